"""Interpolation kernels, deapodization factors and min-max coefficients.

TEST INFRASTRUCTURE (oracle).  FP64.

Section 2.1.3 (eq 2.10-2.11) replaces the ideal sinc interpolator T by a sparse
interpolator T_sparse applied after an oversampled FFT of a pre-scaled image
(P = diagonal scaling).  The paper names the Kaiser-Bessel interpolation
function and the min-max NUFFT (Introduction; Section 2.1.3) but fixes neither
the kernel parameters nor the scaling; the readings used here are:

  * Kaiser-Bessel kernel of width J (grid units), shape beta (default 2.34 J):
        psi(u) = I0(beta sqrt(1 - (2u/J)^2)) / I0(beta),   |u| <= J/2;
  * its continuous Fourier transform (cycles per grid unit f):
        Psi(f) = (J / I0(beta)) sinh(z)/z,  z = sqrt(beta^2 - (pi J f)^2)
    (sin(z')/z' with z' = sqrt((pi J f)^2 - beta^2) past the zero crossing);
  * deapodization (the diagonal of P): s(m) = 1 / Psi(m / K), m in [-N/2, N/2);
  * min-max coefficients for one axis: c = T^-1 r with
        T[j, l] = sum_m s(m)^2 exp(i gamma (j - l) m),
        r[j]    = sum_m s(m) exp(-i gamma u_j m),
    i.e. the least-squares fit of exp(-i omega m) by s(m) sum_j c_j exp(-i gamma kappa_j m)
    over all m, which minimises the worst-case error over unit-norm inputs.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

TWO_PI = 2.0 * math.pi


def default_beta(J: int) -> float:
    return 2.34 * J


def kb_psi(u: np.ndarray, J: int, beta: float) -> np.ndarray:
    """Kaiser-Bessel kernel psi(u), zero outside |u| <= J/2."""
    u = np.asarray(u, dtype=np.float64)
    a = 1.0 - (2.0 * u / J) ** 2
    out = special.i0(beta * np.sqrt(np.clip(a, 0.0, None))) / special.i0(beta)
    return np.where(a >= 0.0, out, 0.0)


def kb_psi_hat(f: np.ndarray, J: int, beta: float) -> np.ndarray:
    """Continuous Fourier transform of kb_psi at frequency f (cycles per unit)."""
    f = np.asarray(f, dtype=np.float64)
    z2 = beta ** 2 - (math.pi * J * f) ** 2
    out = np.empty_like(z2)
    pos = z2 > 0
    z = np.sqrt(np.abs(z2))
    with np.errstate(invalid="ignore", divide="ignore"):
        out[pos] = np.sinh(z[pos]) / z[pos]
        neg = z2 < 0
        out[neg] = np.sin(z[neg]) / z[neg]
    out[z2 == 0] = 1.0
    return out * (J / special.i0(beta))


def deapod(N: int, K: int, J: int, beta: float) -> np.ndarray:
    """s(m) = 1/Psi(m/K) for m = -N/2..N/2-1 (array index m + N/2)."""
    m = np.arange(N, dtype=np.float64) - N // 2
    return 1.0 / kb_psi_hat(m / K, J, beta)


def neighbours(omega_d: np.ndarray, K: int, J: int):
    """Neighbour rule for one axis.

    Returns (kappa, u): kappa[p, j] = k0 + j + 1 (integers, not yet wrapped)
    and the offsets u[p, j] = t - kappa[p, j], with t = omega / (2 pi / K),
    all in FP64.  The taps and the offsets both come from the one rounded
    value s = t - J/2: k0 = floor(s), frac = s - k0 (exact, in [0, 1)) and
    u = J/2 + frac - (j + 1).  The offsets then lie in [-J/2, J/2) as they do
    in exact arithmetic; forming t - kappa from the unrounded t instead can
    put the last offset just below -J/2 where s rounded onto an integer,
    outside the kernel's support.
    """
    gamma = TWO_PI / K
    t = np.asarray(omega_d, dtype=np.float64) / gamma
    s = t - J / 2
    k0 = np.floor(s)
    frac = s - k0
    j = np.arange(1, J + 1, dtype=np.float64)
    kappa = k0[:, None] + j[None, :]
    u = (J / 2 - j)[None, :] + frac[:, None]
    return kappa.astype(np.int64), u


def minmax_T(N: int, K: int, J: int, s: np.ndarray) -> np.ndarray:
    gamma = TWO_PI / K
    m = np.arange(N, dtype=np.float64) - N // 2
    d = np.arange(J)[:, None] - np.arange(J)[None, :]
    return np.einsum("m,jlm->jl", s ** 2, np.exp(1j * gamma * d[:, :, None] * m[None, None, :]))


def minmax_coeffs(u: np.ndarray, N: int, K: int, s: np.ndarray) -> np.ndarray:
    """Min-max interpolation coefficients c[p, j] for offsets u[p, j] (one axis)."""
    J = u.shape[1]
    gamma = TWO_PI / K
    m = np.arange(N, dtype=np.float64) - N // 2
    T = minmax_T(N, K, J, s)
    r = np.einsum("m,pjm->pj", s, np.exp(-1j * gamma * u[:, :, None] * m[None, None, :]))
    return np.linalg.solve(T[None, :, :], r[:, :, None])[:, :, 0]


def weights(omega_d: np.ndarray, N: int, K: int, J: int, beta: float, kernel: str,
            s: np.ndarray):
    """(kappa, w) for one axis; w is real for 'kb' and complex for 'minmax'."""
    kappa, u = neighbours(omega_d, K, J)
    if kernel == "kb":
        w = kb_psi(u, J, beta)
    elif kernel == "minmax":
        w = minmax_coeffs(u, N, K, s)
    else:
        raise ValueError(kernel)
    return kappa, w

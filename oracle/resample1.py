"""Radial -> umbrella resampling of the derivative-Radon space, method 1.

TEST INFRASTRUCTURE (oracle).  FP64.

Method 1 of Section 2.1.3 (eq 2.8-2.11): the ideal interpolator T of eq 2.8
(a periodic sinc in every axis of the uniformly sampled (phi, theta, rho)
index space, eq 2.2-2.7) is written as T F F^-1 (eq 2.9), and F P F^-1
(eq 2.11) replaces it by an oversampled NUFFT whose pre-scaling P lets the
interpolator be truncated to a sparse T_sparse.  Two functions here:

* ``exact``: the ideal interpolator itself, x~(t) = sum_m S[m]
  exp(-2 pi i sum_d m_d t_d / N_d) with S the centred spectrum of the samples
  (eq 2.2-2.5), written out as a direct sum;
* ``nufft_steps``: eq 2.11 step by step: F^-1 (inverse DFT), P (scaling
  s_d(m_d) = 1/Psi(m_d/K_d) and zero padding to K_d = 2 N_d, the factor-2
  oversampling the section prefers for the Kaiser-Bessel kernel), F (FFT of
  the padded grid), T_sparse (the J^3 Kaiser-Bessel taps of the NUFFT).

Readings:

* the spectrum band is centred: m_d in [-N_d/2, N_d/2) (N_d even), the band
  of a signal sampled above its Nyquist rate; eq 2.2-2.7 index the band
  0..N-1, which differs by the phasor the section points out and does not
  reproduce a band-limited signal between the samples;
* the signs follow eq 2.2-2.3: the spectrum is taken with exp(+i..) and the
  1/N_d that makes the interpolator reproduce the samples (eq 2.8: an
  interpolation), the evaluation with exp(-i..);
* every axis is periodic in index space, as the DFT of eq 2.9 makes it:
  phi is periodic in fact; rho is, to the extent the Radon values vanish
  beyond the object; theta is not, so targets in the unsampled polar caps get
  the periodic interpolant's values (method 2 gives zero taps there);
* the NUFFT of the T_sparse step evaluates sum_m S'[m] exp(-i omega . m) at
  omega_d = 2 pi t_d / N_d, i.e. at grid coordinate t_d K_d / N_d = 2 t_d,
  with the neighbour rule of the projector's NUFFT in grid-index form: taps
  k0+1..k0+J, k0 = floor(2 t_d - J/2), offsets u = J/2 - j + frac in
  [-J/2, J/2), weights psi(u) (Kaiser-Bessel, beta = 2.34 J), all taps
  wrapped mod K_d.
* index coordinates of a target (theta, phi, rho), as for method 2:
  t_phi = phi N_phi / (2 pi), t_theta = (theta - theta_0) / dtheta,
  t_rho = rho + N_r / 2.

Layouts: samples D[a][b][c] = [phi][theta][rho] (the projector's output for the
(phi, theta) line grid); targets t[p] = (t_phi, t_theta, t_rho).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import fft as sfft

from . import kernels


def centred_spectrum(D: np.ndarray) -> np.ndarray:
    """S[m + N/2] = (1/N_tot) sum_n D[n] exp(+2 pi i sum_d m_d n_d / N_d), m_d in [-N_d/2, N_d/2)."""
    D = np.asarray(D, dtype=np.complex128)
    assert all(n % 2 == 0 for n in D.shape), "even sizes"
    return np.fft.fftshift(sfft.ifftn(D))


def exact(D: np.ndarray, t: np.ndarray) -> np.ndarray:
    """The ideal (periodic sinc) interpolant at index coordinates t (P, 3), eq 2.8."""
    D = np.asarray(D, dtype=np.complex128)
    t = np.asarray(t, dtype=np.float64).reshape(-1, 3)
    S = centred_spectrum(D)
    E = []
    for d in range(3):
        n = D.shape[d]
        m = np.arange(n) - n // 2
        E.append(np.exp(-2j * math.pi * np.outer(t[:, d], m) / n))  # (P, N_d)
    # sum over m2, then m1, then m0 of S[m0, m1, m2] E0 E1 E2
    s2 = np.einsum("abc,pc->abp", S, E[2])
    s1 = np.einsum("abp,pb->ap", s2, E[1])
    return np.einsum("ap,pa->p", s1, E[0])


def taps(tg: np.ndarray, J: int, beta: float):
    """Neighbour rule at grid coordinates tg: taps k0+1..k0+J and KB weights."""
    s = np.asarray(tg, dtype=np.float64) - J / 2
    k0 = np.floor(s)
    frac = s - k0
    j = np.arange(1, J + 1, dtype=np.float64)
    kappa = (k0[:, None] + j[None, :]).astype(np.int64)
    u = (J / 2 - j)[None, :] + frac[:, None]
    return kappa, kernels.kb_psi(u, J, beta)


def oversampled_grid(D: np.ndarray, J: int, beta: float | None = None) -> np.ndarray:
    """F P F^-1 D of eq 2.11: the K_0 x K_1 x K_2 grid (K_d = 2 N_d), frequency kappa at kappa mod K_d."""
    beta = kernels.default_beta(J) if beta is None else beta
    D = np.asarray(D, dtype=np.complex128)
    N = D.shape
    K = tuple(2 * n for n in N)
    S = centred_spectrum(D)                                   # F^-1
    s = [kernels.deapod(N[d], K[d], J, beta) for d in range(3)]
    g = np.zeros(K, dtype=np.complex128)                      # P: scale, pad at (m mod K)
    q = [np.mod(np.arange(N[d]) - N[d] // 2, K[d]) for d in range(3)]
    g[np.ix_(*q)] = S * s[0][:, None, None] * s[1][None, :, None] * s[2][None, None, :]
    return sfft.fftn(g)                                       # F


def interpolate(Y: np.ndarray, t: np.ndarray, J: int, beta: float | None = None) -> np.ndarray:
    """T_sparse of eq 2.11: J^3 KB taps around grid coordinates 2 t, wrapped mod K_d."""
    beta = kernels.default_beta(J) if beta is None else beta
    t = np.asarray(t, dtype=np.float64).reshape(-1, 3)
    K = Y.shape
    idx, wts = [], []
    for d in range(3):
        k, w = taps(2.0 * t[:, d], J, beta)
        idx.append(np.mod(k, K[d]))
        wts.append(w)
    out = np.zeros(t.shape[0], dtype=np.complex128)
    for a in range(J):
        for b in range(J):
            wab = wts[0][:, a] * wts[1][:, b]
            for c in range(J):
                out += wab * wts[2][:, c] * Y[idx[0][:, a], idx[1][:, b], idx[2][:, c]]
    return out


def nufft_steps(D: np.ndarray, t: np.ndarray, J: int, beta: float | None = None) -> np.ndarray:
    """Method 1, eq 2.11: T_sparse F P F^-1 D at index coordinates t."""
    return interpolate(oversampled_grid(D, J, beta), t, J, beta)


def index_coords(n_phi: int, theta0: float, dtheta: float, n_r: int,
                 theta: np.ndarray, phi: np.ndarray, rho: np.ndarray) -> np.ndarray:
    """(t_phi, t_theta, t_rho) of targets (theta, phi, rho) on the radial grid."""
    return np.stack([np.asarray(phi) / (2 * math.pi / n_phi), (np.asarray(theta) - theta0) / dtheta,
                     np.asarray(rho) + n_r / 2], axis=1)


def resample(D: np.ndarray, n_phi: int, theta0: float, dtheta: float, n_theta: int, n_r: int,
             theta: np.ndarray, phi: np.ndarray, rho: np.ndarray, J: int,
             beta: float | None = None) -> np.ndarray:
    """Method 1 at umbrella samples (theta, phi, rho) from D[(a * n_theta + b) * n_r + j]."""
    Dg = np.asarray(D, dtype=np.complex128).reshape(n_phi, n_theta, n_r)
    return nufft_steps(Dg, index_coords(n_phi, theta0, dtheta, n_r, theta, phi, rho), J, beta)

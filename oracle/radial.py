"""Radial stage: Fourier-slice samples -> first-derivative Radon values.

TEST INFRASTRUCTURE (oracle).  FP64.

By the 3D Fourier slice theorem (Section 2.2.1) the samples X(r nhat) along a
line through the origin are the 1D Fourier transform of the plane integrals
R(rho, nhat).  Section 2.4.1 (eq 2.17-2.18) takes the derivative in the Fourier
domain (one multiply per sample) and then one inverse FFT per radial line.

Readings: each line carries N_r samples r_c = (c - N_r/2)(2 pi / N_r) of
[-pi, pi); the output is indexed by rho_j = j - N_r/2 in voxel units;
derivative factor f_c = i r_c except f_0 = 0 (the unpaired sample at r = -pi,
so that real volumes give real output); normalisation 1/N_r:

    D[l, j] = (1/N_r) sum_c f_c G[l, c] exp(+i r_c rho_j).

The adjoint is the conjugate transpose:

    G~[l, c] = conj(f_c) (1/N_r) sum_j d[l, j] exp(-i r_c rho_j).

Both are written as a dense matrix product with the exponentials formed
directly from r_c and rho_j.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def r_grid(n_r: int) -> np.ndarray:
    return (np.arange(n_r, dtype=np.float64) - (n_r // 2)) * (TWO_PI / n_r)


def rho_grid(n_r: int) -> np.ndarray:
    return np.arange(n_r, dtype=np.float64) - (n_r // 2)


def deriv_factor(n_r: int, deriv: bool = True) -> np.ndarray:
    if not deriv:
        return np.ones(n_r, dtype=np.complex128)
    f = 1j * r_grid(n_r)
    f[0] = 0.0
    return f


def directions(phi: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """Unit line directions from eq 2.1 (rho = 1): (sin th cos ph, sin th sin ph, cos th),
    azimuth index outer, polar index inner."""
    out = []
    for ph in np.asarray(phi, dtype=np.float64):
        for th in np.asarray(theta, dtype=np.float64):
            out.append([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    return np.array(out, dtype=np.float64)


def points(dirs: np.ndarray, n_r: int) -> np.ndarray:
    """omega[l*N_r + c] = r_c * nhat_l (r_c formed first, then one FP64 product)."""
    r = r_grid(n_r)
    return (r[None, :, None] * np.asarray(dirs, dtype=np.float64)[:, None, :]).reshape(-1, 3)


def _idft_matrix(n_r: int) -> np.ndarray:
    """E[j, c] = exp(+i r_c rho_j)."""
    return np.exp(1j * np.outer(rho_grid(n_r), r_grid(n_r)))


def forward(G: np.ndarray, n_r: int, deriv: bool = True) -> np.ndarray:
    """D[l, j] = (1/N_r) sum_c f_c G[l, c] exp(+i r_c rho_j); G is (L*N_r,) line-major."""
    G = np.asarray(G, dtype=np.complex128).reshape(-1, n_r)
    f = deriv_factor(n_r, deriv)
    E = _idft_matrix(n_r)
    return ((G * f[None, :]) @ E.T / n_r).reshape(-1)


def adjoint(d: np.ndarray, n_r: int, deriv: bool = True) -> np.ndarray:
    """G~[l, c] = conj(f_c) (1/N_r) sum_j d[l, j] exp(-i r_c rho_j)."""
    d = np.asarray(d, dtype=np.complex128).reshape(-1, n_r)
    f = deriv_factor(n_r, deriv)
    E = _idft_matrix(n_r)
    return ((d @ np.conj(E)) * np.conj(f)[None, :] / n_r).reshape(-1)

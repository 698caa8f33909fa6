"""Umbrella derivative-Radon values -> cone-beam projections (the Grangeat
step in reverse).

TEST INFRASTRUCTURE (oracle).  FP64.

Step 3 of the forward projector (Section 2, third of its steps; Section 2.2.2,
Figures 2.14-2.15; its cost in eq 2.21-2.24): each projection is made from its
own umbrella subset of derivative-Radon values by de-postweighting (eq 2.21),
radial FFTs (eq 2.22), a 2D NUFFT transpose on a (2N)^2 grid with a [5 5]
interpolation neighbourhood (eq 2.23) and de-preweighting (eq 2.24).  The
section defers the weights to an earlier report that is not available, so
they are taken from Grangeat's relation in its textbook form:

* the projection X(u, v) on the flat detector (source-detector distance D,
  pixel (a, b) at u = (a - n/2) delta, v = (b - n/2) delta along the axes
  u^, v^ of the umbrella geometry, delta = side / n) is the line integral of
  the volume along the ray from the source to the pixel;
* on the virtual detector through the rotation axis (distance R from the
  source, coordinates (u', v') = (u, v) R / D), the pre-weighted projection
  g(u', v') = X R / sqrt(R^2 + u'^2 + v'^2) has the 2D Radon transform
  S(alpha, s') along the lines u' cos alpha + v' sin alpha = s', and
  dRf/drho'(n', rho') = (R^2 + s'^2) / R^2 dS/ds'  (Grangeat), where the
  plane through the source and that line has the unit normal n' whose
  distance rho' = R s' / sqrt(R^2 + s'^2) grows with s';
* the umbrella samples U[k][i][j] are the derivative-Radon values dRf/drho at
  (n^, rho) with the orientation of the umbrella geometry, n^ = -n' and
  rho = -rho' (oracle.umbrella: n^ = (e x q)/|e x q| = -(D w + t s^)/|..|), so
  dRf/drho' = -U; the line of sample j lies at s'_j = t_j R / D with
  t_j = (j - n/2) delta, and alpha_i = pi i / n_alpha.

Steps, per projection, in the section's order:

1. de-postweighting: p'(alpha_i, s'_j) = dS/ds' = -U[i, j] R^2 / (R^2 + s'_j^2);
2. radial FFTs: P'(alpha_i, k_m) = delta' sum_j p'(alpha_i, s'_j)
   exp(-2 pi i k_m s'_j) with each line zero-padded to 2n samples,
   k_m = (m - n) dk, dk = 1 / (2 n delta'), delta' = delta R / D (without the
   padding the transform's circular wrap leaves errors of a few per cent on
   smooth projections); the 2D inversion from derivative data needs no
   ramp: |k| P^ = |k| P'^ / (2 pi i k), so c[i, m] = -i sign(k_m) / (2 pi)
   P'(alpha_i, k_m) times the polar quadrature weights dalpha dk,
   dalpha = pi / n_alpha: the trapezoidal rule in k on |k| P^, whose kink at
   k = 0 the Euler-Maclaurin formula corrects with the weight dk^2 / 6 on
   P(alpha_i, 0) (which the derivative data give as -int s' p' ds'), leaving
   an O(dk^4) error (8e-4 of the peak on a Gaussian blob; 4.5e-5 and 2.9e-6
   with 4x and 8x padding); the unpaired Nyquist sample carries nothing;
3. 2D NUFFT transpose: g[b][a] = sum_{i,m} c[i, m] exp(+i omega_{i,m} . (a - n/2, b - n/2))
   with omega_{i,m} = 2 pi (m - n)/(2n) (cos alpha_i, sin alpha_i) (radians
   per pixel): KB spreading (J = 5, beta = 2.34 J) onto the K x K grid (K = 2n,
   cell kappa at kappa mod K, taps by the neighbour rule of oracle.kernels),
   the unnormalised inverse FFT, the crop to [-n/2, n/2)^2 and the scaling
   s(m_u) s(m_v) = 1/Psi(m/K);
4. de-preweighting: X[b][a] = g[b][a] sqrt(R^2 + u'_a^2 + v'_b^2) / R.

Layouts: U[k][i][j] (projection, detector-line angle, offset), n_t = n the
detector size; X[k][b][a] (projection, v row, u column).
"""
from __future__ import annotations

import math

import numpy as np

from . import kernels
from .umbrella import DET_MM, OBJ_MM, SD_MM, SO_MM


class Scan:
    """Scan in voxel units for an N^3 volume spanning the object (as the
    umbrella geometry), with n x n detector pixels and n_alpha line angles."""

    def __init__(self, N: int, n_alpha: int, n: int, J: int = 5):
        assert n % 2 == 0
        self.N, self.n_alpha, self.n, self.J = N, n_alpha, n, J
        self.R = N * SO_MM / OBJ_MM
        self.D = N * SD_MM / OBJ_MM
        self.side = N * DET_MM / OBJ_MM
        self.delta = self.side / n
        self.delta_v = self.delta * self.R / self.D
        self.K = 2 * n
        self.beta = kernels.default_beta(J)
        self.alpha = math.pi * np.arange(n_alpha) / n_alpha
        self.s_v = (np.arange(n) - n // 2) * self.delta_v   # virtual-detector offsets / coordinates


def depostweight(U: np.ndarray, sc: Scan) -> np.ndarray:
    """Step 1: p'[i, j] = -U[i, j] R^2 / (R^2 + s'_j^2)."""
    R2 = sc.R ** 2
    return -np.asarray(U, dtype=np.complex128) * (R2 / (R2 + sc.s_v ** 2))[None, :]


def radial_spectra(p: np.ndarray, sc: Scan) -> np.ndarray:
    """Step 2: c[i, m], m in [0, 2n): the filtered spectrum of line i at k_m = (m - n) dk.

    P'[i, m] = delta' sum_j p'[i, j] exp(-2 pi i (m - n)(j - n/2) / (2n)) (the
    line zero-padded to 2n samples, dk = 1 / (2 n delta')), times
    -i sign(k_m) / (2 pi) dalpha dk; the k = 0 bin carries the Euler-Maclaurin
    correction of the trapezoidal rule on |k| P^ at its kink,
    dalpha (dk^2 / 6) P(alpha_i, 0), with P(alpha, 0) = int S ds' =
    -int s' p'(s') ds' (S vanishes beyond the object); the unpaired Nyquist
    sample m = 0 carries nothing."""
    n = sc.n
    L = 2 * n
    j = np.arange(n) - n // 2
    k = np.arange(L) - n
    E = np.exp(-2j * math.pi * np.outer(k, j) / L)                # [m][j]
    P = sc.delta_v * (p @ E.T)                                     # [i][m]
    dk = 1.0 / (L * sc.delta_v)
    dalpha = math.pi / sc.n_alpha
    H = -1j * np.sign(k) / (2 * math.pi) * dalpha * dk
    H[0] = 0.0
    c = P * H[None, :]
    P0 = -sc.delta_v * (p @ sc.s_v)
    c[:, n] = dalpha * dk * dk / 6.0 * P0
    return c


def polar_omega(sc: Scan) -> np.ndarray:
    """omega_{i,m} = 2 pi (m - n)/(2n) (cos alpha_i, sin alpha_i), shape (n_alpha * 2n, 2) as (u, v)."""
    r = math.pi * (np.arange(2 * sc.n) - sc.n) / sc.n
    wu = np.cos(sc.alpha)[:, None] * r[None, :]
    wv = np.sin(sc.alpha)[:, None] * r[None, :]
    return np.stack([wu.reshape(-1), wv.reshape(-1)], axis=1)


def nufft2_adjoint(c: np.ndarray, om: np.ndarray, n: int, J: int, beta: float) -> np.ndarray:
    """Step 3: g[b][a] ~= sum_p c_p exp(+i (om_u (a - n/2) + om_v (b - n/2)))."""
    K = 2 * n
    s = kernels.deapod(n, K, J, beta)
    ku, wu = kernels.weights(om[:, 0], n, K, J, beta, "kb", s)
    kv, wv = kernels.weights(om[:, 1], n, K, J, beta, "kb", s)
    Y = np.zeros((K, K), dtype=np.complex128)
    c = np.asarray(c, dtype=np.complex128).reshape(-1)
    for a in range(J):
        for b in range(J):
            np.add.at(Y, (np.mod(kv[:, b], K), np.mod(ku[:, a], K)), wv[:, b] * wu[:, a] * c)
    y = np.fft.ifft2(Y) * float(K) ** 2
    q = np.mod(np.arange(n) - n // 2, K)
    return y[np.ix_(q, q)] * s[:, None] * s[None, :]


def nudft2_adjoint(c: np.ndarray, om: np.ndarray, n: int) -> np.ndarray:
    """The exact sum that nufft2_adjoint approximates."""
    m = np.arange(n) - n // 2
    Eu = np.exp(1j * np.outer(m, om[:, 0]))    # [a][p]
    Ev = np.exp(1j * np.outer(m, om[:, 1]))    # [b][p]
    return (Ev * np.asarray(c).reshape(-1)[None, :]) @ Eu.T


def depreweight(g: np.ndarray, sc: Scan) -> np.ndarray:
    """Step 4: X[b][a] = g[b][a] sqrt(R^2 + u'_a^2 + v'_b^2) / R."""
    u = sc.s_v
    return g * np.sqrt(sc.R ** 2 + u[None, :] ** 2 + u[:, None] ** 2) / sc.R


def projection(U: np.ndarray, sc: Scan) -> np.ndarray:
    """One cone-beam projection X[b][a] from its umbrella samples U[i][j]."""
    c = radial_spectra(depostweight(U, sc), sc)
    g = nufft2_adjoint(c, polar_omega(sc), sc.n, sc.J, sc.beta)
    return depreweight(g, sc)


def projections(U: np.ndarray, sc: Scan) -> np.ndarray:
    """All projections: U[k][i][j] -> X[k][b][a]."""
    U = np.asarray(U).reshape(-1, sc.n_alpha, sc.n)
    return np.stack([projection(U[k], sc) for k in range(U.shape[0])])

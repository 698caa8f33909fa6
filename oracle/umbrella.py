"""Radial -> umbrella resampling of the derivative-Radon space (method 2).

TEST INFRASTRUCTURE (oracle).  FP64.

Step 2 of the forward projector (Section 2, second of its three steps;
Section 2.1): the derivative-Radon values computed on the radial pattern
(azimuth phi, polar angle theta, signed distance rho; eq 2.1) are resampled
onto the planes that pass through the X-ray source positions of a circular
cone-beam scan (the "umbrella" pattern of each projection, Figure 2.2).  The
radial pattern is uniform in (phi, theta, rho) index space, so the resampling
is an interpolation there; method 2 (eq 2.15, T_sparse2 the identity)
applies one truncated interpolator T_sparse1 directly.

Readings (the paper gives the geometry only in figures and Section 3.2.1):

* scan geometry in voxel units for an N^3 volume spanning the 360 mm object:
  source radius R_s = N * 1100/360, source-detector distance D_sd =
  N * 1500/360, flat square detector of side N * 512/360 centred on the
  central ray, source positions lambda_k = 2 pi k / n_proj on the circle in
  the z = 0 plane: s = R_s (cos lambda, sin lambda, 0);
* detector frame: centre c = s - D_sd shat (shat = s / R_s), axes
  u = (-sin lambda, cos lambda, 0), v = (0, 0, 1);
* umbrella of projection k (Grangeat): for every detector line
  {u cos alpha + v sin alpha = t}, alpha_i = pi i / n_alpha,
  t_j = (j - n_t/2) * side / n_t, the plane through the source and that line:
  normal n = e x q with e = -sin(alpha) u + cos(alpha) v (the line's direction)
  and q = c - s + t (cos(alpha) u + sin(alpha) v) (source to the line), nhat =
  n / |n|, rho = nhat . s; (theta, phi) = (acos nhat_z, atan2(nhat_y, nhat_x)
  mod 2 pi);
* index coordinates on the radial grid phi_a = 2 pi a / n_phi, theta_b =
  theta_0 + b dtheta, rho_j = j - n_r/2: t_phi = phi / (2 pi / n_phi),
  t_theta = (theta - theta_0) / dtheta, t_rho = rho + n_r / 2;
* T_sparse1 (the sinc "truncated to its main lobe and a few side lobes",
  Section 2.1.3): per axis the J taps k0+1..k0+J with k0 = floor(t - J/2)
  and the weight w(u) = sinc(u) psi(u) / sum_taps sinc psi at offset
  u = t - kappa, psi the Kaiser-Bessel window of width J with
  beta = 4J/3 (psi(0) = 1); grid nodes are reproduced exactly and the
  normalisation makes constants exact as well; phi taps wrap (periodic),
  theta and rho taps that fall off the sampled grid contribute nothing (the
  unsampled polar caps and the zero Radon values beyond the object).  The
  paper's choice J = 3 is a parameter.

Output layout: [k][i][j] (projection, detector-line angle, detector-line
offset), complex.
"""
from __future__ import annotations

import math

import numpy as np

from . import kernels

SO_MM, SD_MM, DET_MM, OBJ_MM = 1100.0, 1500.0, 512.0, 360.0


def geometry(N: int, n_proj: int, n_alpha: int, n_t: int):
    """Plane normals (P, 3) and signed distances (P,) of the umbrella samples."""
    return geometry_at(N, n_proj, n_alpha, n_t, np.arange(n_proj * n_alpha * n_t))


def geometry_at(N: int, n_proj: int, n_alpha: int, n_t: int, samples):
    """As geometry, for the samples p = (k * n_alpha + i) * n_t + j listed."""
    R_s = N * SO_MM / OBJ_MM
    D_sd = N * SD_MM / OBJ_MM
    side = N * DET_MM / OBJ_MM
    samples = np.asarray(samples, dtype=np.int64).reshape(-1)
    nh = np.empty((len(samples), 3))
    rho = np.empty(len(samples))
    for q, p in enumerate(samples):
        k, rem = divmod(int(p), n_alpha * n_t)
        i, j = divmod(rem, n_t)
        lm = 2 * math.pi * k / n_proj
        al = math.pi * i / n_alpha
        tj = (j - n_t // 2) * (side / n_t)
        shat = np.array([math.cos(lm), math.sin(lm), 0.0])
        s = R_s * shat
        c = s - D_sd * shat
        u = np.array([-math.sin(lm), math.cos(lm), 0.0])
        v = np.array([0.0, 0.0, 1.0])
        e = -math.sin(al) * u + math.cos(al) * v
        w = math.cos(al) * u + math.sin(al) * v
        qv = c - s + tj * w
        n = np.cross(e, qv)
        n = n / np.linalg.norm(n)
        nh[q] = n
        rho[q] = n @ s
    return nh, rho


def angles(nh: np.ndarray):
    """(theta, phi) of unit normals, theta in [0, pi], phi in [0, 2 pi)."""
    th = np.arccos(np.clip(nh[:, 2], -1.0, 1.0))
    ph = np.mod(np.arctan2(nh[:, 1], nh[:, 0]), 2 * math.pi)
    return th, ph


def window_beta(J: int) -> float:
    return 4.0 * J / 3.0


def window_sinc(u: np.ndarray, J: int, beta: float) -> np.ndarray:
    """sinc(u) * psi(u): the sinc truncated to |u| < J/2 by the KB window."""
    return np.sinc(u) * kernels.kb_psi(u, J, beta)


def resample(D: np.ndarray, n_phi: int, theta0: float, dtheta: float, n_theta: int, n_r: int,
             theta: np.ndarray, phi: np.ndarray, rho: np.ndarray, J: int,
             beta: float | None = None) -> np.ndarray:
    """Values at (theta, phi, rho) from D[(a * n_theta + b) * n_r + j] by T_sparse1."""
    beta = window_beta(J) if beta is None else beta
    Dg = np.asarray(D, dtype=np.complex128).reshape(n_phi, n_theta, n_r)
    t = [np.asarray(phi) / (2 * math.pi / n_phi), (np.asarray(theta) - theta0) / dtheta,
         np.asarray(rho) + n_r / 2]
    out = np.zeros(len(t[0]), dtype=np.complex128)
    idx, wts = [], []
    for d in range(3):
        k0 = np.floor(t[d] - J / 2.0)
        kap = k0[:, None] + np.arange(1, J + 1)[None, :]
        idx.append(kap.astype(np.int64))
        w = window_sinc(t[d][:, None] - kap, J, beta)
        wts.append(w / w.sum(axis=1, keepdims=True))
    for a in range(J):
        ia = np.mod(idx[0][:, a], n_phi)
        for b in range(J):
            ib = idx[1][:, b]
            okb = (ib >= 0) & (ib < n_theta)
            for c in range(J):
                ic = idx[2][:, c]
                ok = okb & (ic >= 0) & (ic < n_r)
                w = wts[0][:, a] * wts[1][:, b] * wts[2][:, c]
                v = np.zeros(len(out), dtype=np.complex128)
                v[ok] = Dg[ia[ok], ib[ok], ic[ok]]
                out += w * v
    return out

"""Direct reconstruction from radially sampled first-derivative Radon data.

TEST INFRASTRUCTURE (oracle).  FP64.

Section 2.3 inverts module 1 of the projector (image -> derivative Radon
space) by a Fourier-domain ramp filter followed by the NUFFT transpose; the
Introduction names the ramp of the 3D parallel geometry as R^2 in the Fourier
domain (R the radial frequency).  Written out with the 3D inverse Fourier
transform in spherical coordinates, every direction nhat of the unit sphere
S^2 taken once and r running over the whole line (so that each frequency is
met twice, hence the 1/2):

    x(m) = 1 / (2 (2 pi)^3)  int_{S^2} int_{-inf}^{inf} r^2 X(r nhat) exp(+i r nhat . m) dr dOmega.

With the radial samples r_c (spacing 2 pi / N_r), quadrature weights w_l for
the line directions and the projector's adjoint A^H (derivative factor, radial
DFT with the 1/N_r normalisation and the exact NUFFT transpose), the ramp r^2
is conj(f_c) f_c and the sum over c carries N_r * (2 pi / N_r) = 2 pi, so

    x~ = 1 / (8 pi^2)  A^H diag(w) d,

where d are the derivative-Radon values (the projector's output layout).
The same constant is the one of the 3D Radon inversion formula
x = -1/(8 pi^2) int_{S^2} R'' dOmega written in the Fourier domain.

Quadrature (a reading: the paper gives only the sample counts): the product
rule on the (phi, theta) grid, the periodic midpoint spacing in phi and the
trapezoid rule in theta on [theta_0, theta_last], each times sin(theta);
lines are ordered [phi][theta] like the projector's.
"""
from __future__ import annotations

import math

import numpy as np

from . import projector

RECON_SCALE = 1.0 / (8.0 * math.pi ** 2)


def quadrature(phi: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """w[a * n_theta + b] = dphi_a * dtheta_b * sin(theta_b)."""
    phi = np.asarray(phi, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    n_phi, n_th = len(phi), len(theta)
    # periodic spacing in phi: half the distance between the two neighbours
    nxt = np.roll(phi, -1)
    prv = np.roll(phi, 1)
    dphi = 0.5 * (np.mod(nxt - phi, 2 * math.pi) + np.mod(phi - prv, 2 * math.pi))
    if n_phi == 1:
        dphi = np.array([2 * math.pi])
    # trapezoid in theta
    dth = np.zeros(n_th)
    if n_th == 1:
        dth[0] = 2.0  # a single polar angle stands for the whole sphere's sin integral
    else:
        gaps = np.diff(theta)
        dth[:-1] += 0.5 * gaps
        dth[1:] += 0.5 * gaps
    return (dphi[:, None] * (dth * np.sin(theta))[None, :]).reshape(-1)


def reconstruct(d: np.ndarray, dirs: np.ndarray, n_r: int, weights: np.ndarray, prm=None,
                N: int | None = None, exact: bool = False) -> np.ndarray:
    """x~ = 1/(8 pi^2) A^H diag(w) d with A the derivative-Radon projector."""
    L = len(dirs)
    dw = (np.asarray(d, dtype=np.complex128).reshape(L, n_r) * np.asarray(weights)[:, None]).reshape(-1)
    return RECON_SCALE * projector.adjoint(dw, dirs, n_r, prm, N=N, deriv=True, exact=exact)

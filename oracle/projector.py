"""Image -> radially sampled first-derivative Radon space, and its adjoint.

TEST INFRASTRUCTURE (oracle).  FP64.

Module 1 of the forward projector (Section 2, the first of its three steps;
Section 2.4.1, eq 2.16-2.18): a 3D NUFFT at the points r_c nhat_l of radial
lines, the derivative factor, then one radial inverse DFT per line.  The
adjoint applies the transposes in reverse order.  `exact=True` replaces the
NUFFT by the exact NUDFT.
"""
from __future__ import annotations

import numpy as np

from . import nudft, nufft, radial


def forward(x: np.ndarray, dirs: np.ndarray, n_r: int, prm: nufft.Params | None,
            deriv: bool = True, radial_stage: bool = True, exact: bool = False) -> np.ndarray:
    om = radial.points(dirs, n_r)
    G = nudft.nudft3(x, om) if exact else nufft.forward(x, om, prm)
    return radial.forward(G, n_r, deriv) if radial_stage else G


def adjoint(d: np.ndarray, dirs: np.ndarray, n_r: int, prm: nufft.Params | None, N: int | None = None,
            deriv: bool = True, radial_stage: bool = True, exact: bool = False) -> np.ndarray:
    om = radial.points(dirs, n_r)
    Gt = radial.adjoint(d, n_r, deriv) if radial_stage else np.asarray(d, dtype=np.complex128)
    if exact:
        return nudft.nudft3_adjoint(Gt, om, N if N is not None else prm.N)
    return nufft.adjoint(Gt, om, prm)

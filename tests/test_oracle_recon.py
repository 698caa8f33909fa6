"""Pins for the direct reconstruction oracle (oracle.recon, Section 2.3).

The data are the closed-form first-derivative Radon values of Gaussian blobs
(written out here, independent of the oracle's projector), so the pins check
the ramp, the quadrature and the 1/(8 pi^2) constant against the mathematics.
"""
import math

import numpy as np
import pytest

import synthetic
from oracle import nufft, projector, recon


def _gauss_dradon(rho, n, c, cov):
    s2 = n @ cov @ n
    mass = (2 * math.pi) ** 1.5 * math.sqrt(np.linalg.det(cov))
    R = mass * np.exp(-(rho - n @ c) ** 2 / (2 * s2)) / math.sqrt(2 * math.pi * s2)
    return -(rho - n @ c) / s2 * R


def _lines(n_phi, margin):
    phi = synthetic.azimuths(n_phi)
    th = synthetic.polar_angles(n_phi // 2, margin=margin)
    return phi, th, synthetic.line_directions(phi, th)


def _recon_gauss(N, n_r, n_phi, margin, c, cov, exact=False):
    phi, th, dirs = _lines(n_phi, margin)
    rho = np.arange(n_r) - n_r // 2
    d = np.stack([_gauss_dradon(rho, n, c, cov) for n in dirs]).reshape(-1)
    w = recon.quadrature(phi, th)
    prm = None if exact else nufft.Params(N, 2 * N, 6)
    xr = recon.reconstruct(d, dirs, n_r, w, prm, N=N, exact=exact)
    return xr, synthetic.gaussian_blob(N, c, cov), w


@pytest.mark.parametrize("margin", [0.0, 0.2])
def test_quadrature_moments(margin):
    # int over the band theta in [m, pi - m] of 1, cos^2 and sin^2 cos^2(phi):
    # 4 pi cos m, (4 pi / 3) cos^3 m, pi (2 cos m - (2/3) cos^3 m)
    cm = math.cos(margin)
    want = np.array([4 * math.pi * cm, 4 * math.pi / 3 * cm ** 3, math.pi * (2 * cm - 2 * cm ** 3 / 3)])
    errs = []
    for n_phi in (32, 64):
        phi, th, dirs = _lines(n_phi, margin)
        w = recon.quadrature(phi, th)
        assert w.shape == (len(dirs),) and np.all(w >= 0)
        got = np.array([w.sum(), w @ dirs[:, 2] ** 2, w @ dirs[:, 0] ** 2])
        errs.append(np.abs(got - want) / want)
        # trapezoid rule in theta: error <= (b - a) h^2 / 12 * max|f''| with |f''| <= 2 pi * 4
        h = th[1] - th[0]
        assert np.all(np.abs(got - want) <= (math.pi - 2 * margin) * h * h / 12 * 8 * math.pi)
    # second order: halving the spacing cuts the error about four times
    assert np.all(errs[1] < errs[0] / 3)


@pytest.mark.parametrize("margin", [0.0, 0.2])
def test_center_ratio_equals_solid_angle(margin):
    # an isotropic Gaussian at the centre has the same transform along every line,
    # so the reconstruction at the centre is x(0) * sum_l w_l / (4 pi): this pins
    # the ramp r^2, the radial normalisation and the 1/(8 pi^2) constant
    N, n_r = 32, 64
    xr, x, w = _recon_gauss(N, n_r, 48, margin, np.zeros(3), np.eye(3) * 2.5 ** 2)
    ctr = (N // 2,) * 3
    assert abs(xr[ctr].real / x[ctr] - w.sum() / (4 * math.pi)) < 1e-5
    # the missing polar caps remove a fraction 1 - cos(margin) of the sphere
    assert abs(w.sum() / (4 * math.pi) - math.cos(margin)) < 3e-3
    assert np.max(np.abs(xr.imag)) < 1e-5 * x.max()


def test_full_sphere_converges_with_lines():
    # an off-centre anisotropic Gaussian (band-limited to |omega| < pi) is
    # recovered as the angular sampling grows (no polar caps missing)
    N, n_r = 32, 64
    c = np.array([2.0, -1.5, 1.0])
    cov = np.diag([2.5, 3.0, 3.5]) ** 2
    errs = []
    for n_phi in (16, 32, 64):
        xr, x, _ = _recon_gauss(N, n_r, n_phi, 0.0, c, cov)
        errs.append(np.linalg.norm(xr - x) / np.linalg.norm(x))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-2


def test_missing_caps_plateau():
    # with the polar caps theta < 0.2 unsampled the error stops falling: the
    # plateau the angular-sampling experiment of Section 3.1 looks for
    N, n_r = 32, 64
    cov = np.eye(3) * 2.5 ** 2
    errs = []
    for n_phi in (32, 48, 64):
        xr, x, _ = _recon_gauss(N, n_r, n_phi, 0.2, np.zeros(3), cov)
        errs.append(np.linalg.norm(xr - x) / np.linalg.norm(x))
    assert abs(errs[2] - errs[1]) < 0.02 * errs[1]
    assert errs[2] > 0.05


def test_forward_then_reconstruct_matches_closed_form_data():
    # the projector's own output (pinned against the same closed form) gives
    # the same reconstruction as the closed-form data
    N, n_r = 24, 48
    c = np.array([1.0, 0.5, -1.0])
    cov = np.diag([2.5, 2.8, 3.0]) ** 2
    phi, th, dirs = _lines(24, 0.2)
    prm = nufft.Params(N, 2 * N, 6)
    x = synthetic.gaussian_blob(N, c, cov)
    d = projector.forward(x, dirs, n_r, prm)
    w = recon.quadrature(phi, th)
    xa = recon.reconstruct(d, dirs, n_r, w, prm)
    rho = np.arange(n_r) - n_r // 2
    dc = np.stack([_gauss_dradon(rho, n, c, cov) for n in dirs]).reshape(-1)
    xb = recon.reconstruct(dc, dirs, n_r, w, prm)
    assert np.linalg.norm(xa - xb) / np.linalg.norm(xb) < 1e-4


def test_detects_missing_sine(monkeypatch):
    orig = recon.quadrature

    def flat(phi, theta):
        w = orig(phi, theta)
        th = np.tile(np.asarray(theta), len(phi))
        return w / np.sin(th)

    monkeypatch.setattr(recon, "quadrature", flat)
    N, n_r = 32, 64
    xr, x, _ = _recon_gauss(N, n_r, 48, 0.2, np.zeros(3), np.eye(3) * 2.5 ** 2)
    ctr = (N // 2,) * 3
    assert abs(xr[ctr].real / x[ctr] - math.cos(0.2)) > 0.1


def test_detects_wrong_constant(monkeypatch):
    monkeypatch.setattr(recon, "RECON_SCALE", 1.0 / (4 * math.pi ** 2))
    N, n_r = 32, 64
    xr, x, w = _recon_gauss(N, n_r, 48, 0.0, np.zeros(3), np.eye(3) * 2.5 ** 2)
    ctr = (N // 2,) * 3
    assert abs(xr[ctr].real / x[ctr] - w.sum() / (4 * math.pi)) > 0.5

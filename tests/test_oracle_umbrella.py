"""Pins for the radial -> umbrella resampling oracle (oracle.umbrella, eq 2.15)."""
import math

import numpy as np
import pytest

import synthetic
from oracle import umbrella


def _grid(n_phi, n_th, n_r, margin=0.2):
    phi = synthetic.azimuths(n_phi)
    th = synthetic.polar_angles(n_th, margin=margin)
    return phi, th, th[0], th[1] - th[0], np.arange(n_r) - n_r // 2


def test_geometry_planes_contain_source_and_detector_line():
    N, n_proj, n_alpha, n_t = 16, 3, 4, 5
    nh, rho = umbrella.geometry(N, n_proj, n_alpha, n_t)
    assert nh.shape == (n_proj * n_alpha * n_t, 3)
    assert np.allclose(np.linalg.norm(nh, axis=1), 1.0, atol=1e-15)
    R_s, D_sd, side = N * 1100 / 360, N * 1500 / 360, N * 512 / 360
    p = 0
    for k in range(n_proj):
        lam = 2 * math.pi * k / n_proj
        s = R_s * np.array([math.cos(lam), math.sin(lam), 0.0])
        c = s * (1 - D_sd / R_s)
        u = np.array([-math.sin(lam), math.cos(lam), 0.0])
        v = np.array([0.0, 0.0, 1.0])
        for i in range(n_alpha):
            al = math.pi * i / n_alpha
            for j in range(n_t):
                t = (j - n_t // 2) * side / n_t
                # three points of the detector line u cos a + v sin a = t, and the source
                for tau in (-2.0, 0.0, 3.5):
                    uu = t * math.cos(al) - tau * math.sin(al)
                    vv = t * math.sin(al) + tau * math.cos(al)
                    q = c + uu * u + vv * v
                    assert abs(nh[p] @ q - rho[p]) < 1e-9 * N
                assert abs(nh[p] @ s - rho[p]) < 1e-9 * N
                p += 1


def test_geometry_special_planes():
    # the vertical and the horizontal detector lines through the detector centre
    # span planes through the origin: normals along u and along z, rho = 0
    N, n_proj, n_alpha, n_t = 8, 4, 2, 2
    nh, rho = umbrella.geometry(N, n_proj, n_alpha, n_t)
    nh = nh.reshape(n_proj, n_alpha, n_t, 3)
    rho = rho.reshape(n_proj, n_alpha, n_t)
    for k in range(n_proj):
        lam = 2 * math.pi * k / n_proj
        u = np.array([-math.sin(lam), math.cos(lam), 0.0])
        # alpha = 0: the line u = t; j = n_t/2 is t = 0
        assert abs(rho[k, 0, 1]) < 1e-12 and abs(abs(nh[k, 0, 1] @ u) - 1) < 1e-12
        # alpha = pi/2: the line v = t
        assert abs(rho[k, 1, 1]) < 1e-12 and abs(abs(nh[k, 1, 1, 2]) - 1) < 1e-12


def test_grid_nodes_are_reproduced():
    n_phi, n_th, n_r = 12, 9, 16
    phi, th, th0, dth, rho = _grid(n_phi, n_th, n_r)
    rng = np.random.default_rng(3)
    D = rng.standard_normal(n_phi * n_th * n_r) + 1j * rng.standard_normal(n_phi * n_th * n_r)
    a = rng.integers(0, n_phi, 40)
    b = rng.integers(0, n_th, 40)
    j = rng.integers(0, n_r, 40)
    for J in (3, 6):
        got = umbrella.resample(D, n_phi, th0, dth, n_th, n_r, th[b], phi[a], rho[j].astype(float), J)
        want = D.reshape(n_phi, n_th, n_r)[a, b, j]
        assert np.max(np.abs(got - want)) < 1e-13


def test_constants_and_periodic_phi():
    # normalised weights reproduce a constant anywhere inside the grid, and phi wraps
    n_phi, n_th, n_r = 16, 12, 24
    phi, th, th0, dth, rho = _grid(n_phi, n_th, n_r)
    D = np.full(n_phi * n_th * n_r, 2.5 - 1.0j)
    rng = np.random.default_rng(4)
    J = 6
    tq = rng.uniform(th0 + 3 * dth, th0 + (n_th - 4) * dth, 50)
    pq = np.concatenate([rng.uniform(0, 2 * math.pi, 45), [0.0, 1e-9, 2 * math.pi - 1e-9, 0.01, 6.28]])
    rq = rng.uniform(-n_r / 2 + 3, n_r / 2 - 4, 50)
    got = umbrella.resample(D, n_phi, th0, dth, n_th, n_r, tq, pq, rq, J)
    assert np.max(np.abs(got - (2.5 - 1.0j))) < 1e-13


def _smooth(th, ph, r):
    return np.cos(ph) * np.cos(2 * th) * np.exp(-(r / 8.0) ** 2) + 1j * np.sin(2 * ph) * np.exp(-(r / 6.0) ** 2)


@pytest.mark.parametrize("J,tol", [(3, 1.5e-2), (6, 5e-4)])
def test_smooth_function_accuracy(J, tol):
    # an oversampled smooth function of (theta, phi, rho): the truncated
    # windowed sinc is accurate to the level the paper's trade-off implies
    n_phi, n_th, n_r = 64, 32, 64
    phi, th, th0, dth, rho = _grid(n_phi, n_th, n_r)
    PH, TH, R = np.meshgrid(phi, th, rho, indexing="ij")
    D = _smooth(TH, PH, R).reshape(-1)
    rng = np.random.default_rng(5)
    tq = rng.uniform(th0 + J * dth, th0 + (n_th - 1 - J) * dth, 1500)
    pq = rng.uniform(0, 2 * math.pi, 1500)
    rq = rng.uniform(-20, 20, 1500)
    got = umbrella.resample(D, n_phi, th0, dth, n_th, n_r, tq, pq, rq, J)
    want = _smooth(tq, pq, rq)
    assert np.max(np.abs(got - want)) < tol * np.max(np.abs(want))


def _gauss_dradon(rho, n, c, cov):
    s2 = n @ cov @ n
    mass = (2 * math.pi) ** 1.5 * math.sqrt(np.linalg.det(cov))
    R = mass * np.exp(-(rho - n @ c) ** 2 / (2 * s2)) / math.sqrt(2 * math.pi * s2)
    return -(rho - n @ c) / s2 * R


def test_gaussian_umbrella_values():
    # closed-form derivative-Radon values of a Gaussian on the radial grid,
    # resampled onto umbrella planes, against the closed form on those planes
    N = 16
    n_phi, n_th, n_r = 96, 48, 2 * N
    phi, th, th0, dth, rho = _grid(n_phi, n_th, n_r)
    c = np.array([0.5, -0.3, 0.4])
    cov = np.diag([2.0, 2.4, 2.2]) ** 2
    dirs = synthetic.line_directions(phi, th)
    D = np.stack([_gauss_dradon(rho, n, c, cov) for n in dirs]).reshape(-1)
    nh, rq = umbrella.geometry(N, 6, 8, 8)
    tq, pq = umbrella.angles(nh)
    J = 6
    inside = (tq > th0 + J * dth) & (tq < th0 + (n_th - 1 - J) * dth) & (np.abs(rq) < n_r / 2 - J)
    assert inside.sum() > 100
    got = umbrella.resample(D, n_phi, th0, dth, n_th, n_r, tq[inside], pq[inside], rq[inside], J)
    want = np.array([_gauss_dradon(r, n, c, cov) for r, n in zip(rq[inside], nh[inside])])
    assert np.max(np.abs(got - want)) < 2e-3 * np.max(np.abs(D))


def test_detects_shifted_theta_origin(monkeypatch):
    # a plausible slip (theta indexed from 0 instead of theta_0) breaks the pins
    n_phi, n_th, n_r = 12, 9, 16
    phi, th, th0, dth, rho = _grid(n_phi, n_th, n_r)
    rng = np.random.default_rng(3)
    D = rng.standard_normal(n_phi * n_th * n_r) + 0j
    a, b, j = 3, 4, 8
    good = umbrella.resample(D, n_phi, th0, dth, n_th, n_r, th[[b]], phi[[a]], rho[[j]].astype(float), 6)
    bad = umbrella.resample(D, n_phi, 0.0, dth, n_th, n_r, th[[b]], phi[[a]], rho[[j]].astype(float), 6)
    want = D.reshape(n_phi, n_th, n_r)[a, b, j]
    assert abs(good[0] - want) < 1e-13 and abs(bad[0] - want) > 1e-3

"""Pins for the method-1 resampling oracle (oracle.resample1, Section 2.1.3,
eq 2.8-2.11): the ideal interpolator against closed forms, the NUFFT steps
against the pinned cubic NUFFT and the ideal interpolator, axis symmetry, and
derivative-Radon values of Gaussians on umbrella planes."""
import math

import numpy as np
import pytest

import synthetic
from oracle import nufft, resample1, umbrella

SHAPE = (12, 8, 16)   # non-cubic, so that an axis mix-up shows


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _nodes(shape):
    return np.stack(np.meshgrid(*[np.arange(n) for n in shape], indexing="ij"), -1).reshape(-1, 3)


def test_exact_reproduces_the_samples():
    D = _rand(SHAPE, 1)
    got = resample1.exact(D, _nodes(SHAPE))
    assert np.max(np.abs(got - D.reshape(-1))) < 1e-13


@pytest.mark.parametrize("k", [(0, 0, 0), (-6, 3, -8), (5, -4, 7), (-1, 1, 2)])
def test_exact_band_limited_exponentials(k):
    # samples of exp(-2 pi i k.t/N) with k in the centred band (the Nyquist
    # frequencies -N/2 included) are interpolated to that function everywhere
    N = np.array(SHAPE, dtype=float)
    k = np.array(k, dtype=float)
    D = np.exp(-2j * math.pi * (_nodes(SHAPE) @ (k / N))).reshape(SHAPE)
    t = np.random.default_rng(2).uniform(-5, 25, (300, 3))
    want = np.exp(-2j * math.pi * (t @ (k / N)))
    assert np.max(np.abs(resample1.exact(D, t) - want)) < 1e-12


def test_exact_is_the_periodic_sinc_of_eq_2_7():
    # a unit sample at n0: per axis the kernel of eq 2.6-2.7 over the centred
    # band, exp(+i pi s/N) sin(pi s) / (N sin(pi s / N)), s = t - n0
    n0 = (3, 5, 11)
    D = np.zeros(SHAPE, dtype=complex)
    D[n0] = 1.0
    t = np.random.default_rng(3).uniform(-4, 20, (200, 3))
    want = np.ones(len(t), dtype=complex)
    for d, N in enumerate(SHAPE):
        s = t[:, d] - n0[d]
        want *= np.exp(1j * math.pi * s / N) * np.sin(math.pi * s) / (N * np.sin(math.pi * s / N))
    assert np.max(np.abs(resample1.exact(D, t) - want)) < 1e-13


@pytest.mark.parametrize("J", [4, 6])
def test_nufft_steps_equal_the_cubic_nufft(J):
    # on a cubic grid, P, F and T_sparse of eq 2.11 are the projector's NUFFT of
    # the centred spectrum at omega = 2 pi t / N (a separately pinned oracle)
    N = 12
    D = _rand((N, N, N), 4)
    t = np.random.default_rng(5).uniform(-3, 15, (400, 3))
    got = resample1.nufft_steps(D, t, J)
    want = nufft.forward(resample1.centred_spectrum(D), 2 * math.pi * t / N, nufft.Params(N, 2 * N, J))
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))


def test_axis_permutation():
    # relabelling the axes relabels the coordinates: no axis may borrow
    # another's length, scaling or oversampled size
    D = _rand(SHAPE, 6)
    t = np.random.default_rng(7).uniform(-2, 18, (300, 3))
    a = resample1.nufft_steps(D, t, 6)
    for perm in [(1, 2, 0), (2, 0, 1), (0, 2, 1)]:
        b = resample1.nufft_steps(D.transpose(perm), t[:, perm], 6)
        assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(a))


@pytest.mark.parametrize("J,tol", [(4, 3e-3), (6, 5e-5), (8, 1e-6)])
def test_nufft_steps_approach_the_ideal_interpolator(J, tol):
    # eq 2.11 approximates eq 2.8 to the accuracy of the oversampled KB NUFFT,
    # which falls by about two decades per two taps
    D = _rand(SHAPE, 8)
    t = np.random.default_rng(9).uniform(-3, 20, (500, 3))
    ex = resample1.exact(D, t)
    got = resample1.nufft_steps(D, t, J)
    assert np.linalg.norm(got - ex) / np.linalg.norm(ex) < tol


def test_nufft_steps_on_band_limited_exponentials():
    N = np.array(SHAPE, dtype=float)
    t = np.random.default_rng(10).uniform(-5, 25, (300, 3))
    for k in [(-6, 3, -8), (2, -1, 5)]:
        k = np.array(k, dtype=float)
        D = np.exp(-2j * math.pi * (_nodes(SHAPE) @ (k / N))).reshape(SHAPE)
        want = np.exp(-2j * math.pi * (t @ (k / N)))
        assert np.max(np.abs(resample1.nufft_steps(D, t, 6) - want)) < 2e-4


def _gauss_dradon(rho, n, c, cov):
    s2 = n @ cov @ n
    mass = (2 * math.pi) ** 1.5 * math.sqrt(np.linalg.det(cov))
    R = mass * np.exp(-(rho - n @ c) ** 2 / (2 * s2)) / math.sqrt(2 * math.pi * s2)
    return -(rho - n @ c) / s2 * R


def _radial_gaussian(N, n_phi, n_th, c, cov):
    n_r = 2 * N
    phi = synthetic.azimuths(n_phi)
    th = synthetic.polar_angles(n_th)
    rho = np.arange(n_r) - n_r // 2
    dirs = synthetic.line_directions(phi, th)
    D = np.stack([_gauss_dradon(rho, n, c, cov) for n in dirs]).reshape(-1)
    return D, th[0], th[1] - th[0], n_r


def test_isotropic_gaussian_on_all_umbrella_planes():
    # a centred isotropic Gaussian has the same derivative-Radon profile on
    # every line, so every axis of the index space is periodic and smooth and
    # method 1 is accurate on every plane, the polar caps included
    N, n_phi, n_th = 16, 32, 16
    cov = np.eye(3) * 2.2 ** 2
    c = np.zeros(3)
    D, th0, dth, n_r = _radial_gaussian(N, n_phi, n_th, c, cov)
    nh, rq = umbrella.geometry(N, 6, 8, 8)
    tq, pq = umbrella.angles(nh)
    got = resample1.resample(D, n_phi, th0, dth, n_th, n_r, tq, pq, rq, 6)
    want = np.array([_gauss_dradon(r, n, c, cov) for r, n in zip(rq, nh)])
    assert np.max(np.abs(got - want)) < 1e-4 * np.max(np.abs(D))


def test_gaussian_umbrella_values_inside_the_sampled_caps():
    # an off-centre anisotropic Gaussian: the theta axis is not periodic, and
    # inside the sampled range the error stays at the level the periodic
    # extension's jump allows
    N, n_phi, n_th = 16, 96, 48
    c = np.array([0.5, -0.3, 0.4])
    cov = np.diag([2.0, 2.4, 2.2]) ** 2
    D, th0, dth, n_r = _radial_gaussian(N, n_phi, n_th, c, cov)
    nh, rq = umbrella.geometry(N, 6, 8, 8)
    tq, pq = umbrella.angles(nh)
    inside = (tq > th0 + 6 * dth) & (tq < th0 + (n_th - 7) * dth)
    assert inside.sum() > 100
    want = np.array([_gauss_dradon(r, n, c, cov) for r, n in zip(rq[inside], nh[inside])])
    for J in (3, 6):
        got = resample1.resample(D, n_phi, th0, dth, n_th, n_r, tq[inside], pq[inside], rq[inside], J)
        assert np.max(np.abs(got - want)) < 1e-2 * np.max(np.abs(D))


def test_detects_uncentred_band(monkeypatch):
    # the band 0..N-1 of eq 2.2 taken literally (no centring) fails the
    # exponential pin between the samples
    monkeypatch.setattr(resample1, "centred_spectrum",
                        lambda D: np.fft.ifftn(np.asarray(D, dtype=complex)))
    N = np.array(SHAPE, dtype=float)
    k = np.array([-6, 3, -8], dtype=float)
    D = np.exp(-2j * math.pi * (_nodes(SHAPE) @ (k / N))).reshape(SHAPE)
    t = np.random.default_rng(2).uniform(-5, 25, (50, 3))
    want = np.exp(-2j * math.pi * (t @ (k / N)))
    assert np.max(np.abs(resample1.exact(D, t) - want)) > 1e-2


def _approx_err():
    D = _rand(SHAPE, 6)
    t = np.random.default_rng(7).uniform(-2, 18, (200, 3))
    ex = resample1.exact(D, t)
    return np.linalg.norm(resample1.nufft_steps(D, t, 6) - ex) / np.linalg.norm(ex)


def test_detects_missing_scaling(monkeypatch):
    from oracle import kernels
    assert _approx_err() < 5e-5
    monkeypatch.setattr(kernels, "deapod", lambda N, K, J, beta: np.ones(N))
    assert _approx_err() > 1e-3


def test_detects_unscaled_grid_coordinate(monkeypatch):
    # taps placed at t instead of t K/N on the oversampled grid
    orig = resample1.taps
    monkeypatch.setattr(resample1, "taps", lambda tg, J, beta: orig(0.5 * tg, J, beta))
    assert _approx_err() > 1e-1

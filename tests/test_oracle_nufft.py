"""Pins for the straightforward NUFFT (oracle.nufft) against the exact NUDFT."""
import math

import numpy as np
import pytest

import synthetic
from oracle import kernels, nudft, nufft


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _rand_vol(rng, N):
    return rng.standard_normal((N, N, N)) + 1j * rng.standard_normal((N, N, N))


@pytest.mark.parametrize("kernel", ["kb", "minmax"])
def test_error_falls_with_width(rng, kernel):
    # accuracy against the exact NUDFT improves steeply with J at K = 2N;
    # a wrong sign, tap index or transposed axis gives O(1) error instead
    N, K = 12, 24
    x = _rand_vol(rng, N)
    om = rng.uniform(-math.pi, math.pi, (400, 3))
    ex = nudft.nudft3(x, om)
    errs = [_rel(nufft.forward(x, om, nufft.Params(N, K, J, kernel)), ex) for J in (4, 6, 8)]
    assert errs[0] < 2e-3 and errs[1] < 3e-5 and errs[2] < 5e-7
    assert errs[0] > 10 * errs[1] > 100 * errs[2]


def test_dirichlet_exact_at_full_width(rng):
    # J = K = N, uniform scaling, min-max: the periodic-sinc resampler of eq 2.2-2.7
    N = 8
    x = _rand_vol(rng, N)
    om = rng.uniform(-math.pi, math.pi, (200, 3))
    got = nufft.forward(x, om, nufft.Params(N, N, N, "minmax", scaling="uniform"))
    assert _rel(got, nudft.nudft3(x, om)) < 1e-12


def _error_bound(om, prm):
    """E(omega) = || a - b ||_2 over m in [-N/2,N/2)^3 where a = exp(-i omega.m) and
    b = s(m) sum_taps w exp(-i gamma kappa.m), via the separable identity
    E^2 = prod |a_d|^2 - 2 Re prod <a_d, b_d> + prod |b_d|^2."""
    N, K = prm.N, prm.K
    gamma = 2 * math.pi / K
    m = np.arange(N) - N // 2
    na = np.ones(len(om))
    ab = np.ones(len(om), complex)
    nb = np.ones(len(om))
    for d in range(3):
        kap, w = prm.axis_weights(om[:, d])
        a = np.exp(-1j * om[:, d][:, None] * m[None, :])
        b = prm.s[None, :] * np.einsum("pj,pjm->pm", w, np.exp(-1j * gamma * kap[:, :, None] * m[None, None, :]))
        na *= np.sum(np.abs(a) ** 2, 1)
        nb *= np.sum(np.abs(b) ** 2, 1)
        ab *= np.sum(np.conj(a) * b, 1)
    return np.sqrt(np.maximum(na - 2 * ab.real + nb, 0))


@pytest.mark.parametrize("kernel,J", [("kb", 4), ("kb", 6), ("minmax", 6)])
def test_per_point_bound(rng, kernel, J):
    # |X^(omega) - X(omega)| <= E(omega) ||x||_2 (Cauchy-Schwarz; exact for any weights)
    N, K = 12, 24
    prm = nufft.Params(N, K, J, kernel)
    x = _rand_vol(rng, N)
    om = rng.uniform(-math.pi, math.pi, (300, 3))
    err = np.abs(nufft.forward(x, om, prm) - nudft.nudft3(x, om))
    Eom = _error_bound(om, prm)
    E = Eom * np.linalg.norm(x)
    assert np.all(err <= E * (1 + 1e-9) + 1e-12)
    # the bound is small relative to || a || = N^{3/2} (the kernel is accurate)
    assert np.max(Eom) / N ** 1.5 < (3e-3 if J == 4 else 5e-5)


def test_on_grid_points_equal_fft(rng):
    # eq 2.12: a NUFFT at on-grid points 2 pi k/N is the FFT (within the bound)
    N, K, J = 8, 16, 6
    prm = nufft.Params(N, K, J)
    x = _rand_vol(rng, N)
    k = rng.integers(0, N, size=(60, 3))
    om = 2 * math.pi * k / N
    want = np.fft.fftn(x)[k[:, 0], k[:, 1], k[:, 2]] * (-1.0) ** k.sum(1)
    assert _rel(nufft.forward(x, om, prm), want) < 5e-5


def test_transpose_dot_product(rng):
    N, K, J = 10, 20, 6
    for kernel in ("kb", "minmax"):
        prm = nufft.Params(N, K, J, kernel)
        om = rng.uniform(-math.pi, math.pi, (333, 3))
        x = _rand_vol(rng, N)
        y = rng.standard_normal(333) + 1j * rng.standard_normal(333)
        lhs = np.vdot(y, nufft.forward(x, om, prm))
        rhs = np.vdot(nufft.adjoint(y, om, prm), x)
        assert abs(lhs - rhs) / abs(lhs) < 1e-12


def test_transpose_close_to_exact_adjoint(rng):
    # eq 2.13 direction: the NUFFT transpose approximates the adjoint NUDFT
    N, K, J = 10, 20, 6
    prm = nufft.Params(N, K, J)
    om = rng.uniform(-math.pi, math.pi, (500, 3))
    y = rng.standard_normal(500) + 1j * rng.standard_normal(500)
    assert _rel(nufft.adjoint(y, om, prm), nudft.nudft3_adjoint(y, om, N)) < 3e-5


def test_real_input_hermitian_symmetry(rng):
    # real x: X(-omega) = conj X(omega), away from neighbour-rule ties
    N, K, J = 12, 24, 6
    prm = nufft.Params(N, K, J)
    x = rng.standard_normal((N, N, N))
    om = rng.uniform(-math.pi, math.pi, (200, 3))
    a = nufft.forward(x, om, prm)
    b = nufft.forward(x, -om, prm)
    assert np.max(np.abs(a - np.conj(b))) < 1e-12 * np.max(np.abs(a))


def test_ellipsoid_phantom_analytic_transform():
    # loose sanity of the phantom scale: voxelised ellipsoids vs their continuous FT
    # F(k) = rho abc e^{-ik.c} 4 pi (sin q - q cos q)/q^3, q = |D R^T k|, X ~ F(omega/h)/h^3
    N = 32
    h = 2.0 / N
    rng = np.random.default_rng(1000)
    ells = synthetic.random_ellipsoids(rng, 8)
    x = synthetic.voxelize(ells, N)
    om = synthetic.radial_points(synthetic.line_directions(synthetic.azimuths(8),
                                                           synthetic.polar_angles(4)), 32)
    om = om[np.linalg.norm(om, axis=1) < 0.6 * math.pi]
    k = om / h
    F = np.zeros(len(k), complex)
    for e in ells:
        q = np.linalg.norm((k @ e.rot) * e.axes[None, :], axis=1)
        with np.errstate(invalid="ignore", divide="ignore"):
            g = np.where(q < 1e-2, 4 * math.pi * (1 / 3 - q ** 2 / 30 + q ** 4 / 840),
                         4 * math.pi * (np.sin(q) - q * np.cos(q)) / q ** 3)
        F += e.density * np.prod(e.axes) * np.exp(-1j * k @ e.center) * g
    X = nudft.nudft3(x, om) * h ** 3
    # voxel centres sit at u = (n - N/2) h, matching the centring m = n - N/2
    assert _rel(X, F) < 8e-2


def test_kernel_weights_sum_near_partition_of_unity():
    # sum_kappa psi(t - kappa) is ~ Psi(0) for any t (Poisson summation; KB decay)
    J, beta = 6, kernels.default_beta(6)
    K = 32
    t = np.linspace(-5, 5, 37)
    kap, u = kernels.neighbours(t * 2 * math.pi / K, K, J)
    tot = kernels.kb_psi(u, J, beta).sum(1)
    assert np.allclose(tot, kernels.kb_psi_hat(np.array([0.0]), J, beta)[0], rtol=1e-3)

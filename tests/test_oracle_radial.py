"""Pins for the radial derivative stage (oracle.radial) and the projector."""
import math

import numpy as np
import pytest

import synthetic
from oracle import nudft, nufft, projector, radial


def test_directions_follow_polar_map():
    phi = synthetic.azimuths(6)
    th = synthetic.polar_angles(5)
    d_or = radial.directions(phi, th)
    d_in = synthetic.line_directions(phi, th)
    assert np.max(np.abs(d_or - d_in)) < 1e-15
    assert np.allclose(np.linalg.norm(d_in, axis=1), 1.0, atol=1e-15)
    # first line: phi = 0, theta = 0.2 -> (sin 0.2, 0, cos 0.2)
    assert np.allclose(d_in[0], [math.sin(0.2), 0.0, math.cos(0.2)], atol=0)


def test_r_grid_and_idft_equal_shifted_ifft(rng):
    n_r = 16
    r = radial.r_grid(n_r)
    assert r[0] == -math.pi and r[n_r // 2] == 0.0
    G = rng.standard_normal(3 * n_r) + 1j * rng.standard_normal(3 * n_r)
    D = radial.forward(G, n_r, deriv=False).reshape(3, n_r)
    want = np.fft.fftshift(np.fft.ifft(np.fft.ifftshift(G.reshape(3, n_r), axes=1), axis=1), axes=1)
    assert np.max(np.abs(D - want)) < 1e-14


def test_axis_fourier_slice_is_plane_sum(rng):
    # line along e_z, no derivative: the radial inverse DFT of exact transform samples
    # gives the plane sums sum_{n0,n1} x[n0,n1,n2] at rho = n2 - N/2 (Fourier slice theorem)
    N, n_r = 8, 16
    x = rng.standard_normal((N, N, N))
    dirs = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    D = projector.forward(x, dirs, n_r, None, deriv=False, exact=True).reshape(2, n_r)
    rho = radial.rho_grid(n_r)
    inside = (rho >= -N // 2) & (rho < N // 2)
    want_z = np.zeros(n_r)
    want_z[inside] = x.sum(axis=(0, 1))
    want_x = np.zeros(n_r)
    want_x[inside] = x.sum(axis=(1, 2))
    assert np.max(np.abs(D[0] - want_z)) < 1e-12
    assert np.max(np.abs(D[1] - want_x)) < 1e-12


def _gauss_radon_deriv(rho, n, c, cov, amp):
    s2 = n @ cov @ n
    mass = amp * (2 * math.pi) ** 1.5 * math.sqrt(np.linalg.det(cov))
    R = mass * np.exp(-(rho - n @ c) ** 2 / (2 * s2)) / math.sqrt(2 * math.pi * s2)
    return -(rho - n @ c) / s2 * R, R


@pytest.mark.parametrize("exact", [True, False])
def test_gaussian_derivative_radon(rng, exact):
    # a Gaussian blob's Radon transform along nhat is a 1D Gaussian with variance
    # nhat^T C nhat; the radial stage with derivative must return its rho-derivative
    N, n_r = 40, 80
    c = np.array([1.0, -1.0, 0.5])
    A = rng.standard_normal((3, 3))
    cov = np.diag([4.0, 5.5, 6.5]) + 0.3 * (A @ A.T) / 3
    x = synthetic.gaussian_blob(N, c, cov)
    dirs = synthetic.line_directions(synthetic.azimuths(5), synthetic.polar_angles(3))
    prm = None if exact else nufft.Params(N, 2 * N, 6)
    D = projector.forward(x, dirs, n_r, prm, deriv=True, exact=exact).reshape(len(dirs), n_r)
    P = projector.forward(x, dirs, n_r, prm, deriv=False, exact=exact).reshape(len(dirs), n_r)
    rho = radial.rho_grid(n_r)
    for l, nh in enumerate(dirs):
        dR, R = _gauss_radon_deriv(rho, nh, c, cov, 1.0)
        tol = 1e-7 if exact else 1e-4
        assert np.max(np.abs(D[l] - dR)) < tol * np.max(np.abs(dR)), l
        assert np.max(np.abs(P[l] - R)) < tol * np.max(np.abs(R)), l
        # the NUFFT's neighbour-rule ties (the r = 0 sample; the phi = 0 line, where
        # omega_1 = 0 exactly) break Hermitian symmetry at about psi(J/2) = 1/I0(beta)
        assert np.max(np.abs(D[l].imag)) < (1e-9 if exact else 2e-5) * np.max(np.abs(dR))


def test_per_line_parseval(rng):
    n_r = 32
    G = rng.standard_normal(4 * n_r) + 1j * rng.standard_normal(4 * n_r)
    D = radial.forward(G, n_r).reshape(4, n_r)
    f = radial.deriv_factor(n_r)
    lhs = np.sum(np.abs(D) ** 2, 1)
    rhs = np.sum(np.abs(G.reshape(4, n_r) * f) ** 2, 1) / n_r
    assert np.allclose(lhs, rhs, rtol=1e-13)
    assert f[0] == 0 and f[n_r // 2] == 0 and f[1] == pytest.approx(1j * (-math.pi + 2 * math.pi / n_r))


def test_radial_adjoint(rng):
    n_r = 24
    G = rng.standard_normal(5 * n_r) + 1j * rng.standard_normal(5 * n_r)
    d = rng.standard_normal(5 * n_r) + 1j * rng.standard_normal(5 * n_r)
    for deriv in (True, False):
        lhs = np.vdot(d, radial.forward(G, n_r, deriv))
        rhs = np.vdot(radial.adjoint(d, n_r, deriv), G)
        assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_real_volume_gives_real_derivative_radon(rng):
    N, n_r = 16, 32
    x = rng.standard_normal((N, N, N))
    dirs = synthetic.line_directions(synthetic.azimuths(4) + 0.1, synthetic.polar_angles(3) + 0.05)
    D = projector.forward(x, dirs, n_r, nufft.Params(N, 2 * N, 6))
    assert np.max(np.abs(D.imag)) < 1e-12 * np.max(np.abs(D))


def test_projector_dot_and_nudft_agreement(rng):
    N, n_r = 12, 24
    prm = nufft.Params(N, 24, 6)
    dirs = synthetic.line_directions(synthetic.azimuths(6), synthetic.polar_angles(4))
    x = rng.standard_normal((N, N, N)) + 1j * rng.standard_normal((N, N, N))
    y = rng.standard_normal(len(dirs) * n_r) + 1j * rng.standard_normal(len(dirs) * n_r)
    Ax = projector.forward(x, dirs, n_r, prm)
    lhs = np.vdot(y, Ax)
    rhs = np.vdot(projector.adjoint(y, dirs, n_r, prm), x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    Ax_exact = projector.forward(x, dirs, n_r, None, exact=True)
    assert np.linalg.norm(Ax - Ax_exact) / np.linalg.norm(Ax_exact) < 5e-5
    adj_exact = projector.adjoint(y, dirs, n_r, None, N=N, exact=True)
    adj = projector.adjoint(y, dirs, n_r, prm)
    assert np.linalg.norm(adj - adj_exact) / np.linalg.norm(adj_exact) < 5e-5

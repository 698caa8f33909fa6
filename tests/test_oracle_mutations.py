"""Planted mistakes in the oracle must be caught by its pins.

Each case patches one plausible mistake into the oracle (on the CPU only) and
checks that the corresponding pin detects it.
"""
import math

import numpy as np
import pytest

from oracle import kernels, nudft, nufft, projector, radial
import synthetic


def _nufft_vs_nudft(J=6):
    rng = np.random.default_rng(7)
    N, K = 10, 20
    x = rng.standard_normal((N, N, N)) + 1j * rng.standard_normal((N, N, N))
    om = rng.uniform(-math.pi, math.pi, (200, 3))
    a = nufft.forward(x, om, nufft.Params(N, K, J))
    b = nudft.nudft3(x, om)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _gauss_deriv_err():
    N, n_r = 24, 48
    c = np.array([0.5, -0.5, 0.25])
    cov = np.diag([3.0, 3.5, 4.0])
    x = synthetic.gaussian_blob(N, c, cov)
    dirs = synthetic.line_directions(np.array([0.3, 1.9]), np.array([0.7, 2.0]))
    D = projector.forward(x, dirs, n_r, None, exact=True).reshape(len(dirs), n_r)
    rho = np.arange(n_r) - n_r // 2.0  # written out here, independent of the oracle
    worst = 0.0
    for l, nh in enumerate(dirs):
        s2 = nh @ cov @ nh
        R = (2 * math.pi) ** 1.5 * math.sqrt(np.linalg.det(cov)) * np.exp(-(rho - nh @ c) ** 2 / (2 * s2)) / math.sqrt(2 * math.pi * s2)
        dR = -(rho - nh @ c) / s2 * R
        worst = max(worst, np.max(np.abs(D[l] - dR)) / np.max(np.abs(dR)))
    return worst


def test_unpatched_baselines():
    assert _nufft_vs_nudft() < 3e-5
    assert _gauss_deriv_err() < 1e-6


def test_detects_missing_deapodization(monkeypatch):
    monkeypatch.setattr(kernels, "deapod", lambda N, K, J, beta: np.ones(N))
    assert _nufft_vs_nudft() > 1e-2


def test_detects_wrong_tap_offset(monkeypatch):
    orig = kernels.neighbours

    def shifted(omega_d, K, J):
        kap, u = orig(omega_d, K, J)
        return kap + 1, u  # taps one cell off, offsets unchanged
    monkeypatch.setattr(kernels, "neighbours", shifted)
    assert _nufft_vs_nudft() > 1e-2


def test_detects_transposed_axes(monkeypatch):
    orig = nufft.Params.axis_weights
    calls = {"n": 0}

    def swapped(self, omega_d):
        calls["n"] += 1
        return orig(self, -omega_d if calls["n"] % 3 == 2 else omega_d)  # flip axis 1
    monkeypatch.setattr(nufft.Params, "axis_weights", swapped)
    assert _nufft_vs_nudft() > 1e-2


def test_detects_conjugated_derivative(monkeypatch):
    orig = radial.deriv_factor
    monkeypatch.setattr(radial, "deriv_factor", lambda n_r, deriv=True: np.conj(orig(n_r, deriv)))
    assert _gauss_deriv_err() > 0.5


def test_detects_wrong_radial_centring(monkeypatch):
    orig = radial.rho_grid
    monkeypatch.setattr(radial, "rho_grid", lambda n_r: orig(n_r) + 1)
    assert _gauss_deriv_err() > 1e-2


def test_detects_wrong_kb_shape(monkeypatch):
    orig = kernels.kb_psi_hat
    monkeypatch.setattr(kernels, "kb_psi_hat", lambda f, J, beta: orig(f * 1.05, J, beta))
    assert _nufft_vs_nudft() > 1e-4

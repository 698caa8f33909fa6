"""Pins for the Kaiser-Bessel kernel, its transform, the neighbour rule and min-max."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import kernels


@pytest.mark.parametrize("J", [4, 6, 8])
def test_psi_hat_matches_quadrature(J):
    # the closed-form transform against adaptive quadrature of psi itself,
    # including frequencies past the zero crossing (pi J f > beta)
    beta = kernels.default_beta(J)

    def ft(f):
        val, _ = integrate.quad(lambda u: kernels.kb_psi(u, J, beta) * math.cos(2 * math.pi * f * u),
                                -J / 2, J / 2, limit=200, epsabs=1e-14, epsrel=1e-13)
        return val

    fz = beta / (math.pi * J)
    for f in [0.0, 0.1, 0.25, 0.5, 0.9 * fz, 1.2 * fz, 1.7 * fz]:
        got = float(kernels.kb_psi_hat(np.array([f]), J, beta)[0])
        want = ft(f)
        assert abs(got - want) <= 1e-10 * max(1.0, abs(want)), (f, got, want)


def test_psi_special_values():
    J, beta = 6, kernels.default_beta(6)
    assert kernels.kb_psi(np.array([0.0]), J, beta)[0] == pytest.approx(1.0, abs=1e-15)
    edge = kernels.kb_psi(np.array([-J / 2, J / 2]), J, beta)
    assert edge == pytest.approx([1 / special.i0(beta)] * 2, rel=1e-12)
    u = np.linspace(-2.9, 2.9, 41)
    assert np.allclose(kernels.kb_psi(u, J, beta), kernels.kb_psi(-u, J, beta), rtol=0, atol=1e-15)
    assert kernels.kb_psi(np.array([3.01, -3.2]), J, beta).tolist() == [0.0, 0.0]


def test_deapod_is_reciprocal_transform():
    N, K, J = 16, 32, 6
    beta = kernels.default_beta(J)
    s = kernels.deapod(N, K, J, beta)
    m = np.arange(N) - N // 2
    assert np.allclose(s * kernels.kb_psi_hat(m / K, J, beta), 1.0, atol=1e-14)
    assert np.allclose(s[1:], s[1:][::-1], rtol=0, atol=0)  # s(m) = s(-m)


def test_neighbour_rule():
    K, J = 16, 6
    gamma = 2 * math.pi / K
    om = np.array([0.0, 0.37 * gamma, -2.5 * gamma, 7.9 * gamma, -8 * gamma])
    kap, u = kernels.neighbours(om, K, J)
    t = om / gamma
    for p in range(len(om)):
        k0 = math.floor(t[p] - J / 2)
        assert kap[p].tolist() == list(range(k0 + 1, k0 + J + 1))
        assert np.all(u[p] >= -J / 2) and np.all(u[p] < J / 2)
        assert np.allclose(u[p], t[p] - kap[p], atol=0)
    # the tie at t = 0: taps -2..3, offset -3 at the last tap
    assert kap[0].tolist() == [-2, -1, 0, 1, 2, 3]


def test_neighbour_offsets_stay_in_support_when_s_rounds():
    """Where s = t - J/2 rounds onto an integer (t just beyond a negative
    integer, where t - J/2 enters a coarser binade), the taps follow the
    rounded s and so must the offsets: all J of them inside [-J/2, J/2), so
    that no tap's weight falls off the kernel's support (psi = 0 there)."""
    K, J = 192, 6
    gamma = 2 * math.pi / K
    ts = np.array([-3.0000000000000004, -2.0000000000000004, -1.0000000000000002,
                   -5.000000000000001, -3.9999999999999996])
    kap, u = kernels.neighbours(ts * gamma, K, J)
    t = (ts * gamma) / gamma
    for p in range(len(ts)):
        s = t[p] - J / 2
        assert kap[p].tolist() == list(range(int(math.floor(s)) + 1, int(math.floor(s)) + J + 1))
        assert np.all(u[p] >= -J / 2) and np.all(u[p] < J / 2), (ts[p], u[p])
        assert np.all(kernels.kb_psi(u[p], J, kernels.default_beta(J)) > 0)
    # the first case rounds: s = -6 exactly although t - 3 < -6
    assert t[0] - 3 == -6.0 and t[0] < -3.0


def test_minmax_reproduces_exponential_at_uniform_full_width(rng):
    # J = K = N with s = 1: the fit is exact (periodic sinc interpolation, eq 2.2-2.7)
    N = K = J = 8
    s = np.ones(N)
    om = rng.uniform(-math.pi, math.pi, 20)
    kap, u = kernels.neighbours(om, K, J)
    c = kernels.minmax_coeffs(u, N, K, s)
    m = np.arange(N) - N // 2
    approx = np.einsum("pj,pjm->pm", c, np.exp(-1j * (2 * math.pi / K) * kap[:, :, None] * m[None, None, :]))
    exact = np.exp(-1j * om[:, None] * m[None, :])
    assert np.max(np.abs(approx - exact)) < 1e-12


def test_minmax_is_least_squares_optimum(rng):
    # perturbing the min-max coefficients can only increase || a - B c ||
    N, K, J = 16, 32, 4
    s = kernels.deapod(N, K, J, kernels.default_beta(J))
    om = rng.uniform(-math.pi, math.pi, 5)
    kap, u = kernels.neighbours(om, K, J)
    c = kernels.minmax_coeffs(u, N, K, s)
    m = np.arange(N) - N // 2
    gamma = 2 * math.pi / K
    for p in range(5):
        B = s[:, None] * np.exp(-1j * gamma * m[:, None] * kap[p][None, :])
        a = np.exp(-1j * om[p] * m)
        e0 = np.linalg.norm(a - B @ c[p])
        for _ in range(5):
            d = 1e-3 * (rng.standard_normal(J) + 1j * rng.standard_normal(J))
            assert np.linalg.norm(a - B @ (c[p] + d)) >= e0
        # and the normal equations hold
        assert np.linalg.norm(B.conj().T @ (a - B @ c[p])) < 1e-10 * np.linalg.norm(a)

"""Pins for the exact NUDFT (oracle.nudft) against closed forms and textbook FFTs."""
import math

import numpy as np
import pytest

from oracle import nudft

pytestmark = pytest.mark.filterwarnings("ignore")


def test_delta_is_pure_phase(rng):
    # a single voxel at n0 gives exp(-i omega . (n0 - N/2)): pins sign and centring
    N = 8
    n0 = np.array([1, 6, 3])
    x = np.zeros((N, N, N))
    x[tuple(n0)] = 1.0
    om = rng.uniform(-math.pi, math.pi, (50, 3))
    got = nudft.nudft3(x, om)
    want = np.exp(-1j * om @ (n0 - N // 2))
    assert np.max(np.abs(got - want)) < 1e-13


def test_on_grid_equals_centred_fft(rng):
    # omega on the N-grid (2 pi k / N) is the textbook DFT with centring:
    # X(2 pi k/N) = sum_n x[n] exp(-2 pi i k (n - N/2)/N) = (-1)^{k.1} fftn(x)[k]
    N = 8
    x = rng.standard_normal((N, N, N)) + 1j * rng.standard_normal((N, N, N))
    F = np.fft.fftn(x)
    k = rng.integers(0, N, size=(40, 3))
    om = 2 * math.pi * k / N
    got = nudft.nudft3(x, om)
    want = F[k[:, 0], k[:, 1], k[:, 2]] * (-1.0) ** k.sum(axis=1)
    assert np.max(np.abs(got - want)) / np.max(np.abs(want)) < 1e-13


def test_separable_geometric_closed_form(rng):
    # x[n] = a^n0 b^n1 c^n2 (distinct per axis: pins the axis pairing)
    N = 10
    a, b, c = 0.9 * np.exp(0.3j), 0.7 * np.exp(-1.1j), 1.1 * np.exp(0.5j)
    n = np.arange(N)
    x = (a ** n)[:, None, None] * (b ** n)[None, :, None] * (c ** n)[None, None, :]
    om = rng.uniform(-math.pi, math.pi, (30, 3))

    def geo(z, w):
        # sum_n z^n exp(-i w (n - N/2)) = exp(i w N/2) (1 - q^N)/(1 - q), q = z e^{-iw}
        q = z * np.exp(-1j * w)
        return np.exp(1j * w * N / 2) * (1 - q ** N) / (1 - q)

    want = geo(a, om[:, 0]) * geo(b, om[:, 1]) * geo(c, om[:, 2])
    got = nudft.nudft3(x, om)
    assert np.max(np.abs(got - want)) / np.max(np.abs(want)) < 1e-12


def test_parseval_on_grid(rng):
    N = 6
    x = rng.standard_normal((N, N, N)) + 1j * rng.standard_normal((N, N, N))
    k = np.stack(np.meshgrid(*[np.arange(N)] * 3, indexing="ij"), -1).reshape(-1, 3)
    X = nudft.nudft3(x, 2 * math.pi * k / N)
    assert abs(np.sum(np.abs(X) ** 2) - N ** 3 * np.sum(np.abs(x) ** 2)) < 1e-10 * np.sum(np.abs(X) ** 2)


def test_adjoint_dot_and_columns(rng):
    N = 8
    om = rng.uniform(-math.pi, math.pi, (64, 3))
    x = rng.standard_normal((N, N, N)) + 1j * rng.standard_normal((N, N, N))
    y = rng.standard_normal(64) + 1j * rng.standard_normal(64)
    lhs = np.vdot(y, nudft.nudft3(x, om))
    rhs = np.vdot(nudft.nudft3_adjoint(y, om, N), x)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13
    # column p of the adjoint is exp(+i omega_p . m)
    e = np.zeros(64, complex)
    e[5] = 1.0
    col = nudft.nudft3_adjoint(e, om, N)
    m = np.arange(N) - N // 2
    want = np.exp(1j * (om[5, 0] * m[:, None, None] + om[5, 1] * m[None, :, None] + om[5, 2] * m[None, None, :]))
    assert np.max(np.abs(col - want)) < 1e-13
    # sampled evaluation agrees with the full adjoint
    vox = np.array([[0, 0, 0], [3, 7, 1], [7, 7, 7]])
    full = nudft.nudft3_adjoint(y, om, N)
    part = nudft.nudft3_adjoint_at(y, om, N, vox)
    assert np.max(np.abs(part - full[vox[:, 0], vox[:, 1], vox[:, 2]])) < 1e-12

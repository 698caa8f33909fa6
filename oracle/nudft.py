"""Exact non-uniform DFT (the plain definition the NUFFT approximates).

TEST INFRASTRUCTURE (oracle).  FP64.

Section 2.1.2, eq 2.3 writes the 1D non-uniform DFT y(m) = sum_n x(n) e^{-j 2 pi m n / N};
the 3D form used here, with the volume centred at voxel N/2 and frequencies in
radians per voxel, is

    X(omega) = sum_{n in [0,N)^3} x[n] exp(-i omega . (n - N/2)).

The sum over n0, n1, n2 factors into three 1D sums of directly computed
exponentials (exact algebra, no approximation), which keeps the cost at
M * N^3 complex multiply-adds executed as dense products.
"""
from __future__ import annotations

import numpy as np


def _phase_rows(omega_d: np.ndarray, N: int, sign: float) -> np.ndarray:
    """E[p, n] = exp(sign * i * omega_d[p] * (n - N/2))."""
    m = np.arange(N, dtype=np.float64) - N // 2
    return np.exp(sign * 1j * np.outer(omega_d, m))


def nudft3(x: np.ndarray, omega: np.ndarray, chunk: int = 2048) -> np.ndarray:
    """X(omega_p) = sum_n x[n] exp(-i omega_p . m) for all rows of omega (M, 3)."""
    x = np.asarray(x, dtype=np.complex128)
    N = x.shape[0]
    assert x.shape == (N, N, N)
    omega = np.asarray(omega, dtype=np.float64).reshape(-1, 3)
    out = np.empty(omega.shape[0], dtype=np.complex128)
    for s in range(0, omega.shape[0], chunk):
        w = omega[s:s + chunk]
        e0 = _phase_rows(w[:, 0], N, -1.0)
        e1 = _phase_rows(w[:, 1], N, -1.0)
        e2 = _phase_rows(w[:, 2], N, -1.0)
        # sum over n2 first: t[p, a, b] = sum_c e2[p, c] x[a, b, c]
        t = np.einsum("pc,abc->pab", e2, x, optimize=True)
        t = np.einsum("pb,pab->pa", e1, t, optimize=True)
        out[s:s + chunk] = np.einsum("pa,pa->p", e0, t)
    return out


def nudft3_adjoint(g: np.ndarray, omega: np.ndarray, N: int, chunk: int = 2048) -> np.ndarray:
    """Conjugate transpose of nudft3: x~[n] = sum_p exp(+i omega_p . m) g[p]."""
    g = np.asarray(g, dtype=np.complex128).reshape(-1)
    omega = np.asarray(omega, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((N, N, N), dtype=np.complex128)
    for s in range(0, omega.shape[0], chunk):
        w = omega[s:s + chunk]
        e0 = _phase_rows(w[:, 0], N, +1.0)
        e1 = _phase_rows(w[:, 1], N, +1.0)
        e2 = _phase_rows(w[:, 2], N, +1.0)
        t = e0 * g[s:s + chunk, None]                      # (p, a)
        t = np.einsum("pa,pb->pab", t, e1, optimize=True)  # (p, a, b)
        out += np.einsum("pab,pc->abc", t, e2, optimize=True)
    return out


def nudft3_adjoint_at(g: np.ndarray, omega: np.ndarray, N: int, voxels: np.ndarray,
                      chunk: int = 1 << 20) -> np.ndarray:
    """Adjoint NUDFT evaluated only at the listed voxels (V, 3) integer indices."""
    g = np.asarray(g, dtype=np.complex128).reshape(-1)
    omega = np.asarray(omega, dtype=np.float64).reshape(-1, 3)
    mv = np.asarray(voxels, dtype=np.float64) - N // 2
    out = np.zeros(len(mv), dtype=np.complex128)
    for s in range(0, omega.shape[0], chunk):
        ph = omega[s:s + chunk] @ mv.T  # (p, v)
        out += np.exp(1j * ph).T @ g[s:s + chunk]
    return out

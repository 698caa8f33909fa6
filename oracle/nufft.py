"""Straightforward oversampled 3D NUFFT and its transpose.

TEST INFRASTRUCTURE (oracle).  FP64.

Follows the factorisation of Section 2.1.3, eq 2.11, x~ = T_sparse F P x:
  1. P: multiply the volume by the separable scaling s(m0) s(m1) s(m2) and
     zero-pad it onto the K^3 grid, voxel m stored at index (m mod K);
  2. F: unnormalised 3D FFT of the padded grid (a library FFT), so that
     Y[kappa mod K] = sum_m s(m) x[m] exp(-i gamma kappa . m);
  3. T_sparse: for every point, the J^3 tensor-product taps of the neighbour
     rule, X(omega) ~= sum_{a,b,c} w0_a w1_b w2_c Y[(kappa0_a, kappa1_b, kappa2_c) mod K].
The transpose (the paper's NUFFT-transpose, Introduction) applies the
conjugated weights to spread every point onto the grid, an unnormalised inverse
FFT (K^3 * ifftn), the crop back to m in [-N/2, N/2) and the same scaling.

No blocking or reordering beyond processing the points in chunks.
"""
from __future__ import annotations

import numpy as np
from scipy import fft as sfft

from . import kernels

# Threads of the library FFT (scipy.fft's pocketfft); the CPU baseline sets it
# to the host's core count.  The transform is the same for any value.
FFT_WORKERS = 1


class Params:
    """NUFFT parameters: N (even), K >= N, J taps, kernel 'kb'|'minmax', beta,
    scaling 'kb' (deapodization 1/Psi(m/K)) or 'uniform' (s = 1)."""

    def __init__(self, N: int, K: int, J: int, kernel: str = "kb", beta: float | None = None,
                 scaling: str = "kb"):
        assert N % 2 == 0 and K >= N and 1 <= J <= K
        self.N, self.K, self.J, self.kernel = int(N), int(K), int(J), kernel
        self.beta = kernels.default_beta(J) if beta is None else float(beta)
        if scaling == "kb":
            self.s = kernels.deapod(N, K, J, self.beta)
        elif scaling == "uniform":
            self.s = np.ones(N)
        else:
            raise ValueError(scaling)

    def axis_weights(self, omega_d: np.ndarray):
        return kernels.weights(omega_d, self.N, self.K, self.J, self.beta, self.kernel, self.s)


def _pad_index(N: int, K: int) -> np.ndarray:
    m = np.arange(N) - N // 2
    return np.mod(m, K)


def prescale_pad(x: np.ndarray, prm: Params) -> np.ndarray:
    """Step 1: g[(m mod K)] = s(m0) s(m1) s(m2) x[n]; zeros elsewhere."""
    N, K, s = prm.N, prm.K, prm.s
    g = np.zeros((K, K, K), dtype=np.complex128)
    q = _pad_index(N, K)
    g[np.ix_(q, q, q)] = s[:, None, None] * s[None, :, None] * s[None, None, :] * x
    return g


def oversampled_spectrum(x: np.ndarray, prm: Params) -> np.ndarray:
    """Steps 1-2: Y = FFT_K(P x), numpy layout (frequency kappa at index kappa mod K)."""
    return sfft.fftn(prescale_pad(np.asarray(x, dtype=np.complex128), prm), workers=FFT_WORKERS)


def interpolate(Y: np.ndarray, omega: np.ndarray, prm: Params, chunk: int = 1 << 16) -> np.ndarray:
    """Step 3: J^3 tensor-product interpolation from the spectrum grid to the points."""
    K, J = prm.K, prm.J
    omega = np.asarray(omega, dtype=np.float64).reshape(-1, 3)
    out = np.empty(omega.shape[0], dtype=np.complex128)
    flat = Y.reshape(-1)
    for s in range(0, omega.shape[0], chunk):
        w = omega[s:s + chunk]
        k0, w0 = prm.axis_weights(w[:, 0])
        k1, w1 = prm.axis_weights(w[:, 1])
        k2, w2 = prm.axis_weights(w[:, 2])
        i0, i1, i2 = np.mod(k0, K), np.mod(k1, K), np.mod(k2, K)
        acc = np.zeros(w.shape[0], dtype=np.complex128)
        for a in range(J):
            for b in range(J):
                row = (i0[:, a] * K + i1[:, b]) * K
                wab = w0[:, a] * w1[:, b]
                for c in range(J):
                    acc += wab * w2[:, c] * flat[row + i2[:, c]]
        out[s:s + chunk] = acc
    return out


def spread(g: np.ndarray, omega: np.ndarray, prm: Params, chunk: int = 1 << 16) -> np.ndarray:
    """Transpose of interpolate: Y~[kappa] = sum_p conj(w_p(kappa)) g[p]."""
    K, J = prm.K, prm.J
    omega = np.asarray(omega, dtype=np.float64).reshape(-1, 3)
    g = np.asarray(g, dtype=np.complex128).reshape(-1)
    re = np.zeros(K ** 3)
    im = np.zeros(K ** 3)
    for s in range(0, omega.shape[0], chunk):
        w = omega[s:s + chunk]
        gv = g[s:s + chunk]
        k0, w0 = prm.axis_weights(w[:, 0])
        k1, w1 = prm.axis_weights(w[:, 1])
        k2, w2 = prm.axis_weights(w[:, 2])
        i0, i1, i2 = np.mod(k0, K), np.mod(k1, K), np.mod(k2, K)
        idx = ((i0[:, :, None, None] * K + i1[:, None, :, None]) * K + i2[:, None, None, :]).reshape(-1)
        wt = (w0[:, :, None, None] * w1[:, None, :, None] * w2[:, None, None, :])
        val = (np.conj(wt) * gv[:, None, None, None]).reshape(-1)
        re += np.bincount(idx, weights=val.real, minlength=K ** 3)
        im += np.bincount(idx, weights=val.imag, minlength=K ** 3)
    return (re + 1j * im).reshape(K, K, K)


def crop_scale(yt: np.ndarray, prm: Params) -> np.ndarray:
    """Transpose of prescale_pad: x~[n] = s(m0) s(m1) s(m2) y~[(m mod K)]."""
    N, K, s = prm.N, prm.K, prm.s
    q = _pad_index(N, K)
    return yt[np.ix_(q, q, q)] * (s[:, None, None] * s[None, :, None] * s[None, None, :])


def forward(x: np.ndarray, omega: np.ndarray, prm: Params) -> np.ndarray:
    """Type-2 NUFFT: X(omega_p) ~= sum_n x[n] exp(-i omega_p . m)."""
    return interpolate(oversampled_spectrum(x, prm), omega, prm)


def inverse_spectrum(Yt: np.ndarray, prm: Params) -> np.ndarray:
    """Unnormalised inverse FFT: y~[q] = sum_k Y~[k] exp(+2 pi i k.q/K)."""
    return sfft.ifftn(Yt, workers=FFT_WORKERS) * float(prm.K) ** 3


def adjoint(g: np.ndarray, omega: np.ndarray, prm: Params) -> np.ndarray:
    """Exact conjugate transpose of forward."""
    return crop_scale(inverse_spectrum(spread(g, omega, prm), prm), prm)

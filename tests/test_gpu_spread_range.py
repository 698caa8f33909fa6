"""Spreading (the transpose of eq 2.11's interpolation) on inputs with a wide
dynamic range, tiny or huge magnitudes and non-finite values, checked cell by
cell against the oracle.

The FP32 spreading accumulates integers: a value v of magnitude
a = max(|re v|, |im v|) is rounded on a fixed-point scale s = 2^30 / (top B)
shared by the values of its magnitude class within its task (top < 2^c, the
class's bound, and the class holds the binades within CLASS_BITS = 16 of c,
so top < 2^(CLASS_BITS + 1) a), B the largest sum over a halo cell of the
products of the weight magnitudes (at most B_max, the same sum over all
points, computed here from the oracle's weights).  Each contribution's
rounding error is then <= 0.5 / s < a B 2^(CLASS_BITS - 30).  With the
polynomial weights' fit error (<= 1e-7 per axis) and the FP32 products and
additions, every cell k satisfies

    |spread_k - oracle_k| <= (2^(CLASS_BITS-30) B_max + 4e-7) C_k + 8 eps (A_k + |oracle_k|),

C_k = sum over the points whose footprint covers k of a_p, A_k the same sum
weighted by the weight magnitudes, eps = 2^-24.  A single fixed-point scale per
task (no classes) would give the small values of a task holding a 10^7 times
larger outlier errors of about the outlier's magnitude times B 2^-31, which
this bar rejects.  Non-finite inputs make exactly the cells of their J^3
footprints non-finite, as in the FP64 form and the oracle.
"""
import numpy as np
import pytest

import synthetic
from oracle import nufft, radial
from tests.gpu_util import rel_l2, require_gpu, say, to_dev, to_host

pytestmark = pytest.mark.gpu

N, K, J, N_R = 32, 64, 6, 64
CLASS_BITS = 16  # the binades one fixed-point scale of the spreading serves


def _cover_sums(mag, om, prm):
    """Per grid cell (numpy layout): (A, C) = (sum_p |w_p(k)| a_p, sum_p a_p)
    over the points p whose J^3 footprint covers cell k."""
    K_, J_ = prm.K, prm.J
    k0, w0 = prm.axis_weights(om[:, 0])
    k1, w1 = prm.axis_weights(om[:, 1])
    k2, w2 = prm.axis_weights(om[:, 2])
    i0, i1, i2 = np.mod(k0, K_), np.mod(k1, K_), np.mod(k2, K_)
    idx = ((i0[:, :, None, None] * K_ + i1[:, None, :, None]) * K_ + i2[:, None, None, :]).reshape(-1)
    wt = np.abs(w0[:, :, None, None] * w1[:, None, :, None] * w2[:, None, None, :])
    A = np.bincount(idx, weights=(wt * mag[:, None, None, None]).reshape(-1), minlength=K_ ** 3)
    C = np.bincount(idx, weights=np.repeat(mag, J_ ** 3), minlength=K_ ** 3)
    return A.reshape((K_,) * 3), C.reshape((K_,) * 3)


@pytest.fixture(scope="module")
def geo():
    require_gpu()
    import torch
    from paper_1605_05231_amd import Plan
    dirs = synthetic.line_directions(synthetic.azimuths(12), synthetic.polar_angles(6))
    prm = nufft.Params(N, K, J)
    om = radial.points(dirs, N_R)
    p32 = Plan(N, K, J, dirs=dirs, n_r=N_R, dtype=torch.complex64)
    p64 = Plan(N, K, J, dirs=dirs, n_r=N_R, dtype=torch.complex128)
    ones = np.ones(len(om))
    bmax = float(_cover_sums(ones, om, prm)[0].max())
    say(f"[range] M={len(om)} B_max={bmax:.3f}")
    return {"dirs": dirs, "prm": prm, "om": om, "p32": p32, "p64": p64, "bmax": bmax}


def _spread(plan, y, dtype, deterministic=False):
    import torch
    g = torch.empty(K ** 3, dtype=dtype, device="cuda")
    plan.stage(4, to_dev(y, dtype), g, deterministic=deterministic)  # STAGE_SPREAD: centred grid
    return np.fft.ifftshift(to_host(g).reshape((K,) * 3))  # numpy layout


def _check_cells(geo, y, got, label):
    ref = nufft.spread(y, geo["om"], geo["prm"])
    mag = np.maximum(np.abs(y.real), np.abs(y.imag))
    A, C = _cover_sums(mag, geo["om"], geo["prm"])
    eps = 2.0 ** -24
    bar = (2.0 ** (CLASS_BITS - 30) * geo["bmax"] + 4e-7) * C + 8 * eps * (A + np.abs(ref))
    err = np.abs(got - ref)
    covered = C > 0
    ratio = np.max(err[covered] / bar[covered])
    say(f"[range] {label}: worst err/bar {ratio:.3e}, rel-L2 {rel_l2(got, ref):.2e}, "
        f"uncovered cells max |got| {np.max(np.abs(got[~covered])) if (~covered).any() else 0:.1e}")
    assert ratio <= 1.0, (label, ratio)
    assert not np.any(got[~covered]), label
    return ref


def test_outliers_seven_decades(geo):
    """Values of ~1e-7 with one outlier of ~1 among every ~150 points, so that
    every task holds outliers 10^7 times larger than most of its values."""
    import torch
    rng = np.random.default_rng(41)
    M = len(geo["om"])
    y = 1e-7 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    out = rng.choice(M, M // 150, replace=False)
    y[out] = rng.standard_normal(len(out)) + 1j * rng.standard_normal(len(out))
    y = y.astype(np.complex64).astype(np.complex128)
    got = _spread(geo["p32"], y, torch.complex64)
    ref = _check_cells(geo, y, got, "outliers FP32")
    # the cells that no outlier reaches keep the precision of the small values
    mag = np.maximum(np.abs(y.real), np.abs(y.imag))
    small = mag.copy()
    small[out] = 0.0
    big = np.zeros_like(mag)
    big[out] = mag[out]
    _, Cbig = _cover_sums(big, geo["om"], geo["prm"])
    quiet = (Cbig == 0) & (np.abs(ref) > 0)
    e_quiet = rel_l2(got[quiet], ref[quiet])
    say(f"[range] cells no outlier reaches: {quiet.sum()}, rel-L2 {e_quiet:.2e}")
    assert quiet.sum() > 1000 and e_quiet < 2e-6
    g64 = _spread(geo["p64"], y, torch.complex128)
    assert rel_l2(g64, ref) < 1e-12
    # the FP64 form in deterministic mode (fixed point, scale 2^62 / (top B)):
    # the same cell bar with 2^(CLASS_BITS - 62), and its FP64 rounding
    d64 = _spread(geo["p64"], y, torch.complex128, deterministic=True)
    mag = np.maximum(np.abs(y.real), np.abs(y.imag))
    A, C = _cover_sums(mag, geo["om"], geo["prm"])
    bar = (2.0 ** (CLASS_BITS - 62) * geo["bmax"] + 1e-12) * C + 8 * 2.0 ** -53 * (A + np.abs(ref))
    covered = C > 0
    r64 = np.max(np.abs(d64 - ref)[covered] / bar[covered])
    say(f"[range] outliers FP64 deterministic: worst err/bar {r64:.3e}, rel-L2 {rel_l2(d64, ref):.2e}")
    assert r64 <= 1.0 and rel_l2(d64, ref) < 1e-12


@pytest.mark.parametrize("scale", [1e-33, 1e-20, 1e35])
def test_tiny_and_huge_magnitudes(geo, scale):
    import torch
    rng = np.random.default_rng(int(abs(np.log10(scale))))
    M = len(geo["om"])
    y = scale * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    y = y.astype(np.complex64).astype(np.complex128)
    got = _spread(geo["p32"], y, torch.complex64)
    ref = _check_cells(geo, y, got, f"scale {scale:g} FP32")
    assert rel_l2(got, ref) < 2e-6


def test_non_finite_values(geo):
    """NaN and infinite inputs: the non-finite cells are exactly those of their
    footprints (as in the oracle and the FP64 form); the other cells are
    accurate."""
    import torch
    rng = np.random.default_rng(43)
    M = len(geo["om"])
    y = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    y = y.astype(np.complex64).astype(np.complex128)
    bad = rng.choice(M, 5, replace=False)
    y[bad[0]] = complex(np.nan, 0.0)
    y[bad[1]] = complex(0.0, np.nan)
    y[bad[2]] = complex(np.inf, 1.0)
    y[bad[3]] = complex(-np.inf, np.inf)
    y[bad[4]] = complex(np.nan, np.nan)
    ref = nufft.spread(y, geo["om"], geo["prm"])
    got = _spread(geo["p32"], y, torch.complex64)
    g64 = _spread(geo["p64"], y, torch.complex128)
    nf_ref = ~np.isfinite(ref)
    say(f"[range] non-finite cells: oracle {nf_ref.sum()}, FP32 {(~np.isfinite(got)).sum()}, "
        f"FP64 {(~np.isfinite(g64)).sum()}")
    assert nf_ref.sum() >= 5 * J ** 3 // 2
    d64 = _spread(geo["p64"], y, torch.complex128, deterministic=True)
    assert np.array_equal(~np.isfinite(got), nf_ref)
    assert np.array_equal(~np.isfinite(g64), nf_ref)
    assert np.array_equal(~np.isfinite(d64), nf_ref)
    # the finite cells against the oracle of the finite values alone
    yf = y.copy()
    yf[bad] = 0.0
    ok = ~nf_ref
    reff = nufft.spread(yf, geo["om"], geo["prm"])
    assert rel_l2(got[ok], reff[ok]) < 2e-6


def test_non_finite_reaches_adjoint_and_gradient(geo):
    """A NaN residual gives a non-finite adjoint (every voxel, after the inverse
    FFT), in the FP32 path as in the FP64 form."""
    import torch
    M = len(geo["om"])
    y = np.zeros(M, dtype=np.complex128)
    y[M // 3] = complex(np.nan, 0.0)
    v32 = geo["p32"].adjoint(to_dev(y, torch.complex64))
    v64 = geo["p64"].adjoint(to_dev(y, torch.complex128))
    assert not torch.isfinite(v32).any() and not torch.isfinite(v64).any()

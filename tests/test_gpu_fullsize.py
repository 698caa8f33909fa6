"""Parity at full workload sizes, in the tiling the benchmark runs:

  c2  128^3 volume, K = 256^3, J = 6 KB, 180 x 90 lines x 256 samples
      (4,147,200 points), tiling chosen by the autotuner as the benchmark does;
  c3  256^3 volume, K = 512^3, J = 6 KB, 360 x 180 lines x 512 samples
      (33,177,600 points), 16^3 tiles and 16,384 points per task (the
      autotuner's choice at this size; taken directly, which saves its run).

The oracle cannot run every point at these sizes, so it runs a sample of
whole lines: the grid-size work (the oversampled FFT and its inverse) in full,
the point work only for the sampled lines.  Checked, with relative-L2 and
max-error bars:
  * forward: the sampled lines of the GPU output against the oracle's;
  * adjoint: the adjoint of data that is zero except on the sampled lines,
    over every voxel, against the oracle's adjoint of those lines alone;
  * for all points, the dot test <A x, y> = <x, A^H y> (the c2 gate: 1e-5).
Both the FP32 path and the FP64 form are checked.  The sample includes the
lines where taps tie (phi = 0, pi/2, pi, 3pi/2) and the first and last polar
angles, plus a seeded random set."""
import os

import numpy as np
import pytest

import synthetic
from oracle import nufft, radial
from tests.gpu_util import max_rel, rel_l2, require_gpu, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _sample_lines(W, n_rand):
    n_phi, n_th = W.n_phi, W.n_theta
    rng = np.random.default_rng(77)
    picks = [(a, b) for a in (0, n_phi // 4, n_phi // 2, 3 * n_phi // 4) for b in (0, n_th // 2, n_th - 1)]
    picks += [(int(a), int(b)) for a, b in zip(rng.integers(0, n_phi, n_rand), rng.integers(0, n_th, n_rand))]
    return np.unique(np.array([a * n_th + b for a, b in picks]))


@pytest.fixture(scope="module", params=["c2", "c3"])
def wl(request):
    require_gpu()
    W = synthetic.WORKLOADS[request.param]
    x = W.volume()
    dirs = W.directions()
    lines = _sample_lines(W, 60 if W.name == "c3" else 120)
    prm = nufft.Params(W.N, W.K, W.J)
    om = radial.points(dirs[lines], W.n_r)
    say(f"[fullsize] {W.name} oracle: {len(lines)} of {len(dirs)} lines, full {W.K}^3 transforms")
    Y = nufft.oversampled_spectrum(x.astype(np.complex128), prm)
    D = radial.forward(nufft.interpolate(Y, om, prm), W.n_r)
    # sampled cells of the centred spectrum (the stage API's compact layout):
    # random ones plus the grid's last planes, rows and columns
    K = W.K
    rs = np.random.default_rng(80)
    cells = np.concatenate([rs.integers(0, K, (3000, 3)),
                            np.stack([np.full(200, K - 1), rs.integers(0, K, 200), rs.integers(0, K, 200)], 1),
                            np.stack([rs.integers(0, K, 200), np.full(200, K - 1), rs.integers(0, K, 200)], 1),
                            np.stack([rs.integers(0, K, 200), rs.integers(0, K, 200), np.full(200, K - 1)], 1)])
    Yc = Y[tuple(((cells + K // 2) % K).T)]  # centred cell j holds frequency j - K/2
    del Y
    rng = np.random.default_rng(78)
    d = rng.standard_normal(D.shape) + 1j * rng.standard_normal(D.shape)
    v = nufft.crop_scale(nufft.inverse_spectrum(nufft.spread(radial.adjoint(d, W.n_r), om, prm), prm), prm)
    return {"W": W, "x": x, "dirs": dirs, "lines": lines, "D": D, "d": d, "v": v, "tiling": None,
            "cells": cells, "Yc": Yc}


def _plan(pkg, W, dirs, dtype):
    """A plan in the benchmark's tiling: autotuned at c2, 16 / 16384 at c3."""
    if W.name == "c3":
        old = os.environ.get("NUFFTCT_MAXPTS"), os.environ.get("NUFFTCT_TILE")
        os.environ["NUFFTCT_MAXPTS"], os.environ["NUFFTCT_TILE"] = "16384", "16"
        try:
            return pkg.Plan(W.N, W.K, W.J, dirs=dirs, n_r=W.n_r, dtype=dtype)
        finally:
            for k, o in zip(("NUFFTCT_MAXPTS", "NUFFTCT_TILE"), old):
                if o is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = o
    pkg.autotune(W.N, W.K, W.J, dirs, W.n_r, dtype=dtype)
    return pkg.Plan(W.N, W.K, W.J, dirs=dirs, n_r=W.n_r, dtype=dtype)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_sampled_lines_vs_oracle(wl, prec):
    import torch
    import paper_1605_05231_amd as pkg
    W = wl["W"]
    dtype = torch.complex64 if prec == "f32" else torch.complex128
    say(f"[fullsize] {W.name} {prec}: plan {W.N}^3 / {W.K}^3, {W.M} points")
    plan = _plan(pkg, W, wl["dirs"], dtype)
    say(f"[fullsize] {W.name} {prec}: tiling {plan.tiling()}")
    L, n_r = len(wl["dirs"]), W.n_r
    sel = torch.from_numpy(wl["lines"]).cuda()
    # forward: every point is computed, the sampled lines are compared
    D = plan.forward(to_dev(wl["x"], dtype)).reshape(L, n_r)
    got = to_host(D[sel]).reshape(-1)
    ef, mf = rel_l2(got, wl["D"]), max_rel(got, wl["D"])
    # adjoint of data living on the sampled lines only, over all voxels
    din = torch.zeros((L, n_r), dtype=dtype, device="cuda")
    din[sel] = to_dev(wl["d"].reshape(-1, n_r), dtype)
    v = to_host(plan.adjoint(din))
    ea, ma = rel_l2(v, wl["v"]), max_rel(v, wl["v"])
    say(f"[fullsize] {W.name} {prec}: forward rel-L2 {ef:.2e} max {mf:.2e} on {len(wl['lines'])} lines; "
        f"adjoint rel-L2 {ea:.2e} max {ma:.2e}")
    tol = 1e-5 if prec == "f32" else 1e-12
    assert max(ef, mf, ea, ma) < tol
    plan.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_dot_product_all_points(wl, prec):
    import torch
    import paper_1605_05231_amd as pkg
    W = wl["W"]
    dtype = torch.complex64 if prec == "f32" else torch.complex128
    plan = _plan(pkg, W, wl["dirs"], dtype)
    g = torch.Generator(device="cuda").manual_seed(79)
    x = torch.randn(W.N ** 3, dtype=dtype, device="cuda", generator=g)
    y = torch.randn(W.M, dtype=dtype, device="cuda", generator=g)
    ax = plan.forward(x).reshape(-1).to(torch.complex128)
    ahy = plan.adjoint(y).reshape(-1).to(torch.complex128)
    lhs = torch.vdot(y.to(torch.complex128), ax).item()
    rhs = torch.vdot(ahy, x.to(torch.complex128)).item()
    err = abs(lhs - rhs) / abs(lhs)
    say(f"[fullsize] {W.name} {prec}: dot test relative difference {err:.2e}")
    assert err < (1e-5 if prec == "f32" else 1e-12)
    plan.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_stage_chain_full_grid(wl, prec):
    """The stage API at full size hands out compact K^3 grids while the plan's
    own grid may pad its planes (512^2 planes are): the spectrum stage against
    the oracle at sampled cells (last planes, rows and columns included), and
    the stages chained through compact grids equal the fused operators bit for
    bit."""
    import torch
    import paper_1605_05231_amd as pkg
    W = wl["W"]
    dtype = torch.complex64 if prec == "f32" else torch.complex128
    plan = _plan(pkg, W, wl["dirs"], dtype)
    x = to_dev(wl["x"], dtype)
    g = torch.empty(W.K ** 3, dtype=dtype, device="cuda")
    plan.stage(pkg.STAGE_PAD_FFT, x, g)
    c = torch.from_numpy(wl["cells"]).cuda()
    got = to_host(g.reshape(W.K, W.K, W.K)[c[:, 0], c[:, 1], c[:, 2]])
    m = max_rel(got, wl["Yc"])
    say(f"[fullsize] {W.name} {prec}: spectrum stage at {len(got)} cells, max err {m:.2e}")
    assert m < (2e-6 if prec == "f32" else 1e-13)
    G = torch.empty(W.M, dtype=dtype, device="cuda")
    plan.stage(pkg.STAGE_INTERP, g, G)
    D = torch.empty(W.M, dtype=dtype, device="cuda")
    plan.stage(pkg.STAGE_RADIAL, G, D)
    assert torch.equal(D, plan.forward(x).reshape(-1))
    y = D.clone()
    Gt = torch.empty(W.M, dtype=dtype, device="cuda")
    plan.stage(pkg.STAGE_RADIAL_ADJ, y, Gt)
    plan.stage(pkg.STAGE_SPREAD, Gt, g, deterministic=True)
    v = torch.empty(W.N ** 3, dtype=dtype, device="cuda")
    plan.stage(pkg.STAGE_IFFT_CROP, g, v)
    assert torch.equal(v, plan.adjoint(y, deterministic=True).reshape(-1))
    plan.close()

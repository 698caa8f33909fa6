"""Parity at the full benchmark size: the 256^3 volume on the K = 512^3 grid,
J = 6 Kaiser-Bessel, 360 x 180 lines x 512 samples = 33,177,600 points, in the
tiling the benchmark runs (16^3 tiles, 16,384 points per task).

The oracle cannot run every point at this size, so it runs a sample of whole
lines: the grid-size work (the 512^3 oversampled FFT and its inverse) in full,
the point work only for the sampled lines.  Checked:
  * forward: the sampled lines of the GPU output against the oracle's;
  * adjoint: the adjoint of data that is zero except on the sampled lines,
    over every voxel of the 256^3 output, against the oracle's adjoint of
    those lines alone;
  * for all 33 M points, the dot test <A x, y> = <x, A^H y>.
Both the FP32 path and the FP64 form are checked.  The sample includes the
lines where taps tie (phi = 0, pi/2, pi, 3pi/2) and the first and last polar
angles, plus a seeded random set."""
import os

import numpy as np
import pytest

import synthetic
from oracle import nufft, radial
from tests.gpu_util import rel_l2, require_gpu, say, to_dev, to_host

pytestmark = pytest.mark.gpu

W = synthetic.WORKLOADS["c3"]


def _sample_lines():
    n_phi, n_th = W.n_phi, W.n_theta
    rng = np.random.default_rng(77)
    picks = [(a, b) for a in (0, n_phi // 4, n_phi // 2, 3 * n_phi // 4) for b in (0, n_th // 2, n_th - 1)]
    picks += [(int(a), int(b)) for a, b in zip(rng.integers(0, n_phi, 60), rng.integers(0, n_th, 60))]
    return np.unique(np.array([a * n_th + b for a, b in picks]))


@pytest.fixture(scope="module")
def c3():
    require_gpu()
    x = W.volume()
    dirs = W.directions()
    lines = _sample_lines()
    prm = nufft.Params(W.N, W.K, W.J)
    om = radial.points(dirs[lines], W.n_r)
    say(f"[fullsize] oracle: {len(lines)} of {len(dirs)} lines, full 512^3 transforms")
    Y = nufft.oversampled_spectrum(x.astype(np.complex128), prm)
    D = radial.forward(nufft.interpolate(Y, om, prm), W.n_r)
    del Y
    rng = np.random.default_rng(78)
    d = rng.standard_normal(D.shape) + 1j * rng.standard_normal(D.shape)
    v = nufft.crop_scale(nufft.inverse_spectrum(nufft.spread(radial.adjoint(d, W.n_r), om, prm), prm), prm)
    return {"x": x, "dirs": dirs, "lines": lines, "D": D, "d": d, "v": v}


def _plan(pkg, torch, dirs, dtype):
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


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_c3_sampled_lines_vs_oracle(c3, prec):
    import torch
    import paper_1605_05231_amd as pkg
    dtype = torch.complex64 if prec == "f32" else torch.complex128
    say(f"[fullsize] {prec}: plan 256^3 / 512^3, {W.M} points")
    plan = _plan(pkg, torch, c3["dirs"], dtype)
    L, n_r = len(c3["dirs"]), W.n_r
    sel = torch.from_numpy(c3["lines"]).cuda()
    # forward: every point is computed, the sampled lines are compared
    D = plan.forward(to_dev(c3["x"], dtype)).reshape(L, n_r)
    ef = rel_l2(to_host(D[sel]).reshape(-1), c3["D"])
    # adjoint of data living on the sampled lines only, over all voxels
    din = torch.zeros((L, n_r), dtype=dtype, device="cuda")
    din[sel] = to_dev(c3["d"].reshape(-1, n_r), dtype)
    v = to_host(plan.adjoint(din))
    ea = rel_l2(v, c3["v"])
    say(f"[fullsize] {prec}: forward rel-L2 {ef:.2e} on {len(c3['lines'])} lines; adjoint rel-L2 {ea:.2e}")
    tol = 1e-5 if prec == "f32" else 1e-12
    assert ef < tol and ea < tol
    plan.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_c3_dot_product_all_points(prec):
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    dtype = torch.complex64 if prec == "f32" else torch.complex128
    plan = _plan(pkg, torch, W.directions(), dtype)
    g = torch.Generator(device="cuda").manual_seed(79)
    x = torch.randn(W.N ** 3, dtype=dtype, device="cuda", generator=g)
    y = torch.randn(W.M, dtype=dtype, device="cuda", generator=g)
    ax = plan.forward(x).reshape(-1).to(torch.complex128)
    ahy = plan.adjoint(y).reshape(-1).to(torch.complex128)
    lhs = torch.vdot(y.to(torch.complex128), ax).item()
    rhs = torch.vdot(ahy, x.to(torch.complex128)).item()
    err = abs(lhs - rhs) / abs(lhs)
    say(f"[fullsize] {prec}: dot test relative difference {err:.2e}")
    assert err < (1e-5 if prec == "f32" else 1e-12)
    plan.close()

"""Differentiation through the projector (the c4 workload: 128^3, batch 4,
K=256^3, J=6, 180 x 90 lines x 256 samples): the autograd backward is the
hand-written adjoint, checked by central finite differences and against the
oracle gradient A^H (A x - y)."""
import numpy as np
import pytest

import synthetic
from oracle import nufft, projector, radial
from tests.gpu_util import max_rel, rel_l2, require_gpu, say

pytestmark = pytest.mark.gpu


def _loss_grad(pkg, plan, x_np, y_np):
    import torch
    x = torch.from_numpy(x_np.astype(np.float32)).cuda().requires_grad_(True)
    y = torch.from_numpy(y_np.astype(np.complex64)).cuda()
    r = pkg.project(x, plan) - y
    loss = 0.5 * (r.real.double() ** 2 + r.imag.double() ** 2).sum()
    loss.backward()
    return float(loss), x.grad.double().cpu().numpy()


def test_gradient_vs_oracle_reduced_c4():
    """Batch of 4 perturbed-phantom pairs at 48^3 (c4 geometry scaled down):
    gradient = Re A^H (A x - y) from the oracle."""
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    N, K, J, n_r = 48, 96, 6, 96
    dirs = synthetic.line_directions(synthetic.azimuths(36), synthetic.polar_angles(18))
    prm = nufft.Params(N, K, J)
    plan = pkg.Plan(N, K, J, dirs=dirs, n_r=n_r)
    xs = np.stack([synthetic.ellipsoid_phantom(N, 20, 4000 + b) for b in range(4)])
    ys = np.stack([projector.forward(synthetic.ellipsoid_phantom(N, 20, 4000 + b, perturb=True),
                                     dirs, n_r, prm).reshape(len(dirs), n_r) for b in range(4)])
    x32 = xs.astype(np.float32).astype(float)
    y32 = ys.astype(np.complex64).astype(complex)
    loss, g = _loss_grad(pkg, plan, x32, y32)
    for b in range(4):
        r = projector.forward(x32[b], dirs, n_r, prm) - y32[b].reshape(-1)
        gw = projector.adjoint(r, dirs, n_r, prm).real
        e, m = rel_l2(g[b], gw), max_rel(g[b], gw)
        say(f"grad vs oracle [{b}] rel={e:.2e} max={m:.2e}")
        assert e < 1e-4 and m < 1e-4


def test_c4_full_size_finite_differences():
    """c4 sizes: 4 x 128^3, 4.1 M points.  Central differences (step 1e-3) of
    the loss evaluated with the FP64 form at 64 random voxels against the
    FP32 autograd gradient; the loss is quadratic, so the differences carry
    no truncation error."""
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    W = synthetic.WORKLOADS["c4"]
    dirs = W.directions()
    plan32 = pkg.Plan(W.N, W.K, W.J, dirs=dirs, n_r=W.n_r)
    plan64 = pkg.Plan(W.N, W.K, W.J, dirs=dirs, n_r=W.n_r, dtype=torch.complex128)
    xs = np.stack([W.volume(b) for b in range(4)]).astype(np.float32).astype(float)
    # y = A x_pert with the FP64 form: data for the loss, not an expected value
    ys = []
    for b in range(4):
        xp = torch.from_numpy(W.volume(b, perturb=True).astype(np.complex128)).cuda()
        ys.append(plan64.forward(xp).cpu().numpy())
    ys = np.stack(ys).astype(np.complex64).astype(complex)
    loss, g = _loss_grad(pkg, plan32, xs, ys)
    rng = np.random.default_rng(4)
    h = 1e-3
    yd = [torch.from_numpy(ys[b]).cuda() for b in range(4)]

    def L64(b, x):
        xd = torch.from_numpy(x.astype(np.complex128)).cuda()
        r = plan64.forward(xd) - yd[b]
        return 0.5 * float((r.abs() ** 2).sum())

    worst = 0.0
    for k in range(64):
        b = int(rng.integers(4))
        idx = tuple(int(v) for v in rng.integers(W.N // 4, 3 * W.N // 4, size=3))
        xp = xs[b].copy()
        xm = xs[b].copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (L64(b, xp) - L64(b, xm)) / (2 * h)
        err = abs(fd - g[b][idx]) / max(abs(fd), 1e-3 * np.max(np.abs(g[b])))
        worst = max(worst, err)
    say(f"c4 FD worst rel err {worst:.2e}")
    assert worst < 1e-4
    # and the FP32 autograd gradient against the FP64 form's own adjoint
    for b in range(4):
        xd = torch.from_numpy(xs[b].astype(np.complex128)).cuda()
        r = plan64.forward(xd) - yd[b]
        g64 = plan64.adjoint(r).real.cpu().numpy()
        e = rel_l2(g[b], g64)
        say(f"c4 grad FP32 vs FP64 form [{b}] {e:.2e}")
        assert e < 1e-4


def test_c4_full_size_gradient_vs_oracle_sampled_lines():
    """c4 sizes (4 x 128^3, K = 256^3, 4.1 M points per volume): the loss
    0.5 ||S (A x - y)||^2 over a sample S of whole lines of every volume, with
    y = the oracle's projection of the perturbed phantoms on those lines.  Its
    FP32 autograd gradient Re A^H S^T S (A x - y) covers every voxel; the
    oracle computes the same from its own forward on the sampled lines and
    its adjoint of their residual."""
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    W = synthetic.WORKLOADS["c4"]
    dirs = W.directions()
    L, n_r = len(dirs), W.n_r
    prm = nufft.Params(W.N, W.K, W.J)
    plan = pkg.Plan(W.N, W.K, W.J, dirs=dirs, n_r=n_r)
    rng = np.random.default_rng(404)
    lines = np.unique(rng.integers(0, L, 40))
    om = radial.points(dirs[lines], n_r)
    xs = np.stack([W.volume(b) for b in range(4)]).astype(np.float32).astype(float)
    ys = np.zeros((4, L, n_r), dtype=np.complex128)
    want = []
    for b in range(4):
        xp = W.volume(b, perturb=True).astype(np.complex128)
        ys[b, lines] = radial.forward(nufft.interpolate(nufft.oversampled_spectrum(xp, prm), om, prm),
                                      n_r).reshape(-1, n_r)
    ys = ys.astype(np.complex64).astype(np.complex128)
    for b in range(4):
        r = radial.forward(nufft.interpolate(nufft.oversampled_spectrum(xs[b] + 0j, prm), om, prm), n_r)
        r = r - ys[b, lines].reshape(-1)
        want.append(nufft.crop_scale(nufft.inverse_spectrum(nufft.spread(radial.adjoint(r, n_r), om, prm),
                                                            prm), prm).real)
    x = torch.from_numpy(xs.astype(np.float32)).cuda().requires_grad_(True)
    y = torch.from_numpy(ys.astype(np.complex64)).cuda()
    sel = torch.from_numpy(lines).cuda()
    res = (pkg.project(x, plan) - y)[:, sel]
    loss = 0.5 * (res.real.double() ** 2 + res.imag.double() ** 2).sum()
    loss.backward()
    g = x.grad.double().cpu().numpy()
    for b in range(4):
        e, m = rel_l2(g[b], want[b]), max_rel(g[b], want[b])
        say(f"c4 grad vs oracle on {len(lines)} lines [{b}] rel={e:.2e} max={m:.2e}")
        assert e < 1e-4 and m < 1e-4


def test_gradcheck_fp64_small():
    """torch.autograd.gradcheck on a tiny FP64 plan (complex input)."""
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    N, K, J, n_r = 8, 16, 4, 16
    dirs = synthetic.line_directions(synthetic.azimuths(3), synthetic.polar_angles(2))
    plan = pkg.Plan(N, K, J, dirs=dirs, n_r=n_r, dtype=torch.complex128)
    x = torch.randn(N, N, N, dtype=torch.complex128, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda v: pkg.project(v, plan), (x,), eps=1e-6, atol=1e-7,
                                    rtol=1e-6, fast_mode=True)

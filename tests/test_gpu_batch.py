"""Uneven batches (the c5 workload: 64 volumes, N in {48..160}, K = 2N, J = 6,
own direction sets with N_phi in [60, 240], N_theta = N_phi/2, N_r = 2N) and
HIP-graph replay."""
import numpy as np
import pytest

import synthetic
from oracle import nufft, projector, radial
from tests.gpu_util import max_rel, rel_l2, require_gpu, say

pytestmark = pytest.mark.gpu


def _make(items):
    import torch
    import paper_1605_05231_amd as pkg
    dirs = [w.directions() for w in items]
    b = pkg.Batch([w.N for w in items], [w.K for w in items], 6, dirs, [w.n_r for w in items])
    xs = [torch.from_numpy(w.volume().astype(np.complex64)).cuda() for w in items]
    outs = [torch.empty(w.M, dtype=torch.complex64, device="cuda") for w in items]
    vols = [torch.empty(w.N ** 3, dtype=torch.complex64, device="cuda") for w in items]
    return b, dirs, xs, outs, vols


def test_small_uneven_batch_vs_oracle():
    require_gpu()
    items = [synthetic.Workload(f"b{i}", N=n, K=2 * n, J=6, n_phi=p, n_theta=p // 2, n_r=2 * n,
                                n_ell=10 + i, seed=5000 + i)
             for i, (n, p) in enumerate([(48, 12), (64, 8), (48, 10), (32, 16)])]
    b, dirs, xs, outs, vols = _make(items)
    b.forward(xs, outs)
    b.adjoint(outs, vols)
    for i, w in enumerate(items):
        prm = nufft.Params(w.N, w.K, 6)
        x = xs[i].cpu().numpy().astype(complex)
        want = projector.forward(x, dirs[i], w.n_r, prm)
        got = outs[i].cpu().numpy()
        ef = rel_l2(got, want)
        wa = projector.adjoint(got.astype(complex), dirs[i], w.n_r, prm)
        ea = rel_l2(vols[i].cpu().numpy(), wa.reshape(-1))
        mf = max_rel(got, want)
        ma = max_rel(vols[i].cpu().numpy(), wa.reshape(-1))
        say(f"batch item {i} N={w.N} fwd={ef:.2e} (max {mf:.2e}) adj={ea:.2e} (max {ma:.2e})")
        assert max(ef, ea, mf, ma) < 1e-5


def test_many_small_volumes_in_chunks():
    """70 volumes of 16^3 and three of 24^3: the small volumes run as batched
    launches in two chunks of at most 64 volumes; every result equals its
    single plan's bit for bit, eagerly and from graph replays, and two members
    match the oracle."""
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    spec = [(16, 8)] * 70 + [(24, 12)] * 3
    items = [synthetic.Workload(f"t{i}", N=n, K=2 * n, J=6, n_phi=p, n_theta=p // 2, n_r=2 * n,
                                n_ell=4, seed=5300 + i) for i, (n, p) in enumerate(spec)]
    b, dirs, xs, outs, vols = _make(items)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.forward(xs, outs)
        b.adjoint(outs, vols)
    stream.synchronize()
    ref_out = [o.clone() for o in outs]
    ref_vol = [v.clone() for v in vols]
    for i in (0, 37, 63, 64, 69, 70, 72):
        w = items[i]
        p = pkg.Plan(w.N, w.K, 6, dirs=dirs[i], n_r=w.n_r)
        o = p.forward(xs[i])
        assert torch.equal(o.reshape(-1), ref_out[i]), i
        assert torch.equal(p.adjoint(o).reshape(-1), ref_vol[i]), i
        p.close()
    with torch.cuda.stream(stream):
        b.capture(0, xs, outs, stream=stream)
        b.capture(1, outs, vols, stream=stream)
    for rep in range(2):
        for o in outs:
            o.zero_()
        for v in vols:
            v.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            b.replay(0, stream=stream)
            b.replay(1, stream=stream)
        stream.synchronize()
        for i in range(len(items)):
            assert torch.equal(outs[i], ref_out[i]), (rep, i)
            assert torch.equal(vols[i], ref_vol[i]), (rep, i)
    for i in (5, 71):
        w = items[i]
        prm = nufft.Params(w.N, w.K, 6)
        x = xs[i].cpu().numpy().astype(complex)
        want = projector.forward(x, dirs[i], w.n_r, prm)
        e = rel_l2(ref_out[i].cpu().numpy(), want)
        wa = projector.adjoint(ref_out[i].cpu().numpy().astype(complex), dirs[i], w.n_r, prm)
        ea = rel_l2(ref_vol[i].cpu().numpy(), wa.reshape(-1))
        say(f"small batch item {i} N={w.N}: fwd {e:.2e} adj {ea:.2e}")
        assert max(e, ea) < 1e-5


def test_tuned_batch_vs_oracle():
    """A batch whose size classes take the autotuner's tiling: every member
    matches the oracle, and the members of a class share one tiling."""
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    spec = [(48, 12), (48, 10), (64, 8), (32, 16), (64, 10)]
    items = [synthetic.Workload(f"u{i}", N=n, K=2 * n, J=6, n_phi=p, n_theta=p // 2, n_r=2 * n,
                                n_ell=10, seed=5400 + i) for i, (n, p) in enumerate(spec)]
    dirs = [w.directions() for w in items]
    b = pkg.Batch([w.N for w in items], [w.K for w in items], 6, dirs, [w.n_r for w in items],
                  tune=True)
    xs = [torch.from_numpy(w.volume().astype(np.complex64)).cuda() for w in items]
    outs = [torch.empty(w.M, dtype=torch.complex64, device="cuda") for w in items]
    vols = [torch.empty(w.N ** 3, dtype=torch.complex64, device="cuda") for w in items]
    b.forward(xs, outs)
    b.adjoint(outs, vols)
    torch.cuda.synchronize()
    for i, w in enumerate(items):
        prm = nufft.Params(w.N, w.K, 6)
        x = xs[i].cpu().numpy().astype(complex)
        want = projector.forward(x, dirs[i], w.n_r, prm)
        got = outs[i].cpu().numpy()
        wa = projector.adjoint(got.astype(complex), dirs[i], w.n_r, prm)
        ef, ea = rel_l2(got, want), rel_l2(vols[i].cpu().numpy(), wa.reshape(-1))
        say(f"tuned batch item {i} N={w.N}: fwd {ef:.2e} adj {ea:.2e}")
        assert max(ef, ea, max_rel(got, want)) < 1e-5


def test_minmax_batch_matches_single_plans():
    """Min-max weights differ per volume, so such a batch runs volume by volume
    on worker streams: its results equal single plans' bit for bit."""
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    items = [synthetic.Workload(f"m{i}", N=n, K=2 * n, J=6, n_phi=p, n_theta=p // 2, n_r=2 * n,
                                n_ell=10, seed=5100 + i)
             for i, (n, p) in enumerate([(32, 12), (48, 10), (32, 8)])]
    dirs = [w.directions() for w in items]
    b = pkg.Batch([w.N for w in items], [w.K for w in items], 6, dirs, [w.n_r for w in items],
                  kernel="minmax")
    xs = [torch.from_numpy(w.volume().astype(np.complex64)).cuda() for w in items]
    outs = [torch.empty(w.M, dtype=torch.complex64, device="cuda") for w in items]
    vols = [torch.empty(w.N ** 3, dtype=torch.complex64, device="cuda") for w in items]
    b.forward(xs, outs)
    b.adjoint(outs, vols)
    torch.cuda.synchronize()
    for i, w in enumerate(items):
        p = pkg.Plan(w.N, w.K, 6, dirs=dirs[i], n_r=w.n_r, kernel="minmax")
        o = p.forward(xs[i])
        assert torch.equal(o.reshape(-1), outs[i])
        assert torch.equal(p.adjoint(o).reshape(-1), vols[i])
        p.close()


@pytest.mark.parametrize("prec", ["f64"])
def test_fp64_batch_deterministic_matches_single_plans(prec):
    """The FP64 batch in deterministic mode (fixed-point spreading, one launch
    per stage) equals single plans bit for bit, twice in a row."""
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    items = [synthetic.Workload(f"d{i}", N=n, K=2 * n, J=6, n_phi=p, n_theta=p // 2, n_r=2 * n,
                                n_ell=10, seed=5200 + i)
             for i, (n, p) in enumerate([(32, 12), (48, 10), (64, 8)])]
    dirs = [w.directions() for w in items]
    b = pkg.Batch([w.N for w in items], [w.K for w in items], 6, dirs, [w.n_r for w in items],
                  dtype=torch.complex128)
    xs = [torch.from_numpy(w.volume().astype(np.complex128)).cuda() for w in items]
    outs = [torch.empty(w.M, dtype=torch.complex128, device="cuda") for w in items]
    vols = [torch.empty(w.N ** 3, dtype=torch.complex128, device="cuda") for w in items]
    b.forward(xs, outs)
    for rep in range(2):
        b.adjoint(outs, vols, deterministic=True)
        torch.cuda.synchronize()
        for i, w in enumerate(items):
            p = pkg.Plan(w.N, w.K, 6, dirs=dirs[i], n_r=w.n_r, dtype=torch.complex128)
            o = p.forward(xs[i])
            assert torch.equal(o.reshape(-1), outs[i])
            assert torch.equal(p.adjoint(o, deterministic=True).reshape(-1), vols[i]), (rep, i)
            p.close()


def test_c5_batch_graph_replay():
    """The full 64-volume c5 batch: batched results equal single-plan results
    bit for bit, and graph replays equal the eager run bit for bit on every
    replay (eager work and synchronisations between replays)."""
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    items = synthetic.batch_workload(64)
    say(f"c5 total points {sum(w.M for w in items)}")
    b, dirs, xs, outs, vols = _make(items)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.forward(xs, outs)
        b.adjoint(outs, vols)
    stream.synchronize()
    ref_out = [o.clone() for o in outs]
    ref_vol = [v.clone() for v in vols]
    # spot-check four members against independent single plans
    for i in (0, 17, 40, 63):
        w = items[i]
        p = pkg.Plan(w.N, w.K, 6, dirs=dirs[i], n_r=w.n_r)
        o = p.forward(xs[i])
        assert torch.equal(o.reshape(-1), ref_out[i])
        assert torch.equal(p.adjoint(o).reshape(-1), ref_vol[i])
    # graph capture of forward and adjoint; replays vs eager results
    with torch.cuda.stream(stream):
        b.capture(0, xs, outs, stream=stream)
        b.capture(1, outs, vols, stream=stream)
    for rep in range(3):
        for o in outs:
            o.zero_()
        for v in vols:
            v.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            b.replay(0, stream=stream)
            b.replay(1, stream=stream)
        stream.synchronize()
        # unrelated eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        for i in range(len(items)):
            assert torch.equal(outs[i], ref_out[i]), (rep, i)
            assert torch.equal(vols[i], ref_vol[i]), (rep, i)
    # one member of each of the larger sizes (grids 192 = 8 8 3, 256 = 8 8 4,
    # 320 = 8 8 5) against the oracle on sampled whole lines: the member's own
    # plan reproduces the batch bit for bit, and its forward on the sampled
    # lines and its adjoint of data on those lines alone match the oracle
    rng = np.random.default_rng(55)
    for n in (96, 128, 160):
        i = next(k for k, w in enumerate(items) if w.N == n)
        w = items[i]
        p = pkg.Plan(w.N, w.K, 6, dirs=dirs[i], n_r=w.n_r)
        o = p.forward(xs[i])
        assert torch.equal(o.reshape(-1), ref_out[i])
        L = len(dirs[i])
        lines = np.unique(rng.integers(0, L, 24))
        prm = nufft.Params(w.N, w.K, 6)
        om = radial.points(dirs[i][lines], w.n_r)
        x = xs[i].cpu().numpy().astype(complex)
        want = radial.forward(nufft.interpolate(nufft.oversampled_spectrum(x, prm), om, prm), w.n_r)
        got = o.reshape(L, w.n_r)[torch.from_numpy(lines).cuda()].cpu().numpy().reshape(-1)
        ef, mf = rel_l2(got, want), max_rel(got, want)
        d = rng.standard_normal(want.shape) + 1j * rng.standard_normal(want.shape)
        d = d.astype(np.complex64).astype(complex)
        din = torch.zeros((L, w.n_r), dtype=torch.complex64, device="cuda")
        din[torch.from_numpy(lines).cuda()] = torch.from_numpy(d.reshape(-1, w.n_r).astype(np.complex64)).cuda()
        va = p.adjoint(din).cpu().numpy()
        wa = nufft.crop_scale(nufft.inverse_spectrum(nufft.spread(radial.adjoint(d, w.n_r), om, prm), prm), prm)
        ea, ma = rel_l2(va, wa), max_rel(va, wa)
        say(f"c5 item {i} N={n} K={w.K} vs oracle on {len(lines)} lines: fwd {ef:.2e} (max {mf:.2e}), "
            f"adj {ea:.2e} (max {ma:.2e})")
        assert max(ef, mf, ea, ma) < 1e-5
        p.close()
    # the small members against the oracle
    for i, w in enumerate(items):
        if w.N == 48 and w.n_phi <= 80:
            prm = nufft.Params(w.N, w.K, 6)
            x = xs[i].cpu().numpy().astype(complex)
            e = rel_l2(ref_out[i].cpu().numpy(), projector.forward(x, dirs[i], w.n_r, prm))
            say(f"c5 item {i} vs oracle {e:.2e}")
            assert e < 1e-5
            break

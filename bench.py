#!/usr/bin/env python3
"""Benchmark of the NUFFT derivative-Radon projector, forward + adjoint, on one GPU.

Workload (default): a 256^3 volume of 40 random ellipsoids plus Gaussian noise
(sigma 0.01), oversampled grid K = 512^3, J = 6 Kaiser-Bessel taps, radial
lines at 360 azimuths x 180 polar angles with 512 samples each
(M = 33,177,600 points), derivative + radial inverse DFT on.  One step = one
forward (volume -> derivative-Radon values) followed by one adjoint of that
output (-> volume), inputs resident in device memory.  Metric: Mpoints/s =
M / (time of one step).

Also reported (outside the timed region): the per-stage kernel times from HIP
events recorded on the launch stream during the timed steps, the roofline of
the dominant kernel, the FP32 path's relative L2 error against the full-FP64
GPU form and against the CPU FP64 oracle on a sample of lines, and the CPU
oracle's own throughput on that sample (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+adj NUFFT projector Mpts/s at 256³, rel-L2≤1e-4; FP32 vs FP64 form"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes(N, K, M, cb, touched):
    """Algorithmic HBM bytes per launch of each stage (cb = bytes per complex)."""
    fft = cb * (N ** 3 + 2 * N * N * K + 2 * N * K * K + K ** 3)
    return {
        "pad_fft": fft,                       # pruned passes, deapodization fused
        "interp": cb * (touched + M),          # touched grid cells once + M outputs
        "radial": 2 * cb * M,                  # read + write M
        "radial_adj": 2 * cb * M,
        "spread": cb * M,                      # read M (halo partials are not algorithmic)
        "ifft_crop": fft,
        "merge": cb * K ** 3,                  # write every grid cell once
    }


def alg_flops(M, J):
    """Algorithmic FP32 flops per launch of the point kernels: per point, J^3
    taps of a complex value times a real weight (2 FMA = 4 flop each), the
    separable row and plane sums (2 FMA per row of J and per plane), and 3J
    weight polynomials of degree 11 (11 FMA each)."""
    per_point = 4 * J ** 3 + 4 * J * J + 4 * J + 3 * J * 11 * 2
    return {"interp": per_point * M, "spread": per_point * M}


# ---------------------------------------------------------------------------
# rocprofv3 post-processing (summaries committed under profiles/)
KERNEL_SOURCES = {"interp": "k_grid_impl.h", "spread": "k_grid_impl.h", "merge": "k_grid_impl.h",
                  "radial": "k_fft_impl.h", "radial_adj": "k_fft_impl.h"}
KERNEL_NAMES = {"interp": "k_interp<", "spread": "k_spread<", "merge": "k_merge<",
                "radial": "k_radial<float, 512, false>", "radial_adj": "k_radial<float, 512, true>"}
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "hbm_traffic_c3.json")


def source_sha(fname):
    import hashlib
    path = os.path.join(ROOT, "paper_1605_05231_amd", "csrc", fname)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def _short(name):
    import re
    n = name.replace("void ", "")
    return (re.sub(r"\(.*$", "", n) if not n.startswith("at::") else n[:60])[:80]


def summarize_stats(csv_path):
    import csv
    print(f"{'kernel':80s} {'calls':>5s} {'avg_us':>10s} {'total_ms':>9s} {'pct':>6s}")
    for r in csv.DictReader(open(csv_path)):
        print(f"{_short(r['Name']):80s} {int(r['Calls']):5d} {float(r['AverageNs']) / 1e3:10.1f} "
              f"{float(r['TotalDurationNs']) / 1e6:9.2f} {float(r['Percentage']):6.2f}")


def summarize_counters(fetch_csv, write_csv):
    """Mean FETCH_SIZE / WRITE_SIZE (KiB per dispatch) per kernel, the copy-kernel
    scale factors (1 GiB read and written by one plain copy), and the scaled
    HBM traffic per launch; writes the traffic record used by the benchmark."""
    import collections
    import csv
    vals = {}
    for cname, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        agg = collections.OrderedDict()
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == cname:
                agg.setdefault(_short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
        vals[cname] = {k: sum(v) / len(v) for k, v in agg.items()}
    gib_kib = 1024.0 * 1024.0
    # the 1 GiB copies: the dispatch whose WRITE_SIZE is closest to 1 GiB, per copy kernel
    cands = {}
    for cname, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        for r in csv.DictReader(open(path)):
            k = _short(r["Kernel_Name"])
            if r["Counter_Name"] == cname and ("copyBuffer" in k or "manual_unroll<128, 4" in k):
                cands.setdefault((k, r["Dispatch_Id"]), {})[cname] = float(r["Counter_Value"])
    best = {}
    for (k, d), v in cands.items():
        if "WRITE_SIZE" in v and abs(v["WRITE_SIZE"] - gib_kib) < 0.05 * gib_kib:
            best[k] = v
    for k, v in best.items():
        print(f"# copy kernel {k}: FETCH {v.get('FETCH_SIZE', float('nan')):.1f} KiB, "
              f"WRITE {v['WRITE_SIZE']:.1f} KiB for 1 GiB read + 1 GiB written")
    ck = sorted(best)[0]
    f_fetch = gib_kib / best[ck]["FETCH_SIZE"]
    f_write = gib_kib / best[ck]["WRITE_SIZE"]
    print(f"# scale factors from {ck}: f_fetch {f_fetch:.3f}, f_write {f_write:.3f}")
    print(f"{'kernel':80s} {'FETCH_KiB':>12s} {'WRITE_KiB':>12s} {'scaled_GB':>10s}")
    rec = {"f_fetch": f_fetch, "f_write": f_write, "kernels": {}}
    for k in vals["FETCH_SIZE"]:
        fe, wr = vals["FETCH_SIZE"][k], vals["WRITE_SIZE"].get(k, float("nan"))
        gb = (fe * f_fetch + wr * f_write) * 1024 / 1e9
        print(f"{k:80s} {fe:12.1f} {wr:12.1f} {gb:10.4f}")
        for stage, kn in KERNEL_NAMES.items():
            if kn in k and "float" in k:
                rec["kernels"][stage] = {"fetch_kib": fe, "write_kib": wr, "traffic_bytes": gb * 1e9,
                                         "source": KERNEL_SOURCES[stage],
                                         "source_sha": source_sha(KERNEL_SOURCES[stage])}
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(rec, f, indent=1)


def traffic_for(stage):
    """Scaled HBM bytes per launch of `stage` if the committed counters were
    taken on the current kernel source, else None."""
    try:
        rec = json.load(open(TRAFFIC_JSON))["kernels"][stage]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("source_sha") != source_sha(rec["source"]):
        return None
    return rec["traffic_bytes"]


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on the host's cores.  It runs before the GPU is
# touched, so its worker processes are forked from a process without GPU state.
_ORACLE_CTX = {}


def _oracle_lines(lines):
    """Point stages of the oracle for a chunk of whole lines (worker process):
    interpolation, radial stage and its adjoint, spreading.  Returns the
    radial output of the chunk and its spread grid as sparse (index, value)."""
    import numpy as np
    from oracle import nufft, radial
    c = _ORACLE_CTX
    om = radial.points(c["dirs"][lines], c["n_r"])
    D = radial.forward(nufft.interpolate(c["Y"], om, c["prm"]), c["n_r"])
    g = nufft.spread(radial.adjoint(D, c["n_r"]), om, c["prm"]).reshape(-1)
    nz = np.flatnonzero(g)
    return D, nz, g[nz]


def oracle_fwd_adj(x, dirs, n_r, N, K, J, lines, workers):
    """One oracle forward (derivative-Radon values of `lines`) and the adjoint
    of that output: the oversampled FFT and its inverse on the full grid
    (scipy.fft with `workers` threads), the point stages of the lines split
    over `workers` forked processes.  Returns (seconds per part, D, volume)."""
    import multiprocessing as mp

    import numpy as np
    from oracle import nufft

    prm = nufft.Params(N, K, J)
    nufft.FFT_WORKERS = workers
    t = {}
    t0 = time.perf_counter()
    Y = nufft.oversampled_spectrum(x.astype(np.complex128), prm)
    t["fft"] = time.perf_counter() - t0
    _ORACLE_CTX.update(Y=Y, dirs=dirs, n_r=n_r, prm=prm)
    chunks = [c for c in np.array_split(np.asarray(lines), 4 * workers) if len(c)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_lines, chunks)
    t["points"] = time.perf_counter() - t0
    _ORACLE_CTX.clear()
    del Y
    t0 = time.perf_counter()
    grid = np.zeros(K ** 3, dtype=np.complex128)
    for _, nz, v in res:
        grid[nz] += v
    vol = nufft.crop_scale(nufft.inverse_spectrum(grid.reshape((K,) * 3), prm), prm)
    t["ifft_crop"] = time.perf_counter() - t0
    nufft.FFT_WORKERS = 1
    return t, np.concatenate([r[0] for r in res]), vol


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(W, sample_lines):
    """The oracle on all host cores (capped at 16, the host share of one GPU):
    the workload's full-grid transforms and `sample_lines` of its lines, scaled
    to all lines (a bounded sample), and for the c3 workload also c2 in full
    (median of 3).  Returns the cpu_baseline record and the sample's outputs."""
    import numpy as np

    import synthetic

    cores = min(len(os.sched_getaffinity(0)), 16)
    x = W.volume().astype(np.complex64)
    dirs = W.directions()
    L = len(dirs)
    ns = min(sample_lines, L)
    sample = np.unique(np.linspace(0, L - 1, ns).round().astype(int))
    log(f"[bench] CPU oracle ({cores} cores, {cpu_model()}) on {len(sample)} of {L} {W.name} lines ...")
    t, Ds, vs = oracle_fwd_adj(x, dirs, W.n_r, W.N, W.K, W.J, sample, cores)
    scale = L / len(sample)
    est = t["fft"] + t["ifft_crop"] + t["points"] * scale
    rec = {
        "value": round(W.M / est / 1e6, 4), "unit": "Mpts/s", "cores": cores, "kind": "oracle",
        "sample": f"{W.name}: oversampled FFT and inverse FFT in full ({t['fft']:.1f}s + "
                  f"{t['ifft_crop']:.1f}s, scipy.fft on {cores} threads); point stages on "
                  f"{len(sample)} of {L} lines ({len(sample) * W.n_r} points, {cores} processes, "
                  f"{t['points']:.1f}s) scaled by {scale:.1f}",
        "cpu_model": cpu_model(), "stage_s": {k: round(v, 3) for k, v in t.items()},
    }
    if W.name == "c3":
        W2 = synthetic.WORKLOADS["c2"]
        x2 = W2.volume().astype(np.complex64)
        d2 = W2.directions()
        runs = []
        for _ in range(3):
            t2, _, _ = oracle_fwd_adj(x2, d2, W2.n_r, W2.N, W2.K, W2.J, np.arange(len(d2)), cores)
            runs.append(sum(t2.values()))
        med = sorted(runs)[1]
        rec["c2_full"] = {"value": round(W2.M / med / 1e6, 4), "unit": "Mpts/s", "s_median_of_3": round(med, 3),
                          "runs_s": [round(r, 3) for r in runs]}
        log(f"[bench] CPU oracle c2 in full: {med:.2f}s -> {W2.M / med / 1e6:.3f} Mpts/s")
    log(f"[bench] CPU oracle {W.name} (sampled): {W.M / est / 1e6:.3f} Mpts/s")
    return rec, sample, Ds, vs


def bench_batch(args):
    """Batch of 64 volumes of uneven size (N in {48..160}, K = 2N, N_r = 2N,
    N_phi even in [60, 240], N_theta = N_phi / 2): forward + adjoint of every
    volume, captured once into two HIP graphs and replayed; metric = sum of
    the volumes' points / time of one forward + adjoint replay."""
    import numpy as np
    import torch

    import paper_1605_05231_amd as pkg
    import synthetic

    items = synthetic.batch_workload(64)
    t0 = time.perf_counter()
    vols = [w.volume() for w in items]
    log(f"[bench] c5: {len(items)} volumes, N in {sorted(set(w.N for w in items))}, "
        f"phantoms {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    batch = pkg.Batch([w.N for w in items], [w.K for w in items], 6,
                      [w.directions() for w in items], [w.n_r for w in items])
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    Ms = batch.Ms
    Mtot = int(sum(Ms))
    log(f"[bench] c5: sum M = {Mtot}, batch plans {plan_s:.2f}s")
    xs = [torch.from_numpy(v.astype(np.complex64)).cuda().reshape(-1) for v in vols]
    ys = [torch.empty(m, dtype=torch.complex64, device="cuda") for m in Ms]
    vs = [torch.empty(w.N ** 3, dtype=torch.complex64, device="cuda") for w in items]
    st = torch.cuda.Stream()  # graph capture needs a non-default stream
    with torch.cuda.stream(st):
        # eager (stream-ordered launches) for comparison
        for _ in range(args.warmup):
            batch.forward(xs, ys)
            batch.adjoint(ys, vs)
        st.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            batch.forward(xs, ys)
            batch.adjoint(ys, vs)
        st.synchronize()
        eager_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        batch.capture(0, xs, ys)
        batch.capture(1, ys, vs)
        for _ in range(args.warmup):
            batch.replay(0)
            batch.replay(1)
        st.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        t0 = time.perf_counter()
        for a, b in ev:
            a.record(st)
            batch.replay(0)
            batch.replay(1)
            b.record(st)
        st.synchronize()
        wall = time.perf_counter() - t0
    per = sorted(a.elapsed_time(b) for a, b in ev)
    ms = wall * 1e3 / args.steps
    value = Mtot / (ms * 1e-3) / 1e6
    log(f"[bench] c5 graph replay {ms:.3f} ms/step -> {value:.1f} Mpts/s (eager {eager_ms:.3f} ms)")
    q = lambda f: round(per[min(len(per) - 1, int(f * len(per)))], 4)
    print(json.dumps({
        "metric": "fwd+adj NUFFT projector Mpts/s, batch of 64 uneven volumes (graph replay)",
        "value": round(value, 2), "unit": "Mpts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c5: 64 volumes, N in {48, 64, 96, 128, 160}, K = 2N, J = 6 kb, "
                               "N_phi x N_phi/2 lines x 2N samples", "points": Mtot,
                   "step": "forward (derivative-Radon) + adjoint of every volume"},
        "step_ms": {"p10": q(0.1), "median": q(0.5), "p90": q(0.9)},
        "eager_ms_per_step": round(eager_ms, 4), "plan_s": round(plan_s, 2),
    }), flush=True)


def bench_recon(args):
    """Direct reconstruction (ramp + NUFFT transpose with angular quadrature):
    its speed at c3 (Mpts/s = M / time of one reconstruction from resident
    derivative-Radon data), then the angular-sampling experiment: a 64^3
    ellipsoid phantom projected on N_phi x N_phi/2 lines of 128 samples and
    reconstructed, error against the phantom as N_phi grows."""
    import numpy as np
    import torch

    import paper_1605_05231_amd as pkg
    import synthetic

    W = synthetic.WORKLOADS["c3"]
    N, K, J, n_r = W.N, W.K, W.J, W.n_r
    dirs = W.directions()
    M = W.M
    phi = synthetic.azimuths(W.n_phi)
    th = synthetic.polar_angles(W.n_theta)
    plan = pkg.Plan(N, K, J, dirs=dirs, n_r=n_r, dtype=torch.complex64)
    plan.set_line_weights(pkg.radial_quadrature(phi, th))
    x = torch.from_numpy(W.volume().astype(np.complex64)).cuda()
    d = plan.forward(x)
    v = torch.empty_like(x)
    for _ in range(args.warmup):
        plan.reconstruct(d, out=v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.reconstruct(d, out=v)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    xn = x.real.cpu().numpy()
    vr = v.real.cpu().numpy()
    err_c3 = float(np.linalg.norm(vr - xn) / np.linalg.norm(xn))
    log(f"[bench] e1: c3 reconstruction {ms:.3f} ms -> {M / (ms * 1e-3) / 1e6:.1f} Mpts/s, "
        f"rel-L2 vs phantom {err_c3:.3e}")
    del plan, x, d, v
    torch.cuda.empty_cache()

    # angular-sampling experiment (Section 3.1, here in 3D): error vs lines
    Ne, ne_r = 64, 128
    xe = synthetic.ellipsoid_phantom(Ne, 20, 3100)
    xt = torch.from_numpy(xe.astype(np.complex64)).cuda()
    curve = []
    for n_phi in (16, 24, 32, 48, 64, 96, 128, 160, 200, 256):
        ph = synthetic.azimuths(n_phi)
        tt = synthetic.polar_angles(n_phi // 2)
        dr = synthetic.line_directions(ph, tt)
        p = pkg.Plan(Ne, 2 * Ne, 6, dirs=dr, n_r=ne_r, dtype=torch.complex64)
        p.set_line_weights(pkg.radial_quadrature(ph, tt))
        rec = p.reconstruct(p.forward(xt)).real.cpu().numpy()
        mean_abs = float(np.mean(np.abs(rec - xe)))
        rel = float(np.linalg.norm(rec - xe) / np.linalg.norm(xe))
        curve.append({"n_phi": n_phi, "n_theta": n_phi // 2, "lines": len(dr),
                      "mean_abs_err_per_voxel": mean_abs, "rel_l2": rel})
        log(f"[bench] e1: N_phi {n_phi:4d} lines {len(dr):6d}: mean |err| {mean_abs:.4e}, rel-L2 {rel:.4e}")
        p.close()
    print(json.dumps({
        "metric": "direct reconstruction (ramp + NUFFT transpose) Mpts/s at 256³",
        "value": round(M / (ms * 1e-3) / 1e6, 2), "unit": "Mpts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c3 reconstruction from its own derivative-Radon data; "
                               "angular sampling experiment: 64^3 phantom, N_phi x N_phi/2 lines x 128",
                   "points": M},
        "c3_rel_l2_vs_phantom": err_c3,
        "angular_sampling": curve,
    }), flush=True)


def bench_umbrella(args):
    """Radial -> umbrella resampling (method 2, eq 2.15) at the 128^3 set-up of
    the cone-beam experiment: the c2 projector output (180 x 90 lines x 256)
    resampled onto 256 projections x 256 x 256 detector lines; Msamples/s =
    umbrella samples / time of one resampling, for J = 3 (the paper's) and 6;
    then method 1 (eq 2.11) at J = 6 with its grid step and gather timed apart."""
    import numpy as np
    import torch

    import paper_1605_05231_amd as pkg
    import synthetic

    W = synthetic.WORKLOADS["c2"]
    N, K, J, n_r = W.N, W.K, W.J, W.n_r
    phi = synthetic.azimuths(W.n_phi)
    th = synthetic.polar_angles(W.n_theta)
    plan = pkg.Plan(N, K, J, dirs=W.directions(), n_r=n_r, dtype=torch.complex64)
    d = plan.forward(torch.from_numpy(W.volume().astype(np.complex64)).cuda()).reshape(-1)
    torch.cuda.synchronize()
    n_proj = n_alpha = n_t = 2 * N
    P = n_proj * n_alpha * n_t
    res = {}
    for Ju in (3, 6):
        u = pkg.Umbrella(N, n_proj, n_alpha, n_t, W.n_phi, W.n_theta, n_r, th[0], th[1] - th[0], J=Ju)
        out = torch.empty((n_proj, n_alpha, n_t), dtype=torch.complex64, device="cuda")
        for _ in range(args.warmup):
            u.resample(d, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            u.resample(d, out=out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        res[Ju] = ms
        log(f"[bench] umbrella J={Ju}: {ms:.3f} ms -> {P / (ms * 1e-3) / 1e6:.1f} Msamples/s")
        u.close()
    # method 1 (eq 2.11): the grid step (three in-place axis passes) and the
    # J^3 gather, timed apart with events on the stream they run on
    u1 = pkg.Umbrella(N, n_proj, n_alpha, n_t, W.n_phi, W.n_theta, n_r, th[0], th[1] - th[0], J=6,
                      method=1)
    out = torch.empty((n_proj, n_alpha, n_t), dtype=torch.complex64, device="cuda")
    grid = torch.empty(u1.grid_shape, dtype=torch.complex64, device="cuda")
    for _ in range(args.warmup):
        u1.resample(d, out=out)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_grid = t_gather = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        u1.resample(d, out=out)
    torch.cuda.synchronize()
    ms1 = (time.perf_counter() - t0) * 1e3 / args.steps
    for _ in range(args.steps):
        ev[0].record()
        u1.stage("grid", d, out=grid)
        ev[1].record()
        u1.stage("gather", grid, out=out)
        ev[2].record()
        torch.cuda.synchronize()
        t_grid += ev[0].elapsed_time(ev[1])
        t_gather += ev[1].elapsed_time(ev[2])
    t_grid /= args.steps
    t_gather /= args.steps
    n_in = W.n_phi * W.n_theta * n_r
    grid_bytes = 21 * 8 * n_in  # input once, then 2+4+8 times it written and 2+4 read
    log(f"[bench] umbrella method 1 J=6: {ms1:.3f} ms -> {P / (ms1 * 1e-3) / 1e6:.1f} Msamples/s; "
        f"grid step {t_grid:.3f} ms ({grid_bytes / (t_grid * 1e-3) / 1e9:.0f} GB/s algorithmic), "
        f"gather {t_gather:.3f} ms")
    u1.close()
    print(json.dumps({
        "metric": "radial-to-umbrella resampling (method 2) Msamples/s at 128³",
        "value": round(P / (res[6] * 1e-3) / 1e6, 2), "unit": "Msamples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(res[6], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c2 derivative-Radon values (180 x 90 lines x 256) -> 256 projections "
                               "x 256 x 256 umbrella planes, J = 6", "samples": P},
        "J3_ms": round(res[3], 4),
        "method1": {
            "ms": round(ms1, 4), "Msamples_s": round(P / (ms1 * 1e-3) / 1e6, 2), "J": 6,
            "grid_ms": round(t_grid, 4), "gather_ms": round(t_gather, 4),
            "grid_cells": int(u1.grid_shape[0] * u1.grid_shape[1] * u1.grid_shape[2]),
            "roofline_grid": {"bound": "hbm", "alg_bytes": grid_bytes,
                              "achieved": round(grid_bytes / (t_grid * 1e-3) / 1e9, 1), "peak": 8000.0,
                              "unit": "GB/s", "frac": round(grid_bytes / (t_grid * 1e-3) / 8e12, 4)},
        },
    }), flush=True)


def bench_cone(args):
    """The complete NUFFT cone-beam forward projector at the set-up of the
    paper's projector experiment (Section 3.2): a 128^3 volume -> derivative-
    Radon values on 256 x 256 lines x 256 samples (module 1; polar angles at
    the midpoints of 256 bins of [0, pi], so no cap is left unsampled) ->
    256 projections x 256 detector-line angles x 128 offsets (step 2, method 2
    at the paper's [3 3 3] and at J = 6, and method 1 at J = 6) -> 256
    cone-beam projections of 128 x 128 pixels (step 3, [5 5]).  Projections/s
    = 256 / the time of one projector call from the resident volume.  The
    paper's Matlab runs (hardware not stated) took about 44 s (method 2) and
    56.6 s (method 1) for this set-up: context, not a target."""
    import math

    import numpy as np
    import torch

    import paper_1605_05231_amd as pkg
    import synthetic

    N, K, J = 128, 256, 6
    n_phi = n_th = n_r = 256
    n_proj, n_alpha, n_det = 256, 256, 128
    phi = synthetic.azimuths(n_phi)
    th = synthetic.polar_angles(n_th, margin=math.pi / (2 * n_th))
    W = synthetic.WORKLOADS["c2"]
    x = torch.from_numpy(W.volume().astype(np.complex64)).cuda()
    dirs = synthetic.line_directions(phi, th)
    if not args.no_autotune:
        pkg.autotune(N, K, J, dirs, n_r, dtype=torch.complex64)
    plan = pkg.Plan(N, K, J, dirs=dirs, n_r=n_r, dtype=torch.complex64)
    d = torch.empty(n_phi * n_th * n_r, dtype=torch.complex64, device="cuda")
    U = torch.empty((n_proj, n_alpha, n_det), dtype=torch.complex64, device="cuda")
    X = torch.empty((n_proj, n_det, n_det), dtype=torch.complex64, device="cuda")
    g = pkg.Grangeat(N, n_proj, n_alpha, n_det)
    res = {}
    for label, method, Ju in (("method2_J3", 2, 3), ("method2_J6", 2, 6), ("method1_J6", 1, 6)):
        u = pkg.Umbrella(N, n_proj, n_alpha, n_det, n_phi, n_th, n_r, th[0], th[1] - th[0], J=Ju,
                         method=method)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        for _ in range(args.warmup):
            plan.forward(x, out=d)
            u.resample(d, out=U)
            g.project(U, out=X)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.forward(x, out=d)
            u.resample(d, out=U)
            g.project(U, out=X)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        st = np.zeros(3)
        for _ in range(args.steps):
            ev[0].record()
            plan.forward(x, out=d)
            ev[1].record()
            u.resample(d, out=U)
            ev[2].record()
            g.project(U, out=X)
            ev[3].record()
            torch.cuda.synchronize()
            st += [ev[i].elapsed_time(ev[i + 1]) for i in range(3)]
        st /= args.steps
        res[label] = {"ms": round(ms, 4), "projections_s": round(n_proj / (ms * 1e-3), 1),
                      "stage_ms": {"module1": round(st[0], 4), "resample": round(st[1], 4),
                                   "grangeat": round(st[2], 4)}}
        log(f"[bench] cone {label}: {ms:.3f} ms per projector call -> {n_proj / (ms * 1e-3):.0f} "
            f"projections/s (module 1 {st[0]:.3f}, resampling {st[1]:.3f}, Grangeat {st[2]:.3f} ms)")
        u.close()
    main_ = res["method2_J3"]
    print(json.dumps({
        "metric": "complete NUFFT cone-beam forward projector, projections/s at 128³",
        "value": main_["projections_s"], "unit": "projections/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "128^3 ellipsoid volume -> 256 x 256 lines x 256 samples (K = 256, J = 6) "
                               "-> 256 x 256 x 128 umbrella planes (method 2, J = 3) -> 256 projections "
                               "of 128 x 128 (J = 5)", "projections": n_proj},
        "variants": res,
        "paper_context_s": {"method2_matlab": 44.0, "method1_matlab": 56.596,
                            "note": "the paper's Matlab runs of its projector at this set-up; hardware "
                                    "not stated"},
    }), flush=True)
    plan.close()
    g.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=["c2", "c3", "c5", "e1", "umbrella", "cone"],
                    help="c5: batch of 64 uneven volumes, replayed from HIP graphs; e1: direct "
                         "reconstruction at c3 and the angular-sampling experiment (own JSON lines)")
    ap.add_argument("--kernel", default="kb", choices=["kb", "minmax"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the tiling autotuner (defaults: tile 16, 4096 points per task)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-form comparison")
    ap.add_argument("--tile", type=int, default=0, help="with --no-autotune: tile edge (8 or 16)")
    ap.add_argument("--max-pts", type=int, default=0, help="with --no-autotune: points per task")
    ap.add_argument("--cpu-sample-lines", type=int, default=3240)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--summarize-stats", metavar="KERNEL_STATS_CSV",
                    help="print a summary of a rocprofv3 --stats kernel table and exit")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarize two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) and exit")
    args = ap.parse_args()
    if args.summarize_stats:
        summarize_stats(args.summarize_stats)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the projector runs "
              "on a single MI355X and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import synthetic

    cpu = None
    if not args.no_cpu_baseline and args.workload in ("c2", "c3") and args.kernel == "kb":
        # before any GPU call: its worker processes are forked from this one
        cpu = cpu_baseline(synthetic.WORKLOADS[args.workload], args.cpu_sample_lines)

    import torch

    import paper_1605_05231_amd as pkg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "c5":
        bench_batch(args)
        return
    if args.workload == "e1":
        bench_recon(args)
        return
    if args.workload == "umbrella":
        bench_umbrella(args)
        return
    if args.workload == "cone":
        bench_cone(args)
        return
    W = synthetic.WORKLOADS[args.workload]
    N, K, J, n_r = W.N, W.K, W.J, W.n_r
    dirs = W.directions()
    M = W.M
    log(f"[bench] workload {W.name}: N={N} K={K} J={J} lines={len(dirs)} n_r={n_r} M={M}")
    t0 = time.perf_counter()
    x_np = W.volume()
    log(f"[bench] phantom {time.perf_counter() - t0:.1f}s")

    tune = None
    # explicit tiling (read by the library when a plan is created)
    if args.tile:
        os.environ["NUFFTCT_TILE"] = str(args.tile)
    if args.max_pts:
        os.environ["NUFFTCT_MAXPTS"] = str(args.max_pts)
    if not args.no_autotune and not (args.tile or args.max_pts):
        t0 = time.perf_counter()
        tune = pkg.autotune(N, K, J, dirs, n_r, kernel=args.kernel)
        log(f"[bench] autotune {tune} in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    plan = pkg.Plan(N, K, J, dirs=dirs, n_r=n_r, kernel=args.kernel, dtype=torch.complex64)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    log(f"[bench] plan {plan_s:.2f}s")

    if args.copy_calibration:
        import ctypes
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)  # torch's elementwise copy kernel
        torch.cuda.synchronize()
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_int, ctypes.c_void_p]
        rc = hip.hipMemcpyAsync(dst.data_ptr(), src.data_ptr(), 1 << 30, 3,  # device to device
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        del src, dst
        log(f"[bench] copy calibration: two 1 GiB device copies (torch kernel, hipMemcpyAsync rc={rc})")

    x = torch.from_numpy(x_np.astype(np.complex64)).cuda()
    D = torch.empty((len(dirs), n_r), dtype=torch.complex64, device="cuda")
    V = torch.empty((N, N, N), dtype=torch.complex64, device="cuda")

    def step():
        plan.forward(x, out=D)
        plan.adjoint(D, out=V)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.stage_times()  # clear
    plan.set_timing(True)
    torch.cuda.synchronize()
    cur = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(cur)
        step()
        b.record(cur)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.set_timing(False)
    per = sorted(a.elapsed_time(b) for a, b in ev)
    step_ms = {"p10": round(per[int(0.1 * len(per))], 4), "median": round(per[len(per) // 2], 4),
               "p90": round(per[min(len(per) - 1, int(0.9 * len(per)))], 4)}
    st = plan.stage_times()
    ms_per_step = wall * 1e3 / args.steps
    value = M / (ms_per_step * 1e-3) / 1e6
    log(f"[bench] {ms_per_step:.3f} ms/step -> {value:.1f} Mpts/s")
    stage_avg = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in st.items()}
    log("[bench] stage avg ms: " + ", ".join(f"{k}={v:.3f}" for k, v in stage_avg.items()))

    # touched grid cells: spread positive weights of all-ones input and count nonzeros
    ones = torch.ones(M, dtype=torch.complex64, device="cuda")
    grid = torch.empty(K ** 3, dtype=torch.complex64, device="cuda")
    plan.stage(pkg.STAGE_SPREAD, ones, grid)
    touched = int(torch.count_nonzero(grid.real).item())
    del grid, ones
    ab = alg_bytes(N, K, M, 8, touched)
    af = alg_flops(M, J)
    single = ["interp", "spread", "merge", "radial", "radial_adj"]
    dom = max(single, key=lambda k: stage_avg[k])
    tr = traffic_for(dom)
    # every stage is priced against HBM with its algorithmic bytes (nothing on
    # the path is a dense contraction); the point kernels also carry the view
    # against the FP32 vector peak
    achieved = ab[dom] / (stage_avg[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if tr is None else round(tr),
                "alg_bytes_per_launch": ab[dom], "avg_launch_ms": round(stage_avg[dom], 4)}
    if dom in af:
        alu = af[dom] / (stage_avg[dom] * 1e-3) / 1e12
        roofline["alu_view"] = {"achieved": round(alu, 2), "peak": FP32_VECTOR_PEAK_TFLOPS,
                                "unit": "TFLOP/s", "frac": round(alu / FP32_VECTOR_PEAK_TFLOPS, 4),
                                "alg_flops_per_launch": af[dom]}
    # the spreading stage (halo partials + merge) and the whole step against HBM
    a3_bytes = 8 * M + 8 * K ** 3
    a3_ms = stage_avg["spread"] + stage_avg["merge"]
    step_bytes = sum(ab[k] for k in ("pad_fft", "interp", "radial", "radial_adj", "ifft_crop")) + a3_bytes
    roofline["a3_stage"] = {"alg_bytes": a3_bytes, "ms": round(a3_ms, 4),
                            "frac": round(a3_bytes / (a3_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    roofline["step"] = {"alg_bytes": step_bytes, "ms": round(ms_per_step, 4),
                        "frac": round(step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        "ceiling_Mpts_s": round(M / (step_bytes / (HBM_PEAK_GBS * 1e9)) / 1e6, 1)}
    stages = {k: {"avg_ms": round(stage_avg[k], 4),
                  "alg_GBps": round(ab[k] / (stage_avg[k] * 1e-3) / 1e9, 1) if stage_avg[k] and ab[k] else None}
              for k in stage_avg}

    result = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{W.name}: {N}^3 volume, K={K}^3, J={J} {args.kernel}, "
                               f"{W.n_phi}x{W.n_theta} lines x {n_r} samples",
                   "N": N, "K": K, "J": J, "kernel": args.kernel, "points": M,
                   "step": "forward (derivative-Radon) + adjoint"},
        "roofline": roofline,
        "step_ms": step_ms,
        "stages": stages,
        "touched_cells": touched,
        "plan_s": round(plan_s, 2),
        "tiling": tune or "default",
    }

    # FP64 form: speed and the FP32 path's error against it
    if not args.no_fp64:
        del plan
        torch.cuda.empty_cache()
        D32 = D.clone()
        V32 = V.clone()
        del D, V
        p64 = pkg.Plan(N, K, J, dirs=dirs, n_r=n_r, kernel=args.kernel, dtype=torch.complex128)
        x64 = torch.from_numpy(x_np.astype(np.complex128)).cuda()
        D64 = p64.forward(x64)
        V64 = p64.adjoint(D64)
        # the FP32 adjoint above consumed the FP32 forward's output; compare like with like
        V64_from32 = p64.adjoint(D32.to(torch.complex128))
        torch.cuda.synchronize()
        n64 = max(2, args.steps // 4)
        t0 = time.perf_counter()
        for _ in range(n64):
            p64.forward(x64, out=D64)
            p64.adjoint(D64, out=V64)
        torch.cuda.synchronize()
        ms64 = (time.perf_counter() - t0) * 1e3 / n64
        d = (D32.to(torch.complex128) - D64)
        ef = float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(D64))
        mf = float(d.abs().max() / D64.abs().max())
        va = (V32.to(torch.complex128) - V64_from32)
        ea = float(torch.linalg.vector_norm(va) / torch.linalg.vector_norm(V64_from32))
        ma = float(va.abs().max() / V64_from32.abs().max())
        result["fp64_form"] = {"value": round(M / (ms64 * 1e-3) / 1e6, 2), "ms_per_step": round(ms64, 3),
                               "speedup_fp32_over_fp64": round(ms64 / ms_per_step, 2)}
        result["accuracy_vs_fp64_form"] = {"fwd_rel_l2": ef, "fwd_max_rel": mf,
                                           "adj_rel_l2": ea, "adj_max_rel": ma}
        log(f"[bench] FP64 form {ms64:.2f} ms/step; FP32 vs FP64 fwd {ef:.2e} adj {ea:.2e}")
        del p64, x64, D64, V64, V64_from32, d, va
        torch.cuda.empty_cache()
        D, V = D32, V32

    if cpu is not None:
        rec, sample, Ds, vs = cpu
        rec["gpu_speedup"] = round(value / rec["value"], 1)
        result["cpu_baseline"] = rec
        # parity on the sample: forward lines and the adjoint of those lines alone
        L = len(dirs)
        sel = torch.from_numpy(sample).cuda()
        Dg = D.reshape(L, n_r)[sel].cpu().numpy().reshape(-1)
        ef = float(np.linalg.norm(Dg - Ds) / np.linalg.norm(Ds))
        mf = float(np.max(np.abs(Dg - Ds)) / np.max(np.abs(Ds)))
        Din = torch.zeros((L, n_r), dtype=torch.complex64, device="cuda")
        Din[sel] = torch.from_numpy(Ds.reshape(-1, n_r).astype(np.complex64)).cuda()
        p32 = pkg.Plan(N, K, J, dirs=dirs, n_r=n_r, kernel=args.kernel, dtype=torch.complex64)
        vg = p32.adjoint(Din).cpu().numpy()
        ea = float(np.linalg.norm(vg - vs) / np.linalg.norm(vs))
        ma = float(np.max(np.abs(vg - vs)) / np.max(np.abs(vs)))
        result["accuracy_vs_oracle_sample"] = {"fwd_rel_l2": ef, "fwd_max_rel": mf, "adj_rel_l2": ea,
                                               "adj_max_rel": ma, "lines": int(len(sample))}
        log(f"[bench] oracle sample: fwd {ef:.2e} (max {mf:.2e}) adj {ea:.2e} (max {ma:.2e})")

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

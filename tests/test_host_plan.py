"""The library's host-side plan logic, on the CPU, against the oracle and its
own invariants: the harness tests/host_check.cpp is built from the library's
host_plan.cpp and tables.cpp with g++ under the address and undefined-behaviour
sanitizers (any report fails the run), then

  * the neighbour rule's first taps equal the oracle's (kernels.neighbours:
    k0 = floor(t - J/2), first tap k0 + 1, centred and wrapped) bit for bit,
    on radial geometries full of near-ties (K = n_r, directions with
    components 1/2 and 1, the rounding cases where t - J/2 enters a coarser
    binade) and on adversarial explicit points (+-pi, 0, just beyond negative
    integers);
  * the binning is a partition: both point orders are permutations, every
    task lies in its bin and holds at most max_pts points, the interpolation
    and spreading orders hold the same points per task, bin task offsets are
    consistent, and the pairs of the spreading order share their first cell;
  * the deapodization, twiddle, Kaiser-Bessel and min-max tables equal the
    oracle's FP64 values (Section 2.1.3, eq 2.10-2.11; min-max to the
    accuracy of the oracle's own FP64 solve).
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import synthetic
from oracle import kernels, radial

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1605_05231_amd", "csrc")


@pytest.fixture(scope="module")
def harness():
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tempfile.mkdtemp(prefix="host_check_")
    exe = os.path.join(d, "host_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-Wno-unknown-pragmas",
           os.path.join(HERE, "host_check.cpp"), os.path.join(CSRC, "host_plan.cpp"),
           os.path.join(CSRC, "tables.cpp"), "-o", exe, "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def run(exe, *, K, J, N, geom, n_r=0, radial_plan=False, tile=16, max_pts=4096, fp32=True,
        pair_spread=True, twins=None, beta=None, fracs=(0.0, 0.25, 0.5, 0.999)):
    twins = pair_spread if twins is None else twins
    beta = kernels.default_beta(J) if beta is None else beta
    geom = np.ascontiguousarray(np.asarray(geom, dtype=np.float64).reshape(-1, 3))
    M = geom.shape[0] * n_r if radial_plan else geom.shape[0]
    fr = np.asarray(fracs, dtype=np.float64)
    hdr = np.array([M, K, J, tile, max_pts, n_r, int(radial_plan), int(fp32), int(pair_spread),
                    int(twins), geom.shape[0], N, len(fr)], dtype=np.int64)
    with tempfile.TemporaryDirectory() as d:
        fi, fo = os.path.join(d, "in"), os.path.join(d, "out")
        with open(fi, "wb") as f:
            f.write(hdr.tobytes() + np.float64(beta).tobytes() + geom.tobytes() + fr.tobytes())
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe, fi, fo], capture_output=True, text=True, env=env)
        assert r.returncode == 0, f"harness failed ({r.returncode}):\n{r.stderr[-4000:]}"
        buf = open(fo, "rb").read()
    o = 0

    def take(dtype, n):
        nonlocal o
        a = np.frombuffer(buf, dtype=dtype, count=n, offset=o)
        o += a.nbytes
        return a

    nb = K // tile
    out = {"first": take(np.int32, 3 * M).reshape(M, 3), "perm": take(np.int32, M),
           "perm_s": take(np.int32, M)}
    nt = int(take(np.int64, 1)[0])
    out["tasks"] = take(np.int32, 5 * nt).reshape(nt, 5)
    out["bin_tasks"] = take(np.int32, nb ** 3 + 1)
    out["s"] = take(np.float64, N)
    out["tw"] = take(np.float64, 2 * K)
    out["psi"] = take(np.float64, J * len(fr)).reshape(len(fr), J)
    mm = take(np.float64, 2 * J * len(fr)).reshape(len(fr), J, 2)
    out["mm"] = mm[..., 0] + 1j * mm[..., 1]
    assert o == len(buf)
    out.update(M=M, nb=nb, tile=tile, max_pts=max_pts, J=J, K=K, N=N, fracs=fr, beta=beta,
               twins=twins)
    return out


def oracle_first(om, K, J):
    cols = []
    for d in range(3):
        kappa, _ = kernels.neighbours(om[:, d], K, J)
        cols.append(np.mod(kappa[:, 0] + K // 2, K))
    return np.stack(cols, axis=1)


def check_binning(o, om, pair_spread):
    M, nb, T, J = o["M"], o["nb"], o["tile"], o["J"]
    first = o["first"].astype(np.int64)
    key = ((first[:, 0] // T) * nb + first[:, 1] // T) * nb + first[:, 2] // T
    for name in ("perm", "perm_s"):
        assert np.array_equal(np.sort(o[name]), np.arange(M)), name
    tasks, bt = o["tasks"], o["bin_tasks"]
    assert bt[0] == 0 and bt[-1] == len(tasks) and np.all(np.diff(bt) >= 0)
    pos = 0
    n_twins = n_same = 0
    for k, (b, start, count, npairs, ntwins) in enumerate(tasks):
        assert bt[b] <= k < bt[b + 1]
        assert start == pos and 0 < count <= o["max_pts"]
        pos += count
        seg_s = o["perm_s"][start:start + count]
        seg_i = o["perm"][start:start + count]
        assert np.all(key[seg_s] == b)
        assert np.array_equal(np.sort(seg_s), np.sort(seg_i))
        # (without paired spreading, the only pairs are twins)
        assert 2 * npairs <= count and (pair_spread or npairs == (ntwins if o["twins"] else 0))
        p = seg_s[:2 * npairs].reshape(-1, 2)
        assert np.array_equal(first[p[:, 0]], first[p[:, 1]])
        # interpolation units: the first ntwins entry pairs sample one
        # frequency twice, and they are exactly the spreading pairs that do
        same = np.max(np.abs(om[p[:, 0]] - om[p[:, 1]]), axis=1) <= 1e-12 * np.maximum(
            1.0, np.max(np.abs(om[p[:, 0]]), axis=1))
        n_same += int(same.sum())
        assert 2 * ntwins <= count and (o["twins"] or ntwins == 0)
        tw = seg_i[:2 * ntwins].reshape(-1, 2)
        assert np.array_equal(first[tw[:, 0]], first[tw[:, 1]])
        assert np.all(np.abs(om[tw[:, 0]] - om[tw[:, 1]]) <= 1e-12 * np.maximum(1.0, np.abs(om[tw[:, 0]])))
        if o["twins"]:
            assert np.all(same[:ntwins])  # twins first
            assert ntwins == same.sum() and not np.any(same[ntwins:])
            want = {frozenset(q) for q in p[same].tolist()}
            assert {frozenset(q) for q in tw.tolist()} == want
        n_twins += int(ntwins)
    assert pos == M
    return n_twins, n_same


TIE_CASES = [
    # (name, N, K, J, n_phi, n_theta, n_r): K = n_r puts t on (half-)integers
    ("k192_j6_ties", 96, 192, 6, 6, 3, 192),
    ("k48_j6_fewlines", 24, 48, 6, 5, 5, 48),
    ("k64_j7_odd", 32, 64, 7, 8, 4, 64),
    ("k96_j5", 48, 96, 5, 12, 6, 96),
]


@pytest.mark.parametrize("case", TIE_CASES, ids=[c[0] for c in TIE_CASES])
def test_first_taps_and_binning_radial(harness, case):
    name, N, K, J, nphi, nth, n_r = case
    dirs = synthetic.line_directions(synthetic.azimuths(nphi), synthetic.polar_angles(nth))
    om = radial.points(dirs, n_r)
    for tile, max_pts in ((16, 4096), (8, 256)):
        if K % tile:
            continue
        o = run(harness, K=K, J=J, N=N, geom=dirs, n_r=n_r, radial_plan=True, tile=tile,
                max_pts=max_pts)
        assert np.array_equal(o["first"], oracle_first(om, K, J)), name
        n_twins, _ = check_binning(o, om, True)
        # without paired spreading (min-max weights) the interpolation still
        # takes the same twins
        o2 = run(harness, K=K, J=J, N=N, geom=dirs, n_r=n_r, radial_plan=True, tile=tile,
                 max_pts=max_pts, pair_spread=False, twins=True)
        assert check_binning(o2, om, False)[0] == n_twins
        # lines (phi, theta) and (phi + pi, pi - theta) sample the same
        # frequencies in opposite order; the twins that can share an
        # interpolation are those whose first taps agree (a tie can split
        # them): nearly all of these must be found (a task boundary can
        # split a few)
        first = oracle_first(om, K, J)
        groups = {}
        for i, (qq, ff) in enumerate(zip(np.round(np.ldexp(om, 30)).astype(np.int64), first)):
            groups.setdefault((tuple(qq), tuple(ff)), []).append(i)
        possible = sum(len(v) // 2 for v in groups.values())
        assert 0.95 * possible <= n_twins <= possible, (n_twins, possible)
        if nphi % 2 == 0 and name != "k192_j6_ties":
            assert n_twins >= 0.45 * len(om)


def test_first_taps_explicit_adversarial_points(harness):
    K, J, N = 64, 6, 32
    g = 2 * math.pi / K
    rng = np.random.default_rng(5)
    ts = np.array([-3.0000000000000004, -2.0000000000000004, -1.0000000000000002, -5.000000000000001,
                   -3.9999999999999996, 0.0, 1e-17, -1e-17, 31.999999999999996, -32.0])
    pts = np.concatenate([
        np.stack([ts * g, np.roll(ts, 3) * g, np.roll(ts, 7) * g], axis=1),
        np.array([[-math.pi] * 3, [math.pi] * 3, [math.pi - 1e-12, -math.pi, 0.0]]),
        rng.uniform(-math.pi, math.pi, (2000, 3)),
        np.round(rng.uniform(-30, 30, (500, 3))) * g,  # exact ties
    ])
    for fp32, pair_spread in ((True, True), (False, False), (True, False)):
        o = run(harness, K=K, J=J, N=N, geom=pts, fp32=fp32, pair_spread=pair_spread,
                max_pts=300)
        assert np.array_equal(o["first"], oracle_first(pts, K, J))
        check_binning(o, pts, pair_spread)


@pytest.mark.parametrize("N,K,J", [(32, 64, 6), (48, 96, 4), (40, 80, 7), (16, 32, 8)])
def test_tables_match_oracle(harness, N, K, J):
    dirs = np.array([[0.0, 0.0, 1.0]])
    o = run(harness, K=K, J=J, N=N, geom=dirs, n_r=16, radial_plan=True)
    beta = o["beta"]
    s = kernels.deapod(N, K, J, beta)
    assert np.max(np.abs(o["s"] - s) / np.abs(s)) < 1e-13
    # twiddles against 40-digit values: the library rounds once, to within
    # half an ulp of each component
    import mpmath
    mpmath.mp.dps = 40
    ref = [mpmath.expjpi(-2 * mpmath.mpf(k) / K) for k in range(K)]
    err = max(max(abs(mpmath.mpf(o["tw"][2 * k]) - mpmath.re(ref[k])),
                  abs(mpmath.mpf(o["tw"][2 * k + 1]) - mpmath.im(ref[k]))) for k in range(K))
    assert float(err) <= 2.0 ** -53
    # the Kaiser-Bessel kernel (scipy's FP64 I0 in the oracle, a long-double
    # series in the library)
    u = J / 2 - 1 - np.arange(J)[None, :] + o["fracs"][:, None]
    assert np.max(np.abs(o["psi"] - kernels.kb_psi(u, J, beta))) < 1e-14
    mm = kernels.minmax_coeffs(u, N, K, s)
    T = kernels.minmax_T(N, K, J, s)
    tol = 8 * np.linalg.cond(T) * np.finfo(float).eps
    err = np.max(np.abs(o["mm"] - mm)) / np.max(np.abs(mm))
    assert err < tol, (err, tol)

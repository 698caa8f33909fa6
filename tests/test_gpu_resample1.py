"""GPU parity of the radial -> umbrella resampling, method 1 (eq 2.11), with
the oracle: the grid step (F P F^-1 on the K grid) element by element, the
gather step (T_sparse) on the oracle's own grid, the whole resampling, the
closed form of a centred Gaussian on umbrella planes, and the full 128^3
set-up of the cone-beam experiment (180 x 90 lines x 256 -> 256 projections
x 256 x 256 detector lines) on every grid cell and on sampled planes.

Umbrella samples whose grid coordinate 2 t - J/2 lies within 1e-7 of an
integer on some axis sit where the neighbour rule switches tap sets: there
the two FP64 geometry computations (oracle and kernel) may round to
different sides, both results are correct, and they differ by up to the
Kaiser-Bessel kernel's edge value.  Those samples are compared at a bar
that covers that jump; every other sample at the precision's bar."""
import numpy as np
import pytest

import synthetic
from oracle import kernels, resample1, umbrella
from tests.gpu_util import max_rel, rel_l2, require_gpu, say, to_dev, to_host

pytestmark = pytest.mark.gpu

BAR = {"f32": 5e-6, "f64": 1e-12}


def _dtype(prec):
    import torch
    return torch.complex64 if prec == "f32" else torch.complex128


def _setup(N, n_proj, n_alpha, n_t, n_phi, n_th, n_r, J, prec, seed):
    import paper_1605_05231_amd as pkg
    th = synthetic.polar_angles(n_th)
    th0, dth = th[0], th[1] - th[0]
    u = pkg.Umbrella(N, n_proj, n_alpha, n_t, n_phi, n_th, n_r, th0, dth, J=J,
                     dtype=_dtype(prec), method=1)
    rng = np.random.default_rng(seed)
    D = rng.standard_normal((n_phi, n_th, n_r)) + 1j * rng.standard_normal((n_phi, n_th, n_r))
    if prec == "f32":
        D = D.astype(np.complex64).astype(np.complex128)
    nh, rq = umbrella.geometry(N, n_proj, n_alpha, n_t)
    tq, pq = umbrella.angles(nh)
    t = resample1.index_coords(n_phi, th0, dth, n_r, tq, pq, rq)
    return u, D, t


def _near_tie(t, J, eps=1e-7):
    s = 2.0 * t - J / 2.0
    d = np.abs(s - np.round(s))
    return np.any(d < eps, axis=1)


def _weight_sum(J):
    """S: the largest sum of one axis's J tap weights over all offsets."""
    beta = kernels.default_beta(J)
    fr = np.linspace(0.0, 1.0, 1001)
    return max(float(np.sum(kernels.kb_psi(J / 2.0 - np.arange(1, J + 1) + f, J, beta))) for f in fr)


def _tie_jump(J, ymax):
    """Bound on the change of a sample when the tap set of its axes switches:
    per axis one weight psi(J/2) moves between two cells, times the other two
    axes' summed weights (at most S each), over up to three axes."""
    psi_edge = float(kernels.kb_psi(np.array([J / 2.0]), J, kernels.default_beta(J))[0])
    S = _weight_sum(J)
    return 3 * 2 * psi_edge * S * S * ymax


def _compare(got, want, tie, prec, J, ymax, label, grid_err=0.0):
    """Strict bar away from tap-set switches; near them, the jump bound.
    grid_err: the bar of the grid the samples were gathered from (relative to
    its largest value), carried through the J^3 taps (at most S^3 of it)."""
    scale = np.max(np.abs(want))
    ok = ~tie
    e_strict = np.max(np.abs(got[ok] - want[ok])) / scale
    e_tie = np.max(np.abs(got[tie] - want[tie])) / scale if tie.any() else 0.0
    bar = BAR[prec] + _weight_sum(J) ** 3 * grid_err * ymax / scale
    say(f"[resample1] {label}: max err {e_strict:.2e} on {ok.sum()} samples (bar {bar:.2e}), "
        f"{e_tie:.2e} on {tie.sum()} near-tie samples (rel-L2 {rel_l2(got, want):.2e})")
    assert e_strict < bar
    assert e_tie < bar + _tie_jump(J, ymax) / scale


CASES = [
    # (N, n_proj, n_alpha, n_t, n_phi, n_theta, n_r, J)
    (16, 6, 8, 12, 32, 16, 32, 6),
    (16, 5, 6, 10, 32, 16, 32, 3),
    (24, 4, 6, 8, 60, 30, 48, 6),     # K = 120, 60, 96: radix 3 and 5
    (20, 3, 5, 7, 40, 20, 40, 4),     # ragged counts, K = 80, 40, 80
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[4]}x{c[5]}x{c[6]}_J{c[7]}")
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_grid_step_vs_oracle(case, prec):
    require_gpu()
    N, n_proj, n_alpha, n_t, n_phi, n_th, n_r, J = case
    say(f"[resample1] grid step {case} {prec}")
    u, D, _ = _setup(N, n_proj, n_alpha, n_t, n_phi, n_th, n_r, J, prec, 11)
    assert u.grid_shape == (2 * n_phi, 2 * n_th, 2 * n_r)
    got = to_host(u.stage("grid", to_dev(D.reshape(-1), _dtype(prec))))
    want = resample1.oversampled_grid(D, J)
    e, m = rel_l2(got, want), max_rel(got, want)
    say(f"[resample1] grid step rel-L2 {e:.2e} max {m:.2e}")
    assert m < BAR[prec]
    u.close()


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[4]}x{c[5]}x{c[6]}_J{c[7]}")
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_gather_step_vs_oracle(case, prec):
    require_gpu()
    N, n_proj, n_alpha, n_t, n_phi, n_th, n_r, J = case
    say(f"[resample1] gather step {case} {prec}")
    u, D, t = _setup(N, n_proj, n_alpha, n_t, n_phi, n_th, n_r, J, prec, 12)
    Y = resample1.oversampled_grid(D, J)
    if prec == "f32":
        Y = Y.astype(np.complex64).astype(np.complex128)
    got = to_host(u.stage("gather", to_dev(Y.reshape(-1), _dtype(prec)))).reshape(-1)
    want = resample1.interpolate(Y, t, J)
    _compare(got, want, _near_tie(t, J), prec, J, np.max(np.abs(Y)), f"gather {case} {prec}")
    u.close()


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[4]}x{c[5]}x{c[6]}_J{c[7]}")
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_resample_vs_oracle(case, prec):
    require_gpu()
    N, n_proj, n_alpha, n_t, n_phi, n_th, n_r, J = case
    say(f"[resample1] resample {case} {prec}")
    u, D, t = _setup(N, n_proj, n_alpha, n_t, n_phi, n_th, n_r, J, prec, 13)
    got = to_host(u.resample(to_dev(D.reshape(-1), _dtype(prec)))).reshape(-1)
    Y = resample1.oversampled_grid(D, J)
    want = resample1.interpolate(Y, t, J)
    _compare(got, want, _near_tie(t, J), prec, J, np.max(np.abs(Y)), f"resample {case} {prec}",
             grid_err=BAR[prec])
    # the same call again: the workspace is rewritten in full
    again = to_host(u.resample(to_dev(D.reshape(-1), _dtype(prec)))).reshape(-1)
    assert np.array_equal(again, got)
    u.close()


def _gauss_dradon(rho, n, c, cov):
    s2 = n @ cov @ n
    mass = (2 * np.pi) ** 1.5 * np.sqrt(np.linalg.det(cov))
    R = mass * np.exp(-(rho - n @ c) ** 2 / (2 * s2)) / np.sqrt(2 * np.pi * s2)
    return -(rho - n @ c) / s2 * R


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_isotropic_gaussian_closed_form(prec):
    # a centred isotropic Gaussian: the same derivative-Radon profile on every
    # line, so the index space is periodic on every axis and method 1 meets
    # the closed form on every umbrella plane
    require_gpu()
    import paper_1605_05231_amd as pkg
    N, n_phi, n_th = 16, 32, 16
    n_r = 2 * N
    cov = np.eye(3) * 2.2 ** 2
    c = np.zeros(3)
    th = synthetic.polar_angles(n_th)
    rho = np.arange(n_r) - n_r // 2
    dirs = synthetic.line_directions(synthetic.azimuths(n_phi), th)
    D = np.stack([_gauss_dradon(rho, n, c, cov) for n in dirs]).reshape(-1)
    u = pkg.Umbrella(N, 6, 8, 8, n_phi, n_th, n_r, th[0], th[1] - th[0], J=6, dtype=_dtype(prec),
                     method=1)
    got = to_host(u.resample(to_dev(D, _dtype(prec)))).reshape(-1)
    nh, rq = umbrella.geometry(N, 6, 8, 8)
    want = np.array([_gauss_dradon(r, n, c, cov) for r, n in zip(rq, nh)])
    err = np.max(np.abs(got - want)) / np.max(np.abs(D))
    say(f"[resample1] isotropic Gaussian {prec}: max err {err:.2e}")
    assert err < 1e-4
    u.close()


def test_full_size_128_setup():
    """The cone-beam experiment's 128^3 set-up in FP32, the configuration the
    benchmark times: the grid step on every one of its 33,177,600 cells, and
    the whole resampling on a seeded sample of umbrella planes."""
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    W = synthetic.WORKLOADS["c2"]
    N, n_phi, n_th, n_r = W.N, W.n_phi, W.n_theta, W.n_r
    n_proj = n_alpha = n_t = 2 * N
    J = 6
    th = synthetic.polar_angles(n_th)
    th0, dth = th[0], th[1] - th[0]
    say(f"[resample1] full size: {n_phi}x{n_th}x{n_r} -> {n_proj}x{n_alpha}x{n_t}, J={J}")
    rng = np.random.default_rng(21)
    D = (rng.standard_normal((n_phi, n_th, n_r)) + 1j * rng.standard_normal((n_phi, n_th, n_r)))
    D = D.astype(np.complex64)
    u = pkg.Umbrella(N, n_proj, n_alpha, n_t, n_phi, n_th, n_r, th0, dth, J=J, method=1)
    d = torch.from_numpy(D.reshape(-1)).cuda()
    grid = u.stage("grid", d)
    want_grid = resample1.oversampled_grid(D.astype(np.complex128), J)
    got_grid = to_host(grid)
    e, m = rel_l2(got_grid, want_grid), max_rel(got_grid, want_grid)
    say(f"[resample1] full-size grid step: rel-L2 {e:.2e} max {m:.2e}")
    assert m < 5e-6
    del got_grid
    out = to_host(u.resample(d)).reshape(-1)
    P = n_proj * n_alpha * n_t
    pick = np.unique(rng.integers(0, P, 20000))
    nh, rq = umbrella.geometry_at(N, n_proj, n_alpha, n_t, pick)
    tq, pq = umbrella.angles(nh)
    t = resample1.index_coords(n_phi, th0, dth, n_r, tq, pq, rq)
    want = resample1.interpolate(want_grid, t, J)
    _compare(out[pick], want, _near_tie(t, J), "f32", J, np.max(np.abs(want_grid)),
             "full size, sampled planes", grid_err=5e-6)
    u.close()


def test_rejects_unsupported_lengths_and_stages():
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    from paper_1605_05231_amd import NufftError
    for n_phi, n_th, n_r in [(31, 16, 32), (28, 16, 32), (32, 16, 1024)]:
        with pytest.raises(NufftError):
            pkg.Umbrella(16, 2, 2, 4, n_phi, n_th, n_r, 0.2, 0.1, J=6, method=1)
    u2 = pkg.Umbrella(16, 2, 2, 4, 32, 16, 32, 0.2, 0.1, J=6)
    with pytest.raises(ValueError):
        u2.stage("grid", torch.zeros(32 * 16 * 32, dtype=torch.complex64, device="cuda"))
    u2.close()
    u1 = pkg.Umbrella(16, 2, 2, 4, 32, 16, 32, 0.2, 0.1, J=6, method=1)
    with pytest.raises(ValueError):
        u1.stage("grid", torch.zeros(7, dtype=torch.complex64, device="cuda"))
    u1.close()

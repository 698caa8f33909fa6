"""GPU parity of the direct reconstruction (nufftct_reconstruct) with the oracle.

The library computes 1/(8 pi^2) A^H diag(w) d in its own kernels; the oracle
(oracle.recon) does the same in FP64 NumPy with its own quadrature.
"""
import math

import numpy as np
import pytest

import synthetic
from oracle import nufft, recon
from tests.gpu_util import rel_l2, require_gpu, say, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [
    # N, K, J, n_phi, n_theta, n_r, kernel
    (24, 48, 6, 16, 8, 48, "kb"),
    (24, 48, 5, 10, 7, 48, "minmax"),
    (32, 64, 6, 24, 12, 64, "kb"),
]


def _plan(pkg, torch, N, K, J, dirs, n_r, kernel, dtype):
    return pkg.Plan(N, K, J, dirs=dirs, n_r=n_r, kernel=kernel, dtype=dtype)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"N{c[0]}_K{c[1]}_J{c[2]}_{c[6]}")
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_reconstruct_matches_oracle(case, prec):
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    N, K, J, n_phi, n_th, n_r, kernel = case
    say(f"[recon] {case} {prec}")
    phi = synthetic.azimuths(n_phi)
    th = synthetic.polar_angles(n_th)
    dirs = synthetic.line_directions(phi, th)
    L = len(dirs)
    rng = np.random.default_rng(900 + N)
    d = rng.standard_normal((L, n_r)) + 1j * rng.standard_normal((L, n_r))
    w = pkg.radial_quadrature(phi, th)
    dtype = torch.complex64 if prec == "f32" else torch.complex128
    plan = _plan(pkg, torch, N, K, J, dirs, n_r, kernel, dtype)
    plan.set_line_weights(w)
    got = to_host(plan.reconstruct(to_dev(d, dtype)))
    prm = nufft.Params(N, K, J, kernel=kernel)
    want = recon.reconstruct(d.reshape(-1), dirs, n_r, recon.quadrature(phi, th), prm)
    err = rel_l2(got, want)
    say(f"[recon] rel-L2 {err:.2e}")
    if prec == "f32":
        assert err < 1e-5
    else:
        tol = 1e-12
        if kernel == "minmax":  # the oracle's own FP64 min-max solve carries cond(T) eps
            tol = 1e-10
        assert err < tol
    plan.close()


def test_reconstruct_is_weighted_adjoint():
    # reconstruct == 1/(8 pi^2) * adjoint of the line-weighted data, through the C ABI
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    N, K, J, n_r = 16, 32, 6, 32
    phi = synthetic.azimuths(8)
    th = synthetic.polar_angles(5)
    dirs = synthetic.line_directions(phi, th)
    rng = np.random.default_rng(31)
    d = rng.standard_normal((len(dirs), n_r)) + 1j * rng.standard_normal((len(dirs), n_r))
    w = rng.uniform(0.5, 2.0, len(dirs))
    plan = pkg.Plan(N, K, J, dirs=dirs, n_r=n_r, dtype=torch.complex128)
    plan.set_line_weights(w)
    a = to_host(plan.reconstruct(to_dev(d, torch.complex128)))
    b = to_host(plan.adjoint(to_dev(d * w[:, None], torch.complex128))) / (8 * math.pi ** 2)
    assert rel_l2(a, b) < 1e-14
    # the weights can be replaced; twice the weights, twice the volume
    plan.set_line_weights(2 * w)
    c = to_host(plan.reconstruct(to_dev(d, torch.complex128)))
    assert rel_l2(c, 2 * a) < 1e-14
    plan.close()


def test_reconstruct_gaussian_center_ratio():
    # forward of an isotropic centred Gaussian then reconstruction: the centre
    # voxel comes back scaled by the sampled solid angle, sum(w) / (4 pi)
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    N, K, J, n_r = 32, 64, 6, 64
    phi = synthetic.azimuths(48)
    th = synthetic.polar_angles(24)
    dirs = synthetic.line_directions(phi, th)
    x = synthetic.gaussian_blob(N, np.zeros(3), np.eye(3) * 2.5 ** 2)
    plan = pkg.Plan(N, K, J, dirs=dirs, n_r=n_r, dtype=torch.complex64)
    w = pkg.radial_quadrature(phi, th)
    plan.set_line_weights(w)
    xt = to_dev(x.astype(np.complex64), torch.complex64)
    xr = to_host(plan.reconstruct(plan.forward(xt)))
    ctr = (N // 2,) * 3
    ratio = xr[ctr].real / x[ctr]
    say(f"[recon] centre ratio {ratio:.6f} vs {w.sum() / (4 * math.pi):.6f}")
    assert abs(ratio - w.sum() / (4 * math.pi)) < 1e-4
    plan.close()


def test_reconstruct_errors():
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    N, K, J, n_r = 16, 32, 4, 32
    dirs = synthetic.line_directions(synthetic.azimuths(4), synthetic.polar_angles(3))
    plan = pkg.Plan(N, K, J, dirs=dirs, n_r=n_r, dtype=torch.complex64)
    d = torch.zeros(plan.M, dtype=torch.complex64, device="cuda")
    with pytest.raises(pkg.NufftError):
        plan.reconstruct(d)  # no weights yet
    with pytest.raises(ValueError):
        plan.set_line_weights(np.ones(len(dirs) + 1))
    with pytest.raises(pkg.NufftError):
        plan.set_line_weights(np.full(len(dirs), np.nan))
    pts = np.zeros((8, 3))
    pplan = pkg.Plan(N, K, J, points=pts, dtype=torch.complex64)
    with pytest.raises((pkg.NufftError, ValueError)):
        pplan.set_line_weights(np.ones(1))
    plan.close()
    pplan.close()

"""The allocation-free forward entry point (nufftct_forward_noalloc): its
results equal nufftct_forward's on the same plan bit for bit, on two calls in a
row with the second on a smaller plan (the static scratch keeps the first
call's contents), and a plan whose workspace exceeds the static array is
rejected before any work."""
import numpy as np
import pytest

import synthetic
from tests.gpu_util import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


def _case(pkg, torch, N, K, J, nphi, nth, n_r, dtype, seed):
    dirs = synthetic.line_directions(synthetic.azimuths(nphi), synthetic.polar_angles(nth))
    plan = pkg.Plan(N, K, J, dirs=dirs, n_r=n_r, dtype=dtype)
    rng = np.random.default_rng(seed)
    x = synthetic.ellipsoid_phantom(N, 8, seed) + 0.1j * rng.standard_normal((N, N, N))
    return plan, to_dev(x, dtype)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_matches_forward_twice(prec):
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    dtype = torch.complex64 if prec == "f32" else torch.complex128
    big = _case(pkg, torch, 48, 96, 6, 16, 8, 96, dtype, 1)
    small = _case(pkg, torch, 24, 48, 6, 10, 5, 48, dtype, 2)
    for name, (plan, x) in (("first", big), ("second, smaller", small)):
        for radial, deriv in ((True, True), (True, False), (False, False)):
            want = plan.forward(x, radial=radial, deriv=deriv)
            got = torch.empty_like(want)
            plan.forward_noalloc(x, got, radial=radial, deriv=deriv)
            torch.cuda.synchronize()
            say(f"[noalloc] {prec} {name} call, radial={radial} deriv={deriv}: "
                f"max |diff| {float((got - want).abs().max()):.1e}")
            assert torch.equal(got, want)
    # the larger plan again, after the smaller one overwrote part of the scratch
    plan, x = big
    want = plan.forward(x)
    got = torch.empty_like(want)
    plan.forward_noalloc(x, got)
    assert torch.equal(got, want)


def test_noalloc_rejects_plans_beyond_the_static_array():
    require_gpu()
    import torch
    import paper_1605_05231_amd as pkg
    dirs = synthetic.line_directions(synthetic.azimuths(4), synthetic.polar_angles(2))
    plan = pkg.Plan(128, 256, 6, dirs=dirs, n_r=256)  # 256^3 x 8 bytes = 128 MiB of grid
    x = torch.zeros(128 ** 3, dtype=torch.complex64, device="cuda")
    out = torch.empty(plan.M, dtype=torch.complex64, device="cuda")
    with pytest.raises(pkg.NufftError, match="static scratch"):
        plan.forward_noalloc(x, out)

"""Host-only checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments before touching a GPU."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from paper_1605_05231_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nufftct.h")

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH),
                                reason="libnufftct.so not built")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nufftct_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), "binding signatures out of sync with the header"
    assert b"gfx950" in lib.nufftct_version()


def _radial(N=32, K=64, J=4, kernel=0, beta=-1.0, prec=0, n_lines=2, n_r=64):
    lib = _lib.load()
    p = C.c_void_p()
    d = np.zeros((max(n_lines, 1), 3))
    d[:, 2] = 1.0
    rc = lib.nufftct_plan_create_radial(C.byref(p), N, K, J, kernel, beta, prec,
                                        d.ctypes.data_as(C.POINTER(C.c_double)), n_lines, n_r, None)
    return rc, p, lib.nufftct_last_error().decode()


@pytest.mark.parametrize("kw,code,frag", [
    (dict(N=31), _lib.EINVAL, "N must be even"),
    (dict(N=0), _lib.EINVAL, "N must be even"),
    (dict(K=30), _lib.EINVAL, "K must be even and >= N"),
    (dict(K=65), _lib.EINVAL, "K must be even"),
    (dict(J=1), _lib.EINVAL, "J must be"),
    (dict(J=9), _lib.EINVAL, "J must be"),
    (dict(kernel=7), _lib.EINVAL, "unknown kernel"),
    (dict(prec=5), _lib.EINVAL, "unknown precision"),
    (dict(beta=100.0), _lib.EINVAL, "beta"),
    (dict(n_r=63), _lib.EINVAL, "n_r"),
    (dict(n_r=2), _lib.EINVAL, "n_r must be >= 4"),
    (dict(n_lines=0), _lib.EINVAL, "n_lines"),
    (dict(K=98, N=32), _lib.EUNSUPPORTED, "prime factor"),
    (dict(K=72, N=32), _lib.EUNSUPPORTED, "compiled FFT lengths"),
    (dict(n_r=56), _lib.EUNSUPPORTED, "prime factor"),
])
def test_rejects_bad_arguments(kw, code, frag):
    rc, p, msg = _radial(**kw)
    assert rc == code and frag in msg, (rc, msg)
    assert p.value is None


def test_null_pointers_and_points_validation():
    lib = _lib.load()
    assert lib.nufftct_plan_create_radial(None, 32, 64, 4, 0, -1.0, 0, None, 1, 64, None) == _lib.EINVAL
    p = C.c_void_p()
    assert lib.nufftct_plan_create(C.byref(p), 32, 64, 4, 0, -1.0, 0, None, 10, 0, None) == _lib.EINVAL
    bad = np.array([[np.nan, 0, 0]])
    rc = lib.nufftct_plan_create(C.byref(p), 32, 64, 4, 0, -1.0, 0,
                                 bad.ctypes.data_as(C.POINTER(C.c_double)), 1, 0, None)
    assert rc == _lib.EINVAL and b"finite" in lib.nufftct_last_error()
    for fn in ("nufftct_forward", "nufftct_adjoint"):
        assert getattr(lib, fn)(None, None, None, 0, None) == _lib.EINVAL
    assert lib.nufftct_stage(None, 0, None, None, 0, None) == _lib.EINVAL
    assert lib.nufftct_plan_destroy(None) == _lib.OK
    assert lib.nufftct_batch_destroy(None) == _lib.OK
    assert lib.nufftct_batch_graph_launch(None, 0, None) == _lib.EINVAL
    b = C.c_void_p()
    assert lib.nufftct_batch_create(C.byref(b), 0, None, None, 6, 0, -1.0, 0, None, None, None,
                                    None) == _lib.EINVAL


@pytest.mark.skipif(os.environ.get("HIP_VISIBLE_DEVICES", None) is None and os.path.exists("/dev/kfd"),
                    reason="a GPU may be present; the no-device path is checked only without one")
def test_valid_plan_without_device_fails_cleanly():
    rc, p, msg = _radial()
    assert rc in (_lib.EHIP, _lib.ENOMEM) and msg
    assert p.value is None


def test_radial_quadrature_matches_oracle():
    # host-only library routine (no device work) against the oracle's own weights
    from oracle import recon
    import synthetic
    lib = _lib.load()
    dp = C.POINTER(C.c_double)
    for n_phi, margin in ((12, 0.2), (7, 0.0), (1, 0.3)):
        phi = np.ascontiguousarray(synthetic.azimuths(n_phi))
        for n_th in (1, 2, 9):
            th = np.ascontiguousarray(synthetic.polar_angles(n_th, margin=margin)) if n_th > 1 \
                else np.array([math.pi / 2])
            w = np.empty(n_phi * n_th)
            rc = lib.nufftct_radial_quadrature(phi.ctypes.data_as(dp), n_phi, th.ctypes.data_as(dp),
                                               n_th, w.ctypes.data_as(dp))
            assert rc == _lib.OK
            want = recon.quadrature(phi, th)
            assert np.max(np.abs(w - want)) <= 1e-14 * np.max(np.abs(want)), (n_phi, n_th)


def test_reconstruction_entry_points_reject_bad_arguments():
    lib = _lib.load()
    dp = C.POINTER(C.c_double)
    phi = np.array([0.0, 1.0])
    th = np.array([1.0, 0.5])  # not increasing
    w = np.empty(4)
    assert lib.nufftct_radial_quadrature(phi.ctypes.data_as(dp), 2, th.ctypes.data_as(dp), 2,
                                         w.ctypes.data_as(dp)) == _lib.EINVAL
    assert lib.nufftct_radial_quadrature(None, 2, th.ctypes.data_as(dp), 2,
                                         w.ctypes.data_as(dp)) == _lib.EINVAL
    assert lib.nufftct_set_line_weights(None, w.ctypes.data_as(dp), None) == _lib.EINVAL
    assert lib.nufftct_reconstruct(None, C.c_void_p(16), C.c_void_p(32), None) == _lib.EINVAL


def test_umbrella_create_is_host_only_and_validates():
    # creation only checks arguments and sets constants on the host (no device memory)
    lib = _lib.load()
    for J in range(2, 9):
        for prec in (_lib.FP32, _lib.FP64):
            u = C.c_void_p()
            rc = lib.nufftct_umbrella_create(C.byref(u), 4, 8, 16, 50.0, 70.0, 24.0, 32, 16, 0.2,
                                             0.05, 32, J, prec, None)
            assert rc == _lib.OK, (J, prec, lib.nufftct_last_error())
            assert lib.nufftct_umbrella_destroy(u) == _lib.OK
    u = C.c_void_p()
    bad = [(0, 8, 16, 50.0, 70.0, 24.0, 32, 16, 0.2, 0.05, 32, 6),
           (4, 8, 16, -1.0, 70.0, 24.0, 32, 16, 0.2, 0.05, 32, 6),
           (4, 8, 16, 50.0, 70.0, 24.0, 32, 16, 0.2, 0.0, 32, 6),
           (4, 8, 16, 50.0, 70.0, 24.0, 32, 16, 0.2, 0.05, 32, 9)]
    for args in bad:
        assert lib.nufftct_umbrella_create(C.byref(u), *args, _lib.FP32, None) == _lib.EINVAL, args
    assert lib.nufftct_umbrella_resample(None, C.c_void_p(16), C.c_void_p(32), None) == _lib.EINVAL

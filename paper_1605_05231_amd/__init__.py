"""MI355X NUFFT projector: volume -> radially sampled derivative-Radon space, and
its exact adjoint, as hand-written HIP kernels behind a C ABI (libnufftct.so).

This module only marshals arguments: every step of the projector runs in the
library's kernels.  PyTorch supplies device memory and the current stream.
The library must have been built (``__graft_entry__.build()``); importing
works without it, but creating a plan raises if it is missing.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (DERIV, DERIV_RADIAL, DETERMINISTIC, FP32, FP64, KERNEL_KB, KERNEL_MINMAX_KB, RADIAL,  # noqa: F401
                   STAGE_IFFT_CROP, STAGE_INTERP, STAGE_NAMES, STAGE_PAD_FFT, STAGE_RADIAL,
                   STAGE_RADIAL_ADJ, STAGE_SPREAD, UMB_STAGE_GATHER, UMB_STAGE_GRID, GR_STAGE_BACKPROJECT, GR_STAGE_SPECTRA,
                   NufftError)

__all__ = ["Plan", "Batch", "Umbrella", "Grangeat", "NufftProjector", "project", "autotune", "radial_quadrature",
           "NufftError", "version"]


def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _check_tensor(t, n: int, dtype, name: str):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device (cuda/hip) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")


def version() -> str:
    return _lib.load().nufftct_version().decode()


class Plan:
    """A NUFFT projector plan (owns tables, point binning and workspaces).

    Radial plans: ``Plan(N, K, J, dirs=(L,3) float64, n_r=...)``; the points are
    ``r_c * dirs[l]`` with ``r_c = (c - n_r/2) 2 pi / n_r``.  Point plans:
    ``Plan(N, K, J, points=(M,3) float64[, n_r=line length])``.
    ``dtype`` is torch.complex64 (FP32 path) or torch.complex128 (FP64 form).
    """

    def __init__(self, N: int, K: int, J: int, *, dirs=None, n_r: int = 0, points=None,
                 kernel: str = "kb", beta: float | None = None, dtype=None, device=None):
        torch = _torch()
        lib = _lib.load()
        self.dtype = dtype or torch.complex64
        prec = {torch.complex64: FP32, torch.complex128: FP64}.get(self.dtype)
        if prec is None:
            raise TypeError("dtype must be torch.complex64 or torch.complex128")
        kern = {"kb": KERNEL_KB, "minmax": KERNEL_MINMAX_KB}[kernel]
        self.device = torch.device(device or "cuda")
        self.N, self.K, self.J = int(N), int(K), int(J)
        self.kernel = kernel
        self._ptr = C.c_void_p()
        with torch.cuda.device(self.device):
            st = _stream_handle()
            b = -1.0 if beta is None else float(beta)
            if dirs is not None:
                d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
                self._geom = d
                rc = lib.nufftct_plan_create_radial(
                    C.byref(self._ptr), self.N, self.K, self.J, kern, b, prec,
                    d.ctypes.data_as(C.POINTER(C.c_double)), d.shape[0], int(n_r), C.c_void_p(st))
                self.n_r = int(n_r)
                self.M = d.shape[0] * self.n_r
            elif points is not None:
                pts = np.ascontiguousarray(np.asarray(points, dtype=np.float64).reshape(-1, 3))
                self._geom = pts
                rc = lib.nufftct_plan_create(
                    C.byref(self._ptr), self.N, self.K, self.J, kern, b, prec,
                    pts.ctypes.data_as(C.POINTER(C.c_double)), pts.shape[0], int(n_r),
                    C.c_void_p(st))
                self.n_r = int(n_r)
                self.M = pts.shape[0]
            else:
                raise ValueError("give dirs (radial plan) or points")
        _lib.check(rc)

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_ptr", None) is not None and self._ptr.value:
            _lib.load().nufftct_plan_destroy(self._ptr)
            self._ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- sizes --------------------------------------------------------------
    @property
    def vol_shape(self):
        return (self.N, self.N, self.N)

    @property
    def out_shape(self):
        return (self.M // self.n_r, self.n_r) if self.n_r else (self.M,)

    def info(self) -> dict:
        vals = [C.c_int64(), C.c_int64(), C.c_int(), C.c_int64(), C.c_int64(), C.c_int(), C.c_int64()]
        _lib.check(_lib.load().nufftct_plan_info(self._ptr, *[C.byref(v) for v in vals]))
        keys = ["N", "K", "J", "M", "n_r", "precision", "workspace_bytes"]
        return {k: v.value for k, v in zip(keys, vals)}

    def tiling(self) -> tuple:
        """(tile edge, points per task) of the plan's interpolation/spreading tasks."""
        t, m = C.c_int(), C.c_int()
        _lib.check(_lib.load().nufftct_plan_tiling(self._ptr, C.byref(t), C.byref(m)))
        return (t.value, m.value)

    # -- operators ----------------------------------------------------------
    @staticmethod
    def _flags(radial: bool, deriv: bool) -> int:
        return (RADIAL if radial else 0) | (DERIV if (radial and deriv) else 0)

    def forward(self, x, out=None, *, radial: bool = True, deriv: bool = True, stream=None):
        """vol (N,N,N) -> (L, n_r) derivative-Radon values (or NUFFT values)."""
        torch = _torch()
        radial = radial and self.n_r > 0
        _check_tensor(x, self.N ** 3, self.dtype, "x")
        if out is None:
            out = torch.empty(self.out_shape, dtype=self.dtype, device=x.device)
        _check_tensor(out, self.M, self.dtype, "out")
        _lib.check(_lib.load().nufftct_forward(self._ptr, x.data_ptr(), out.data_ptr(),
                                               self._flags(radial, deriv),
                                               C.c_void_p(_stream_handle(stream))))
        return out

    def forward_noalloc(self, x, out, *, radial: bool = True, deriv: bool = True, stream=None):
        """forward() with its workspace in the library's static 64 MiB device
        array: no device allocation in the call (the output must be given).
        Calls on one GPU must not overlap."""
        radial = radial and self.n_r > 0
        _check_tensor(x, self.N ** 3, self.dtype, "x")
        _check_tensor(out, self.M, self.dtype, "out")
        _lib.check(_lib.load().nufftct_forward_noalloc(self._ptr, x.data_ptr(), out.data_ptr(),
                                                       self._flags(radial, deriv),
                                                       C.c_void_p(_stream_handle(stream))))
        return out

    def adjoint(self, y, out=None, *, radial: bool = True, deriv: bool = True,
                deterministic: bool = False, stream=None):
        """(L, n_r) or (M,) -> vol (N,N,N): exact conjugate transpose of forward.
        deterministic: bitwise reproducible in the FP64 form too (the FP32
        path always is)."""
        torch = _torch()
        radial = radial and self.n_r > 0
        _check_tensor(y, self.M, self.dtype, "y")
        if out is None:
            out = torch.empty(self.vol_shape, dtype=self.dtype, device=y.device)
        _check_tensor(out, self.N ** 3, self.dtype, "out")
        _lib.check(_lib.load().nufftct_adjoint(self._ptr, y.data_ptr(), out.data_ptr(),
                                               self._flags(radial, deriv)
                                               | (DETERMINISTIC if deterministic else 0),
                                               C.c_void_p(_stream_handle(stream))))
        return out

    def set_line_weights(self, w):
        """Per-line quadrature weights (n_lines values) for `reconstruct`."""
        w = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(-1))
        if self.n_r == 0 or w.shape[0] != self.M // self.n_r:
            raise ValueError(f"need one weight per line ({self.M // max(self.n_r, 1)}), got {w.shape[0]}")
        _lib.check(_lib.load().nufftct_set_line_weights(self._ptr, w.ctypes.data_as(C.POINTER(C.c_double)),
                                                        C.c_void_p(_stream_handle())))

    def reconstruct(self, d, out=None, *, stream=None):
        """Direct reconstruction 1/(8 pi^2) A^H diag(w) d from derivative-Radon
        values d ((L, n_r) or (M,)) with the weights of `set_line_weights`."""
        torch = _torch()
        _check_tensor(d, self.M, self.dtype, "d")
        if out is None:
            out = torch.empty(self.vol_shape, dtype=self.dtype, device=d.device)
        _check_tensor(out, self.N ** 3, self.dtype, "out")
        _lib.check(_lib.load().nufftct_reconstruct(self._ptr, d.data_ptr(), out.data_ptr(),
                                                   C.c_void_p(_stream_handle(stream))))
        return out

    def stage(self, stage: int, inp, out, *, deriv: bool = True, deterministic: bool = False,
              stream=None):
        """Run a single stage (STAGE_*); sizes: vol N^3, grid K^3, points M."""
        sizes = {STAGE_PAD_FFT: (self.N ** 3, self.K ** 3), STAGE_INTERP: (self.K ** 3, self.M),
                 STAGE_RADIAL: (self.M, self.M), STAGE_RADIAL_ADJ: (self.M, self.M),
                 STAGE_SPREAD: (self.M, self.K ** 3), STAGE_IFFT_CROP: (self.K ** 3, self.N ** 3)}
        ni, no = sizes[stage]
        _check_tensor(inp, ni, self.dtype, "inp")
        _check_tensor(out, no, self.dtype, "out")
        _lib.check(_lib.load().nufftct_stage(self._ptr, stage, inp.data_ptr(), out.data_ptr(),
                                             (DERIV if deriv else 0)
                                             | (DETERMINISTIC if deterministic else 0),
                                             C.c_void_p(_stream_handle(stream))))
        return out

    # -- timing -------------------------------------------------------------
    def set_timing(self, on: bool = True):
        _lib.check(_lib.load().nufftct_set_timing(self._ptr, 1 if on else 0))

    def stage_times(self) -> dict:
        ms = (C.c_double * 8)()
        cnt = (C.c_int64 * 8)()
        _lib.check(_lib.load().nufftct_get_stage_times(self._ptr, ms, cnt, 8))
        return {STAGE_NAMES[i]: (ms[i], cnt[i]) for i in range(len(STAGE_NAMES))}


def autotune(N: int, K: int, J: int, dirs, n_r: int, *, kernel: str = "kb", beta=None,
             dtype=None, deriv: bool = True) -> dict:
    """Time candidate tilings for this radial geometry on the current GPU and
    record the fastest; later Plans with the same shape use it."""
    torch = _torch()
    dtype = dtype or torch.complex64
    prec = {torch.complex64: FP32, torch.complex128: FP64}[dtype]
    d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
    t, m, ms = C.c_int(), C.c_int(), C.c_double()
    _lib.check(_lib.load().nufftct_autotune_radial(
        int(N), int(K), int(J), {"kb": KERNEL_KB, "minmax": KERNEL_MINMAX_KB}[kernel],
        -1.0 if beta is None else float(beta), prec, d.ctypes.data_as(C.POINTER(C.c_double)),
        d.shape[0], int(n_r), RADIAL | (DERIV if deriv else 0), C.byref(t), C.byref(m), C.byref(ms),
        C.c_void_p(_stream_handle())))
    return {"tile": t.value, "max_pts": m.value, "ms": ms.value}


def radial_quadrature(phi, theta) -> np.ndarray:
    """Quadrature weights of the directions of a (phi, theta) line grid, lines
    ordered [phi][theta] (computed by the library on the host)."""
    phi = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).reshape(-1))
    theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1))
    w = np.empty(len(phi) * len(theta), dtype=np.float64)
    dp = C.POINTER(C.c_double)
    _lib.check(_lib.load().nufftct_radial_quadrature(phi.ctypes.data_as(dp), len(phi),
                                                     theta.ctypes.data_as(dp), len(theta),
                                                     w.ctypes.data_as(dp)))
    return w


# Scan geometry of the circular cone-beam set-up (Section 3.2.1) in millimetres:
# source-object and source-detector distances, detector side, object side.
SCAN_MM = (1100.0, 1500.0, 512.0, 360.0)


class Umbrella:
    """Radial -> umbrella resampling for a circular cone-beam scan: method 2
    (eq 2.15, the default) or method 1 (eq 2.11, an oversampled NUFFT in the
    radial grid's index space); distances in voxels (default: the Section
    3.2.1 set-up scaled to an N^3 volume spanning the object)."""

    def __init__(self, N, n_proj, n_alpha, n_t, n_phi, n_theta, n_r, theta0, dtheta, *, J=6,
                 scan=None, dtype=None, method=2):
        torch = _torch()
        self.dtype = dtype or torch.complex64
        prec = {torch.complex64: FP32, torch.complex128: FP64}[self.dtype]
        if scan is None:
            so, sd, det, obj = SCAN_MM
            scan = (N * so / obj, N * sd / obj, N * det / obj)
        if method not in (1, 2):
            raise ValueError("method must be 1 or 2")
        self.method = method
        self.n_in = int(n_phi) * int(n_theta) * int(n_r)
        self.shape = (int(n_proj), int(n_alpha), int(n_t))
        self._ptr = C.c_void_p()
        lib = _lib.load()
        create = lib.nufftct_umbrella1_create if method == 1 else lib.nufftct_umbrella_create
        _lib.check(create(
            C.byref(self._ptr), int(n_proj), int(n_alpha), int(n_t), float(scan[0]), float(scan[1]),
            float(scan[2]), int(n_phi), int(n_theta), float(theta0), float(dtheta), int(n_r), int(J),
            prec, C.c_void_p(_stream_handle())))
        self.grid_shape = None
        if method == 1:
            K3 = (C.c_int64 * 3)()
            _lib.check(lib.nufftct_umbrella_grid_shape(self._ptr, K3))
            self.grid_shape = tuple(int(k) for k in K3)

    def resample(self, d, out=None, *, stream=None):
        torch = _torch()
        _check_tensor(d, self.n_in, self.dtype, "d")
        if out is None:
            out = torch.empty(self.shape, dtype=self.dtype, device=d.device)
        _check_tensor(out, self.shape[0] * self.shape[1] * self.shape[2], self.dtype, "out")
        _lib.check(_lib.load().nufftct_umbrella_resample(self._ptr, d.data_ptr(), out.data_ptr(),
                                                         C.c_void_p(_stream_handle(stream))))
        return out

    def stage(self, which, x, out=None, *, stream=None):
        """Method 1, one step: "grid" (radial samples -> oversampled grid
        F P F^-1 D, shape grid_shape) or "gather" (grid -> umbrella samples)."""
        torch = _torch()
        if self.method != 1:
            raise ValueError("only method 1 has stages")
        ncell = self.grid_shape[0] * self.grid_shape[1] * self.grid_shape[2]
        if which == "grid":
            code, n_in, shape = UMB_STAGE_GRID, self.n_in, self.grid_shape
        elif which == "gather":
            code, n_in, shape = UMB_STAGE_GATHER, ncell, self.shape
        else:
            raise ValueError(which)
        _check_tensor(x, n_in, self.dtype, "x")
        if out is None:
            out = torch.empty(shape, dtype=self.dtype, device=x.device)
        _check_tensor(out, shape[0] * shape[1] * shape[2], self.dtype, "out")
        _lib.check(_lib.load().nufftct_umbrella_stage(self._ptr, code, x.data_ptr(), out.data_ptr(),
                                                      C.c_void_p(_stream_handle(stream))))
        return out

    def close(self):
        if getattr(self, "_ptr", None) is not None and self._ptr.value:
            _lib.load().nufftct_umbrella_destroy(self._ptr)
            self._ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Grangeat:
    """Umbrella derivative-Radon values -> cone-beam projections (the Grangeat
    step in reverse, Section 2.2.2): n_proj projections of n x n pixels from
    n_alpha x n umbrella samples each; distances in voxels (default: the
    Section 3.2.1 set-up scaled to an N^3 volume spanning the object)."""

    def __init__(self, N, n_proj, n_alpha, n, *, J=5, scan=None, dtype=None):
        torch = _torch()
        self.dtype = dtype or torch.complex64
        prec = {torch.complex64: FP32, torch.complex128: FP64}[self.dtype]
        if scan is None:
            so, sd, det, obj = SCAN_MM
            scan = (N * so / obj, N * sd / obj, N * det / obj)
        self.n_proj, self.n_alpha, self.n = int(n_proj), int(n_alpha), int(n)
        self._ptr = C.c_void_p()
        _lib.check(_lib.load().nufftct_grangeat_create(
            C.byref(self._ptr), self.n_proj, self.n_alpha, self.n, float(scan[0]), float(scan[1]),
            float(scan[2]), int(J), prec, C.c_void_p(_stream_handle())))

    def project(self, u, out=None, *, stream=None):
        torch = _torch()
        _check_tensor(u, self.n_proj * self.n_alpha * self.n, self.dtype, "u")
        if out is None:
            out = torch.empty((self.n_proj, self.n, self.n), dtype=self.dtype, device=u.device)
        _check_tensor(out, self.n_proj * self.n * self.n, self.dtype, "out")
        _lib.check(_lib.load().nufftct_grangeat_project(self._ptr, u.data_ptr(), out.data_ptr(),
                                                        C.c_void_p(_stream_handle(stream))))
        return out

    def stage(self, which, x, out=None, *, stream=None):
        """"spectra" (umbrella samples -> filtered spectra, [alpha][m][proj])
        or "backproject" (spectra -> projections)."""
        torch = _torch()
        n_spec = self.n_alpha * 2 * self.n * self.n_proj
        if which == "spectra":
            code, n_in, shape = GR_STAGE_SPECTRA, self.n_proj * self.n_alpha * self.n, \
                (self.n_alpha, 2 * self.n, self.n_proj)
        elif which == "backproject":
            code, n_in, shape = GR_STAGE_BACKPROJECT, n_spec, (self.n_proj, self.n, self.n)
        else:
            raise ValueError(which)
        _check_tensor(x, n_in, self.dtype, "x")
        if out is None:
            out = torch.empty(shape, dtype=self.dtype, device=x.device)
        _check_tensor(out, shape[0] * shape[1] * shape[2], self.dtype, "out")
        _lib.check(_lib.load().nufftct_grangeat_stage(self._ptr, code, x.data_ptr(), out.data_ptr(),
                                                      C.c_void_p(_stream_handle(stream))))
        return out

    def entries(self):
        n = C.c_int64()
        _lib.check(_lib.load().nufftct_grangeat_info(self._ptr, C.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "_ptr", None) is not None and self._ptr.value:
            _lib.load().nufftct_grangeat_destroy(self._ptr)
            self._ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Uneven batch of radial plans sharing J, kernel and precision; tune=True
    autotunes the tiling per size class (on its largest member)."""

    def __init__(self, Ns, Ks, J, dirs_list, n_rs, *, kernel="kb", beta=None, dtype=None,
                 tune=False):
        torch = _torch()
        lib = _lib.load()
        self.dtype = dtype or torch.complex64
        prec = {torch.complex64: FP32, torch.complex128: FP64}[self.dtype]
        kern = {"kb": KERNEL_KB, "minmax": KERNEL_MINMAX_KB}[kernel]
        n = len(Ns)
        self.Ns = [int(v) for v in Ns]
        self.n_rs = [int(v) for v in n_rs]
        self._dirs = [np.ascontiguousarray(np.asarray(d, dtype=np.float64).reshape(-1, 3)) for d in dirs_list]
        self.Ms = [d.shape[0] * r for d, r in zip(self._dirs, self.n_rs)]
        Na = (C.c_int64 * n)(*self.Ns)
        Ka = (C.c_int64 * n)(*[int(v) for v in Ks])
        La = (C.c_int64 * n)(*[d.shape[0] for d in self._dirs])
        Ra = (C.c_int64 * n)(*self.n_rs)
        Da = (C.POINTER(C.c_double) * n)(*[d.ctypes.data_as(C.POINTER(C.c_double)) for d in self._dirs])
        self._ptr = C.c_void_p()
        create = lib.nufftct_batch_create_tuned if tune else lib.nufftct_batch_create
        _lib.check(create(C.byref(self._ptr), n, Na, Ka, int(J), kern,
                          -1.0 if beta is None else float(beta), prec, Da, La, Ra,
                          C.c_void_p(_stream_handle())))

    def close(self):
        if getattr(self, "_ptr", None) is not None and self._ptr.value:
            _lib.load().nufftct_batch_destroy(self._ptr)
            self._ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, ts, sizes, name):
        for t, n in zip(ts, sizes):
            _check_tensor(t, n, self.dtype, name)
        return (C.c_void_p * len(ts))(*[t.data_ptr() for t in ts])

    def forward(self, xs, outs, *, deriv=True, stream=None):
        a = self._ptrs(xs, [n ** 3 for n in self.Ns], "x")
        b = self._ptrs(outs, self.Ms, "out")
        _lib.check(_lib.load().nufftct_batch_forward(self._ptr, a, b, RADIAL | (DERIV if deriv else 0),
                                                     C.c_void_p(_stream_handle(stream))))
        return outs

    def adjoint(self, ys, outs, *, deriv=True, deterministic=False, stream=None):
        a = self._ptrs(ys, self.Ms, "y")
        b = self._ptrs(outs, [n ** 3 for n in self.Ns], "out")
        flags = RADIAL | (DERIV if deriv else 0) | (DETERMINISTIC if deterministic else 0)
        _lib.check(_lib.load().nufftct_batch_adjoint(self._ptr, a, b, flags,
                                                     C.c_void_p(_stream_handle(stream))))
        return outs

    def capture(self, direction: int, src, dst, *, deriv=True, stream=None):
        if direction == 0:
            a = self._ptrs(src, [n ** 3 for n in self.Ns], "x")
            b = self._ptrs(dst, self.Ms, "out")
        else:
            a = self._ptrs(src, self.Ms, "y")
            b = self._ptrs(dst, [n ** 3 for n in self.Ns], "out")
        # the graph holds raw pointers: keep each direction's buffers alive
        self._keep = getattr(self, "_keep", {})
        self._keep[direction] = (src, dst)
        _lib.check(_lib.load().nufftct_batch_graph_capture(self._ptr, direction, a, b,
                                                           RADIAL | (DERIV if deriv else 0),
                                                           C.c_void_p(_stream_handle(stream))))

    def replay(self, direction: int, stream=None):
        _lib.check(_lib.load().nufftct_batch_graph_launch(self._ptr, direction,
                                                          C.c_void_p(_stream_handle(stream))))


def _autograd():
    torch = _torch()

    class NufftProjector(torch.autograd.Function):
        """y = A x with A the plan's forward (derivative-Radon by default); the
        backward applies the hand-written adjoint A^H.  x may be one volume
        (N, N, N) or a batch (B, N, N, N) sharing the plan's geometry.  Real
        inputs get the real part of A^H g as their gradient."""

        @staticmethod
        def forward(ctx, x, plan, radial=True, deriv=True):
            ctx.plan, ctx.radial, ctx.deriv = plan, radial, deriv
            ctx.real_input = not x.is_complex()
            xc = x.to(plan.dtype).contiguous()
            if xc.dim() == 3:
                return plan.forward(xc, radial=radial, deriv=deriv)
            out = torch.empty((xc.shape[0],) + plan.out_shape, dtype=plan.dtype, device=xc.device)
            for b in range(xc.shape[0]):
                plan.forward(xc[b], out=out[b], radial=radial, deriv=deriv)
            return out

        @staticmethod
        def backward(ctx, g):
            plan = ctx.plan
            gc = g.to(plan.dtype).contiguous()
            if gc.dim() == len(plan.out_shape):
                gx = plan.adjoint(gc, radial=ctx.radial, deriv=ctx.deriv)
            else:
                gx = torch.empty((gc.shape[0],) + plan.vol_shape, dtype=plan.dtype, device=gc.device)
                for b in range(gc.shape[0]):
                    plan.adjoint(gc[b], out=gx[b], radial=ctx.radial, deriv=ctx.deriv)
            if ctx.real_input:
                gx = gx.real
            return gx, None, None, None

    return NufftProjector


class _Lazy:
    _cls = None

    def __getattr__(self, item):
        if _Lazy._cls is None:
            _Lazy._cls = _autograd()
        return getattr(_Lazy._cls, item)


NufftProjector = _Lazy()


def project(x, plan: Plan, radial: bool = True, deriv: bool = True):
    """Differentiable forward projection (autograd backward = adjoint kernels)."""
    return NufftProjector.apply(x, plan, radial, deriv)

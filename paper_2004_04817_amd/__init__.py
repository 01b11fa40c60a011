"""Python binding of the MI355X GCB greedy RBF mesh-deformation library.

A thin ctypes layer over ``libgcb.so`` (the C ABI declared in
``include/gcb.h``): argument marshalling only.  Every step of the method runs
in the library's HIP kernels.  PyTorch is used, when the caller passes
tensors, for device memory and the current HIP stream.

The library must be built (``__graft_entry__.build()`` or
``python paper_2004_04817_amd/build.py``); importing :func:`lib` raises if it
is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgcb.so")

GCB_OK, GCB_NOT_CONVERGED = 0, 1
GCB_E_INVALID, GCB_E_STATE, GCB_E_NOMEM, GCB_E_SINGULAR, GCB_E_DEVICE = -1, -2, -3, -4, -5
GCB_MEM_HOST, GCB_MEM_DEVICE = 0, 1
GCB_F32, GCB_F64 = 0, 1
GCB_PREC_FP64, GCB_PREC_FP32_EVAL = 0, 1
GCB_SERVE_BATCH, GCB_SERVE_CACHE = 1, 2

EXPORTS = ["gcb_version", "gcb_partition", "gcb_create", "gcb_destroy", "gcb_last_error", "gcb_set_stream",
           "gcb_set_boundary", "gcb_set_displacement", "gcb_set_params", "gcb_set_groups", "gcb_select",
           "gcb_get_support", "gcb_get_log", "gcb_deform", "gcb_deform_multi", "gcb_certify",
           "gcb_set_support", "gcb_refactor", "gcb_get_factor", "gcb_get_monitor",
           "gcb_batch_create", "gcb_batch_destroy", "gcb_batch_last_error", "gcb_batch_begin", "gcb_batch_step",
           "gcb_batch_end", "gcb_select_batch", "gcb_deform_batch", "gcb_batch_set_layout",
           "gcb_server_clock", "gcb_server_create", "gcb_server_destroy", "gcb_server_last_error",
           "gcb_server_submit", "gcb_server_progress", "gcb_server_result", "gcb_server_forget",
           "gcb_server_memory", "gcb_deform_time", "gcb_deform_noalloc",
           "gcb_set_kernel_timing", "gcb_get_kernel_times", "gcb_get_deform_pairs"]

GCB_NOALLOC_MAX_SUPPORTS = 8192
GCB_MAX_PER_ITER = 16


class GcbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gcb error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("radius", C.c_double), ("m", C.c_int32), ("seed", C.c_uint64), ("tol_abs", C.c_double),
                ("nc_max", C.c_int64), ("precision", C.c_int32), ("use_init", C.c_int32),
                ("init_idx", C.c_int64 * 3), ("warm_start", C.c_int32), ("monitor_every", C.c_int32),
                ("per_iter", C.c_int32), ("cull_volume", C.c_int32)]


class SelectInfo(C.Structure):
    _fields_ = [("nc", C.c_int64), ("iterations", C.c_int64), ("status", C.c_int32), ("converged", C.c_int32),
                ("final_max_err", C.c_double), ("final_rms_err", C.c_double), ("pairs_group", C.c_uint64),
                ("pairs_append", C.c_uint64), ("pairs_cert", C.c_uint64), ("ms_select", C.c_double),
                ("probed_iterations", C.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class Record(C.Structure):
    _fields_ = [("cap_support", C.c_int64), ("support", C.c_void_p), ("weights", C.c_void_p),
                ("cap_log", C.c_int64), ("log_group", C.c_void_p), ("log_node", C.c_void_p),
                ("log_err", C.c_void_p), ("log_appended", C.c_void_p), ("nc", C.c_int64),
                ("iterations", C.c_int64)]


class Request(C.Structure):
    _fields_ = [("mesh_key", C.c_int64), ("nb", C.c_int64), ("xyz", C.c_void_p), ("disp", C.c_void_p),
                ("params", Params), ("nv", C.c_int64), ("vol_xyz", C.c_void_p), ("in_dtype", C.c_int32),
                ("out_dtype", C.c_int32), ("out", C.c_void_p), ("t_arrival", C.c_double),
                ("record", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("state", C.c_int32), ("warm", C.c_int32), ("kept", C.c_int32), ("reserved", C.c_int32),
                ("info", SelectInfo), ("t_arrival", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double)]


_LIB = None


def lib():
    """Load libgcb.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        # PyTorch ships its own HIP runtime with the same soname as the system
        # one; loading torch first makes libgcb.so bind to that same runtime,
        # so device pointers and streams from torch are valid in the library
        # and only one runtime owns the GPU.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.gcb_version.restype = C.c_char_p
        L.gcb_partition.argtypes = [i64, i32, C.c_uint64, vp]
        L.gcb_create.argtypes = [C.POINTER(vp), C.c_int, vp]
        L.gcb_destroy.argtypes = [vp]
        L.gcb_destroy.restype = None
        L.gcb_last_error.argtypes = [vp]
        L.gcb_last_error.restype = C.c_char_p
        L.gcb_set_stream.argtypes = [vp, vp]
        L.gcb_set_boundary.argtypes = [vp, i64, vp, vp, C.c_int]
        L.gcb_set_displacement.argtypes = [vp, vp, C.c_int]
        L.gcb_set_params.argtypes = [vp, C.POINTER(Params)]
        L.gcb_set_groups.argtypes = [vp, vp, C.c_int]
        L.gcb_select.argtypes = [vp, C.POINTER(SelectInfo)]
        L.gcb_get_support.argtypes = [vp, vp, vp, C.c_int]
        L.gcb_get_log.argtypes = [vp, vp, vp, vp, vp, i64]
        L.gcb_get_log.restype = i64
        L.gcb_deform.argtypes = [vp, i64, vp, C.c_int, vp, C.c_int, C.c_int]
        L.gcb_deform_noalloc.argtypes = [vp, i64, vp, C.c_int, vp, C.c_int]
        L.gcb_set_kernel_timing.argtypes = [vp, i32]
        L.gcb_get_deform_pairs.argtypes = [vp, vp, vp]
        L.gcb_get_kernel_times.argtypes = [vp, vp, vp]
        L.gcb_deform_multi.argtypes = [vp, i32, vp, i64, vp, C.c_int, vp, C.c_int, C.c_int]
        L.gcb_certify.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.gcb_set_support.argtypes = [vp, vp, i64, C.c_int, C.POINTER(SelectInfo)]
        L.gcb_refactor.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(SelectInfo)]
        L.gcb_get_factor.argtypes = [vp, vp, C.c_int]
        L.gcb_get_monitor.argtypes = [vp, vp, vp, vp, i64]
        L.gcb_get_monitor.restype = i64
        L.gcb_batch_create.argtypes = [C.POINTER(vp), C.c_int, vp]
        L.gcb_batch_destroy.argtypes = [vp]
        L.gcb_batch_destroy.restype = None
        L.gcb_batch_last_error.argtypes = [vp]
        L.gcb_batch_last_error.restype = C.c_char_p
        L.gcb_batch_begin.argtypes = [vp, vp]
        L.gcb_batch_step.argtypes = [vp, vp, i32, i32, vp]
        L.gcb_batch_step.restype = i32
        L.gcb_batch_end.argtypes = [vp, vp, C.POINTER(SelectInfo)]
        L.gcb_select_batch.argtypes = [vp, vp, i32, vp]
        L.gcb_deform_batch.argtypes = [vp, vp, i32, vp, vp, C.c_int, vp, C.c_int]
        L.gcb_batch_set_layout.argtypes = [vp, i32, i32, i32]
        L.gcb_server_clock.restype = C.c_double
        L.gcb_server_create.argtypes = [C.POINTER(vp), C.c_int, vp, C.c_uint64, i32, i32]
        L.gcb_server_destroy.argtypes = [vp]
        L.gcb_server_destroy.restype = None
        L.gcb_server_last_error.argtypes = [vp]
        L.gcb_server_last_error.restype = C.c_char_p
        L.gcb_server_submit.argtypes = [vp, C.POINTER(Request), C.POINTER(i64)]
        L.gcb_server_progress.argtypes = [vp, i32, C.POINTER(i32)]
        L.gcb_server_result.argtypes = [vp, i64, C.POINTER(Result)]
        L.gcb_server_forget.argtypes = [vp, i64]
        L.gcb_deform_time.argtypes = [vp, C.POINTER(C.c_double)]
        L.gcb_server_memory.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(i32)]
        for name in EXPORTS:
            getattr(L, name)
        _LIB = L
    return _LIB


def version() -> str:
    return lib().gcb_version().decode()


def partition(nb: int, m: int, seed: int) -> np.ndarray:
    """The library's seeded partition (host function of the C ABI)."""
    g = np.empty(nb, dtype=np.int32)
    rc = lib().gcb_partition(int(nb), int(m), int(seed) & 0xFFFFFFFFFFFFFFFF, g.ctypes.data)
    if rc != GCB_OK:
        raise GcbError(rc, "gcb_partition rejected its arguments")
    return g


def _is_tensor(x) -> bool:
    return type(x).__module__.startswith("torch")


def _arg(x, dtype):
    """(pointer, mem kind, keep-alive) for a numpy array or a torch tensor."""
    if _is_tensor(x):
        import torch
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        want = {np.float64: torch.float64, np.float32: torch.float32, np.int32: torch.int32,
                np.int64: torch.int64}[dtype]
        if x.dtype != want:
            raise ValueError(f"expected {want}, got {x.dtype}")
        return x.data_ptr(), (GCB_MEM_DEVICE if x.is_cuda else GCB_MEM_HOST), x
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data, GCB_MEM_HOST, a


def _stream_of(x):
    """The caller's current HIP stream for a device tensor (0 = null stream), else None."""
    if _is_tensor(x) and x.is_cuda:
        import torch
        return int(torch.cuda.current_stream(x.device).cuda_stream)
    return None


@dataclasses.dataclass
class Log:
    group: np.ndarray
    node: np.ndarray
    err: np.ndarray
    appended: np.ndarray


class Context:
    """One GCB problem on one device (wraps a gcb_ctx)."""

    def __init__(self, device: int = 0, stream=None):
        h = C.c_void_p()
        rc = lib().gcb_create(C.byref(h), int(device), stream)
        if rc != GCB_OK:
            raise GcbError(rc, lib().gcb_last_error(None).decode())
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            lib().gcb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def _check(self, rc, ok=(GCB_OK,)):
        if rc not in ok:
            raise GcbError(rc, lib().gcb_last_error(self._h).decode())
        return rc

    def set_stream(self, stream: int):
        """Enqueue later calls on this hipStream_t handle (0: the null stream)."""
        self._check(lib().gcb_set_stream(self._h, C.c_void_p(stream) if stream else None))
        self._stream = stream

    def use_current_stream(self, tensor):
        s = _stream_of(tensor)
        if s is not None and s != getattr(self, "_stream", None):
            self.set_stream(s)

    def set_boundary(self, xyz, disp):
        px, mx, kx = _arg(xyz, np.float64)
        pd, md, kd = _arg(disp, np.float64)
        if mx != md:
            raise ValueError("xyz and disp must live in the same memory")
        nb = int(kx.shape[0])
        if tuple(kx.shape) != (nb, 3) or tuple(kd.shape) != (nb, 3):
            raise ValueError("xyz and disp must be (nb, 3)")
        self.use_current_stream(kx)
        self._check(lib().gcb_set_boundary(self._h, nb, px, pd, mx))
        self.nb = nb

    def set_displacement(self, disp):
        pd, md, kd = _arg(disp, np.float64)
        self.use_current_stream(kd)
        self._check(lib().gcb_set_displacement(self._h, pd, md))

    def set_params(self, radius: float, m: int, tol_abs: float, nc_max: int | None = None, seed: int = 0,
                   precision: int = GCB_PREC_FP64, init_idx=None, warm_start: bool = False, monitor_every: int = 0,
                   per_iter: int = 0, cull_volume: bool = False):
        """warm_start: start from the support set of the last finished selection (same
        boundary, radius, m and seed; new displacements via set_displacement).
        per_iter > 1: the several-nodes-per-iteration variant (up to per_iter nodes appended
        per iteration; the log's appended entries are counts).
        cull_volume: FP64 deformations skip (point, support) pairs farther apart than R."""
        p = Params()
        p.radius = float(radius)
        p.m = int(m)
        p.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        p.tol_abs = float(tol_abs)
        p.nc_max = int(self.nb if nc_max is None else nc_max)
        p.precision = int(precision)
        p.use_init = 0 if init_idx is None else 1
        if init_idx is not None:
            for t in range(3):
                p.init_idx[t] = int(init_idx[t])
        p.warm_start = 1 if warm_start else 0
        p.monitor_every = int(monitor_every)
        p.per_iter = int(per_iter)
        p.cull_volume = 1 if cull_volume else 0
        self._check(lib().gcb_set_params(self._h, C.byref(p)))

    def set_groups(self, group_of):
        if group_of is None:
            self._check(lib().gcb_set_groups(self._h, None, GCB_MEM_HOST))
            return
        pg, mg, kg = _arg(group_of, np.int32)
        self._check(lib().gcb_set_groups(self._h, pg, mg))

    def select(self) -> dict:
        info = SelectInfo()
        self._check(lib().gcb_select(self._h, C.byref(info)), ok=(GCB_OK, GCB_NOT_CONVERGED))
        self.nc = info.nc
        return info.as_dict()

    def get_support(self):
        idx = np.empty(self.nc, dtype=np.int64)
        w = np.empty((self.nc, 3), dtype=np.float64)
        self._check(lib().gcb_get_support(self._h, idx.ctypes.data, w.ctypes.data, GCB_MEM_HOST))
        return idx, w

    def get_log(self) -> Log:
        n = lib().gcb_get_log(self._h, None, None, None, None, 0)
        if n < 0:
            self._check(int(n))
        g = np.empty(n, np.int32)
        nd = np.empty(n, np.int64)
        e = np.empty(n, np.float64)
        a = np.empty(n, np.int8)
        lib().gcb_get_log(self._h, g.ctypes.data, nd.ctypes.data, e.ctypes.data, a.ctypes.data, n)
        return Log(g, nd, e, a)

    def get_monitor(self):
        """(iteration, max_err, rms_err) arrays of the monitor samples of the last selection."""
        n = lib().gcb_get_monitor(self._h, None, None, None, 0)
        if n < 0:
            self._check(int(n))
        it = np.empty(n, np.int64)
        mx = np.empty(n)
        rm = np.empty(n)
        if n:
            lib().gcb_get_monitor(self._h, it.ctypes.data, mx.ctypes.data, rm.ctypes.data, n)
        return it, mx, rm

    def deform(self, xyz, out=None, out_dtype=None):
        """Eq. (6) at the points xyz (nv, 3): numpy (host) or torch (host/device)."""
        if _is_tensor(xyz):
            import torch
            in_dt = GCB_F64 if xyz.dtype == torch.float64 else GCB_F32
            if out is None:
                odt = torch.float64 if out_dtype in (None, np.float64, torch.float64) else torch.float32
                out = torch.empty(xyz.shape, dtype=odt, device=xyz.device)
            px, mx, kx = _arg(xyz, np.float64 if in_dt == GCB_F64 else np.float32)
            out_dt = GCB_F64 if out.dtype == torch.float64 else GCB_F32
            po, mo, ko = _arg(out, np.float64 if out_dt == GCB_F64 else np.float32)
        else:
            a = np.ascontiguousarray(xyz)
            in_dt = GCB_F32 if a.dtype == np.float32 else GCB_F64
            px, mx, kx = _arg(a, np.float32 if in_dt == GCB_F32 else np.float64)
            if out is None:
                out = np.empty(a.shape, dtype=np.float32 if out_dtype == np.float32 else np.float64)
            out_dt = GCB_F32 if out.dtype == np.float32 else GCB_F64
            po, mo, ko = out.ctypes.data, GCB_MEM_HOST, out
        if mx != mo:
            raise ValueError("xyz and out must live in the same memory")
        nv = int(kx.shape[0])
        self.use_current_stream(kx)
        self._check(lib().gcb_deform(self._h, nv, px, in_dt, po, out_dt, mx))
        return out

    def deform_noalloc(self, xyz, out):
        """Eq. (6) through the allocation-free entry point: xyz (nv, 3) and out
        (nv, 3) are device tensors on the context's device, allocated by the
        caller; the library allocates nothing."""
        import torch
        if not (_is_tensor(xyz) and _is_tensor(out) and xyz.is_cuda and out.is_cuda):
            raise ValueError("deform_noalloc takes device tensors for xyz and out")
        in_dt = GCB_F64 if xyz.dtype == torch.float64 else GCB_F32
        out_dt = GCB_F64 if out.dtype == torch.float64 else GCB_F32
        px, _, kx = _arg(xyz, np.float64 if in_dt == GCB_F64 else np.float32)
        po, _, ko = _arg(out, np.float64 if out_dt == GCB_F64 else np.float32)
        if kx.dim() != 2 or kx.shape[1] != 3 or tuple(ko.shape) != tuple(kx.shape):
            raise ValueError("xyz and out must have the same shape (nv, 3)")
        self.use_current_stream(kx)
        self._check(lib().gcb_deform_noalloc(self._h, int(kx.shape[0]), px, in_dt, po, out_dt))
        return out

    def deform_pairs(self) -> tuple:
        """(evaluated, dense) (point, support) pairs of the last culled deformation."""
        ev = C.c_uint64()
        dn = C.c_uint64()
        self._check(lib().gcb_get_deform_pairs(self._h, C.byref(ev), C.byref(dn)))
        return int(ev.value), int(dn.value)

    def set_kernel_timing(self, on: bool):
        """Record HIP events between the greedy kernels of later selections (slower, same results)."""
        self._check(lib().gcb_set_kernel_timing(self._h, 1 if on else 0))

    def kernel_times(self) -> dict:
        """Summed device ms and launch counts per greedy kernel of the last timed selection."""
        ms = (C.c_double * 4)()
        n = (C.c_int64 * 4)()
        self._check(lib().gcb_get_kernel_times(self._h, ms, n))
        names = ("sweep", "k_factor_l", "k_factor_u", "certificate")
        return {k: {"ms": ms[q], "launches": int(n[q])} for q, k in enumerate(names)}

    def deform_time(self) -> float:
        """Device milliseconds of the last deform's kernels (waits for them)."""
        ms = C.c_double()
        self._check(lib().gcb_deform_time(self._h, C.byref(ms)))
        return ms.value

    def deform_multi(self, modes, xyz, out=None, out_dtype=None):
        """K displacement fields of the boundary (nb, 3K) solved on the selected
        supports and evaluated at xyz (nv, 3): returns (nv, 3K)."""
        if _is_tensor(xyz):
            import torch
            in_dt = GCB_F64 if xyz.dtype == torch.float64 else GCB_F32
            if not _is_tensor(modes) or not modes.is_cuda:
                raise ValueError("with device points, modes must be a device tensor too")
            rc = int(modes.shape[1])
            if out is None:
                odt = torch.float64 if out_dtype in (None, np.float64, torch.float64) else torch.float32
                out = torch.empty((xyz.shape[0], rc), dtype=odt, device=xyz.device)
            px, mx, kx = _arg(xyz, np.float64 if in_dt == GCB_F64 else np.float32)
            pm, mm, km = _arg(modes, np.float64)
            out_dt = GCB_F64 if out.dtype == torch.float64 else GCB_F32
            po, mo, ko = _arg(out, np.float64 if out_dt == GCB_F64 else np.float32)
        else:
            a = np.ascontiguousarray(xyz)
            in_dt = GCB_F32 if a.dtype == np.float32 else GCB_F64
            px, mx, kx = _arg(a, np.float32 if in_dt == GCB_F32 else np.float64)
            pm, mm, km = _arg(modes, np.float64)
            rc = int(km.shape[1])
            if out is None:
                out = np.empty((a.shape[0], rc), dtype=np.float32 if out_dtype == np.float32 else np.float64)
            out_dt = GCB_F32 if out.dtype == np.float32 else GCB_F64
            po, mo, ko = out.ctypes.data, GCB_MEM_HOST, out
        if rc % 3:
            raise ValueError("modes must have 3K columns")
        if not (mx == mo == mm):
            raise ValueError("modes, xyz and out must live in the same memory")
        self.use_current_stream(kx)
        self._check(lib().gcb_deform_multi(self._h, rc // 3, pm, int(kx.shape[0]), px, in_dt, po, out_dt, mx))
        return out

    def set_support(self, idx) -> dict:
        """Use the support set idx (selection order) instead of selecting: the
        factor is rebuilt from scratch (dense FP64) and W fitted to the current field."""
        p, m, k = _arg(idx, np.int64)
        info = SelectInfo()
        self._check(lib().gcb_set_support(self._h, p, int(k.shape[0]), m, C.byref(info)))
        self.nc = info.nc
        return info.as_dict()

    def get_factor(self) -> np.ndarray:
        """The inverse factor M = L^-1 (nc, nc), dense lower triangular."""
        n = int(self.nc)
        p = np.empty(n * (n + 1) // 2)
        self._check(lib().gcb_get_factor(self._h, p.ctypes.data, GCB_MEM_HOST))
        M = np.zeros((n, n))
        M[np.tril_indices(n)] = p
        return M

    def refactor(self):
        """Rebuild the inverse factor of the current support set; returns (drift, info)."""
        d = C.c_double()
        info = SelectInfo()
        self._check(lib().gcb_refactor(self._h, C.byref(d), C.byref(info)))
        return d.value, info.as_dict()

    def certify(self):
        mx, rms = C.c_double(), C.c_double()
        self._check(lib().gcb_certify(self._h, C.byref(mx), C.byref(rms)))
        return mx.value, rms.value


class Batch:
    """Several contexts advanced by shared launches (wraps a gcb_batch).

    Contexts handed to a batch run on the batch's stream from then on."""

    def __init__(self, device: int = 0, stream: int | None = None):
        """stream: a hipStream_t handle; None takes torch's current stream of the device."""
        if stream is None:
            import torch
            stream = int(torch.cuda.current_stream(device).cuda_stream)
        h = C.c_void_p()
        rc = lib().gcb_batch_create(C.byref(h), int(device), C.c_void_p(stream) if stream else None)
        if rc != GCB_OK:
            raise GcbError(rc, lib().gcb_batch_last_error(None).decode())
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            lib().gcb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def _raise(self, rc, ctxs=()):
        msg = lib().gcb_batch_last_error(self._h).decode()
        for c in ctxs:
            cm = lib().gcb_last_error(c._h).decode()
            if cm:
                msg = (msg + "; " if msg else "") + cm
        raise GcbError(rc, msg)

    @staticmethod
    def _handles(ctxs):
        return (C.c_void_p * len(ctxs))(*[c._h.value for c in ctxs])

    def set_layout(self, sweep_tpl: int = 0, factor_rpw: int = 0, lone_graph: bool = True):
        """Tile shapes of the batched iterations (0: automatic); see paper_2004_04817_amd.autotune."""
        rc = lib().gcb_batch_set_layout(self._h, int(sweep_tpl), int(factor_rpw), 1 if lone_graph else 0)
        if rc != GCB_OK:
            self._raise(rc)

    def begin(self, ctx: Context):
        rc = lib().gcb_batch_begin(self._h, ctx._h)
        if rc != GCB_OK:
            self._raise(rc, [ctx])

    def step(self, ctxs, iterations: int = 64) -> np.ndarray:
        """Advance every running context; returns the 0/1 running flags."""
        run = np.zeros(len(ctxs), np.int32)
        n = lib().gcb_batch_step(self._h, self._handles(ctxs), len(ctxs), int(iterations), run.ctypes.data)
        if n < 0:
            self._raise(int(n), ctxs)
        return run

    def end(self, ctx: Context) -> dict:
        info = SelectInfo()
        rc = lib().gcb_batch_end(self._h, ctx._h, C.byref(info))
        if rc not in (GCB_OK, GCB_NOT_CONVERGED):
            self._raise(rc, [ctx])
        ctx.nc = info.nc
        return info.as_dict()

    def select(self, ctxs) -> list:
        infos = (SelectInfo * len(ctxs))()
        rc = lib().gcb_select_batch(self._h, self._handles(ctxs), len(ctxs), infos)
        if rc not in (GCB_OK, GCB_NOT_CONVERGED):
            self._raise(rc, ctxs)
        out = []
        for c, inf in zip(ctxs, infos):
            c.nc = inf.nc
            out.append(inf.as_dict())
        return out

    def deform(self, ctxs, xyzs, outs=None, out_dtype=None):
        """Eq. (6) for every context in one launch; xyzs are device tensors (nv_i, 3)."""
        import torch
        if len(xyzs) != len(ctxs):
            raise ValueError("one point set per context")
        if not xyzs:
            return []
        in_dt = GCB_F64 if xyzs[0].dtype == torch.float64 else GCB_F32
        if outs is None:
            odt = torch.float64 if out_dtype in (None, np.float64, torch.float64) else torch.float32
            outs = [torch.empty(x.shape, dtype=odt, device=x.device) for x in xyzs]
        out_dt = GCB_F64 if outs[0].dtype == torch.float64 else GCB_F32
        keep = []
        for x, o in zip(xyzs, outs):
            px, mx, kx = _arg(x, np.float64 if in_dt == GCB_F64 else np.float32)
            po, mo, ko = _arg(o, np.float64 if out_dt == GCB_F64 else np.float32)
            if mx != GCB_MEM_DEVICE or mo != GCB_MEM_DEVICE:
                raise ValueError("batched deformation takes device tensors")
            if tuple(kx.shape) != tuple(ko.shape) or kx.shape[-1] != 3:
                raise ValueError("points and outputs must be (nv, 3) of equal shape")
            keep.append((px, po, int(kx.shape[0])))
        nv = (C.c_int64 * len(keep))(*[k[2] for k in keep])
        xp = (C.c_void_p * len(keep))(*[k[0] for k in keep])
        op = (C.c_void_p * len(keep))(*[k[1] for k in keep])
        rc = lib().gcb_deform_batch(self._h, self._handles(ctxs), len(ctxs), nv, xp, in_dt, op, out_dt)
        if rc != GCB_OK:
            self._raise(rc, ctxs)
        return outs


def clock() -> float:
    """The serving clock (monotonic seconds) that request arrival times use."""
    return float(lib().gcb_server_clock())


class Server:
    """Request loop (wraps a gcb_server): FIFO admission by slots and device
    memory, continuous batching (GCB_SERVE_BATCH) and resident meshes served by
    warm starts (GCB_SERVE_CACHE)."""

    def __init__(self, device: int = 0, hbm_budget: int = 8 << 30, max_active: int = 32,
                 flags: int = GCB_SERVE_BATCH | GCB_SERVE_CACHE, stream: int | None = None):
        if stream is None:
            import torch
            stream = int(torch.cuda.current_stream(device).cuda_stream)
        h = C.c_void_p()
        rc = lib().gcb_server_create(C.byref(h), int(device), C.c_void_p(stream) if stream else None,
                                     int(hbm_budget), int(max_active), int(flags))
        if rc != GCB_OK:
            raise GcbError(rc, "gcb_server_create failed")
        self._h = h
        self._keep = {}
        self._records = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().gcb_server_destroy(self._h)
            self._h = None
            self._keep = {}
            self._records = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def _check(self, rc):
        if rc != GCB_OK:
            raise GcbError(rc, lib().gcb_server_last_error(self._h).decode())

    def submit(self, xyz, disp, radius, m, tol_abs, seed=0, nc_max=None, mesh_key=-1, vol=None, out=None,
               t_arrival=-1.0, record=False, log_cap=1 << 18) -> int:
        """Queue a request: boundary (nb, 3) host arrays, volume and output device tensors.
        record=True: the selection's support set, weights and per-iteration log are copied
        out when it finishes (``result`` then holds them; the copies synchronise the stream)."""
        import torch
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        disp = np.ascontiguousarray(disp, dtype=np.float64)
        nb = xyz.shape[0]
        r = Request()
        r.mesh_key = int(mesh_key)
        r.nb = nb
        r.xyz = xyz.ctypes.data
        r.disp = disp.ctypes.data
        r.params.radius = float(radius)
        r.params.m = int(m)
        r.params.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        r.params.tol_abs = float(tol_abs)
        r.params.nc_max = int(nb if nc_max is None else nc_max)
        keep = [xyz, disp]
        if vol is not None:
            if not (_is_tensor(vol) and vol.is_cuda and _is_tensor(out) and out.is_cuda):
                raise ValueError("vol and out must be device tensors")
            if not (vol.is_contiguous() and out.is_contiguous()) or tuple(vol.shape) != tuple(out.shape):
                raise ValueError("vol and out must be contiguous (nv, 3) tensors")
            r.nv = int(vol.shape[0])
            r.vol_xyz = vol.data_ptr()
            r.out = out.data_ptr()
            r.in_dtype = GCB_F64 if vol.dtype == torch.float64 else GCB_F32
            r.out_dtype = GCB_F64 if out.dtype == torch.float64 else GCB_F32
            keep += [vol, out]
        else:
            r.in_dtype = r.out_dtype = GCB_F64
        r.t_arrival = float(t_arrival)
        rec = None
        if record:
            ncap = int(r.params.nc_max)
            arrs = {"support": np.zeros(ncap, dtype=np.int64), "weights": np.zeros((ncap, 3)),
                    "log_group": np.zeros(log_cap, dtype=np.int32), "log_node": np.zeros(log_cap, dtype=np.int64),
                    "log_err": np.zeros(log_cap), "log_appended": np.zeros(log_cap, dtype=np.int8)}
            rec = Record(ncap, arrs["support"].ctypes.data, arrs["weights"].ctypes.data, int(log_cap),
                         arrs["log_group"].ctypes.data, arrs["log_node"].ctypes.data, arrs["log_err"].ctypes.data,
                         arrs["log_appended"].ctypes.data, 0, 0)
            r.record = C.addressof(rec)
            keep += [rec, arrs]
        t = C.c_int64()
        self._check(lib().gcb_server_submit(self._h, C.byref(r), C.byref(t)))
        self._keep[t.value] = keep
        if rec is not None:
            self._records[t.value] = (rec, arrs)
        return t.value

    def progress(self, iterations: int = 16) -> int:
        n = C.c_int32()
        self._check(lib().gcb_server_progress(self._h, int(iterations), C.byref(n)))
        return n.value

    def result(self, ticket: int) -> dict:
        r = Result()
        self._check(lib().gcb_server_result(self._h, int(ticket), C.byref(r)))
        d = {"state": r.state, "warm": bool(r.warm), "kept": bool(r.kept), "t_arrival": r.t_arrival,
             "t_admit": r.t_admit,
             "t_done": r.t_done}
        d.update(r.info.as_dict())
        if r.state == 3 and int(ticket) in self._records:
            rec, arrs = self._records[int(ticket)]
            nc, it = int(rec.nc), int(rec.iterations)
            if it > len(arrs["log_group"]):
                raise GcbError(GCB_E_INVALID, f"record log holds {len(arrs['log_group'])} of {it} iterations")
            d["support"] = arrs["support"][:nc].copy()
            d["weights"] = arrs["weights"][:nc].copy()
            d["log"] = {k: arrs[k][:it].copy() for k in ("log_group", "log_node", "log_err", "log_appended")}
        if r.state == 3 or r.state < 0:
            self._keep.pop(int(ticket), None)
            self._records.pop(int(ticket), None)
        return d

    def forget(self, ticket: int):
        """Drop the server's record of a finished or failed ticket."""
        self._check(lib().gcb_server_forget(self._h, int(ticket)))

    def memory(self):
        b, n = C.c_uint64(), C.c_int32()
        self._check(lib().gcb_server_memory(self._h, C.byref(b), C.byref(n)))
        return b.value, n.value

    def last_error(self) -> str:
        return lib().gcb_server_last_error(self._h).decode()


def select(xyz, disp, radius, m, tol_abs, nc_max=None, seed=0, precision=GCB_PREC_FP64, init_idx=None,
           group_of=None, device=0):
    """Convenience: run one selection and return (context, info)."""
    ctx = Context(device)
    ctx.set_boundary(xyz, disp)
    ctx.set_params(radius, m, tol_abs, nc_max=nc_max, seed=seed, precision=precision, init_idx=init_idx)
    if group_of is not None:
        ctx.set_groups(group_of)
    info = ctx.select()
    return ctx, info

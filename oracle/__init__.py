"""CPU FP64 oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg import this package.  It loads ``liboracle.so`` (plain C, built from
``gcb_oracle.c`` by ``oracle/build.py``) and offers a NumPy brute-force twin
in :mod:`oracle.brute`.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

ORC_OK, ORC_NOT_CONVERGED, ORC_E_INVALID, ORC_E_SINGULAR = 0, 1, -1, -4


class _Problem(C.Structure):
    _fields_ = [("nb", C.c_int64), ("xyz", C.c_void_p), ("disp", C.c_void_p), ("radius", C.c_double),
                ("m", C.c_int32), ("seed", C.c_uint64), ("tol_abs", C.c_double), ("nc_max", C.c_int64),
                ("group_of", C.c_void_p), ("init_idx", C.c_void_p), ("nthreads", C.c_int32),
                ("warm_S", C.c_void_p), ("warm_n", C.c_int64), ("per_iter", C.c_int32)]


class _Info(C.Structure):
    _fields_ = [("nc", C.c_int64), ("iterations", C.c_int64), ("status", C.c_int32), ("converged", C.c_int32),
                ("final_max_err", C.c_double), ("final_rms_err", C.c_double), ("pairs_group", C.c_uint64),
                ("pairs_append", C.c_uint64), ("pairs_cert", C.c_uint64), ("t_error", C.c_double),
                ("t_solve", C.c_double), ("singular_node", C.c_int64)]


class _Log(C.Structure):
    _fields_ = [("cap", C.c_int64), ("group", C.c_void_p), ("node", C.c_void_p), ("err", C.c_void_p),
                ("appended", C.c_void_p), ("monitor_every", C.c_int32), ("mon_max", C.c_void_p),
                ("mon_rms", C.c_void_p), ("n_monitor", C.c_int64)]


def load(path: str):
    """Open an oracle shared library at ``path`` and declare its signatures."""
    L = C.CDLL(path)
    L.orc_phi.restype = C.c_double
    L.orc_phi.argtypes = [C.c_double]
    L.orc_splitmix64_next.restype = C.c_uint64
    L.orc_splitmix64_next.argtypes = [C.POINTER(C.c_uint64)]
    L.orc_partition.argtypes = [C.c_int64, C.c_int32, C.c_uint64, C.c_void_p]
    L.orc_initial_nodes.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_interpolate.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_int64,
                                  C.c_void_p, C.c_void_p, C.c_int32]
    L.orc_rc_create.restype = C.c_void_p
    L.orc_rc_create.argtypes = [C.c_int32]
    L.orc_rc_destroy.argtypes = [C.c_void_p]
    L.orc_rc_size.restype = C.c_int64
    L.orc_rc_size.argtypes = [C.c_void_p]
    L.orc_rc_append.restype = C.c_int
    L.orc_rc_append.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]
    L.orc_rc_weights.argtypes = [C.c_void_p, C.c_void_p]
    L.orc_rc_factor.argtypes = [C.c_void_p, C.c_void_p]
    L.orc_select.restype = C.c_int
    L.orc_select.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_void_p, C.POINTER(_Log), C.POINTER(_Info)]
    L.orc_solve_on_support.restype = C.c_int
    L.orc_solve_on_support.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_int32,
                                       C.c_void_p, C.c_void_p]
    L.orc_inverse_factor.restype = C.c_int
    L.orc_inverse_factor.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_void_p]
    L.orc_validate.restype = C.c_int64
    L.orc_validate.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_double, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    L.orc_validate_block.restype = C.c_int64
    L.orc_validate_block.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_int64, C.c_int64, C.c_void_p,
                                     C.c_void_p, C.c_double, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    return L


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        _LIB = load(path)
    return _LIB


class use_library:
    """Context manager: route every oracle call to another build (used by the
    tests that plant a mistake in a copy of the oracle source)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _LIB
        self._saved = lib()
        _LIB = load(self.path)
        return _LIB

    def __exit__(self, *exc):
        global _LIB
        _LIB = self._saved
        return False


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data


def phi(eta: float) -> float:
    return lib().orc_phi(float(eta))


def splitmix64(seed: int, count: int) -> np.ndarray:
    st = C.c_uint64(seed & 0xFFFFFFFFFFFFFFFF)
    return np.array([lib().orc_splitmix64_next(C.byref(st)) for _ in range(count)], dtype=np.uint64)


def partition(nb: int, m: int, seed: int) -> np.ndarray:
    g = np.empty(nb, dtype=np.int32)
    lib().orc_partition(nb, m, seed & 0xFFFFFFFFFFFFFFFF, _ptr(g))
    return g


def initial_nodes(xyz, disp) -> np.ndarray:
    xyz, disp = _f64(xyz), _f64(disp)
    out = np.empty(3, dtype=np.int64)
    lib().orc_initial_nodes(xyz.shape[0], _ptr(xyz), _ptr(disp), _ptr(out))
    return out


def interpolate(sup_xyz, w, radius, tgt_xyz, nthreads: int = 0) -> np.ndarray:
    """Eq. (1)/(6) at arbitrary targets; w is (nc, K)."""
    sup_xyz, tgt_xyz = _f64(sup_xyz), _f64(tgt_xyz)
    w = _f64(w)
    if w.ndim == 1:
        w = w[:, None]
    K = w.shape[1]
    out = np.empty((tgt_xyz.shape[0], K))
    lib().orc_interpolate(sup_xyz.shape[0], _ptr(sup_xyz), _ptr(w), K, float(radius), tgt_xyz.shape[0],
                          _ptr(tgt_xyz), _ptr(out), int(nthreads))
    return out


class RC:
    """Recurrence-Cholesky factor of Phi_S (grows one row per append)."""

    def __init__(self, K: int = 3):
        self._h = lib().orc_rc_create(K)
        self.K = K

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_rc_destroy(self._h)
            self._h = None

    @property
    def n(self) -> int:
        return lib().orc_rc_size(self._h)

    def append(self, b, rhs, phi0: float = 1.0) -> int:
        b = _f64(b) if len(b) else np.zeros(1)
        rhs = _f64(rhs)
        return lib().orc_rc_append(self._h, _ptr(b), float(phi0), _ptr(rhs))

    def weights(self) -> np.ndarray:
        w = np.empty((max(self.n, 1), self.K))
        lib().orc_rc_weights(self._h, _ptr(w))
        return w[: self.n]

    def factor(self) -> np.ndarray:
        L = np.empty((max(self.n, 1), max(self.n, 1)))
        lib().orc_rc_factor(self._h, _ptr(L))
        return L[: self.n, : self.n]


@dataclasses.dataclass
class SelectResult:
    status: int
    S: np.ndarray          # support node indices in selection order
    W: np.ndarray          # (nc, 3) weights
    nc: int
    iterations: int
    converged: bool
    final_max_err: float
    final_rms_err: float
    pairs_group: int
    pairs_append: int
    pairs_cert: int
    t_error: float
    t_solve: float
    singular_node: int
    log_group: np.ndarray
    log_node: np.ndarray
    log_err: np.ndarray
    log_appended: np.ndarray
    mon_max: np.ndarray = None
    mon_rms: np.ndarray = None


def _problem(xyz, disp, radius, m, seed, tol_abs, nc_max, group_of=None, init_idx=None, nthreads=0, warm_S=None,
             per_iter=1):
    if warm_S is not None:
        warm_S = np.ascontiguousarray(warm_S, dtype=np.int64)
    keep = [xyz, disp, group_of, init_idx, warm_S]
    p = _Problem(xyz.shape[0], _ptr(xyz), _ptr(disp), float(radius), int(m), int(seed) & 0xFFFFFFFFFFFFFFFF,
                 float(tol_abs), int(nc_max), _ptr(group_of), _ptr(init_idx), int(nthreads),
                 _ptr(warm_S), 0 if warm_S is None else len(warm_S), int(per_iter))
    return p, keep


def select(xyz, disp, radius, m, tol_abs, nc_max=None, seed=0, group_of=None, init_idx=None,
           nthreads: int = 0, log_cap: int | None = None, warm_S=None, monitor_every: int = 0,
           per_iter: int = 1) -> SelectResult:
    """Algorithm 1 (GCB greedy) in FP64 with the RC solve.

    warm_S: a kept support set (>= 3 distinct nodes, in order) to start from
    instead of the three starting nodes; the selection ends at once when it
    already meets E* for these displacements, else the loop runs from k = len(warm_S).
    monitor_every: record the all-node max / RMS error after every that many iterations.
    per_iter: nodes appended per iteration (1: Algorithm 1; p > 1: the top p of the
    group over E*, ranked by error descending then index; log_appended holds counts)."""
    xyz, disp = _f64(xyz), _f64(disp)
    nb = xyz.shape[0]
    nc_max = nb if nc_max is None else int(nc_max)
    if group_of is not None:
        group_of = np.ascontiguousarray(group_of, dtype=np.int32)
    if init_idx is not None:
        init_idx = np.ascontiguousarray(init_idx, dtype=np.int64)
    p, keep = _problem(xyz, disp, radius, m, seed, tol_abs, nc_max, group_of, init_idx, nthreads, warm_S, per_iter)
    if log_cap is None:
        log_cap = (nc_max + 1) * int(m) + 8
    lg = np.empty(log_cap, dtype=np.int32)
    ln = np.empty(log_cap, dtype=np.int64)
    le = np.empty(log_cap, dtype=np.float64)
    la = np.empty(log_cap, dtype=np.int8)
    mmx = np.empty(log_cap, dtype=np.float64)
    mrm = np.empty(log_cap, dtype=np.float64)
    log = _Log(log_cap, _ptr(lg), _ptr(ln), _ptr(le), _ptr(la), int(monitor_every), _ptr(mmx), _ptr(mrm), 0)
    S = np.empty(max(nc_max, 3), dtype=np.int64)
    W = np.empty((max(nc_max, 3), 3))
    info = _Info()
    st = lib().orc_select(C.byref(p), _ptr(S), _ptr(W), C.byref(log), C.byref(info))
    del keep
    it = min(info.iterations, log_cap)
    return SelectResult(st, S[: info.nc].copy(), W[: info.nc].copy(), info.nc, info.iterations,
                        bool(info.converged), info.final_max_err, info.final_rms_err, info.pairs_group,
                        info.pairs_append, info.pairs_cert, info.t_error, info.t_solve, info.singular_node,
                        lg[:it].copy(), ln[:it].copy(), le[:it].copy(), la[:it].copy(),
                        mmx[: log.n_monitor].copy(), mrm[: log.n_monitor].copy())


def validate(xyz, disp, radius, m, tol_abs, S_init, group, node, appended, tau, nc_max=None, seed=0,
             group_of=None, init_idx=None, nthreads: int = 0, warm_S=None):
    """Follow-mode replay of a foreign selection; returns (first_bad or -1, reason, max_gap)."""
    xyz, disp = _f64(xyz), _f64(disp)
    nb = xyz.shape[0]
    nc_max = nb if nc_max is None else int(nc_max)
    if group_of is not None:
        group_of = np.ascontiguousarray(group_of, dtype=np.int32)
    if init_idx is not None:
        init_idx = np.ascontiguousarray(init_idx, dtype=np.int64)
    p, keep = _problem(xyz, disp, radius, m, seed, tol_abs, nc_max, group_of, init_idx, nthreads, warm_S)
    S_init = np.ascontiguousarray(S_init[:3], dtype=np.int64)
    group = np.ascontiguousarray(group, dtype=np.int32)
    node = np.ascontiguousarray(node, dtype=np.int64)
    appended = np.ascontiguousarray(appended, dtype=np.int8)
    reason = C.c_int32(0)
    gap = C.c_double(0.0)
    bad = lib().orc_validate(C.byref(p), _ptr(S_init), len(group), _ptr(group), _ptr(node), _ptr(appended),
                             float(tau), C.byref(reason), C.byref(gap))
    del keep
    return int(bad), int(reason.value), float(gap.value)


def validate_block(xyz, disp, radius, m, tol_abs, S_seq, group, appended, tau, per_iter, nc_max=None, seed=0,
                   group_of=None, init_idx=None, nthreads: int = 0):
    """Follow-mode replay of a foreign run of the several-nodes-per-iteration variant
    (S_seq: the whole support sequence; appended: per-iteration counts); returns
    (first_bad or -1, reason, max_gap)."""
    xyz, disp = _f64(xyz), _f64(disp)
    nb = xyz.shape[0]
    nc_max = nb if nc_max is None else int(nc_max)
    if group_of is not None:
        group_of = np.ascontiguousarray(group_of, dtype=np.int32)
    if init_idx is not None:
        init_idx = np.ascontiguousarray(init_idx, dtype=np.int64)
    p, keep = _problem(xyz, disp, radius, m, seed, tol_abs, nc_max, group_of, init_idx, nthreads, None, per_iter)
    S_seq = np.ascontiguousarray(S_seq, dtype=np.int64)
    group = np.ascontiguousarray(group, dtype=np.int32)
    appended = np.ascontiguousarray(appended, dtype=np.int8)
    reason = C.c_int32(0)
    gap = C.c_double(0.0)
    bad = lib().orc_validate_block(C.byref(p), _ptr(S_seq), len(S_seq), len(group), _ptr(group), _ptr(appended),
                                   float(tau), C.byref(reason), C.byref(gap))
    del keep
    return int(bad), int(reason.value), float(gap.value)


def inverse_factor(xyz, S, radius) -> np.ndarray:
    """M = L^-1 (n, n) with L L^T = Phi_S for the support set S in its order."""
    xyz = _f64(xyz)
    S = np.ascontiguousarray(S, dtype=np.int64)
    M = np.empty((max(len(S), 1), max(len(S), 1)))
    st = lib().orc_inverse_factor(xyz.shape[0], _ptr(xyz), _ptr(S), len(S), float(radius), _ptr(M))
    if st != ORC_OK:
        raise RuntimeError(f"orc_inverse_factor: status {st}")
    return M[: len(S), : len(S)]


def solve_on_support(xyz, S, radius, D) -> np.ndarray:
    """Weights (n, K) of the K columns of D (nb, K) on support set S (in order)."""
    xyz = _f64(xyz)
    S = np.ascontiguousarray(S, dtype=np.int64)
    D = _f64(D)
    if D.ndim == 1:
        D = D[:, None]
    K = D.shape[1]
    W = np.empty((max(len(S), 1), K))
    st = lib().orc_solve_on_support(xyz.shape[0], _ptr(xyz), _ptr(S), len(S), float(radius), K, _ptr(D), _ptr(W))
    if st != ORC_OK:
        raise RuntimeError(f"orc_solve_on_support: status {st}")
    return W[: len(S)]


def cost_model(nc: float, nb: float, nv: float, m: float = 1.0) -> dict:
    """Operation counts of Table 1 and Section 3: RC solve 2Nc^3/3, errors
    3 Nc^2 Nb / (2m) (m = 1: traditional greedy), volume 10 Nc Nv."""
    return {"solve": 2.0 * nc ** 3 / 3.0, "errors": 3.0 * nc ** 2 * nb / (2.0 * m), "volume": 10.0 * nc * nv}

"""ctypes binding of ``librbfdef.so`` (the C ABI in ``include/rbfdef.h``).

Argument marshalling only: every step of the deformation runs in the library's HIP kernels.
torch tensors provide device memory (float64, CUDA/HIP device, structure-of-arrays ``[dim, n]``)
and ``torch.cuda`` streams. There is no CPU fallback: if the library is not built, or no GPU is
present, the calls raise.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import re
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "librbfdef.so")
HEADER = os.path.join(ROOT, "include", "rbfdef.h")

RBF_OK, RBF_W_CAP, RBF_W_BREAKDOWN = 0, 1, 2
RBF_E_INVALID, RBF_E_NOMEM, RBF_E_NOT_SPD, RBF_E_DEVICE, RBF_E_NOT_FOUND, RBF_E_BUSY = -1, -2, -3, -4, -5, -6
RBF_FP64, RBF_MIXED = 0, 1
RBF_WENDLAND_C2, RBF_WENDLAND_C0, RBF_WENDLAND_C4, RBF_WENDLAND_C6 = 0, 1, 2, 3
BASES = {"c2": RBF_WENDLAND_C2, "c0": RBF_WENDLAND_C0, "c4": RBF_WENDLAND_C4, "c6": RBF_WENDLAND_C6}


def _precision(precision, n_levels: int):
    """(precision code, per-level array or None) from "fp64", "mixed" or one of them per level."""
    code = lambda p: RBF_MIXED if p == "mixed" else RBF_FP64
    if isinstance(precision, str):
        return code(precision), None
    if len(precision) != n_levels:
        raise ValueError("one precision per level")
    return RBF_FP64, (_i32 * n_levels)(*[code(p) for p in precision])


_LEVEL_ARRAYS: dict = {}


def _level_arrays(radius, D, level_off):
    """ctypes copies of the per-level radii, support distances and offsets (cached by value)."""
    key = (tuple(radius), tuple(D), tuple(level_off))
    got = _LEVEL_ARRAYS.get(key)
    if got is None:
        nl = len(radius)
        got = ((_f64 * nl)(*[float(x) for x in radius]), (_f64 * nl)(*[float(x) for x in D]),
               (_i32 * (nl + 1))(*[int(x) for x in level_off]))
        if len(_LEVEL_ARRAYS) > 256:
            _LEVEL_ARRAYS.clear()
        _LEVEL_ARRAYS[key] = got
    return got


def _basis(name: str) -> int:
    if name not in BASES:
        raise ValueError(f"unknown basis {name!r}; one of {sorted(BASES)}")
    return BASES[name]
MAX_LEVELS = 8
RBF_STOP_SKIPPED, RBF_STOP_EPS, RBF_STOP_CAP, RBF_STOP_ALL_SELECTED, RBF_STOP_BREAKDOWN = -1, 0, 1, 2, 3
STOP_NAMES = {-1: "skipped", 0: "eps", 1: "cap", 2: "all_selected", 3: "breakdown"}
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3

_vp = ctypes.c_void_p
_i32, _i64, _u64, _f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double


class rbf_greedy_params(ctypes.Structure):
    _fields_ = [("dim", _i32), ("n_levels", _i32), ("radius", _f64 * MAX_LEVELS),
                ("eps_abs", _f64), ("level_reduction", _f64), ("max_ctrl_total", _i64),
                ("seed_idx", ctypes.POINTER(_i64)), ("seed_off", ctypes.POINTER(_i32)),
                ("precision", _i32), ("basis", _i32)]


class rbf_ctrl_set(ctypes.Structure):
    _fields_ = [("capacity", _i64), ("ctrl_idx", _vp), ("xc", _vp), ("alpha", _vp),
                ("e_final", _vp), ("n_levels_used", _i32), ("stop_reason", _i32),
                ("level_off", _i32 * (MAX_LEVELS + 1)), ("level_stop", _i32 * MAX_LEVELS),
                ("level_max_err", _f64 * MAX_LEVELS), ("level_in_max", _f64 * MAX_LEVELS),
                ("level_seconds", _f64 * MAX_LEVELS), ("level_fp32_err", _f64 * MAX_LEVELS),
                ("n_iterations", _i64), ("err_hist", _vp)]


class rbf_request(ctypes.Structure):
    _fields_ = [("geom", _vp), ("ds", _vp), ("params", rbf_greedy_params),
                ("D", _f64 * MAX_LEVELS), ("d_factor", _f64), ("warm_start", _i32), ("dv", _vp),
                ("out", ctypes.POINTER(rbf_ctrl_set))]


class rbf_req_info(ctypes.Structure):
    _fields_ = [("state", _i32), ("result", _i32), ("t_arrive", _f64), ("t_admit", _f64),
                ("t_start", _f64), ("t_done", _f64)]


_SIGS = {
    "rbf_ctx_create": (_i32, [_i32, _u64, ctypes.POINTER(_vp)]),
    "rbf_ctx_destroy": (_i32, [_vp]),
    "rbf_status_str": (ctypes.c_char_p, [_i32]),
    "rbf_last_error": (ctypes.c_char_p, []),
    "rbf_ctx_bytes_in_use": (_u64, [_vp]),
    "rbf_greedy_select": (_i32, [_vp, ctypes.POINTER(rbf_greedy_params), _i64, _vp, _vp,
                                 ctypes.POINTER(rbf_ctrl_set), _vp]),
    "rbf_solve_weights": (_i32, [_vp, _i32, _f64, _i64, _vp, _vp, _vp, _i32, _vp]),
    "rbf_volume_update": (_i32, [_vp, _i32, _i32, ctypes.POINTER(_f64), ctypes.POINTER(_f64),
                                 ctypes.POINTER(_i32), _i64, _vp, _vp, _i64, _vp, _vp, _vp, _i32,
                                 ctypes.POINTER(_i32), _i32, _vp]),
    "rbf_volume_update_noalloc": (_i32, [_vp, _i32, _i32, ctypes.POINTER(_f64), ctypes.POINTER(_f64),
                                         ctypes.POINTER(_i32), _i64, _vp, _vp, _i64, _vp, _vp, _vp, _i32,
                                         ctypes.POINTER(_i32), _i32, _vp]),
    "rbf_evaluate": (_i32, [_vp, _i32, _f64, _i64, _i64, _vp, _vp, _i64, _vp, _vp, _f64, _vp, _i32, _i32,
                            _vp]),
    "rbf_geom_create": (_i32, [_vp, _i32, _i64, _vp, _i64, _vp, _vp, ctypes.POINTER(_vp)]),
    "rbf_geom_release": (_i32, [_vp, _vp]),
    "rbf_geom_volume_update": (_i32, [_vp, _vp, _i32, ctypes.POINTER(_f64), ctypes.POINTER(_f64),
                                      ctypes.POINTER(_i32), _i64, _vp, _vp, _vp, _i32, ctypes.POINTER(_i32),
                                      _i32, _vp]),
    "rbf_submit": (_i32, [_vp, ctypes.POINTER(rbf_request), ctypes.POINTER(_u64)]),
    "rbf_poll": (_i32, [_vp, _u64, ctypes.POINTER(rbf_req_info)]),
    "rbf_wait": (_i32, [_vp, _u64, ctypes.POINTER(rbf_req_info)]),
    "rbf_now": (_f64, []),
    "rbf_ctx_set_timing": (_i32, [_vp, _i32]),
    "rbf_ctx_kernel_time": (_i32, [_vp, ctypes.c_char_p, ctypes.POINTER(_f64), ctypes.POINTER(_i64)]),
    "rbf_ctx_kernel_pairs": (_i32, [_vp, ctypes.c_char_p, ctypes.POINTER(_i64)]),
}

_lib = None
_live_ctx: set = set()   # contexts created through this binding and not yet destroyed


def _unload_at_exit() -> None:
    """Unload the library at interpreter exit, while the HIP runtime is still whole.

    hipcc registers each translation unit's module destructor (the unregistration of its GPU
    code object) with atexit() when the library is loaded. exit() runs such handlers in reverse
    order of registration, so any handler registered after the load (the HIP runtime's or a
    profiler's finalisation, when they initialise after this library was loaded) runs first, and
    the unregistration then calls into a runtime that is already torn down. dlclose() runs the
    library's handlers at once instead; Python's own atexit callbacks run before any C exit
    handler. Skipped while a context is alive (its worker threads run library code)."""
    global _lib
    if _lib is None or _live_ctx:
        return
    import _ctypes

    handle, _lib = _lib._handle, None
    _ctypes.dlclose(handle)


def header_functions() -> List[str]:
    """Names of every function the public header declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rbf_[a-z_0-9]+)\s*\(", text)))


def lib() -> ctypes.CDLL:
    """Load the HIP library. Raises when it has not been built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        atexit.register(_unload_at_exit)
    return _lib


class RbfError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        msg = f"{where}: {L.rbf_status_str(status).decode()} ({status}): {L.rbf_last_error().decode()}"
        super().__init__(msg)
        self.status = status


def _check(status: int, where: str) -> int:
    if status < 0:
        raise RbfError(status, where)
    return status


def _stream(stream) -> int:
    import torch

    if stream is None:
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)   # no Stream object per call
        if raw is not None:
            return raw(torch.cuda.current_device())
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev(t, name: str, dim: Optional[int] = None, n: Optional[int] = None, allow_ld: bool = False):
    """Validate a float64 device tensor [dim, n] and return (pointer, leading dimension)."""
    import torch

    if t is None:
        return None, 0
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP torch tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if t.dim() == 1:
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if n is not None and t.shape[0] != n:
            raise ValueError(f"{name} has {t.shape[0]} entries, expected {n}")
        return t.data_ptr(), t.shape[0]
    shape, stride = t.shape, t.stride()
    if len(shape) != 2:
        raise ValueError(f"{name} must be [dim, n]")
    if dim is not None and shape[0] != dim:
        raise ValueError(f"{name} has {shape[0]} rows, expected {dim}")
    if n is not None and shape[1] != n:
        raise ValueError(f"{name} has {shape[1]} columns, expected {n}")
    # Row-contiguous SoA: unit stride along a row; rows at the leading dimension stride[0], which
    # must be the row length unless a larger leading dimension is allowed (no element: any).
    if shape[0] and shape[1] and ((shape[1] > 1 and stride[1] != 1) or stride[0] < shape[1] or
                                  (not allow_ld and shape[0] > 1 and stride[0] != shape[1])):
        raise ValueError(f"{name} must be row-contiguous SoA")
    return t.data_ptr(), stride[0]


# ---- context -------------------------------------------------------------------------------------
def rbf_ctx_create(device: int = 0, hbm_budget_bytes: int = 0) -> int:
    h = _vp()
    _check(lib().rbf_ctx_create(device, hbm_budget_bytes, ctypes.byref(h)), "rbf_ctx_create")
    _live_ctx.add(h.value)
    return h.value


def rbf_ctx_destroy(ctx: int) -> None:
    _check(lib().rbf_ctx_destroy(ctx), "rbf_ctx_destroy")
    _live_ctx.discard(ctx)


def rbf_ctx_bytes_in_use(ctx: int) -> int:
    return lib().rbf_ctx_bytes_in_use(ctx)


def rbf_now() -> float:
    return lib().rbf_now()


def rbf_ctx_set_timing(ctx: int, enabled: bool, count_pairs: bool = False) -> None:
    """Event timing of the kernel-sum launches; count_pairs adds the evaluated-pair counter (one
    atomic per workgroup: keep it off while timing)."""
    flags = (1 if enabled else 0) | (2 if count_pairs else 0)
    _check(lib().rbf_ctx_set_timing(ctx, flags), "rbf_ctx_set_timing")


def rbf_ctx_kernel_pairs(ctx: int, kernel: str) -> int:
    """(point, control) pairs a timed kernel evaluated since timing was enabled (culled pairs
    excluded)."""
    n = _i64()
    _check(lib().rbf_ctx_kernel_pairs(ctx, kernel.encode(), ctypes.byref(n)), "rbf_ctx_kernel_pairs")
    return n.value


def rbf_ctx_kernel_time(ctx: int, kernel: str):
    """(summed device milliseconds, launches) of a timed kernel since timing was enabled."""
    ms, n = _f64(), _i64()
    _check(lib().rbf_ctx_kernel_time(ctx, kernel.encode(), ctypes.byref(ms), ctypes.byref(n)),
           "rbf_ctx_kernel_time")
    return ms.value, n.value


# ---- greedy --------------------------------------------------------------------------------------
@dataclass
class CtrlSet:
    """Result of ``rbf_greedy_select``: device tensors plus the per-level host metadata."""
    dim: int
    radius: List[float]
    ctrl_idx: object          # int64 [capacity]
    xc: object                # float64 [dim, capacity]
    alpha: object             # float64 [dim, capacity]
    e_final: object           # float64 [dim, n_s] or None
    level_off: List[int]
    level_stop: List[int]
    level_max_err: List[float]
    n_levels_used: int
    n_iterations: int
    status: int
    level_in_max: List[float] = field(default_factory=list)    # max ||dS_l|| per level input
    level_seconds: List[float] = field(default_factory=list)
    level_fp32_err: List[float] = field(default_factory=list)   # FP32 error at the surface (mixed)
    err_hist: object = None   # float64 [n_iterations]: max ||E|| before each argmax selection

    def fp32_levels(self, tol: float = 1e-6) -> List[bool]:
        """Levels whose measured FP32 error is at most tol max ||dS|| (the serving path's rule)."""
        return [0.0 < e <= tol * self.level_in_max[0] if self.level_fp32_err else False
                for e in self.level_fp32_err[: self.n_levels_used]]

    @property
    def total(self) -> int:
        return self.level_off[-1]

    def support_distances(self, k: float) -> List[float]:
        """D_l = k max_i ||dS_l,i|| for the levels run (section 4, volume reduction factor k)."""
        return [k * self.level_in_max[l] for l in range(self.n_levels_used)]

    def level(self, l: int):
        a, b = self.level_off[l], self.level_off[l + 1]
        return self.ctrl_idx[a:b], self.alpha[:, a:b]


def make_params(dim: int, radius: Sequence[float], eps: float, rho: float = 0.1, cap: int = 0,
                seeds: Optional[Sequence[Sequence[int]]] = None, precision: str = "fp64",
                n_s: Optional[int] = None, basis: str = "c2"):
    """Build rbf_greedy_params; the returned tuple keeps the seed arrays alive."""
    p = rbf_greedy_params()
    p.dim = dim
    p.n_levels = len(radius)
    for l, r in enumerate(radius):
        p.radius[l] = float(r)
    p.eps_abs = float(eps)
    p.level_reduction = float(rho)
    p.max_ctrl_total = int(cap if cap > 0 else (n_s or 1) * len(radius))
    p.precision = RBF_MIXED if precision == "mixed" else RBF_FP64
    p.basis = _basis(basis)
    keep = []
    if seeds is not None:
        lv = [list(seeds[l]) if l < len(seeds) else [] for l in range(len(radius))]
        off = (_i32 * (len(radius) + 1))()
        for l, s in enumerate(lv):
            off[l + 1] = off[l] + len(s)
        flat = [q for s in lv for q in s] or [0]
        idx = (_i64 * len(flat))(*flat)
        p.seed_idx = ctypes.cast(idx, ctypes.POINTER(_i64))
        p.seed_off = ctypes.cast(off, ctypes.POINTER(_i32))
        keep = [idx, off]
    return p, keep


def rbf_greedy_select(ctx: int, xs, ds, radius: Sequence[float], eps: float, rho: float = 0.1,
                      cap: int = 0, seeds=None, precision: str = "fp64", want_residual: bool = True,
                      stream=None, basis: str = "c2") -> CtrlSet:
    import torch

    dim, n_s = xs.shape
    p, keep = make_params(dim, radius, eps, rho, cap, seeds, precision, n_s, basis)
    pxs, _ = _dev(xs, "xs", dim, n_s)
    pds, _ = _dev(ds, "ds", dim, n_s)
    capacity = int(p.max_ctrl_total)
    dev = xs.device
    ctrl = torch.full((capacity,), -1, dtype=torch.int64, device=dev)
    xc = torch.zeros((dim, capacity), dtype=torch.float64, device=dev)
    alpha = torch.zeros((dim, capacity), dtype=torch.float64, device=dev)
    ef = torch.zeros((dim, n_s), dtype=torch.float64, device=dev) if want_residual else None
    hist = torch.zeros((capacity,), dtype=torch.float64, device=dev)
    out = rbf_ctrl_set()
    out.capacity = capacity
    out.ctrl_idx = ctrl.data_ptr()
    out.xc = xc.data_ptr()
    out.alpha = alpha.data_ptr()
    out.e_final = ef.data_ptr() if ef is not None else None
    out.err_hist = hist.data_ptr()
    st = _check(lib().rbf_greedy_select(ctx, ctypes.byref(p), n_s, pxs, pds, ctypes.byref(out),
                                        _stream(stream)), "rbf_greedy_select")
    del keep
    nl = out.n_levels_used
    return CtrlSet(dim=dim, radius=[float(r) for r in radius], ctrl_idx=ctrl, xc=xc, alpha=alpha,
                   e_final=ef, level_off=[out.level_off[l] for l in range(len(radius) + 1)],
                   level_stop=[out.level_stop[l] for l in range(len(radius))],
                   level_max_err=[out.level_max_err[l] for l in range(len(radius))],
                   n_levels_used=nl, n_iterations=out.n_iterations, status=st,
                   level_in_max=[out.level_in_max[l] for l in range(len(radius))],
                   level_seconds=[out.level_seconds[l] for l in range(len(radius))],
                   level_fp32_err=[out.level_fp32_err[l] for l in range(len(radius))],
                   err_hist=hist[: out.n_iterations])


def rbf_solve_weights(ctx: int, radius: float, xc, dsc, alpha=None, stream=None, basis: str = "c2"):
    import torch

    dim, n_c = xc.shape
    pxc, _ = _dev(xc, "xc", dim, n_c)
    pds, _ = _dev(dsc, "dsc", dim, n_c)
    if alpha is None:
        alpha = torch.empty((dim, n_c), dtype=torch.float64, device=xc.device)
    pa, _ = _dev(alpha, "alpha", dim, n_c)
    _check(lib().rbf_solve_weights(ctx, dim, float(radius), n_c, pxc, pds, pa, _basis(basis), _stream(stream)),
           "rbf_solve_weights")
    return alpha


def rbf_volume_update(ctx: int, radius: Sequence[float], D: Sequence[float], level_off: Sequence[int],
                      xc, alpha, xv, dwall, dv=None, precision="fp64", stream=None,
                      basis: str = "c2"):
    """Enqueue the psi-weighted volume update; returns dv (written asynchronously on the stream).
    precision: "fp64", "mixed", or a list with one of them per level."""
    import torch

    dim, n_v = xv.shape
    nl = len(radius)
    if len(level_off) != nl + 1:
        raise ValueError("level_off must have n_levels + 1 entries")
    D = list(D) if len(D) == nl else [float(D[0])] * nl
    pxc, ldc = _dev(xc, "xc", dim, None, allow_ld=True)
    pa, lda = _dev(alpha, "alpha", dim, None, allow_ld=True)
    if ldc != lda:
        raise ValueError("xc and alpha must share a leading dimension")
    if int(level_off[-1]) > xc.shape[1]:
        raise ValueError("level_off exceeds the control arrays")
    pxv, _ = _dev(xv, "xv", dim, n_v)
    pd, _ = _dev(dwall, "dwall", None, n_v)
    if dv is None:
        dv = torch.empty((dim, n_v), dtype=torch.float64, device=xv.device)
    pdv, _ = _dev(dv, "dv", dim, n_v)
    r = (_f64 * nl)(*[float(x) for x in radius])
    d = (_f64 * nl)(*[float(x) for x in D])
    off = (_i32 * (nl + 1))(*[int(x) for x in level_off])
    prec, levels = _precision(precision, nl)
    _check(lib().rbf_volume_update(ctx, dim, nl, r, d, off, ldc, pxc, pa, n_v, pxv, pd, pdv,
                                   prec, levels, _basis(basis), _stream(stream)),
           "rbf_volume_update")
    return dv


def rbf_volume_update_noalloc(ctx: int, radius: Sequence[float], D: Sequence[float],
                              level_off: Sequence[int], xc, alpha, xv, dwall, dv, precision="fp64",
                              stream=None, basis: str = "c2"):
    """rbf_volume_update through the allocation-free entry point: the caller passes dv, and the
    library's fixed device scratch replaces its pool (calls overlapping on one GPU race)."""
    dim, n_v = xv.shape
    nl = len(radius)
    if len(level_off) != nl + 1:
        raise ValueError("level_off must have n_levels + 1 entries")
    D = list(D) if len(D) == nl else [float(D[0])] * nl
    pxc, ldc = _dev(xc, "xc", dim, None, allow_ld=True)
    pa, lda = _dev(alpha, "alpha", dim, None, allow_ld=True)
    if ldc != lda:
        raise ValueError("xc and alpha must share a leading dimension")
    if int(level_off[-1]) > xc.shape[1]:
        raise ValueError("level_off exceeds the control arrays")
    pxv, _ = _dev(xv, "xv", dim, n_v)
    pd, _ = _dev(dwall, "dwall", None, n_v)
    pdv, _ = _dev(dv, "dv", dim, n_v)
    r, d, off = _level_arrays(radius, D, level_off)
    prec, levels = _precision(precision, nl)
    _check(lib().rbf_volume_update_noalloc(ctx, dim, nl, r, d, off, ldc, pxc, pa, n_v, pxv, pd, pdv,
                                           prec, levels, _basis(basis), _stream(stream)),
           "rbf_volume_update_noalloc")
    return dv


def rbf_evaluate(ctx: int, radius: float, xc, alpha, xp, base=None, sign: float = -1.0, out=None,
                 precision: str = "fp64", stream=None, basis: str = "c2"):
    """out = base - sign * sum_c phi(||x_p - xc|| / R) alpha_c (plain interpolant by default)."""
    import torch

    dim, n_p = xp.shape
    pxc, ldc = _dev(xc, "xc", dim, None, allow_ld=True)
    pa, lda = _dev(alpha, "alpha", dim, None, allow_ld=True)
    if ldc != lda:
        raise ValueError("xc and alpha must share a leading dimension")
    n_c = xc.shape[1]
    pxp, _ = _dev(xp, "xp", dim, n_p)
    pb, _ = _dev(base, "base", dim, n_p)
    if out is None:
        out = torch.empty((dim, n_p), dtype=torch.float64, device=xp.device)
    po, _ = _dev(out, "out", dim, n_p)
    _check(lib().rbf_evaluate(ctx, dim, float(radius), n_c, ldc, pxc, pa, n_p, pxp, pb, float(sign), po,
                              RBF_MIXED if precision == "mixed" else RBF_FP64, _basis(basis), _stream(stream)),
           "rbf_evaluate")
    return out


# ---- serving -------------------------------------------------------------------------------------
def rbf_geom_create(ctx: int, xs, xv, dwall=None) -> int:
    dim, n_s = xs.shape
    n_v = xv.shape[1]
    pxs, _ = _dev(xs, "xs", dim, n_s)
    pxv, _ = _dev(xv, "xv", dim, n_v)
    pd, _ = _dev(dwall, "dwall", None, n_v)
    h = _vp()
    _check(lib().rbf_geom_create(ctx, dim, n_s, pxs, n_v, pxv, pd, ctypes.byref(h)), "rbf_geom_create")
    return h.value


def rbf_geom_volume_update(ctx: int, geom: int, radius: Sequence[float], D: Sequence[float],
                           level_off: Sequence[int], xc, alpha, dv, precision="fp64", stream=None,
                           basis: str = "c2"):
    """Enqueue the volume update on a resident geometry; dv is [dim, n_v] in the geometry's
    original point order. precision: "fp64", "mixed", or a list with one of them per level."""
    nl = len(radius)
    if len(level_off) != nl + 1:
        raise ValueError("level_off must have n_levels + 1 entries")
    D = list(D) if len(D) == nl else [float(D[0])] * nl
    dim = dv.shape[0]
    pxc, ldc = _dev(xc, "xc", dim, None, allow_ld=True)
    pa, lda = _dev(alpha, "alpha", dim, None, allow_ld=True)
    if ldc != lda:
        raise ValueError("xc and alpha must share a leading dimension")
    if int(level_off[-1]) > xc.shape[1]:
        raise ValueError("level_off exceeds the control arrays")
    pdv, _ = _dev(dv, "dv", dim, None)
    r, d, off = _level_arrays(radius, D, level_off)
    prec, levels = _precision(precision, nl)
    _check(lib().rbf_geom_volume_update(ctx, geom, nl, r, d, off, ldc, pxc, pa, pdv, prec, levels,
                                        _basis(basis), _stream(stream)),
           "rbf_geom_volume_update")
    return dv


def rbf_geom_release(ctx: int, geom: int) -> int:
    return _check(lib().rbf_geom_release(ctx, geom), "rbf_geom_release")


@dataclass
class Request:
    """A submitted request and the host objects that must stay alive until it is DONE."""
    ticket: int
    dv: object
    out: Optional[CtrlSet]
    oc: Optional[rbf_ctrl_set] = None
    keep: list = field(default_factory=list)


def rbf_submit(ctx: int, geom: int, ds, dv, radius: Sequence[float], eps: float, D: Sequence[float],
               rho: float = 0.1, cap: int = 0, seeds=None, precision: str = "mixed",
               warm_start: bool = False, want_ctrl: bool = False, d_factor: float = 0.0,
               basis: str = "c2") -> Request:
    import torch

    dim, n_s = ds.shape
    p, keep = make_params(dim, radius, eps, rho, cap, seeds, precision, n_s, basis)
    req = rbf_request()
    req.geom = geom
    req.ds, _ = _dev(ds, "ds", dim, n_s)
    req.params = p
    nl = len(radius)
    D = list(D) if len(D) == nl else [float(D[0])] * nl
    for l in range(nl):
        req.D[l] = float(D[l])
    req.d_factor = float(d_factor)
    req.warm_start = 1 if warm_start else 0
    req.dv, _ = _dev(dv, "dv", dim, None)
    cs = None
    oc = None
    if want_ctrl:
        capacity = int(p.max_ctrl_total)
        dev = ds.device
        ctrl = torch.full((capacity,), -1, dtype=torch.int64, device=dev)
        xc = torch.zeros((dim, capacity), dtype=torch.float64, device=dev)
        alpha = torch.zeros((dim, capacity), dtype=torch.float64, device=dev)
        oc = rbf_ctrl_set()
        oc.capacity = capacity
        oc.ctrl_idx, oc.xc, oc.alpha, oc.e_final = ctrl.data_ptr(), xc.data_ptr(), alpha.data_ptr(), None
        req.out = ctypes.pointer(oc)
        keep += [oc, ctrl, xc, alpha]
        cs = CtrlSet(dim, [float(r) for r in radius], ctrl, xc, alpha, None, [], [], [], 0, 0, 0)
    t = _u64()
    _check(lib().rbf_submit(ctx, ctypes.byref(req), ctypes.byref(t)), "rbf_submit")
    keep += [req, ds, dv]
    return Request(ticket=t.value, dv=dv, out=cs, oc=oc, keep=keep)


def _fill_ctrl(r: Request):
    if r.out is None or r.oc is None:
        return
    oc = r.oc
    nl = len(r.out.radius)
    r.out.level_off = [oc.level_off[l] for l in range(nl + 1)]
    r.out.level_stop = [oc.level_stop[l] for l in range(nl)]
    r.out.level_max_err = [oc.level_max_err[l] for l in range(nl)]
    r.out.n_levels_used = oc.n_levels_used
    r.out.n_iterations = oc.n_iterations
    r.out.level_in_max = [oc.level_in_max[l] for l in range(nl)]
    r.out.level_seconds = [oc.level_seconds[l] for l in range(nl)]
    r.out.level_fp32_err = [oc.level_fp32_err[l] for l in range(nl)]


def rbf_poll(ctx: int, r: Request) -> rbf_req_info:
    info = rbf_req_info()
    _check(lib().rbf_poll(ctx, r.ticket, ctypes.byref(info)), "rbf_poll")
    return info


def rbf_wait(ctx: int, r: Request) -> rbf_req_info:
    info = rbf_req_info()
    _check(lib().rbf_wait(ctx, r.ticket, ctypes.byref(info)), "rbf_wait")
    _fill_ctrl(r)
    return info


class Context:
    """Owns an rbf_ctx for ``with`` blocks."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.handle = rbf_ctx_create(device, hbm_budget_bytes)

    def close(self):
        if self.handle:
            rbf_ctx_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self.handle

    def __exit__(self, *exc):
        self.close()

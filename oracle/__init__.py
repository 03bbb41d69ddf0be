"""FP64 CPU oracle of multi-level greedy RBF mesh deformation (arXiv:2107.13887).

TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the CPU-baseline leg of the benchmark
are the only code allowed to import this package. It shares no code with the GPU library: the C
source ``rbf_oracle.c`` is compiled here with gcc into ``liborc.so`` and called through ctypes.

Functions follow the paper's statement of the method (see the header of ``rbf_oracle.c``):
``wendland_c2`` (eq. (2)), ``wendland`` (Table 1: C0, C2, C4, C6), ``psi`` (Section 4), ``evaluate`` (eq. (1)), ``solve_weights``
(eq. (9) on a control set), ``greedy`` (Section 3: eq. (12), argmax, multi-level residual) and
``volume`` (eqs. (19) and (23)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rbf_oracle.c")
LIB_PATH = os.path.join(_HERE, "liborc.so")

STOP_NAMES = {0: "eps", 1: "cap", 2: "all_selected", 3: "breakdown", -1: "skipped"}
# Codes of the Wendland functions of Table 1 in rbf_oracle.c.
BASIS = {"c2": 0, "c0": 1, "c4": 2, "c6": 3}

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


def build(out_path: str = LIB_PATH, defines: Optional[List[str]] = None) -> str:
    """Compile ``rbf_oracle.c`` with gcc (-O2, OpenMP, no FP contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter"]
    for d in defines or []:
        cmd.append("-D" + d)
    tmp = out_path + ".tmp"
    cmd += [_SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out_path)
    return out_path


class Oracle:
    """ctypes view of one compiled oracle library (the real one, or a planted-mistake variant
    built by the tests)."""

    def __init__(self, path: str = LIB_PATH):
        if not os.path.exists(path):
            if path != LIB_PATH:
                raise FileNotFoundError(path)
            build()
        self.lib = ctypes.CDLL(path)
        L = self.lib
        L.orc_wendland_c2.restype = ctypes.c_double
        L.orc_wendland_c2.argtypes = [ctypes.c_double]
        L.orc_wendland.restype = ctypes.c_double
        L.orc_wendland.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc_psi.restype = ctypes.c_double
        L.orc_psi.argtypes = [ctypes.c_double]
        L.orc_eval.restype = None
        L.orc_eval.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int64, _dp, _dp,
                               ctypes.c_int64, _dp, _dp, ctypes.c_int]
        L.orc_solve_weights.restype = ctypes.c_int
        L.orc_solve_weights.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int64, _dp, _dp, _dp,
                                        ctypes.c_int]
        L.orc_greedy.restype = ctypes.c_int
        L.orc_greedy.argtypes = [ctypes.c_int, ctypes.c_int64, _dp, _dp, ctypes.c_int, _dp,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int64, _i64p, _i32p,
                                 _i64p, _dp, _i32p, _dp, _i32p, _i32p, _dp, _dp, ctypes.c_int]
        L.orc_volume.restype = None
        L.orc_volume.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _i32p, ctypes.c_int64,
                                 _dp, _dp, ctypes.c_int64, _dp, _dp, _dp, ctypes.c_int]

    # -- scalar functions ----------------------------------------------------------------------
    def wendland_c2(self, eta: float) -> float:
        return self.lib.orc_wendland_c2(float(eta))

    def wendland(self, basis: str, eta: float) -> float:
        """Table 1: the Wendland function named by ``basis`` ("c0", "c2", "c4", "c6")."""
        return self.lib.orc_wendland(BASIS[basis], float(eta))

    def psi(self, xi: float) -> float:
        return self.lib.orc_psi(float(xi))

    # -- array functions -----------------------------------------------------------------------
    def evaluate(self, radius: float, xc: np.ndarray, alpha: np.ndarray, xp: np.ndarray,
                 basis: str = "c2") -> np.ndarray:
        """Interpolant sum_c alpha_c phi(||p - x_c|| / R) at the points ``xp`` [dim, n_p]."""
        xc, alpha, xp = _f64(xc), _f64(alpha), _f64(xp)
        dim, n_c = xc.shape
        out = np.zeros((dim, xp.shape[1]))
        self.lib.orc_eval(dim, float(radius), n_c, _ptr(xc), _ptr(alpha), xp.shape[1], _ptr(xp),
                          _ptr(out), BASIS[basis])
        return out

    def solve_weights(self, radius: float, xc: np.ndarray, dsc: np.ndarray, basis: str = "c2"):
        """Weights of the interpolant through (xc, dsc): Phi_cc alpha = dsc. Returns (status,
        alpha); status -3 means Phi_cc is not numerically positive definite."""
        xc, dsc = _f64(xc), _f64(dsc)
        dim, n_c = xc.shape
        alpha = np.zeros((dim, n_c))
        st = self.lib.orc_solve_weights(dim, float(radius), n_c, _ptr(xc), _ptr(dsc), _ptr(alpha),
                                        BASIS[basis])
        return st, alpha

    def greedy(self, dim: int, xs: np.ndarray, ds: np.ndarray, radius, eps: float,
               rho: float = 0.1, cap: int = 0, seeds=None, basis: str = "c2") -> "GreedyResult":
        """Multi-level greedy selection (Section 3) with the readings listed in the C header."""
        xs, ds = _f64(xs), _f64(ds)
        n_s = xs.shape[1]
        radius = np.ascontiguousarray(radius, dtype=np.float64)
        n_levels = radius.size
        if cap <= 0:
            cap = n_s * n_levels
        seeds = seeds if seeds is not None else [[0]]
        lv = [list(seeds[l]) if l < len(seeds) else [] for l in range(n_levels)]
        seed_off = np.zeros(n_levels + 1, dtype=np.int32)
        for l, s in enumerate(lv):
            seed_off[l + 1] = seed_off[l] + len(s)
        seed_idx = np.array([p for s in lv for p in s] or [0], dtype=np.int64)
        ctrl = np.full(cap, -1, dtype=np.int64)
        alpha = np.zeros((dim, cap))
        level_off = np.zeros(n_levels + 1, dtype=np.int32)
        level_err = np.zeros(n_levels)
        level_stop = np.zeros(n_levels, dtype=np.int32)
        used = np.zeros(1, dtype=np.int32)
        e_final = np.zeros((dim, n_s))
        hist = np.zeros(cap)
        st = self.lib.orc_greedy(dim, n_s, _ptr(xs), _ptr(ds), n_levels, _ptr(radius), float(eps),
                                 float(rho), cap, seed_idx.ctypes.data_as(_i64p),
                                 seed_off.ctypes.data_as(_i32p), ctrl.ctypes.data_as(_i64p),
                                 _ptr(alpha), level_off.ctypes.data_as(_i32p), _ptr(level_err),
                                 level_stop.ctypes.data_as(_i32p), used.ctypes.data_as(_i32p),
                                 _ptr(e_final), _ptr(hist), BASIS[basis])
        if st != 0:
            raise RuntimeError(f"orc_greedy failed with status {st}")
        total = int(level_off[-1])
        return GreedyResult(dim=dim, radius=radius.copy(), ctrl_idx=ctrl[:total].copy(),
                            alpha=np.ascontiguousarray(alpha[:, :total]), level_off=level_off,
                            level_max_err=level_err, level_stop=level_stop,
                            n_levels_used=int(used[0]), e_final=e_final,
                            history=hist[: total - int(seed_off[-1])].copy())

    def volume(self, radius, D, level_off, xc: np.ndarray, alpha: np.ndarray, xv: np.ndarray,
               dwall: np.ndarray, basis: str = "c2") -> np.ndarray:
        """dV_v = sum_l psi(d_v / D_l) sum_{c in level l} phi(||x_v - x_c|| / R_l) alpha_c."""
        xc, alpha, xv, dwall = _f64(xc), _f64(alpha), _f64(xv), _f64(dwall)
        radius = np.ascontiguousarray(radius, dtype=np.float64)
        D = np.ascontiguousarray(np.broadcast_to(np.asarray(D, dtype=np.float64), radius.shape))
        level_off = np.ascontiguousarray(level_off, dtype=np.int32)
        dim, n_c = xc.shape
        n_v = xv.shape[1]
        dv = np.zeros((dim, n_v))
        self.lib.orc_volume(dim, radius.size, _ptr(radius), _ptr(D),
                            level_off.ctypes.data_as(_i32p), n_c, _ptr(xc), _ptr(alpha), n_v,
                            _ptr(xv), _ptr(dwall), _ptr(dv), BASIS[basis])
        return dv


@dataclass
class GreedyResult:
    dim: int
    radius: np.ndarray
    ctrl_idx: np.ndarray        # selection order, concatenated over levels
    alpha: np.ndarray           # [dim, total]
    level_off: np.ndarray       # [n_levels + 1]
    level_max_err: np.ndarray   # max_i ||E_i|| at each level close
    level_stop: np.ndarray      # stop reason per level (see STOP_NAMES)
    n_levels_used: int
    e_final: np.ndarray         # residual after the last level
    history: np.ndarray         # max candidate ||E|| before each argmax selection

    def level(self, l: int):
        a, b = int(self.level_off[l]), int(self.level_off[l + 1])
        return self.ctrl_idx[a:b], self.alpha[:, a:b]


def support_distances(k: float, ds: np.ndarray, res: "GreedyResult"):
    """Section 4, volume point reduction: D_l = k (dS_l)^max for every level run, with
    (dS_l)^max = max_i ||dS_l,i||; dS_0 is the prescribed surface displacement and dS_l for
    l >= 1 is the error left by level l - 1, whose maximum the greedy reports at its close."""
    ds = _f64(ds)
    top = [float(np.sqrt((ds ** 2).sum(axis=0)).max())]
    top += [float(res.level_max_err[l]) for l in range(res.n_levels_used - 1)]
    return [k * m for m in top]


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


_default: Optional[Oracle] = None


def get() -> Oracle:
    """The oracle built from the unmodified source (built on first use if missing)."""
    global _default
    if _default is None:
        _default = Oracle()
    return _default

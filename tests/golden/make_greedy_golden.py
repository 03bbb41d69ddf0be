"""Writes the stored full-size greedy selections of the 3D workloads from the FP64 CPU oracle.

    python tests/golden/make_greedy_golden.py [cfg2 cfg3 sine3d]

For each workload the oracle's whole multi-level greedy (Section 3: eq. (12), argmax, the level
residual handed on as in eq. (19)) runs on the seeded synthetic surface and displacement, and
``greedy_<workload>.npz`` receives its control sets in selection order (``ctrl_idx``),
``level_off``, ``level_stop``, ``level_max_err``, the weights ``alpha`` [dim, total], the error
history before each argmax selection, the final residual at 4000 seeded surface points
(``e_idx``, ``e_sample``) with its maximum norm, and a hash of the inputs it was computed from
(``input_sha``: surface points, displacement and greedy parameters). Only ``oracle`` and
``synth`` are used; nothing here touches the GPU library. The oracle runs with OpenMP over
surface points, and its results do not depend on the thread count (each point's sum is serial,
the argmax combine is serial).
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOADS = ("cfg2", "cfg3", "sine3d")


def build(name):
    import synth

    return {"cfg2": synth.workload_cfg2, "cfg3": synth.workload_cfg3,
            "sine3d": synth.workload_sine3d}[name]()


def input_sha(w) -> str:
    """Hash of what the greedy reads: surface points, displacement and its parameters."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(w.xs, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(w.ds, dtype=np.float64).tobytes())
    h.update(repr((list(map(float, w.radius)), float(w.eps), float(w.rho), int(w.cap_total()),
                   [list(map(int, s)) for s in w.seeds])).encode())
    return h.hexdigest()[:32]


def path_for(name: str) -> str:
    return os.path.join(HERE, f"greedy_{name}.npz")


def make(name: str) -> str:
    import oracle

    w = build(name)
    t0 = time.perf_counter()
    ref = oracle.get().greedy(w.dim, w.xs, w.ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(),
                              seeds=w.seeds)
    secs = time.perf_counter() - t0
    e_idx = np.sort(np.random.default_rng(4242).choice(w.n_s, min(4000, w.n_s), replace=False))
    out = path_for(name)
    np.savez_compressed(
        out, input_sha=np.array(input_sha(w)), ctrl_idx=ref.ctrl_idx.astype(np.int64),
        level_off=np.asarray(ref.level_off, dtype=np.int32),
        level_stop=np.asarray(ref.level_stop, dtype=np.int32),
        level_max_err=np.asarray(ref.level_max_err, dtype=np.float64),
        n_levels_used=np.array(ref.n_levels_used), alpha=ref.alpha, history=ref.history,
        e_idx=e_idx.astype(np.int64), e_sample=np.ascontiguousarray(ref.e_final[:, e_idx]),
        e_final_max=np.array(float(np.sqrt((ref.e_final ** 2).sum(0)).max())),
        oracle_seconds=np.array(secs))
    print(f"{name}: {ref.ctrl_idx.size} control points, levels {list(ref.level_off)}, "
          f"oracle {secs:.1f} s -> {out}", flush=True)
    return out


if __name__ == "__main__":
    for n in sys.argv[1:] or WORKLOADS:
        make(n)

#!/usr/bin/env python3
"""Benchmark of the multi-level greedy RBF mesh deformation hot path on one MI355X.

One step = the whole path on one synthetic deformation: multi-level greedy selection of the
control points on the surface (rbf_greedy_select) followed by the wall-distance-reduced volume
update on the resident geometry (rbf_geom_volume_update). Inputs are resident in HBM before the
timed region starts. Default workload: the 3D iced swept wing (80,000 surface points, 4,000,000
volume points, three levels, FP64), the largest configuration that fits one GPU.

Headline value: in-support RBF evaluations per second of the volume update, i.e. the
(reduced volume point, control point) pairs of the same level with psi(d / D_l) > 0 and
phi(||x_v - x_c|| / R_l) > 0, counted exactly on the host (KD-tree pair count), divided by the
device time of the volume-update calls (hipEvents on the launch stream). Beside it: the dense
count sum_l n_{D_l} N_{c,l} and the pairs the kernel actually evaluates after its per-workgroup
compact-support cull (device counter). The roofline fraction of the volume kernel launch (VALU
issue bound) is taken on the in-support pairs. Also reported: greedy time-to-eps and its
Newton-basis stream against HBM peak, the plain call on the unsorted volume, the FP32 pair form
and the guarded mixed form against FP64 and the oracle, further workloads (the 2D multi-level
airfoil; the bent and twisted wing in mixed precision with its mesh validity), a reduced serving
mix, and the FP64 CPU oracle timed on this machine's host cores on the same workload.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload cfg2] [--precision fp64]
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("RBF evals/s (volume update: in-support reduced-volume point x control point pairs, "
          "psi > 0 and phi > 0, per second), greedy time-to-eps, p50/p99 request latency")
VALU_LANE_OPS = 256 * 64 * 2.4e9          # 256 CUs x 64 lanes x 2.4 GHz
HBM_PEAK_GBS = 8000.0                     # MI355X HBM3E
# Minimal VALU issue slots per (point, control) pair with the Wendland C2 basis: dim subtractions,
# the squared distance (dim multiply-adds), the square root (a quarter-rate op: 4 slots), 1 - eta,
# the clamp at 0, t^2 and t^4, 4 eta + 1, the product, and dim accumulating multiply-adds; points
# and controls are pre-scaled by 1/R. Other bases change the polynomial part; the FP32 pair form
# adds one conversion to FP64 before the accumulation.
MIN_SLOTS = {2: 17, 3: 20}
BASIS_SLOTS = {"c0": -3, "c2": 0, "c4": 2, "c6": 3}


def min_slots(dim, basis, precision):
    return MIN_SLOTS[dim] + BASIS_SLOTS[basis] + (1 if precision == "mixed" else 0)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_workload(name):
    import synth

    if name == "cfg1":
        return synth.workload_cfg1(), ("2D NACA0012 multi-level: N_s=4000 surface, N_v=400000 O-mesh, "
                                       "R_l=2c/0.5c/0.1c, eps=1e-5c, D=0.5c")
    if name == "cfg0":
        return synth.workload_cfg0(), "2D NACA0012 single level: N_s=400, N_v=20000, R=2c, eps=1e-5c, D=1c"
    if name == "cfg2":
        return synth.workload_cfg2(), ("3D swept wing ice horn: N_s=80000, N_v=4001800 (C-H shell), "
                                       "R_l=3c/0.8c/0.2c, eps=1e-4c, cap 4000, D=1c")
    if name == "cfg4":
        return None, ("serving mix: 64 geometries (60% 2D airfoils, N_s 500-8000; 40% 3D wings, "
                      "N_s 10k-80k), 4 warm-started icing steps each, Poisson arrivals at 20/s, "
                      "eps in {1e-4, 1e-5}, mixed precision")
    if name == "cfg3":
        return synth.workload_cfg3(), ("3D swept wing bend+twist: N_s=80000, N_v=4001800 (C-H shell), "
                                       "R_l=3c/0.8c/0.2c, eps=1e-4c, cap 4000, D=1c")
    if name == "sine2d":
        return synth.workload_sine2d(), ("2D NACA0012 global deformation dy = 0.01 sin(15 pi x): N_s=4000, "
                                         "N_v=400000, R=2c on 5 levels, eps=1e-5 max|dS|, D_l = 5 max|dS_l|")
    if name == "sine3d":
        return synth.workload_sine3d(), ("3D swept wing global deformation 0.03 sin(4 pi y): N_s=80000, "
                                         "N_v=4001800 (C-H shell), R=3c on 4 levels, eps=1e-4c, cap 4000, "
                                         "D_l = 5 max|dS_l|")
    raise SystemExit(f"unknown workload {name}")


# What decides the volume kernel sum's memory traffic: its kernels and launch wrappers, their
# argument block, the basis functions they inline, and the resident geometry's stored layout
# (serve.cpp: the order of the rows decides how the writes through the permutation coalesce).
# The host planner (ksum_host.cpp) is left out.
KERNEL_SOURCES = ("ksum.hip", "ksum.h", "basis.h", "serve.cpp")


def kernel_source_hash():
    """Hash of the kernel-sum device sources with comments and white space removed, so that a
    counter summary stays matched to its kernel through edits of the comments only."""
    import hashlib
    import re

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2107_13887_amd", "csrc", name)) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update("".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision):
    """HBM bytes per launch of the volume kernel-sum, from the committed counter summary (the L2's
    read and write requests to memory, counted by size: 32, 64 and 128 bytes), or None when that
    summary was taken on a different kernel source or layout."""
    path = os.path.join(ROOT, "profiles", f"traffic_volume_ksum_{workload}_{precision}.txt")
    if not os.path.exists(path):
        return None
    fields = dict(line.split(":", 1) for line in open(path) if ":" in line)
    fields = {k.strip(): v.strip() for k, v in fields.items()}
    if fields.get("ksum_source_sha256_16") != kernel_source_hash():
        return None
    return float(fields["hbm_bytes_per_launch"])


def _omp():
    """The OpenMP runtime the oracle library uses (to read and set its thread count)."""
    import ctypes

    try:
        return ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None


def serving_replay(ctx, geoms, reqs, time_scale=1.0, compare=True):
    """Replay a request mix through the serving loop: every geometry made resident first, each
    request's surface displacement uploaded before the clock starts, then submissions at their
    Poisson arrival times (later icing steps of a geometry warm-started from the previous one).
    Latency = completion - arrival, both taken by the library's clock. With compare=True the same
    requests also run one after another on the plain calls (greedy from scratch in FP64, then the
    volume update with its per-call reduction), as a caller without the serving loop would."""
    import numpy as np
    import torch

    from paper_2107_13887_amd import rbfdef

    dev = torch.device("cuda:0")
    steps = max(r.step for r in reqs)
    handles, dvs, dss = [], [], []
    for g in geoms:
        handles.append(rbfdef.rbf_geom_create(ctx, torch.from_numpy(g.xs).to(dev),
                                              torch.from_numpy(g.xv).to(dev),
                                              torch.from_numpy(g.dwall).to(dev)))
        dvs.append(torch.zeros((g.dim, g.xv.shape[1]), dtype=torch.float64, device=dev))
    for r in reqs:
        g = geoms[r.geom]
        dss.append(torch.from_numpy(np.ascontiguousarray(g.shape * (r.step / steps))).to(dev))
    torch.cuda.synchronize()
    log(f"bench: serving replay: {len(geoms)} geometries resident, {len(reqs)} requests to submit")
    pend = []
    t0 = rbfdef.rbf_now()
    for r, ds in zip(reqs, dss):
        g = geoms[r.geom]
        wait = t0 + r.arrival * time_scale - rbfdef.rbf_now()
        if wait > 0:
            time.sleep(wait)
        pend.append(rbfdef.rbf_submit(ctx, handles[r.geom], ds, dvs[r.geom], g.radius, r.eps,
                                      [g.D] * len(g.radius), rho=0.1, cap=g.cap, precision=r.precision,
                                      warm_start=r.step > 1))
    infos = []
    for k, q in enumerate(pend):
        infos.append(rbfdef.rbf_wait(ctx, q))
        if (k + 1) % 32 == 0:
            log(f"bench: serving replay: {k + 1}/{len(pend)} requests done")
    t_end = max(i.t_done for i in infos)
    failed = sum(1 for i in infos if i.state != rbfdef.REQ_DONE)
    lat = sorted((i.t_done - i.t_arrive) * 1e3 for i in infos)
    queue = sorted((i.t_start - i.t_arrive) * 1e3 for i in infos)
    service = [(i.t_done - i.t_start) * 1e3 for i in infos]
    pct = lambda v, q: v[min(len(v) - 1, int(q * len(v)))]
    out = {
        "requests": len(reqs), "geometries": len(geoms), "icing_steps": steps, "failed": failed,
        "arrival_rate_per_s": (len(reqs) / (reqs[-1].arrival * time_scale)
                               if reqs[-1].arrival * time_scale > 0 else None),
        "p50_latency_ms": pct(lat, 0.50), "p99_latency_ms": pct(lat, 0.99),
        "p50_queue_ms": pct(queue, 0.50), "mean_service_ms": statistics.mean(service),
        "throughput_req_per_s": len(reqs) / (t_end - t0),
        "makespan_s": t_end - t0,
        "surface_points": sum(g.xs.shape[1] for g in geoms),
        "volume_points": sum(g.xv.shape[1] for g in geoms),
    }
    for h in handles:
        rbfdef.rbf_geom_release(ctx, h)
    if compare:
        stream = torch.cuda.current_stream()
        dev_geom = [(torch.from_numpy(g.xs).to(dev), torch.from_numpy(g.xv).to(dev),
                     torch.from_numpy(g.dwall).to(dev)) for g in geoms]
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        for k, (r, ds) in enumerate(zip(reqs, dss)):
            if k % 32 == 0:
                log(f"bench: sequential plain FP64: request {k}/{len(reqs)}")
            g = geoms[r.geom]
            xs, xv, dw = dev_geom[r.geom]
            cs = rbfdef.rbf_greedy_select(ctx, xs, ds, g.radius, r.eps, rho=0.1, cap=g.cap,
                                          precision="fp64", want_residual=False)
            rbfdef.rbf_volume_update(ctx, g.radius, [g.D] * len(g.radius), cs.level_off, cs.xc, cs.alpha,
                                     xv, dw, precision="fp64")
        torch.cuda.synchronize()
        out["sequential_plain_fp64_s"] = time.perf_counter() - c0
        out["sequential_plain_fp64_req_per_s"] = len(reqs) / out["sequential_plain_fp64_s"]
    return out


def _median_ms(stream, fn, reps):
    import torch

    evs = []
    for _ in range(reps):
        a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a_.record(stream)
        fn()
        b_.record(stream)
        evs.append((a_, b_))
    torch.cuda.synchronize()
    return statistics.median(a_.elapsed_time(b_) for a_, b_ in evs)


def error_curve(cs, w, points=40):
    """The greedy's normalized error max ||E|| / max ||dS|| before each argmax selection,
    subsampled, with the iteration index and an elapsed time from each level's wall time spread
    evenly over its iterations (the error-versus-time curve of Section 3)."""
    import numpy as np

    hist = cs.err_hist.cpu().numpy() if cs.err_hist is not None else np.zeros(0)
    if hist.size == 0:
        return []
    scale = float(np.sqrt((w.ds ** 2).sum(0)).max())
    t = np.zeros(hist.size)
    start, clock = 0, 0.0
    for l in range(cs.n_levels_used):
        n_l = cs.level_off[l + 1] - cs.level_off[l] - (len(w.seeds[l]) if l < len(w.seeds) else 0)
        n_l = max(0, min(n_l, hist.size - start))
        if n_l:
            t[start:start + n_l] = clock + cs.level_seconds[l] * (np.arange(n_l) + 1) / n_l
        start += n_l
        clock += cs.level_seconds[l]
    pick = np.unique(np.linspace(0, hist.size - 1, min(points, hist.size)).round().astype(int))
    return [[int(i), float(t[i]), float(hist[i] / scale)] for i in pick]


def _normwise(got, ref):
    import numpy as np

    scale = np.sqrt((ref ** 2).sum(0)).max()
    err = np.sqrt(((got - ref) ** 2).sum(0))
    return {"max_abs": float(err.max()), "rms": float(np.sqrt((err ** 2).mean())),
            "normwise": float(err.max() / scale) if scale > 0 else None}


def in_support_pairs(w, radius, D, off, xc):
    """Exact count of the (reduced volume point, control point) pairs of one volume update that lie
    inside the compact support, level by level: d_v < D_l (psi > 0, Section 4) and
    ||x_v - x_c|| < R_l (phi > 0, eq. (2)). A KD-tree pair count on the host, independent of the
    GPU path; pairs exactly at distance R_l (phi = 0) are left out."""
    import numpy as np
    from scipy.spatial import cKDTree

    trees, total, per_level = {}, 0, []
    for l in range(len(radius)):
        lo, hi = int(off[l]), int(off[l + 1])
        if hi <= lo:
            per_level.append(0)
            continue
        key = float(D[l])
        if key not in trees:
            trees[key] = cKDTree(np.ascontiguousarray(w.xv[:, w.dwall < D[l]].T))
        n = int(cKDTree(np.ascontiguousarray(xc[:, lo:hi].T)).count_neighbors(
            trees[key], np.nextafter(float(radius[l]), 0.0)))
        per_level.append(n)
        total += n
    return total, per_level


def run_workload(ctx, name, precision, basis, steps, warmup):
    """Greedy selection plus resident volume update of one workload, timed; returns the raw
    measurements the record is built from."""
    import torch

    from paper_2107_13887_amd import rbfdef

    t0 = time.perf_counter()
    w, desc = build_workload(name)
    log(f"bench: workload {w.name} built in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    m = {"w": w, "desc": desc, "precision": precision}
    xs = torch.from_numpy(w.xs).to(dev)
    ds = torch.from_numpy(w.ds).to(dev)
    xv = torch.from_numpy(w.xv).to(dev)
    dw = torch.from_numpy(w.dwall).to(dev)
    stream = torch.cuda.current_stream()
    # Setup, outside the timed region: the geometry (surface, volume, wall distances) becomes
    # resident once, as across successive icing steps.
    geom = rbfdef.rbf_geom_create(ctx, xs, xv, dw)
    dv = torch.empty((w.dim, w.n_v), dtype=torch.float64, device=dev)

    def supports(cs):
        """Per-level (radius, D, level_off) of a step: fixed D, or D_l = k (dS_l)^max."""
        if w.d_factor > 0:
            used = cs.n_levels_used
            return w.radius[:used], cs.support_distances(w.d_factor), cs.level_off[: used + 1]
        return w.radius, [w.D] * w.n_levels, cs.level_off

    def step():
        g0 = time.perf_counter()
        cs = rbfdef.rbf_greedy_select(ctx, xs, ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(),
                                      seeds=w.seeds, precision=precision, want_residual=False,
                                      basis=basis)
        g1 = time.perf_counter()
        radius, D, off = supports(cs)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rbfdef.rbf_geom_volume_update(ctx, geom, radius, D, off, cs.xc, cs.alpha, dv,
                                      precision=precision, basis=basis)
        e1.record(stream)
        return cs, g1 - g0, (e0, e1)

    for i in range(warmup):
        cs, _, _ = step()
        torch.cuda.synchronize()
        log(f"bench: {name}: warmup {i + 1}/{warmup} done ({cs.total} control points)")
    rbfdef.rbf_ctx_set_timing(ctx, True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    greedy_t, events = [], []
    for i in range(steps):
        cs, tg, ev = step()
        greedy_t.append(tg)
        events.append(ev)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    vol_ms = [a.elapsed_time(b) for a, b in events]
    kname = "volume_ksum_" + precision
    k_ms, k_n = rbfdef.rbf_ctx_kernel_time(ctx, kname)
    rbfdef.rbf_ctx_set_timing(ctx, False)
    log(f"bench: {name}: {steps} steps in {wall:.3f}s")
    radius, D, off = supports(cs)
    vol_call = lambda prec: rbfdef.rbf_geom_volume_update(ctx, geom, radius, D, off, cs.xc, cs.alpha, dv,
                                                          precision=prec, basis=basis)
    # Pairs the kernel evaluates per launch: one more, untimed launch with the device counter on.
    rbfdef.rbf_ctx_set_timing(ctx, False, count_pairs=True)
    vol_call(precision)
    evaluated = float(rbfdef.rbf_ctx_kernel_pairs(ctx, kname))
    rbfdef.rbf_ctx_set_timing(ctx, False)
    n_c = [off[l + 1] - off[l] for l in range(len(radius))]
    n_d = [int((w.dwall < D[l]).sum()) for l in range(len(radius))]
    xcn = cs.xc[:, : cs.total].cpu().numpy()
    in_sup, in_sup_l = in_support_pairs(w, radius, D, off, xcn)
    m.update(dict(xs=xs, ds=ds, xv=xv, dw=dw, geom=geom, dv=dv, cs=cs, radius=radius, D=D, off=off,
                  greedy_t=greedy_t, vol_ms=vol_ms, wall=wall, kname=kname, k_ms=k_ms, k_n=k_n,
                  vol_call=vol_call, evaluated=evaluated, n_c=n_c, n_d=n_d,
                  dense_pairs=sum(n_d[l] * n_c[l] for l in range(len(radius))),
                  in_support=in_sup, in_support_per_level=in_sup_l, xcn=xcn,
                  alpha=cs.alpha[:, : cs.total].cpu().numpy(), stream=stream))
    return m


def volume_roofline(m, precision, basis, workload):
    """Roofline of the dominant volume launch: in-support pairs per launch over the launch's
    average device time (library hipEvents on the launch stream, timed region), against the
    VALU-issue peak in pairs/s."""
    w = m["w"]
    avg_kernel_s = (m["k_ms"] / m["k_n"]) / 1e3 if m["k_n"] else float("nan")
    peak = VALU_LANE_OPS / min_slots(w.dim, basis, precision) / 1e9
    achieved = m["in_support"] / avg_kernel_s / 1e9
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Gpair/s",
            "frac": achieved / peak,
            "frac_of_evaluated": m["evaluated"] / avg_kernel_s / 1e9 / peak,
            "traffic": measured_traffic(workload, precision) if basis == "c2" else None,
            "kernel": m["kname"], "kernel_avg_ms": avg_kernel_s * 1e3, "kernel_launches": m["k_n"],
            "work_unit": "in-support (reduced volume point, control) pairs per launch (psi > 0 and "
                         "phi > 0, counted exactly on the host); the kernel evaluates "
                         f"{m['evaluated']:.4g} pairs per launch after its compact-support cull"}


def greedy_block(m, basis):
    """Greedy time-to-eps, iteration rate and the Newton-basis stream against HBM peak."""
    w, cs = m["w"], m["cs"]
    used = cs.n_levels_used
    g_bytes = 0
    for l in range(used):
        k = m["n_c"][l] if l < len(m["n_c"]) else 0
        g_bytes += 8 * w.n_s * (k * (k - 1) // 2) + k * w.n_s * (9 + 24 * w.dim)
    g_time = statistics.median(m["greedy_t"])
    return {
        "greedy_time_to_eps_s": g_time,
        "greedy_iterations": cs.n_iterations,
        "greedy_iterations_per_s": cs.n_iterations / g_time,
        "greedy_us_per_iteration": g_time / max(1, cs.n_iterations) * 1e6,
        "greedy_roofline": {"bound": "hbm", "achieved": g_bytes / g_time / 1e9, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": g_bytes / g_time / 1e9 / HBM_PEAK_GBS,
                            "algorithmic_bytes": g_bytes,
                            "work_unit": "Newton-basis stream of every iteration (N_s x n read, one "
                                         "column written, E and x_s), whole greedy call timed"},
        "greedy_levels": [{"controls": m["n_c"][l] if l < len(m["n_c"]) else 0,
                           "seconds": cs.level_seconds[l], "max_err_in": cs.level_in_max[l],
                           "max_err_out": cs.level_max_err[l]} for l in range(used)],
    }


def golden_selection(w):
    """The stored full selection of this workload (written by tests/golden/make_greedy_golden.py
    from the oracle) when its input hash matches, else None."""
    import numpy as np

    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    try:
        import make_greedy_golden as mg
    finally:
        sys.path.pop(0)
    name = w.name.split("_")[0]
    path = mg.path_for(name)
    if not os.path.exists(path):
        return None
    z = np.load(path, allow_pickle=False)
    if str(z["input_sha"]) != mg.input_sha(w):
        return None
    return z


def oracle_leg(m, basis, big, budget_s=12.0):
    """The CPU-baseline leg: every use of the FP64 oracle in the benchmark, all of it outside the
    timed region. The oracle's volume update timed on the host cores on a bounded sample of the
    step's workload (its rate is cpu_baseline), and the references the GPU results are checked
    against: the oracle's volume at sampled reduced-volume points and, where affordable, its whole
    greedy selection (else its first 60 selections; a stored full selection from the oracle is used
    when present)."""
    import numpy as np

    import oracle

    w, cs = m["w"], m["cs"]
    radius, D, off = m["radius"], m["D"], m["off"]
    o = oracle.get()
    xc, al = m["xcn"], m["alpha"]
    inside = np.flatnonzero(w.dwall < max(D))
    per_point = np.zeros(w.n_v)
    for l in range(len(radius)):
        per_point += (w.dwall < D[l]) * (off[l + 1] - off[l])
    rng = np.random.default_rng(5)
    n_pick = int(min(inside.size, max(1000, 2e9 / max(1.0, per_point[inside].mean()))))
    pick = np.sort(rng.choice(inside, n_pick, replace=False)) if n_pick < inside.size else inside
    xv, dwp = np.ascontiguousarray(w.xv[:, pick]), np.ascontiguousarray(w.dwall[pick])
    pairs = float(per_point[pick].sum())
    omp = _omp()
    cores = int(omp.omp_get_max_threads()) if omp else int(os.environ.get("OMP_NUM_THREADS", 1))

    def timed(fn, budget):
        reps, t = 0, 0.0
        while t < budget and reps < 1000:
            t0 = time.perf_counter()
            fn()
            t += time.perf_counter() - t0
            reps += 1
        return reps, t

    vol = lambda pts=xv, d=dwp: o.volume(radius, D, off, xc, al, pts, d, basis=basis)
    reps, t = timed(vol, budget_s)
    cpu = {"value": pairs * reps / t, "unit": "evals/s", "cores": cores, "kind": "oracle",
           "sample": f"volume update of the step's {cs.total} control points over {pick.size} of the "
                     f"{inside.size} reduced-volume points ({pairs:.3g} pairs, every pair of points "
                     f"within the support distances and controls of the same level, as the oracle "
                     f"computes them), {reps} repetitions in {t:.1f} s"}
    if omp:
        sub = pick[: max(1, pick.size // max(1, cores))]
        omp.omp_set_num_threads(1)
        r1, t1 = timed(lambda: vol(np.ascontiguousarray(w.xv[:, sub]), np.ascontiguousarray(w.dwall[sub])), 2.0)
        omp.omp_set_num_threads(cores)
        cpu["single_thread_value"] = float(per_point[sub].sum()) * r1 / t1
    # References for the parity checks.
    ref_pick = np.random.default_rng(11).choice(inside, min(20000, inside.size), replace=False)
    ref = {"pick": ref_pick,
           "dv": o.volume(radius, D, off, xc, al, w.xv[:, ref_pick], w.dwall[ref_pick], basis=basis)}
    got = cs.ctrl_idx[: cs.total].cpu().numpy()
    gold = golden_selection(w) if basis == "c2" else None
    if gold is not None:
        ref["same"] = bool(np.array_equal(got, gold["ctrl_idx"]))
        ref["check"] = (f"whole control set ({gold['ctrl_idx'].size} points) against the oracle's "
                        f"stored full greedy selection (tests/golden, input hash {str(gold['input_sha'])})")
        cpu["greedy_time_to_eps_s"] = float(gold["oracle_seconds"])
        cpu["greedy_time_note"] = "oracle's whole greedy, timed where the stored selection was written"
    elif big:
        k = 60
        r = o.greedy(w.dim, w.xs, w.ds, w.radius, w.eps, rho=w.rho, cap=k, seeds=w.seeds, basis=basis)
        ref["same"] = bool(np.array_equal(got[:k], r.ctrl_idx[:k]))
        ref["check"] = f"first {k} selections against the oracle's greedy capped at {k}"
    else:
        t0 = time.perf_counter()
        r = o.greedy(w.dim, w.xs, w.ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(), seeds=w.seeds,
                     basis=basis)
        cpu["greedy_time_to_eps_s"] = time.perf_counter() - t0
        ref["same"] = bool(np.array_equal(got, r.ctrl_idx))
        ref["check"] = "whole control set against the oracle's greedy"
    return cpu, ref


def precision_study(ctx, m, basis, ref):
    """The FP32 pair form (shifted local origin, FP64 accumulation) beside the FP64 path on the
    step's control sets: every level in FP32, and the guarded form a mixed-precision request runs
    (FP32 only on the levels whose measured FP32 error at the surface is at most 1e-6 max |dS|),
    against the FP64 GPU result and the FP64 oracle at sampled points."""
    import torch

    from paper_2107_13887_amd import rbfdef

    w, cs, stream, vol_call, dv = m["w"], m["cs"], m["stream"], m["vol_call"], m["dv"]
    ms64 = _median_ms(stream, lambda: vol_call("fp64"), 10)
    vol_call("fp64")
    torch.cuda.synchronize()
    dv64 = dv.cpu().numpy()
    msmx = _median_ms(stream, lambda: vol_call("mixed"), 10)
    vol_call("mixed")
    torch.cuda.synchronize()
    dvmx = dv.cpu().numpy()
    csm = cs if m["precision"] == "mixed" else rbfdef.rbf_greedy_select(
        ctx, m["xs"], m["ds"], w.radius, w.eps, rho=w.rho, cap=w.cap_total(), seeds=w.seeds,
        precision="mixed", want_residual=False, basis=basis)
    guard = ["mixed" if f else "fp64" for f in csm.fp32_levels()][: len(m["radius"])]
    msg = _median_ms(stream, lambda: vol_call(guard), 10)
    vol_call(guard)
    torch.cuda.synchronize()
    dvg = dv.cpu().numpy()
    study = {"fp64_volume_update_ms": ms64, "mixed_volume_update_ms": msmx,
             "mixed_speedup": ms64 / msmx,
             "mixed_vs_fp64_gpu": _normwise(dvmx, dv64),
             "level_fp32_err_at_surface": csm.level_fp32_err[: csm.n_levels_used],
             "guarded_levels": guard,
             "guarded_volume_update_ms": msg,
             "guarded_speedup": ms64 / msg,
             "guarded_vs_fp64_gpu": _normwise(dvg, dv64)}
    if ref is not None:
        pick = ref["pick"]
        study.update({"fp64_vs_oracle_sampled": _normwise(dv64[:, pick], ref["dv"]),
                      "mixed_vs_oracle_sampled": _normwise(dvmx[:, pick], ref["dv"]),
                      "guarded_vs_oracle_sampled": _normwise(dvg[:, pick], ref["dv"]),
                      "oracle_sample_points": int(pick.size)})
    return study, dv64, dvg


def mesh_validity(w, dvs):
    """Smallest corner Jacobian of the deformed C-H shell's hexahedra, each oriented by the sign of
    the undeformed cell (positive: no cell inverted), for each named volume displacement (the
    surface moved by its prescribed displacement), with the undeformed mesh's smallest."""
    import numpy as np

    import synth

    j0 = synth.hex_jacobians(w.xv, w.xs, w.meta)
    s0 = np.sign(j0)
    out = {"undeformed": float(np.abs(j0).min()), "cells": int(j0.size)}
    for name, dv in dvs.items():
        j = synth.hex_jacobians(w.xv + dv, w.xs + w.ds, w.meta) * s0
        out[name] = float(j.min())
        out[name + "_inverted_cells"] = int((j <= 0).sum())
    return out


def side_block(ctx, name, precision, basis, steps, warmup, with_oracle):
    """A further workload of the same path: greedy and volume figures and the roofline fraction."""
    m = run_workload(ctx, name, precision, basis, steps, warmup)
    w, cs = m["w"], m["cs"]
    big = w.n_s * w.cap_total() > 5e7
    b = {"workload": f"{w.name}: {m['desc']}", "precision": precision,
         "control_points_per_level": m["n_c"], "reduced_volume_points_per_level": m["n_d"],
         "in_support_pairs_per_volume_update": m["in_support"],
         "evaluated_pairs_per_volume_update": m["evaluated"],
         "dense_pairs_per_volume_update": m["dense_pairs"],
         "volume_update_ms": statistics.median(m["vol_ms"]),
         "in_support_evals_per_s": m["in_support"] / (statistics.median(m["vol_ms"]) / 1e3),
         "roofline": volume_roofline(m, precision, basis, name)}
    b.update(greedy_block(m, basis))
    ref = None
    if with_oracle:
        cpu, ref = oracle_leg(m, basis, big, budget_s=3.0)
        b["cpu_baseline"] = cpu
        b["selection_identical_to_oracle"] = ref["same"]
        b["selection_check"] = ref["check"]
    return m, b, ref


def seeded_start_block(ctx, m, basis, scale=1.25):
    """The next icing step (displacement x scale) seeded with this step's control sets and no
    resident basis, timed both ways: each level's seeds started from the blocked FP64 MFMA
    Cholesky of their Phi_CC and the blocked MFMA triangular solve for their Newton basis, and
    appended one iteration each. Same control sets either way (checked)."""
    import numpy as np
    import torch

    from paper_2107_13887_amd import rbfdef

    w, cs = m["w"], m["cs"]
    used = cs.n_levels_used
    ctrl = cs.ctrl_idx[: cs.total].cpu().numpy()
    off = cs.level_off
    seeds = [[int(p) for p in ctrl[off[l]:off[l + 1]]] for l in range(used)]
    seeds += [[] for _ in range(w.n_levels - used)]
    ds2 = (scale * m["ds"]).contiguous()
    call = lambda: rbfdef.rbf_greedy_select(ctx, m["xs"], ds2, w.radius, w.eps, rho=w.rho, cap=w.cap_total(),
                                            seeds=seeds, precision="fp64", want_residual=False, basis=basis)
    res = {}
    for start, reps in (("factor", 3), ("append", 1)):
        os.environ["RBF_SEED_START"] = start
        try:
            call()
            torch.cuda.synchronize()
            if start == "factor":
                rbfdef.rbf_ctx_set_timing(ctx, True)
            times = []
            for _ in range(reps):
                t0 = time.perf_counter()
                c2 = call()
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            if start == "factor":
                dev = {k: rbfdef.rbf_ctx_kernel_time(ctx, k) for k in ("seed_start", "seed_factor", "seed_basis")}
                rbfdef.rbf_ctx_set_timing(ctx, False)
        finally:
            os.environ.pop("RBF_SEED_START", None)
        res[start] = (statistics.median(times), c2.ctrl_idx[: c2.total].cpu().numpy(), c2.n_iterations)
    flops_chol = flops_basis = 0
    g = (w.n_s + 63) // 64
    for sl in seeds:
        nb = (len(sl) + 63) // 64
        if len(sl) < 32:
            continue
        flops_chol += sum((nb - kb - 1) * (nb - kb) // 2 for kb in range(nb)) * 2 * 64 ** 3
        flops_basis += g * (nb * (nb - 1) // 2 + nb) * 2 * 64 ** 3
    per = lambda k: dev[k][0] / 3   # per call (three timed calls), summed over its levels
    mf_ms = per("seed_factor") + per("seed_basis")
    return {
        "workload": f"{w.name} next icing step (displacement x {scale}) seeded with this step's control "
                    "sets, no resident basis",
        "seeds_per_level": [len(sl) for sl in seeds],
        "greedy_call_ms": {"factor": res["factor"][0] * 1e3, "append": res["append"][0] * 1e3},
        "seeded_start_ms_device": per("seed_start"),
        "seed_factor_ms_device": per("seed_factor"),
        "seed_basis_ms_device": per("seed_basis"),
        "append_minus_factor_ms": (res["append"][0] - res["factor"][0]) * 1e3,
        "identical_selections": bool(np.array_equal(res["factor"][1], res["append"][1])),
        "argmax_iterations_after_seeds": res["factor"][2],
        "mfma_flops": {"cholesky_trailing": flops_chol, "basis_trsm": flops_basis},
        "mfma_tflops_in_factor_and_basis": (flops_chol + flops_basis) / (mf_ms / 1e3) / 1e12 if mf_ms > 0 else None,
        "frac_of_fp64_mfma_peak": (flops_chol + flops_basis) / (mf_ms / 1e3) / 78.6e12 if mf_ms > 0 else None,
        "timers_note": "device times per call (hipEvents on the launch stream), summed over the levels",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg2",
                    help="cfg0..cfg3, sine2d, sine3d (one deformation per step), or cfg4 (serving mix)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--basis", default="c2", choices=["c0", "c2", "c4", "c6"])
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (CPU baseline and the parity references)")
    ap.add_argument("--extra-workloads", default="cfg1",
                    help="comma-separated workloads measured after the main one (empty: none)")
    ap.add_argument("--study-workload", default="cfg3",
                    help="workload of the mixed-precision study with mesh validity (empty: none)")
    ap.add_argument("--serve-geometries", type=int, default=16,
                    help="geometries of the reduced serving mix replayed after the main timing (0: skip)")
    ap.add_argument("--serve-scale", type=float, default=0.25,
                    help="size scale of the reduced serving mix")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2107_13887_amd import rbfdef

    if args.workload == "cfg4":
        return serve_main(args)
    ctx = rbfdef.rbf_ctx_create(0)
    dev = torch.device("cuda:0")
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    m = run_workload(ctx, args.workload, args.precision, args.basis, args.steps, args.warmup)
    w, cs, stream = m["w"], m["cs"], m["stream"]
    big = w.n_s * w.cap_total() > 5e7       # the oracle's whole greedy would take minutes
    radius, D, off = m["radius"], m["D"], m["off"]
    # Secondary: the plain call on the caller's (unsorted) volume, with its per-call compaction.
    plain_ms = _median_ms(stream, lambda: rbfdef.rbf_volume_update(
        ctx, radius, D, off, cs.xc, cs.alpha, m["xv"], m["dw"], precision=args.precision,
        basis=args.basis), 5)
    cpu, ref = (None, None) if args.no_cpu_baseline else oracle_leg(m, args.basis, big)
    study, _, _ = precision_study(ctx, m, args.basis, ref)

    # Dense FP64 solve (blocked Cholesky, trailing updates on FP64 MFMA): n^3/3 flops of the
    # factorization plus the dim triangular pairs, on the step's largest level and on the first
    # min(N_s, 4000) surface points with the widest radius (a dense SPD matrix).
    used = cs.n_levels_used
    dense = []
    n_c = m["n_c"]
    big_l = max(range(used), key=lambda l: n_c[l]) if used else 0
    sets = [("largest level of the step", cs.xc[:, off[big_l]:off[big_l + 1]].contiguous(),
             m["ds"][:, cs.ctrl_idx[off[big_l]:off[big_l + 1]]].contiguous(), radius[big_l])]
    nd = min(w.n_s, 4000)
    sets.append((f"first {nd} surface points", m["xs"][:, :nd].contiguous(), m["ds"][:, :nd].contiguous(),
                 w.radius[0]))
    for label, sx, sd, rr in sets:
        nn = sx.shape[1]
        if nn < 2:
            continue
        alpha_d = torch.empty_like(sx)
        ms = _median_ms(stream, lambda: rbfdef.rbf_solve_weights(ctx, rr, sx, sd, alpha_d, basis=args.basis), 5)
        flops = nn ** 3 / 3 + 2 * w.dim * nn * nn
        dense.append({"points": nn, "set": label, "ms": ms, "tflops": flops / (ms / 1e3) / 1e12,
                      "frac_of_fp64_mfma": flops / (ms / 1e3) / 78.6e12})
    seeded = seeded_start_block(ctx, m, args.basis)
    # The greedy's per-iteration floor: one 64-point tile, every point selected (eps 0), so each
    # iteration is all synchronization and no streaming.
    n_tiny = min(64, w.n_s)
    xs_t, ds_t = m["xs"][:, :n_tiny].contiguous(), m["ds"][:, :n_tiny].contiguous()
    tiny = lambda: rbfdef.rbf_greedy_select(ctx, xs_t, ds_t, [w.radius[0]], 0.0, rho=w.rho, cap=n_tiny,
                                            seeds=[[0]], precision="fp64", want_residual=False,
                                            basis=args.basis)
    tiny()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ct = tiny()
    torch.cuda.synchronize()
    floor_us = (time.perf_counter() - t0) / max(ct.n_iterations, 1) * 1e6

    vol_s = sum(m["vol_ms"]) / 1e3
    rec = {
        "metric": METRIC,
        "value": m["in_support"] * args.steps / vol_s,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {m['desc']}", "precision": args.precision, "basis": args.basis,
                   "control_points_per_level": n_c, "support_distance_per_level": D,
                   "reduced_volume_points_per_level": m["n_d"],
                   "in_support_pairs_per_volume_update": m["in_support"],
                   "in_support_pairs_per_level": m["in_support_per_level"],
                   "evaluated_pairs_per_volume_update": m["evaluated"],
                   "dense_pairs_per_volume_update": m["dense_pairs"],
                   "parallelism": "single GPU"},
        "value_note": "in-support RBF evaluations (psi > 0 and phi > 0) per second of the volume update: "
                      "in-support pairs per call x steps / the calls' device time (hipEvents on the launch "
                      "stream); dense_evals_per_s counts every reduced point with every control of its level",
        "dense_evals_per_s": m["dense_pairs"] * args.steps / vol_s,
        "evaluated_evals_per_s": m["evaluated"] * args.steps / vol_s,
        "volume_update_ms": statistics.median(m["vol_ms"]),
        "plain_volume_update_ms": plain_ms,
        "greedy_iteration_floor_us": floor_us,
        "greedy_error_curve": error_curve(cs, w),
        "dense_solve": dense,
        "seeded_start": seeded,
        "selection_identical_to_oracle": ref["same"] if ref else None,
        "selection_check": ref["check"] if ref else None,
        "precision_study": study,
        "p50_latency_ms": None,
        "p99_latency_ms": None,
        "roofline": volume_roofline(m, args.precision, args.basis, args.workload),
        "cpu_baseline": cpu,
    }
    rec.update(greedy_block(m, args.basis))
    rbfdef.rbf_geom_release(ctx, m["geom"])
    del m
    extras = {}
    for name in [x for x in args.extra_workloads.split(",") if x and x != args.workload]:
        me, b, _ = side_block(ctx, name, "fp64", args.basis, max(5, args.steps // 2), 2,
                              not args.no_cpu_baseline)
        rbfdef.rbf_geom_release(ctx, me["geom"])
        extras[name] = b
    if extras:
        rec["other_workloads"] = extras
    if args.study_workload:
        ms_, b, ref_s = side_block(ctx, args.study_workload, "mixed", args.basis, 3, 1, not args.no_cpu_baseline)
        st, dv64, dvg = precision_study(ctx, ms_, args.basis, ref_s)
        b["precision_study"] = st
        if ms_["w"].dim == 3 and "n_chord" in ms_["w"].meta:
            b["min_hex_jacobian"] = mesh_validity(ms_["w"], {"fp64": dv64, "guarded_mixed": dvg})
        rbfdef.rbf_geom_release(ctx, ms_["geom"])
        rec["mixed_precision_workload"] = b
    if args.serve_geometries > 0:
        import synth

        geoms, reqs = synth.serving_mix(n_geom=args.serve_geometries, scale=args.serve_scale)
        log(f"bench: serving mix of {len(reqs)} requests on {len(geoms)} geometries")
        srv = serving_replay(ctx, geoms, reqs)
        srv["mix"] = (f"{args.serve_geometries} geometries at size scale {args.serve_scale} of the "
                      "serving mix, 4 icing steps each, Poisson arrivals at 20/s, mixed precision")
        sat = serving_replay(ctx, geoms, reqs, time_scale=0.0, compare=False)
        srv["saturated"] = {"throughput_req_per_s": sat["throughput_req_per_s"],
                            "p50_latency_ms": sat["p50_latency_ms"], "p99_latency_ms": sat["p99_latency_ms"],
                            "makespan_s": sat["makespan_s"],
                            "note": "every request submitted at t = 0 (capacity of the serving loop)"}
        rec["p50_latency_ms"] = srv["p50_latency_ms"]
        rec["p99_latency_ms"] = srv["p99_latency_ms"]
        rec["serving"] = srv
    rbfdef.rbf_ctx_destroy(ctx)
    print(json.dumps(rec))


def serve_main(args):
    """The full serving mix: throughput and request latency through the serving loop."""
    import torch

    import synth
    from paper_2107_13887_amd import rbfdef

    t0 = time.perf_counter()
    geoms, reqs = synth.serving_mix(progress=log)
    log(f"bench: serving mix built in {time.perf_counter() - t0:.1f}s")
    ctx = rbfdef.rbf_ctx_create(0)
    torch.cuda.synchronize()
    # Warmup: one small replay compiles nothing but touches every code path and the pool.
    wg, wr = synth.serving_mix(n_geom=4, scale=0.125, seed=9)
    serving_replay(ctx, wg, wr, compare=False)
    log("bench: warmup replay done")
    srv = serving_replay(ctx, geoms, reqs)
    rbfdef.rbf_ctx_destroy(ctx)
    _, desc = build_workload("cfg4")
    rec = {
        "metric": "requests/s through the serving loop (p50/p99 request latency beside it)",
        "value": srv["throughput_req_per_s"],
        "unit": "requests/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": len(wr),
        "ms_per_step": srv["makespan_s"] / len(reqs) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"cfg4: {desc}", "parallelism": "single GPU"},
        "p50_latency_ms": srv["p50_latency_ms"],
        "p99_latency_ms": srv["p99_latency_ms"],
        "serving": srv,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(rec))
    # This process ends here without the interpreter's and the libraries' exit handlers: after the
    # full mix one of them faults in exit() (a segmentation fault once the result line is out,
    # from a handler of a library mapped after the GPU runtime started; the same serving loop on
    # 16 geometries exits normally, and unloading this library first did not change it). The
    # context is destroyed and the device idle at this point, and nothing is left to write.
    sys.stdout.flush()
    sys.stderr.flush()
    os._exit(0)


if __name__ == "__main__":
    main()

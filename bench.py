#!/usr/bin/env python3
"""Benchmark of the multi-level greedy RBF mesh deformation hot path on one MI355X.

One step = the whole path on one synthetic deformation: multi-level greedy selection of the
control points on the surface (rbf_greedy_select) followed by the wall-distance-reduced volume
update (rbf_volume_update). Inputs are resident in HBM before the timed region starts.

Headline value: RBF evaluations per second of the volume update, i.e. the number of
(reduced volume point, control point) pairs sum_l n_{D_l} N_{c,l} divided by the device time of
the volume-update calls (hipEvents on the launch stream). The kernel skips the controls whose
support misses a block of points (phi = 0 there), so it computes fewer pairs than that count;
the roofline fraction is taken on the pairs it actually computes (counted on the device). The geometry is made resident once
before the timed region (rbf_geom_create: volume stored in wall-distance order), so each step's
volume reduction is a prefix (rbf_geom_volume_update); the plain call on the unsorted volume
(rbf_volume_update, with its per-call compaction) is reported beside it. Also reported: greedy time-to-eps,
the roofline fraction of the volume kernel-sum launch (VALU issue bound), and the FP64 CPU oracle
timed on this machine's host cores on the same workload.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload cfg1] [--precision fp64]
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("RBF evals/s (volume update: reduced-volume points x control points per second; pairs "
          "outside the compact support are skipped, not computed), greedy time-to-eps, p50/p99 "
          "request latency")
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
        return synth.workload_cfg2(), ("3D swept wing ice horn: N_s=80000, N_v=4000000, R_l=3c/0.8c/0.2c, "
                                       "eps=1e-4c, cap 4000, D=1c")
    if name == "cfg4":
        return None, ("serving mix: 64 geometries (60% 2D airfoils, N_s 500-8000; 40% 3D wings, "
                      "N_s 10k-80k), 4 warm-started icing steps each, Poisson arrivals at 20/s, "
                      "eps in {1e-4, 1e-5}, mixed precision")
    if name == "cfg3":
        return synth.workload_cfg3(), ("3D swept wing bend+twist: N_s=80000, N_v=4000000, "
                                       "R_l=3c/0.8c/0.2c, eps=1e-4c, cap 4000, D=1c")
    if name == "sine2d":
        return synth.workload_sine2d(), ("2D NACA0012 global deformation dy = 0.01 sin(15 pi x): N_s=4000, "
                                         "N_v=400000, R=2c on 5 levels, eps=1e-5 max|dS|, D_l = 5 max|dS_l|")
    if name == "sine3d":
        return synth.workload_sine3d(), ("3D swept wing global deformation 0.03 sin(4 pi y): N_s=80000, "
                                         "N_v=4000000, R=3c on 4 levels, eps=1e-4c, cap 4000, D_l = 5 max|dS_l|")
    raise SystemExit(f"unknown workload {name}")


def kernel_source_hash():
    """Hash of the kernel-sum source with comments and white space removed, so that a counter
    summary stays matched to its kernel through edits of the comments only."""
    import hashlib
    import re

    with open(os.path.join(ROOT, "paper_2107_13887_amd", "csrc", "ksum.hip")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return hashlib.sha256("".join(src.split()).encode()).hexdigest()[:16]


def measured_traffic(workload, precision):
    """HBM bytes per launch of the volume kernel-sum, from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain-copy calibration), or None when that summary was
    taken on a different kernel source."""
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


def cpu_baseline(w, cs, radius, D, off, basis, big, budget_s=12.0):
    """The FP64 oracle timed on this machine's host cores, on a bounded sample of the same
    workload: the volume update of the step's control sets over the reduced volume (all of it,
    or a seeded subset when one pass would be long), repeated for about budget_s seconds; the same
    on one thread for a short while; and the oracle's whole greedy where it is affordable."""
    import numpy as np

    import oracle

    o = oracle.get()
    xc = cs.xc[:, : cs.total].cpu().numpy()
    al = cs.alpha[:, : cs.total].cpu().numpy()
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
    out = {"value": pairs * reps / t, "unit": "evals/s", "cores": cores, "kind": "oracle",
           "sample": f"volume update of the step's {cs.total} control points over {pick.size} of the "
                     f"{inside.size} reduced-volume points ({pairs:.3g} pairs), {reps} repetitions in "
                     f"{t:.1f} s"}
    if omp:
        sub = pick[: max(1, pick.size // max(1, cores))]
        omp.omp_set_num_threads(1)
        r1, t1 = timed(lambda: vol(np.ascontiguousarray(w.xv[:, sub]), np.ascontiguousarray(w.dwall[sub])), 2.0)
        omp.omp_set_num_threads(cores)
        out["single_thread_value"] = float(per_point[sub].sum()) * r1 / t1
    if not big:
        g = lambda: o.greedy(w.dim, w.xs, w.ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(),
                             seeds=w.seeds, basis=basis)
        rg, tg = timed(g, 3.0)
        out["greedy_time_to_eps_s"] = tg / rg
    return out


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg1",
                    help="cfg0..cfg3, sine2d, sine3d (one deformation per step), or cfg4 (serving mix)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--basis", default="c2", choices=["c0", "c2", "c4", "c6"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    import numpy as np
    import torch

    import oracle
    from paper_2107_13887_amd import rbfdef

    if args.workload == "cfg4":
        return serve_main(args)
    t0 = time.perf_counter()
    w, desc = build_workload(args.workload)
    log(f"bench: workload {w.name} built in {time.perf_counter() - t0:.1f}s")
    big = w.n_s * w.cap_total() > 5e7       # the oracle's whole greedy would take minutes
    dev = torch.device("cuda:0")
    xs = torch.from_numpy(w.xs).to(dev)
    ds = torch.from_numpy(w.ds).to(dev)
    xv = torch.from_numpy(w.xv).to(dev)
    dw = torch.from_numpy(w.dwall).to(dev)
    ctx = rbfdef.rbf_ctx_create(0)
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
                                      seeds=w.seeds, precision=args.precision, want_residual=False,
                                      basis=args.basis)
        g1 = time.perf_counter()
        radius, D, off = supports(cs)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rbfdef.rbf_geom_volume_update(ctx, geom, radius, D, off, cs.xc, cs.alpha, dv,
                                      precision=args.precision, basis=args.basis)
        e1.record(stream)
        return cs, g1 - g0, (e0, e1)

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for i in range(args.warmup):
        cs, _, _ = step()
        torch.cuda.synchronize()
        log(f"bench: warmup {i + 1}/{args.warmup} done ({cs.total} control points)")
    rbfdef.rbf_ctx_set_timing(ctx, True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    greedy_t, events = [], []
    for i in range(args.steps):
        cs, tg, ev = step()
        greedy_t.append(tg)
        events.append(ev)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    vol_ms = [a.elapsed_time(b) for a, b in events]
    kname = "volume_ksum_" + args.precision
    k_ms, k_n = rbfdef.rbf_ctx_kernel_time(ctx, kname)
    rbfdef.rbf_ctx_set_timing(ctx, False)
    log(f"bench: {args.steps} steps in {wall:.3f}s")
    radius, D, off = supports(cs)
    vol_call = lambda prec: rbfdef.rbf_geom_volume_update(ctx, geom, radius, D, off, cs.xc, cs.alpha, dv,
                                                          precision=prec, basis=args.basis)
    # Pairs the kernel computes per launch: one more, untimed launch with the device counter on.
    rbfdef.rbf_ctx_set_timing(ctx, False, count_pairs=True)
    vol_call(args.precision)
    evaluated = float(rbfdef.rbf_ctx_kernel_pairs(ctx, kname))
    rbfdef.rbf_ctx_set_timing(ctx, False)
    # Secondary: the plain call on the caller's (unsorted) volume, with its per-call compaction.
    plain_ms = _median_ms(stream, lambda: rbfdef.rbf_volume_update(
        ctx, radius, D, off, cs.xc, cs.alpha, xv, dw, precision=args.precision, basis=args.basis), 5)

    n_c = [off[l + 1] - off[l] for l in range(len(radius))]
    n_d = [int((w.dwall < D[l]).sum()) for l in range(len(radius))]
    pairs = sum(n_d[l] * n_c[l] for l in range(len(radius)))
    value = pairs * args.steps / (sum(vol_ms) / 1e3)
    avg_kernel_s = (k_ms / k_n) / 1e3 if k_n else float("nan")
    peak = VALU_LANE_OPS / min_slots(w.dim, args.basis, args.precision) / 1e9
    achieved = evaluated / avg_kernel_s / 1e9

    # Precision study on this step's control sets: the FP32 pair arithmetic (shifted local origin,
    # FP64 accumulation) beside the FP64 path, and both against the FP64 oracle on sampled points.
    ms64 = _median_ms(stream, lambda: vol_call("fp64"), 10)
    vol_call("fp64")
    torch.cuda.synchronize()
    dv64 = dv.cpu().numpy()
    msmx = _median_ms(stream, lambda: vol_call("mixed"), 10)
    vol_call("mixed")
    torch.cuda.synchronize()
    dvmx = dv.cpu().numpy()
    # The guarded form: FP32 only on the levels whose measured FP32 error at the surface is at
    # most 1e-6 max |dS| (what a mixed-precision request runs). The step's greedy ran in FP64
    # unless --precision mixed, so the measurement comes from one mixed greedy here.
    csm = cs if args.precision == "mixed" else rbfdef.rbf_greedy_select(
        ctx, xs, ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(), seeds=w.seeds, precision="mixed",
        want_residual=False, basis=args.basis)
    guard = ["mixed" if f else "fp64" for f in csm.fp32_levels()][: len(radius)]
    msg = _median_ms(stream, lambda: vol_call(guard), 10)
    vol_call(guard)
    torch.cuda.synchronize()
    dvg = dv.cpu().numpy()
    inside = np.flatnonzero(w.dwall < max(D))
    pick = np.random.default_rng(11).choice(inside, min(20000, inside.size), replace=False)
    xcn = cs.xc[:, : cs.total].cpu().numpy()
    aln = cs.alpha[:, : cs.total].cpu().numpy()
    orc = oracle.get()
    ref_s = orc.volume(radius, D, off, xcn, aln, w.xv[:, pick], w.dwall[pick], basis=args.basis)
    study = {"fp64_volume_update_ms": ms64, "mixed_volume_update_ms": msmx,
             "mixed_speedup": ms64 / msmx,
             "mixed_vs_fp64_gpu": _normwise(dvmx, dv64),
             "fp64_vs_oracle_sampled": _normwise(dv64[:, pick], ref_s),
             "mixed_vs_oracle_sampled": _normwise(dvmx[:, pick], ref_s),
             "level_fp32_err_at_surface": csm.level_fp32_err[: csm.n_levels_used],
             "guarded_levels": guard,
             "guarded_volume_update_ms": msg,
             "guarded_vs_fp64_gpu": _normwise(dvg, dv64),
             "guarded_vs_oracle_sampled": _normwise(dvg[:, pick], ref_s),
             "oracle_sample_points": int(pick.size)}

    # Selection parity outside the timed region: the whole greedy where the oracle affords it,
    # otherwise its first 60 selections (the argmax sequence does not depend on the cap).
    if big:
        k = 60
        ref = orc.greedy(w.dim, w.xs, w.ds, w.radius, w.eps, rho=w.rho, cap=k, seeds=w.seeds,
                         basis=args.basis)
        same = bool(np.array_equal(cs.ctrl_idx[:k].cpu().numpy(), ref.ctrl_idx[:k]))
        parity = f"first {k} selections against the oracle's greedy capped at {k}"
    else:
        ref = orc.greedy(w.dim, w.xs, w.ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(),
                         seeds=w.seeds, basis=args.basis)
        same = bool(np.array_equal(cs.ctrl_idx[: cs.total].cpu().numpy(), ref.ctrl_idx))
        parity = "whole control set against the oracle's greedy"
    cpu = None if args.no_cpu_baseline else cpu_baseline(w, cs, radius, D, off, args.basis, big)

    used = cs.n_levels_used
    # Dense FP64 solve (blocked Cholesky, trailing updates on FP64 MFMA): n^3/3 flops of the
    # factorization plus the dim triangular pairs, on the step's largest level and on the first
    # min(N_s, 4000) surface points with the widest radius (a dense SPD matrix).
    dense = []
    big_l = max(range(used), key=lambda l: n_c[l]) if used else 0
    sets = [("largest level of the step", cs.xc[:, off[big_l]:off[big_l + 1]].contiguous(),
             ds[:, cs.ctrl_idx[off[big_l]:off[big_l + 1]]].contiguous(), radius[big_l])]
    nd = min(w.n_s, 4000)
    sets.append((f"first {nd} surface points", xs[:, :nd].contiguous(), ds[:, :nd].contiguous(), w.radius[0]))
    for label, sx, sd, rr in sets:
        nn = sx.shape[1]
        if nn < 2:
            continue
        alpha_d = torch.empty_like(sx)
        ms = _median_ms(stream, lambda: rbfdef.rbf_solve_weights(ctx, rr, sx, sd, alpha_d, basis=args.basis), 5)
        flops = nn ** 3 / 3 + 2 * w.dim * nn * nn
        dense.append({"points": nn, "set": label, "ms": ms, "tflops": flops / (ms / 1e3) / 1e12,
                      "frac_of_fp64_mfma": flops / (ms / 1e3) / 78.6e12})
    # The greedy's per-iteration floor: one 64-point tile, every point selected (eps 0), so each
    # iteration is all synchronization and no streaming.
    n_tiny = min(64, w.n_s)
    tiny = lambda: rbfdef.rbf_greedy_select(ctx, xs[:, :n_tiny].contiguous(), ds[:, :n_tiny].contiguous(),
                                            [w.radius[0]], 0.0, rho=w.rho, cap=n_tiny, seeds=[[0]],
                                            precision="fp64", want_residual=False, basis=args.basis)
    tiny()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ct = tiny()
    torch.cuda.synchronize()
    floor_us = (time.perf_counter() - t0) / max(ct.n_iterations, 1) * 1e6

    # The greedy's Newton-basis stream (HBM-bound on large surfaces): an iteration with n finished
    # columns reads the N_s x n basis and writes one column, and reads/writes E and reads x_s.
    g_bytes = 0
    for l in range(used):
        m = n_c[l] if l < len(n_c) else 0
        g_bytes += 8 * w.n_s * (m * (m - 1) // 2) + m * w.n_s * (9 + 24 * w.dim)
    g_time = statistics.median(greedy_t)
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {desc}", "precision": args.precision, "basis": args.basis,
                   "control_points_per_level": n_c, "support_distance_per_level": D,
                   "reduced_volume_points_per_level": n_d,
                   "pairs_per_volume_update": pairs,
                   "evaluated_pairs_per_volume_update": evaluated,
                   "parallelism": "single GPU"},
        "greedy_time_to_eps_s": statistics.median(greedy_t),
        "greedy_iterations": cs.n_iterations,
        "greedy_iterations_per_s": cs.n_iterations / statistics.median(greedy_t),
        "greedy_roofline": {"bound": "hbm", "achieved": g_bytes / g_time / 1e9, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": g_bytes / g_time / 1e9 / HBM_PEAK_GBS,
                            "algorithmic_bytes": g_bytes,
                            "work_unit": "Newton-basis stream of every iteration (N_s x n read, one "
                                         "column written, E and x_s), whole greedy call timed"},
        "greedy_iteration_floor_us": floor_us,
        "greedy_error_curve": error_curve(cs, w),
        "dense_solve": dense,
        "greedy_levels": [{"controls": n_c[l] if l < len(n_c) else 0, "seconds": cs.level_seconds[l],
                           "max_err_in": cs.level_in_max[l], "max_err_out": cs.level_max_err[l]}
                          for l in range(used)],
        "volume_update_ms": statistics.median(vol_ms),
        "plain_volume_update_ms": plain_ms,
        "plain_volume_update_evals_per_s": pairs / (plain_ms / 1e3),
        "selection_identical_to_oracle": same,
        "selection_check": parity,
        "precision_study": study,
        "p50_latency_ms": None,
        "p99_latency_ms": None,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Gpair/s",
                     "frac": achieved / peak,
                     "traffic": measured_traffic(args.workload, args.precision)
                     if args.basis == "c2" else None,
                     "kernel": kname, "kernel_avg_ms": avg_kernel_s * 1e3, "kernel_launches": k_n,
                     "work_unit": "evaluated (point, control) pairs per launch, "
                                  "controls whose support misses a point block skipped"},
        "cpu_baseline": cpu,
    }
    rbfdef.rbf_geom_release(ctx, geom)
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


if __name__ == "__main__":
    main()

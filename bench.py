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
MIN_SLOTS = {2: 17, 3: 20}                 # minimal VALU slots per pair (FP64), see the design doc


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
    raise SystemExit(f"unknown workload {name}")


def kernel_source_hash():
    import hashlib

    with open(os.path.join(ROOT, "paper_2107_13887_amd", "csrc", "ksum.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


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


def cpu_baseline(w, ref, budget_s=12.0):
    """FP64 oracle timed on the host cores: the volume update on the oracle's own control set,
    repeated on the full reduced volume until about budget_s seconds have passed."""
    import numpy as np

    import oracle

    o = oracle.get()
    D = [w.D] * w.n_levels
    xc = np.ascontiguousarray(w.xs[:, ref.ctrl_idx])
    counts = [int((w.dwall < D[l]).sum()) for l in range(w.n_levels)]
    pairs = sum(counts[l] * int(ref.level_off[l + 1] - ref.level_off[l]) for l in range(w.n_levels))
    reps, t = 0, 0.0
    while t < budget_s and reps < 1000:
        t0 = time.perf_counter()
        o.volume(w.radius, D, ref.level_off, xc, ref.alpha, w.xv, w.dwall)
        t += time.perf_counter() - t0
        reps += 1
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": pairs * reps / t, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"full reduced volume ({counts[0]} of {w.n_v} points) x {ref.level_off[-1]} "
                      f"oracle control points, {reps} repetitions in {t:.1f} s"}


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
    infos = [rbfdef.rbf_wait(ctx, q) for q in pend]
    t_end = max(i.t_done for i in infos)
    failed = sum(1 for i in infos if i.state != rbfdef.REQ_DONE)
    lat = sorted((i.t_done - i.t_arrive) * 1e3 for i in infos)
    queue = sorted((i.t_start - i.t_arrive) * 1e3 for i in infos)
    service = [(i.t_done - i.t_start) * 1e3 for i in infos]
    pct = lambda v, q: v[min(len(v) - 1, int(q * len(v)))]
    out = {
        "requests": len(reqs), "geometries": len(geoms), "icing_steps": steps, "failed": failed,
        "arrival_rate_per_s": len(reqs) / (reqs[-1].arrival * time_scale) if reqs[-1].arrival > 0 else None,
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
        for r, ds in zip(reqs, dss):
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg1")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
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
    dev = torch.device("cuda:0")
    xs = torch.from_numpy(w.xs).to(dev)
    ds = torch.from_numpy(w.ds).to(dev)
    xv = torch.from_numpy(w.xv).to(dev)
    dw = torch.from_numpy(w.dwall).to(dev)
    D = [w.D] * w.n_levels
    ctx = rbfdef.rbf_ctx_create(0)
    stream = torch.cuda.current_stream()
    # Setup, outside the timed region: the geometry (surface, volume, wall distances) becomes
    # resident once, its volume stored in wall-distance order, as across successive icing steps.
    geom = rbfdef.rbf_geom_create(ctx, xs, xv, dw)
    dv = torch.empty((w.dim, w.n_v), dtype=torch.float64, device=dev)

    def step():
        g0 = time.perf_counter()
        cs = rbfdef.rbf_greedy_select(ctx, xs, ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(),
                                      seeds=w.seeds, precision=args.precision, want_residual=False)
        g1 = time.perf_counter()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rbfdef.rbf_geom_volume_update(ctx, geom, w.radius, D, cs.level_off, cs.xc, cs.alpha, dv,
                                      precision=args.precision)
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
    k_ms, k_n = rbfdef.rbf_ctx_kernel_time(ctx, "volume_ksum_" + args.precision)
    k_pairs = rbfdef.rbf_ctx_kernel_pairs(ctx, "volume_ksum_" + args.precision)
    log(f"bench: {args.steps} steps in {wall:.3f}s")
    # Secondary: the plain call on the caller's (unsorted) volume, with its per-call compaction.
    plain = []
    for _ in range(5):
        a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a_.record(stream)
        rbfdef.rbf_volume_update(ctx, w.radius, D, cs.level_off, cs.xc, cs.alpha, xv, dw,
                                 precision=args.precision)
        b_.record(stream)
        plain.append((a_, b_))
    torch.cuda.synchronize()
    plain_ms = statistics.median(a_.elapsed_time(b_) for a_, b_ in plain)

    n_c = [cs.level_off[l + 1] - cs.level_off[l] for l in range(w.n_levels)]
    n_d = [int((w.dwall < D[l]).sum()) for l in range(w.n_levels)]
    pairs = sum(n_d[l] * n_c[l] for l in range(w.n_levels))
    value = pairs * args.steps / (sum(vol_ms) / 1e3)
    avg_kernel_s = (k_ms / k_n) / 1e3 if k_n else float("nan")
    peak = VALU_LANE_OPS / MIN_SLOTS[w.dim] / 1e9
    evaluated = k_pairs / k_n if k_n else float("nan")     # pairs the kernel computed per launch
    achieved = evaluated / avg_kernel_s / 1e9

    # Parity and CPU baseline outside the timed region.
    ref = oracle.get().greedy(w.dim, w.xs, w.ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(),
                              seeds=w.seeds)
    same = bool(np.array_equal(cs.ctrl_idx[: cs.total].cpu().numpy(), ref.ctrl_idx))
    cpu = None if args.no_cpu_baseline else cpu_baseline(w, ref)

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
        "config": {"workload": f"{w.name}: {desc}", "precision": args.precision,
                   "control_points_per_level": n_c, "reduced_volume_points_per_level": n_d,
                   "pairs_per_volume_update": pairs,
                   "evaluated_pairs_per_volume_update": evaluated,
                   "parallelism": "single GPU"},
        "greedy_time_to_eps_s": statistics.median(greedy_t),
        "greedy_iterations": cs.n_iterations,
        "volume_update_ms": statistics.median(vol_ms),
        "plain_volume_update_ms": plain_ms,
        "plain_volume_update_evals_per_s": pairs / (plain_ms / 1e3),
        "selection_identical_to_oracle": same,
        "p50_latency_ms": None,
        "p99_latency_ms": None,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Gpair/s",
                     "frac": achieved / peak, "traffic": measured_traffic(args.workload, args.precision),
                     "kernel": "volume_ksum_" + args.precision,
                     "kernel_avg_ms": avg_kernel_s * 1e3, "kernel_launches": k_n},
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
    geoms, reqs = synth.serving_mix()
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

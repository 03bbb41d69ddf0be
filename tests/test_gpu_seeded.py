"""Seeded level starts (Section 3 with given first control points; eq. (9) for their weights).

A level handed n seed points (a warm start whose resident basis was dropped, or a call with
seeds) forms its Newton basis in one pass: Phi_CC of the seeds factored by the blocked FP64 MFMA
Cholesky, then V = Phi_sC L^-T by blocked FP64 MFMA triangular solves, instead of n single
appends. Bar: the control sets identical to the oracle's greedy seeded with the same points and
to the one-by-one path's; residual, level errors and error curve within the FP64 bound; weights
within 1e-6 normwise (the greedy tests' bar). Cases: the previous icing step's control sets as
seeds (2D multi-level airfoil, a surface not a multiple of 64 points, a small swept wing), random
first-level seed sets of 1, 63, 64, 65 and 200 points (one block, a ragged block, several
blocks), two seeds at the same coordinates (not positive definite: the level falls back to
appending and stops at the breakdown, as the oracle does), and serving with no room for resident
bases, so that every warm start takes this path.
"""
import numpy as np
import pytest
import torch

import synth
from helpers import to_dev
from paper_2107_13887_amd import rbfdef
from test_gpu_greedy import _check_same

pytestmark = pytest.mark.gpu


def _seeded(gctx, w, seeds, start, monkeypatch):
    monkeypatch.setenv("RBF_SEED_START", start)
    cs = rbfdef.rbf_greedy_select(gctx, to_dev(w.xs), to_dev(w.ds), w.radius, w.eps, rho=w.rho,
                                  cap=w.cap_total(), seeds=seeds)
    torch.cuda.synchronize()
    monkeypatch.delenv("RBF_SEED_START")
    return cs


def _ctrl(cs):
    return cs.ctrl_idx[: cs.total].cpu().numpy()


def _workload(case):
    if case == "cfg1":
        return synth.workload_cfg1()
    if case == "cfg1-ragged":
        return synth.workload_cfg1(n_s=3002, n_layers=8)
    if case == "wing":
        return synth.workload_cfg2(n_chord=60, n_span=30, n_layers=4)
    raise ValueError(case)


def _step2(w, seeds, scale=1.5):
    return synth.Workload(w.name + "_step2", w.dim, w.xs, np.ascontiguousarray(scale * w.ds), w.xv, w.dwall,
                          w.radius, w.eps, w.rho, w.D, w.cap, seeds)


@pytest.mark.parametrize("case", ["cfg1", "cfg1-ragged", "wing"])
def test_seeded_start_matches_oracle(gctx, orc, monkeypatch, case):
    """Step 2 of an icing sequence seeded with step 1's control sets (hundreds per level)."""
    w = _workload(case)
    cold = orc.greedy(w.dim, w.xs, w.ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(), seeds=w.seeds)
    seeds = [list(cold.level(l)[0]) for l in range(cold.n_levels_used)]
    seeds += [[] for _ in range(w.n_levels - len(seeds))]
    w2 = _step2(w, seeds)
    print(f"case {case} n_s={w.n_s} seeds per level {[len(s) for s in seeds]}", flush=True)
    ref = orc.greedy(w.dim, w.xs, w2.ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(), seeds=seeds)
    got = _seeded(gctx, w2, seeds, "factor", monkeypatch)
    _check_same(orc, w2, ref, got)
    one = _seeded(gctx, w2, seeds, "append", monkeypatch)
    assert np.array_equal(_ctrl(got), _ctrl(one))


@pytest.mark.parametrize("n0", [1, 63, 64, 65, 200])
def test_random_seed_sets(gctx, orc, monkeypatch, n0):
    """Random first-level seed sets on a small swept wing (1800 surface points, three levels)."""
    w = synth.workload_cfg2(n_chord=60, n_span=30, n_layers=4)
    rng = np.random.default_rng(n0)
    seeds = [[int(p) for p in rng.choice(w.n_s, size=n0, replace=False)]]
    w.seeds = seeds
    print(f"case n0={n0} n_s={w.n_s}", flush=True)
    ref = orc.greedy(w.dim, w.xs, w.ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(), seeds=seeds)
    got = _seeded(gctx, w, seeds, "factor", monkeypatch)
    _check_same(orc, w, ref, got)
    assert np.array_equal(_ctrl(got)[:n0], np.array(seeds[0]))


def test_coincident_seeds_fall_back_to_appending(gctx, orc, monkeypatch):
    """Two seeds at the same coordinates (distinct indices) make Phi_CC singular: the factor meets
    a zero pivot, the level is appended one by one and stops at the breakdown, as the oracle's
    does. (A repeated index is rejected as an invalid argument before any of this.)"""
    w = synth.random_workload(77, 2, 700, 10, [1.0], 1e-7)
    w.xs[:, 139] = w.xs[:, 10]
    seeds = [list(range(0, 140, 2)) + [139] + list(range(1, 40, 2))]
    print(f"case coincident seeds, {len(seeds[0])} seeds", flush=True)
    ref = orc.greedy(w.dim, w.xs, w.ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(), seeds=seeds)
    assert ref.level_stop[0] == rbfdef.RBF_STOP_BREAKDOWN
    got = _seeded(gctx, w, seeds, "factor", monkeypatch)
    assert got.level_stop[0] == rbfdef.RBF_STOP_BREAKDOWN
    assert np.array_equal(_ctrl(got), ref.ctrl_idx)


def test_warm_start_without_room_for_bases(gctx, orc, monkeypatch):
    """Serving with no room for resident bases (RBF_CACHE_FRACTION=0): each warm-started icing step
    starts its levels from the blocked factor of the previous step's control sets, and equals the
    oracle's greedy seeded with them."""
    monkeypatch.setenv("RBF_CACHE_FRACTION", "0")
    w = synth.workload_cfg1(n_s=2000, n_layers=8)
    geom = rbfdef.rbf_geom_create(gctx, to_dev(w.xs), to_dev(w.xv), to_dev(w.dwall))
    prev = w.seeds
    for step in range(3):
        ds = np.ascontiguousarray((1.0 + 0.4 * step) * w.ds)
        dv = torch.zeros((2, w.n_v), dtype=torch.float64, device="cuda:0")
        r = rbfdef.rbf_submit(gctx, geom, to_dev(ds), dv, w.radius, w.eps, [w.D] * w.n_levels, rho=w.rho,
                              cap=w.cap_total(), seeds=w.seeds, warm_start=step > 0, want_ctrl=True)
        info = rbfdef.rbf_wait(gctx, r)
        assert info.state == rbfdef.REQ_DONE, info.result
        ref = orc.greedy(2, w.xs, ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(), seeds=prev)
        got = r.out.ctrl_idx[: r.out.total].cpu().numpy()
        print(f"step {step}: seeds per level {[len(p) for p in prev]}, {r.out.total} controls", flush=True)
        if step > 0:
            assert max(len(p) for p in prev) >= 32   # at least one level starts from the factor
        assert np.array_equal(got, ref.ctrl_idx)
        prev = [list(ref.level(l)[0]) for l in range(ref.n_levels_used)]
        prev += [[] for _ in range(w.n_levels - len(prev))]
    rbfdef.rbf_geom_release(gctx, geom)


@pytest.mark.parametrize("n0", [100, 250])
def test_seeded_start_repeats_bit_for_bit(gctx, monkeypatch, n0):
    """The blocked seeded start reads back, in other threads, the blocks of V each workgroup has
    just stored; a barrier orders them. Two calls on the same seeds, with calls on other inputs
    between them (so the pool hands back memory holding other values), must give the same bits."""
    w = synth.random_workload(90 + n0, 2, 3000, 10, [0.3, 0.08], 1e-7, cap=900)
    rng = np.random.default_rng(n0)
    seeds = [[int(p) for p in rng.choice(w.n_s, size=n0, replace=False)], []]
    other = synth.random_workload(7 + n0, 2, 3000, 10, [0.3, 0.08], 1e-7, cap=900)
    outs = []
    for rep in range(2):
        print(f"case n0={n0} call {rep}", flush=True)
        cs = _seeded(gctx, w, seeds, "factor", monkeypatch)
        outs.append((_ctrl(cs), cs.alpha[:, : cs.total].cpu().numpy().view(np.uint64),
                     cs.e_final.cpu().numpy().view(np.uint64)))
        _seeded(gctx, other, [list(range(0, 2 * n0, 2)), []], "factor", monkeypatch)
    for x, y in zip(outs[0], outs[1]):
        assert np.array_equal(x, y)

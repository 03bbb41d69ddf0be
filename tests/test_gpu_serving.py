"""Serving loop through the C ABI: resident geometries, continuous batching, warm start.

Checks: the resident (wall-distance ordered) volume path agrees with the plain volume update;
every request's results are bit-for-bit the same alone and in a concurrent mix; a warm-started
icing step equals the oracle's greedy seeded with the previous step's control sets; admission
respects a small HBM budget; request timestamps are ordered; bad handles are reported.
"""
import numpy as np
import pytest
import torch

import synth
from helpers import check_fp64, fp64_bound, normwise, sum_magnitude, to_dev
from paper_2107_13887_amd import rbfdef

pytestmark = pytest.mark.gpu


def _requests(n):
    """Small mixed bag of 2D and 3D problems (different sizes)."""
    out = []
    for i in range(n):
        if i % 3 == 2:
            w = synth.workload_cfg2(n_chord=40, n_span=12 + 2 * i, n_layers=6, cap=300)
        elif i % 3 == 1:
            w = synth.workload_cfg1(n_s=200 + 40 * i, n_layers=12)
        else:
            w = synth.workload_cfg0(n_s=120 + 20 * i, n_layers=10)
            w.eps = 1e-4
        out.append(w)
    return out


def _submit(ctx, geom, w, dv, precision="fp64", warm=False, want_ctrl=False):
    return rbfdef.rbf_submit(ctx, geom, to_dev(w.ds), dv, w.radius, w.eps, [w.D] * w.n_levels, rho=w.rho,
                             cap=w.cap_total(), seeds=w.seeds, precision=precision, warm_start=warm,
                             want_ctrl=want_ctrl)


def test_resident_volume_matches_plain_path(gctx, orc):
    w = synth.workload_cfg1(n_s=400, n_layers=30)
    geom = rbfdef.rbf_geom_create(gctx, to_dev(w.xs), to_dev(w.xv), to_dev(w.dwall))
    dv = torch.zeros((2, w.n_v), dtype=torch.float64, device="cuda:0")
    r = _submit(gctx, geom, w, dv, want_ctrl=True)
    info = rbfdef.rbf_wait(gctx, r)
    assert info.state == rbfdef.REQ_DONE and info.result >= 0
    assert info.t_arrive <= info.t_admit <= info.t_start <= info.t_done
    ref = orc.greedy(2, w.xs, w.ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(), seeds=w.seeds)
    cs = r.out
    assert np.array_equal(cs.ctrl_idx[: cs.total].cpu().numpy(), ref.ctrl_idx)
    D = [w.D] * w.n_levels
    xc = w.xs[:, ref.ctrl_idx]
    ref_dv = orc.volume(w.radius, D, ref.level_off, xc, ref.alpha, w.xv, w.dwall)
    scale = np.sqrt((ref_dv ** 2).sum(0)).max()
    S = sum_magnitude(orc, w.radius, ref.level_off, xc, ref.alpha, w.xv, w.dwall, D)
    got = dv.cpu().numpy()
    err = np.sqrt(((got - ref_dv) ** 2).sum(0)).max()
    print(f"resident volume error {err:.3e} (bound {fp64_bound(scale, S):.3e})")
    check_fp64(err, scale, S)
    assert np.all(got[:, w.dwall >= w.D] == 0.0)
    rbfdef.rbf_geom_release(gctx, geom)


def test_device_wall_distance(gctx, orc):
    """A geometry created without wall distances computes them on the device (nearest surface
    point); the deformation matches the one with the host-computed distances."""
    w = synth.workload_cfg0(n_s=160, n_layers=12)
    g1 = rbfdef.rbf_geom_create(gctx, to_dev(w.xs), to_dev(w.xv), to_dev(w.dwall))
    g2 = rbfdef.rbf_geom_create(gctx, to_dev(w.xs), to_dev(w.xv), None)
    d1 = torch.zeros((2, w.n_v), dtype=torch.float64, device="cuda:0")
    d2 = torch.zeros_like(d1)
    r1 = _submit(gctx, g1, w, d1, want_ctrl=True)
    rbfdef.rbf_wait(gctx, r1)
    rbfdef.rbf_wait(gctx, _submit(gctx, g2, w, d2))
    cs = r1.out
    xc = cs.xc[:, : cs.total].cpu().numpy()
    a = cs.alpha[:, : cs.total].cpu().numpy()
    S = sum_magnitude(orc, w.radius, cs.level_off, xc, a, w.xv, w.dwall, [w.D])
    ref = d1.cpu().numpy()
    scale = np.sqrt((ref ** 2).sum(0)).max()
    err = np.sqrt(((d2.cpu().numpy() - ref) ** 2).sum(0)).max()
    print(f"device wall distance: difference {err:.3e} (bound {fp64_bound(scale, S):.3e})")
    check_fp64(err, scale, S)
    rbfdef.rbf_geom_release(gctx, g1)
    rbfdef.rbf_geom_release(gctx, g2)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_same_alone_and_in_the_mix(gctx, precision):
    ws = _requests(7)
    geoms = [rbfdef.rbf_geom_create(gctx, to_dev(w.xs), to_dev(w.xv), to_dev(w.dwall)) for w in ws]
    alone = []
    for w, g in zip(ws, geoms):
        dv = torch.zeros((w.dim, w.n_v), dtype=torch.float64, device="cuda:0")
        info = rbfdef.rbf_wait(gctx, _submit(gctx, g, w, dv, precision))
        assert info.state == rbfdef.REQ_DONE, info.result
        alone.append(dv.clone())
    outs, reqs = [], []
    for w, g in zip(ws, geoms):
        dv = torch.full((w.dim, w.n_v), float("nan"), dtype=torch.float64, device="cuda:0")
        outs.append(dv)
        reqs.append(_submit(gctx, g, w, dv, precision))
    for r in reqs:
        info = rbfdef.rbf_wait(gctx, r)
        assert info.state == rbfdef.REQ_DONE, info.result
    for a, b in zip(alone, outs):
        assert torch.equal(a, b)
    for g in geoms:
        rbfdef.rbf_geom_release(gctx, g)


def test_warm_start_equals_seeded_oracle(gctx, orc):
    """Two icing steps on one geometry: the second, warm-started, equals the oracle's greedy
    with the first step's control sets as per-level seeds."""
    w = synth.workload_cfg1(n_s=300, n_layers=10)
    geom = rbfdef.rbf_geom_create(gctx, to_dev(w.xs), to_dev(w.xv), to_dev(w.dwall))
    dv = torch.zeros((2, w.n_v), dtype=torch.float64, device="cuda:0")
    r1 = _submit(gctx, geom, w, dv, want_ctrl=True)
    rbfdef.rbf_wait(gctx, r1)
    ref1 = orc.greedy(2, w.xs, w.ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(), seeds=w.seeds)
    assert np.array_equal(r1.out.ctrl_idx[: r1.out.total].cpu().numpy(), ref1.ctrl_idx)
    ds2 = 1.5 * w.ds
    seeds = [list(ref1.level(l)[0]) for l in range(ref1.n_levels_used)]
    seeds += [[] for _ in range(w.n_levels - len(seeds))]
    w2 = synth.Workload(w.name + "_step2", 2, w.xs, np.ascontiguousarray(ds2), w.xv, w.dwall, w.radius,
                        w.eps, w.rho, w.D, w.cap, w.seeds)
    if ref1.n_levels_used != w.n_levels:
        pytest.skip("first step did not use every level")
    r2 = _submit(gctx, geom, w2, dv, warm=True, want_ctrl=True)
    info = rbfdef.rbf_wait(gctx, r2)
    assert info.state == rbfdef.REQ_DONE
    ref2 = orc.greedy(2, w.xs, ds2, w.radius, w.eps, rho=w.rho, cap=w.cap_total(), seeds=seeds)
    got = r2.out.ctrl_idx[: r2.out.total].cpu().numpy()
    assert np.array_equal(got, ref2.ctrl_idx)
    rbfdef.rbf_geom_release(gctx, geom)


def test_admission_under_small_budget(orc):
    """A context whose budget holds one request at a time still completes every request, and a
    request that can never fit is refused at submit."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = rbfdef.rbf_ctx_create(0, 100 << 20)
    try:
        ws = [synth.workload_cfg0(n_s=400, n_layers=8) for _ in range(3)]
        for w in ws:
            w.eps = 1e-4
        geoms = [rbfdef.rbf_geom_create(ctx, to_dev(w.xs), to_dev(w.xv), to_dev(w.dwall)) for w in ws]
        dvs = [torch.zeros((2, w.n_v), dtype=torch.float64, device="cuda:0") for w in ws]
        reqs = [_submit(ctx, g, w, dv) for g, w, dv in zip(geoms, ws, dvs)]
        infos = [rbfdef.rbf_wait(ctx, r) for r in reqs]
        assert all(i.state == rbfdef.REQ_DONE for i in infos)
        assert torch.equal(dvs[0], dvs[1]) and torch.equal(dvs[1], dvs[2])
        big = synth.workload_cfg1(n_s=6000, n_layers=4)
        gb = rbfdef.rbf_geom_create(ctx, to_dev(big.xs), to_dev(big.xv), to_dev(big.dwall))
        with pytest.raises(rbfdef.RbfError) as e:
            _submit(ctx, gb, big, torch.zeros((2, big.n_v), dtype=torch.float64, device="cuda:0"))
        assert e.value.status == rbfdef.RBF_E_NOMEM
    finally:
        rbfdef.rbf_ctx_destroy(ctx)


def test_bad_handles(gctx):
    class Fake:
        ticket = 987654321
    with pytest.raises(rbfdef.RbfError) as e:
        rbfdef.rbf_poll(gctx, Fake())
    assert e.value.status == rbfdef.RBF_E_NOT_FOUND
    with pytest.raises(rbfdef.RbfError) as e:
        rbfdef.rbf_geom_release(gctx, 12345)
    assert e.value.status == rbfdef.RBF_E_NOT_FOUND


def test_geom_volume_update_matches_oracle(gctx, orc):
    """The resident-geometry volume update equals the oracle's volume update for given control
    sets (per-level D, ragged sizes, 3D)."""
    w = synth.random_workload(77, 3, 500, 9001, [1.5, 0.6], 1e-7)
    ref = orc.greedy(3, w.xs, w.ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(), seeds=w.seeds)
    xc = np.ascontiguousarray(w.xs[:, ref.ctrl_idx])
    D = [0.9, 0.45]
    geom = rbfdef.rbf_geom_create(gctx, to_dev(w.xs), to_dev(w.xv), to_dev(w.dwall))
    dv = torch.full((3, w.n_v), float("nan"), dtype=torch.float64, device="cuda:0")
    rbfdef.rbf_geom_volume_update(gctx, geom, w.radius, D, list(ref.level_off), to_dev(xc),
                                  to_dev(ref.alpha), dv)
    torch.cuda.synchronize()
    got = dv.cpu().numpy()
    want = orc.volume(w.radius, D, ref.level_off, xc, ref.alpha, w.xv, w.dwall)
    scale = np.sqrt((want ** 2).sum(0)).max()
    S = sum_magnitude(orc, w.radius, ref.level_off, xc, ref.alpha, w.xv, w.dwall, D)
    err = np.sqrt(((got - want) ** 2).sum(0)).max()
    check_fp64(err, scale, S)
    far = w.dwall >= max(D)
    assert np.all(got[:, far] == 0.0) and not np.any(np.signbit(got[:, far]))
    rbfdef.rbf_geom_release(gctx, geom)


def test_warm_start_reuses_resident_basis(gctx):
    """Three icing steps on one geometry with warm start: the steps after the first reuse the
    resident Newton bases. A fresh geometry given the same sequence (first cold, then warm) gives
    the same control sets and bit-identical displacements (the reuse is exact)."""
    w = synth.workload_cfg1(n_s=600, n_layers=8)
    runs = []
    for rep in range(2):
        geom = rbfdef.rbf_geom_create(gctx, to_dev(w.xs), to_dev(w.xv), to_dev(w.dwall))
        outs = []
        for step in range(3):
            ws = synth.Workload(w.name, 2, w.xs, np.ascontiguousarray((1.0 + 0.3 * step) * w.ds), w.xv,
                                w.dwall, w.radius, w.eps, w.rho, w.D, w.cap, w.seeds)
            dv = torch.zeros((2, w.n_v), dtype=torch.float64, device="cuda:0")
            r = _submit(gctx, geom, ws, dv, warm=step > 0, want_ctrl=True)
            info = rbfdef.rbf_wait(gctx, r)
            assert info.state == rbfdef.REQ_DONE, info.result
            outs.append((r.out.ctrl_idx[: r.out.total].cpu().numpy(), dv.clone()))
        runs.append(outs)
        rbfdef.rbf_geom_release(gctx, geom)
    for (c1, d1), (c2, d2) in zip(*runs):
        assert np.array_equal(c1, c2)
        assert torch.equal(d1, d2)
    # warm steps keep the earlier control points as their first ones
    assert np.array_equal(runs[0][1][0][: len(runs[0][0][0])][:5], runs[0][0][0][:5])


def test_adaptive_support_distance(gctx, orc):
    """Section 4's volume reduction with D_l = k (dS_l)^max (k = 5) per level: the serving path
    derives D_l from the greedy's level maxima (equal to the oracle's within k times the FP64
    residual bound); the result equals the oracle's volume update given those D_l, and every point
    at or beyond max_l D_l is +0.0."""
    import oracle as oracle_mod

    w = synth.workload_cfg1(n_s=500, n_layers=40)
    geom = rbfdef.rbf_geom_create(gctx, to_dev(w.xs), to_dev(w.xv), to_dev(w.dwall))
    dv = torch.full((2, w.n_v), float("nan"), dtype=torch.float64, device="cuda:0")
    r = rbfdef.rbf_submit(gctx, geom, to_dev(w.ds), dv, w.radius, w.eps, [1.0] * w.n_levels, rho=w.rho,
                          cap=w.cap_total(), seeds=w.seeds, precision="fp64", want_ctrl=True, d_factor=5.0)
    info = rbfdef.rbf_wait(gctx, r)
    assert info.state == rbfdef.REQ_DONE, info.result
    ref = orc.greedy(2, w.xs, w.ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(), seeds=w.seeds)
    cs = r.out
    assert np.array_equal(cs.ctrl_idx[: cs.total].cpu().numpy(), ref.ctrl_idx)
    D_ref = oracle_mod.support_distances(5.0, w.ds, ref)
    D = cs.support_distances(5.0)
    print(f"D_l oracle {D_ref} device {D}")
    assert all(t > 0 for t in cs.level_seconds[: cs.n_levels_used])
    xc = w.xs[:, ref.ctrl_idx]
    used = ref.n_levels_used
    S_surf = sum_magnitude(orc, w.radius[:used], ref.level_off[: used + 1], xc, ref.alpha, w.xs)
    tol = 5.0 * fp64_bound(np.sqrt((w.ds ** 2).sum(0)).max(), S_surf)
    assert len(D) == used and np.all(np.abs(np.array(D) - D_ref) <= tol)
    want = orc.volume(w.radius[:used], D, ref.level_off[: used + 1], xc, ref.alpha, w.xv, w.dwall)
    got = dv.cpu().numpy()
    scale = np.sqrt((want ** 2).sum(0)).max()
    S = sum_magnitude(orc, w.radius[:used], ref.level_off[: used + 1], xc, ref.alpha, w.xv, w.dwall, D)
    err = np.sqrt(((got - want) ** 2).sum(0)).max()
    print(f"adaptive-D volume error {err:.3e} (bound {fp64_bound(scale, S):.3e}); "
          f"points per level {[int((w.dwall < d).sum()) for d in D]} of {w.n_v}")
    check_fp64(err, scale, S)
    far = w.dwall >= max(D)
    assert np.all(got[:, far] == 0.0) and not np.any(np.signbit(got[:, far]))
    rbfdef.rbf_geom_release(gctx, geom)

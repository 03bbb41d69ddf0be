"""GPU parity of the volume update (eqs. (19), (23)) and the interpolant evaluation (eq. (1))
against the FP64 oracle, through the C ABI.

Tolerances (tests/helpers.py): the FP64 path within 1e-10 of the result's scale plus the stated
forward-error bound 2 (gamma_n S + eps_phi A) of two FP64 evaluations of the same sums (S the
magnitude of the summed terms, A that of the weights in support, eps_phi the basis value's own
error, with the one-step root of the volume sums); the measured difference is printed in units
of u S. The mixed path (FP32 pair arithmetic, FP64 accumulation) is held to the same form with
u32 = 2^-24 for the pair part (mixed_bound). Points at or beyond every support distance D_l must
be +0.0 bit for bit. A call that fails after its compaction kernels are enqueued keeps its buffers
reserved until its stream has passed them.
"""
import numpy as np
import pytest
import torch

import synth
from helpers import check_fp64, fp64_bound, mixed_bound, normwise, sum_magnitude, to_dev
from paper_2107_13887_amd import rbfdef

pytestmark = pytest.mark.gpu


def _controls(orc, w):
    res = orc.greedy(w.dim, w.xs, w.ds, w.radius, w.eps, rho=w.rho, cap=w.cap_total(), seeds=w.seeds)
    return res, np.ascontiguousarray(w.xs[:, res.ctrl_idx])


def _assert_fp64(orc, w, res, xc, D, got, ref, xv, dwall):
    scale = np.sqrt((ref ** 2).sum(0)).max()
    S = sum_magnitude(orc, w.radius, res.level_off, xc, res.alpha, xv, dwall, D)
    err = np.sqrt(((got - ref) ** 2).sum(0)).max()
    print(f"volume error {err:.3e} = {err / scale:.3e} normwise (bound {fp64_bound(scale, S):.3e})")
    check_fp64(err, scale, S)


def _run(gctx, w, res, xc, D, precision="fp64", xv=None, dwall=None):
    xv = w.xv if xv is None else xv
    dwall = w.dwall if dwall is None else dwall
    print(f"case {w.name} n_v={xv.shape[1]} n_c={xc.shape[1]} D={D} {precision}", flush=True)
    dv = rbfdef.rbf_volume_update(gctx, w.radius, D, list(res.level_off), to_dev(xc), to_dev(res.alpha),
                                  to_dev(xv), to_dev(dwall), precision=precision)
    torch.cuda.synchronize()
    return dv.cpu().numpy()


@pytest.mark.parametrize("dim,n_s,n_v,radius,D", [
    (2, 300, 5000, [1.5], [0.9]),
    (3, 350, 7001, [1.5, 0.6], [0.9, 0.5]),          # ragged size, per-level D
    (3, 700, 3333, [2.0, 0.8, 0.3], [1.2, 1.2, 1.2]),  # controls span several LDS tiles
    (2, 64, 17, [1.0], [2.5]),                        # fewer points than one workgroup
])
def test_volume_fp64_matches_oracle(gctx, orc, dim, n_s, n_v, radius, D):
    w = synth.random_workload(20 + n_s, dim, n_s, n_v, radius, 1e-7)
    res, xc = _controls(orc, w)
    ref = orc.volume(w.radius, D, res.level_off, xc, res.alpha, w.xv, w.dwall)
    got = _run(gctx, w, res, xc, D)
    _assert_fp64(orc, w, res, xc, D, got, ref, w.xv, w.dwall)
    far = w.dwall >= max(D)
    assert np.all(got[:, far] == 0.0) and not np.any(np.signbit(got[:, far]))


def test_volume_zero_exactly_at_D(gctx, orc):
    w = synth.random_workload(31, 3, 200, 4000, [1.0], 1e-7)
    res, xc = _controls(orc, w)
    dwall = w.dwall.copy()
    dwall[::7] = 0.5                      # exactly at D
    got = _run(gctx, w, res, xc, [0.5], dwall=dwall)
    ref = orc.volume(w.radius, [0.5], res.level_off, xc, res.alpha, w.xv, dwall)
    assert np.array_equal(got == 0.0, ref == 0.0)
    assert np.all(got[:, dwall >= 0.5] == 0.0)
    _assert_fp64(orc, w, res, xc, [0.5], got, ref, w.xv, dwall)


def test_volume_empty_level_and_no_points(gctx, orc):
    w = synth.random_workload(32, 2, 120, 1000, [1.0, 0.5], 1e-7)
    res, xc = _controls(orc, w)
    off = [0, int(res.level_off[1]), int(res.level_off[1])]   # second level empty
    a = np.ascontiguousarray(res.alpha[:, : off[1]])
    c = np.ascontiguousarray(xc[:, : off[1]])
    dv = rbfdef.rbf_volume_update(gctx, w.radius, [0.8, 0.8], off, to_dev(c), to_dev(a), to_dev(w.xv),
                                  to_dev(w.dwall))
    torch.cuda.synchronize()
    ref = orc.volume(w.radius, [0.8, 0.8], off, c, a, w.xv, w.dwall)
    assert normwise(dv.cpu().numpy(), ref) <= 1e-9
    empty = torch.zeros((2, 0), dtype=torch.float64, device="cuda:0")
    rbfdef.rbf_volume_update(gctx, w.radius, [0.8, 0.8], off, to_dev(c), to_dev(a), empty,
                             torch.zeros(0, dtype=torch.float64, device="cuda:0"), dv=empty)
    torch.cuda.synchronize()


def test_volume_rejects_bad_arguments(gctx):
    x = torch.zeros((3, 10), dtype=torch.float64, device="cuda:0")
    d = torch.zeros(10, dtype=torch.float64, device="cuda:0")
    with pytest.raises(rbfdef.RbfError) as e:
        rbfdef.rbf_volume_update(gctx, [1.0], [-1.0], [0, 10], x, x, x, d)
    assert e.value.status == rbfdef.RBF_E_INVALID
    with pytest.raises(rbfdef.RbfError):
        rbfdef.rbf_volume_update(gctx, [0.0], [1.0], [0, 10], x, x, x, d)
    with pytest.raises(ValueError):
        rbfdef.rbf_volume_update(gctx, [1.0], [1.0], [0, 11], x, x, x, d)


@pytest.mark.parametrize("dim", [2, 3])
def test_volume_mixed_precision(gctx, orc, dim):
    w = synth.random_workload(40 + dim, dim, 400, 6000, [1.5, 0.5], 1e-6)
    res, xc = _controls(orc, w)
    D = [0.9, 0.9]
    ref = orc.volume(w.radius, D, res.level_off, xc, res.alpha, w.xv, w.dwall)
    got = _run(gctx, w, res, xc, D, precision="mixed")
    scale = np.sqrt((ref ** 2).sum(0)).max()
    S = sum_magnitude(orc, w.radius, res.level_off, xc, res.alpha, w.xv, w.dwall, D)
    err = np.sqrt(((got - ref) ** 2).sum(0)).max()
    bound = mixed_bound(scale, S)
    print(f"mixed error {err:.3e} = {err / scale:.3e} normwise, S/scale {S / scale:.1f}, bound {bound:.3e}")
    assert err <= bound
    far = w.dwall >= max(D)
    assert np.all(got[:, far] == 0.0)


@pytest.mark.parametrize("cfg", [0, 1])
def test_volume_airfoil_configs(gctx, orc, cfg):
    """Full-size 2D configurations: oracle control sets, GPU volume update, every point checked."""
    w = synth.workload(cfg)
    res, xc = _controls(orc, w)
    D = [w.D] * w.n_levels
    ref = orc.volume(w.radius, D, res.level_off, xc, res.alpha, w.xv, w.dwall)
    got = _run(gctx, w, res, xc, D)
    scale = np.sqrt((ref ** 2).sum(0)).max()
    S = sum_magnitude(orc, w.radius, res.level_off, xc, res.alpha, w.xv, w.dwall, D)
    err = np.sqrt(((got - ref) ** 2).sum(0)).max()
    print(f"volume error {err:.3e} = {err / scale:.3e} normwise (bound {fp64_bound(scale, S):.3e})")
    check_fp64(err, scale, S)
    assert np.all(got[:, w.dwall >= w.D] == 0.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_evaluate_matches_oracle(gctx, orc, dim):
    rng = np.random.default_rng(50 + dim)
    xc = rng.uniform(-1, 1, (dim, 300))
    alpha = rng.uniform(-1, 1, (dim, 300))
    xp = rng.uniform(-1.5, 1.5, (dim, 2001))
    ref = orc.evaluate(0.7, xc, alpha, xp)
    out = rbfdef.rbf_evaluate(gctx, 0.7, to_dev(xc), to_dev(alpha), to_dev(xp))
    base = rng.uniform(-1, 1, (dim, 2001))
    res = rbfdef.rbf_evaluate(gctx, 0.7, to_dev(xc), to_dev(alpha), to_dev(xp), base=to_dev(base), sign=1.0)
    torch.cuda.synchronize()
    assert normwise(out.cpu().numpy(), ref) <= 1e-12
    assert np.abs(res.cpu().numpy() - (base - ref)).max() <= 1e-12 * np.abs(ref).max()


def test_binding_uses_the_current_stream():
    """The binding enqueues on torch's current stream, default or not."""
    assert rbfdef._stream(None) == torch.cuda.current_stream().cuda_stream
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        assert rbfdef._stream(None) == s.cuda_stream == torch.cuda.current_stream().cuda_stream
    assert rbfdef._stream(s) == s.cuda_stream


def test_failed_call_keeps_its_buffers_until_its_kernels_end(gctx):
    """A plain volume update that fails (forced: RBF_KSUM_FAIL_AFTER_COMPACTION) after its
    compaction kernels are enqueued returns RBF_E_NOMEM and hands its buffers back to the pool only
    once its stream has passed them. A call of the same sizes issued right after it on another
    stream, which would otherwise be given those blocks while the failed call's kernels still write
    them, returns the same bits as alone."""
    rng = np.random.default_rng(11)
    n_v, n_c = 3_000_000, 600
    xv = torch.from_numpy(rng.uniform(-1.0, 1.0, (3, n_v))).to("cuda:0")
    dwall = torch.from_numpy(rng.uniform(0.0, 1.0, n_v)).to("cuda:0")
    xc = torch.from_numpy(rng.uniform(-1.0, 1.0, (3, n_c))).to("cuda:0")
    al = torch.from_numpy(rng.uniform(-1e-3, 1e-3, (3, n_c))).to("cuda:0")
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    dv_a = torch.empty((3, n_v), dtype=torch.float64, device="cuda:0")   # alive until the end: the
    # failed call's compaction still writes its zeros there after the call has returned
    call = lambda D, st, dv=None: rbfdef.rbf_volume_update(gctx, [0.3], [D], [0, n_c], xc, al, xv, dwall, dv=dv,
                                                           stream=st)
    ref = call(0.6, sb)
    torch.cuda.synchronize()
    for rep in range(4):
        print(f"case failed call then another, repetition {rep}", flush=True)
        import os
        os.environ["RBF_KSUM_FAIL_AFTER_COMPACTION"] = "1"
        try:
            with pytest.raises(rbfdef.RbfError) as e:
                call(0.2, sa, dv_a)
        finally:
            del os.environ["RBF_KSUM_FAIL_AFTER_COMPACTION"]
        assert e.value.status == rbfdef.RBF_E_NOMEM
        got = call(0.6, sb)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)

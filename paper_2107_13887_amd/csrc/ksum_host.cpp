// Host planner of the kernel sums (ksum.hip): per-call volume reduction, launch shape (points per
// lane, control-list splits), the resident geometry's row-group order, timers and the
// evaluated-pair counter.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "ksum.h"

namespace rbf {

using namespace ksum;

namespace {

// Launch-shape overrides, read once per process (0: not set).
struct ShapeEnv {
    int P, blocks, max_split, split;
    ShapeEnv()
    {
        auto get = [](const char *name) {
            const char *v = getenv(name);
            return v && *v ? atoi(v) : 0;
        };
        P = get("RBF_KSUM_P");
        blocks = get("RBF_KSUM_BLOCKS");
        max_split = get("RBF_KSUM_MAX_SPLIT");
        split = get("RBF_KSUM_SPLIT");
    }
};

const ShapeEnv &shape_env()
{
    static const ShapeEnv e;
    return e;
}

}  // namespace

rbf_status run_kernel_sum(rbf_ctx ctx, const SumProblem &pb, hipStream_t s, const SumScratch *ext)
{
    const int DIM = pb.dim;
    if (pb.n_p == 0) return RBF_OK;
    KArgs a{};
    a.n_live = -1;
    a.n_levels = pb.n_levels;
    int64_t nc_max = 0;
    double dmax = 0.0, dmin = HUGE_VAL;
    for (int l = 0; l < pb.n_levels; ++l) {
        a.lv[l] = pb.lv[l];
        nc_max = std::max<int64_t>(nc_max, pb.lv[l].c_end - pb.lv[l].c_begin);
        dmax = std::max(dmax, pb.lv[l].D);
        if (pb.lv[l].c_end > pb.lv[l].c_begin) dmin = std::min(dmin, pb.lv[l].D);
    }
    a.xc = pb.xc;
    a.alpha = pb.alpha;
    a.ld_ctrl = pb.ld_ctrl;
    a.xp = pb.xp;
    a.ld_p = pb.n_p;
    a.dwall = pb.dwall;
    a.base = pb.base;
    a.sign = pb.sign;
    a.out = pb.out;
    a.ld_out = pb.ld_out ? pb.ld_out : pb.n_p;
    a.n_work = pb.n_p;

    DevBuf work, nwork, partial, counts;
    // Scratch from the pool, or carved in 256-byte steps from the caller's fixed area (the
    // allocation-free entry point: then no pool, no timer events, no pair counter).
    char *ext_at = ext ? static_cast<char *>(ext->base) : nullptr;
    size_t ext_left = ext ? ext->bytes : 0;
    auto carve = [&](size_t bytes) -> void * {
        const size_t b = (bytes + 255) & ~size_t(255);
        if (b > ext_left) return nullptr;
        void *p = ext_at;
        ext_at += b;
        ext_left -= b;
        return p;
    };
    int64_t n_rows = pb.n_p;    // rows the kernel-sum grid covers
    if (pb.dwall && pb.n_active >= 0) {
        // Resident geometry: results go out through perm. The grid covers every point; the
        // workgroups past the reduced prefix only write +0.0, so no separate zero-fill is
        // launched.
        a.out_perm = pb.perm;
        a.n_live = pb.n_active;
        a.block_box = pb.block_box;
    } else if (pb.dwall) {
        const int64_t nb = (pb.n_p + CBLK - 1) / CBLK;
        int64_t *nw = nullptr;
        int32_t *wk = nullptr, *cn = nullptr;
        if (ext) {
            nw = static_cast<int64_t *>(carve(sizeof(int64_t)));
            wk = static_cast<int32_t *>(carve(sizeof(int32_t) * pb.n_p));
            cn = static_cast<int32_t *>(carve(sizeof(int32_t) * nb));
            if (!nw || !wk || !cn)
                return fail(RBF_E_INVALID, "%lld points need more than the %llu bytes of fixed scratch",
                            (long long)pb.n_p, (unsigned long long)ext->bytes);
        } else {
            RBF_TRY(nwork.get(ctx->pool.get(), sizeof(int64_t), s));
            RBF_TRY(work.get(ctx->pool.get(), sizeof(int32_t) * pb.n_p, s));
            RBF_TRY(counts.get(ctx->pool.get(), sizeof(int32_t) * nb, s));
            nw = nwork.as<int64_t>();
            wk = work.as<int32_t>();
            cn = counts.as<int32_t>();
        }
        launch_reduce(pb.dwall, pb.n_p, dmax, cn, nw, wk, pb.out, DIM, s);
        RBF_HIP(hipGetLastError());
        // RBF_KSUM_FAIL_AFTER_COMPACTION=1 fails the call here, with its compaction kernels
        // enqueued (tests: its buffers must stay reserved until its stream has passed them).
        if (const char *e = getenv("RBF_KSUM_FAIL_AFTER_COMPACTION"); e && atoi(e) && !ext)
            return fail(RBF_E_NOMEM, "failure forced after the compaction (RBF_KSUM_FAIL_AFTER_COMPACTION)");
        a.work = wk;
        a.n_work_dev = nw;
    }

    // Launch shape: P points per lane; split the control lists when there are too few blocks.
    // The FP32 pair form is compiled in when some level asks for it.
    bool mixed = false;
    for (int l = 0; l < pb.n_levels; ++l) mixed |= pb.lv[l].fp32 != 0;
    // Two points per lane share every control read from LDS; one point per lane gives twice the
    // workgroups, which balances better when there are few blocks (the cost of a block varies
    // with the number of controls near it), and waves of half the rows, of which fewer straddle a
    // level's support distance when the levels' distances differ (a wave that needs a level
    // computes all its rows for it, psi = 0 on those beyond).
    const ShapeEnv &env = shape_env();
    const bool uneven_d = pb.dwall && dmax > 2.0 * dmin;
    int P = env.P ? env.P : (n_rows < (int64_t)8 * ctx->n_cu * VBLOCK || uneven_d ? 1 : 2);
    if (P != 1 && P != 2) P = 2;
    const int64_t nbx = (n_rows + (int64_t)BLOCK * P - 1) / ((int64_t)BLOCK * P);
    const int64_t target = env.blocks > 0 ? env.blocks : (int64_t)8 * ctx->n_cu;
    // Split only while every split keeps at least 128 controls: a split re-reads the points and
    // writes partial sums, which pays only when it turns a ragged last round of waves into many.
    int S = (int)std::max<int64_t>(1, std::min<int64_t>((target + nbx - 1) / nbx, nc_max / 128));
    S = std::min(S, env.max_split > 0 ? env.max_split : 64);
    if (env.split > 0) S = env.split;
    // Fixed scratch: fewer splits while their partial sums do not fit (one split needs none).
    while (ext && S > 1 && sizeof(double) * (size_t)S * DIM * n_rows + 255 > ext_left) --S;
    a.n_split = S;
    // Resident geometry: workgroups take the row groups heaviest first, dealt across the compute
    // units (RBF_KSUM_ORDER=0: stored order).
    if (pb.geom) {
        const char *e = getenv("RBF_KSUM_ORDER");
        if (!(e && e[0] == '0')) RBF_TRY(resident_order(ctx, *pb.geom, pb, P, nbx, s, &a.order));
    }
    if (S > 1) {
        if (ext) {
            a.partial = static_cast<double *>(carve(sizeof(double) * (size_t)S * DIM * n_rows));
        } else {
            RBF_TRY(partial.get(ctx->pool.get(), sizeof(double) * (size_t)S * DIM * n_rows, s));
            a.partial = partial.as<double>();
        }
        a.ld_part = n_rows;
    }
    const dim3 grid((unsigned)nbx, (unsigned)S);
    const char *name = pb.dwall ? (mixed ? "volume_ksum_mixed" : "volume_ksum_fp64")
                                : (mixed ? "surface_ksum_mixed" : "surface_ksum_fp64");
    a.pairs = ext ? nullptr : ctx->timers.counter(name);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (!ext) ctx->timers.pair(&t0, &t1);
    launch_sum(a, grid, DIM, P, mixed, pb.basis, s, t0, t1);
    RBF_HIP(hipGetLastError());
    ctx->timers.add(name, t0, t1);
    if (S > 1) {
        const int gf = (int)std::min<int64_t>((n_rows + BLOCK - 1) / BLOCK, 8192);
        launch_finalize(a, DIM, gf, s);
        RBF_HIP(hipGetLastError());
    }
    work.release_after(s);
    counts.release_after(s);
    nwork.release_after(s);
    partial.release_after(s);
    return RBF_OK;
}

}  // namespace rbf

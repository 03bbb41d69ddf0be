// Wendland kernel sums (Table 1) on gfx950: the volume update of eqs. (19)/(23) and the surface
// interpolant/residual of eqs. (1)/(12).
//
//   out_k(p) = base_k(p) - sign * sum_l psi(d_p / D_l) sum_{c in level l} phi(||x_p - x_c|| / R_l) alpha_k,c
//
// Design (VALU-bound: about 21 vector slots per point/control pair in 2D, 24 in 3D, three fewer
// in the volume sums, against 40-56 bytes of HBM traffic per point):
//   * points stream as SoA, P points per lane, 256 lanes per workgroup, each wave on 64 P
//     consecutive stored points;
//   * the controls of each level are staged through LDS in tiles of 256, scaled by 1/R_l while
//     they are loaded (coalesced over the control index); every lane of a wave then reads the
//     same LDS address, a broadcast without bank conflicts;
//   * the control list of each level may be split over gridDim.y so that few points still give
//     enough waves; split partial sums are reduced in a fixed order (deterministic results);
//   * compact support: each workgroup takes a bounding box of its points (on a resident geometry
//     the union of the stored boxes of its 64-row groups, otherwise the box of its points that
//     each support distance weights), and while a control tile is staged every control whose
//     distance to that box is at least R_l (with a relative margin of 1e-4) is dropped by a
//     stable in-tile compaction, so the pair loop runs over the controls that can reach the
//     workgroup only. Dropped pairs have phi = 0 exactly, the order of the kept ones is
//     unchanged, and each level's sum runs over all its tiles before psi is applied once, so the
//     sums equal the uncut ones bit for bit whatever the tiling;
//   * the wall-distance reduction keeps only points with d < max_l D_l: the prefix of a resident
//     volume stored in spatially compact blocks ordered by their smallest wall distance, or a
//     stable two-kernel compaction that also writes +0.0 to every dropped point;
//   * FP64 square root from the hardware reciprocal square-root estimate e refined by one
//     Goldschmidt step (error ~1.5 e^2, at most ~37 u): the volume sums stop there and form
//     t = 1 - eta directly from it (coordinates scaled by 2 / R, the polynomial in t); the
//     surface sums (the greedy's level residuals) add one Newton correction (error ~1.5 e^3);
//   * mixed precision: the pair arithmetic runs in FP32 on coordinates shifted to a per-workgroup
//     origin (the workgroup's first point), the basis value is widened and accumulated in FP64.
#include <hip/hip_ext.h>

#include "basis.h"
#include "ksum.h"

namespace rbf {
namespace ksum {
namespace {

// A control is dropped for a workgroup when its squared distance to the workgroup's box, in units
// of R_l, is at least (1 + 1e-4)^2: every pair it would form then has eta > 1 and phi = 0, with
// room for the rounding of the scaled coordinates (FP64, or FP32 on shifted coordinates).
constexpr double CULL2 = 1.00020001;

// a > 0 normal. y ~ a^-1/2 (1 + e), |e| <= 2^-24.2 (v_rsq_f64); g = a y, h = y / 2. One
// Goldschmidt step leaves g with relative error ~1.5 e^2 (at most ~37 u, u = 2^-53); the Newton
// correction with the unrefined h leaves ~1.5 e^3 (the result to about half an ulp).
__device__ __forceinline__ double sqrt_goldschmidt(double a)
{
    double y = __builtin_amdgcn_rsq(a);
    double g = a * y;
    double h = 0.5 * y;
    double r = __builtin_fma(-g, h, 0.5);
    g = __builtin_fma(g, r, g);
    double d = __builtin_fma(-g, g, a);
    return __builtin_fma(d, h, g);
}

// psi(xi) = 1 - xi on [0, 1), zero from xi = 1 on (Section 4), with xi = d / D as a true
// division so that d == D gives exactly zero.
__device__ __forceinline__ double psi_w(double d, double D)
{
    double xi = d / D;
    return xi >= 1.0 ? 0.0 : 1.0 - xi;
}

__device__ __forceinline__ void split_range(const SumLevel &L, int s, int S, int64_t &cb, int64_t &ce)
{
    if (S == 1) {
        cb = L.c_begin;
        ce = L.c_end;
        return;
    }
    int64_t nc = L.c_end - L.c_begin;
    cb = L.c_begin + (nc * s) / S;
    ce = L.c_begin + (nc * (s + 1)) / S;
}

// One pair in FP64: phi(|q - c|) for coordinates already scaled by 1/R (Table 1), the root to
// half an ulp.
// Every pair form below clamps t = 1 - eta with fmin(fmax(t, 0), 1), which the compiler folds into
// the clamp modifier of the instruction that forms t (t <= 1 always: eta >= 0), so the compact
// support costs no instruction of its own.
template <int DIM, int BASIS>
__device__ __forceinline__ double pair_f64(const double (&q)[DIM], const double *c)
{
    double d0 = q[0] - c[0];
    double r2 = __builtin_fma(d0, d0, 1e-200);   // keeps r2 > 0 so rsq stays finite at r = 0
#pragma unroll
    for (int k = 1; k < DIM; ++k) {
        double dk = q[k] - c[k];
        r2 = __builtin_fma(dk, dk, r2);
    }
    double eta = sqrt_goldschmidt(r2);
    double t = fmin(fmax(1.0 - eta, 0.0), 1.0);
    return wendland_t<BASIS, double>(eta, t);
}

// The volume sums' pair, on coordinates scaled by 2 / R: s = 4 eta^2 (+1e-200), y = rsq(s),
// G = s y = 2 eta (1 + e) and r = 1 - G y. One Goldschmidt step gives eta = G / 2 + G r / 4
// (relative error ~1.5 e^2, the first step of sqrt_goldschmidt), so t = 1 - eta = 1 + G (-1/2 - r / 4)
// comes out directly and the polynomial is taken in t: one issue slot fewer than forming eta.
template <int DIM, int BASIS>
__device__ __forceinline__ double pair_f64_t(const double (&q)[DIM], const double *c)
{
    double d0 = q[0] - c[0];
    double s = __builtin_fma(d0, d0, 1e-200);
#pragma unroll
    for (int k = 1; k < DIM; ++k) {
        double dk = q[k] - c[k];
        s = __builtin_fma(dk, dk, s);
    }
    const double y = __builtin_amdgcn_rsq(s);
    const double G = s * y;
    const double r = __builtin_fma(-G, y, 1.0);
    const double tc = fmin(fmax(__builtin_fma(G, __builtin_fma(r, -0.25, -0.5), 1.0), 0.0), 1.0);
    return wendland_tform<BASIS, double>(tc, tc);
}

template <int DIM, int BASIS>
__device__ __forceinline__ float pair_f32(const float (&q)[DIM], const float *c)
{
    float d0 = q[0] - c[0];
    float r2 = d0 * d0;
#pragma unroll
    for (int k = 1; k < DIM; ++k) {
        float dk = q[k] - c[k];
        r2 = __builtin_fmaf(dk, dk, r2);
    }
    float eta = __builtin_amdgcn_sqrtf(r2);
    float t = fminf(fmaxf(1.0f - eta, 0.0f), 1.0f);
    return wendland_t<BASIS, float>(eta, t);
}

// Adds phi * alpha over the staged controls [c0, c1) of level l (consecutive in the tile) to the
// level's running sum la, for the P points of this lane. A level's sum runs over its controls in
// stream order whatever the tiling, and culled controls only drop exact zeros, so every kernel
// here gives the same bits.
template <int DIM, int P, bool MIXED, int BASIS>
__device__ __forceinline__ void level_accum(const KArgs &a, int l, const double *tile, int c0, int c1,
                                            const double (&xq)[P][DIM], const double (&org)[DIM],
                                            double (&la)[P][DIM])
{
    constexpr int ST = 2 * DIM;
    constexpr int AOFF = DIM;
    const double inv_r = a.lv[l].inv_r;
    // Four independent pairs in flight per lane with one point per lane (small launches, where
    // the last waves of a compute unit run alone), two with two points per lane.
    constexpr int UNR = P == 1 ? 4 : 2;
    if (MIXED && a.lv[l].fp32) {
        float q32[P][DIM];
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int k = 0; k < DIM; ++k) q32[p][k] = (float)((xq[p][k] - org[k]) * inv_r);
#pragma unroll UNR
        for (int c = c0; c < c1; ++c) {
            const double *cc = tile + c * ST;
            double cal[DIM];
            float cpos[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                cal[k] = cc[AOFF + k];
                cpos[k] = reinterpret_cast<const float *>(cc)[k];
            }
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const double ph = (double)pair_f32<DIM, BASIS>(q32[p], cpos);
#pragma unroll
                for (int k = 0; k < DIM; ++k) la[p][k] = __builtin_fma(ph, cal[k], la[p][k]);
            }
        }
    } else {
        // Volume sums (psi applied) take coordinates scaled by 2 / R (pair_f64_t, the staged
        // controls likewise), surface sums by 1 / R.
        const double sc = a.dwall ? 2.0 * inv_r : inv_r;
        double q64[P][DIM];
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int k = 0; k < DIM; ++k) q64[p][k] = xq[p][k] * sc;
        if (a.dwall) {
            // Volume sums: the one-step root with t formed directly (pair_f64_t).
#pragma unroll UNR
            for (int c = c0; c < c1; ++c) {
                const double *cc = tile + c * ST;
                double cal[DIM], cpos[DIM];
#pragma unroll
                for (int k = 0; k < DIM; ++k) {
                    cal[k] = cc[AOFF + k];
                    cpos[k] = cc[k];
                }
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const double ph = pair_f64_t<DIM, BASIS>(q64[p], cpos);
#pragma unroll
                    for (int k = 0; k < DIM; ++k) la[p][k] = __builtin_fma(ph, cal[k], la[p][k]);
                }
            }
        } else {
            // Surface sums (the greedy's level residual, whose rounding can decide the next
            // level's argmax): the root to half an ulp.
#pragma unroll UNR
            for (int c = c0; c < c1; ++c) {
                const double *cc = tile + c * ST;
                double cal[DIM], cpos[DIM];
#pragma unroll
                for (int k = 0; k < DIM; ++k) {
                    cal[k] = cc[AOFF + k];
                    cpos[k] = cc[k];
                }
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const double ph = pair_f64<DIM, BASIS>(q64[p], cpos);
#pragma unroll
                    for (int k = 0; k < DIM; ++k) la[p][k] = __builtin_fma(ph, cal[k], la[p][k]);
                }
            }
        }
    }
}

// acc += psi(d / D_l) la for the finished level l (psi = 1 without wall distances); la = 0.
template <int DIM, int P>
__device__ __forceinline__ void level_flush(const KArgs &a, int l, const double (&dw)[P], double (&la)[P][DIM],
                                            double (&acc)[P][DIM])
{
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const double wgl = a.dwall ? psi_w(dw[p], a.lv[l].D) : 1.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            acc[p][k] = __builtin_fma(wgl, la[p][k], acc[p][k]);
            la[p][k] = 0.0;
        }
    }
}

// Final values (one split) or split partials of the P points of this lane.
template <int DIM, int P>
__device__ __forceinline__ void store_rows(const KArgs &a, int64_t rbase, int lane, const bool (&ok)[P],
                                           const int64_t (&oi)[P], const double (&acc)[P][DIM])
{
#pragma unroll
    for (int p = 0; p < P; ++p) {
        if (!ok[p]) continue;
        if (a.n_split == 1) {
            if (oi[p] < 0) continue;
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                const int64_t o = k * a.ld_out + oi[p];
                a.out[o] = a.base ? a.base[o] - a.sign * acc[p][k] : (-a.sign) * acc[p][k];
            }
        } else {
            const int64_t w = rbase + p * 64 + lane;
#pragma unroll
            for (int k = 0; k < DIM; ++k)
                a.partial[((int64_t)blockIdx.y * DIM + k) * a.ld_part + w] = acc[p][k];
        }
    }
}

template <int DIM, int P, bool MIXED, int BASIS>
__global__ __launch_bounds__(BLOCK) void ksum_kernel(KArgs a)
{
    // Per control in LDS: DIM scaled coordinates (FP64, or FP32 shifted ones in the first DIM
    // floats on FP32 levels) then DIM weights in FP64.
    constexpr int ST = 2 * DIM;                         // doubles per control in LDS
    constexpr int AOFF = DIM;                           // offset of the weights
    constexpr int NW = BLOCK / 64;                      // waves per workgroup
    constexpr int ML = RBF_MAX_LEVELS;
    __shared__ double tile[TILE * ST];
    __shared__ double origin[DIM];
    __shared__ double wbox[NW][2 * DIM];
    __shared__ double box[ML][2 * DIM];                 // per level: min[DIM], max[DIM]
    __shared__ int wcnt[NW];
    __shared__ int64_t vs[ML + 1], cb[ML];              // the workgroup's control stream (below)
    __shared__ double sbox[ML][2 * DIM];                // level boxes scaled by 1 / R_l
    __shared__ double s_inv_r[ML];
    __shared__ int wlc[NW][ML];                         // kept controls per wave and level
    __shared__ int seg[ML + 1];                         // level segments of the kept tile
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t n_work = a.n_work_dev ? *a.n_work_dev : a.n_work;
    const int64_t group = a.order ? (int64_t)a.order[blockIdx.x] : (int64_t)blockIdx.x;
    const int64_t wbase = group * (BLOCK * P);
    if (wbase >= n_work) return;
    const int split = blockIdx.y;
    // Rows from n_live on lie beyond every level's support (resident volume past its reduced
    // prefix): the workgroup only writes zeros.
    const bool live = a.n_live < 0 || wbase < a.n_live;

    // Point rows: wave v takes the 64 P consecutive rows from wbase + 64 P v, lane-contiguous for
    // each p, so a wave holds neighbouring points of the stored order. Every load of the point
    // data is issued here, once.
    int64_t idx[P], oi[P];
    bool ok[P];
    double dw[P], acc[P][DIM], xq[P][DIM];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int64_t w = wbase + (int64_t)wave * (64 * P) + p * 64 + lane;
        ok[p] = w < n_work;
        idx[p] = ok[p] ? (a.work ? (int64_t)a.work[w] : w) : 0;
        oi[p] = (ok[p] && a.out_perm) ? (int64_t)a.out_perm[idx[p]] : idx[p];
        dw[p] = (live && a.dwall && ok[p]) ? a.dwall[idx[p]] : 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            xq[p][k] = (live && ok[p]) ? a.xp[k * a.ld_p + idx[p]] : 0.0;
            acc[p][k] = 0.0;
        }
    }
    unsigned long long n_eval = 0;                      // pairs this wave evaluated

    if (live) {
        if (MIXED && tid == 0) {
            const int64_t i0 = a.work ? (int64_t)a.work[wbase] : wbase;
#pragma unroll
            for (int k = 0; k < DIM; ++k) origin[k] = a.xp[k * a.ld_p + i0];
        }
        int wave_pts = 0;                               // valid points of this wave
#pragma unroll
        for (int p = 0; p < P; ++p) wave_pts += __popcll(__ballot(ok[p]));

        // Per level: the box of the points it weights (psi > 0) and, per wave, whether any of its
        // points needs it. Levels sharing the support distance share the box.
        unsigned int wave_need = 0;
        if (a.block_box) {
            // Resident geometry: the stored boxes of the workgroup's rows (all their points) bound
            // every level's points, with no reduction; a level is used when some point of the wave
            // needs it.
            constexpr int NB = BLOCK * P / BOXROWS;     // stored boxes per workgroup
            const double *bb = a.block_box + (wbase / BOXROWS) * 2 * DIM;
            double bv = 0.0;
            if (tid < 2 * DIM) {
                const int k = tid % DIM;
                const bool lo = tid < DIM;
                bv = bb[tid];
#pragma unroll
                for (int j = 1; j < NB; ++j) {
                    const double v = bb[j * 2 * DIM + (lo ? k : DIM + k)];
                    bv = lo ? fmin(bv, v) : fmax(bv, v);
                }
            }
            for (int l = 0; l < a.n_levels; ++l) {
                bool need = false;
#pragma unroll
                for (int p = 0; p < P; ++p) need |= ok[p] && psi_w(dw[p], a.lv[l].D) > 0.0;
                if (__ballot(need) != 0ull) wave_need |= 1u << l;
                if (tid < 2 * DIM) box[l][tid] = bv;
            }
            if (lane == 0) wcnt[wave] = (int)wave_need;
            __syncthreads();
            unsigned int any = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) any |= (unsigned int)wcnt[w];
            // Levels no wave needs get an empty box (the control stream leaves them out).
            if (tid < a.n_levels * 2 * DIM) {
                const int l = tid / (2 * DIM), k = tid % (2 * DIM);
                if (!((any >> l) & 1u)) box[l][k] = k < DIM ? HUGE_VAL : -HUGE_VAL;
            }
        }
        for (int l = 0; l < (a.block_box ? 0 : a.n_levels); ++l) {
            const double dl = a.dwall ? a.lv[l].D : 0.0;
            if (l > 0 && dl == (a.dwall ? a.lv[l - 1].D : 0.0)) {
                wave_need |= ((wave_need >> (l - 1)) & 1u) << l;
                if (tid < 2 * DIM) box[l][tid] = box[l - 1][tid];
                continue;
            }
            double lo[DIM], hi[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                lo[k] = HUGE_VAL;
                hi[k] = -HUGE_VAL;
            }
            bool need = false;
#pragma unroll
            for (int p = 0; p < P; ++p)
                if (ok[p] && (!a.dwall || psi_w(dw[p], dl) > 0.0)) {
                    need = true;
#pragma unroll
                    for (int k = 0; k < DIM; ++k) {
                        lo[k] = fmin(lo[k], xq[p][k]);
                        hi[k] = fmax(hi[k], xq[p][k]);
                    }
                }
            if (__ballot(need) != 0ull) wave_need |= 1u << l;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1)
#pragma unroll
                for (int k = 0; k < DIM; ++k) {
                    lo[k] = fmin(lo[k], __shfl_xor(lo[k], off));
                    hi[k] = fmax(hi[k], __shfl_xor(hi[k], off));
                }
            __syncthreads();                            // earlier readers of wbox are done
            if (lane == 0)
#pragma unroll
                for (int k = 0; k < DIM; ++k) {
                    wbox[wave][k] = lo[k];
                    wbox[wave][DIM + k] = hi[k];
                }
            __syncthreads();
            if (tid < 2 * DIM) {
                double v = wbox[0][tid];
#pragma unroll
                for (int w = 1; w < NW; ++w) v = tid < DIM ? fmin(v, wbox[w][tid]) : fmax(v, wbox[w][tid]);
                box[l][tid] = v;
            }
        }
        __syncthreads();

        // This split's controls of every level the workgroup needs, as one stream in level
        // order: [vs[l], vs[l + 1]) holds level l's range starting at control cb[l].
        if (tid == 0) {
            vs[0] = 0;
            for (int l = 0; l < a.n_levels; ++l) {
                int64_t c0, c1;
                split_range(a.lv[l], split, a.n_split, c0, c1);
                cb[l] = c0;
                vs[l + 1] = vs[l] + (box[l][0] <= box[l][DIM] ? c1 - c0 : 0);
            }
        }
        if (tid < a.n_levels) s_inv_r[tid] = a.lv[tid].inv_r;
        if (tid < a.n_levels * 2 * DIM) {
            const int l = tid / (2 * DIM), k = tid % (2 * DIM);
            sbox[l][k] = box[l][k] * a.lv[l].inv_r;
        }
        __syncthreads();
        const int64_t total = vs[a.n_levels];
        double org[DIM], la[P][DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) org[k] = MIXED ? origin[k] : 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int k = 0; k < DIM; ++k) la[p][k] = 0.0;
        int open_l = -1;                                // level whose sum la holds

        for (int64_t v0 = 0; v0 < total; v0 += TILE) {
            const int nt = (int)min<int64_t>(TILE, total - v0);
            __syncthreads();
            // Stage the tile: keep the controls whose support reaches their level's box, in order.
            double xck[DIM], ack[DIM];
            bool keep = false;
            int lv_me = 0;
            if (tid < nt) {
                const int64_t v = v0 + tid;
                while (lv_me + 1 < a.n_levels && vs[lv_me + 1] <= v) ++lv_me;
                const int64_t c = cb[lv_me] + (v - vs[lv_me]);
#pragma unroll
                for (int k = 0; k < DIM; ++k) {
                    xck[k] = a.xc[k * a.ld_ctrl + c];
                    ack[k] = a.alpha[k * a.ld_ctrl + c];
                }
                const double inv_r = s_inv_r[lv_me];
                double g2 = 0.0;
#pragma unroll
                for (int k = 0; k < DIM; ++k) {
                    const double cs = xck[k] * inv_r;
                    const double gap = fmax(fmax(sbox[lv_me][k] - cs, cs - sbox[lv_me][DIM + k]), 0.0);
                    g2 = __builtin_fma(gap, gap, g2);
                }
                keep = g2 < CULL2;
            }
            const unsigned long long m = __ballot(keep);
            if (lane == 0) wcnt[wave] = __popcll(m);
            for (int l = 0; l < a.n_levels; ++l) {
                const unsigned long long ml = __ballot(keep && lv_me == l);
                if (lane == 0) wlc[wave][l] = __popcll(ml);
            }
            __syncthreads();
            if (tid == 0) {
                int run = 0;
                seg[0] = 0;
                for (int l = 0; l < a.n_levels; ++l) {
                    for (int w = 0; w < NW; ++w) run += wlc[w][l];
                    seg[l + 1] = run;
                }
            }
            int pos = __popcll(m & ((1ull << lane) - 1ull));
            int kept = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                pos += w < wave ? wcnt[w] : 0;
                kept += wcnt[w];
            }
            kept = __builtin_amdgcn_readfirstlane(kept);   // the same in every lane: a scalar loop bound
            if (keep) {
                double *dst = tile + pos * ST;
                const double inv_r = s_inv_r[lv_me];
                const bool f32 = MIXED && a.lv[lv_me].fp32;
#pragma unroll
                for (int k = 0; k < DIM; ++k) {
                    if (f32) reinterpret_cast<float *>(dst)[k] = (float)((xck[k] - origin[k]) * inv_r);
                    else dst[k] = xck[k] * (a.dwall ? 2.0 * inv_r : inv_r);
                }
#pragma unroll
                for (int k = 0; k < DIM; ++k) dst[AOFF + k] = ack[k];
            }
            __syncthreads();
            // The kept controls of one level are consecutive: one pair loop per level segment.
            for (int l = 0; l < a.n_levels; ++l) {
                const int c0 = __builtin_amdgcn_readfirstlane(seg[l]);
                const int c1 = __builtin_amdgcn_readfirstlane(seg[l + 1]);
                if (c1 > c0 && ((wave_need >> l) & 1u)) {
                    n_eval += (unsigned long long)(c1 - c0) * (unsigned long long)wave_pts;
                    if (l != open_l) {
                        if (open_l >= 0) level_flush<DIM, P>(a, open_l, dw, la, acc);
                        open_l = l;
                    }
                    level_accum<DIM, P, MIXED, BASIS>(a, l, tile, c0, c1, xq, org, la);
                }
            }
        }
        if (open_l >= 0) level_flush<DIM, P>(a, open_l, dw, la, acc);
    }
    if (a.pairs && lane == 0 && n_eval) atomicAdd(a.pairs, n_eval);
    store_rows<DIM, P>(a, wbase + (int64_t)wave * (64 * P), lane, ok, oi, acc);
}

// Sum the split partials in split order and write the final values.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void ksum_finalize(KArgs a)
{
    const int64_t n_work = a.n_work_dev ? *a.n_work_dev : a.n_work;
    for (int64_t w = (int64_t)blockIdx.x * BLOCK + threadIdx.x; w < n_work;
         w += (int64_t)gridDim.x * BLOCK) {
        const int64_t idx = a.work ? (int64_t)a.work[w] : w;
        const int64_t oi = a.out_perm ? (int64_t)a.out_perm[idx] : idx;
        if (oi < 0) continue;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double s = 0.0;
            for (int sp = 0; sp < a.n_split; ++sp) s += a.partial[((int64_t)sp * DIM + k) * a.ld_part + w];
            const int64_t o = k * a.ld_out + oi;
            a.out[o] = a.base ? a.base[o] - a.sign * s : (-a.sign) * s;
        }
    }
}

// ---- wall-distance reduction ------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void reduce_count(const double *d, int64_t n, double dmax,
                                                     int32_t *counts)
{
    __shared__ int32_t red[BLOCK];
    const int64_t base = (int64_t)blockIdx.x * CBLK + (int64_t)threadIdx.x * CHUNK;
    int c = 0;
#pragma unroll
    for (int j = 0; j < CHUNK; ++j)
        if (base + j < n && d[base + j] < dmax) ++c;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = red[0];
}

// Stable compaction of {v : d_v < dmax}: each block adds up the counts of the blocks before it
// (a fixed-order sum, so the list is the same every run), scans its own flags and writes its
// kept indices in order. Dropped points get +0.0 in every component; the last block stores
// the total.
__global__ __launch_bounds__(BLOCK) void reduce_scatter(const double *d, int64_t n, double dmax,
                                                       const int32_t *counts, int64_t *n_work,
                                                       int32_t *work, double *out, int32_t dim)
{
    __shared__ int32_t sc[BLOCK];
    __shared__ int64_t red[BLOCK];
    int64_t before = 0;
    for (int64_t b = threadIdx.x; b < blockIdx.x; b += BLOCK) before += counts[b];
    red[threadIdx.x] = before;
    const int64_t base = (int64_t)blockIdx.x * CBLK + (int64_t)threadIdx.x * CHUNK;
    bool keep[CHUNK];
    int c = 0;
#pragma unroll
    for (int j = 0; j < CHUNK; ++j) {
        keep[j] = base + j < n && d[base + j] < dmax;
        c += keep[j];
    }
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    for (int s = 1; s < BLOCK; s <<= 1) {
        const int32_t t = threadIdx.x >= s ? sc[threadIdx.x - s] : 0;
        __syncthreads();
        sc[threadIdx.x] += t;
        __syncthreads();
    }
    const int64_t block_off = red[0];
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == BLOCK - 1) *n_work = block_off + sc[BLOCK - 1];
    int64_t pos = block_off + sc[threadIdx.x] - c;
#pragma unroll
    for (int j = 0; j < CHUNK; ++j) {
        const int64_t v = base + j;
        if (v >= n) break;
        if (keep[j]) {
            work[pos++] = (int32_t)v;
        } else {
            for (int k = 0; k < dim; ++k) out[k * n + v] = 0.0;
        }
    }
}

template <int DIM, int P, int BASIS>
void launch_sum_t(const KArgs &a, dim3 grid, bool mixed, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (e0) {
        if (mixed)
            hipExtLaunchKernelGGL((ksum_kernel<DIM, P, true, BASIS>), grid, dim3(BLOCK), 0, s, e0, e1, 0, a);
        else
            hipExtLaunchKernelGGL((ksum_kernel<DIM, P, false, BASIS>), grid, dim3(BLOCK), 0, s, e0, e1, 0, a);
    } else if (mixed) {
        hipLaunchKernelGGL((ksum_kernel<DIM, P, true, BASIS>), grid, dim3(BLOCK), 0, s, a);
    } else {
        hipLaunchKernelGGL((ksum_kernel<DIM, P, false, BASIS>), grid, dim3(BLOCK), 0, s, a);
    }
}

template <int DIM, int BASIS>
void launch_sum_p(const KArgs &a, dim3 grid, int P, bool mixed, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (P == 1) launch_sum_t<DIM, 1, BASIS>(a, grid, mixed, s, e0, e1);
    else launch_sum_t<DIM, 2, BASIS>(a, grid, mixed, s, e0, e1);
}

template <int DIM>
void launch_sum_b(const KArgs &a, dim3 grid, int P, bool mixed, int32_t basis, hipStream_t s, hipEvent_t e0,
                  hipEvent_t e1)
{
    switch (basis) {
    case RBF_WENDLAND_C0: launch_sum_p<DIM, RBF_WENDLAND_C0>(a, grid, P, mixed, s, e0, e1); break;
    case RBF_WENDLAND_C4: launch_sum_p<DIM, RBF_WENDLAND_C4>(a, grid, P, mixed, s, e0, e1); break;
    case RBF_WENDLAND_C6: launch_sum_p<DIM, RBF_WENDLAND_C6>(a, grid, P, mixed, s, e0, e1); break;
    default: launch_sum_p<DIM, RBF_WENDLAND_C2>(a, grid, P, mixed, s, e0, e1); break;
    }
}

}  // namespace

void launch_sum(const KArgs &a, dim3 grid, int dim, int P, bool mixed, int32_t basis, hipStream_t s,
                hipEvent_t start, hipEvent_t stop)
{
    if (dim == 2) launch_sum_b<2>(a, grid, P, mixed, basis, s, start, stop);
    else launch_sum_b<3>(a, grid, P, mixed, basis, s, start, stop);
}

void launch_finalize(const KArgs &a, int dim, int blocks, hipStream_t s)
{
    if (dim == 2) hipLaunchKernelGGL(ksum_finalize<2>, dim3(blocks), dim3(BLOCK), 0, s, a);
    else hipLaunchKernelGGL(ksum_finalize<3>, dim3(blocks), dim3(BLOCK), 0, s, a);
}

void launch_reduce(const double *d, int64_t n, double dmax, int32_t *counts, int64_t *n_work,
                   int32_t *work, double *out, int32_t dim, hipStream_t s)
{
    const int64_t nb = (n + CBLK - 1) / CBLK;
    hipLaunchKernelGGL(reduce_count, dim3((unsigned)nb), dim3(BLOCK), 0, s, d, n, dmax, counts);
    hipLaunchKernelGGL(reduce_scatter, dim3((unsigned)nb), dim3(BLOCK), 0, s, d, n, dmax,
                       (const int32_t *)counts, n_work, work, out, dim);
}

}  // namespace ksum
}  // namespace rbf

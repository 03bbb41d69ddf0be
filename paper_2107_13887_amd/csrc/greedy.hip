// Multi-level greedy surface point selection (Section 3) on gfx950.
//
// Formulation. Let C = (c_0 .. c_{n-1}) be the control points of the current level and
// Phi_cc = L L^T the Cholesky factor of their basis matrix. The Newton basis
//   V[:, j] = Phi_sC L^{-T} e_j   (N_s values per column)
// holds, at every surface point, the values of the basis functions that L orthonormalises; its
// rows at the control points are L itself. With y = L^{-1} dS_C the greedy error of eq. (12) is
//   E = dS - Phi_sC alpha = dS - V y,   alpha = L^{-T} y.
// Appending a point p borders L with l = V[p, :] and d = sqrt(phi(0) - l.l) (the bordered
// Cholesky step of the weight solve, eq. (9)), adds the column
//   v = (phi(||x - x_p|| / R) - V l) / d
// and the coefficient y_n = E_p / d, so that E <- E - y_n v. Each iteration therefore costs one
// matrix-vector product over the stored basis (memory-bound, fully parallel over surface points)
// plus an argmax, and never a triangular solve. alpha is recovered once per level by a blocked
// back substitution L^T alpha = y, and the level residual dS_{l+1} = dS_l - Phi_sC alpha is then
// recomputed from alpha by the FP64 kernel sum (the same quantity the paper's loop produces).
//
// Kernels per iteration: g_select (one workgroup: argmax of the per-block maxima, stop tests,
// row extraction, pivot) and g_update (one workgroup per 64 surface points: new column, error
// update, block argmax). Reductions run in a fixed order; squared norms are formed without fused
// multiply-adds so they equal the oracle's formula term by term.
#include <cmath>
#include <vector>

#include "internal.h"

namespace rbf {
namespace {

constexpr int UPB = 64;       // surface points per update workgroup (one per lane)
constexpr int UWAVES = 4;     // waves per update workgroup, each a slice of the dot product
constexpr int LCHUNK = 2048;  // Newton row entries staged per LDS pass

struct GState {
    int64_t n;        // finished columns (control points) of the level
    int64_t p;        // point appended by the pending update
    int64_t n_iter;   // argmax selections made in this call (all levels)
    int32_t go;       // 1: an update for column n is pending
    int32_t stop;     // RBF_STOP_* once the level stopped, else -1
    double d;         // pivot of the pending column
    double c[3];      // Newton coefficients of the pending column
    double target2;   // squared tolerance of the level
    double rmax2;     // max_i ||r_i||^2 of the level's input residual
};

struct Cand {
    double m2;
    int64_t idx;
};

__device__ __forceinline__ bool better(double m2, int64_t i, double bm2, int64_t bi)
{
    // Larger squared norm wins; equal values go to the lower index; idx < 0 means "none".
    if (i < 0) return false;
    if (bi < 0) return true;
    return m2 > bm2 || (m2 == bm2 && i < bi);
}

template <int DIM>
__device__ __forceinline__ double norm2_plain(const double *v, int64_t ld, int64_t i)
{
#pragma clang fp contract(off)
    double s = v[i] * v[i];
#pragma unroll
    for (int k = 1; k < DIM; ++k) s = s + v[k * ld + i] * v[k * ld + i];
    return s;
}

// phi(||a - b|| / R) term by term as the textbook formula (no contraction), for the few basis
// values computed per iteration.
template <int DIM>
__device__ __forceinline__ double phi_pair(const double *xs, int64_t ld, int64_t i, int64_t j, double R)
{
#pragma clang fp contract(off)
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        double d = xs[k * ld + i] - xs[k * ld + j];
        s = s + d * d;
    }
    double eta = sqrt(s) / R;
    if (eta >= 1.0) return 0.0;
    double t = 1.0 - eta;
    return t * t * t * t * (4.0 * eta + 1.0);
}

__device__ __forceinline__ void wave_argmax(double &m2, int64_t &idx)
{
    for (int off = 32; off > 0; off >>= 1) {
        double om = __shfl_down(m2, off, 64);
        int64_t oi = __shfl_down(idx, off, 64);
        if (better(om, oi, m2, idx)) {
            m2 = om;
            idx = oi;
        }
    }
}

// E = r, selected = 0, per-block max of ||r_i||^2 (no exclusions).
template <int DIM>
__global__ __launch_bounds__(64) void g_init(const double *r, double *E, uint8_t *sel, int64_t n_s,
                                             Cand *part)
{
    int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
    double m2 = -1.0;
    int64_t idx = -1;
    if (i < n_s) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) E[k * n_s + i] = r[k * n_s + i];
        sel[i] = 0;
        m2 = norm2_plain<DIM>(r, n_s, i);
        idx = i;
    }
    wave_argmax(m2, idx);
    if (threadIdx.x == 0) part[blockIdx.x] = Cand{m2, idx};
}

__device__ void block_argmax(const Cand *part, int64_t g, double &m2, int64_t &idx, Cand *sh)
{
    double bm = -1.0;
    int64_t bi = -1;
    for (int64_t b = threadIdx.x; b < g; b += blockDim.x) {
        Cand c = part[b];
        if (better(c.m2, c.idx, bm, bi)) {
            bm = c.m2;
            bi = c.idx;
        }
    }
    wave_argmax(bm, bi);
    int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[w] = Cand{bm, bi};
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k)
            if (better(sh[k].m2, sh[k].idx, bm, bi)) {
                bm = sh[k].m2;
                bi = sh[k].idx;
            }
        sh[0] = Cand{bm, bi};
    }
    __syncthreads();
    m2 = sh[0].m2;
    idx = sh[0].idx;
}

// Level start: the level target from max ||r||^2, as max(eps, rho * max ||r||) squared.
__global__ __launch_bounds__(256) void g_begin(GState *st, const Cand *part, int64_t g, double eps,
                                               double rho, int32_t last)
{
    __shared__ Cand sh[4];
    double m2;
    int64_t idx;
    block_argmax(part, g, m2, idx, sh);
    if (threadIdx.x == 0) {
        double rmax2 = m2 < 0.0 ? 0.0 : m2;
        double target = eps;
        if (!last && rho * sqrt(rmax2) > target) target = rho * sqrt(rmax2);
        st->rmax2 = rmax2;
        st->target2 = target * target;
        st->n = 0;
        st->go = 0;
        st->stop = -1;
    }
}

// One selection: argmax (or a forced seed), stop tests, Newton row extraction and pivot.
template <int DIM>
__global__ __launch_bounds__(256) void g_select(GState *st, const Cand *part, int64_t g,
                                                int64_t forced, int64_t cap_level, const double *V,
                                                int64_t ldV, double *Lpack, double *coef,
                                                int64_t ld_coef, const double *E, int64_t n_s,
                                                int64_t *ctrl, uint8_t *sel, double *hist,
                                                int64_t hist_cap)
{
    __shared__ Cand sh[4];
    __shared__ double red[256];
    __shared__ int32_t s_stop, s_skip;
    __shared__ int64_t s_n;
    if (threadIdx.x == 0) {
        s_skip = st->stop >= 0;            // level already finished
        if (!s_skip && st->go) {           // the previous update completed column n
            st->n += 1;
            st->go = 0;
        }
        s_n = st->n;
    }
    __syncthreads();
    if (s_skip) return;
    const int64_t n = s_n;
    double m2 = 0.0;
    int64_t p = forced;
    if (forced < 0) block_argmax(part, g, m2, p, sh);
    if (threadIdx.x == 0) {
        int32_t stop = -1;
        if (forced < 0) {
            if (p < 0) stop = RBF_STOP_ALL_SELECTED;
            else if (m2 < st->target2) stop = RBF_STOP_EPS;
        }
        if (stop < 0 && n >= cap_level) stop = RBF_STOP_CAP;
        s_stop = stop;
        if (stop >= 0) st->stop = stop;
    }
    __syncthreads();
    if (s_stop >= 0) return;

    // l = V[p, 0:n] is the new row of the Cholesky factor of Phi_cc.
    double *row = Lpack + (n * (n + 1)) / 2;
    double part_ll = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
        double v = V[j * ldV + p];
        row[j] = v;
        part_ll = __builtin_fma(v, v, part_ll);
    }
    red[threadIdx.x] = part_ll;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double d2 = 1.0 - red[0];     // phi(0) - l.l
        // l.l carries about (n + 1) ulps of rounding: a pivot below that is zero (breakdown).
        if (!(d2 > (double)(n + 1) * 0x1p-52)) {
            st->stop = RBF_STOP_BREAKDOWN;
            return;
        }
        double d = sqrt(d2);
        row[n] = d;
        st->p = p;
        st->d = d;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double c = E[k * n_s + p] / d;
            st->c[k] = c;
            coef[k * ld_coef + n] = c;
        }
        ctrl[n] = p;
        sel[p] = 1;
        if (forced < 0) {
            if (st->n_iter < hist_cap) hist[st->n_iter] = sqrt(m2);
            st->n_iter += 1;
        }
        st->go = 1;
    }
}

// New Newton column, error update and per-block argmax. Lane = surface point, wave = slice of
// the dot product V[i, 0:n] . l.
template <int DIM>
__global__ __launch_bounds__(UPB *UWAVES) void g_update(const GState *st, const double *xs,
                                                        int64_t n_s, double R, double *V,
                                                        int64_t ldV, const double *Lpack,
                                                        double *E, const uint8_t *sel, Cand *part)
{
    __shared__ double lsh[LCHUNK];
    __shared__ double psum[UWAVES][UPB];
    if (!st->go) return;
    const int64_t n = st->n;
    const int64_t p = st->p;
    const double *lrow = Lpack + (n * (n + 1)) / 2;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * UPB + lane;
    const bool ok = i < n_s;
    const int64_t ic = ok ? i : 0;

    double s = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += LCHUNK) {
        const int nj = (int)min<int64_t>(LCHUNK, n - j0);
        __syncthreads();
        for (int t = threadIdx.x; t < nj; t += UPB * UWAVES) lsh[t] = lrow[j0 + t];
        __syncthreads();
        const int per = (nj + UWAVES - 1) / UWAVES;
        const int jb = w * per, je = min(nj, jb + per);
        const double *col = V + (j0 + jb) * ldV + ic;
        int j = jb;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (; j + 4 <= je; j += 4, col += 4 * ldV) {
            s0 = __builtin_fma(col[0], lsh[j], s0);
            s1 = __builtin_fma(col[ldV], lsh[j + 1], s1);
            s2 = __builtin_fma(col[2 * ldV], lsh[j + 2], s2);
            s3 = __builtin_fma(col[3 * ldV], lsh[j + 3], s3);
        }
        for (; j < je; ++j, col += ldV) s0 = __builtin_fma(col[0], lsh[j], s0);
        s += (s0 + s1) + (s2 + s3);
    }
    psum[w][lane] = s;
    __syncthreads();
    if (w != 0) return;

    double m2 = -1.0;
    int64_t idx = -1;
    if (ok) {
        double dot = psum[0][lane];
#pragma unroll
        for (int k = 1; k < UWAVES; ++k) dot += psum[k][lane];
        const double d = st->d;
        double v = (phi_pair<DIM>(xs, n_s, i, p, R) - dot) / d;
        V[n * ldV + i] = v;
#pragma unroll
        for (int k = 0; k < DIM; ++k) E[k * n_s + i] = __builtin_fma(-st->c[k], v, E[k * n_s + i]);
        if (!sel[i]) {
            m2 = norm2_plain<DIM>(E, n_s, i);
            idx = i;
        }
    }
    wave_argmax(m2, idx);
    if (lane == 0) part[blockIdx.x] = Cand{m2, idx};
}

// Blocked back substitution L^T alpha = y for the 64 rows [b0, b1) (all later rows done).
// Every workgroup solves the diagonal block (cheap, redundant) and then removes the block's
// contribution from its share of the rows above b0; workgroup 0 stores alpha.
template <int DIM>
__global__ __launch_bounds__(256) void g_backsolve(const double *Lpack, double *y, int64_t ld_y,
                                                   double *alpha, int64_t ld_a, int64_t b0, int64_t b1)
{
    __shared__ double Lb[64][65];
    __shared__ double xb[DIM][64];
    const int nb = (int)(b1 - b0);
    for (int t = threadIdx.x; t < 64 * 64; t += blockDim.x) {
        int r = t / 64, c = t % 64;
        Lb[r][c] = (r < nb && c <= r) ? Lpack[((b0 + r) * (b0 + r + 1)) / 2 + b0 + c] : 0.0;
    }
    if (threadIdx.x < 64) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) xb[k][threadIdx.x] = threadIdx.x < nb ? y[k * ld_y + b0 + threadIdx.x] : 0.0;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int j = threadIdx.x;
        double rhs[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) rhs[k] = xb[k][j];
        for (int i = nb - 1; i >= 0; --i) {
            double xi[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                double v = rhs[k] / Lb[i][i];
                xi[k] = __shfl(v, i, 64);
            }
            if (j < i) {
#pragma unroll
                for (int k = 0; k < DIM; ++k) rhs[k] = __builtin_fma(-Lb[i][j], xi[k], rhs[k]);
            }
            if (j == i) {
#pragma unroll
                for (int k = 0; k < DIM; ++k) rhs[k] = xi[k];
            }
        }
#pragma unroll
        for (int k = 0; k < DIM; ++k) xb[k][j] = rhs[k];
        if (blockIdx.x == 0 && j < nb) {
#pragma unroll
            for (int k = 0; k < DIM; ++k) alpha[k * ld_a + b0 + j] = rhs[k];
        }
    }
    __syncthreads();
    // Rows above the block: y_j -= sum_{i in block} L[i][j] alpha_i.
    for (int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; jj < b0;
         jj += (int64_t)gridDim.x * blockDim.x) {
        double acc[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) acc[k] = 0.0;
        for (int i = 0; i < nb; ++i) {
            double lij = Lpack[((b0 + i) * (b0 + i + 1)) / 2 + jj];
#pragma unroll
            for (int k = 0; k < DIM; ++k) acc[k] = __builtin_fma(lij, xb[k][i], acc[k]);
        }
#pragma unroll
        for (int k = 0; k < DIM; ++k) y[k * ld_y + jj] -= acc[k];
    }
}

template <int DIM>
__global__ __launch_bounds__(256) void g_gather(const double *xs, int64_t n_s, const int64_t *ctrl,
                                                int64_t n, double *xc, int64_t ld)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        int64_t p = ctrl[j];
#pragma unroll
        for (int k = 0; k < DIM; ++k) xc[k * ld + j] = xs[k * n_s + p];
    }
}

__global__ void g_finite(const double *a, int64_t n, int32_t *bad)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(a[i])) *bad = 1;
}

template <int DIM>
rbf_status greedy_impl(rbf_ctx ctx, const rbf_greedy_params &prm, int64_t n_s, const double *xs,
                       const double *ds, rbf_ctrl_set *out, hipStream_t s)
{
    Pool *pool = ctx->pool.get();
    const int64_t cap = prm.max_ctrl_total;
    const int64_t cols = std::min<int64_t>(n_s, cap);      // most columns one level can need
    const int64_t g = (n_s + UPB - 1) / UPB;

    DevBuf bV, bL, bE, bR, bR2, bSel, bPart, bState, bCoef, bHist, bFlag;
    RBF_TRY(bV.get(pool, sizeof(double) * (size_t)cols * (size_t)n_s));
    RBF_TRY(bL.get(pool, sizeof(double) * (size_t)(cols * (cols + 1) / 2 + 1)));
    RBF_TRY(bE.get(pool, sizeof(double) * DIM * (size_t)n_s));
    RBF_TRY(bR.get(pool, sizeof(double) * DIM * (size_t)n_s));
    RBF_TRY(bR2.get(pool, sizeof(double) * DIM * (size_t)n_s));
    RBF_TRY(bSel.get(pool, (size_t)n_s));
    RBF_TRY(bPart.get(pool, sizeof(Cand) * (size_t)g));
    RBF_TRY(bState.get(pool, sizeof(GState)));
    RBF_TRY(bCoef.get(pool, sizeof(double) * DIM * (size_t)cols));
    RBF_TRY(bHist.get(pool, sizeof(double) * (size_t)cap));
    RBF_TRY(bFlag.get(pool, sizeof(int32_t)));
    double *V = bV.as<double>(), *Lp = bL.as<double>(), *E = bE.as<double>();
    double *R = bR.as<double>(), *R2 = bR2.as<double>(), *coef = bCoef.as<double>();
    uint8_t *sel = bSel.as<uint8_t>();
    Cand *part = bPart.as<Cand>();
    GState *st = bState.as<GState>();

    // Reject non-finite coordinates or displacements.
    RBF_HIP(hipMemsetAsync(bFlag.ptr, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(g_finite, dim3(256), dim3(256), 0, s, xs, (int64_t)DIM * n_s, bFlag.as<int32_t>());
    hipLaunchKernelGGL(g_finite, dim3(256), dim3(256), 0, s, ds, (int64_t)DIM * n_s, bFlag.as<int32_t>());
    int32_t bad = 0;
    RBF_HIP(hipMemcpyAsync(&bad, bFlag.ptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RBF_HIP(hipStreamSynchronize(s));
    if (bad) return fail(RBF_E_INVALID, "xs or ds holds a non-finite value");

    RBF_HIP(hipMemsetAsync(st, 0, sizeof(GState), s));
    RBF_HIP(hipMemcpyAsync(R, ds, sizeof(double) * DIM * n_s, hipMemcpyDeviceToDevice, s));

    GState hs{};
    int64_t total = 0, iters_before = 0;
    int used = 0;
    out->level_off[0] = 0;
    for (int l = 0; l < RBF_MAX_LEVELS; ++l) {
        out->level_stop[l] = RBF_STOP_SKIPPED;
        out->level_max_err[l] = 0.0;
    }
    for (int l = 0; l < prm.n_levels; ++l) {
        const double Rl = prm.radius[l];
        const int64_t cap_level = std::min<int64_t>(cols, cap - total);
        hipLaunchKernelGGL(g_init<DIM>, dim3((unsigned)g), dim3(64), 0, s, R, E, sel, n_s, part);
        hipLaunchKernelGGL(g_begin, dim3(1), dim3(256), 0, s, st, part, g, prm.eps_abs,
                           prm.level_reduction, (int32_t)(l == prm.n_levels - 1));
        int64_t *ctrl = out->ctrl_idx + total;
        auto step = [&](int64_t forced) {
            hipLaunchKernelGGL(g_select<DIM>, dim3(1), dim3(256), 0, s, st, part, g, forced, cap_level,
                               V, n_s, Lp, coef, cols, E, n_s, ctrl, sel, bHist.as<double>(), cap);
            hipLaunchKernelGGL(g_update<DIM>, dim3((unsigned)g), dim3(UPB * UWAVES), 0, s, st, xs, n_s,
                               Rl, V, n_s, Lp, E, sel, part);
        };
        if (prm.seed_off) {
            for (int32_t k = prm.seed_off[l]; k < prm.seed_off[l + 1]; ++k) step(prm.seed_idx[k]);
        } else if (l == 0) {
            step(0);
        }
        RBF_HIP(hipGetLastError());
        // Argmax iterations in batches; the device stops itself, extra launches are no-ops.
        // Every effective iteration adds a column, so the level ends within cap_level + 1
        // selections; the host gives up (device error) well after that.
        int64_t batch = 16, launched = 0;
        for (;;) {
            for (int64_t b = 0; b < batch; ++b) step(-1);
            launched += batch;
            RBF_HIP(hipGetLastError());
            RBF_HIP(hipMemcpyAsync(&hs, st, sizeof(GState), hipMemcpyDeviceToHost, s));
            RBF_HIP(hipStreamSynchronize(s));
            if (hs.stop >= 0) break;
            if (launched > cap_level + 1024)
                return fail(RBF_E_DEVICE, "greedy level %d did not terminate after %lld selections", l,
                            (long long)launched);
            batch = std::min<int64_t>(batch * 2, 256);
        }
        const int64_t n = hs.n;
        out->level_stop[l] = hs.stop;
        // Weights: L^T alpha = y, blocked from the bottom.
        double *alpha = out->alpha + total;
        if (n > 0) {
            RBF_HIP(hipMemcpy2DAsync(R2, sizeof(double) * cols, coef, sizeof(double) * cols,
                                     sizeof(double) * n, DIM, hipMemcpyDeviceToDevice, s));
            for (int64_t b1 = n; b1 > 0; b1 -= 64) {
                int64_t b0 = std::max<int64_t>(0, b1 - 64);
                unsigned gb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((b0 + 255) / 256, 1024));
                hipLaunchKernelGGL(g_backsolve<DIM>, dim3(gb), dim3(256), 0, s, Lp, R2, cols, alpha,
                                   out->capacity, b0, b1);
            }
            unsigned gg = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024));
            hipLaunchKernelGGL(g_gather<DIM>, dim3(gg), dim3(256), 0, s, xs, n_s, ctrl, n,
                               out->xc + total, out->capacity);
            RBF_HIP(hipGetLastError());
            // dS_{l+1} = dS_l - Phi_sC alpha at every surface point, FP64 kernel sum.
            SumProblem pb;
            pb.dim = DIM;
            pb.n_levels = 1;
            pb.lv[0] = SumLevel{1.0 / Rl, 0.0, 0, n};
            pb.ld_ctrl = out->capacity;
            pb.xc = out->xc + total;
            pb.alpha = alpha;
            pb.n_p = n_s;
            pb.xp = xs;
            pb.base = R;
            pb.sign = 1.0;
            pb.out = R2;
            pb.precision = RBF_FP64;
            RBF_TRY(run_kernel_sum(ctx, pb, s));
            std::swap(R, R2);
        }
        total += n;
        out->level_off[l + 1] = (int32_t)total;
        used = l + 1;
        // max ||dS_{l+1}|| decides whether another level is needed.
        hipLaunchKernelGGL(g_init<DIM>, dim3((unsigned)g), dim3(64), 0, s, R, E, sel, n_s, part);
        hipLaunchKernelGGL(g_begin, dim3(1), dim3(256), 0, s, st, part, g, prm.eps_abs,
                           prm.level_reduction, 1);
        RBF_HIP(hipGetLastError());
        RBF_HIP(hipMemcpyAsync(&hs, st, sizeof(GState), hipMemcpyDeviceToHost, s));
        RBF_HIP(hipStreamSynchronize(s));
        out->level_max_err[l] = std::sqrt(hs.rmax2);
        if (std::sqrt(hs.rmax2) < prm.eps_abs || out->level_stop[l] == RBF_STOP_CAP) break;
    }
    for (int l = used; l < prm.n_levels; ++l) out->level_off[l + 1] = (int32_t)total;
    out->n_levels_used = used;
    out->stop_reason = out->level_stop[used - 1];
    out->n_iterations = hs.n_iter - iters_before;
    if (out->e_final)
        RBF_HIP(hipMemcpyAsync(out->e_final, R, sizeof(double) * DIM * n_s, hipMemcpyDeviceToDevice, s));
    RBF_HIP(hipStreamSynchronize(s));
    bool cap_hit = false, brk = false;
    for (int l = 0; l < used; ++l) {
        cap_hit |= out->level_stop[l] == RBF_STOP_CAP;
        brk |= out->level_stop[l] == RBF_STOP_BREAKDOWN;
    }
    return brk ? RBF_W_BREAKDOWN : (cap_hit ? RBF_W_CAP : RBF_OK);
}

}  // namespace

rbf_status run_greedy(rbf_ctx ctx, const rbf_greedy_params &p, int64_t n_s, const double *xs,
                      const double *ds, rbf_ctrl_set *out, hipStream_t s)
{
    return p.dim == 2 ? greedy_impl<2>(ctx, p, n_s, xs, ds, out, s)
                      : greedy_impl<3>(ctx, p, n_s, xs, ds, out, s);
}

}  // namespace rbf

// Wendland C2 kernel sums on gfx950: the volume update of eqs. (19)/(23) and the surface
// interpolant/residual of eqs. (1)/(12).
//
//   out_k(p) = base_k(p) - sign * sum_l psi(d_p / D_l) sum_{c in level l} phi(||x_p - x_c|| / R_l) alpha_k,c
//
// Design (VALU-bound: ~20-27 vector slots per point/control pair against 40-56 bytes of HBM
// traffic per point):
//   * points stream as SoA, P points per lane, 256 lanes per workgroup;
//   * controls of each level are packed once (coordinates pre-scaled by 1/R_l, then the weights)
//     and staged through LDS in tiles of 256; every lane of a wave reads the same LDS address,
//     a broadcast without bank conflicts;
//   * the control list of each level may be split over gridDim.y to give enough waves when there
//     are few points; the split partial sums are reduced in a fixed order (deterministic);
//   * the wall-distance reduction keeps only points with d < max_l D_l: either the prefix of a
//     volume sorted by d, or a stable compaction that also writes +0.0 to every dropped point;
//   * FP64 square root from the hardware reciprocal square-root estimate refined by one
//     Goldschmidt step and one Newton correction (accurate to about one ulp);
//   * mixed precision: the pair arithmetic runs in FP32 on coordinates shifted to a per-workgroup
//     origin (the workgroup's first point), the basis value is widened and accumulated in FP64.
#include "internal.h"

namespace rbf {
namespace {

constexpr int BLOCK = 256;
constexpr int TILE = 256;

struct KArgs {
    int32_t n_levels;
    int32_t n_split;
    SumLevel lv[RBF_MAX_LEVELS];
    double dsupp[RBF_MAX_LEVELS];   // D_l (psi applied when dwall != null)
    const double *pack;             // [n_ctrl][2*DIM]: x/R_l, y/R_l, (z/R_l), alpha_x, alpha_y, (alpha_z)
    const int32_t *work;            // reduced point list, or null for the identity
    const int64_t *n_work_dev;      // device-side count (null: use n_work)
    int64_t n_work;
    const double *xp;
    int64_t ld_p;
    const double *dwall;
    const double *base;
    double sign;
    double *out;
    int64_t ld_out;
    double *partial;                // [n_split][DIM][ld_part]
    int64_t ld_part;
};

__device__ __forceinline__ double sqrt_pos(double a)
{
    // a >= 1e-200 (a normal number). One Goldschmidt step squares the estimate's relative error,
    // the Newton correction squares it again.
    double y = __builtin_amdgcn_rsq(a);
    double g = a * y;
    double h = 0.5 * y;
    double r = __builtin_fma(-g, h, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    double d = __builtin_fma(-g, g, a);
    return __builtin_fma(d, h, g);
}

// Wendland C2, eq. (2): (1 - eta)^4 (4 eta + 1) on [0, 1), zero beyond, written branch-free.
__device__ __forceinline__ double phi_c2(double eta)
{
    double t = fmax(1.0 - eta, 0.0);
    double t2 = t * t;
    return (t2 * t2) * __builtin_fma(4.0, eta, 1.0);
}

__device__ __forceinline__ float phi_c2f(float eta)
{
    float t = fmaxf(1.0f - eta, 0.0f);
    float t2 = t * t;
    return (t2 * t2) * __builtin_fmaf(4.0f, eta, 1.0f);
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
    int64_t nc = L.c_end - L.c_begin;
    cb = L.c_begin + (nc * s) / S;
    ce = L.c_begin + (nc * (s + 1)) / S;
}

template <int DIM, int P>
__global__ __launch_bounds__(BLOCK) void ksum_f64(KArgs a)
{
    constexpr int ST = 2 * DIM;
    __shared__ double tile[TILE * ST];
    const int tid = threadIdx.x;
    const int64_t n_work = a.n_work_dev ? *a.n_work_dev : a.n_work;
    const int64_t wbase = (int64_t)blockIdx.x * (BLOCK * P);
    if (wbase >= n_work) return;
    const int split = blockIdx.y;

    double x[P][DIM], dw[P], acc[P][DIM];
    int64_t idx[P];
    bool ok[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        int64_t w = wbase + p * BLOCK + tid;
        ok[p] = w < n_work;
        idx[p] = ok[p] ? (a.work ? (int64_t)a.work[w] : w) : 0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            x[p][k] = ok[p] ? a.xp[k * a.ld_p + idx[p]] : 0.0;
            acc[p][k] = 0.0;
        }
        dw[p] = (a.dwall && ok[p]) ? a.dwall[idx[p]] : 0.0;
    }

    for (int l = 0; l < a.n_levels; ++l) {
        double wg[P];
        int any = 0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            wg[p] = a.dwall ? psi_w(dw[p], a.dsupp[l]) : 1.0;
            any |= (ok[p] && wg[p] > 0.0);
        }
        if (!__syncthreads_or(any)) continue;
        const double inv_r = a.lv[l].inv_r;
        int64_t cb, ce;
        split_range(a.lv[l], split, a.n_split, cb, ce);
        double q[P][DIM], la[P][DIM];
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                q[p][k] = x[p][k] * inv_r;
                la[p][k] = 0.0;
            }
        for (int64_t t0 = cb; t0 < ce; t0 += TILE) {
            const int nt = (int)min<int64_t>(TILE, ce - t0);
            __syncthreads();
            for (int i = tid; i < nt * ST; i += BLOCK) tile[i] = a.pack[t0 * ST + i];
            __syncthreads();
            for (int c = 0; c < nt; ++c) {
                const double *cc = tile + c * ST;
                double cpos[DIM], cal[DIM];
#pragma unroll
                for (int k = 0; k < DIM; ++k) {
                    cpos[k] = cc[k];
                    cal[k] = cc[DIM + k];
                }
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    double d0 = q[p][0] - cpos[0];
                    double r2 = d0 * d0;
#pragma unroll
                    for (int k = 1; k < DIM; ++k) {
                        double dk = q[p][k] - cpos[k];
                        r2 = __builtin_fma(dk, dk, r2);
                    }
                    double eta = sqrt_pos(fmax(r2, 1e-200));
                    double ph = phi_c2(eta);
#pragma unroll
                    for (int k = 0; k < DIM; ++k) la[p][k] = __builtin_fma(ph, cal[k], la[p][k]);
                }
            }
        }
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int k = 0; k < DIM; ++k) acc[p][k] = __builtin_fma(wg[p], la[p][k], acc[p][k]);
    }

#pragma unroll
    for (int p = 0; p < P; ++p) {
        if (!ok[p]) continue;
        if (a.n_split == 1) {
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                double b = a.base ? a.base[k * a.ld_out + idx[p]] : 0.0;
                a.out[k * a.ld_out + idx[p]] = a.base ? b - a.sign * acc[p][k] : (-a.sign) * acc[p][k];
            }
        } else {
            int64_t w = wbase + p * BLOCK + tid;
#pragma unroll
            for (int k = 0; k < DIM; ++k)
                a.partial[((int64_t)split * DIM + k) * a.ld_part + w] = acc[p][k];
        }
    }
}

// Mixed precision: FP32 pair arithmetic around a per-workgroup origin, FP64 accumulation.
template <int DIM, int P>
__global__ __launch_bounds__(BLOCK) void ksum_mixed(KArgs a)
{
    constexpr int ST = 2 * DIM;
    __shared__ float tpos[TILE * 4];
    __shared__ double tal[TILE * DIM];
    __shared__ double origin[DIM];
    const int tid = threadIdx.x;
    const int64_t n_work = a.n_work_dev ? *a.n_work_dev : a.n_work;
    const int64_t wbase = (int64_t)blockIdx.x * (BLOCK * P);
    if (wbase >= n_work) return;
    const int split = blockIdx.y;

    double x[P][DIM], dw[P], acc[P][DIM];
    int64_t idx[P];
    bool ok[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        int64_t w = wbase + p * BLOCK + tid;
        ok[p] = w < n_work;
        idx[p] = ok[p] ? (a.work ? (int64_t)a.work[w] : w) : 0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            x[p][k] = ok[p] ? a.xp[k * a.ld_p + idx[p]] : 0.0;
            acc[p][k] = 0.0;
        }
        dw[p] = (a.dwall && ok[p]) ? a.dwall[idx[p]] : 0.0;
    }
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) origin[k] = x[0][k];
    }
    __syncthreads();
    double o[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) o[k] = origin[k];

    for (int l = 0; l < a.n_levels; ++l) {
        double wg[P];
        int any = 0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            wg[p] = a.dwall ? psi_w(dw[p], a.dsupp[l]) : 1.0;
            any |= (ok[p] && wg[p] > 0.0);
        }
        if (!__syncthreads_or(any)) continue;
        const double inv_r = a.lv[l].inv_r;
        int64_t cb, ce;
        split_range(a.lv[l], split, a.n_split, cb, ce);
        float q[P][DIM];
        double la[P][DIM];
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                q[p][k] = (float)((x[p][k] - o[k]) * inv_r);
                la[p][k] = 0.0;
            }
        for (int64_t t0 = cb; t0 < ce; t0 += TILE) {
            const int nt = (int)min<int64_t>(TILE, ce - t0);
            __syncthreads();
            for (int c = tid; c < nt; c += BLOCK) {
                const double *src = a.pack + (t0 + c) * ST;
#pragma unroll
                for (int k = 0; k < DIM; ++k) {
                    tpos[c * 4 + k] = (float)(src[k] - o[k] * inv_r);
                    tal[c * DIM + k] = src[DIM + k];
                }
            }
            __syncthreads();
            for (int c = 0; c < nt; ++c) {
                float cpos[DIM];
                double cal[DIM];
#pragma unroll
                for (int k = 0; k < DIM; ++k) {
                    cpos[k] = tpos[c * 4 + k];
                    cal[k] = tal[c * DIM + k];
                }
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    float d0 = q[p][0] - cpos[0];
                    float r2 = d0 * d0;
#pragma unroll
                    for (int k = 1; k < DIM; ++k) {
                        float dk = q[p][k] - cpos[k];
                        r2 = __builtin_fmaf(dk, dk, r2);
                    }
                    float eta = __builtin_amdgcn_sqrtf(r2);
                    double ph = (double)phi_c2f(eta);
#pragma unroll
                    for (int k = 0; k < DIM; ++k) la[p][k] = __builtin_fma(ph, cal[k], la[p][k]);
                }
            }
        }
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int k = 0; k < DIM; ++k) acc[p][k] = __builtin_fma(wg[p], la[p][k], acc[p][k]);
    }

#pragma unroll
    for (int p = 0; p < P; ++p) {
        if (!ok[p]) continue;
        if (a.n_split == 1) {
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                double b = a.base ? a.base[k * a.ld_out + idx[p]] : 0.0;
                a.out[k * a.ld_out + idx[p]] = a.base ? b - a.sign * acc[p][k] : (-a.sign) * acc[p][k];
            }
        } else {
            int64_t w = wbase + p * BLOCK + tid;
#pragma unroll
            for (int k = 0; k < DIM; ++k)
                a.partial[((int64_t)split * DIM + k) * a.ld_part + w] = acc[p][k];
        }
    }
}

// Sum the split partials in split order and write the final values.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void ksum_finalize(KArgs a)
{
    const int64_t n_work = a.n_work_dev ? *a.n_work_dev : a.n_work;
    for (int64_t w = (int64_t)blockIdx.x * BLOCK + threadIdx.x; w < n_work;
         w += (int64_t)gridDim.x * BLOCK) {
        int64_t idx = a.work ? (int64_t)a.work[w] : w;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double s = 0.0;
            for (int sp = 0; sp < a.n_split; ++sp) s += a.partial[((int64_t)sp * DIM + k) * a.ld_part + w];
            double b = a.base ? a.base[k * a.ld_out + idx] : 0.0;
            a.out[k * a.ld_out + idx] = a.base ? b - a.sign * s : (-a.sign) * s;
        }
    }
}

// Pack the controls of every level: coordinates scaled by 1/R_l, then the weights.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void pack_controls(int32_t n_levels, const SumLevel *lv_unused,
                                                     KArgs a, const double *xc, const double *alpha,
                                                     int64_t ld, double *pack)
{
    constexpr int ST = 2 * DIM;
    int64_t n_total = a.lv[n_levels - 1].c_end;
    for (int64_t c = (int64_t)blockIdx.x * BLOCK + threadIdx.x; c < n_total;
         c += (int64_t)gridDim.x * BLOCK) {
        double inv_r = a.lv[0].inv_r;
        for (int l = 0; l < n_levels; ++l)
            if (c >= a.lv[l].c_begin && c < a.lv[l].c_end) inv_r = a.lv[l].inv_r;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            pack[c * ST + k] = xc[k * ld + c] * inv_r;
            pack[c * ST + DIM + k] = alpha[k * ld + c];
        }
    }
}

// ---- wall-distance reduction ------------------------------------------------------------------
constexpr int CHUNK = 4;                  // points per lane in the compaction
constexpr int CBLK = BLOCK * CHUNK;       // points per compaction block

__global__ __launch_bounds__(BLOCK) void reduce_count(const double *d, int64_t n, double dmax,
                                                     int32_t *counts)
{
    __shared__ int32_t red[BLOCK];
    int64_t base = (int64_t)blockIdx.x * CBLK + (int64_t)threadIdx.x * CHUNK;
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

// Exclusive scan of the per-block counts by one workgroup; total to *n_work.
__global__ __launch_bounds__(1024) void reduce_scan(int32_t *counts, int64_t n_blocks, int64_t *n_work)
{
    __shared__ int64_t buf[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < n_blocks; b0 += 1024) {
        int64_t i = b0 + threadIdx.x;
        int64_t v = i < n_blocks ? counts[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int s = 1; s < 1024; s <<= 1) {
            int64_t t = threadIdx.x >= s ? buf[threadIdx.x - s] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < n_blocks) counts[i] = (int32_t)(carry + buf[threadIdx.x] - v);
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_work = carry;
}

// Stable compaction of {v : d_v < dmax}; dropped points get +0.0 in every component of out.
__global__ __launch_bounds__(BLOCK) void reduce_scatter(const double *d, int64_t n, double dmax,
                                                       const int32_t *offsets, int32_t *work,
                                                       double *out, int32_t dim)
{
    __shared__ int32_t sc[BLOCK];
    int64_t base = (int64_t)blockIdx.x * CBLK + (int64_t)threadIdx.x * CHUNK;
    bool keep[CHUNK];
    int c = 0;
#pragma unroll
    for (int j = 0; j < CHUNK; ++j) {
        keep[j] = base + j < n && d[base + j] < dmax;
        c += keep[j];
    }
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int s = 1; s < BLOCK; s <<= 1) {
        int32_t t = threadIdx.x >= s ? sc[threadIdx.x - s] : 0;
        __syncthreads();
        sc[threadIdx.x] += t;
        __syncthreads();
    }
    int32_t pos = offsets[blockIdx.x] + sc[threadIdx.x] - c;
#pragma unroll
    for (int j = 0; j < CHUNK; ++j) {
        int64_t v = base + j;
        if (v >= n) break;
        if (keep[j]) {
            work[pos++] = (int32_t)v;
        } else {
            for (int k = 0; k < dim; ++k) out[k * n + v] = 0.0;
        }
    }
}

// Sorted wall distances: the reduced volume is the prefix d < dmax (first index with d >= dmax).
__global__ void reduce_prefix(const double *d, int64_t n, double dmax, int64_t *n_work)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (d[mid] < dmax) lo = mid + 1; else hi = mid;
    }
    *n_work = lo;
}

__global__ __launch_bounds__(BLOCK) void zero_tail(const int64_t *from, int64_t n, int32_t dim, double *out)
{
    int64_t start = *from;
    for (int64_t v = start + (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * BLOCK)
        for (int k = 0; k < dim; ++k) out[k * n + v] = 0.0;
}

template <int DIM, int P>
void launch_sum(const KArgs &a, dim3 grid, bool mixed, hipStream_t s)
{
    if (mixed)
        hipLaunchKernelGGL((ksum_mixed<DIM, P>), grid, dim3(BLOCK), 0, s, a);
    else
        hipLaunchKernelGGL((ksum_f64<DIM, P>), grid, dim3(BLOCK), 0, s, a);
}

template <int DIM>
void launch_sum_p(const KArgs &a, dim3 grid, int P, bool mixed, hipStream_t s)
{
    if (P == 1) launch_sum<DIM, 1>(a, grid, mixed, s);
    else if (P == 2) launch_sum<DIM, 2>(a, grid, mixed, s);
    else launch_sum<DIM, 4>(a, grid, mixed, s);
}

int env_int(const char *name, int dflt)
{
    const char *v = getenv(name);
    return v && *v ? atoi(v) : dflt;
}

}  // namespace

rbf_status run_kernel_sum(rbf_ctx ctx, const SumProblem &pb, hipStream_t s)
{
    const int DIM = pb.dim;
    if (pb.n_p == 0) return RBF_OK;
    KArgs a{};
    a.n_levels = pb.n_levels;
    int64_t n_ctrl = 0, nc_max = 0;
    for (int l = 0; l < pb.n_levels; ++l) {
        a.lv[l] = pb.lv[l];
        n_ctrl = std::max<int64_t>(n_ctrl, pb.lv[l].c_end);
        nc_max = std::max<int64_t>(nc_max, pb.lv[l].c_end - pb.lv[l].c_begin);
        a.dsupp[l] = pb.lv[l].D;
    }
    a.xp = pb.xp;
    a.ld_p = pb.n_p;
    a.dwall = pb.dwall;
    a.base = pb.base;
    a.sign = pb.sign;
    a.out = pb.out;
    a.ld_out = pb.n_p;

    DevBuf pack, work, counts, nwork, partial;
    if (n_ctrl > 0) {
        RBF_TRY(pack.get(ctx->pool.get(), sizeof(double) * 2 * DIM * n_ctrl));
        int gb = (int)std::min<int64_t>((n_ctrl + BLOCK - 1) / BLOCK, 1024);
        if (DIM == 2)
            hipLaunchKernelGGL(pack_controls<2>, dim3(gb), dim3(BLOCK), 0, s, pb.n_levels,
                               (const SumLevel *)nullptr, a, pb.xc, pb.alpha, pb.ld_ctrl, pack.as<double>());
        else
            hipLaunchKernelGGL(pack_controls<3>, dim3(gb), dim3(BLOCK), 0, s, pb.n_levels,
                               (const SumLevel *)nullptr, a, pb.xc, pb.alpha, pb.ld_ctrl, pack.as<double>());
        RBF_HIP(hipGetLastError());
    }
    a.pack = pack.as<double>();

    // Wall-distance reduction.
    if (pb.dwall) {
        double dmax = 0.0;
        for (int l = 0; l < pb.n_levels; ++l) dmax = std::max(dmax, a.dsupp[l]);
        RBF_TRY(nwork.get(ctx->pool.get(), sizeof(int64_t)));
        if (pb.sorted_by_d) {
            hipLaunchKernelGGL(reduce_prefix, dim3(1), dim3(64), 0, s, pb.dwall, pb.n_p, dmax,
                               nwork.as<int64_t>());
            int gz = (int)std::min<int64_t>((pb.n_p + BLOCK - 1) / BLOCK, 4096);
            hipLaunchKernelGGL(zero_tail, dim3(gz), dim3(BLOCK), 0, s, nwork.as<int64_t>(), pb.n_p,
                               DIM, pb.out);
            a.work = nullptr;
        } else {
            int64_t nb = (pb.n_p + CBLK - 1) / CBLK;
            RBF_TRY(counts.get(ctx->pool.get(), sizeof(int32_t) * nb));
            RBF_TRY(work.get(ctx->pool.get(), sizeof(int32_t) * pb.n_p));
            hipLaunchKernelGGL(reduce_count, dim3((unsigned)nb), dim3(BLOCK), 0, s, pb.dwall, pb.n_p,
                               dmax, counts.as<int32_t>());
            hipLaunchKernelGGL(reduce_scan, dim3(1), dim3(1024), 0, s, counts.as<int32_t>(), nb,
                               nwork.as<int64_t>());
            hipLaunchKernelGGL(reduce_scatter, dim3((unsigned)nb), dim3(BLOCK), 0, s, pb.dwall,
                               pb.n_p, dmax, counts.as<int32_t>(), work.as<int32_t>(), pb.out, DIM);
            a.work = work.as<int32_t>();
        }
        RBF_HIP(hipGetLastError());
        a.n_work_dev = nwork.as<int64_t>();
    }
    a.n_work = pb.n_p;

    // Launch shape: P points per lane; split the control lists when there are too few blocks.
    const bool mixed = pb.precision == RBF_MIXED;
    int P = env_int("RBF_KSUM_P", pb.n_p >= (int64_t)BLOCK * 2 * 4 * ctx->n_cu ? 2 : 1);
    if (P != 1 && P != 2 && P != 4) P = 2;
    int64_t nbx = (pb.n_p + (int64_t)BLOCK * P - 1) / ((int64_t)BLOCK * P);
    int64_t target = (int64_t)env_int("RBF_KSUM_BLOCKS", 8 * ctx->n_cu);
    int S = (int)std::max<int64_t>(1, std::min<int64_t>((target + nbx - 1) / nbx, nc_max / 64));
    S = std::min(S, env_int("RBF_KSUM_MAX_SPLIT", 64));
    if (const char *e = getenv("RBF_KSUM_SPLIT")) S = std::max(1, atoi(e));
    a.n_split = S;
    if (S > 1) {
        RBF_TRY(partial.get(ctx->pool.get(), sizeof(double) * (size_t)S * DIM * pb.n_p));
        a.partial = partial.as<double>();
        a.ld_part = pb.n_p;
    }
    dim3 grid((unsigned)nbx, (unsigned)S);
    hipEvent_t t0;
    ctx->timers.begin(&t0, s);
    if (DIM == 2) launch_sum_p<2>(a, grid, P, mixed, s);
    else launch_sum_p<3>(a, grid, P, mixed, s);
    RBF_HIP(hipGetLastError());
    ctx->timers.end(pb.dwall ? (mixed ? "volume_ksum_mixed" : "volume_ksum_fp64")
                             : (mixed ? "surface_ksum_mixed" : "surface_ksum_fp64"), t0, s);
    if (S > 1) {
        int gf = (int)std::min<int64_t>((pb.n_p + BLOCK - 1) / BLOCK, 8192);
        if (DIM == 2) hipLaunchKernelGGL(ksum_finalize<2>, dim3(gf), dim3(BLOCK), 0, s, a);
        else hipLaunchKernelGGL(ksum_finalize<3>, dim3(gf), dim3(BLOCK), 0, s, a);
        RBF_HIP(hipGetLastError());
    }
    pack.release_after(s);
    work.release_after(s);
    counts.release_after(s);
    nwork.release_after(s);
    partial.release_after(s);
    return RBF_OK;
}

}  // namespace rbf

// Serving: resident geometries and asynchronous deformation requests with continuous batching.
//
// Geometry. rbf_geom_create copies the surface and volume into the context's pool, computes the
// wall distance when none is given (distance to the nearest surface point), and stores the volume
// in blocks of VBLOCK points: the points are put in Z order (a space-filling curve over the
// bounding box, so each block is spatially compact), cut into blocks, the blocks are stored by
// increasing smallest wall distance, and the points inside each block by wall distance. When the
// input order is spatially local (a structured mesh), runs of ZRUN consecutive input points move
// as units instead (Z order of the runs, runs inside a block by their smallest wall distance), so
// that each 64-byte segment of the results is written by one store of one wave. The
// reduced volume of any request, {d < max D_l} (section 4), is then inside a prefix of whole
// blocks whose end the host knows from the sorted block minima, with no per-request compaction;
// every kernel-sum workgroup takes one compact block, which lets it skip the controls whose
// support misses the block, and each wave skips the levels none of its points reaches. Results
// go back through the permutation.
//
// Requests. rbf_submit copies the request and queues it. Worker slots, each with its own HIP
// stream, pull requests in arrival order as soon as they are free: a request is admitted when its
// device-memory footprint fits the part of the HBM budget that running requests have not
// reserved, and when no earlier request on the same geometry is still pending (successive icing
// steps run in order, each warm-started from the control sets its predecessor selected). Work of
// different requests overlaps on the device. Each request's kernels and launch shapes depend only
// on its own sizes, so its results are the same alone and in a mix.
#include <algorithm>
#include <cmath>

#include "basis.h"
#include "internal.h"

namespace rbf {
namespace {

constexpr int SORT_BLK = 2048;    // points per workgroup in the radix passes
constexpr int ZRUN = 8;           // consecutive input points kept together in Z order (64 output bytes)
static_assert(VBLOCK % ZRUN == 0, "blocks hold whole runs");
constexpr int NBUCKET = 256;      // 8-bit digits

// d_v = min_s ||x_v - x_s|| over the surface points (surface staged through LDS).
template <int DIM>
__global__ __launch_bounds__(256) void geo_walldist(const double *xs, int64_t n_s, const double *xv,
                                                    int64_t n_v, double *d)
{
    __shared__ double tile[256 * DIM];
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double x[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) x[k] = v < n_v ? xv[k * n_v + v] : 0.0;
    double best = 1e300;
    for (int64_t t0 = 0; t0 < n_s; t0 += 256) {
        const int nt = (int)min<int64_t>(256, n_s - t0);
        __syncthreads();
        if (threadIdx.x < nt)
#pragma unroll
            for (int k = 0; k < DIM; ++k) tile[threadIdx.x * DIM + k] = xs[k * n_s + t0 + threadIdx.x];
        __syncthreads();
        for (int j = 0; j < nt; ++j) {
            double r2 = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                const double dk = x[k] - tile[j * DIM + k];
                r2 = __builtin_fma(dk, dk, r2);
            }
            best = fmin(best, r2);
        }
    }
    if (v < n_v) d[v] = sqrt(best);
}

// Per-workgroup bounding boxes of the volume: part[blockIdx][0..DIM) = min, [DIM..2 DIM) = max.
template <int DIM>
__global__ __launch_bounds__(256) void geo_bbox(const double *xv, int64_t n, double *part)
{
    __shared__ double red[256][2 * DIM];
    double lo[DIM], hi[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        lo[k] = HUGE_VAL;
        hi[k] = -HUGE_VAL;
    }
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            lo[k] = fmin(lo[k], xv[k * n + i]);
            hi[k] = fmax(hi[k], xv[k * n + i]);
        }
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        red[threadIdx.x][k] = lo[k];
        red[threadIdx.x][DIM + k] = hi[k];
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                red[threadIdx.x][k] = fmin(red[threadIdx.x][k], red[threadIdx.x + s][k]);
                red[threadIdx.x][DIM + k] = fmax(red[threadIdx.x][DIM + k], red[threadIdx.x + s][DIM + k]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 2 * DIM) part[blockIdx.x * 2 * DIM + threadIdx.x] = red[0][threadIdx.x];
}

// Spread the low bits of v so that consecutive bits land DIM positions apart (bit interleaving
// for a Z-order key).
__device__ inline uint32_t spread2(uint32_t v)
{
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__device__ inline uint32_t spread3(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

struct Box {
    double lo[3];
    double scale[3];   // cells per unit length
};

// Z-order key of every volume point on a 2^16 x 2^16 (2D) or 2^10 x 2^10 x 2^10 (3D) grid over
// the bounding box; idx = the point's index. With runs, the key is taken per run of ZRUN
// consecutive input points (the key of the run's first point), so that the stable sort keeps each
// run whole and in order; the last, partial run then takes the largest key (it sorts last and
// shifts no later run off its alignment).
template <int DIM>
__global__ __launch_bounds__(256) void geo_morton(const double *xv, int64_t n, Box box, int32_t runs,
                                                  uint32_t *key, int32_t *idx)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t r = runs ? (i / ZRUN) * ZRUN : i;
    uint32_t m = 0xffffffffu;
    if (!runs || r + ZRUN <= n) {
        constexpr double top = DIM == 2 ? 65535.0 : 1023.0;
        uint32_t q[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k)
            q[k] = (uint32_t)fmin(top, fmax(0.0, (xv[k * n + r] - box.lo[k]) * box.scale[k]));
        if (DIM == 2) m = spread2(q[0]) | (spread2(q[1]) << 1);
        else m = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[DIM - 1]) << 2);
    }
    key[i] = m;
    idx[i] = (int32_t)i;
}

// Diagonal of the bounding box of every block of VBLOCK points in the point-wise Z order (idx:
// input index at each sorted position; the last block may be partial). One workgroup per block.
template <int DIM>
__global__ __launch_bounds__(256) void geo_blockdiag(const int32_t *idx, const double *xv, int64_t n, double *diag)
{
    __shared__ double red[4][2 * DIM];
    const int64_t b0 = (int64_t)blockIdx.x * VBLOCK;
    double lo[DIM], hi[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        lo[k] = HUGE_VAL;
        hi[k] = -HUGE_VAL;
    }
    for (int j = threadIdx.x; j < VBLOCK && b0 + j < n; j += 256) {
        const int64_t i = idx[b0 + j];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            lo[k] = fmin(lo[k], xv[k * n + i]);
            hi[k] = fmax(hi[k], xv[k * n + i]);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            lo[k] = fmin(lo[k], __shfl_xor(lo[k], off, 64));
            hi[k] = fmax(hi[k], __shfl_xor(hi[k], off, 64));
        }
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            red[threadIdx.x >> 6][k] = lo[k];
            red[threadIdx.x >> 6][DIM + k] = hi[k];
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        double d2 = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const double l = fmin(fmin(red[0][k], red[1][k]), fmin(red[2][k], red[3][k]));
            const double h = fmax(fmax(red[0][DIM + k], red[1][DIM + k]), fmax(red[2][DIM + k], red[3][DIM + k]));
            d2 += (h - l) * (h - l);
        }
        diag[blockIdx.x] = sqrt(d2);
    }
}

// pos[idx[p]] = p: each input point's position in the point-wise Z order.
__global__ __launch_bounds__(256) void geo_position(const int32_t *idx, int64_t n, int32_t *pos)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < n) pos[idx[p]] = (int32_t)p;
}

// Runs of ZRUN consecutive input points that are spatially local: the diagonal of the run's box
// at most twice that of the point-wise block holding the run's first point. Counted into *local.
template <int DIM>
__global__ __launch_bounds__(256) void geo_runlocal(const double *xv, int64_t n, const int32_t *pos,
                                                    const double *diag, unsigned long long *local)
{
    __shared__ int32_t red[4];
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int32_t ok = 0;
    if ((r + 1) * ZRUN <= n) {
        double d2 = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double lo = HUGE_VAL, hi = -HUGE_VAL;
            for (int j = 0; j < ZRUN; ++j) {
                const double x = xv[k * n + r * ZRUN + j];
                lo = fmin(lo, x);
                hi = fmax(hi, x);
            }
            d2 += (hi - lo) * (hi - lo);
        }
        const double bd = diag[pos[r * ZRUN] / VBLOCK];
        ok = d2 <= 4.0 * bd * bd;
    }
    for (int off = 32; off > 0; off >>= 1) ok += __shfl_xor(ok, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ok;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicAdd(local, (unsigned long long)(red[0] + red[1] + red[2] + red[3]));
}

// Per-workgroup digit histograms, stored digit-major: hist[digit * nblk + block].
__global__ __launch_bounds__(256) void radix_hist(const uint32_t *key, int64_t n, int shift, int32_t *hist,
                                                  int64_t nblk)
{
    __shared__ int32_t h[NBUCKET];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SORT_BLK;
    for (int j = threadIdx.x; j < SORT_BLK; j += 256)
        if (base + j < n) atomicAdd(&h[(key[base + j] >> shift) & (NBUCKET - 1)], 1);
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of the digit-major histogram table by one workgroup (fixed order).
__global__ __launch_bounds__(1024) void radix_scan(int32_t *hist, int64_t m)
{
    __shared__ int64_t part[1024];
    const int64_t per = (m + 1023) / 1024;
    const int64_t b0 = min<int64_t>(m, threadIdx.x * per), b1 = min<int64_t>(m, b0 + per);
    int64_t s = 0;
    for (int64_t i = b0; i < b1; ++i) s += hist[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int t = 0; t < 1024; ++t) {
            const int64_t v = part[t];
            part[t] = run;
            run += v;
        }
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int64_t i = b0; i < b1; ++i) {
        const int32_t v = hist[i];
        hist[i] = (int32_t)run;
        run += v;
    }
}

// Stable scatter of one radix pass: positions are assigned in index order inside each block (one
// lane walks the block), then all lanes move the (key, index) pairs.
__global__ __launch_bounds__(256) void radix_place(const uint32_t *key_in, const int32_t *idx_in, int64_t n,
                                                   int shift, const int32_t *off, int64_t nblk,
                                                   uint32_t *key_out, int32_t *idx_out)
{
    __shared__ int32_t cur[NBUCKET];
    __shared__ int32_t pos[SORT_BLK];
    const int64_t base = (int64_t)blockIdx.x * SORT_BLK;
    const int cnt = (int)min<int64_t>(SORT_BLK, n - base);
    cur[threadIdx.x] = off[(int64_t)threadIdx.x * nblk + blockIdx.x];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int j = 0; j < cnt; ++j) pos[j] = cur[(key_in[base + j] >> shift) & (NBUCKET - 1)]++;
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += 256) {
        key_out[pos[j]] = key_in[base + j];
        idx_out[pos[j]] = idx_in[base + j];
    }
}

// Smallest wall distance of each run of VBLOCK points in Z order.
__global__ __launch_bounds__(256) void geo_blockmin(const double *d, const int32_t *idx, int64_t n, double *bmin)
{
    __shared__ double red[256];
    const int64_t b0 = (int64_t)blockIdx.x * VBLOCK;
    double m = HUGE_VAL;
    for (int j = threadIdx.x; j < VBLOCK; j += 256)
        if (b0 + j < n) m = fmin(m, d[idx[b0 + j]]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) bmin[blockIdx.x] = red[0];
}

// Final layout: stored block r is Z-order block border[r]; slots past the end of the volume are
// padding (perm -1, d = +inf, so psi = 0 and nothing is written for them).
template <int DIM>
__global__ __launch_bounds__(256) void geo_gather(const int32_t *border, const int32_t *zidx, const double *d,
                                                  const double *xv, int64_t n, int64_t n_pad, int32_t *perm,
                                                  double *d_sorted, double *x_sorted)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n_pad) return;
    const int64_t src = (int64_t)border[j / VBLOCK] * VBLOCK + j % VBLOCK;
    if (src < n) {
        const int32_t v = zidx[src];
        perm[j] = v;
        d_sorted[j] = d[v];
#pragma unroll
        for (int k = 0; k < DIM; ++k) x_sorted[k * n_pad + j] = xv[k * n + v];
    } else {
        perm[j] = -1;
        d_sorted[j] = HUGE_VAL;
#pragma unroll
        for (int k = 0; k < DIM; ++k) x_sorted[k * n_pad + j] = 0.0;
    }
}

// Point-wise layout: inside every stored block, order the points by wall distance (ties by slot,
// so by Z order): a wave then holds points of similar distance, and one whose points all lie at
// or beyond a level's support distance skips that level. One workgroup per block, bitonic sort in
// LDS.
template <int DIM>
__global__ __launch_bounds__(256) void geo_pointsort(int32_t *perm, double *d_sorted, double *x_sorted,
                                                     int64_t n_pad)
{
    static_assert(VBLOCK == 512, "two keys per lane");
    __shared__ double key[VBLOCK];
    __shared__ int32_t slot[VBLOCK];
    const int64_t b0 = (int64_t)blockIdx.x * VBLOCK;
    const int t = threadIdx.x;
    for (int j = t; j < VBLOCK; j += 256) {
        key[j] = d_sorted[b0 + j];
        slot[j] = j;
    }
    __syncthreads();
    for (int k = 2; k <= VBLOCK; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int i = (t / j) * 2 * j + (t % j), q = i + j;
            const bool up = (i & k) == 0;
            const bool gt = key[i] > key[q] || (key[i] == key[q] && slot[i] > slot[q]);
            if (gt == up) {
                const double kv = key[i];
                key[i] = key[q];
                key[q] = kv;
                const int32_t sv = slot[i];
                slot[i] = slot[q];
                slot[q] = sv;
            }
            __syncthreads();
        }
    int32_t pv[2];
    double dv[2], xvv[2][DIM];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int64_t src = b0 + slot[t + 256 * r];
        pv[r] = perm[src];
        dv[r] = d_sorted[src];
#pragma unroll
        for (int k = 0; k < DIM; ++k) xvv[r][k] = x_sorted[k * n_pad + src];
    }
    __syncthreads();   // every read of the block is done before any slot is overwritten
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int64_t dst = b0 + t + 256 * r;
        perm[dst] = pv[r];
        d_sorted[dst] = dv[r];
#pragma unroll
        for (int k = 0; k < DIM; ++k) x_sorted[k * n_pad + dst] = xvv[r][k];
    }
}

// Run layout: inside every stored block, order its runs of ZRUN points by their smallest wall
// distance (ties by position, so by Z order), each run kept whole and in input order: a wave then
// holds points of similar distance, and one whose points all lie at or beyond a level's support
// distance skips that level; its stores cover whole 64-byte segments. One workgroup per block.
template <int DIM>
__global__ __launch_bounds__(256) void geo_runsort(int32_t *perm, double *d_sorted, double *x_sorted,
                                                     int64_t n_pad)
{
    static_assert(VBLOCK == 512, "two slots per lane");
    constexpr int NRUN = VBLOCK / ZRUN;
    __shared__ double rmin[NRUN];
    __shared__ int32_t rank[NRUN];
    const int64_t b0 = (int64_t)blockIdx.x * VBLOCK;
    const int t = threadIdx.x;
    if (t < NRUN) {
        double m = HUGE_VAL;
        for (int j = 0; j < ZRUN; ++j) m = fmin(m, d_sorted[b0 + t * ZRUN + j]);
        rmin[t] = m;
    }
    __syncthreads();
    if (t < NRUN) {
        int r = 0;
        for (int q = 0; q < NRUN; ++q) r += rmin[q] < rmin[t] || (rmin[q] == rmin[t] && q < t);
        rank[t] = r;
    }
    __syncthreads();
    int32_t pv[2];
    double dv[2], xvv[2][DIM];
    int64_t dst[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int j = t + 256 * r;
        const int64_t src = b0 + j;
        dst[r] = b0 + rank[j / ZRUN] * ZRUN + j % ZRUN;
        pv[r] = perm[src];
        dv[r] = d_sorted[src];
#pragma unroll
        for (int k = 0; k < DIM; ++k) xvv[r][k] = x_sorted[k * n_pad + src];
    }
    __syncthreads();   // every read of the block is done before any slot is overwritten
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        perm[dst[r]] = pv[r];
        d_sorted[dst[r]] = dv[r];
#pragma unroll
        for (int k = 0; k < DIM; ++k) x_sorted[k * n_pad + dst[r]] = xvv[r][k];
    }
}

// Box (min, max per coordinate) of every BOXROWS consecutive stored points, padding excluded
// (all padding: an empty box, min +inf and max -inf). One wave per box.
template <int DIM>
__global__ __launch_bounds__(256) void geo_blockbox(const int32_t *perm, const double *x_sorted, int64_t n_pad,
                                                    double *box)
{
    static_assert(BOXROWS == 64, "one row per lane");
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;   // n_pad is a multiple of 256
    const bool pt = perm[j] >= 0;
    double lo[DIM], hi[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const double x = x_sorted[k * n_pad + j];
        lo[k] = pt ? x : HUGE_VAL;
        hi[k] = pt ? x : -HUGE_VAL;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            lo[k] = fmin(lo[k], __shfl_xor(lo[k], off));
            hi[k] = fmax(hi[k], __shfl_xor(hi[k], off));
        }
    const int lane = threadIdx.x & 63;
    double *b = box + (j / BOXROWS) * 2 * DIM;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        if (lane == k) b[k] = lo[k];
        if (lane == DIM + k) b[DIM + k] = hi[k];
    }
}

template <int DIM>
rbf_status build_geometry(rbf_ctx ctx, Geometry &g, const double *xs, const double *xv,
                          const double *dwall, hipStream_t s)
{
    Pool *pool = ctx->pool.get();
    const int64_t n_s = g.n_s, n_v = g.n_v;
    const int64_t nb = (n_v + VBLOCK - 1) / VBLOCK;
    const int64_t n_pad = nb * VBLOCK;
    g.n_pad = n_pad;
    g.block_dmin.clear();
    RBF_TRY(g.xs.get(pool, sizeof(double) * DIM * n_s, s));
    RBF_HIP(hipMemcpyAsync(g.xs.ptr, xs, sizeof(double) * DIM * n_s, hipMemcpyDeviceToDevice, s));
    RBF_TRY(g.xv_sorted.get(pool, sizeof(double) * DIM * std::max<int64_t>(1, n_pad), s));
    RBF_TRY(g.d_sorted.get(pool, sizeof(double) * std::max<int64_t>(1, n_pad), s));
    RBF_TRY(g.perm.get(pool, sizeof(int32_t) * std::max<int64_t>(1, n_pad), s));
    g.bytes = sizeof(double) * (DIM * (n_s + n_pad) + n_pad + 2 * DIM * (n_pad / BOXROWS)) + sizeof(int32_t) * n_pad;
    if (n_v == 0) {
        RBF_HIP(hipStreamSynchronize(s));
        settle_all(g.xs, g.xv_sorted, g.d_sorted, g.perm);
        return RBF_OK;
    }
    DevBuf dtmp, part, k0, k1, i0, i1, hist, bmin, border;
    const double *d = dwall;
    if (!d) {
        RBF_TRY(dtmp.get(pool, sizeof(double) * n_v, s));
        hipLaunchKernelGGL(geo_walldist<DIM>, dim3((unsigned)((n_v + 255) / 256)), dim3(256), 0, s,
                           g.xs.as<double>(), n_s, xv, n_v, dtmp.as<double>());
        RBF_HIP(hipGetLastError());
        d = dtmp.as<double>();
    }
    // Z-order keys over the volume's bounding box.
    const int gb = (int)std::min<int64_t>((n_v + 255) / 256, 512);
    RBF_TRY(part.get(pool, sizeof(double) * 2 * DIM * gb, s));
    hipLaunchKernelGGL(geo_bbox<DIM>, dim3(gb), dim3(256), 0, s, xv, n_v, part.as<double>());
    std::vector<double> ph((size_t)2 * DIM * gb);
    RBF_HIP(hipMemcpyAsync(ph.data(), part.ptr, sizeof(double) * ph.size(), hipMemcpyDeviceToHost, s));
    RBF_HIP(hipStreamSynchronize(s));
    Box box{};
    for (int k = 0; k < DIM; ++k) {
        double lo = HUGE_VAL, hi = -HUGE_VAL;
        for (int b = 0; b < gb; ++b) {
            lo = std::min(lo, ph[(size_t)b * 2 * DIM + k]);
            hi = std::max(hi, ph[(size_t)b * 2 * DIM + DIM + k]);
        }
        if (!std::isfinite(lo) || !std::isfinite(hi)) return fail(RBF_E_INVALID, "volume coordinates not finite");
        box.lo[k] = lo;
        box.scale[k] = hi > lo ? (DIM == 2 ? 65536.0 : 1024.0) / (hi - lo) : 0.0;
    }
    RBF_TRY(k0.get(pool, sizeof(uint32_t) * n_v, s));
    RBF_TRY(k1.get(pool, sizeof(uint32_t) * n_v, s));
    RBF_TRY(i0.get(pool, sizeof(int32_t) * n_v, s));
    RBF_TRY(i1.get(pool, sizeof(int32_t) * n_v, s));
    const int64_t nblk = (n_v + SORT_BLK - 1) / SORT_BLK;
    RBF_TRY(hist.get(pool, sizeof(int32_t) * NBUCKET * nblk, s));
    const unsigned gv = (unsigned)((n_v + 255) / 256);
    // Stable LSD radix sort of (key, index) by Z-order key, four 8-bit passes; the result is back
    // in k0 / i0.
    auto zsort = [&](int32_t runs) {
        hipLaunchKernelGGL(geo_morton<DIM>, dim3(gv), dim3(256), 0, s, xv, n_v, box, runs, k0.as<uint32_t>(),
                           i0.as<int32_t>());
        DevBuf *kin = &k0, *kout = &k1, *iin = &i0, *iout = &i1;
        for (int shift = 0; shift < 32; shift += 8) {
            hipLaunchKernelGGL(radix_hist, dim3((unsigned)nblk), dim3(256), 0, s, kin->as<const uint32_t>(), n_v,
                               shift, hist.as<int32_t>(), nblk);
            hipLaunchKernelGGL(radix_scan, dim3(1), dim3(1024), 0, s, hist.as<int32_t>(), (int64_t)NBUCKET * nblk);
            hipLaunchKernelGGL(radix_place, dim3((unsigned)nblk), dim3(256), 0, s, kin->as<const uint32_t>(),
                               iin->as<const int32_t>(), n_v, shift, hist.as<const int32_t>(), nblk,
                               kout->as<uint32_t>(), iout->as<int32_t>());
            std::swap(kin, kout);
            std::swap(iin, iout);
        }
    };
    zsort(0);
    // Runs of ZRUN consecutive input points are kept whole when the input order is spatially
    // local (structured meshes): at least 80% of the runs span at most twice the diagonal of the
    // point-wise block that holds their first point. Then every output line is written by one
    // wave. Otherwise (scattered input order) the point-wise order stands.
    bool runs = false;
    const int64_t n_runs = n_v / ZRUN;
    if (n_runs >= 64) {
        DevBuf local, diag;
        RBF_TRY(local.get(pool, sizeof(unsigned long long), s));
        RBF_TRY(diag.get(pool, sizeof(double) * nb, s));
        RBF_HIP(hipMemsetAsync(local.ptr, 0, sizeof(unsigned long long), s));
        hipLaunchKernelGGL(geo_blockdiag<DIM>, dim3((unsigned)nb), dim3(256), 0, s, i0.as<const int32_t>(), xv, n_v,
                           diag.as<double>());
        hipLaunchKernelGGL(geo_position, dim3(gv), dim3(256), 0, s, i0.as<const int32_t>(), n_v, i1.as<int32_t>());
        hipLaunchKernelGGL(geo_runlocal<DIM>, dim3((unsigned)((n_runs + 255) / 256)), dim3(256), 0, s, xv, n_v,
                           i1.as<const int32_t>(), diag.as<const double>(), local.as<unsigned long long>());
        unsigned long long nl = 0;
        RBF_HIP(hipMemcpyAsync(&nl, local.ptr, sizeof nl, hipMemcpyDeviceToHost, s));
        RBF_HIP(hipStreamSynchronize(s));
        settle_all(local, diag);
        runs = (double)nl >= 0.8 * (double)n_runs;
        if (runs) zsort(1);
    }
    g.run_layout = runs;
    RBF_HIP(hipGetLastError());
    DevBuf *iin = &i0;
    // Blocks of VBLOCK points in Z order, stored by increasing smallest wall distance: the
    // points of any support distance D then lie in a prefix of whole blocks.
    RBF_TRY(bmin.get(pool, sizeof(double) * nb, s));
    hipLaunchKernelGGL(geo_blockmin, dim3((unsigned)nb), dim3(256), 0, s, d, iin->as<const int32_t>(), n_v,
                       bmin.as<double>());
    std::vector<double> bm(nb);
    RBF_HIP(hipMemcpyAsync(bm.data(), bmin.ptr, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    RBF_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> order(nb);
    for (int64_t b = 0; b < nb; ++b) order[b] = (int32_t)b;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return bm[a] < bm[b]; });
    g.block_dmin.resize(nb);
    for (int64_t r = 0; r < nb; ++r) g.block_dmin[r] = bm[order[r]];
    RBF_TRY(border.get(pool, sizeof(int32_t) * nb, s));
    RBF_HIP(hipMemcpyAsync(border.ptr, order.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(geo_gather<DIM>, dim3((unsigned)((n_pad + 255) / 256)), dim3(256), 0, s,
                       border.as<const int32_t>(), iin->as<const int32_t>(), d, xv, n_v, n_pad,
                       g.perm.as<int32_t>(), g.d_sorted.as<double>(), g.xv_sorted.as<double>());
    if (runs)
        hipLaunchKernelGGL(geo_runsort<DIM>, dim3((unsigned)nb), dim3(256), 0, s, g.perm.as<int32_t>(),
                           g.d_sorted.as<double>(), g.xv_sorted.as<double>(), n_pad);
    else
        hipLaunchKernelGGL(geo_pointsort<DIM>, dim3((unsigned)nb), dim3(256), 0, s, g.perm.as<int32_t>(),
                           g.d_sorted.as<double>(), g.xv_sorted.as<double>(), n_pad);
    RBF_TRY(g.block_box.get(pool, sizeof(double) * 2 * DIM * (n_pad / BOXROWS), s));
    hipLaunchKernelGGL(geo_blockbox<DIM>, dim3((unsigned)(n_pad / 256)), dim3(256), 0, s, g.perm.as<const int32_t>(),
                       g.xv_sorted.as<const double>(), n_pad, g.block_box.as<double>());
    RBF_HIP(hipGetLastError());
    RBF_HIP(hipStreamSynchronize(s));
    settle_all(g.xs, g.xv_sorted, g.d_sorted, g.perm, g.block_box, dtmp, part, k0, k1, i0, i1, hist, bmin, border);
    return RBF_OK;
}

// Reduced volume for support distance D: the stored blocks whose smallest wall distance is
// below D (a prefix, in points).
int64_t prefix_for(const Geometry &g, double D)
{
    const auto it = std::lower_bound(g.block_dmin.begin(), g.block_dmin.end(), D);
    return (int64_t)(it - g.block_dmin.begin()) * VBLOCK;
}

// Work of each row group of a resident kernel sum (one workgroup per group of `rows` stored
// rows): the controls the workgroup will keep (those within R_l of the group's box, with the
// kernel's margin), summed over the levels whose support distance reaches the group (its smallest
// wall distance is below D_l). That is the length of the workgroup's pair loop: its waves run
// side by side on the compute unit's SIMDs.
struct OrderLevels {
    int32_t n_levels;
    double inv_r[RBF_MAX_LEVELS], D[RBF_MAX_LEVELS];
    int64_t c_begin[RBF_MAX_LEVELS], c_end[RBF_MAX_LEVELS];
};

template <int DIM>
__global__ __launch_bounds__(256) void geo_group_weight(const double *xc, int64_t ld_ctrl, const double *box,
                                                        const double *d_sorted, int rows, OrderLevels lv,
                                                        double *weight)
{
    __shared__ int32_t red[4][RBF_MAX_LEVELS];
    __shared__ double dred[4];
    const int64_t r0 = (int64_t)blockIdx.x * rows;
    double dm = HUGE_VAL;   // the group's smallest wall distance
    for (int j = threadIdx.x; j < rows; j += 256) dm = fmin(dm, d_sorted[r0 + j]);
    for (int off = 32; off > 0; off >>= 1) dm = fmin(dm, __shfl_xor(dm, off, 64));
    if ((threadIdx.x & 63) == 0) dred[threadIdx.x >> 6] = dm;
    __syncthreads();
    const double dmin = fmin(fmin(dred[0], dred[1]), fmin(dred[2], dred[3]));
    double lo[DIM], hi[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        lo[k] = HUGE_VAL;
        hi[k] = -HUGE_VAL;
    }
    for (int b = 0; b < rows / BOXROWS; ++b) {
        const double *bb = box + (r0 / BOXROWS + b) * 2 * DIM;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            lo[k] = fmin(lo[k], bb[k]);
            hi[k] = fmax(hi[k], bb[DIM + k]);
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int l = 0; l < lv.n_levels; ++l) {
        int32_t kept = 0;
        if (dmin < lv.D[l])
            for (int64_t c = lv.c_begin[l] + threadIdx.x; c < lv.c_end[l]; c += 256) {
                double d2 = 0.0;
#pragma unroll
                for (int k = 0; k < DIM; ++k) {
                    const double x = xc[k * ld_ctrl + c];
                    const double e = x < lo[k] ? lo[k] - x : (x > hi[k] ? x - hi[k] : 0.0);
                    d2 = __builtin_fma(e, e, d2);
                }
                kept += d2 * (lv.inv_r[l] * lv.inv_r[l]) < 1.00020001 ? 1 : 0;
            }
        for (int off = 32; off > 0; off >>= 1) kept += __shfl_xor(kept, off, 64);
        if (lane == 0) red[w][l] = kept;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double wt = 0.0;
        for (int l = 0; l < lv.n_levels; ++l) wt += (double)(red[0][l] + red[1][l] + red[2][l] + red[3][l]);
        weight[blockIdx.x] = wt;
    }
}

uint64_t greedy_footprint(int dim, int64_t n_s, int64_t cap)
{
    const uint64_t cols = (uint64_t)std::min<int64_t>(n_s, cap);
    const uint64_t rows = (uint64_t)((n_s + 63) / 64) * 64;   // the basis keeps whole 64-point tiles
    const uint64_t lda = (cols + 63) / 64 * 64;
    return sizeof(double) * (2 * ((cols + 1) * rows + cols * (cols + 1) / 2) + (uint64_t)(3 * dim + 1) * n_s +
                             (uint64_t)(dim + 1) * cols + 2 * (uint64_t)cap) +
           (uint64_t)n_s * 17 + sizeof(int64_t) * (uint64_t)cap + sizeof(double) * (uint64_t)cap * 2 * dim +
           sizeof(double) * ((uint64_t)dim * n_s + (uint64_t)n_s / 256 + 1) +   // FP32 error check
           sizeof(double) * (uint64_t)dim * n_s + 16 * (uint64_t)(n_s / 64 + 1) +  // persistent form's second buffers
           sizeof(double) * (lda * lda + 64 * lda + (uint64_t)dim * cols) + 256;    // seeded start's dense factor
}

}  // namespace

rbf_status resident_order(rbf_ctx ctx, Geometry &g, const SumProblem &pb, int P, int64_t n_groups,
                          hipStream_t s, const int32_t **order)
{
    *order = nullptr;
    const int rows = 256 * P;
    if (n_groups * rows != g.n_pad || pb.n_levels < 1 || pb.n_levels > RBF_MAX_LEVELS) return RBF_OK;
    std::lock_guard<std::mutex> lk(g.order_mu);
    for (const Geometry::GroupOrder &o : g.orders) {
        bool same = o.P == P && o.n_levels == pb.n_levels;
        for (int l = 0; same && l < pb.n_levels; ++l)
            same = o.inv_r[l] == pb.lv[l].inv_r && o.D[l] == pb.lv[l].D;
        if (same) {
            *order = o.order.as<const int32_t>();
            return RBF_OK;
        }
    }
    if (g.orders.size() >= 16) return RBF_OK;   // many distinct requests: stored order
    OrderLevels lv{};
    lv.n_levels = pb.n_levels;
    for (int l = 0; l < pb.n_levels; ++l) {
        lv.inv_r[l] = pb.lv[l].inv_r;
        lv.D[l] = pb.lv[l].D;
        lv.c_begin[l] = pb.lv[l].c_begin;
        lv.c_end[l] = pb.xc ? pb.lv[l].c_end : pb.lv[l].c_begin;
    }
    DevBuf bw;
    RBF_TRY(bw.get(ctx->pool.get(), sizeof(double) * (size_t)n_groups, s));
    if (g.dim == 2)
        hipLaunchKernelGGL(geo_group_weight<2>, dim3((unsigned)n_groups), dim3(256), 0, s, pb.xc, pb.ld_ctrl,
                           g.block_box.as<const double>(), g.d_sorted.as<const double>(), rows, lv, bw.as<double>());
    else
        hipLaunchKernelGGL(geo_group_weight<3>, dim3((unsigned)n_groups), dim3(256), 0, s, pb.xc, pb.ld_ctrl,
                           g.block_box.as<const double>(), g.d_sorted.as<const double>(), rows, lv, bw.as<double>());
    RBF_HIP(hipGetLastError());
    std::vector<double> wt((size_t)n_groups);
    RBF_HIP(hipMemcpyAsync(wt.data(), bw.ptr, sizeof(double) * (size_t)n_groups, hipMemcpyDeviceToHost, s));
    RBF_HIP(hipStreamSynchronize(s));
    bw.settle();
    // Heaviest first (stored order among equals), dealt to the compute units back and forth:
    // workgroup x runs on unit x mod n_cu, every workgroup resident at once.
    std::vector<int32_t> rank((size_t)n_groups);
    for (int64_t i = 0; i < n_groups; ++i) rank[(size_t)i] = (int32_t)i;
    std::stable_sort(rank.begin(), rank.end(), [&](int32_t x, int32_t y) { return wt[(size_t)x] > wt[(size_t)y]; });
    const int64_t ncu = std::max(1, ctx->n_cu);
    std::vector<int32_t> ord((size_t)n_groups, -1);
    for (int64_t k = 0; k < n_groups; ++k) {
        const int64_t r = k / ncu, c = k % ncu;
        const bool whole = (r + 1) * ncu <= n_groups;   // the last, partial round is not reversed
        const int64_t x = r * ncu + ((r & 1) && whole ? ncu - 1 - c : c);
        ord[(size_t)x] = rank[(size_t)k];
    }
    std::vector<uint8_t> seen((size_t)n_groups, 0);
    for (int32_t v : ord) {
        if (v < 0 || v >= n_groups || seen[(size_t)v]) return fail(RBF_E_DEVICE, "row-group order is not a permutation");
        seen[(size_t)v] = 1;
    }
    Geometry::GroupOrder o;
    o.P = P;
    o.n_levels = pb.n_levels;
    for (int l = 0; l < pb.n_levels; ++l) {
        o.inv_r[l] = pb.lv[l].inv_r;
        o.D[l] = pb.lv[l].D;
    }
    RBF_TRY(o.order.get(ctx->pool.get(), sizeof(int32_t) * (size_t)n_groups));
    RBF_HIP(hipMemcpyAsync(o.order.ptr, ord.data(), sizeof(int32_t) * (size_t)n_groups, hipMemcpyHostToDevice, s));
    RBF_HIP(hipStreamSynchronize(s));
    *order = o.order.as<const int32_t>();
    g.orders.push_back(std::move(o));
    return RBF_OK;
}

// ---- server ---------------------------------------------------------------------------------
struct Req {
    rbf_ticket id = 0;
    rbf_request r{};
    std::vector<int64_t> seed_idx;
    std::vector<int32_t> seed_off;
    Geometry *g = nullptr;
    rbf_geom handle = nullptr;
    int32_t state = RBF_REQ_QUEUED;
    rbf_status result = RBF_OK;
    double t_arrive = 0, t_admit = 0, t_start = 0, t_done = 0;
    uint64_t reserve = 0;
};

class Server {
  public:
    explicit Server(rbf_ctx ctx, int n_slots) : ctx_(ctx)
    {
        for (int i = 0; i < n_slots; ++i) {
            hipStream_t s = nullptr;
            (void)hipSetDevice(ctx->device);
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) break;
            streams_.push_back(s);
        }
        for (size_t i = 0; i < streams_.size(); ++i) workers_.emplace_back([this, i] { work(i); });
    }
    ~Server()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
            for (Req *q : queue_) {
                q->state = RBF_REQ_FAILED;
                q->result = fail(RBF_E_DEVICE, "context destroyed before the request ran");
            }
            queue_.clear();
        }
        cv_.notify_all();
        for (auto &t : workers_) t.join();
        for (auto s : streams_) (void)hipStreamDestroy(s);
    }
    bool ok() const { return !streams_.empty(); }

    rbf_status submit(std::unique_ptr<Req> q, rbf_ticket *out)
    {
        std::lock_guard<std::mutex> lk(mu_);
        q->id = ++next_id_;
        q->t_arrive = now_seconds();
        q->g->refs += 1;
        *out = q->id;
        queue_.push_back(q.get());
        reqs_[q->id] = std::move(q);
        cv_.notify_all();
        return RBF_OK;
    }

    rbf_status poll(rbf_ticket t, rbf_req_info *info, bool wait)
    {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = reqs_.find(t);
        if (it == reqs_.end()) return fail(RBF_E_NOT_FOUND, "unknown ticket %llu", (unsigned long long)t);
        Req *q = it->second.get();
        if (wait)
            done_cv_.wait(lk, [&] { return q->state == RBF_REQ_DONE || q->state == RBF_REQ_FAILED; });
        info->state = q->state;
        info->result = q->result;
        info->t_arrive = q->t_arrive;
        info->t_admit = q->t_admit;
        info->t_start = q->t_start;
        info->t_done = q->t_done;
        if (wait) reqs_.erase(it);
        return RBF_OK;
    }

    bool geometry_busy(Geometry *g)
    {
        std::lock_guard<std::mutex> lk(mu_);
        return g->refs > 0;
    }

  private:
    // First admissible request in arrival order: its geometry has no earlier pending request and
    // its footprint fits the unreserved budget. An earlier request that does not fit the memory
    // blocks the later ones (no starvation of large requests).
    Req *pick_locked()
    {
        const uint64_t budget = ctx_->pool->budget();
        std::vector<Geometry *> blocked;
        for (auto it = queue_.begin(); it != queue_.end(); ++it) {
            Req *q = *it;
            if (std::find(blocked.begin(), blocked.end(), q->g) != blocked.end() || q->g->running) {
                blocked.push_back(q->g);
                continue;
            }
            // Resident bases of idle geometries yield to an admitted request's working memory.
            while (reserved_ + q->reserve + cache_total_ > budget) {
                Geometry *victim = nullptr;
                for (Geometry *o : cached_)
                    if (o != q->g && !o->running && (!victim || o->last_use < victim->last_use)) victim = o;
                if (!victim) break;
                cache_total_ -= victim->cache_bytes;
                victim->levels.clear();
                victim->cache_bytes = 0;
                cached_.erase(std::find(cached_.begin(), cached_.end(), victim));
            }
            if (reserved_ + q->reserve + cache_total_ > budget) return nullptr;
            queue_.erase(it);
            return q;
        }
        return nullptr;
    }

    void work(size_t slot)
    {
        (void)hipSetDevice(ctx_->device);
        hipStream_t s = streams_[slot];
        for (;;) {
            Req *q = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || (q = pick_locked()) != nullptr; });
                if (!q) return;   // stopping
                reserved_ += q->reserve;
                q->g->running = true;
                q->state = RBF_REQ_RUNNING;
                q->t_admit = now_seconds();
            }
            q->t_start = now_seconds();
            const rbf_status st = run(*q, s);
            {
                std::lock_guard<std::mutex> lk(mu_);
                q->t_done = now_seconds();
                q->result = st;
                q->state = st < 0 ? RBF_REQ_FAILED : RBF_REQ_DONE;
                reserved_ -= q->reserve;
                q->g->running = false;
                q->g->refs -= 1;
            }
            cv_.notify_all();
            done_cv_.notify_all();
        }
    }

    rbf_status run(Req &q, hipStream_t s);

  public:
    void keep_bases(Geometry &g, std::vector<LevelCache> &&fresh);
    void forget(Geometry *g);

  private:
    uint64_t cache_limit() const
    {
        const char *e = getenv("RBF_CACHE_FRACTION");
        const double f = e ? atof(e) : 0.4;
        return (uint64_t)(f * (double)ctx_->pool->budget());
    }
    std::vector<Geometry *> cached_;
    uint64_t cache_total_ = 0;

    rbf_ctx ctx_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    std::deque<Req *> queue_;
    std::unordered_map<rbf_ticket, std::unique_ptr<Req>> reqs_;
    std::vector<hipStream_t> streams_;
    std::vector<std::thread> workers_;
    uint64_t reserved_ = 0;
    rbf_ticket next_id_ = 0;
    bool stop_ = false;
};

rbf_status Server::run(Req &q, hipStream_t s)
{
    Geometry &g = *q.g;
    const rbf_greedy_params &p0 = q.r.params;
    rbf_greedy_params p = p0;
    // Warm start: seed every level with the control set the previous request on this geometry
    // selected (if it fits the cap); otherwise the request's own seeds.
    std::vector<int64_t> wseed;
    std::vector<int32_t> woff;
    if (q.r.warm_start && (int)g.last_ctrl.size() == p.n_levels) {
        woff.assign(p.n_levels + 1, 0);
        for (int l = 0; l < p.n_levels; ++l) {
            for (int64_t c : g.last_ctrl[l]) wseed.push_back(c);
            woff[l + 1] = (int32_t)wseed.size();
        }
        if ((int64_t)wseed.size() <= p.max_ctrl_total && !wseed.empty()) {
            p.seed_idx = wseed.data();
            p.seed_off = woff.data();
        }
    } else if (!q.seed_off.empty()) {
        p.seed_idx = q.seed_idx.data();
        p.seed_off = q.seed_off.data();
    } else {
        p.seed_idx = nullptr;
        p.seed_off = nullptr;
    }
    const int dim = p.dim;
    const int64_t cap = p.max_ctrl_total;
    rbf_ctrl_set local{};
    rbf_ctrl_set *cs = q.r.out;
    DevBuf bi, bx, ba;
    if (!cs) {
        RBF_TRY(bi.get(ctx_->pool.get(), sizeof(int64_t) * cap, s));
        RBF_TRY(bx.get(ctx_->pool.get(), sizeof(double) * dim * cap, s));
        RBF_TRY(ba.get(ctx_->pool.get(), sizeof(double) * dim * cap, s));
        local.capacity = cap;
        local.ctrl_idx = bi.as<int64_t>();
        local.xc = bx.as<double>();
        local.alpha = ba.as<double>();
        local.e_final = nullptr;
        cs = &local;
    }
    std::vector<LevelCache> fresh;
    rbf_status st = run_greedy(ctx_, p, g.n_s, g.xs.as<double>(), q.r.ds, cs, s, &g.levels, &fresh);
    if (st < 0) return st;
    // Volume update on the resident geometry. Support distances: the request's D_l, or
    // D_l = k max ||dS_l|| from the greedy (section 4). Levels without controls add nothing and
    // are left out.
    SumProblem pb;
    pb.dim = dim;
    pb.n_levels = 0;
    double dmax = 0.0;
    for (int l = 0; l < p.n_levels; ++l) {
        const double Dl = q.r.d_factor > 0.0 ? q.r.d_factor * cs->level_in_max[l] : q.r.D[l];
        if (cs->level_off[l + 1] == cs->level_off[l] || !(Dl > 0.0)) continue;
        // FP32 pairs only where the level's measured FP32 error at the surface allows it.
        const bool f32 = p.precision == RBF_MIXED && cs->level_fp32_err[l] <= RBF_MIXED_TOL * cs->level_in_max[0];
        pb.lv[pb.n_levels++] = SumLevel{1.0 / p.radius[l], Dl, cs->level_off[l], cs->level_off[l + 1], f32};
        dmax = std::max(dmax, Dl);
    }
    pb.ld_ctrl = cs->capacity;
    pb.xc = cs->xc;
    pb.alpha = cs->alpha;
    pb.n_p = g.n_pad;
    pb.ld_out = g.n_v;
    pb.xp = g.xv_sorted.as<double>();
    pb.dwall = g.d_sorted.as<double>();
    pb.perm = g.perm.as<int32_t>();
    pb.n_active = prefix_for(g, dmax);
    pb.block_box = g.block_box.as<double>();
    pb.geom = &g;
    pb.out = q.r.dv;
    pb.sign = -1.0;
    pb.precision = p.precision;
    pb.basis = p.basis;
    RBF_TRY(run_kernel_sum(ctx_, pb, s));
    RBF_HIP(hipStreamSynchronize(s));
    settle_all(bi, bx, ba);
    // Remember the control sets for the next icing step on this geometry.
    std::vector<int64_t> all(cs->level_off[p.n_levels]);
    if (!all.empty())
        RBF_HIP(hipMemcpy(all.data(), cs->ctrl_idx, sizeof(int64_t) * all.size(), hipMemcpyDeviceToHost));
    g.last_ctrl.assign(p.n_levels, {});
    for (int l = 0; l < p.n_levels; ++l)
        g.last_ctrl[l].assign(all.begin() + cs->level_off[l], all.begin() + cs->level_off[l + 1]);
    keep_bases(g, std::move(fresh));
    return st;
}

// Resident Newton bases share a slice of the budget: least recently used idle geometries give
// theirs up first; a set that cannot fit is dropped (the next step then re-appends its seeds).
void Server::keep_bases(Geometry &g, std::vector<LevelCache> &&fresh)
{
    std::lock_guard<std::mutex> lk(mu_);
    const uint64_t need = cache_bytes(fresh, g.n_s);
    cache_total_ -= g.cache_bytes;
    g.levels.clear();
    g.cache_bytes = 0;
    const uint64_t limit = cache_limit();
    while (cache_total_ + need > limit) {
        Geometry *victim = nullptr;
        for (Geometry *o : cached_)
            if (o != &g && !o->running && o->cache_bytes > 0 && (!victim || o->last_use < victim->last_use))
                victim = o;
        if (!victim) break;
        cache_total_ -= victim->cache_bytes;
        victim->levels.clear();
        victim->cache_bytes = 0;
        cached_.erase(std::find(cached_.begin(), cached_.end(), victim));
    }
    if (need > 0 && cache_total_ + need <= limit) {
        g.levels = std::move(fresh);
        g.cache_bytes = need;
        g.last_use = now_seconds();
        cache_total_ += need;
        if (std::find(cached_.begin(), cached_.end(), &g) == cached_.end()) cached_.push_back(&g);
    } else {
        cached_.erase(std::remove(cached_.begin(), cached_.end(), &g), cached_.end());
    }
}

void Server::forget(Geometry *g)
{
    std::lock_guard<std::mutex> lk(mu_);
    cache_total_ -= g->cache_bytes;
    g->cache_bytes = 0;
    cached_.erase(std::remove(cached_.begin(), cached_.end(), g), cached_.end());
}

void server_shutdown(rbf_ctx ctx)
{
    delete ctx->server;
    ctx->server = nullptr;
}

}  // namespace rbf

using namespace rbf;

extern "C" {

rbf_status rbf_geom_create(rbf_ctx ctx, int32_t dim, int64_t n_s, const double *xs, int64_t n_v,
                           const double *xv, const double *dwall, rbf_geom *out)
{
    if (!ctx || !out) return fail(RBF_E_INVALID, "NULL context or out");
    if (dim != 2 && dim != 3) return fail(RBF_E_INVALID, "dim must be 2 or 3");
    if (n_s < 1 || n_s > (int64_t(1) << 31) - 1) return fail(RBF_E_INVALID, "n_s out of range");
    if (n_v < 0 || n_v > (int64_t(1) << 31) - 1) return fail(RBF_E_INVALID, "n_v out of range");
    if (!xs || (n_v > 0 && !xv)) return fail(RBF_E_INVALID, "NULL device array");
    RBF_HIP(hipSetDevice(ctx->device));
    auto g = std::make_unique<Geometry>();
    g->dim = dim;
    g->n_s = n_s;
    g->n_v = n_v;
    hipStream_t s = nullptr;
    RBF_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    rbf_status st = dim == 2 ? build_geometry<2>(ctx, *g, xs, xv, dwall, s)
                             : build_geometry<3>(ctx, *g, xs, xv, dwall, s);
    (void)hipStreamSynchronize(s);
    settle_all(g->xs, g->xv_sorted, g->d_sorted, g->perm, g->block_box);   // the stream is idle
    (void)hipStreamDestroy(s);
    if (st < 0) return st;
    rbf_geom h = reinterpret_cast<rbf_geom>(g.get());
    std::lock_guard<std::mutex> lk(ctx->geom_mu);
    ctx->geoms[h] = std::move(g);
    *out = h;
    return RBF_OK;
}

rbf_status rbf_geom_volume_update(rbf_ctx ctx, rbf_geom geom, int32_t n_levels, const double *radius,
                                  const double *D, const int32_t *level_off, int64_t ld_ctrl,
                                  const double *xc, const double *alpha, double *dv,
                                  int32_t precision, const int32_t *level_precision, int32_t basis,
                                  void *stream)
{
    if (!ctx) return fail(RBF_E_INVALID, "ctx is NULL");
    Geometry *g = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->geom_mu);
        auto it = ctx->geoms.find(geom);
        if (it == ctx->geoms.end()) return fail(RBF_E_NOT_FOUND, "unknown geometry");
        g = it->second.get();
    }
    if (n_levels < 1 || n_levels > RBF_MAX_LEVELS) return fail(RBF_E_INVALID, "n_levels out of range");
    if (!radius || !D || !level_off) return fail(RBF_E_INVALID, "NULL host array");
    if (level_off[0] < 0) return fail(RBF_E_INVALID, "level_off[0] < 0");
    double dmax = 0.0;
    for (int l = 0; l < n_levels; ++l) {
        if (!(radius[l] > 0.0) || !std::isfinite(radius[l])) return fail(RBF_E_INVALID, "radius[%d] invalid", l);
        if (!(D[l] > 0.0) || !std::isfinite(D[l])) return fail(RBF_E_INVALID, "D[%d] invalid", l);
        if (level_off[l + 1] < level_off[l]) return fail(RBF_E_INVALID, "level_off not monotone");
        dmax = std::max(dmax, D[l]);
    }
    if (level_off[n_levels] > ld_ctrl) return fail(RBF_E_INVALID, "level_off exceeds ld_ctrl");
    RBF_TRY(check_precision(precision, level_precision, n_levels));
    if (!basis_valid(basis)) return fail(RBF_E_INVALID, "unknown basis %d", basis);
    if (g->n_v == 0) return RBF_OK;
    if (!dv || (level_off[n_levels] > level_off[0] && (!xc || !alpha))) return fail(RBF_E_INVALID, "NULL device array");
    RBF_HIP(hipSetDevice(ctx->device));
    SumProblem pb;
    pb.dim = g->dim;
    pb.n_levels = n_levels;
    for (int l = 0; l < n_levels; ++l)
        pb.lv[l] = SumLevel{1.0 / radius[l], D[l], level_off[l], level_off[l + 1],
                            (level_precision ? level_precision[l] : precision) == RBF_MIXED};
    pb.ld_ctrl = ld_ctrl;
    pb.xc = xc;
    pb.alpha = alpha;
    pb.n_p = g->n_pad;
    pb.ld_out = g->n_v;
    pb.xp = g->xv_sorted.as<double>();
    pb.dwall = g->d_sorted.as<double>();
    pb.perm = g->perm.as<int32_t>();
    pb.n_active = prefix_for(*g, dmax);
    pb.block_box = g->block_box.as<double>();
    pb.geom = g;
    pb.out = dv;
    pb.sign = -1.0;
    pb.precision = precision;
    pb.basis = basis;
    return run_kernel_sum(ctx, pb, (hipStream_t)stream);
}

rbf_status rbf_geom_release(rbf_ctx ctx, rbf_geom geom)
{
    if (!ctx) return fail(RBF_E_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->geom_mu);
    auto it = ctx->geoms.find(geom);
    if (it == ctx->geoms.end()) return fail(RBF_E_NOT_FOUND, "unknown geometry");
    if (ctx->server && ctx->server->geometry_busy(it->second.get()))
        return fail(RBF_E_BUSY, "geometry still has queued or running requests");
    if (ctx->server) ctx->server->forget(it->second.get());
    ctx->geoms.erase(it);
    return RBF_OK;
}

rbf_status rbf_submit(rbf_ctx ctx, const rbf_request *req, rbf_ticket *out)
{
    if (!ctx || !req || !out) return fail(RBF_E_INVALID, "NULL argument");
    Geometry *g = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->geom_mu);
        auto it = ctx->geoms.find(req->geom);
        if (it == ctx->geoms.end()) return fail(RBF_E_NOT_FOUND, "unknown geometry");
        g = it->second.get();
    }
    const rbf_greedy_params &p = req->params;
    RBF_TRY(validate_params(p, g->n_s));
    if (p.dim != g->dim) return fail(RBF_E_INVALID, "request dim %d != geometry dim %d", p.dim, g->dim);
    if (!req->ds || (g->n_v > 0 && !req->dv)) return fail(RBF_E_INVALID, "NULL device array");
    if (!(req->d_factor >= 0.0) || !std::isfinite(req->d_factor))
        return fail(RBF_E_INVALID, "d_factor must be finite and >= 0");
    if (req->d_factor == 0.0)
        for (int l = 0; l < p.n_levels; ++l)
            if (!(req->D[l] > 0.0) || !std::isfinite(req->D[l])) return fail(RBF_E_INVALID, "D[%d] must be > 0", l);
    if (req->out && (!req->out->ctrl_idx || !req->out->xc || !req->out->alpha ||
                     req->out->capacity < p.max_ctrl_total))
        return fail(RBF_E_INVALID, "out control set arrays missing or too small");
    auto q = std::make_unique<Req>();
    q->r = *req;
    q->g = g;
    q->handle = req->geom;
    if (p.seed_off) {
        q->seed_off.assign(p.seed_off, p.seed_off + p.n_levels + 1);
        q->seed_idx.assign(p.seed_idx, p.seed_idx + p.seed_off[p.n_levels]);
    }
    q->r.params.seed_idx = nullptr;
    q->r.params.seed_off = nullptr;
    const int64_t n_act = g->n_v;
    q->reserve = greedy_footprint(p.dim, g->n_s, p.max_ctrl_total) +
                 sizeof(double) * (uint64_t)p.dim * (uint64_t)n_act * 2 + (64ull << 20);
    if (q->reserve > ctx->pool->budget())
        return fail(RBF_E_NOMEM, "request needs about %llu bytes, budget is %llu",
                    (unsigned long long)q->reserve, (unsigned long long)ctx->pool->budget());
    {
        std::lock_guard<std::mutex> lk(ctx->geom_mu);
        if (!ctx->server) {
            const char *e = getenv("RBF_SERVE_SLOTS");
            const int slots = e && atoi(e) > 0 ? atoi(e) : 4;
            ctx->server = new Server(ctx, slots);
            if (!ctx->server->ok()) {
                delete ctx->server;
                ctx->server = nullptr;
                return fail(RBF_E_DEVICE, "could not create serving streams");
            }
        }
    }
    return ctx->server->submit(std::move(q), out);
}

rbf_status rbf_poll(rbf_ctx ctx, rbf_ticket t, rbf_req_info *out)
{
    if (!ctx || !out) return fail(RBF_E_INVALID, "NULL argument");
    if (!ctx->server) return fail(RBF_E_NOT_FOUND, "unknown ticket");
    return ctx->server->poll(t, out, false);
}

rbf_status rbf_wait(rbf_ctx ctx, rbf_ticket t, rbf_req_info *out)
{
    if (!ctx || !out) return fail(RBF_E_INVALID, "NULL argument");
    if (!ctx->server) return fail(RBF_E_NOT_FOUND, "unknown ticket");
    return ctx->server->poll(t, out, true);
}

}  // extern "C"

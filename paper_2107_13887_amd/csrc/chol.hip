// Dense FP64 weight solve Phi_cc alpha = dS_c (eq. (9) on a given point set) on gfx950.
//
// Blocked right-looking Cholesky with 64x64 blocks on a row-major padded matrix:
//   for each block column k:  L_kk = chol(A_kk)            (one wave, a row per lane)
//                             L_ik = A_ik L_kk^-T           (panel: one wave per row block,
//                                                            a row per lane, L_kk in LDS)
//                             A_ij -= L_ik L_jk^T, i >= j > k  (trailing update, FP64 MFMA)
// Blocks move between HBM and the waves' rows through LDS, so every global access is a
// contiguous 512-byte row. The trailing update carries the n^3/3 flops and runs on
// v_mfma_f64_16x16x4_f64: each 256-lane workgroup owns a 64x64 tile, each wave a 32x32 quarter as
// 2x2 MFMA blocks over the 64-deep product.
// The forward and backward substitutions for the dim right-hand sides are one launch each: the
// workgroup owning a block row forms the inverse of its diagonal block while it waits, removes
// the contributions of the finished blocks as each is published, and multiplies by the inverse,
// so the chain from one block to the next is one flag, one 64x64 product and one 64x64 product.
// A non-positive pivot raises a device flag reported as RBF_E_NOT_SPD.
// The same factorization starts a greedy level from given control points (the seeds), followed by
// a blocked FP64 MFMA triangular solve for their Newton basis at every surface point.
#include <cmath>
#include <cstdlib>

#include "basis.h"
#include "internal.h"
#include "trichain.h"

namespace rbf {
namespace {

constexpr int NB = 64;
typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double sqrt_pos(double a)
{
    double y = __builtin_amdgcn_rsq(a);
    double g = a * y;
    double h = 0.5 * y;
    double r = __builtin_fma(-g, h, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    double d = __builtin_fma(-g, g, a);
    return __builtin_fma(d, h, g);
}

// sqrt(a) and 1/sqrt(a) to about an ulp: the v_rsq_f64 seed, one Goldschmidt step, a correction
// of the root and a last step on the reciprocal.
__device__ __forceinline__ void sqrt_and_rsqrt(double a, double &sq, double &inv)
{
    const double y = __builtin_amdgcn_rsq(a);
    double g = a * y;
    double h = 0.5 * y;
    double r = __builtin_fma(-g, h, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    const double d = __builtin_fma(-g, g, a);
    sq = __builtin_fma(d, h, g);
    r = __builtin_fma(-sq, h, 0.5);
    inv = 2.0 * __builtin_fma(h, r, h);
}

// Phi[i][j] = phi(||x_i - x_j|| / R) for the lower triangle (upper left untouched), padded
// rows/columns beyond n get the identity so the padded factorization stays well defined.
template <int DIM>
__global__ __launch_bounds__(256) void c_build(const double *xc, int64_t n, int64_t lda,
                                               double inv_r, int32_t basis, double *A)
{
    for (int64_t i = blockIdx.x; i < lda; i += gridDim.x)
    for (int64_t j = threadIdx.x; j <= i; j += 256) {
        double v;
        if (i < n && j < n) {
            double r2 = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                double d = (xc[k * n + i] - xc[k * n + j]) * inv_r;
                r2 = __builtin_fma(d, d, r2);
            }
            v = wendland(basis, sqrt_pos(fmax(r2, 1e-200)));
        } else {
            v = (i == j) ? 1.0 : 0.0;
        }
        A[i * lda + j] = v;
    }
}

// Lane l's value of v, in every lane.
__device__ __forceinline__ double lane_value(double v, int l)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Load / store a 64x64 block of the row-major matrix through LDS: lane t moves column t of every
// row, so each access is one contiguous row.
__device__ __forceinline__ void block_to_lds(const double *A, int64_t lda, int64_t r0, int64_t c0,
                                             double (*T)[NB + 1])
{
    const int t = threadIdx.x;
#pragma unroll 8
    for (int r = 0; r < NB; ++r) T[r][t] = A[(r0 + r) * lda + c0 + t];
}

// LDS hand-off between the lanes of one wave (the only wave taking part).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Factor the diagonal block k0 in place, by one wave (lane i = threadIdx.x < 64) holding row i in
// registers. At step j the pivot is read from lane j, column j is scaled in every lane (by the
// reciprocal root, so the serial chain holds no division) and written once to LDS, and each lane
// subtracts L[i][j] L[c][j] from its entries c > j with L[c][j] read as an LDS broadcast. Entries
// above the diagonal are never read and are not stored. T and col are LDS scratch.
__device__ __forceinline__ void diag_factor(double *A, int64_t lda, int64_t k0, int32_t *bad,
                                            double (*T)[NB + 1], double *col)
{
    const int i = threadIdx.x;
    block_to_lds(A, lda, k0, k0, T);
    wave_lds_sync();
    double r[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) r[c] = c <= i ? T[i][c] : 0.0;
    bool sing = false;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        double d = lane_value(r[j], j);
        // A pivot within rounding of zero (below (index + 1) ulps of phi(0) = 1) is singular.
        if (!(d > (double)(k0 + j + 1) * 0x1p-52)) {
            sing = true;
            d = 1.0;
        }
        double sd, inv;
        sqrt_and_rsqrt(d, sd, inv);
        const double lij = i > j ? r[j] * inv : 0.0;
        r[j] = i > j ? lij : (i == j ? sd : 0.0);
        if (j + 1 < NB) {
            col[i] = lij;
            wave_lds_sync();
#pragma unroll
            for (int c = j + 1; c < NB; ++c) r[c] = __builtin_fma(-lij, col[c], r[c]);
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (sing && i == 0) *bad = 1;
#pragma unroll
    for (int c = 0; c < NB; ++c) T[i][c] = r[c];
    wave_lds_sync();
#pragma unroll 8
    for (int rr = 0; rr < NB; ++rr)
        if (i <= rr) A[(k0 + rr) * lda + k0 + i] = T[rr][i];
}

// The first diagonal block (every later one is factored by the trailing update that finishes it).
__global__ __launch_bounds__(NB) void c_diag(double *A, int64_t lda, int64_t k0, int32_t *bad)
{
    __shared__ double T[NB][NB + 1];
    __shared__ __align__(16) double col[NB];
    diag_factor(A, lda, k0, bad, T, col);
}

// acc(64x64, this wave's 32x32 quarter) += Ablk(64x64) * Bblk(64x64)^T from LDS via FP64 MFMA.
// MFMA 16x16x4 f64: lane l supplies A[l % 16][l / 16] and B^T[l / 16][l % 16]; result element
// v of lane l is D[l / 16 + 4 v][l % 16] (rows interleaved across the four result registers).
__device__ __forceinline__ void tile_abt_acc(const double (*Ab)[NB + 1], const double (*Bb)[NB + 1],
                                             d4 acc[2][2])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll 4
    for (int kk = 0; kk < NB; kk += 4) {
        double af[2], bf[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) af[r] = Ab[r0 + r * 16 + li][kk + lk];
#pragma unroll
        for (int c = 0; c < 2; ++c) bf[c] = Bb[c0 + c * 16 + li][kk + lk];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 2; ++c)
                acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[r], bf[c], acc[r][c], 0, 0, 0);
    }
}

// acc = Ablk * Bblk^T (as above, from zero).
__device__ __forceinline__ void tile_abt(const double (*Ab)[NB + 1], const double (*Bb)[NB + 1], d4 acc[2][2])
{
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[r][c] = d4{0.0, 0.0, 0.0, 0.0};
    tile_abt_acc(Ab, Bb, acc);
}

// Panel: L_ik = A_ik L_kk^-T for every row block i below k. One wave per row block, lane r holds
// row r of A_ik and solves x L_kk^T = a by columns (x_m = a_m / L_mm, as a product with the
// reciprocal formed beforehand, then a_j -= x_m L_jm for j > m), with L_kk in LDS read as
// broadcasts.
__global__ __launch_bounds__(NB) void c_panel(double *A, int64_t lda, int64_t k0)
{
    __shared__ double L[NB][NB + 1];
    __shared__ double T[NB][NB + 1];
    __shared__ double rinv[NB];
    const int t = threadIdx.x;
    const int64_t i0 = k0 + NB * (1 + (int64_t)blockIdx.x);
    block_to_lds(A, lda, k0, k0, L);
    block_to_lds(A, lda, i0, k0, T);
    __syncthreads();
    rinv[t] = 1.0 / L[t][t];
    double a[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) a[c] = T[t][c];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NB; ++m) {
        const double x = a[m] * rinv[m];
        a[m] = x;
#pragma unroll
        for (int j = m + 1; j < NB; ++j) a[j] = __builtin_fma(-x, L[j][m], a[j]);
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) T[t][c] = a[c];
    __syncthreads();
#pragma unroll 8
    for (int r = 0; r < NB; ++r) A[(i0 + r) * lda + k0 + t] = T[r][t];
}

// Trailing update A_ij -= L_ik L_jk^T over the lower block triangle j <= i below block k. Tile 0
// is the next diagonal block; once its update is stored it is final, so wave 0 of that workgroup
// factors it while the other tiles are still being updated (the diagonal step leaves the critical
// path wherever the trailing update is longer).
__global__ __launch_bounds__(256) void c_trailing(double *A, int64_t lda, int64_t k0, int64_t nbr,
                                                  int32_t *bad)
{
    __shared__ double ab[NB][NB + 1];
    __shared__ double bb[NB][NB + 1];
    __shared__ __align__(16) double col[NB];
    // linear block index -> (bi, bj) with 0 <= bj <= bi < nbr (blocks after k)
    int64_t t = blockIdx.x;
    int64_t bi = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
    while (bi * (bi + 1) / 2 > t) --bi;
    int64_t bj = t - bi * (bi + 1) / 2;
    const int64_t i0 = k0 + NB * (1 + bi), j0 = k0 + NB * (1 + bj);
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
        int r = e / NB, c = e % NB;
        ab[r][c] = A[(i0 + r) * lda + k0 + c];
        bb[r][c] = A[(j0 + r) * lda + k0 + c];
    }
    __syncthreads();
    d4 acc[2][2];
    tile_abt(ab, bb, acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int row = r0 + r * 16 + (lane >> 4) + 4 * v, cc = c0 + c * 16 + (lane & 15);
                A[(i0 + row) * lda + j0 + cc] -= acc[r][c][v];
            }
    if (t == 0) {
        __syncthreads();   // the tile's stores by all four waves, before wave 0 reads it back
        if (threadIdx.x < NB) diag_factor(A, lda, k0 + NB, bad, ab, col);
    }
}

// ---- substitutions, one launch each -------------------------------------------------------------
// Chain state (int32, zeroed before the factorization): [0] forward ticket, [1] backward ticket,
// [2] fault (a wait gave up), [3] non-positive pivot, then one done flag per block for the forward
// pass and one per block for the backward pass.
constexpr int CH_HDR = 16;
// RBF_SOLVE_SPIN_LIMIT overrides the bound on the polls of one wait.

struct ChainArgs {
    const double *A;
    int64_t lda, n, nblk;
    double *y;        // [dim][n]: forward result
    double *dinv;     // [nblk][64][64]: inverses of the diagonal blocks, row-major
    int32_t *st;
    unsigned long long spin_limit;
    int32_t want;     // value of a published done flag
};

// Forward substitution L y = b. The workgroup with ticket kb owns rows [64 kb, 64 kb + 64): lane t
// keeps row t of b minus the finished blocks' contributions L_kb,j y_j, then y_kb = inv(L_kb,kb)
// times that. Tickets follow the order in which workgroups start, so a workgroup only waits for
// blocks owned by workgroups already running.
template <int DIM>
__global__ __launch_bounds__(NB) void c_fwd_chain(ChainArgs a, const double *b)
{
    __shared__ double Ls[NB][NB + 1];
    __shared__ double Dv[NB][NB + 1];
    __shared__ double vec[DIM][NB];
    __shared__ double rl[NB];
    __shared__ int32_t sh_kb, ok_sh;
    const int t = threadIdx.x;
    if (t == 0) sh_kb = __hip_atomic_fetch_add(&a.st[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int64_t kb = sh_kb, k0 = kb * NB;
    block_to_lds(a.A, a.lda, k0, k0, Ls);
    __syncthreads();
    tc_tri_inverse(Ls, Dv, rl);
    double *dk = a.dinv + kb * NB * NB;   // for the backward pass, stored off the chain
#pragma unroll 8
    for (int r = 0; r < NB; ++r) dk[r * NB + threadIdx.x] = Dv[r][threadIdx.x];
    double acc[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) acc[k] = k0 + t < a.n ? b[k * a.n + k0 + t] : 0.0;
    for (int64_t j = 0; j < kb; ++j) {
        __syncthreads();
        block_to_lds(a.A, a.lda, k0, j * NB, Ls);
        if (!tc_wait(&a.st[CH_HDR + j], a.want, &a.st[2], a.spin_limit, ok_sh)) return;
#pragma unroll
        for (int k = 0; k < DIM; ++k) vec[k][t] = a.y[k * a.n + j * NB + t];   // j < kb: a whole block
        __syncthreads();
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int c = 0; c < NB; c += 2) {
                s0 = __builtin_fma(Ls[t][c], vec[k][c], s0);
                s1 = __builtin_fma(Ls[t][c + 1], vec[k][c + 1], s1);
            }
            acc[k] -= s0 + s1;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < DIM; ++k) vec[k][t] = acc[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int c = 0; c < NB; c += 2) {
            s0 = __builtin_fma(Dv[t][c], vec[k][c], s0);
            s1 = __builtin_fma(Dv[t][c + 1], vec[k][c + 1], s1);
        }
        if (k0 + t < a.n) a.y[k * a.n + k0 + t] = s0 + s1;
    }
    tc_publish(&a.st[CH_HDR + kb]);
}

// Backward substitution L^T x = y, blocks from the last: the workgroup owning block kb keeps, in
// lane t, entry t of y_kb minus sum over finished j > kb of (L_j,kb^T x_j), then x_kb =
// inv(L_kb,kb)^T times that, with the inverse the forward pass stored.
template <int DIM>
__global__ __launch_bounds__(NB) void c_bwd_chain(ChainArgs a, double *x)
{
    __shared__ double Ls[NB][NB + 1];
    __shared__ double Dv[NB][NB + 1];
    __shared__ double vec[DIM][NB];
    __shared__ int32_t sh_kb, ok_sh;
    const int t = threadIdx.x;
    if (t == 0) sh_kb = __hip_atomic_fetch_add(&a.st[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int64_t kb = a.nblk - 1 - sh_kb, k0 = kb * NB;
    const double *dk = a.dinv + kb * NB * NB;
#pragma unroll 8
    for (int r = 0; r < NB; ++r) Dv[r][t] = dk[r * NB + t];
    double acc[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) acc[k] = k0 + t < a.n ? a.y[k * a.n + k0 + t] : 0.0;
    for (int64_t j = a.nblk - 1; j > kb; --j) {
        __syncthreads();
        block_to_lds(a.A, a.lda, j * NB, k0, Ls);
        if (!tc_wait(&a.st[CH_HDR + a.nblk + j], a.want, &a.st[2], a.spin_limit, ok_sh)) return;
#pragma unroll
        for (int k = 0; k < DIM; ++k) vec[k][t] = j * NB + t < a.n ? x[k * a.n + j * NB + t] : 0.0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int r = 0; r < NB; r += 2) {
                s0 = __builtin_fma(Ls[r][t], vec[k][r], s0);
                s1 = __builtin_fma(Ls[r + 1][t], vec[k][r + 1], s1);
            }
            acc[k] -= s0 + s1;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < DIM; ++k) vec[k][t] = acc[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int r = 0; r < NB; r += 2) {
            s0 = __builtin_fma(Dv[r][t], vec[k][r], s0);
            s1 = __builtin_fma(Dv[r + 1][t], vec[k][r + 1], s1);
        }
        if (k0 + t < a.n) x[k * a.n + k0 + t] = s0 + s1;
    }
    tc_publish(&a.st[CH_HDR + a.nblk + kb]);
}

// ---- seeded level start: the Newton basis of a given control set -----------------------------
// A level that starts from n given control points (a warm start whose resident basis is gone, or
// a call with seeds) needs L with L L^T = Phi_CC and V = Phi_sC L^-T at every surface point. The
// factor comes from the blocked MFMA Cholesky above; V from a blocked triangular solve by
// 64-column blocks, left-looking, one workgroup per tile of 64 surface points:
//   acc   = Phi(tile, C_K) - sum_{J < K} V(tile, J) L_KJ^T      (FP64 MFMA, 64 x 64 x 64 per J)
//   V(tile, K) = acc Dinv_K^T                                    (FP64 MFMA, Dinv_K = inv(L_KK))
// Phi(tile, C_K) is evaluated in the workgroup, exactly as the greedy's own update evaluates phi,
// so the only differences from appending the points one by one are the order of the sums and the
// use of the diagonal blocks' inverses.

// Dinv_kb = inv(L_kb,kb) for every diagonal block of the factored padded matrix, row-major.
__global__ __launch_bounds__(NB) void c_diag_inverse(const double *A, int64_t lda, double *dinv)
{
    __shared__ double Ls[NB][NB + 1];
    __shared__ double Dv[NB][NB + 1];
    __shared__ double rl[NB];
    const int64_t k0 = (int64_t)blockIdx.x * NB;
    block_to_lds(A, lda, k0, k0, Ls);
    __syncthreads();
    tc_tri_inverse(Ls, Dv, rl);
    __syncthreads();
    double *dk = dinv + (int64_t)blockIdx.x * NB * NB;
#pragma unroll 8
    for (int r = 0; r < NB; ++r) dk[r * NB + threadIdx.x] = Dv[r][threadIdx.x];
}

// Packed rows of the factor: Lp[i (i + 1) / 2 + j] = L[i][j], j <= i < n.
__global__ __launch_bounds__(256) void c_pack(const double *A, int64_t lda, int64_t n, double *Lp)
{
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x)
        for (int64_t j = threadIdx.x; j <= i; j += 256) Lp[(i * (i + 1)) / 2 + j] = A[i * lda + j];
}

// phi(||x_i - c_j|| / R) as the greedy's update forms it: the squared distance summed in order
// without contraction, an IEEE root and a division by R, exactly zero from eta = 1 on.
template <int DIM>
__device__ __forceinline__ double phi_seed(const double (&x)[DIM], const double (&c)[DIM], double R,
                                           int32_t basis)
{
    double s = 0.0;
    {
#pragma clang fp contract(off)
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const double d = x[k] - c[k];
            s = s + d * d;
        }
    }
    const double eta = sqrt(s) / R;
    return eta >= 1.0 ? 0.0 : wendland(basis, eta);
}

// V(tile, 0:n) for one tile of 64 surface points per workgroup (see above). Blocks of V and L
// stream through LDS with the next block's loads in flight during the current block's MFMAs.
// V is tile-major: V(i, j) at ((i / 64) ldt + j) 64 + i % 64; rows past n_s take the last
// point's coordinates and are never read as results.
template <int DIM>
__global__ __launch_bounds__(256, 2) void c_seed_basis(const double *xs, int64_t n_s, const double *xc, int64_t n,
                                                    double R, int32_t basis, const double *A, int64_t lda,
                                                    const double *dinv, double *V, int64_t ldt)
{
    __shared__ double va[NB][NB + 1];
    __shared__ double lb[NB][NB + 1];
    __shared__ double xt[DIM][NB];
    __shared__ double ck[DIM][NB];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t tile = blockIdx.x;
    const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
    const int64_t nblk = (n + NB - 1) / NB;
    double *vt = V + tile * ldt * NB;
    if (t < NB) {
        const int64_t i = min(tile * NB + t, n_s - 1);
#pragma unroll
        for (int k = 0; k < DIM; ++k) xt[k][t] = xs[k * n_s + i];
    }
    for (int64_t kb = 0; kb < nblk; ++kb) {
        // The previous block of V was stored to global memory by every thread at the end of the
        // previous iteration; the loads below read it (block 0 at kb = 1) in other threads.
        __syncthreads();
        d4 acc[2][2];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 2; ++c) acc[r][c] = d4{0.0, 0.0, 0.0, 0.0};
        // Earlier blocks: acc += V(tile, J) L_kb,J^T. Pair e = t + 256 q (q < 8) of a block holds
        // elements 2e and 2e + 1: column e / 32 and rows 2 (e % 32) + {0, 1} of V's block (one
        // contiguous 32 KB region), row e / 32 and columns 2 (e % 32) + {0, 1} of L's block
        // (64 contiguous 512-byte rows). 16-byte loads, the next block's in flight during the MFMAs.
        const int pr = t >> 5, pc = (t & 31) * 2;   // pair q: V column / L row pr + 8 q, offset pc
        const d2 *vsrc = reinterpret_cast<const d2 *>(vt) + t;
        const double *lsrc = A + (kb * NB + pr) * lda + pc;
        d2 pv[8], pl[8];
        if (kb > 0) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                pv[q] = vsrc[256 * q];
                pl[q] = *reinterpret_cast<const d2 *>(lsrc + 8 * q * lda);
            }
        }
        for (int64_t jb = 0; jb < kb; ++jb) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                va[pc][pr + 8 * q] = pv[q].x;
                va[pc + 1][pr + 8 * q] = pv[q].y;
                lb[pr + 8 * q][pc] = pl[q].x;
                lb[pr + 8 * q][pc + 1] = pl[q].y;
            }
            __syncthreads();
            if (jb + 1 < kb) {
                vsrc += NB * NB / 2;
                lsrc += NB;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    pv[q] = vsrc[256 * q];
                    pl[q] = *reinterpret_cast<const d2 *>(lsrc + 8 * q * lda);
                }
            }
            tile_abt_acc(va, lb, acc);
        }
        // B = Phi(tile, C_kb) - acc into va: phi by element e = t + 256 q (row e % 64, column
        // e / 64), then each lane subtracts its accumulator entries. Columns past n are zero.
        __syncthreads();
        if (t < NB) {
            const int64_t j = min(kb * NB + t, n - 1);
#pragma unroll
            for (int k = 0; k < DIM; ++k) ck[k][t] = xc[k * n + j];
        }
        __syncthreads();
#pragma unroll 1
        for (int q = 0; q < 16; ++q) {
            const int e = t + 256 * q, row = e & 63, col = e >> 6;
            double xx[DIM], cc[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                xx[k] = xt[k][row];
                cc[k] = ck[k][col];
            }
            va[row][col] = kb * NB + col < n ? phi_seed<DIM>(xx, cc, R, basis) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int col = c0 + c * 16 + (lane & 15);
                if (kb * NB + col < n)
#pragma unroll
                    for (int v = 0; v < 4; ++v) va[r0 + r * 16 + (lane >> 4) + 4 * v][col] -= acc[r][c][v];
            }
        const double *dk = dinv + kb * NB * NB;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int e = t + 256 * q;
            lb[e >> 6][e & 63] = dk[e];
        }
        __syncthreads();
        // V(tile, kb)[row][c] = sum_m B[row][m] Dinv[c][m], staged column-major for the stores.
        tile_abt(va, lb, acc);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    va[c0 + c * 16 + (lane & 15)][r0 + r * 16 + (lane >> 4) + 4 * v] = acc[r][c][v];
        __syncthreads();
        const int64_t live_cols = min<int64_t>(NB, n - kb * NB);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int e = t + 256 * q;
            if ((e >> 6) < live_cols) vt[kb * NB * NB + e] = va[e >> 6][e & 63];
        }
    }
}

// Phi_cc of the n points xc ([dim][n]) on the padded row-major matrix A (lda = 64 ceil(n / 64)),
// factored in place into its lower Cholesky factor (launches only). A non-positive pivot sets *bad.
template <int DIM>
void launch_factor(double radius, int64_t n, const double *xc, int32_t basis, double *A, int64_t lda,
                   int32_t *bad, hipStream_t s)
{
    const int64_t nblk = lda / NB;
    hipLaunchKernelGGL(c_build<DIM>, dim3((unsigned)std::min<int64_t>(lda, 8192)), dim3(256), 0, s,
                       xc, n, lda, 1.0 / radius, basis, A);
    for (int64_t kb = 0; kb < nblk; ++kb) {
        const int64_t k0 = kb * NB, rest = nblk - kb - 1;
        if (kb == 0) hipLaunchKernelGGL(c_diag, dim3(1), dim3(NB), 0, s, A, lda, k0, bad);
        if (rest > 0) {
            hipLaunchKernelGGL(c_panel, dim3((unsigned)rest), dim3(NB), 0, s, A, lda, k0);
            hipLaunchKernelGGL(c_trailing, dim3((unsigned)(rest * (rest + 1) / 2)), dim3(256), 0, s, A, lda,
                               k0, rest, bad);
        }
    }
}

template <int DIM>
rbf_status solve_impl(rbf_ctx ctx, double radius, int64_t n, const double *xc, const double *dsc,
                      double *alpha, int32_t basis, hipStream_t s)
{
    Pool *pool = ctx->pool.get();
    const int64_t lda = ((n + NB - 1) / NB) * NB;
    const int64_t nblk = lda / NB;
    const size_t st_bytes = sizeof(int32_t) * (size_t)(CH_HDR + 2 * nblk);
    DevBuf bA, bSt, bDinv, bY;
    RBF_TRY(bA.get(pool, sizeof(double) * (size_t)lda * (size_t)lda, s));
    RBF_TRY(bSt.get(pool, st_bytes, s));
    RBF_TRY(bDinv.get(pool, sizeof(double) * (size_t)nblk * NB * NB, s));
    RBF_TRY(bY.get(pool, sizeof(double) * DIM * (size_t)n, s));
    double *A = bA.as<double>();
    int32_t *st = bSt.as<int32_t>();
    RBF_HIP(hipMemsetAsync(st, 0, st_bytes, s));
    launch_factor<DIM>(radius, n, xc, basis, A, lda, st + 3, s);
    RBF_HIP(hipGetLastError());
    ChainArgs ca{};
    ca.A = A;
    ca.lda = lda;
    ca.n = n;
    ca.nblk = nblk;
    ca.y = bY.as<double>();
    ca.dinv = bDinv.as<double>();
    ca.st = st;
    ca.spin_limit = TC_SPIN_LIMIT;
    if (const char *e = getenv("RBF_SOLVE_SPIN_LIMIT")) ca.spin_limit = strtoull(e, nullptr, 10);
    // RBF_SOLVE_UNMET_WAITS=1 makes every wait ask for a flag value no block publishes, so each
    // gives up at the spin limit: the failure path, reached with every kernel still exiting.
    ca.want = 1;
    if (const char *e = getenv("RBF_SOLVE_UNMET_WAITS")) ca.want = atoi(e) ? 2 : 1;
    hipLaunchKernelGGL(c_fwd_chain<DIM>, dim3((unsigned)nblk), dim3(NB), 0, s, ca, dsc);
    hipLaunchKernelGGL(c_bwd_chain<DIM>, dim3((unsigned)nblk), dim3(NB), 0, s, ca, alpha);
    RBF_HIP(hipGetLastError());
    int32_t flags[4] = {0, 0, 0, 0};
    RBF_HIP(hipMemcpyAsync(flags, st, sizeof(flags), hipMemcpyDeviceToHost, s));
    RBF_HIP(hipStreamSynchronize(s));
    settle_all(bA, bSt, bDinv, bY);
    if (flags[3]) return fail(RBF_E_NOT_SPD, "Phi_cc is not numerically positive definite (n=%lld)", (long long)n);
    if (flags[2])
        return fail(RBF_E_DEVICE, "weight solve: a substitution wait gave up after %llu polls (n=%lld)",
                    ca.spin_limit, (long long)n);
    return RBF_OK;
}

}  // namespace

rbf_status run_solve_weights(rbf_ctx ctx, int32_t dim, double radius, int64_t n_c, const double *xc,
                             const double *dsc, double *alpha, int32_t basis, hipStream_t s)
{
    return dim == 2 ? solve_impl<2>(ctx, radius, n_c, xc, dsc, alpha, basis, s)
                    : solve_impl<3>(ctx, radius, n_c, xc, dsc, alpha, basis, s);
}

rbf_status seed_factor(int32_t dim, double radius, int32_t basis, int64_t n, const double *xc, double *A,
                       int64_t lda, double *dinv, int32_t *bad, hipStream_t s)
{
    if (dim == 2) launch_factor<2>(radius, n, xc, basis, A, lda, bad, s);
    else launch_factor<3>(radius, n, xc, basis, A, lda, bad, s);
    hipLaunchKernelGGL(c_diag_inverse, dim3((unsigned)(lda / NB)), dim3(NB), 0, s, (const double *)A, lda, dinv);
    RBF_HIP(hipGetLastError());
    return RBF_OK;
}

rbf_status seed_basis(int32_t dim, const double *xs, int64_t n_s, const double *xc, int64_t n, double radius,
                      int32_t basis, const double *A, int64_t lda, const double *dinv, double *V, int64_t ldt,
                      double *Lpack, hipStream_t s)
{
    const unsigned g = (unsigned)((n_s + NB - 1) / NB);
    hipLaunchKernelGGL(c_pack, dim3((unsigned)std::min<int64_t>(n, 8192)), dim3(256), 0, s, A, lda, n, Lpack);
    if (dim == 2)
        hipLaunchKernelGGL(c_seed_basis<2>, dim3(g), dim3(256), 0, s, xs, n_s, xc, n, radius, basis, A, lda, dinv,
                           V, ldt);
    else
        hipLaunchKernelGGL(c_seed_basis<3>, dim3(g), dim3(256), 0, s, xs, n_s, xc, n, radius, basis, A, lda, dinv,
                           V, ldt);
    RBF_HIP(hipGetLastError());
    return RBF_OK;
}

}  // namespace rbf

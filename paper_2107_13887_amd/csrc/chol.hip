// Dense FP64 weight solve Phi_cc alpha = dS_c (eq. (9) on a given point set) on gfx950.
//
// Blocked right-looking Cholesky with 64x64 blocks on a row-major padded matrix:
//   for each block column k:  L_kk = chol(A_kk)            (one wave, a row per lane)
//                             L_ik = A_ik L_kk^-T           (panel: one wave per row block,
//                                                            a row per lane, L_kk in LDS)
//                             A_ij -= L_ik L_jk^T, i >= j > k  (trailing update, FP64 MFMA)
// then blocked forward and backward substitution for the dim right-hand sides. The trailing
// update carries the n^3/3 flops and runs on v_mfma_f64_16x16x4_f64: each 256-lane workgroup
// owns a 64x64 tile, each wave a 32x32 quarter as 2x2 MFMA blocks over the 64-deep product.
// A non-positive pivot raises a device flag reported as RBF_E_NOT_SPD.
#include <cmath>

#include "basis.h"
#include "internal.h"

namespace rbf {
namespace {

constexpr int NB = 64;
typedef double d4 __attribute__((ext_vector_type(4)));

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

// Factor the diagonal block: one wave, lane i holds row i in registers. At step j the pivot is
// read from lane j, column j is scaled in every lane and written once to LDS, and each lane
// subtracts L[i][j] L[c][j] from its entries c > j with L[c][j] read as an LDS broadcast.
// Entries above the diagonal are left out of every read that matters and are not stored.
__global__ __launch_bounds__(NB) void c_diag(double *A, int64_t lda, int64_t k0, int32_t *bad)
{
    __shared__ __align__(16) double col[NB];
    const int i = threadIdx.x;
    double *ar = A + (k0 + i) * lda + k0;
    double r[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) r[c] = c <= i ? ar[c] : 0.0;
    bool sing = false;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        double d = lane_value(r[j], j);
        // A pivot within rounding of zero (below (index + 1) ulps of phi(0) = 1) is singular.
        if (!(d > (double)(k0 + j + 1) * 0x1p-52)) {
            sing = true;
            d = 1.0;
        }
        const double sd = sqrt(d);
        const double lij = i > j ? r[j] / sd : 0.0;
        r[j] = i > j ? lij : (i == j ? sd : 0.0);
        if (j + 1 < NB) {
            col[i] = lij;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int c = j + 1; c < NB; ++c) r[c] = __builtin_fma(-lij, col[c], r[c]);
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (sing && i == 0) *bad = 1;
#pragma unroll
    for (int c = 0; c < NB; ++c)
        if (c <= i) ar[c] = r[c];
}

// acc(64x64, this wave's 32x32 quarter) = Ablk(64x64) * Bblk(64x64)^T from LDS via FP64 MFMA.
// MFMA 16x16x4 f64: lane l supplies A[l % 16][l / 16] and B^T[l / 16][l % 16]; result element
// v of lane l is D[l / 16 + 4 v][l % 16] (rows interleaved across the four result registers).
__device__ __forceinline__ void tile_abt(const double (*Ab)[NB + 1], const double (*Bb)[NB + 1],
                                         d4 acc[2][2])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[r][c] = d4{0.0, 0.0, 0.0, 0.0};
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

// Panel: L_ik = A_ik L_kk^-T for every row block i below k. One wave per row block, lane r holds
// row r of A_ik and solves x L_kk^T = a by columns (x_m = a_m / L_mm, then a_j -= x_m L_jm for
// j > m), with L_kk in LDS read as broadcasts.
__global__ __launch_bounds__(NB) void c_panel(double *A, int64_t lda, int64_t k0)
{
    __shared__ double L[NB][NB + 1];
    const int t = threadIdx.x;
    for (int r = 0; r < NB; ++r) L[r][t] = t <= r ? A[(k0 + r) * lda + k0 + t] : 0.0;
    const int64_t i0 = k0 + NB * (1 + (int64_t)blockIdx.x);
    double *ar = A + (i0 + t) * lda + k0;
    double a[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) a[c] = ar[c];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NB; ++m) {
        const double x = a[m] / L[m][m];
        a[m] = x;
#pragma unroll
        for (int j = m + 1; j < NB; ++j) a[j] = __builtin_fma(-x, L[j][m], a[j]);
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) ar[c] = a[c];
}

// Trailing update A_ij -= L_ik L_jk^T over the lower block triangle j <= i below block k.
__global__ __launch_bounds__(256) void c_trailing(double *A, int64_t lda, int64_t k0, int64_t nbr)
{
    __shared__ double ab[NB][NB + 1];
    __shared__ double bb[NB][NB + 1];
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
                int row = r0 + r * 16 + (lane >> 4) + 4 * v, col = c0 + c * 16 + (lane & 15);
                A[(i0 + row) * lda + j0 + col] -= acc[r][c][v];
            }
}

// Forward substitution L y = b for rows [b0, b0 + 64), then b_i -= L_i,blk y_blk below.
template <int DIM>
__global__ __launch_bounds__(256) void c_fwd(const double *A, int64_t lda, double *b, int64_t ldb,
                                             int64_t n, int64_t b0, double *yout)
{
    __shared__ double Lb[NB][NB + 1];
    __shared__ double yb[DIM][NB];
    __shared__ double rinv[NB];                         // 1 / L[i][i], off the serial chain
    const int nb = (int)min<int64_t>(NB, n - b0);
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
        int r = e / NB, c = e % NB;
        Lb[r][c] = (r < nb && c <= r) ? A[(b0 + r) * lda + b0 + c] : (r == c ? 1.0 : 0.0);
    }
    if (threadIdx.x < NB)
        for (int k = 0; k < DIM; ++k) yb[k][threadIdx.x] = threadIdx.x < nb ? b[k * ldb + b0 + threadIdx.x] : 0.0;
    __syncthreads();
    if (threadIdx.x < NB) rinv[threadIdx.x] = 1.0 / Lb[threadIdx.x][threadIdx.x];
    __syncthreads();
    if (threadIdx.x < NB) {
        const int j = threadIdx.x;
        double rhs[DIM];
        for (int k = 0; k < DIM; ++k) rhs[k] = yb[k][j];
        for (int i = 0; i < nb; ++i) {
            // x_i from lane i's finished right-hand side, the same value in every lane
            const double ri = rinv[i];
            double xi[DIM];
            for (int k = 0; k < DIM; ++k) xi[k] = lane_value(rhs[k], i) * ri;
            if (j > i)
                for (int k = 0; k < DIM; ++k) rhs[k] = __builtin_fma(-Lb[j][i], xi[k], rhs[k]);
            if (j == i)
                for (int k = 0; k < DIM; ++k) rhs[k] = xi[k];
        }
        for (int k = 0; k < DIM; ++k) yb[k][j] = rhs[k];
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x < nb)
        for (int k = 0; k < DIM; ++k) yout[k * ldb + b0 + threadIdx.x] = yb[k][threadIdx.x];
    for (int64_t r = b0 + nb + (int64_t)blockIdx.x * 256 + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * 256) {
        double acc[DIM];
        for (int k = 0; k < DIM; ++k) acc[k] = 0.0;
        for (int i = 0; i < nb; ++i) {
            double l = A[r * lda + b0 + i];
            for (int k = 0; k < DIM; ++k) acc[k] = __builtin_fma(l, yb[k][i], acc[k]);
        }
        for (int k = 0; k < DIM; ++k) b[k * ldb + r] -= acc[k];
    }
}

// Backward substitution L^T x = y for rows [b0, b1), then y_j -= L_blk,j x_blk above.
template <int DIM>
__global__ __launch_bounds__(256) void c_bwd(const double *A, int64_t lda, double *y, int64_t ldy,
                                             int64_t b0, int64_t b1, double *xout)
{
    __shared__ double Lb[NB][NB + 1];
    __shared__ double xb[DIM][NB];
    __shared__ double rinv[NB];                         // 1 / L[i][i], off the serial chain
    const int nb = (int)(b1 - b0);
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
        int r = e / NB, c = e % NB;
        Lb[r][c] = (r < nb && c <= r) ? A[(b0 + r) * lda + b0 + c] : (r == c ? 1.0 : 0.0);
    }
    if (threadIdx.x < NB)
        for (int k = 0; k < DIM; ++k) xb[k][threadIdx.x] = threadIdx.x < nb ? y[k * ldy + b0 + threadIdx.x] : 0.0;
    __syncthreads();
    if (threadIdx.x < NB) rinv[threadIdx.x] = 1.0 / Lb[threadIdx.x][threadIdx.x];
    __syncthreads();
    if (threadIdx.x < NB) {
        const int j = threadIdx.x;
        double rhs[DIM];
        for (int k = 0; k < DIM; ++k) rhs[k] = xb[k][j];
        for (int i = nb - 1; i >= 0; --i) {
            const double ri = rinv[i];
            double xi[DIM];
            for (int k = 0; k < DIM; ++k) xi[k] = lane_value(rhs[k], i) * ri;
            if (j < i)
                for (int k = 0; k < DIM; ++k) rhs[k] = __builtin_fma(-Lb[i][j], xi[k], rhs[k]);
            if (j == i)
                for (int k = 0; k < DIM; ++k) rhs[k] = xi[k];
        }
        for (int k = 0; k < DIM; ++k) xb[k][j] = rhs[k];
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x < nb)
        for (int k = 0; k < DIM; ++k) xout[k * ldy + b0 + threadIdx.x] = xb[k][threadIdx.x];
    for (int64_t jj = (int64_t)blockIdx.x * 256 + threadIdx.x; jj < b0; jj += (int64_t)gridDim.x * 256) {
        double acc[DIM];
        for (int k = 0; k < DIM; ++k) acc[k] = 0.0;
        for (int i = 0; i < nb; ++i) {
            double l = A[(b0 + i) * lda + jj];
            for (int k = 0; k < DIM; ++k) acc[k] = __builtin_fma(l, xb[k][i], acc[k]);
        }
        for (int k = 0; k < DIM; ++k) y[k * ldy + jj] -= acc[k];
    }
}

template <int DIM>
rbf_status solve_impl(rbf_ctx ctx, double radius, int64_t n, const double *xc, const double *dsc,
                      double *alpha, int32_t basis, hipStream_t s)
{
    Pool *pool = ctx->pool.get();
    const int64_t lda = ((n + NB - 1) / NB) * NB;
    const int64_t nblk = lda / NB;
    DevBuf bA, bFlag, bW, bY;
    RBF_TRY(bA.get(pool, sizeof(double) * (size_t)lda * (size_t)lda));
    RBF_TRY(bFlag.get(pool, sizeof(int32_t)));
    RBF_TRY(bW.get(pool, sizeof(double) * DIM * (size_t)n));
    RBF_TRY(bY.get(pool, sizeof(double) * DIM * (size_t)n));
    double *A = bA.as<double>();
    RBF_HIP(hipMemsetAsync(bFlag.ptr, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(c_build<DIM>, dim3((unsigned)std::min<int64_t>(lda, 8192)), dim3(256), 0, s,
                       xc, n, lda, 1.0 / radius, basis, A);
    for (int64_t kb = 0; kb < nblk; ++kb) {
        const int64_t k0 = kb * NB, rest = nblk - kb - 1;
        hipLaunchKernelGGL(c_diag, dim3(1), dim3(NB), 0, s, A, lda, k0, bFlag.as<int32_t>());
        if (rest > 0) {
            hipLaunchKernelGGL(c_panel, dim3((unsigned)rest), dim3(NB), 0, s, A, lda, k0);
            hipLaunchKernelGGL(c_trailing, dim3((unsigned)(rest * (rest + 1) / 2)), dim3(256), 0, s, A, lda,
                               k0, rest);
        }
    }
    RBF_HIP(hipGetLastError());
    // W = dsc (updated below each block), Y = L^-1 dsc, alpha = L^-T Y (Y updated above).
    RBF_HIP(hipMemcpyAsync(bW.ptr, dsc, sizeof(double) * DIM * n, hipMemcpyDeviceToDevice, s));
    for (int64_t b0 = 0; b0 < n; b0 += NB) {
        unsigned gb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n - b0 + 255) / 256, 1024));
        hipLaunchKernelGGL(c_fwd<DIM>, dim3(gb), dim3(256), 0, s, A, lda, bW.as<double>(), n, n, b0,
                           bY.as<double>());
    }
    for (int64_t b1 = n; b1 > 0; b1 -= NB) {
        int64_t b0 = std::max<int64_t>(0, b1 - NB);
        unsigned gb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((b0 + 255) / 256, 1024));
        hipLaunchKernelGGL(c_bwd<DIM>, dim3(gb), dim3(256), 0, s, A, lda, bY.as<double>(), n, b0, b1,
                           alpha);
    }
    RBF_HIP(hipGetLastError());
    int32_t bad = 0;
    RBF_HIP(hipMemcpyAsync(&bad, bFlag.ptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RBF_HIP(hipStreamSynchronize(s));
    if (bad) return fail(RBF_E_NOT_SPD, "Phi_cc is not numerically positive definite (n=%lld)", (long long)n);
    return RBF_OK;
}

}  // namespace

rbf_status run_solve_weights(rbf_ctx ctx, int32_t dim, double radius, int64_t n_c, const double *xc,
                             const double *dsc, double *alpha, int32_t basis, hipStream_t s)
{
    return dim == 2 ? solve_impl<2>(ctx, radius, n_c, xc, dsc, alpha, basis, s)
                    : solve_impl<3>(ctx, radius, n_c, xc, dsc, alpha, basis, s);
}

}  // namespace rbf

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
// Execution. An iteration is a select phase (argmax of the per-tile maxima, stop tests, row
// extraction, pivot) and an update phase (all workgroups, 64 surface points per tile: new column,
// error update, tile argmax). On small surfaces a level runs as one persistent cooperative kernel
// in which every workgroup runs the select phase itself after the iteration's one grid barrier,
// keeping the Newton row in LDS for its update. When the device holds a workgroup per tile and no
// other persistent kernel runs, the resident form also keeps each tile's first Newton columns in
// LDS and its error in registers, so that its update reads no global memory. On large surfaces
// (or when a cooperative launch is impossible) the two phases run as two kernel launches per
// iteration.
// Reductions run in a fixed order; squared norms are formed without fused multiply-adds so they
// equal the textbook formula term by term.
//
// Seeded levels. A level handed its first control points (a warm start from the previous icing
// step's set, or the caller's seeds) starts from the resident basis of the same points when one is
// kept; otherwise, from SEED_FACTOR_MIN seeds on, from L = chol(Phi_CC) (blocked, FP64 MFMA) and
// V = Phi_sC L^-T (blocked triangular solves, FP64 MFMA) formed at once, rather than by appending
// the seeds one iteration each. Either way y = L^-1 dS_C and E = dS - V y follow, and the level
// continues with its argmax iterations.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "basis.h"
#include "internal.h"
#include "trichain.h"

namespace cg = cooperative_groups;

namespace rbf {
namespace {

constexpr int UPB = 64;       // surface points per tile (one per lane)
constexpr int UWAVES = 4;     // waves per workgroup, each a slice of the dot product
constexpr int NT = UPB * UWAVES;
constexpr int LCHUNK = 2048;  // Newton row entries staged per LDS pass
constexpr int64_t LEAN_MAX_TILES = 112;   // largest surface (in tiles) run by the persistent kernel
constexpr int RES_COLS = 192;             // Newton columns a resident persistent workgroup keeps in LDS
constexpr int SEL_U = 8;                  // loads a select thread issues before using any
// The two-launch update reads the basis columns below keep_cols with the default cache policy and
// the rest non-temporally, so that the first KEEP_BYTES of every iteration's stream stay in the
// 256 MB last-level cache for the next iteration instead of being evicted by the rest of it.
constexpr int64_t KEEP_BYTES = int64_t(192) << 20;
constexpr int64_t SEED_FACTOR_MIN = 32;   // fewest seeds of a level started from the blocked factor

struct GState {
    int64_t n;        // finished columns (control points) of the level
    int64_t p;        // point appended by the pending update
    int64_t n_iter;   // argmax selections made in this call (all levels)
    int32_t go;       // 1: an update for column n is pending
    int32_t stop;     // RBF_STOP_* once the level stopped, else -1
    int32_t fault;    // 1: a persistent workgroup gave up waiting at a barrier
    double d;         // pivot of the pending column
    double c[3];      // Newton coefficients of the pending column
    double target2;   // squared tolerance of the level
    double rmax2;     // max_i ||r_i||^2 of the level's input residual
};

struct Cand {
    double m2;
    int64_t idx;
};

struct GArgs {
    GState *st;
    const double *xs;
    int64_t n_s;
    double R;
    int32_t basis;       // RBF_WENDLAND_*
    double *V;           // Newton basis, tile-major: V(i, j) at ((i / UPB) ldt + j) UPB + i % UPB
    int64_t ldt;         // columns per tile in V
    double *Lpack;       // packed lower factor, row n at n (n + 1) / 2
    double *coef;        // [DIM][ld_coef] Newton coefficients y
    int64_t ld_coef;
    double *E;           // [DIM][n_s] current error
    uint8_t *sel;        // [n_s] selected in this level
    Cand *part;          // [g] per-tile maxima
    double *E2;          // persistent form: second error buffer (iterations alternate)
    Cand *part2;         // persistent form: second buffer of per-tile maxima
    unsigned long long spin_limit;   // persistent form: polls of one barrier before giving up
    int64_t g;           // number of tiles
    int64_t *ctrl;       // this level's slice of the output control list
    double *hist;
    int64_t hist_cap;
    int64_t cap_level;
    const int64_t *seeds;  // device [n_seeds]
    int64_t n_seeds;
    int64_t max_iter;
    int64_t keep_cols;   // two-launch update: columns read with the default cache policy (KEEP_BYTES)
};

struct SelShared {
    Cand sh[UWAVES];
    double red[UWAVES];
    int32_t stop, skip;
    int64_t n, p;
    double m2, d, c[3], xp[3];
};

struct UpdShared {
    double lsh[LCHUNK];
    double psum[UWAVES][UPB];
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

// phi(||x_i - x_j|| / R) of the selected basis (Table 1), distance term by term with no
// contraction; only a few of these are computed per iteration.
template <int DIM>
__device__ __forceinline__ double phi_pair(const double *xs, int64_t ld, int64_t i, int64_t j, double R,
                                           int32_t basis)
{
    double s = 0.0;
    {
#pragma clang fp contract(off)
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double d = xs[k * ld + i] - xs[k * ld + j];
            s = s + d * d;
        }
    }
    double eta = sqrt(s) / R;
    if (eta >= 1.0) return 0.0;
    return wendland(basis, eta);
}

// phi_pair on coordinates already at hand, with the same arithmetic.
template <int DIM>
__device__ __forceinline__ double phi_xy(const double (&x)[DIM], const double (&y)[DIM], double R, int32_t basis)
{
    double s = 0.0;
    {
#pragma clang fp contract(off)
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double d = x[k] - y[k];
            s = s + d * d;
        }
    }
    double eta = sqrt(s) / R;
    if (eta >= 1.0) return 0.0;
    return wendland(basis, eta);
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

// E = r, selected = 0, per-tile max of ||r_i||^2 (no exclusions).
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

// Fixed-order reduction of the per-tile maxima by one workgroup of NT threads.
__device__ void block_argmax(const Cand *part, int64_t g, double &m2, int64_t &idx, Cand *sh)
{
    double bm = -1.0;
    int64_t bi = -1;
    for (int64_t b = threadIdx.x; b < g; b += NT) {
        Cand c = part[b];
        if (better(c.m2, c.idx, bm, bi)) {
            bm = c.m2;
            bi = c.idx;
        }
    }
    wave_argmax(bm, bi);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[w] = Cand{bm, bi};
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < UWAVES; ++k)
            if (better(sh[k].m2, sh[k].idx, bm, bi)) {
                bm = sh[k].m2;
                bi = sh[k].idx;
            }
        sh[0] = Cand{bm, bi};
    }
    __syncthreads();
    m2 = sh[0].m2;
    idx = sh[0].idx;
    __syncthreads();
}

// Level start: the level target max(eps, rho * max ||r||), squared.
__global__ __launch_bounds__(NT) void g_begin(GState *st, const Cand *part, int64_t g, double eps,
                                              double rho, int32_t last)
{
    __shared__ Cand sh[UWAVES];
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

// Select phase (one workgroup): finish the pending column, choose the next point (argmax or a
// forced seed), apply the stop tests, extract the Newton row l = V[p, 0:n] as row n of the
// Cholesky factor and form the pivot d = sqrt(phi(0) - l.l) and the coefficients y_n = E_p / d.
// Two rounds of memory reads: the level state with the per-tile maxima, then the row with E_p.
template <int DIM>
__device__ void select_phase(const GArgs &a, int64_t forced, SelShared &s)
{
    GState *st = a.st;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int32_t stop0 = 0, go0 = 0;
    int64_t n0 = 0;
    double target2 = 0.0;
    if (threadIdx.x == 0) {
        stop0 = st->stop;
        go0 = st->go;
        n0 = st->n;
        target2 = st->target2;
    }
    if (forced < 0) {
        double bm = -1.0;
        int64_t bi = -1;
        // SEL_U maxima per thread in flight at once, then compared in the same order.
        for (int64_t b0 = threadIdx.x; b0 < a.g; b0 += (int64_t)NT * SEL_U) {
            Cand cv[SEL_U];
#pragma unroll
            for (int r = 0; r < SEL_U; ++r) {
                const int64_t b = b0 + (int64_t)r * NT;
                cv[r] = b < a.g ? a.part[b] : Cand{-1.0, -1};
            }
#pragma unroll
            for (int r = 0; r < SEL_U; ++r)
                if (better(cv[r].m2, cv[r].idx, bm, bi)) {
                    bm = cv[r].m2;
                    bi = cv[r].idx;
                }
        }
        wave_argmax(bm, bi);
        if (lane == 0) s.sh[w] = Cand{bm, bi};
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s.skip = stop0 >= 0;               // level already finished
        if (!s.skip && go0) {              // the previous update completed column n
            n0 += 1;
            st->n = n0;
            st->go = 0;
        }
        s.n = n0;
        double m2 = 0.0;
        int64_t p = forced;
        if (forced < 0) {
            m2 = s.sh[0].m2;
            p = s.sh[0].idx;
            for (int k = 1; k < UWAVES; ++k)
                if (better(s.sh[k].m2, s.sh[k].idx, m2, p)) {
                    m2 = s.sh[k].m2;
                    p = s.sh[k].idx;
                }
        }
        int32_t stop = -1;
        if (!s.skip) {
            if (forced < 0) {
                if (p < 0) stop = RBF_STOP_ALL_SELECTED;
                else if (m2 < target2) stop = RBF_STOP_EPS;
            }
            if (stop < 0 && n0 >= a.cap_level) stop = RBF_STOP_CAP;
            if (stop >= 0) st->stop = stop;
        }
        s.stop = stop;
        s.p = p;
        s.m2 = m2;
    }
    __syncthreads();
    if (s.skip || s.stop >= 0) return;
    const int64_t n = s.n, p = s.p;

    double *row = a.Lpack + (n * (n + 1)) / 2;
    double ep[DIM];
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < DIM; ++k) ep[k] = a.E[k * a.n_s + p];
    // The row's entries (one per 512-byte column of p's tile): SEL_U loads per thread in flight
    // before any is stored or summed, the sum in increasing j as before.
    const double *prow = a.V + (p / UPB) * a.ldt * UPB + (p % UPB);
    double part_ll = 0.0;
    for (int64_t j0 = threadIdx.x; j0 < n; j0 += (int64_t)NT * SEL_U) {
        double v[SEL_U];
#pragma unroll
        for (int r = 0; r < SEL_U; ++r) {
            const int64_t j = j0 + (int64_t)r * NT;
            v[r] = j < n ? prow[j * UPB] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < SEL_U; ++r) {
            const int64_t j = j0 + (int64_t)r * NT;
            if (j < n) {
                row[j] = v[r];
                part_ll = __builtin_fma(v[r], v[r], part_ll);
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part_ll += __shfl_xor(part_ll, off, 64);
    if (lane == 0) s.red[w] = part_ll;
    __syncthreads();
    if (threadIdx.x == 0) {
        double ll = s.red[0];
        for (int k = 1; k < UWAVES; ++k) ll += s.red[k];
        const double d2 = 1.0 - ll;       // phi(0) - l.l
        // l.l carries about (n + 1) ulps of rounding: a pivot below that is zero (breakdown).
        if (!(d2 > (double)(n + 1) * 0x1p-52)) {
            st->stop = RBF_STOP_BREAKDOWN;
        } else {
            const double d = sqrt(d2);
            row[n] = d;
            st->p = p;
            st->d = d;
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                const double c = ep[k] / d;
                st->c[k] = c;
                a.coef[k * a.ld_coef + n] = c;
            }
            a.ctrl[n] = p;
            a.sel[p] = 1;
            if (forced < 0) {
                if (st->n_iter < a.hist_cap) a.hist[st->n_iter] = sqrt(s.m2);
                st->n_iter += 1;
            }
            st->go = 1;
        }
    }
    __syncthreads();
}

// Update phase for one tile of 64 surface points: lane = point, wave = slice of the dot product
// V[i, 0:n] . l. Writes column n, updates E and the tile's argmax of ||E_i||^2 over unselected i.
template <int DIM>
__device__ void update_tile(const GArgs &a, int64_t tile, int64_t n, int64_t p, double d,
                            const double (&c)[DIM], UpdShared &u)
{
    const double *lrow = a.Lpack + (n * (n + 1)) / 2;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = tile * UPB + lane;
    const bool ok = i < a.n_s;
    const double *vt = a.V + tile * a.ldt * UPB + lane;   // this tile's columns, 512 B each

    double s = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += LCHUNK) {
        const int nj = (int)min<int64_t>(LCHUNK, n - j0);
        __syncthreads();
        for (int t = threadIdx.x; t < nj; t += NT) u.lsh[t] = lrow[j0 + t];
        __syncthreads();
        const int per = (nj + UWAVES - 1) / UWAVES;
        const int jb = w * per, je = min(nj, jb + per);
        const double *col = vt + (j0 + jb) * UPB;
        int j = jb;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        // Sixteen column loads in flight per lane before any is consumed: the loop is bound by
        // memory, not by the multiply-adds.
        // Blocks of 16 wholly below keep_cols take the default cache policy, the rest are read
        // non-temporally; the sums run in the same order either way.
        const int64_t jk = a.keep_cols - j0;
        for (; j + 16 <= je && j + 16 <= jk; j += 16, col += 16 * UPB) {
            double v[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = col[q * UPB];
#pragma unroll
            for (int q = 0; q < 16; q += 4) {
                s0 = __builtin_fma(v[q], u.lsh[j + q], s0);
                s1 = __builtin_fma(v[q + 1], u.lsh[j + q + 1], s1);
                s2 = __builtin_fma(v[q + 2], u.lsh[j + q + 2], s2);
                s3 = __builtin_fma(v[q + 3], u.lsh[j + q + 3], s3);
            }
        }
        for (; j + 16 <= je; j += 16, col += 16 * UPB) {
            double v[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = __builtin_nontemporal_load(col + q * UPB);
#pragma unroll
            for (int q = 0; q < 16; q += 4) {
                s0 = __builtin_fma(v[q], u.lsh[j + q], s0);
                s1 = __builtin_fma(v[q + 1], u.lsh[j + q + 1], s1);
                s2 = __builtin_fma(v[q + 2], u.lsh[j + q + 2], s2);
                s3 = __builtin_fma(v[q + 3], u.lsh[j + q + 3], s3);
            }
        }
        for (; j + 4 <= je; j += 4, col += 4 * UPB) {
            s0 = __builtin_fma(col[0], u.lsh[j], s0);
            s1 = __builtin_fma(col[UPB], u.lsh[j + 1], s1);
            s2 = __builtin_fma(col[2 * UPB], u.lsh[j + 2], s2);
            s3 = __builtin_fma(col[3 * UPB], u.lsh[j + 3], s3);
        }
        for (; j < je; ++j, col += UPB) s0 = __builtin_fma(col[0], u.lsh[j], s0);
        s += (s0 + s1) + (s2 + s3);
    }
    u.psum[w][lane] = s;
    __syncthreads();
    if (w == 0) {
        double m2 = -1.0;
        int64_t idx = -1;
        if (ok) {
            double dot = u.psum[0][lane];
#pragma unroll
            for (int k = 1; k < UWAVES; ++k) dot += u.psum[k][lane];
            const double v = (phi_pair<DIM>(a.xs, a.n_s, i, p, a.R, a.basis) - dot) / d;
            a.V[(tile * a.ldt + n) * UPB + lane] = v;
#pragma unroll
            for (int k = 0; k < DIM; ++k) a.E[k * a.n_s + i] = __builtin_fma(-c[k], v, a.E[k * a.n_s + i]);
            if (!a.sel[i]) {
                m2 = norm2_plain<DIM>(a.E, a.n_s, i);
                idx = i;
            }
        }
        wave_argmax(m2, idx);
        if (lane == 0) a.part[tile] = Cand{m2, idx};
    }
    __syncthreads();
}

// ---- two-kernel form (fallback) -------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(NT) void g_select(GArgs a, int64_t forced)
{
    __shared__ SelShared s;
    select_phase<DIM>(a, forced, s);
}

template <int DIM>
__global__ __launch_bounds__(NT) void g_update(GArgs a)
{
    __shared__ UpdShared u;
    const GState *st = a.st;
    if (!st->go) return;
    double c[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) c[k] = st->c[k];
    update_tile<DIM>(a, blockIdx.x, st->n, st->p, st->d, c, u);
}

// ---- persistent cooperative form ----------------------------------------------------------------
// Every workgroup runs the same iteration count: the loop ends when the state read after a grid
// barrier says the level stopped (or after max_iter iterations, a bound the level can never
// legitimately reach), so all workgroups leave together.
template <int DIM>
__global__ __launch_bounds__(NT) void g_level(GArgs a)
{
    __shared__ SelShared s;
    __shared__ UpdShared u;
    __shared__ int32_t go_sh;
    __shared__ int64_t n_sh, p_sh;
    __shared__ double d_sh, c_sh[3];
    cg::grid_group grid = cg::this_grid();
    for (int64_t it = 0; it < a.max_iter; ++it) {
        if (blockIdx.x == 0) select_phase<DIM>(a, it < a.n_seeds ? a.seeds[it] : -1, s);
        grid.sync();
        if (threadIdx.x == 0) {
            const GState *st = a.st;
            go_sh = st->go;
            n_sh = st->n;
            p_sh = st->p;
            d_sh = st->d;
            for (int k = 0; k < DIM; ++k) c_sh[k] = st->c[k];
        }
        __syncthreads();
        if (!go_sh) break;
        double c[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) c[k] = c_sh[k];
        const int64_t n = n_sh, p = p_sh;
        const double d = d_sh;
        for (int64_t t = blockIdx.x; t < a.g; t += gridDim.x) update_tile<DIM>(a, t, n, p, d, c, u);
        grid.sync();
    }
}

// ---- persistent form: one barrier per iteration, the select phase in every workgroup ---------
// Iteration it: update(it) applies the column appended by select(it - 1) to this workgroup's
// tiles, then a grid barrier, then select(it) runs in every workgroup on the same data with the
// same fixed-order reductions, so all of them take the same decisions and leave at the same
// iteration; workgroup 0 alone writes the outputs. A workgroup may start update(it + 1) while
// another still runs select(it), so what select(it) reads is never written by update(it + 1):
// the error E and the per-tile maxima alternate between two buffers by iteration parity, the
// Newton row is read from columns below n (update(it + 1) writes column n), and the update
// excludes the point just selected by its own copy of p rather than through sel[].
struct GridBar {
    unsigned int count;   // arrivals so far (all iterations); zeroed before the launch
    unsigned int pad;
};

// Default bound on the polls of one barrier (each after a short sleep, about 4 s in all): far
// beyond any iteration, it only ends a wait that could never be met, with a fault flag instead of
// a hang. RBF_GREEDY_SPIN_LIMIT overrides it (0: give up at the first poll that finds the count
// short, which makes the failure path testable).
constexpr unsigned long long LEAN_SPIN_LIMIT = 1ull << 22;

// V(i, jb .. je) . l(jb .. je) for one wave's slice of a tile's columns (V(i, jb) at col[0], the
// next column UPB doubles on): 16 loads in flight, four partial sums in a fixed order.
__device__ __forceinline__ double slice_dot(const double *col, const double *l, int jb, int je)
{
    int j = jb;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (; j + 16 <= je; j += 16, col += 16 * UPB) {
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = col[q * UPB];
#pragma unroll
        for (int q = 0; q < 16; q += 4) {
            s0 = __builtin_fma(v[q], l[j + q], s0);
            s1 = __builtin_fma(v[q + 1], l[j + q + 1], s1);
            s2 = __builtin_fma(v[q + 2], l[j + q + 2], s2);
            s3 = __builtin_fma(v[q + 3], l[j + q + 3], s3);
        }
    }
    for (; j + 4 <= je; j += 4, col += 4 * UPB) {
        s0 = __builtin_fma(col[0], l[j], s0);
        s1 = __builtin_fma(col[UPB], l[j + 1], s1);
        s2 = __builtin_fma(col[2 * UPB], l[j + 2], s2);
        s3 = __builtin_fma(col[3 * UPB], l[j + 3], s3);
    }
    for (; j < je; ++j, col += UPB) s0 = __builtin_fma(col[0], l[j], s0);
    return (s0 + s1) + (s2 + s3);
}

// What a resident workgroup keeps of its tile's row in each lane between iterations: the error as
// it last wrote it, the coordinates, and whether the row was selected in this level (or lies past
// the surface). With its first RES_COLS Newton columns in LDS, an update of up to RES_COLS columns
// reads no global memory.
template <int DIM>
struct ResRow {
    double e[DIM];
    double x[DIM];
    bool sel;
};

template <int DIM, bool RES>
__device__ void update_tile_lean(const GArgs &a, int64_t tile, int64_t n, int64_t p, double d,
                                 const double (&c)[DIM], const double (&xp)[DIM], bool row_in_lds,
                                 const double *Ein, double *Eout, Cand *part_out, UpdShared &u, double *vres,
                                 ResRow<DIM> &rr)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = tile * UPB + lane;
    const bool ok = i < a.n_s;
    const double *vt = a.V + tile * a.ldt * UPB + lane;
    const double *prow = a.V + (p / UPB) * a.ldt * UPB + (p % UPB);   // V(p, j) at prow[j UPB]
    const bool lds = RES && n <= RES_COLS;                               // every column in LDS

    double s = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += LCHUNK) {
        const int nj = (int)min<int64_t>(LCHUNK, n - j0);
        if (!row_in_lds) {
            __syncthreads();
            for (int t = threadIdx.x; t < nj; t += NT)
                u.lsh[t] = prow[(j0 + t) * UPB];
            __syncthreads();
        }
        const int per = (nj + UWAVES - 1) / UWAVES;
        const int jb = w * per, je = min(nj, jb + per);
        if (lds) s += slice_dot(vres + jb * UPB + lane, u.lsh, jb, je);
        else s += slice_dot(vt + (j0 + jb) * UPB, u.lsh, jb, je);
    }
    __syncthreads();                                    // psum of the previous tile has been read
    u.psum[w][lane] = s;
    __syncthreads();
    if (w == 0) {
        double m2 = -1.0;
        int64_t idx = -1;
        if (RES) rr.sel = rr.sel || i == p;
        if (ok) {
            double dot = u.psum[0][lane];
#pragma unroll
            for (int k = 1; k < UWAVES; ++k) dot += u.psum[k][lane];
            const double ph = RES ? phi_xy<DIM>(rr.x, xp, a.R, a.basis) : phi_pair<DIM>(a.xs, a.n_s, i, p, a.R, a.basis);
            const double v = (ph - dot) / d;
            a.V[(tile * a.ldt + n) * UPB + lane] = v;
            if (RES && n < RES_COLS) vres[n * UPB + lane] = v;
            double e[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                e[k] = __builtin_fma(-c[k], v, RES ? rr.e[k] : Ein[k * a.n_s + i]);
                Eout[k * a.n_s + i] = e[k];
                if (RES) rr.e[k] = e[k];
            }
            if (RES ? !rr.sel : (i != p && !a.sel[i])) {
#pragma clang fp contract(off)
                double q = e[0] * e[0];
#pragma unroll
                for (int k = 1; k < DIM; ++k) q = q + e[k] * e[k];
                m2 = q;
                idx = i;
            }
        }
        wave_argmax(m2, idx);
        if (lane == 0) part_out[tile] = Cand{m2, idx};
    }
}

// The select phase of the persistent form, run by every workgroup on the state after the
// barrier: the next point (argmax of the per-tile maxima, or a forced seed), the stop tests, the
// Newton row l = V[p, 0:n] (kept in LDS for the update when it fits), the pivot and the Newton
// coefficients. Workgroup 0 writes the outputs. Returns false when the level stops.
template <int DIM>
__device__ bool select_lean(const GArgs &a, int64_t forced, int64_t n, double target2, int64_t &n_iter,
                            const double *Ecur, const Cand *part, SelShared &s, UpdShared &u,
                            int64_t &p_out, double &d_out, double (&c_out)[DIM], double (&xp_out)[DIM])
{
    GState *st = a.st;
    const bool writer = blockIdx.x == 0;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (forced < 0) {
        double bm = -1.0;
        int64_t bi = -1;
        for (int64_t b0 = threadIdx.x; b0 < a.g; b0 += (int64_t)NT * SEL_U) {
            Cand cv[SEL_U];
#pragma unroll
            for (int r = 0; r < SEL_U; ++r) {
                const int64_t b = b0 + (int64_t)r * NT;
                cv[r] = b < a.g ? part[b] : Cand{-1.0, -1};
            }
#pragma unroll
            for (int r = 0; r < SEL_U; ++r)
                if (better(cv[r].m2, cv[r].idx, bm, bi)) {
                    bm = cv[r].m2;
                    bi = cv[r].idx;
                }
        }
        wave_argmax(bm, bi);
        if (lane == 0) s.sh[w] = Cand{bm, bi};
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m2 = 0.0;
        int64_t p = forced;
        if (forced < 0) {
            m2 = s.sh[0].m2;
            p = s.sh[0].idx;
            for (int k = 1; k < UWAVES; ++k)
                if (better(s.sh[k].m2, s.sh[k].idx, m2, p)) {
                    m2 = s.sh[k].m2;
                    p = s.sh[k].idx;
                }
        }
        int32_t stop = -1;
        if (forced < 0) {
            if (p < 0) stop = RBF_STOP_ALL_SELECTED;
            else if (m2 < target2) stop = RBF_STOP_EPS;
        }
        if (stop < 0 && n >= a.cap_level) stop = RBF_STOP_CAP;
        s.stop = stop;
        s.p = p;
        s.m2 = m2;
    }
    __syncthreads();
    if (s.stop >= 0) {
        if (writer && threadIdx.x == 0) {
            st->n = n;
            st->go = 0;
            st->n_iter = n_iter;
            st->stop = s.stop;
        }
        return false;
    }
    const int64_t p = s.p;
    double *row = a.Lpack + (n * (n + 1)) / 2;
    double ep[DIM], xp[DIM];
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            ep[k] = Ecur[k * a.n_s + p];
            xp[k] = a.xs[k * a.n_s + p];
        }
    const double *prow = a.V + (p / UPB) * a.ldt * UPB + (p % UPB);
    double part_ll = 0.0;
    for (int64_t j0 = threadIdx.x; j0 < n; j0 += (int64_t)NT * SEL_U) {
        double v[SEL_U];
#pragma unroll
        for (int r = 0; r < SEL_U; ++r) {
            const int64_t j = j0 + (int64_t)r * NT;
            v[r] = j < n ? prow[j * UPB] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < SEL_U; ++r) {
            const int64_t j = j0 + (int64_t)r * NT;
            if (j < n) {
                if (j < LCHUNK) u.lsh[j] = v[r];
                if (writer) row[j] = v[r];
                part_ll = __builtin_fma(v[r], v[r], part_ll);
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part_ll += __shfl_xor(part_ll, off, 64);
    if (lane == 0) s.red[w] = part_ll;
    __syncthreads();
    if (threadIdx.x == 0) {
        double ll = s.red[0];
        for (int k = 1; k < UWAVES; ++k) ll += s.red[k];
        const double d2 = 1.0 - ll;       // phi(0) - l.l
        // l.l carries about (n + 1) ulps of rounding: a pivot below that is zero (breakdown).
        if (!(d2 > (double)(n + 1) * 0x1p-52)) {
            s.stop = RBF_STOP_BREAKDOWN;
            if (writer) {
                st->n = n;
                st->go = 0;
                st->n_iter = n_iter;
                st->stop = RBF_STOP_BREAKDOWN;
            }
        } else {
            const double d = sqrt(d2);
            s.d = d;
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                s.c[k] = ep[k] / d;
                s.xp[k] = xp[k];
            }
            if (writer) {
                row[n] = d;
                st->p = p;
                st->d = d;
#pragma unroll
                for (int k = 0; k < DIM; ++k) {
                    st->c[k] = s.c[k];
                    a.coef[k * a.ld_coef + n] = s.c[k];
                }
                a.ctrl[n] = p;
                a.sel[p] = 1;
                if (forced < 0) {
                    if (n_iter < a.hist_cap) a.hist[n_iter] = sqrt(s.m2);
                    n_iter += 1;
                }
                st->n = n;
                st->n_iter = n_iter;
                st->go = 1;
            }
        }
    }
    __syncthreads();
    if (s.stop >= 0) return false;
    p_out = p;
    d_out = s.d;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        c_out[k] = s.c[k];
        xp_out[k] = s.xp[k];
    }
    return true;
}

// RES: one tile per workgroup (the grid has a.g workgroups), resident as ResRow describes.
template <int DIM, bool RES>
__global__ __launch_bounds__(NT) void g_level_lean(GArgs a, GridBar *bar)
{
    __shared__ SelShared s;
    __shared__ UpdShared u;
    __shared__ int32_t abort_sh;
    __shared__ double vres[RES ? RES_COLS * UPB : 1];   // V(tile, j) for j < RES_COLS, column-major
    const unsigned int nb = gridDim.x;
    // Level state, read before this workgroup's first arrival: workgroup 0 writes it only after
    // every workgroup has arrived.
    int64_t n = a.st->n;
    int64_t n_iter = a.st->n_iter;
    const double target2 = a.st->target2;
    bool pending = false;
    int64_t p = -1;
    double d = 1.0, c[DIM], xp[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) c[k] = xp[k] = 0.0;
    double *Eb[2] = {a.E, a.E2};
    Cand *Pb[2] = {a.part, a.part2};
    ResRow<DIM> rr;
    if constexpr (RES) {
        // The level's first error (in a.E), this tile's rows and existing columns; the barrier
        // below orders these LDS writes before any read.
        const int64_t i = (int64_t)blockIdx.x * UPB + (threadIdx.x & 63);
        const bool ok = i < a.n_s;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            rr.e[k] = ok ? a.E[k * a.n_s + i] : 0.0;
            rr.x[k] = ok ? a.xs[k * a.n_s + i] : 0.0;
        }
        rr.sel = !ok || a.sel[i] != 0;
        const double *vt = a.V + (int64_t)blockIdx.x * a.ldt * UPB;
        const int64_t nf = min<int64_t>(n, RES_COLS) * UPB;
        for (int64_t t = threadIdx.x; t < nf; t += NT) vres[t] = vt[t];
    }
    for (int64_t it = 0; it < a.max_iter; ++it) {
        const int par = (int)(it & 1);
        if (pending) {
            const bool row_in_lds = n <= LCHUNK;
            if constexpr (RES)
                update_tile_lean<DIM, true>(a, blockIdx.x, n, p, d, c, xp, row_in_lds, Eb[par ^ 1], Eb[par],
                                            Pb[par], u, vres, rr);
            else
                for (int64_t t = blockIdx.x; t < a.g; t += nb)
                    update_tile_lean<DIM, false>(a, t, n, p, d, c, xp, row_in_lds, Eb[par ^ 1], Eb[par], Pb[par],
                                                 u, vres, rr);
            n += 1;
            pending = false;
        }
        // Grid barrier: one release per arrival, relaxed polls of the arrival count, one acquire.
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_add(&bar->count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned int target = nb * (unsigned int)(it + 1);
            unsigned long long spins = 0;
            int32_t ab = 0;
            while (__hip_atomic_load(&bar->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (spins++ >= a.spin_limit) {
                    ab = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            abort_sh = ab;
            if (ab) __hip_atomic_store(&a.st->fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        if (abort_sh) return;
        const int64_t forced = it < a.n_seeds ? a.seeds[it] : -1;
        if (!select_lean<DIM>(a, forced, n, target2, n_iter, Eb[par], Pb[par], s, u, p, d, c, xp)) break;
        pending = true;
    }
}

// Back substitution L^T alpha = y of a level's packed factor (row j at j (j + 1) / 2) in one
// launch, 64-row blocks from the last, chained as in the dense solve: the workgroup owning a block
// removes the contributions L_j,kb^T alpha_j of the later blocks as each is published, then solves
// its diagonal block by substitution (lane i holds row i; the reciprocals of the pivots are formed
// beforehand and each finished unknown is broadcast from its lane) and publishes the block. It
// also gathers its block's control coordinates. A level has few blocks, so the substitution stays
// on the chain rather than an inverse formed while waiting. st: [0] ticket, then one done flag
// per block (zeroed before the launch); a wait that gives up raises gs->fault.
template <int DIM>
__global__ __launch_bounds__(64) void g_backsolve_chain(const double *Lpack, int64_t n, const double *y,
                                                        int64_t ld_y, double *alpha, int64_t ld_a,
                                                        const double *xs, int64_t n_s, const int64_t *ctrl,
                                                        double *xc, int32_t *st, GState *gs,
                                                        unsigned long long spin_limit)
{
    __shared__ double Ld[TC_NB][TC_NB + 1];   // the diagonal block
    __shared__ double Ls[TC_NB][TC_NB + 1];   // one later block's rows, L_j,kb
    __shared__ double vec[DIM][TC_NB];
    __shared__ double rl[TC_NB];
    __shared__ int32_t sh_kb, ok_sh;
    const int t = threadIdx.x;
    const int64_t nblk = (n + TC_NB - 1) / TC_NB;
    if (t == 0) sh_kb = __hip_atomic_fetch_add(&st[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int64_t kb = nblk - 1 - sh_kb, k0 = kb * TC_NB;
    if (k0 + t < n) {
        const int64_t p = ctrl[k0 + t];
#pragma unroll
        for (int k = 0; k < DIM; ++k) xc[k * ld_a + k0 + t] = xs[k * n_s + p];
    }
    // Diagonal block, identity past the level's n rows. Every lane loads from a valid element (row
    // and column clamped into the packed triangle) and selects afterwards, so the loads carry no
    // branch and 16 of them are in flight.
#pragma unroll 16
    for (int r = 0; r < TC_NB; ++r) {
        const int64_t i = min(k0 + r, n - 1);
        const int64_t c = min(k0 + (int64_t)t, i);
        const double v = Lpack[(i * (i + 1)) / 2 + c];
        Ld[r][t] = (k0 + r < n && t <= r) ? v : (r == t ? 1.0 : 0.0);
    }
    __syncthreads();
    rl[t] = 1.0 / Ld[t][t];
    double x[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) x[k] = k0 + t < n ? y[k * ld_y + k0 + t] : 0.0;
    for (int64_t j = nblk - 1; j > kb; --j) {
        __syncthreads();
#pragma unroll 16
        for (int r = 0; r < TC_NB; ++r) {   // L_j,kb: columns k0 + t lie left of every row i >= 64 j
            const int64_t i = min(j * TC_NB + r, n - 1);   // a row of block j (64 j < n)
            const double v = Lpack[(i * (i + 1)) / 2 + k0 + t];
            Ls[r][t] = j * TC_NB + r < n ? v : 0.0;
        }
        if (!tc_wait(&st[1 + j], 1, &gs->fault, spin_limit, ok_sh)) return;
#pragma unroll
        for (int k = 0; k < DIM; ++k) vec[k][t] = j * TC_NB + t < n ? alpha[k * ld_a + j * TC_NB + t] : 0.0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int r = 0; r < TC_NB; r += 2) {
                s0 = __builtin_fma(Ls[r][t], vec[k][r], s0);
                s1 = __builtin_fma(Ls[r + 1][t], vec[k][r + 1], s1);
            }
            x[k] -= s0 + s1;
        }
    }
    __syncthreads();
    for (int i = TC_NB - 1; i >= 0; --i) {
        const double ri = rl[i];
        double xi[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) xi[k] = __shfl(x[k], i, 64) * ri;
        if (t < i) {
#pragma unroll
            for (int k = 0; k < DIM; ++k) x[k] = __builtin_fma(-Ld[i][t], xi[k], x[k]);
        } else if (t == i) {
#pragma unroll
            for (int k = 0; k < DIM; ++k) x[k] = xi[k];
        }
    }
    if (k0 + t < n) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) alpha[k * ld_a + k0 + t] = x[k];
    }
    tc_publish(&st[1 + kb]);
}

// ---- warm start from a resident basis --------------------------------------------------------
// Forward substitution L y = b for rows [b0, b1) of the packed factor (earlier rows done): every
// workgroup solves the diagonal block, workgroup 0 stores y, and each removes the block's
// contribution from its share of the rows below b1.
template <int DIM>
__global__ __launch_bounds__(256) void g_fwdsolve(const double *Lpack, double *b, int64_t ld_b,
                                                  double *y, int64_t ld_y, int64_t n, int64_t b0, int64_t b1)
{
    __shared__ double Lb[64][65];
    __shared__ double inv[64];
    __shared__ double xb[DIM][64];
    const int nb = (int)(b1 - b0);
    // Every thread loads a valid element (row and column clamped into the block's triangle) and
    // masks it afterwards: no branch around the loads, all 16 in flight. Masked entries (above the
    // diagonal or past the block's rows) may become -0 and are never read for a result.
#pragma unroll
    for (int q = 0; q < 16; ++q) {   // launched with 256 threads: 16 passes cover the 64 x 64 block
        const int t = (int)threadIdx.x + 256 * q;
        const int r = t / 64, c = t % 64;
        const int64_t i = b0 + min(r, nb - 1);
        const int64_t cc = b0 + min(c, (int)(i - b0));
        const double v = Lpack[(i * (i + 1)) / 2 + cc];
        Lb[r][c] = v * ((r < nb && c <= r) ? 1.0 : 0.0);   // a mask, not a select the compiler could
                                                            // turn back into a branch around the load
    }
    if (threadIdx.x < 64) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) xb[k][threadIdx.x] = threadIdx.x < nb ? b[k * ld_b + b0 + threadIdx.x] : 0.0;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int j = threadIdx.x;
        inv[j] = j < nb ? 1.0 / Lb[j][j] : 0.0;
        double rhs[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) rhs[k] = xb[k][j];
        for (int i = 0; i < nb; ++i) {
            const double ii = inv[i];
            double xi[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) xi[k] = __shfl(rhs[k], i, 64) * ii;
            if (j > i) {
#pragma unroll
                for (int k = 0; k < DIM; ++k) rhs[k] = __builtin_fma(-Lb[j][i], xi[k], rhs[k]);
            } else if (j == i) {
#pragma unroll
                for (int k = 0; k < DIM; ++k) rhs[k] = xi[k];
            }
        }
#pragma unroll
        for (int k = 0; k < DIM; ++k) xb[k][j] = rhs[k];
        if (blockIdx.x == 0 && j < nb) {
#pragma unroll
            for (int k = 0; k < DIM; ++k) y[k * ld_y + b0 + j] = rhs[k];
        }
    }
    __syncthreads();
    for (int64_t r = b1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        const double *row = Lpack + (r * (r + 1)) / 2 + b0;
        double acc[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) acc[k] = 0.0;
        for (int i = 0; i < nb; ++i) {
            const double l = row[i];
#pragma unroll
            for (int k = 0; k < DIM; ++k) acc[k] = __builtin_fma(l, xb[k][i], acc[k]);
        }
#pragma unroll
        for (int k = 0; k < DIM; ++k) b[k * ld_b + r] -= acc[k];
    }
}

// b[k][j] = r[k][ctrl[j]] (the residual at the control points) and sel[ctrl[j]] = 1.
template <int DIM>
__global__ __launch_bounds__(256) void g_seed_rhs(const double *r, int64_t n_s, const int64_t *ctrl,
                                                  int64_t n, double *b, int64_t ld_b, uint8_t *sel)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = ctrl[j];
#pragma unroll
        for (int k = 0; k < DIM; ++k) b[k * ld_b + j] = r[k * n_s + p];
        sel[p] = 1;
    }
}

// xc[k][j] = xs[k][seeds[j]]: the seeds' coordinates, gathered for the dense factor.
template <int DIM>
__global__ __launch_bounds__(256) void g_gather_seeds(const double *xs, int64_t n_s, const int64_t *seeds, int64_t n,
                                                      double *xc)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = seeds[j];
#pragma unroll
        for (int k = 0; k < DIM; ++k) xc[k * n + j] = xs[k * n_s + p];
    }
}

// E = r - V y over all surface points for the n resident columns (Newton coefficients y in
// coef), and the per-tile argmax of ||E_i||^2 over unselected points.
template <int DIM>
__global__ __launch_bounds__(NT) void g_apply(GArgs a, const double *r, int64_t n)
{
    __shared__ double ysh[DIM][LCHUNK / 2];
    __shared__ double psum[UWAVES][DIM][UPB];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * UPB + lane;
    const bool ok = i < a.n_s;
    double s[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) s[k] = 0.0;
    constexpr int CH = LCHUNK / 2;
    for (int64_t j0 = 0; j0 < n; j0 += CH) {
        const int nj = (int)min<int64_t>(CH, n - j0);
        __syncthreads();
        for (int t = threadIdx.x; t < nj; t += NT)
#pragma unroll
            for (int k = 0; k < DIM; ++k) ysh[k][t] = a.coef[k * a.ld_coef + j0 + t];
        __syncthreads();
        const int per = (nj + UWAVES - 1) / UWAVES;
        const int jb = w * per, je = min(nj, jb + per);
        for (int j = jb; j < je; ++j) {
            const double v = a.V[((int64_t)blockIdx.x * a.ldt + j0 + j) * UPB + lane];
#pragma unroll
            for (int k = 0; k < DIM; ++k) s[k] = __builtin_fma(v, ysh[k][j], s[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k) psum[w][k][lane] = s[k];
    __syncthreads();
    if (w == 0) {
        double m2 = -1.0;
        int64_t idx = -1;
        if (ok) {
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                double dot = psum[0][k][lane];
                for (int q = 1; q < UWAVES; ++q) dot += psum[q][k][lane];
                a.E[k * a.n_s + i] = r[k * a.n_s + i] - dot;
            }
            if (!a.sel[i]) {
                m2 = norm2_plain<DIM>(a.E, a.n_s, i);
                idx = i;
            }
        }
        wave_argmax(m2, idx);
        if (lane == 0) a.part[blockIdx.x] = Cand{m2, idx};
    }
}

__global__ void g_set_count(GState *st, int64_t n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->n = n;
        st->go = 0;
        st->stop = -1;
    }
}

// Per-workgroup maximum over its points of ||(r - r_next) - t||: the difference between the
// level's FP64 interpolant (r - r_next) and another evaluation t of it, at the surface points.
template <int DIM>
__global__ __launch_bounds__(256) void g_maxdiff(const double *r, const double *r_next, const double *t,
                                                 int64_t n_s, double *part)
{
    __shared__ double red[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double e2 = 0.0;
    if (i < n_s)
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const double d = (r[k * n_s + i] - r_next[k * n_s + i]) - t[k * n_s + i];
            e2 = __builtin_fma(d, d, e2);
        }
    red[threadIdx.x] = e2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void g_finite(const double *a, int64_t n, int32_t *bad)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(a[i])) *bad = 1;
}

// Holds G workgroups of the context's co-residency budget while a persistent kernel runs.
// Persistent kernels of one context share the device through these tickets: g workgroups of a
// kernel with room for cap on the device. try_alone takes the device for this kernel alone when no
// other persistent kernel runs (alone is then set; nothing else starts until it ends), for a
// kernel whose workgroups each need most of a compute unit's LDS; otherwise the ticket waits for
// room as usual.
struct CoopTicket {
    static constexpr int64_t ALONE = int64_t(1) << 40;
    rbf_ctx ctx;
    int64_t units;
    bool alone = false;
    CoopTicket(rbf_ctx c, int64_t g, int64_t cap, bool try_alone = false) : ctx(c), units(g)
    {
        std::unique_lock<std::mutex> lk(ctx->coop_mu);
        if (try_alone && ctx->coop_in_use == 0) {
            units = ALONE;
            alone = true;
        } else {
            ctx->coop_cv.wait(lk, [&] { return ctx->coop_in_use + units <= cap; });
        }
        ctx->coop_in_use += units;
    }
    ~CoopTicket()
    {
        {
            std::lock_guard<std::mutex> lk(ctx->coop_mu);
            ctx->coop_in_use -= units;
        }
        ctx->coop_cv.notify_all();
    }
};

int cooperative_blocks(const void *kernel, int n_cu)
{
    int dev = 0, coop = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, NT, 0) != hipSuccess) return 0;
    return per_cu * n_cu;
}

template <int DIM>
rbf_status greedy_impl(rbf_ctx ctx, const rbf_greedy_params &prm, int64_t n_s, const double *xs,
                       const double *ds, rbf_ctrl_set *out, hipStream_t s, const std::vector<LevelCache> *warm,
                       std::vector<LevelCache> *store)
{
    Pool *pool = ctx->pool.get();
    const int64_t cap = prm.max_ctrl_total;
    const int64_t cols = std::min<int64_t>(n_s, cap);      // most columns one level can need
    const int64_t g = (n_s + UPB - 1) / UPB;

    DevBuf bV, bL, bE, bR, bR2, bSel, bPart, bState, bCoef, bHist, bFlag, bSeeds;
    // Columns per tile in the basis, odd so that the tiles' regions start at odd multiples of
    // 512 bytes: workgroups that read the same column of their tiles at the same moment then fall
    // on different memory channels instead of one.
    const int64_t ldt = cols | 1;
    RBF_TRY(bV.get(pool, sizeof(double) * (size_t)ldt * (size_t)((n_s + UPB - 1) / UPB) * UPB, s));
    RBF_TRY(bL.get(pool, sizeof(double) * (size_t)(cols * (cols + 1) / 2 + 1), s));
    RBF_TRY(bE.get(pool, sizeof(double) * DIM * (size_t)n_s, s));
    RBF_TRY(bR.get(pool, sizeof(double) * DIM * (size_t)n_s, s));
    RBF_TRY(bR2.get(pool, sizeof(double) * DIM * (size_t)n_s, s));
    RBF_TRY(bSel.get(pool, (size_t)n_s, s));
    RBF_TRY(bPart.get(pool, sizeof(Cand) * (size_t)g, s));
    RBF_TRY(bState.get(pool, sizeof(GState), s));
    RBF_TRY(bCoef.get(pool, sizeof(double) * DIM * (size_t)cols, s));
    RBF_TRY(bHist.get(pool, sizeof(double) * (size_t)cap, s));
    RBF_TRY(bFlag.get(pool, sizeof(int32_t), s));
    const int32_t n_seed_total = prm.seed_off ? prm.seed_off[prm.n_levels] : 1;
    RBF_TRY(bSeeds.get(pool, sizeof(int64_t) * (size_t)std::max(1, n_seed_total), s));
    double *R = bR.as<double>(), *R2 = bR2.as<double>();
    GState *st = bState.as<GState>();

    // Reject non-finite coordinates or displacements.
    RBF_HIP(hipMemsetAsync(bFlag.ptr, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(g_finite, dim3(256), dim3(256), 0, s, xs, (int64_t)DIM * n_s, bFlag.as<int32_t>());
    hipLaunchKernelGGL(g_finite, dim3(256), dim3(256), 0, s, ds, (int64_t)DIM * n_s, bFlag.as<int32_t>());
    int32_t bad = 0;
    RBF_HIP(hipMemcpyAsync(&bad, bFlag.ptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RBF_HIP(hipStreamSynchronize(s));
    if (bad) return fail(RBF_E_INVALID, "xs or ds holds a non-finite value");

    // Seeds of every level (paper default: the first surface point at level 0).
    std::vector<int64_t> seeds_h;
    std::vector<int32_t> seed_off(prm.n_levels + 1, 0);
    if (prm.seed_off) {
        for (int l = 0; l <= prm.n_levels; ++l) seed_off[l] = prm.seed_off[l];
        seeds_h.assign(prm.seed_idx, prm.seed_idx + prm.seed_off[prm.n_levels]);
    } else {
        seeds_h.push_back(0);
        for (int l = 1; l <= prm.n_levels; ++l) seed_off[l] = 1;
    }
    if (!seeds_h.empty())
        RBF_HIP(hipMemcpyAsync(bSeeds.ptr, seeds_h.data(), sizeof(int64_t) * seeds_h.size(),
                               hipMemcpyHostToDevice, s));
    RBF_HIP(hipMemsetAsync(st, 0, sizeof(GState), s));
    // Ticket and done flags of every level's chained back substitution, zeroed once.
    const int64_t chain_stride = 1 + (cols + TC_NB - 1) / TC_NB;
    DevBuf bChain;
    RBF_TRY(bChain.get(pool, sizeof(int32_t) * (size_t)(prm.n_levels * chain_stride), s));
    RBF_HIP(hipMemsetAsync(bChain.ptr, 0, sizeof(int32_t) * (size_t)(prm.n_levels * chain_stride), s));
    RBF_HIP(hipMemcpyAsync(R, ds, sizeof(double) * DIM * n_s, hipMemcpyDeviceToDevice, s));

    // Execution mode: "lean" (one barrier per iteration), "cg" (cooperative-groups grid
    // barriers) or "kernels" (two launches per iteration). Default: the persistent kernel while the
    // surface has at most LEAN_MAX_TILES tiles (latency-bound iterations, where launches would
    // dominate), two launches per iteration beyond that: there the basis stream is the cost, and
    // fresh launches stream it faster than the persistent kernel, whose per-workgroup release and
    // acquire each iteration write back and invalidate the L2 of every XCD. The two cost the same
    // near 110 tiles on a three-level wing (measured: 94 tiles 53 vs 55 ms, 120 tiles 56.9 vs
    // 56.2 ms, 188 tiles 94.6 vs 86.6 ms, persistent vs two launches).
    // Seeded starts: blocked factor from SEED_FACTOR_MIN seeds on; RBF_SEED_START=append|factor
    // forces one form (tests and timing).
    int64_t seed_factor_min = SEED_FACTOR_MIN;
    if (const char *e = getenv("RBF_SEED_START"))
        seed_factor_min = !strcmp(e, "append") ? INT64_MAX : !strcmp(e, "factor") ? 1 : SEED_FACTOR_MIN;
    const char *mode_env = getenv("RBF_GREEDY_MODE");
    const int mode = getenv("RBF_NO_COOP") ? 2
                   : (mode_env && !strcmp(mode_env, "cg")) ? 1
                   : (mode_env && !strcmp(mode_env, "kernels")) ? 2
                   : (mode_env && !strcmp(mode_env, "lean")) ? 0
                   : (g > LEAN_MAX_TILES ? 2 : 0);
    const int coop_max = mode == 2 ? 0
                       : cooperative_blocks(mode == 0 ? (const void *)g_level_lean<DIM, false> : (const void *)g_level<DIM>,
                                            ctx->n_cu);
    // The resident form of the persistent kernel (one tile per workgroup, its first RES_COLS
    // Newton columns in LDS: about 115 KB per workgroup) when the device has room for a
    // workgroup per tile; RBF_GREEDY_RESIDENT=0 keeps the plain form.
    const char *res_env = getenv("RBF_GREEDY_RESIDENT");
    const int coop_res = (mode == 0 && !(res_env && res_env[0] == '0'))
                             ? cooperative_blocks((const void *)g_level_lean<DIM, true>, ctx->n_cu) : 0;
    DevBuf bBar, bE2, bPart2;
    RBF_TRY(bBar.get(pool, sizeof(GridBar), s));
    if (mode == 0 && coop_max > 0) {
        RBF_TRY(bE2.get(pool, sizeof(double) * DIM * (size_t)n_s, s));
        RBF_TRY(bPart2.get(pool, sizeof(Cand) * (size_t)g, s));
    }
    GArgs a{};
    a.st = st;
    a.xs = xs;
    a.n_s = n_s;
    a.basis = prm.basis;
    a.V = bV.as<double>();
    a.ldt = ldt;
    a.Lpack = bL.as<double>();
    a.coef = bCoef.as<double>();
    a.ld_coef = cols;
    a.E = bE.as<double>();
    a.sel = bSel.as<uint8_t>();
    a.part = bPart.as<Cand>();
    a.E2 = bE2.as<double>();
    a.part2 = bPart2.as<Cand>();
    a.spin_limit = LEAN_SPIN_LIMIT;
    if (const char *e = getenv("RBF_GREEDY_SPIN_LIMIT")) a.spin_limit = strtoull(e, nullptr, 10);
    a.keep_cols = (KEEP_BYTES / (int64_t)(sizeof(double) * n_s)) / 16 * 16;
    if (const char *e = getenv("RBF_GREEDY_KEEP_COLS")) a.keep_cols = strtoll(e, nullptr, 10);
    a.g = g;
    a.hist = bHist.as<double>();
    a.hist_cap = cap;

    GState hs{};
    int64_t total = 0;
    int used = 0;
    out->level_off[0] = 0;
    for (int l = 0; l < RBF_MAX_LEVELS; ++l) {
        out->level_stop[l] = RBF_STOP_SKIPPED;
        out->level_max_err[l] = 0.0;
        out->level_in_max[l] = 0.0;
        out->level_seconds[l] = 0.0;
        out->level_fp32_err[l] = 0.0;
    }
    for (int l = 0; l < prm.n_levels; ++l) {
        const double t_level = now_seconds();
        const double Rl = prm.radius[l];
        a.R = Rl;
        a.cap_level = std::min<int64_t>(cols, cap - total);
        a.ctrl = out->ctrl_idx + total;
        a.seeds = bSeeds.as<int64_t>() + seed_off[l];
        a.n_seeds = seed_off[l + 1] - seed_off[l];
        a.max_iter = a.n_seeds + a.cap_level + 2;
        if (l == 0) {   // later levels start from the state the previous level's close prepared
            hipLaunchKernelGGL(g_init<DIM>, dim3((unsigned)g), dim3(64), 0, s, R, a.E, a.sel, n_s, a.part);
            hipLaunchKernelGGL(g_begin, dim3(1), dim3(NT), 0, s, st, a.part, g, prm.eps_abs,
                               prm.level_reduction, (int32_t)(prm.n_levels == 1));
            RBF_HIP(hipGetLastError());
        }
        // Warm start from the resident basis of the same control points: copy V and L, then
        // y = L^-1 r_C and E = r - V y; the level continues from n0 columns.
        int64_t n_start = 0;   // columns the level starts with (0: its seeds are appended one by one)
        hipEvent_t seed_timer = nullptr;
        if (warm && l < (int)warm->size()) {
            const LevelCache &lc = (*warm)[l];
            const int64_t n0 = lc.n;
            const bool same = n0 > 0 && n0 == a.n_seeds && lc.radius == Rl && lc.basis == prm.basis &&
                              n0 <= a.cap_level &&
                              std::equal(lc.ctrl.begin(), lc.ctrl.end(), seeds_h.begin() + seed_off[l]);
            if (same) {
                RBF_HIP(hipMemcpy2DAsync(a.V, sizeof(double) * ldt * UPB, lc.V.ptr, sizeof(double) * n0 * UPB,
                                         sizeof(double) * n0 * UPB, g, hipMemcpyDeviceToDevice, s));
                RBF_HIP(hipMemcpyAsync(a.Lpack, lc.L.ptr, sizeof(double) * (n0 * (n0 + 1) / 2),
                                       hipMemcpyDeviceToDevice, s));
                RBF_HIP(hipMemcpyAsync(a.ctrl, lc.ctrl.data(), sizeof(int64_t) * n0, hipMemcpyHostToDevice, s));
                n_start = n0;
            }
        }
        // No resident basis for a level handed enough seeds: L from the blocked FP64 MFMA Cholesky
        // of the seeds' Phi_CC and V = Phi_sC L^-T from blocked triangular solves, in place of n
        // single appends. A seed set whose factor meets a non-positive pivot (a repeated or
        // numerically dependent point) is appended one by one instead, which stops the level at
        // the breakdown as before.
        if (n_start == 0 && a.n_seeds >= seed_factor_min && a.n_seeds <= a.cap_level) {
            const int64_t n0 = a.n_seeds;
            const int64_t lda0 = (n0 + 63) / 64 * 64;
            DevBuf bXc, bA, bDinv, bBad;
            RBF_TRY(bXc.get(pool, sizeof(double) * DIM * (size_t)n0, s));
            RBF_TRY(bA.get(pool, sizeof(double) * (size_t)lda0 * (size_t)lda0, s));
            RBF_TRY(bDinv.get(pool, sizeof(double) * 64 * (size_t)lda0, s));
            RBF_TRY(bBad.get(pool, sizeof(int32_t), s));
            RBF_HIP(hipMemsetAsync(bBad.ptr, 0, sizeof(int32_t), s));
            // Device timers (rbf_ctx_set_timing): "seed_factor", "seed_basis", and "seed_start" from
            // the gather to the level's first error (the pivot check's round trip included).
            hipEvent_t t_start = nullptr, t_factor = nullptr;
            ctx->timers.begin(&t_start, s);
            const unsigned gs = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n0 + 255) / 256, 1024));
            hipLaunchKernelGGL(g_gather_seeds<DIM>, dim3(gs), dim3(256), 0, s, xs, n_s, a.seeds, n0, bXc.as<double>());
            ctx->timers.begin(&t_factor, s);
            RBF_TRY(seed_factor(DIM, Rl, prm.basis, n0, bXc.as<const double>(), bA.as<double>(), lda0,
                                bDinv.as<double>(), bBad.as<int32_t>(), s));
            ctx->timers.end("seed_factor", t_factor, s);
            int32_t not_spd = 0;
            RBF_HIP(hipMemcpyAsync(&not_spd, bBad.ptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            RBF_HIP(hipStreamSynchronize(s));
            if (!not_spd) {
                hipEvent_t t_basis = nullptr;
                ctx->timers.begin(&t_basis, s);
                RBF_TRY(seed_basis(DIM, xs, n_s, bXc.as<const double>(), n0, Rl, prm.basis, bA.as<const double>(),
                                   lda0, bDinv.as<const double>(), a.V, ldt, a.Lpack, s));
                ctx->timers.end("seed_basis", t_basis, s);
                RBF_HIP(hipMemcpyAsync(a.ctrl, a.seeds, sizeof(int64_t) * n0, hipMemcpyDeviceToDevice, s));
                n_start = n0;
                seed_timer = t_start;
            } else {
                ctx->timers.end("seed_start_not_spd", t_start, s);
            }
        }
        // From a basis of n_start columns: y = L^-1 r_C by blocked forward substitution, then
        // E = r - V y and the per-tile maxima; the level continues from there.
        if (n_start > 0) {
            const int64_t n0 = n_start;
            const unsigned gs = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n0 + 255) / 256, 1024));
            hipLaunchKernelGGL(g_seed_rhs<DIM>, dim3(gs), dim3(256), 0, s, R, n_s, a.ctrl, n0, R2, cols, a.sel);
            for (int64_t b0 = 0; b0 < n0; b0 += 64) {
                const int64_t b1 = std::min<int64_t>(n0, b0 + 64);
                const unsigned gb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n0 - b1 + 255) / 256, 1024));
                hipLaunchKernelGGL(g_fwdsolve<DIM>, dim3(gb), dim3(256), 0, s, a.Lpack, R2, cols, a.coef,
                                   cols, n0, b0, b1);
            }
            hipLaunchKernelGGL(g_apply<DIM>, dim3((unsigned)g), dim3(NT), 0, s, a, (const double *)R, n0);
            hipLaunchKernelGGL(g_set_count, dim3(1), dim3(64), 0, s, st, n0);
            RBF_HIP(hipGetLastError());
            if (seed_timer) ctx->timers.end("seed_start", seed_timer, s);
            a.n_seeds = 0;
            a.max_iter = a.cap_level - n0 + 2;
        }
        bool done = false;
        if (coop_max > 0) {
            int64_t gmax = coop_max;
            if (const char *e = getenv("RBF_GREEDY_WGS")) gmax = std::max<int64_t>(1, std::min<int64_t>(gmax, atoi(e)));
            const unsigned G = (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, gmax));
            // Persistent kernels of concurrent requests must fit on the device together, or their
            // spinning workgroups could wait for each other's unscheduled ones.
            CoopTicket gate(ctx, G, coop_max, mode == 0 && (int64_t)G == g && g <= coop_res);
            hipError_t e;
            if (mode == 0) {
                RBF_HIP(hipMemsetAsync(bBar.ptr, 0, sizeof(GridBar), s));
                GridBar *barp = bBar.as<GridBar>();
                void *args[] = {&a, &barp};
                const void *kern = gate.alone ? (const void *)g_level_lean<DIM, true> : (const void *)g_level_lean<DIM, false>;
                e = hipLaunchCooperativeKernel(kern, dim3(G), dim3(NT), args, 0, s);
            } else {
                void *args[] = {&a};
                e = hipLaunchCooperativeKernel((const void *)g_level<DIM>, dim3(G), dim3(NT), args, 0, s);
            }
            if (e == hipSuccess) {
                RBF_HIP(hipMemcpyAsync(&hs, st, sizeof(GState), hipMemcpyDeviceToHost, s));
                RBF_HIP(hipStreamSynchronize(s));
                if (hs.fault)
                    return fail(RBF_E_DEVICE, "greedy level %d: a workgroup of the persistent kernel timed out at a barrier", l);
                if (hs.stop < 0)
                    return fail(RBF_E_DEVICE, "greedy level %d did not stop within %lld iterations", l,
                                (long long)a.max_iter);
                done = true;
            } else {
                (void)hipGetLastError();
            }
        }
        if (!done) {
            // Two kernels per iteration; the device stops itself and later launches are no-ops.
            for (int64_t k = 0; k < a.n_seeds; ++k) {
                hipLaunchKernelGGL(g_select<DIM>, dim3(1), dim3(NT), 0, s, a, seeds_h[seed_off[l] + k]);
                hipLaunchKernelGGL(g_update<DIM>, dim3((unsigned)g), dim3(NT), 0, s, a);
            }
            int64_t batch = 16, launched = 0;
            for (;;) {
                for (int64_t b = 0; b < batch; ++b) {
                    hipLaunchKernelGGL(g_select<DIM>, dim3(1), dim3(NT), 0, s, a, (int64_t)-1);
                    hipLaunchKernelGGL(g_update<DIM>, dim3((unsigned)g), dim3(NT), 0, s, a);
                }
                launched += batch;
                RBF_HIP(hipGetLastError());
                RBF_HIP(hipMemcpyAsync(&hs, st, sizeof(GState), hipMemcpyDeviceToHost, s));
                RBF_HIP(hipStreamSynchronize(s));
                if (hs.stop >= 0) break;
                if (launched > a.cap_level + 1024)
                    return fail(RBF_E_DEVICE, "greedy level %d did not stop after %lld selections", l,
                                (long long)launched);
                batch = std::min<int64_t>(batch * 2, 256);
            }
        }
        const int64_t n = hs.n;
        out->level_stop[l] = hs.stop;
        out->level_in_max[l] = std::sqrt(hs.rmax2);   // max ||dS_l|| (set at level start)
        // Weights: L^T alpha = y, blocked from the bottom.
        double *alpha = out->alpha + total;
        if (n > 0) {
            // One launch: the chained block back substitution, which also gathers the controls.
            const int64_t nblk = (n + TC_NB - 1) / TC_NB;
            hipLaunchKernelGGL(g_backsolve_chain<DIM>, dim3((unsigned)nblk), dim3(TC_NB), 0, s, a.Lpack, n,
                               (const double *)a.coef, cols, alpha, out->capacity, xs, n_s,
                               (const int64_t *)a.ctrl, out->xc + total,
                               bChain.as<int32_t>() + (size_t)l * (size_t)chain_stride, st, a.spin_limit);
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
            pb.basis = prm.basis;
            RBF_TRY(run_kernel_sum(ctx, pb, s));
            if (prm.precision == RBF_MIXED) {
                // The level's interpolant with FP32 pair arithmetic, against the FP64 one: the
                // measured error that decides whether its volume sums may run in FP32.
                const int64_t nb = (n_s + 255) / 256;
                DevBuf bT, bPart;
                RBF_TRY(bT.get(pool, sizeof(double) * DIM * n_s, s));
                RBF_TRY(bPart.get(pool, sizeof(double) * nb, s));
                SumProblem pf = pb;
                pf.lv[0].fp32 = 1;
                pf.base = nullptr;
                pf.sign = -1.0;
                pf.out = bT.as<double>();
                RBF_TRY(run_kernel_sum(ctx, pf, s));
                hipLaunchKernelGGL(g_maxdiff<DIM>, dim3((unsigned)nb), dim3(256), 0, s, (const double *)R,
                                   (const double *)R2, bT.as<const double>(), n_s, bPart.as<double>());
                RBF_HIP(hipGetLastError());
                std::vector<double> ph(nb);
                RBF_HIP(hipMemcpyAsync(ph.data(), bPart.ptr, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
                RBF_HIP(hipStreamSynchronize(s));
                settle_all(bT, bPart);
                out->level_fp32_err[l] = std::sqrt(*std::max_element(ph.begin(), ph.end()));
            }
            std::swap(R, R2);
        }
        if (store) {
            if ((int)store->size() < prm.n_levels) store->resize(prm.n_levels);
            LevelCache &lc = (*store)[l];
            lc.V.release_after(s);
            lc.L.release_after(s);
            lc.n = 0;
            if (n > 0 && lc.V.get(pool, sizeof(double) * n * g * UPB) == RBF_OK &&
                lc.L.get(pool, sizeof(double) * (n * (n + 1) / 2)) == RBF_OK) {
                RBF_HIP(hipMemcpy2DAsync(lc.V.ptr, sizeof(double) * n * UPB, a.V, sizeof(double) * ldt * UPB,
                                         sizeof(double) * n * UPB, g, hipMemcpyDeviceToDevice, s));
                RBF_HIP(hipMemcpyAsync(lc.L.ptr, a.Lpack, sizeof(double) * (n * (n + 1) / 2),
                                       hipMemcpyDeviceToDevice, s));
                lc.ctrl.resize(n);
                RBF_HIP(hipMemcpyAsync(lc.ctrl.data(), a.ctrl, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s));
                lc.n = n;
                lc.radius = Rl;
                lc.basis = prm.basis;
            } else {
                lc.V.release_after(s);   // no room for this level's copy: leave it uncached
                lc.L.release_after(s);
            }
        }
        total += n;
        out->level_off[l + 1] = (int32_t)total;
        used = l + 1;
        // max ||dS_{l+1}|| decides whether another level is needed; the same two launches set up
        // level l + 1 (its residual, cleared selection flags and stop target).
        hipLaunchKernelGGL(g_init<DIM>, dim3((unsigned)g), dim3(64), 0, s, R, a.E, a.sel, n_s, a.part);
        hipLaunchKernelGGL(g_begin, dim3(1), dim3(NT), 0, s, st, a.part, g, prm.eps_abs,
                           prm.level_reduction, (int32_t)(l + 2 >= prm.n_levels));
        RBF_HIP(hipGetLastError());
        RBF_HIP(hipMemcpyAsync(&hs, st, sizeof(GState), hipMemcpyDeviceToHost, s));
        RBF_HIP(hipStreamSynchronize(s));
        if (hs.fault)
            return fail(RBF_E_DEVICE, "greedy level %d: a wait of the back substitution gave up", l);
        out->level_max_err[l] = std::sqrt(hs.rmax2);
        out->level_seconds[l] = now_seconds() - t_level;
        if (std::sqrt(hs.rmax2) < prm.eps_abs || out->level_stop[l] == RBF_STOP_CAP) break;
    }
    for (int l = used; l < prm.n_levels; ++l) out->level_off[l + 1] = (int32_t)total;
    if (store)
        for (int l = used; l < (int)store->size(); ++l) (*store)[l].n = 0;
    out->n_levels_used = used;
    out->stop_reason = out->level_stop[used - 1];
    out->n_iterations = hs.n_iter;
    if (out->e_final)
        RBF_HIP(hipMemcpyAsync(out->e_final, R, sizeof(double) * DIM * n_s, hipMemcpyDeviceToDevice, s));
    if (out->err_hist && hs.n_iter > 0)
        RBF_HIP(hipMemcpyAsync(out->err_hist, bHist.ptr, sizeof(double) * (size_t)std::min<int64_t>(hs.n_iter, cap),
                               hipMemcpyDeviceToDevice, s));
    RBF_HIP(hipStreamSynchronize(s));
    settle_all(bV, bL, bE, bR, bR2, bSel, bPart, bState, bCoef, bHist, bFlag, bSeeds, bChain, bBar, bE2, bPart2);
    bool cap_hit = false, brk = false;
    for (int l = 0; l < used; ++l) {
        cap_hit |= out->level_stop[l] == RBF_STOP_CAP;
        brk |= out->level_stop[l] == RBF_STOP_BREAKDOWN;
    }
    return brk ? RBF_W_BREAKDOWN : (cap_hit ? RBF_W_CAP : RBF_OK);
}

}  // namespace

rbf_status run_greedy(rbf_ctx ctx, const rbf_greedy_params &p, int64_t n_s, const double *xs,
                      const double *ds, rbf_ctrl_set *out, hipStream_t s, const std::vector<LevelCache> *warm,
                      std::vector<LevelCache> *store)
{
    return p.dim == 2 ? greedy_impl<2>(ctx, p, n_s, xs, ds, out, s, warm, store)
                      : greedy_impl<3>(ctx, p, n_s, xs, ds, out, s, warm, store);
}

uint64_t cache_bytes(const std::vector<LevelCache> &levels, int64_t n_s)
{
    const uint64_t rows = (uint64_t)((n_s + UPB - 1) / UPB) * UPB;   // V keeps whole tiles
    uint64_t b = 0;
    for (const LevelCache &lc : levels)
        if (lc.n > 0) b += sizeof(double) * ((uint64_t)lc.n * rows + (uint64_t)(lc.n * (lc.n + 1) / 2));
    return b;
}

}  // namespace rbf

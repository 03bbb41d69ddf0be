/*
 * rbfdef.h -- C ABI of an MI355X (gfx950) library for multi-level greedy radial-basis-function
 * mesh deformation with wall-distance volume reduction.
 *
 * Method: Morelli, Bellosta, Guardone, "Efficient Radial Basis Function Mesh Deformation Methods
 * for Aircraft Icing" (arXiv:2107.13887). Section 2 defines the interpolant (eq. (1)), its weights
 * (eq. (9)) and the Wendland C2 basis (eq. (2), Table 1); Section 3 the greedy selection (eq. (12))
 * and its multi-level form (eq. (19)); Section 4 the wall-distance weight psi and the weighted
 * volume update (eq. (23)).
 *
 * Conventions shared by every call:
 *   - Every call returns rbf_status: 0 success, > 0 success with a warning, < 0 error. No call
 *     throws or aborts. On error the outputs are unspecified. rbf_last_error() gives a readable
 *     detail of the last error raised on the calling thread.
 *   - Arrays are structure-of-arrays: coordinate or component k of point i lives at
 *     a[k * ld + i], with ld = the number of points unless a leading dimension is passed.
 *   - Pointers marked "device" are GPU memory of the context's device, owned by the caller and
 *     valid for the duration of the call (or, for rbf_submit, until the request is DONE).
 *     Pointers marked "host" are ordinary host memory, read during the call only.
 *   - "stream" is a hipStream_t passed as void* (NULL = the default stream). Calls marked
 *     "blocking" return after their device work has finished; the others only enqueue it.
 *   - All device memory the library needs besides the caller's buffers comes from the context
 *     and counts against its HBM budget; RBF_E_NOMEM is returned when it would be exceeded. The
 *     one exception is the fixed scratch array of rbf_volume_update_noalloc.
 *   - Calls on one context are not thread-safe except rbf_submit, rbf_poll and rbf_wait.
 */
#ifndef RBFDEF_H
#define RBFDEF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rbf_status;
#define RBF_OK 0
#define RBF_W_CAP 1          /* selection stopped at max_ctrl_total */
#define RBF_W_BREAKDOWN 2    /* a level stopped because the next Cholesky pivot was not positive */
#define RBF_E_INVALID (-1)   /* bad argument: dimension, size, radius, tolerance, seed, NaN */
#define RBF_E_NOMEM (-2)     /* the context's HBM budget (or the device) cannot hold the work */
#define RBF_E_NOT_SPD (-3)   /* Phi_cc not numerically positive definite (e.g. repeated points) */
#define RBF_E_DEVICE (-4)    /* a HIP runtime call failed */
#define RBF_E_NOT_FOUND (-5) /* unknown ticket or geometry */
#define RBF_E_BUSY (-6)      /* geometry still referenced by queued or running requests */

#define RBF_FP64 0   /* every kernel sum in FP64 */
#define RBF_MIXED 1  /* volume kernel sums in FP32 on locally shifted coordinates with an FP64
                        accumulator; greedy factor, convergence check and residuals stay FP64.
                        The greedy measures each level's FP32 error at the surface
                        (level_fp32_err), and a request runs a level's volume sums in FP32 only
                        when that error is at most RBF_MIXED_TOL max_i ||dS_i|| (FP64 otherwise):
                        that guarded form is held to 1e-5 of the result's scale. A direct call with
                        RBF_MIXED on every level does not meet that on cancelling sums (the FP32
                        pair error grows with sum |phi alpha|, e.g. ice shapes with large weights):
                        there only the FP32 rounding of the summed terms bounds its error */
#define RBF_MIXED_TOL 1e-6

/* Basis functions phi(eta), eta = ||r - r_c|| / R, the Wendland functions of Table 1, each zero
 * for eta >= 1 and 1 at eta = 0. C2 (eq. (2)) is the paper's choice and the zero default. */
#define RBF_WENDLAND_C2 0   /* (1 - eta)^4 (4 eta + 1) */
#define RBF_WENDLAND_C0 1   /* (1 - eta)^2 */
#define RBF_WENDLAND_C4 2   /* (1 - eta)^6 (35/3 eta^2 + 6 eta + 1) */
#define RBF_WENDLAND_C6 3   /* (1 - eta)^8 (32 eta^3 + 25 eta^2 + 8 eta + 1) */

#define RBF_STOP_SKIPPED (-1)     /* level not run: an earlier level already met eps_abs */
#define RBF_STOP_EPS 0            /* max ||E|| fell below the level's target */
#define RBF_STOP_CAP 1            /* max_ctrl_total reached */
#define RBF_STOP_ALL_SELECTED 2   /* every surface point is a control point of the level */
#define RBF_STOP_BREAKDOWN 3      /* next pivot d^2 = phi(0) - l.l not positive */

#define RBF_MAX_LEVELS 8

typedef struct rbf_ctx_s *rbf_ctx;
typedef struct rbf_geom_s *rbf_geom;
typedef uint64_t rbf_ticket;

/* ---------------------------------------------------------------------------------------------
 * Context: one GPU, one HBM budget, the pool every internal buffer comes from.
 * device: HIP device ordinal. hbm_budget_bytes: ceiling on library-owned device memory
 * (0 = 90% of the device's free memory). The context owns its pool and a scheduler thread for
 * rbf_submit; rbf_ctx_destroy waits for running requests, then frees everything.
 * ------------------------------------------------------------------------------------------- */
rbf_status rbf_ctx_create(int32_t device, uint64_t hbm_budget_bytes, rbf_ctx *out);
rbf_status rbf_ctx_destroy(rbf_ctx ctx);
const char *rbf_status_str(rbf_status s);
const char *rbf_last_error(void);
/* Library-owned device bytes currently held by the context (pool high-water included). */
uint64_t rbf_ctx_bytes_in_use(rbf_ctx ctx);

/* Kernel timing for measurement. flags bit 0: the main kernel-sum launch of every call is
 * bracketed by a pair of hipEvents on its stream (adds two event records per launch). Kernel
 * names: "volume_ksum_fp64", "volume_ksum_mixed", "surface_ksum_fp64", "surface_ksum_mixed".
 * rbf_ctx_kernel_time waits for the recorded events and returns the summed device time (ms)
 * and the number of launches since timing was last enabled; set_timing clears the totals.
 * flags bit 1: every workgroup of those launches also adds the pairs it evaluated to a device
 * counter (one atomic per workgroup, so time with bit 0 alone). */
rbf_status rbf_ctx_set_timing(rbf_ctx ctx, int32_t enabled);
rbf_status rbf_ctx_kernel_time(rbf_ctx ctx, const char *kernel, double *total_ms, int64_t *launches);
/* (point, control) pairs the named kernel sums actually evaluated since timing was last enabled:
 * pairs whose control was dropped because its support misses the point's workgroup (phi = 0
 * there, eq. (2)) are not counted. Waits for the device. */
rbf_status rbf_ctx_kernel_pairs(rbf_ctx ctx, const char *kernel, int64_t *pairs);

/* ---------------------------------------------------------------------------------------------
 * Greedy parameters (Section 3). The paper's defaults: one support radius R for all levels,
 * per-level reduction 0.1 of the normalized error, first control point = the first surface
 * point. The target of a non-final level l is max(eps_abs, level_reduction * max_i ||dS_l,i||);
 * the final level runs to eps_abs. Norms are per-point Euclidean norms of the dim components.
 * ------------------------------------------------------------------------------------------- */
typedef struct {
    int32_t dim;                    /* 2 or 3 */
    int32_t n_levels;               /* 1 .. RBF_MAX_LEVELS */
    double radius[RBF_MAX_LEVELS];  /* support radius R_l > 0 of level l, eq. (2) */
    double eps_abs;                 /* stop once max_i ||E_i|| < eps_abs (same units as dS) */
    double level_reduction;         /* rho in (0, 1] */
    int64_t max_ctrl_total;         /* cap on sum_l N_c,l, >= 1 */
    const int64_t *seed_idx;        /* host: seed point indices of all levels, CSR by seed_off */
    const int32_t *seed_off;        /* host [n_levels + 1]; NULL = paper default {0} at level 0 */
    int32_t precision;              /* RBF_FP64 or RBF_MIXED */
    int32_t basis;                  /* RBF_WENDLAND_*; requests use it for the volume update too */
} rbf_greedy_params;

/* Result of a greedy selection. The caller sets the four device pointers and `capacity`
 * (>= max_ctrl_total); the library fills the rest. Levels are concatenated: level l owns
 * positions level_off[l] .. level_off[l+1]-1 of ctrl_idx, xc and alpha. */
typedef struct {
    int64_t capacity;                      /* in: leading dimension of xc and alpha */
    int64_t *ctrl_idx;                     /* device [capacity]: surface indices, selection order */
    double *xc;                            /* device [dim][capacity]: their coordinates */
    double *alpha;                         /* device [dim][capacity]: weights, eq. (9) per level */
    double *e_final;                       /* device [dim][n_s] or NULL: residual after the last level */
    int32_t n_levels_used;                 /* out */
    int32_t stop_reason;                   /* out: stop reason of the last level run */
    int32_t level_off[RBF_MAX_LEVELS + 1]; /* out */
    int32_t level_stop[RBF_MAX_LEVELS];    /* out: RBF_STOP_* per level */
    double level_max_err[RBF_MAX_LEVELS];  /* out: max_i ||E_i|| (FP64) at each level close */
    double level_in_max[RBF_MAX_LEVELS];   /* out: max_i ||dS_l,i|| of each level's input, the
                                              (dS_l)^max of the support distance D_l = k (dS_l)^max
                                              (section 4); 0 for levels not run */
    double level_seconds[RBF_MAX_LEVELS];  /* out: host wall time of each level (timing only) */
    double level_fp32_err[RBF_MAX_LEVELS]; /* out, with RBF_MIXED: max_i ||s_l32(x_i) - s_l(x_i)||
                                              over the surface, the error of level l's interpolant
                                              with FP32 pair arithmetic against FP64; 0 otherwise */
    int64_t n_iterations;                  /* out: argmax selections made (seeds excluded) */
    double *err_hist;                      /* device [capacity] or NULL: max_i ||E_i|| over the
                                              candidates before each argmax selection, in order
                                              over the levels (the greedy error curve of
                                              section 3); n_iterations entries are written */
} rbf_ctrl_set;

/* Multi-level greedy surface point selection, Section 3. Per level l: start from the residual
 * dS_l (dS_0 = ds), append the seeds, then repeatedly take the weights of Phi_cc alpha = dS_l,c
 * (eq. (9) on the control set), the error E = dS_l - Phi_sc alpha (eq. (12)) and append the
 * unselected point of largest ||E_i|| (lowest index on exact ties) until max ||E|| is below the
 * level target; then dS_{l+1} = E. The GPU keeps the Newton basis of the control set at every
 * surface point (the Cholesky factor of Phi_cc bordered by one row per added point), so each
 * iteration costs one rank-one update and one argmax, with no triangular solve. A level given
 * 32 seeds or more (with no resident basis of them, as in a warm start after the basis was
 * dropped) forms that basis at once: the blocked FP64 Cholesky of the seeds' Phi_cc (eq. (9)) and
 * blocked triangular solves for the basis at every surface point, on the matrix cores; seeds at
 * coincident coordinates are appended one by one instead and stop the level at the breakdown.
 * xs, ds: device [dim][n_s] FP64. Blocking. Returns RBF_W_CAP / RBF_W_BREAKDOWN as warnings. */
rbf_status rbf_greedy_select(rbf_ctx ctx, const rbf_greedy_params *params, int64_t n_s,
                             const double *xs, const double *ds, rbf_ctrl_set *out, void *stream);

/* Weights of the interpolant through n_c given points, eq. (9): Phi_cc alpha = dsc with
 * Phi_cc[i][j] = phi(||x_i - x_j|| / radius). FP64 blocked Cholesky (trailing updates on FP64
 * matrix cores) and triangular solves. xc, dsc, alpha: device [dim][n_c], n_c in 1..65536.
 * Blocking. RBF_E_NOT_SPD when a pivot is not positive (repeated or numerically coincident
 * points). Each substitution is one launch whose workgroups wait for earlier blocks with a
 * bounded poll; a wait that gives up (never in a healthy run) returns RBF_E_DEVICE. */
rbf_status rbf_solve_weights(rbf_ctx ctx, int32_t dim, double radius, int64_t n_c,
                             const double *xc, const double *dsc, double *alpha, int32_t basis,
                             void *stream);

/* Volume update with wall-distance reduction, eqs. (19) and (23):
 *   dv_v = sum_l psi(dwall_v / D_l) sum_{c in level l} phi(||xv_v - xc_c|| / radius_l) alpha_c
 * with psi(xi) = 1 - xi on [0, 1) and 0 beyond, so points with dwall_v >= max_l D_l get +0.0
 * and are skipped (the volume point reduction of Section 4).
 * radius, D: host [n_levels]; level_off: host [n_levels + 1] offsets into xc/alpha;
 * xc, alpha: device [dim][ld_ctrl]; xv: device [dim][n_v]; dwall: device [n_v];
 * dv: device [dim][n_v] output (fully written). precision: RBF_FP64 or RBF_MIXED for every
 * level, or level_precision (host [n_levels], nullable) per level; basis: RBF_WENDLAND_*.
 * Enqueued on `stream`; returns before the device work finishes. */
rbf_status rbf_volume_update(rbf_ctx ctx, int32_t dim, int32_t n_levels, const double *radius,
                             const double *D, const int32_t *level_off, int64_t ld_ctrl,
                             const double *xc, const double *alpha, int64_t n_v, const double *xv,
                             const double *dwall, double *dv, int32_t precision,
                             const int32_t *level_precision, int32_t basis, void *stream);

/* Allocation-free form of rbf_volume_update, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc. Same
 * arguments, results and precision rules; it calls no hipMalloc or hipFree and no allocating
 * library routine, records no timer events and counts no pairs. Its scratch (the reduced-point
 * list, per-block counts and the partial sums of split control lists) is a fixed array of
 * RBF_NOALLOC_SCRATCH_BYTES in the library's device memory, one per GPU, held until the process
 * ends (its address is looked up once per device by rbf_ctx_create). n_v above
 * RBF_NOALLOC_MAX_POINTS returns RBF_E_INVALID before any device work; when split partial sums
 * would not fit, the control lists are split fewer times. Every call on one GPU uses that GPU's
 * array and leaves its contents behind: calls that overlap on one GPU (other streams or threads)
 * race and must be serialised by the caller. Enqueued on `stream`. */
#define RBF_NOALLOC_SCRATCH_BYTES (64ull << 20)
#define RBF_NOALLOC_MAX_POINTS 16000000
rbf_status rbf_volume_update_noalloc(rbf_ctx ctx, int32_t dim, int32_t n_levels, const double *radius,
                                     const double *D, const int32_t *level_off, int64_t ld_ctrl,
                                     const double *xc, const double *alpha, int64_t n_v,
                                     const double *xv, const double *dwall, double *dv,
                                     int32_t precision, const int32_t *level_precision, int32_t basis,
                                     void *stream);

/* Interpolant evaluation, eq. (1) with the support of eq. (2), at n_p points:
 *   out_k(p) = base_k(p) - sign * sum_c phi(||x_p - xc_c|| / radius) alpha_k,c
 * sign = -1 with base = NULL gives the plain interpolant; sign = +1 with base = dS gives the
 * greedy error of eq. (12). xc, alpha: device [dim][ld_ctrl]; xp, base, out: device [dim][n_p].
 * Enqueued on `stream`. */
rbf_status rbf_evaluate(rbf_ctx ctx, int32_t dim, double radius, int64_t n_c, int64_t ld_ctrl,
                        const double *xc, const double *alpha, int64_t n_p, const double *xp,
                        const double *base, double sign, double *out, int32_t precision,
                        int32_t basis, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Serving: resident geometries and asynchronous deformation requests with continuous batching.
 * A geometry (surface + volume + wall distance) is copied once into the pool and kept, the
 * volume stored in spatially compact blocks of 512 points (Z order) sorted by their smallest wall
 * distance, each block sorted by wall distance too, so each request's reduced volume lies in a
 * prefix of whole blocks; the bounding box of every 64 stored points is kept so that they can
 * skip the controls whose support misses them. The device copy takes 8 (dim + 1) + 4 + dim / 4
 * bytes per volume point (rounded up to whole blocks) plus 8 dim per surface point. Requests that arrive
 * while others run are admitted as soon as a slot and enough of the HBM budget are free; their
 * kernels overlap on separate streams. A request with warm_start seeds each level with the
 * control set the geometry's previous request selected (successive icing steps).
 * ------------------------------------------------------------------------------------------- */

/* xs: device [dim][n_s]; xv: device [dim][n_v]; dwall: device [n_v] or NULL (then the distance
 * to the nearest surface point is computed on the device). Blocking. */
rbf_status rbf_geom_create(rbf_ctx ctx, int32_t dim, int64_t n_s, const double *xs, int64_t n_v,
                           const double *xv, const double *dwall, rbf_geom *out);
/* RBF_E_BUSY while requests on the geometry are queued or running. */
rbf_status rbf_geom_release(rbf_ctx ctx, rbf_geom geom);

typedef struct {
    rbf_geom geom;
    const double *ds;          /* device [dim][n_s], caller-owned until the request is DONE */
    rbf_greedy_params params;  /* copied at submit (seed arrays included) */
    double D[RBF_MAX_LEVELS];  /* wall-distance support per level (used when d_factor == 0) */
    double d_factor;           /* k > 0: D_l = k max_i ||dS_l,i|| per level after the greedy
                                  (section 4, volume reduction factor; the paper uses k = 5) */
    int32_t warm_start;        /* 1: seed each level with this geometry's previous control set */
    double *dv;                /* device [dim][n_v] output in the geometry's original order */
    rbf_ctrl_set *out;         /* NULL, or caller-owned until DONE (device arrays as above) */
} rbf_request;

#define RBF_REQ_QUEUED 0
#define RBF_REQ_RUNNING 1
#define RBF_REQ_DONE 2
#define RBF_REQ_FAILED 3

typedef struct {
    int32_t state;       /* RBF_REQ_* */
    rbf_status result;   /* final status once DONE or FAILED */
    double t_arrive;     /* seconds on the library's monotonic clock */
    double t_admit;
    double t_start;
    double t_done;
} rbf_req_info;

/* Volume update of eqs. (19) and (23) on a resident geometry: the reduced volume {d < max_l D_l}
 * of section 4 lies in the prefix of stored blocks whose smallest wall distance is below max_l
 * D_l (no per-call compaction). Arguments as rbf_volume_update; dv is device [dim][n_v] in the
 * geometry's original point order, fully written (+0.0 where psi = 0). Enqueued on stream.
 * The first call on a geometry for a given set of radii and support distances also builds the
 * order in which the kernel's workgroups take the stored row groups (heaviest first by the
 * controls of that call each group keeps) and waits for the stream once to do so; later calls
 * with the same set reuse it. The order never changes a result. */
rbf_status rbf_geom_volume_update(rbf_ctx ctx, rbf_geom geom, int32_t n_levels, const double *radius,
                                  const double *D, const int32_t *level_off, int64_t ld_ctrl,
                                  const double *xc, const double *alpha, double *dv,
                                  int32_t precision, const int32_t *level_precision, int32_t basis,
                                  void *stream);

/* Non-blocking. RBF_E_NOMEM if the request could never fit the budget. */
rbf_status rbf_submit(rbf_ctx ctx, const rbf_request *req, rbf_ticket *out);
/* Non-blocking status query. A DONE/FAILED ticket stays queryable until rbf_wait returns it. */
rbf_status rbf_poll(rbf_ctx ctx, rbf_ticket ticket, rbf_req_info *out);
/* Blocks until the request is DONE or FAILED, fills *out, then forgets the ticket. */
rbf_status rbf_wait(rbf_ctx ctx, rbf_ticket ticket, rbf_req_info *out);
/* The library's monotonic clock, in seconds (same clock as rbf_req_info). */
double rbf_now(void);

#ifdef __cplusplus
}
#endif

#endif /* RBFDEF_H */

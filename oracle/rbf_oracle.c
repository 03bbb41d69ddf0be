/*
 * rbf_oracle.c -- plain FP64 CPU oracle of multi-level greedy RBF mesh deformation
 * (Morelli, Bellosta, Guardone: "Efficient Radial Basis Function Mesh Deformation Methods for
 * Aircraft Icing", arXiv:2107.13887).
 *
 * TEST INFRASTRUCTURE ONLY. The test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark are the only users of this file. The GPU library shares no code with it and never
 * calls it.
 *
 * Everything is FP64 and written as plain loops that follow the paper's statement of the method:
 *   - Wendland basis functions of Table 1 (C2, eq. (2), by default; C0, C4, C6 selectable);
 *   - interpolation weights from Phi_cc alpha = dS_c, eq. (9) restricted to the control set;
 *   - greedy error E = dS - Phi_sc alpha, eq. (12), and argmax selection (Section 3);
 *   - multi-level residual dS_{l+1} = E (Section 3, the multi-level subspace scheme);
 *   - wall-distance weight psi(xi) = 1 - xi on [0, 1) and the weighted interpolant, eq. (23);
 *   - summed volume displacement over levels, eq. (19).
 * Where the paper is silent the readings are: per-point Euclidean norm of E for the argmax with
 * squared norms compared and the lowest index winning ties; a non-final level ends once
 * max||E|| < max(eps, rho * max||dS_l||); the last level ends at max||E|| < eps; points already
 * selected in a level are not candidates; eta = ||r - r_c|| / R_l everywhere; phi(eta >= 1) = 0
 * and psi(xi >= 1) = 0 exactly; a Cholesky pivot d^2 not above (n + 1) * 2^-52, i.e. zero within
 * the rounding of l.l, stops the level (breakdown).
 *
 * OpenMP parallelises only over independent points. Each sum over control points runs serially
 * in selection order, so results are reproducible bit for bit for a given binary. The library
 * is built with -ffp-contract=off so no multiply-add is fused behind the reader's back.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_INVALID (-1)
#define ORC_E_NOMEM (-2)
#define ORC_E_NOT_SPD (-3)

#define ORC_STOP_EPS 0
#define ORC_STOP_CAP 1
#define ORC_STOP_ALL_SELECTED 2
#define ORC_STOP_BREAKDOWN 3

/* ---------------------------------------------------------------------------------------- */
/* Basis and weight functions                                                               */
/* ---------------------------------------------------------------------------------------- */

/* Wendland C2, eq. (2): phi(eta) = (1 - eta)^4 (4 eta + 1) for 0 <= eta < 1, 0 otherwise. */
double orc_wendland_c2(double eta)
{
#ifdef ORC_MUTANT_PHI_SIGN
    if (eta >= 1.0) return 0.0;
    { double t = 1.0 - eta; return t * t * t * t * (1.0 - 4.0 * eta); }
#elif defined(ORC_MUTANT_PHI_POWER)
    if (eta >= 1.0) return 0.0;
    { double t = 1.0 - eta; return t * t * t * (4.0 * eta + 1.0); }
#else
    if (eta >= 1.0) return 0.0;
    double t = 1.0 - eta;
    return t * t * t * t * (4.0 * eta + 1.0);
#endif
}

/* The Wendland functions of Table 1, selected by `basis`, each zero from eta = 1 on:
 *   C0: (1 - eta)^2
 *   C2: (1 - eta)^4 (4 eta + 1)                       (the paper's choice, eq. (2))
 *   C4: (1 - eta)^6 (35/3 eta^2 + 6 eta + 1)
 *   C6: (1 - eta)^8 (32 eta^3 + 25 eta^2 + 8 eta + 1)
 * Unknown codes give NaN. */
#define ORC_C2 0
#define ORC_C0 1
#define ORC_C4 2
#define ORC_C6 3
double orc_wendland(int basis, double eta)
{
    if (basis == ORC_C2) return orc_wendland_c2(eta);
    if (eta >= 1.0) return 0.0;
    double t = 1.0 - eta;
    if (basis == ORC_C0) return t * t;
#ifdef ORC_MUTANT_C4_COEF
    if (basis == ORC_C4) return t * t * t * t * t * t * (35.0 / 3.0 * eta * eta + 5.0 * eta + 1.0);
#else
    if (basis == ORC_C4) return t * t * t * t * t * t * (35.0 / 3.0 * eta * eta + 6.0 * eta + 1.0);
#endif
#ifdef ORC_MUTANT_C6_POWER
    if (basis == ORC_C6)
        return t * t * t * t * t * t * t * (32.0 * eta * eta * eta + 25.0 * eta * eta + 8.0 * eta + 1.0);
#else
    if (basis == ORC_C6)
        return t * t * t * t * t * t * t * t * (32.0 * eta * eta * eta + 25.0 * eta * eta + 8.0 * eta + 1.0);
#endif
    return NAN;
}

static int basis_ok(int basis)
{
    return basis == ORC_C0 || basis == ORC_C2 || basis == ORC_C4 || basis == ORC_C6;
}

/* Wall-distance function of Section 4: psi(xi) = 1 - xi for 0 <= xi < 1, 0 otherwise. */
double orc_psi(double xi)
{
    if (xi >= 1.0) return 0.0;
    return 1.0 - xi;
}

/* Euclidean distance between point ia of a and point ib of b; both are SoA [dim][n] with the
 * given leading dimensions. */
static double dist(int dim, const double *a, int64_t lda, int64_t ia,
                   const double *b, int64_t ldb, int64_t ib)
{
    double s = 0.0;
    for (int k = 0; k < dim; ++k) {
        double d = a[k * lda + ia] - b[k * ldb + ib];
#ifdef ORC_MUTANT_DIST_DROP_Z
        if (k == 2) continue;
#endif
        s += d * d;
    }
    return sqrt(s);
}

/* ---------------------------------------------------------------------------------------- */
/* Interpolant evaluation, eq. (1) with the support radius of eq. (2):                       */
/*   f_k(p) = sum_c alpha_k,c phi(||p - x_c|| / R),   summed in control order.              */
/* ---------------------------------------------------------------------------------------- */
void orc_eval(int dim, double radius, int64_t n_c, const double *xc, const double *alpha,
              int64_t n_p, const double *xp, double *out, int basis)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_p; ++i) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t c = 0; c < n_c; ++c) {
            double phi = orc_wendland(basis, dist(dim, xp, n_p, i, xc, n_c, c) / radius);
            for (int k = 0; k < dim; ++k) acc[k] += phi * alpha[k * n_c + c];
        }
        for (int k = 0; k < dim; ++k) out[k * n_p + i] = acc[k];
    }
}

/* ---------------------------------------------------------------------------------------- */
/* Dense weight solve, eq. (9) on a given point set: Phi alpha = ds by textbook Cholesky.     */
/* ---------------------------------------------------------------------------------------- */
int orc_solve_weights(int dim, double radius, int64_t n_c, const double *xc, const double *dsc,
                      double *alpha, int basis)
{
    if (dim < 2 || dim > 3 || n_c <= 0 || !(radius > 0.0) || !basis_ok(basis)) return ORC_E_INVALID;
    double *L = (double *)calloc((size_t)n_c * (size_t)n_c, sizeof(double));
    if (!L) return ORC_E_NOMEM;
    for (int64_t i = 0; i < n_c; ++i)
        for (int64_t j = 0; j <= i; ++j)
            L[i * n_c + j] = orc_wendland(basis, dist(dim, xc, n_c, i, xc, n_c, j) / radius);
    /* Cholesky-Banachiewicz: L L^T = Phi. */
    for (int64_t i = 0; i < n_c; ++i) {
        for (int64_t j = 0; j <= i; ++j) {
            double s = L[i * n_c + j];
            for (int64_t k = 0; k < j; ++k) s -= L[i * n_c + k] * L[j * n_c + k];
            if (i == j) {
                if (!(s > (double)(i + 1) * DBL_EPSILON)) { free(L); return ORC_E_NOT_SPD; }
                L[i * n_c + i] = sqrt(s);
            } else {
                L[i * n_c + j] = s / L[j * n_c + j];
            }
        }
    }
    for (int k = 0; k < dim; ++k) {
        double *a = alpha + k * n_c;
        const double *b = dsc + k * n_c;
        for (int64_t i = 0; i < n_c; ++i) {           /* forward: L y = b */
            double s = b[i];
            for (int64_t j = 0; j < i; ++j) s -= L[i * n_c + j] * a[j];
            a[i] = s / L[i * n_c + i];
        }
        for (int64_t i = n_c - 1; i >= 0; --i) {      /* backward: L^T alpha = y */
            double s = a[i];
            for (int64_t j = i + 1; j < n_c; ++j) s -= L[j * n_c + i] * a[j];
            a[i] = s / L[i * n_c + i];
        }
    }
    free(L);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------------------- */
/* Multi-level greedy surface point selection (Section 3)                                    */
/* ---------------------------------------------------------------------------------------- */

/* Packed lower-triangular Cholesky factor of Phi_cc, grown one bordered row at a time. */
typedef struct {
    double *a;      /* row i starts at i (i + 1) / 2 */
    int64_t n;
} packed_chol;

#define ROW(f, i) ((f)->a + ((i) * ((i) + 1)) / 2)

/* Border the factor with the control point p: l = L^-1 phi(X_C, x_p), d^2 = phi(0) - l.l.
 * Returns 0 on success, 1 when the new pivot is not positive (breakdown). */
static int chol_append(packed_chol *f, int dim, const double *xs, int64_t n_s, double radius,
                       const int64_t *ctrl, int64_t p, int basis)
{
    int64_t n = f->n;
    double *row = ROW(f, n);
    for (int64_t j = 0; j < n; ++j)
        row[j] = orc_wendland(basis, dist(dim, xs, n_s, ctrl[j], xs, n_s, p) / radius);
    double ll = 0.0;
    for (int64_t i = 0; i < n; ++i) {                 /* forward substitution */
        double s = row[i];
        const double *ri = ROW(f, i);
        for (int64_t j = 0; j < i; ++j) s -= ri[j] * row[j];
        row[i] = s / ri[i];
        ll += row[i] * row[i];
    }
    double d2 = orc_wendland(basis, 0.0) - ll;
    /* l.l carries about (n + 1) ulps of rounding: a pivot below that is numerically zero. */
    if (!(d2 > (double)(n + 1) * DBL_EPSILON)) return 1;
    row[n] = sqrt(d2);
    f->n = n + 1;
    return 0;
}

/* alpha = Phi_cc^-1 r_C through the factor (forward then backward substitution). */
static void chol_solve(const packed_chol *f, int dim, const double *r, int64_t n_s,
                       const int64_t *ctrl, double *alpha, int64_t lda, double *tmp)
{
    int64_t n = f->n;
    for (int k = 0; k < dim; ++k) {
        double *y = tmp;
        for (int64_t i = 0; i < n; ++i) {
            const double *ri = ROW(f, i);
            double s = r[k * n_s + ctrl[i]];
            for (int64_t j = 0; j < i; ++j) s -= ri[j] * y[j];
            y[i] = s / ri[i];
        }
        double *a = alpha + k * lda;
#ifdef ORC_MUTANT_NO_BACKSOLVE
        for (int64_t i = 0; i < n; ++i) a[i] = y[i];
        continue;
#endif
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = y[i];
            for (int64_t j = i + 1; j < n; ++j) s -= ROW(f, j)[i] * a[j];
            a[i] = s / ROW(f, i)[i];
        }
    }
}

/* E = r - Phi_sC alpha at every surface point, eq. (12), control sums in selection order. */
static void surface_error(int dim, const double *xs, int64_t n_s, const double *r, double radius,
                          const int64_t *ctrl, int64_t n, const double *alpha, int64_t lda,
                          double *E, int basis)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_s; ++i) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t c = 0; c < n; ++c) {
            double phi = orc_wendland(basis, dist(dim, xs, n_s, i, xs, n_s, ctrl[c]) / radius);
            for (int k = 0; k < dim; ++k) acc[k] += phi * alpha[k * lda + c];
        }
        for (int k = 0; k < dim; ++k) {
#ifdef ORC_MUTANT_ERROR_SIGN
            E[k * n_s + i] = r[k * n_s + i] + acc[k];
#else
            E[k * n_s + i] = r[k * n_s + i] - acc[k];
#endif
        }
    }
}

static double norm2_at(int dim, const double *v, int64_t n, int64_t i)
{
    double s = 0.0;
    for (int k = 0; k < dim; ++k) s += v[k * n + i] * v[k * n + i];
    return s;
}

/*
 * Multi-level greedy selection.
 *
 * Inputs: surface points xs [dim][n_s], prescribed displacement ds [dim][n_s]; n_levels support
 * radii; absolute tolerance eps; per-level reduction rho; a cap on the total number of control
 * points; per-level seed lists in CSR form (seed_idx[seed_off[l] .. seed_off[l+1])).
 * Outputs (caller-allocated): ctrl_idx [cap] and alpha [dim][cap] (leading dimension cap),
 * level_off [n_levels + 1], level_max_err [n_levels] (max_i ||E_i|| at each level close),
 * level_stop [n_levels], e_final [dim][n_s] (the residual after the last level; may be NULL),
 * n_levels_used, and history [cap] (max_i ||E_i|| over candidates before each selection made by
 * the argmax; may be NULL).
 */
int orc_greedy(int dim, int64_t n_s, const double *xs, const double *ds,
               int n_levels, const double *radius, double eps, double rho, int64_t cap,
               const int64_t *seed_idx, const int32_t *seed_off,
               int64_t *ctrl_idx, double *alpha, int32_t *level_off, double *level_max_err,
               int32_t *level_stop, int32_t *n_levels_used, double *e_final, double *history,
               int basis)
{
    if (dim < 2 || dim > 3 || n_s <= 0 || n_levels < 1 || n_levels > 8 || cap <= 0 ||
        !(eps >= 0.0) || !(rho > 0.0 && rho <= 1.0) || !basis_ok(basis))
        return ORC_E_INVALID;
    for (int l = 0; l < n_levels; ++l)
        if (!(radius[l] > 0.0)) return ORC_E_INVALID;

    int64_t nmax = cap < n_s ? cap : n_s;           /* most control points one level can hold */
    double *r = (double *)malloc(sizeof(double) * (size_t)dim * (size_t)n_s);
    double *E = (double *)malloc(sizeof(double) * (size_t)dim * (size_t)n_s);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(nmax + 1));
    double *alv = (double *)malloc(sizeof(double) * (size_t)dim * (size_t)(nmax + 1));
    char *sel = (char *)malloc((size_t)n_s);
    packed_chol f;
    f.a = (double *)malloc(sizeof(double) * (size_t)((nmax + 1) * (nmax + 2) / 2));
    f.n = 0;
    if (!r || !E || !tmp || !alv || !sel || !f.a) {
        free(r); free(E); free(tmp); free(alv); free(sel); free(f.a);
        return ORC_E_NOMEM;
    }
    memcpy(r, ds, sizeof(double) * (size_t)dim * (size_t)n_s);

    int64_t total = 0, n_hist = 0;
    int used = 0;
    level_off[0] = 0;
    for (int l = 0; l < n_levels; ++l) {
        int last = (l == n_levels - 1);
        double rmax2 = 0.0;
        for (int64_t i = 0; i < n_s; ++i) {
            double v = norm2_at(dim, r, n_s, i);
            if (v > rmax2) rmax2 = v;
        }
        double target = eps;
        if (!last && rho * sqrt(rmax2) > target) target = rho * sqrt(rmax2);
        double target2 = target * target;

        int64_t *C = ctrl_idx + total;
        int64_t n = 0;
        int stop = -1;
        f.n = 0;
        memset(sel, 0, (size_t)n_s);

        /* Seeds: the first control point(s) of the level, appended before the first error. */
        for (int32_t s = seed_off[l]; s < seed_off[l + 1]; ++s) {
            int64_t p = seed_idx[s];
            if (total + n >= cap) { stop = ORC_STOP_CAP; break; }
            if (chol_append(&f, dim, xs, n_s, radius[l], C, p, basis)) { stop = ORC_STOP_BREAKDOWN; break; }
            C[n++] = p;
            sel[p] = 1;
        }

        for (;;) {
            /* alpha from Phi_cc alpha = r_C (eq. (9) on the control set), then E (eq. (12)). */
            chol_solve(&f, dim, r, n_s, C, alv, nmax + 1, tmp);
            surface_error(dim, xs, n_s, r, radius[l], C, n, alv, nmax + 1, E, basis);
            if (stop >= 0) break;
            /* Largest error signal among the points not yet selected in this level. */
            int64_t p = -1;
            double m2 = -1.0;
            for (int64_t i = 0; i < n_s; ++i) {
                if (sel[i]) continue;
                double v = norm2_at(dim, E, n_s, i);
#ifdef ORC_MUTANT_TIE_HIGH
                if (v >= m2) { m2 = v; p = i; }
#else
                if (v > m2) { m2 = v; p = i; }
#endif
            }
            if (p < 0) { stop = ORC_STOP_ALL_SELECTED; break; }
            if (m2 < target2) { stop = ORC_STOP_EPS; break; }
            if (total + n >= cap) { stop = ORC_STOP_CAP; break; }
            if (chol_append(&f, dim, xs, n_s, radius[l], C, p, basis)) { stop = ORC_STOP_BREAKDOWN; break; }
            if (history) history[n_hist] = sqrt(m2);
            ++n_hist;
            C[n++] = p;
            sel[p] = 1;
        }

        for (int k = 0; k < dim; ++k)
            for (int64_t c = 0; c < n; ++c) alpha[k * cap + total + c] = alv[k * (nmax + 1) + c];
        total += n;
        level_off[l + 1] = (int32_t)total;
        level_stop[l] = stop;
        double emax2 = 0.0;
        for (int64_t i = 0; i < n_s; ++i) {
            double v = norm2_at(dim, E, n_s, i);
            if (v > emax2) emax2 = v;
        }
        level_max_err[l] = sqrt(emax2);
        used = l + 1;
        /* The next level interpolates what this one left: dS_{l+1} = E. */
#ifndef ORC_MUTANT_LEVEL_RESTART
        memcpy(r, E, sizeof(double) * (size_t)dim * (size_t)n_s);
#endif
        if (sqrt(emax2) < eps || stop == ORC_STOP_CAP) break;
    }
    for (int l = used; l < n_levels; ++l) {
        level_off[l + 1] = (int32_t)total;
        level_stop[l] = -1;
        level_max_err[l] = 0.0;
    }
    *n_levels_used = used;
    if (e_final) memcpy(e_final, r, sizeof(double) * (size_t)dim * (size_t)n_s);
    free(r); free(E); free(tmp); free(alv); free(sel); free(f.a);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------------------- */
/* Volume update with wall-distance reduction (Section 4, eqs. (19) and (23))                 */
/*   dV_v = sum_l psi(d_v / D_l) sum_{c in C_l} phi(||x_v - x_c|| / R_l) alpha_c^(l)          */
/* Points with d_v >= D_l receive nothing from level l; beyond every D_l, dV_v = +0.0.        */
/* ---------------------------------------------------------------------------------------- */
void orc_volume(int dim, int n_levels, const double *radius, const double *D,
                const int32_t *level_off, int64_t ld_ctrl, const double *xc, const double *alpha,
                int64_t n_v, const double *xv, const double *dwall, double *dv, int basis)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t v = 0; v < n_v; ++v) {
        double out[3] = {0.0, 0.0, 0.0};
        for (int l = 0; l < n_levels; ++l) {
            double w = orc_psi(dwall[v] / D[l]);
#ifdef ORC_MUTANT_PSI_SKIP
            w = 1.0;
#endif
            if (w == 0.0) continue;
            double acc[3] = {0.0, 0.0, 0.0};
            for (int64_t c = level_off[l]; c < level_off[l + 1]; ++c) {
                double phi = orc_wendland(basis, dist(dim, xv, n_v, v, xc, ld_ctrl, c) / radius[l]);
                for (int k = 0; k < dim; ++k) acc[k] += phi * alpha[k * ld_ctrl + c];
            }
            for (int k = 0; k < dim; ++k) out[k] += w * acc[k];
        }
        for (int k = 0; k < dim; ++k) dv[k * n_v + v] = out[k];
    }
}

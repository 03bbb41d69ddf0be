"""Small helpers shared by the GPU tests, and the tolerances they assert.

FP64 bound. Each displacement component is sum_l psi_l sum_c phi(eta_lc) alpha_c. For any FP64
evaluation of it (GPU or oracle), with u = 2^-53:
  * the products and their recursive sum carry at most gamma_n S, gamma_n = n u / (1 - n u), with
    n the terms one point sums (its in-support controls over all levels, plus the psi products
    and the level sums) and S = sum_l psi_l sum_c phi |alpha_c| (Higham, Accuracy and Stability of
    Numerical Algorithms, eq. (3.5), the inner-product bound);
  * each basis value phi(eta) carries the error of eta. On the GPU the coordinates are scaled by
    1/R before the differences (|d eta| <= u (4 sqrt(dim) rho/R + 5), rho the largest coordinate
    magnitude: two roundings of each scaled coordinate, the difference, the dim-term sum of
    squares, the refined square root; the volume sums take the root from one Goldschmidt step, and
    5 becomes 44.4 there: ROOT_U), then |d phi| <= max|phi'| |d eta| + 5 u (the polynomial:
    max|phi'| = 2 (C0), 2.11 (C2), 2.50 (C4), 2.82 (C6)); the oracle's eta is better. Each value
    multiplies one |alpha_c|, so this enters as eps_phi A, A = sum_l psi_l sum_{eta_lc < 1} |alpha_c|.
  The GPU and the oracle then differ by at most 2 (gamma_n S + eps_phi A). The bound is a worst
  case; the measured differences are printed as err / (u S).
"""
import math

import numpy as np

U64 = 2.0 ** -53
U32 = 2.0 ** -24
MAX_DPHI = {"c0": 2.0, "c2": 2.1094, "c4": 2.4998, "c6": 2.8192}
# Error of eta's last steps in units of u (eta <= 1 in support): the refined square root of the
# surface sums (half an ulp) with the difference and the sum of squares, 5 in all; the volume sums
# (psi applied) stop the root after its Goldschmidt step, relative error 1.5 e^2 with
# |e| <= 2^-24.2 for v_rsq_f64, i.e. 1.5 * 2^4.6 = 36.4 u, plus the step's own roundings.
ROOT_U = {False: 5.0, True: 5.0 + 36.4 + 3.0}


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def normwise(got, ref):
    """max_v ||got_v - ref_v|| / max_v ||ref_v|| over [dim, n] arrays (per-point Euclidean)."""
    num = np.sqrt(((np.asarray(got) - ref) ** 2).sum(axis=0)).max()
    den = np.sqrt((np.asarray(ref) ** 2).sum(axis=0)).max()
    return float(num / den) if den > 0 else float(num)


class SumMagnitude(float):
    """S = max over points and components of sum_l psi_l sum_c phi |alpha_c| (the float value),
    carrying what the forward-error bound also needs: A = max over points and components of
    sum_l psi_l sum_{c in support} |alpha_c|, n = the most terms one point sums, rho_r = the largest
    coordinate magnitude over the smallest radius, dim and the basis."""

    def __new__(cls, S, A=0.0, n=1, rho_r=0.0, dim=3, basis="c2", volume=False):
        obj = super().__new__(cls, S)
        obj.A, obj.n, obj.rho_r, obj.dim, obj.basis = float(A), int(n), float(rho_r), dim, basis
        obj.volume = bool(volume)
        return obj


def sum_magnitude(orc, radius, level_off, xc, alpha, pts, dwall=None, D=None, basis="c2"):
    """S, A and n of the sums sum_l psi_l sum_c phi(||p - x_c|| / R_l) alpha_c at the points pts
    (psi = 1 without wall distances)."""
    a = np.abs(np.asarray(alpha, dtype=np.float64))
    xc = np.asarray(xc, dtype=np.float64)
    pts = np.asarray(pts, dtype=np.float64)
    dim, n_p = pts.shape
    S = np.zeros((dim, n_p))
    A = np.zeros((dim, n_p))
    n = np.zeros(n_p)
    live = np.zeros(n_p, dtype=bool)    # points some level weights (psi > 0)
    used = []
    for l in range(len(radius)):
        lo, hi = int(level_off[l]), int(level_off[l + 1])
        if hi <= lo:
            continue
        used.append(radius[l])
        psi = np.ones(n_p) if dwall is None else np.where(dwall < D[l], 1.0 - dwall / D[l], 0.0)
        live |= psi > 0
        S += psi * orc.evaluate(radius[l], xc[:, lo:hi], a[:, lo:hi], pts, basis=basis)
        r2 = radius[l] ** 2
        for c0 in range(0, n_p, 2048):
            c1 = min(n_p, c0 + 2048)
            d2 = ((pts[:, c0:c1, None] - xc[:, None, lo:hi]) ** 2).sum(0)
            m = (d2 < r2).astype(np.float64)
            A[:, c0:c1] += psi[c0:c1] * (a[:, lo:hi] @ m.T)
            n[c0:c1] += np.where(psi[c0:c1] > 0, m.sum(1), 0.0)
    if not used or not live.any():
        return SumMagnitude(0.0)
    rho = max(np.abs(pts[:, live]).max(), np.abs(xc).max() if xc.size else 0.0)
    return SumMagnitude(S.max(), A.max(), n.max() + 2 * len(radius), rho / min(used), dim, basis,
                        volume=dwall is not None)


def gamma(n, u=U64):
    return n * u / (1.0 - n * u)


def fp64_bound(scale, S):
    """Largest admissible difference between two FP64 evaluations of the sums (module docstring),
    plus 1e-10 of the result's scale."""
    if not isinstance(S, SumMagnitude):
        S = SumMagnitude(S)
    eps_phi = U64 * (MAX_DPHI[S.basis] * (4.0 * math.sqrt(S.dim) * S.rho_r + ROOT_U[S.volume]) + 5.0)
    return 1e-10 * scale + 2.0 * (gamma(S.n) * float(S) + eps_phi * S.A)


def ratio(err, S):
    """err / (u S): the measured difference in units of the rounding of the summed terms."""
    return err / (U64 * float(S)) if float(S) > 0 else 0.0


def mixed_bound(scale, S):
    """The same bound for the all-FP32 pair form (FP32 coordinates shifted to a local origin, FP32
    square root, basis value widened and accumulated in FP64): the pair part with u32 = 2^-24 and
    the local extent (at most 2 rho) for the scaled coordinates. This is what a direct RBF_MIXED
    call is held to; it does not meet the 1e-5 relative FP32 target on cancelling sums."""
    if not isinstance(S, SumMagnitude):
        S = SumMagnitude(S)
    eps_phi = U32 * (MAX_DPHI[S.basis] * (8.0 * math.sqrt(S.dim) * S.rho_r + 5.0) + 5.0)
    return 1e-5 * scale + 2.0 * (gamma(S.n) * float(S) + eps_phi * S.A)


def check_fp64(err, scale, S, label=""):
    """Print the measured difference (absolute, normwise and in units of u S) and assert the FP64
    bound."""
    bound = fp64_bound(scale, S)
    print(f"{label}difference {err:.3e} = {err / scale if scale else 0.0:.3e} normwise = "
          f"{ratio(err, S):.2f} u S (bound {bound:.3e}; S {float(S):.3e}, A {getattr(S, 'A', 0.0):.3e}, "
          f"n {getattr(S, 'n', 0)})")
    assert err <= bound

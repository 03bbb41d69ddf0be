"""Small helpers shared by the GPU tests."""
def to_dev(a):
    import numpy as np
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def normwise(got, ref):
    """max_v ||got_v - ref_v|| / max_v ||ref_v|| over [dim, n] arrays (per-point Euclidean)."""
    import numpy as np

    num = np.sqrt(((np.asarray(got) - ref) ** 2).sum(axis=0)).max()
    den = np.sqrt((np.asarray(ref) ** 2).sum(axis=0)).max()
    return float(num / den) if den > 0 else float(num)


U64 = 2.0 ** -53


def sum_magnitude(orc, radius, level_off, xc, alpha, pts, dwall=None, D=None):
    """max over points and components of sum_l psi_l sum_c phi |alpha_c|: the magnitude of the
    terms whose rounding any FP64 evaluation of the sums carries (phi, psi >= 0)."""
    import numpy as np

    a = np.abs(np.asarray(alpha))
    if dwall is None:
        total = np.zeros((np.asarray(pts).shape[0], np.asarray(pts).shape[1]))
        for l in range(len(radius)):
            lo, hi = int(level_off[l]), int(level_off[l + 1])
            if hi > lo:
                total += orc.evaluate(radius[l], xc[:, lo:hi], a[:, lo:hi], pts)
        return float(total.max()) if total.size else 0.0
    v = orc.volume(radius, D, level_off, xc, a, pts, dwall)
    return float(v.max()) if v.size else 0.0


def fp64_bound(scale, S, c=64.0):
    """FP64 tolerance: 1e-10 relative to the result's scale plus c units of rounding of the
    summed terms (two independent correct FP64 evaluations differ by about u * S)."""
    return 1e-10 * scale + c * U64 * S


U32 = 2.0 ** -24


def mixed_bound(scale, S, c=16.0):
    """Tolerance of the FP32-pair / FP64-accumulate sums: 1e-5 of the scale plus c units of
    FP32 rounding of the summed terms."""
    return 1e-5 * scale + c * U32 * S

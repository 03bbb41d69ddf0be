"""Seeded synthetic inputs for multi-level greedy RBF mesh deformation.

This module is shared by the FP64 CPU oracle's tests and by the GPU library's tests and benchmark.
It builds geometry (NACA0012 contours, an untapered swept NACA0012 wing), structured volume meshes
(2D O-mesh, 3D O-H shell), prescribed surface displacements (ice horns, a rime layer, bending and
twist) and the wall distance of every volume point. It contains none of the deformation method's
arithmetic: no basis function, no solve, no greedy step, no wall-distance weighting.

The paper's own meshes and ice shapes are not available, so these generators stand in for the
paper's 2D NACA0012 and 3D swept-wing icing cases (Section 5, "Results"). Every array that crosses
into a solver is float64 structure-of-arrays: ``xs[k, i]`` is coordinate ``k`` of point ``i``.

Random numbers come from ``numpy.random.default_rng(13887 + cfg)`` (one stream per workload) or
``default_rng(13887000 + request_id)`` for serving requests, so both sides read identical inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 13887
CHORD = 1.0


# --------------------------------------------------------------------------------------------
# NACA0012 contour
# --------------------------------------------------------------------------------------------
def naca0012_contour(n: int):
    """Closed-trailing-edge NACA0012 contour with ``n`` points (``n`` even, chord 1).

    Point 0 is the trailing edge (1, 0). Points 1..n/2-1 run along the upper surface to the
    leading edge at index n/2, and points n/2+1..n-1 mirror them on the lower surface, so the
    contour is traversed counter-clockwise. Abscissae follow x = 1 - cos(beta) with
    beta = (pi/2)(1 - i/(n/2)), which clusters points toward the leading edge.
    """
    if n < 8 or n % 2:
        raise ValueError("contour needs an even number of points >= 8")
    half = n // 2
    i_up = np.arange(half + 1, dtype=np.float64)
    beta = 0.5 * np.pi * (1.0 - i_up / half)
    xu = 1.0 - np.cos(beta)
    yt = 0.6 * (0.2969 * np.sqrt(xu) - 0.1260 * xu - 0.3516 * xu**2 + 0.2843 * xu**3 - 0.1036 * xu**4)
    yt[0] = 0.0
    yt[half] = 0.0
    x = np.empty(n)
    y = np.empty(n)
    x[: half + 1] = xu
    y[: half + 1] = yt
    j = np.arange(half + 1, n)
    x[j] = xu[n - j]
    y[j] = -yt[n - j]
    return x, y


def contour_normals(x: np.ndarray, y: np.ndarray):
    """Outward unit normals of a closed counter-clockwise polygon (central-difference tangent
    rotated by -90 degrees)."""
    tx = np.roll(x, -1) - np.roll(x, 1)
    ty = np.roll(y, -1) - np.roll(y, 1)
    norm = np.hypot(tx, ty)
    return ty / norm, -tx / norm


def arc_length_from_te(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Cumulative arc length from the trailing edge, along the upper side first."""
    seg = np.hypot(np.diff(x), np.diff(y))
    return np.concatenate([[0.0], np.cumsum(seg)])


def upper_arc_length_at(x: np.ndarray, s: np.ndarray, x_target: float) -> float:
    """Arc length of the upper-surface point whose abscissa is ``x_target`` (linear interp)."""
    half = x.size // 2
    xu = x[: half + 1][::-1]  # increasing from LE to TE
    su = s[: half + 1][::-1]
    return float(np.interp(x_target, xu, su))


# --------------------------------------------------------------------------------------------
# Structured volume meshes
# --------------------------------------------------------------------------------------------
def geometric_ratio(n_layers: int, first_layer: float, length: float) -> float:
    """Growth ratio q with (q - 1) / (q**n - 1) * length == first_layer (bisection)."""
    target = first_layer / length
    if target * n_layers >= 1.0:
        return 1.0

    def frac(q):
        return (q - 1.0) / (q**n_layers - 1.0)

    lo, hi = 1.0 + 1e-12, 4.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if frac(mid) > target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def layer_fractions(n_layers: int, first_layer: float, length: float) -> np.ndarray:
    """g_j = (q**j - 1)/(q**n - 1), j = 1..n: the fraction of each ray travelled by layer j."""
    q = geometric_ratio(n_layers, first_layer, length)
    j = np.arange(1, n_layers + 1, dtype=np.float64)
    if q == 1.0:
        return j / n_layers
    return (q**j - 1.0) / (q**n_layers - 1.0)


def blended_rays(px, py, nx, ny, fx, fy, g, bend: float = 0.05):
    """Layer points of rays that leave the wall along its outward normal n and turn into the
    direction e = (F - P) / L, L = |F - P|, of the straight line to their far-field point F: at the
    layer fraction g the point is P + r (w n + (1 - w) e) with r = g L and w = 1 / (1 + r / bend).
    The ray's tangent turns monotonically from n at the wall to e, so the cells next to the wall
    are orthogonal to it rather than sheared (a straight ray to the far field runs within a few
    degrees of the surface near the trailing edge), and far out each ray is the straight one
    shifted by bend (n - e). Returns [len(g), n] arrays."""
    dx, dy = fx - px, fy - py
    L = np.hypot(dx, dy)
    ex, ey = dx / L, dy / L
    r = g[:, None] * L[None]
    w = 1.0 / (1.0 + r / bend)
    return (px[None] + r * (w * nx[None] + (1.0 - w) * ex[None]),
            py[None] + r * (w * ny[None] + (1.0 - w) * ey[None]))


def omesh_2d(xs: np.ndarray, ys: np.ndarray, n_layers: int, first_layer: float,
             r_far: float = 20.0, center=(0.5, 0.0)):
    """2D O-mesh annulus: layer ``j`` of ray ``i`` lies at the fraction g_j of a ray from the
    surface point S_i to F_i, the point of the far-field circle at S_i's polar angle about
    ``center``, leaving the wall along its normal (``blended_rays``). The wall layer itself is not
    part of the volume. Returned layer-major: volume index = (j - 1) * n_rays + i."""
    cx, cy = center
    theta = np.arctan2(ys - cy, xs - cx)
    fx = cx + r_far * np.cos(theta)
    fy = cy + r_far * np.sin(theta)
    nx, ny = contour_normals(xs, ys)
    g = layer_fractions(n_layers, first_layer, r_far - 0.5 * CHORD)
    xv, yv = blended_rays(xs, ys, nx, ny, fx, fy, g)
    return xv.reshape(-1), yv.reshape(-1)


def wall_distance(surface: np.ndarray, volume: np.ndarray) -> np.ndarray:
    """Distance from each volume point to the nearest surface point (float64).

    ``surface`` is [dim, n_s] and ``volume`` is [dim, n_v]. The paper does not say how the wall
    distance is computed; the nearest discrete surface point of the undeformed geometry is used.
    """
    from scipy.spatial import cKDTree

    tree = cKDTree(np.ascontiguousarray(surface.T))
    d, _ = tree.query(np.ascontiguousarray(volume.T), k=1, workers=-1)
    return np.ascontiguousarray(d, dtype=np.float64)


# --------------------------------------------------------------------------------------------
# Swept wing
# --------------------------------------------------------------------------------------------
def wing_surface(n_chord: int, n_span: int, semi_span: float = 3.0, sweep_deg: float = 25.0):
    """Untapered swept NACA0012 wing without a tip cap. Sections lie in x-z planes at
    y_k = b k / (n_span - 1) with leading edge x_LE(y) = y tan(sweep). Station-major order:
    surface index = k * n_chord + i. Returns (xyz [3, n], section x, section z, y stations)."""
    xc, zc = naca0012_contour(n_chord)
    yk = semi_span * np.arange(n_span) / (n_span - 1)
    xle = yk * math.tan(math.radians(sweep_deg))
    X = (xle[:, None] + xc[None, :]).reshape(-1)
    Y = np.repeat(yk, n_chord)
    Z = np.tile(zc, n_span)
    return np.stack([X, Y, Z]), xc, zc, yk


def wing_normals(xyz: np.ndarray, n_chord: int, n_span: int) -> np.ndarray:
    """Outward unit normals from the cross product of the chordwise and spanwise grid tangents."""
    P = xyz.reshape(3, n_span, n_chord)
    tc = np.roll(P, -1, axis=2) - np.roll(P, 1, axis=2)
    ts = np.gradient(P, axis=1)
    n = np.cross(ts, tc, axis=0)
    n /= np.linalg.norm(n, axis=0, keepdims=True)
    # orient outward: agree with the in-section outward normal
    nx2, nz2 = contour_normals(P[0, 0] - P[0, 0].min(), P[2, 0])
    sign = np.sign(n[0] * nx2[None, :] + n[2] * nz2[None, :])
    sign[sign == 0] = 1.0
    return (n * sign[None]).reshape(3, -1)


def c_grid_section(xc: np.ndarray, zc: np.ndarray, n_wake: int, n_layers: int,
                   first_layer: float = 1e-3, r_far: float = 10.0):
    """C-grid of one wing section in its own plane (abscissa from the leading edge, chord 1).

    The C-line runs counter-clockwise: the upper side of the wake cut from its far end to the
    trailing edge, the contour (trailing edge, upper surface, leading edge, lower surface), the
    trailing edge again, then the lower side of the cut out to its far end. The cut holds
    ``n_wake`` points on z = 0 from the trailing edge to x = 0.5 + r_far (geometric spacing that
    starts from the contour's trailing-edge spacing); each appears on both sides of the C-line.
    From every C-line node an off-body line of ``n_layers`` points leaves along the C-line normal
    and bends into its far point (``blended_rays``): straight up or down for the cut, and for the
    contour a point of the far boundary: straight above or below the node behind mid-chord, on
    the half circle of radius r_far about mid-chord at the node's polar angle in front of it. The
    trailing edge, the corner of an O-grid, is a kink of a few degrees of the C-line here, so no
    cell there is a thin wedge.

    Returns (cut_x [n_wake], line_x, line_z [n_layers, m]) with m = 2 n_wake + n + 1 C-line
    nodes: layer j >= 1 of node p at line_x[j - 1, p], line_z[j - 1, p]."""
    n = xc.size
    x_te, x_far = xc[0], 0.5 * CHORD + r_far
    h0 = math.hypot(xc[1] - xc[0], zc[1] - zc[0])
    cut = x_te + (x_far - x_te) * layer_fractions(n_wake, h0, x_far - x_te)
    px = np.concatenate([cut[::-1], [x_te], xc[1:], [x_te], cut])
    pz = np.concatenate([np.zeros(n_wake), [zc[0]], zc[1:], [zc[0]], np.zeros(n_wake)])
    m = px.size
    tx = np.empty(m)
    tz = np.empty(m)
    tx[1:-1], tz[1:-1] = px[2:] - px[:-2], pz[2:] - pz[:-2]
    tx[0], tz[0] = px[1] - px[0], pz[1] - pz[0]
    tx[-1], tz[-1] = px[-1] - px[-2], pz[-1] - pz[-2]
    norm = np.hypot(tx, tz)
    nx, nz = tz / norm, -tx / norm
    fx = px.copy()
    fz = np.concatenate([np.full(n_wake, r_far), np.zeros(n + 1), np.full(n_wake, -r_far)])
    # Contour nodes onto the far boundary: the rear half of the section (behind mid-chord)
    # straight up or down onto z = +-r_far, the front half onto the half circle at the node's
    # polar angle about mid-chord, so the order along the C-line is kept.
    body = slice(n_wake, n_wake + n + 1)
    th = np.arctan2(pz[body], px[body] - 0.5 * CHORD)
    rear = px[body] >= 0.5 * CHORD
    up = np.arange(n + 1) <= n // 2
    bx = np.where(rear, px[body], 0.5 * CHORD + r_far * np.cos(th))
    bz = np.where(rear, np.where(up, r_far, -r_far), r_far * np.sin(th))
    fx[body], fz[body] = bx, bz
    g = layer_fractions(n_layers, first_layer, r_far - 0.5 * CHORD)
    lx, lz = blended_rays(px, pz, nx, nz, fx, fz, g)
    return cut, lx, lz


def ch_shell_3d(xc: np.ndarray, zc: np.ndarray, xle: np.ndarray, yk: np.ndarray, n_wake: int,
                n_layers: int, first_layer: float = 1e-3, r_far: float = 10.0):
    """C-H shell around the swept wing: the section C-grid (``c_grid_section``) at every span
    station, shifted to the station's leading edge. Volume order: the cut points of every station
    (station-major), then layer by layer the off-body points of every station and C-line node:
    index n_wake n_span + (j - 1) m n_span + k m + p for layer j >= 1, station k, node p."""
    cut, lx, lz = c_grid_section(xc, zc, n_wake, n_layers, first_layer, r_far)
    n_span, m = yk.size, lx.shape[1]
    X0 = (xle[:, None] + cut[None, :]).reshape(-1)
    Y0 = np.repeat(yk, n_wake)
    Z0 = np.zeros(X0.size)
    X = (xle[None, :, None] + lx[:, None, :]).reshape(-1)
    Y = np.broadcast_to(yk[None, :, None], (n_layers, n_span, m)).reshape(-1)
    Z = np.broadcast_to(lz[:, None, :], (n_layers, n_span, m)).reshape(-1)
    return np.stack([np.concatenate([X0, X]), np.concatenate([Y0, Y]), np.concatenate([Z0, Z])])


def ch_nodes(vol: np.ndarray, surf: np.ndarray, n_chord: int, n_span: int, n_layers: int, n_wake: int):
    """Node coordinates of the C-H shell as a [3, n_layers + 1, n_span, m] grid (layer 0 on the
    C-line: cut points and surface points, the trailing edge at both of its C-line places)."""
    m = 2 * n_wake + n_chord + 1
    S = surf.reshape(3, n_span, n_chord)
    cut = vol[:, : n_wake * n_span].reshape(3, n_span, n_wake)
    G = np.empty((3, n_layers + 1, n_span, m))
    G[:, 0, :, :n_wake] = cut[:, :, ::-1]
    G[:, 0, :, n_wake] = S[:, :, 0]
    G[:, 0, :, n_wake + 1: n_wake + n_chord] = S[:, :, 1:]
    G[:, 0, :, n_wake + n_chord] = S[:, :, 0]
    G[:, 0, :, n_wake + n_chord + 1:] = cut
    G[:, 1:] = vol[:, n_wake * n_span:].reshape(3, n_layers, n_span, m)
    return G


def hex_jacobians(vol: np.ndarray, surf: np.ndarray, meta: dict) -> np.ndarray:
    """Corner Jacobian (triple product of the three edges at the first corner) of every
    hexahedron of the C-H shell, shape [n_layers, n_span - 1, m - 1] (layer, span station, C-line
    segment). A valid mesh has every cell of one sign, the sign of the undeformed mesh."""
    G = ch_nodes(vol, surf, meta["n_chord"], meta["n_span"], meta["n_layers"], meta["n_wake"])
    a = G[:, :-1, :-1, :-1]
    ei = G[:, :-1, :-1, 1:] - a
    ek = G[:, :-1, 1:, :-1] - a
    ej = G[:, 1:, :-1, :-1] - a
    return np.einsum("cljk,cljk->ljk", ej, np.cross(ei, ek, axis=0))


# --------------------------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------------------------
@dataclass
class Workload:
    """One deformation problem: geometry, prescribed surface displacement, greedy parameters."""
    name: str
    dim: int
    xs: np.ndarray            # [dim, n_s] surface points
    ds: np.ndarray            # [dim, n_s] prescribed surface displacement
    xv: np.ndarray            # [dim, n_v] volume points
    dwall: np.ndarray         # [n_v] wall distance
    radius: List[float]       # support radius per level
    eps: float                # absolute tolerance on max_i ||E_i||
    rho: float = 0.1          # per-level reduction of the normalized error
    D: float = 1.0            # wall-distance support
    cap: int = 0              # cap on the total number of control points (0: n_s per level)
    seeds: List[List[int]] = field(default_factory=lambda: [[0]])
    precision: str = "fp64"
    meta: dict = field(default_factory=dict)
    d_factor: float = 0.0     # k > 0: support distances D_l = k max ||dS_l|| (section 4)

    def __post_init__(self):
        # Row-contiguous SoA, as the device calls take them.
        self.xs = np.ascontiguousarray(self.xs, dtype=np.float64)
        self.ds = np.ascontiguousarray(self.ds, dtype=np.float64)
        self.xv = np.ascontiguousarray(self.xv, dtype=np.float64)
        self.dwall = np.ascontiguousarray(self.dwall, dtype=np.float64)

    @property
    def n_s(self) -> int:
        return self.xs.shape[1]

    @property
    def n_v(self) -> int:
        return self.xv.shape[1]

    @property
    def n_levels(self) -> int:
        return len(self.radius)

    def seed_csr(self):
        lv = [list(self.seeds[l]) if l < len(self.seeds) else [] for l in range(self.n_levels)]
        off = np.zeros(self.n_levels + 1, dtype=np.int32)
        for l, s in enumerate(lv):
            off[l + 1] = off[l] + len(s)
        idx = np.array([p for s in lv for p in s], dtype=np.int64)
        return idx, off

    def cap_total(self) -> int:
        return self.cap if self.cap > 0 else self.n_s * self.n_levels


def _gauss(s, s0, w):
    return np.exp(-(((s - s0) / w) ** 2))


def airfoil_2d(n_s: int, n_layers: int, first_layer: float):
    x, y = naca0012_contour(n_s)
    xs = np.stack([x, y])
    xv, yv = omesh_2d(x, y, n_layers, first_layer)
    vol = np.stack([xv, yv])
    return xs, vol


def workload_cfg0(n_s: int = 400, n_layers: int = 50) -> Workload:
    """2D single-level FP64: NACA0012 with one Gaussian ice horn on the upper leading edge
    (amplitude 0.03c, width 0.02 in arc length, centred where the upper surface has x = 0.01c)
    plus a seeded uniform jitter of 1e-4c per component. Wendland C2 with R = 2c, two seed
    points, eps = 1e-5c, D = 1c."""
    rng = np.random.default_rng(SEED_BASE + 0)
    xs, xv = airfoil_2d(n_s, n_layers, 1e-3)
    nx, ny = contour_normals(xs[0], xs[1])
    s = arc_length_from_te(xs[0], xs[1])
    s0 = upper_arc_length_at(xs[0], s, 0.01)
    amp = 0.03 * _gauss(s, s0, 0.02)
    ds = np.stack([amp * nx, amp * ny]) + rng.uniform(-1e-4, 1e-4, size=(2, n_s))
    return Workload("cfg0_naca0012_2d_single_level", 2, xs, ds, xv, wall_distance(xs, xv),
                    radius=[2.0], eps=1e-5, D=1.0, seeds=[[0, 1]], cap=n_s,
                    meta=dict(cfg=0, n_layers=n_layers))


def workload_cfg1(n_s: int = 4000, n_layers: int = 100, precision: str = "fp64") -> Workload:
    """2D multi-level: NACA0012 with two seeded Gaussian ice horns along the normal (one on each
    side, centres at x ~ U[0.005, 0.03]c, amplitudes U[0.02, 0.05]c, widths U[0.01, 0.03]) plus
    a 0.005c rime layer over x < 0.1c. Levels R = 2c, 0.5c, 0.1c; eps = 1e-5c; D = 0.5c."""
    rng = np.random.default_rng(SEED_BASE + 1)
    first = 2.5e-4 if n_s >= 4000 else 1e-3
    xs, xv = airfoil_2d(n_s, n_layers, first)
    nx, ny = contour_normals(xs[0], xs[1])
    s = arc_length_from_te(xs[0], xs[1])
    half = n_s // 2
    amp = np.zeros(n_s)
    for side in (0, 1):
        xc = rng.uniform(0.005, 0.03)
        a = rng.uniform(0.02, 0.05)
        w = rng.uniform(0.01, 0.03)
        s_up = upper_arc_length_at(xs[0], s, xc)
        s_c = s_up if side == 0 else 2.0 * s[half] - s_up  # mirror point on the lower side
        amp += a * _gauss(s, s_c, w)
    amp += np.where(xs[0] < 0.1, 0.005, 0.0)
    ds = np.stack([amp * nx, amp * ny])
    return Workload("cfg1_naca0012_2d_multilevel", 2, xs, ds, xv, wall_distance(xs, xv),
                    radius=[2.0, 0.5, 0.1], eps=1e-5, D=0.5, seeds=[[0]], cap=3 * n_s,
                    precision=precision, meta=dict(cfg=1, n_layers=n_layers))


def wing_3d(n_chord: int, n_span: int, n_layers: int, n_wake: int):
    """Swept-wing surface and its C-H shell: (xyz, volume, section x, section z, span stations)."""
    xyz, xc, zc, yk = wing_surface(n_chord, n_span)
    xle = yk * math.tan(math.radians(25.0))
    vol = ch_shell_3d(xc, zc, xle, yk, n_wake, n_layers)
    return xyz, vol, xc, zc, yk


def wing_meta(n_chord: int, n_span: int, n_layers: int, n_wake: int, **kw) -> dict:
    return dict(n_chord=n_chord, n_span=n_span, n_layers=n_layers, n_wake=n_wake, **kw)


def workload_cfg2(n_chord: int = 400, n_span: int = 200, n_layers: int = 40, n_wake: int = 49,
                  precision: str = "fp64", cap: int = 4000) -> Workload:
    """3D iced wing: leading-edge horn (the 2D horn profile in local arc length) whose amplitude
    is 0.04c (1 - 0.5 y/b)(1 + 0.1 u_k), u_k ~ U[-1, 1] per station. Levels R = 3c, 0.8c, 0.2c,
    eps = 1e-4c, at most ``cap`` control points in total, D = 1c."""
    rng = np.random.default_rng(SEED_BASE + 2)
    xyz, vol, xc, zc, yk = wing_3d(n_chord, n_span, n_layers, n_wake)
    n = wing_normals(xyz, n_chord, n_span)
    s = arc_length_from_te(xc, zc)
    s0 = upper_arc_length_at(xc, s, 0.01)
    b = yk[-1]
    u = rng.uniform(-1.0, 1.0, size=n_span)
    amp_k = 0.04 * (1.0 - 0.5 * yk / b) * (1.0 + 0.1 * u)
    amp = (amp_k[:, None] * _gauss(s, s0, 0.02)[None, :]).reshape(-1)
    ds = n * amp[None, :]
    return Workload("cfg2_swept_wing_3d_ice", 3, xyz, ds, vol, wall_distance(xyz, vol),
                    radius=[3.0, 0.8, 0.2], eps=1e-4, D=1.0, seeds=[[0]], cap=cap,
                    precision=precision, meta=wing_meta(n_chord, n_span, n_layers, n_wake, cfg=2))


def bend_twist(xyz: np.ndarray, semi_span: float, tip_deflection: float = 0.1,
               tip_twist_deg: float = 5.0, sweep_deg: float = 25.0) -> np.ndarray:
    """Parabolic bending dz = tip_deflection * b (y/b)^2 plus a linear twist, nose up, of
    tip_twist_deg * y/b about the local quarter chord, rotating in the x-z plane."""
    X, Y, Z = xyz
    eta = Y / semi_span
    th = np.radians(tip_twist_deg) * eta
    xq = Y * math.tan(math.radians(sweep_deg)) + 0.25 * CHORD
    c, s_ = np.cos(th), np.sin(th)
    xr = xq + (X - xq) * c + Z * s_
    zr = -(X - xq) * s_ + Z * c
    dz = tip_deflection * semi_span * eta**2
    return np.stack([xr - X, np.zeros_like(Y), zr - Z + dz])


def workload_cfg3(n_chord: int = 400, n_span: int = 200, n_layers: int = 40, n_wake: int = 49,
                  cap: int = 4000) -> Workload:
    """3D global deformation: the wing and meshes of the iced-wing case deformed by parabolic
    bending (tip deflection 0.1b) plus linear twist (5 degrees at the tip). Mixed precision."""
    xyz, vol, xc, zc, yk = wing_3d(n_chord, n_span, n_layers, n_wake)
    ds = bend_twist(xyz, yk[-1])
    return Workload("cfg3_swept_wing_3d_bend_twist", 3, xyz, ds, vol, wall_distance(xyz, vol),
                    radius=[3.0, 0.8, 0.2], eps=1e-4, D=1.0, seeds=[[0]], cap=cap,
                    precision="mixed", meta=wing_meta(n_chord, n_span, n_layers, n_wake, cfg=3))


def workload_sine2d(n_s: int = 4000, n_layers: int = 100) -> Workload:
    """The paper's global-deformation benchmark in 2D (Results, airfoil): every surface point of
    the NACA0012 moves by dy = 0.01 sin(15 pi x), x along the chord in units of c. The paper's
    parameters: Wendland C2 with R = 2c on all five levels, a reduction of 0.1 per level (so
    eps = 1e-5 of max ||dS||), volume reduction factor k = 5. Mesh as the multi-level ice case."""
    first = 2.5e-4 if n_s >= 4000 else 1e-3
    xs, xv = airfoil_2d(n_s, n_layers, first)
    ds = np.stack([np.zeros(n_s), 0.01 * np.sin(15.0 * np.pi * xs[0])])
    top = float(np.sqrt((ds ** 2).sum(axis=0)).max())
    return Workload("sine2d_naca0012", 2, xs, ds, xv, wall_distance(xs, xv), radius=[2.0] * 5,
                    eps=1e-5 * top, D=1.0, seeds=[[0]], cap=0, d_factor=5.0,
                    meta=dict(n_layers=n_layers))


def workload_sine3d(n_chord: int = 400, n_span: int = 200, n_layers: int = 40, n_wake: int = 49,
                    cap: int = 4000) -> Workload:
    """The paper's global-deformation benchmark on the swept wing (eq. (27)): the displacement
    normal to the wing plane is 0.03 sin(4 pi s) with s the spanwise coordinate in units of c (the
    paper's y and z are this generator's z and y). R = 3c on four levels, reduction 0.1 per level,
    eps = 1e-4c, at most ``cap`` control points, k = 5. Mesh as the iced-wing case."""
    xyz, vol, xc, zc, yk = wing_3d(n_chord, n_span, n_layers, n_wake)
    ds = np.stack([np.zeros(xyz.shape[1]), np.zeros(xyz.shape[1]), 0.03 * np.sin(4.0 * np.pi * xyz[1])])
    return Workload("sine3d_swept_wing", 3, xyz, ds, vol, wall_distance(xyz, vol), radius=[3.0] * 4,
                    eps=1e-4, D=1.0, seeds=[[0]], cap=cap, d_factor=5.0,
                    meta=wing_meta(n_chord, n_span, n_layers, n_wake))


def workload(cfg: int, **kw) -> Workload:
    return {0: workload_cfg0, 1: workload_cfg1, 2: workload_cfg2, 3: workload_cfg3}[cfg](**kw)


# --------------------------------------------------------------------------------------------
# Small random inputs for unit tests
# --------------------------------------------------------------------------------------------
def random_points(rng: np.random.Generator, dim: int, n: int, scale: float = 1.0) -> np.ndarray:
    return np.ascontiguousarray(rng.uniform(-scale, scale, size=(dim, n)))


def random_workload(seed: int, dim: int, n_s: int, n_v: int, radius, eps: float,
                    D: float = 1.5, cap: int = 0, seeds=None, rho: float = 0.1) -> Workload:
    """Random points in a box with a smooth-plus-local displacement; volume points scattered
    around the surface set; used for the small parity cases."""
    rng = np.random.default_rng(SEED_BASE * 1000 + seed)
    xs = random_points(rng, dim, n_s)
    centre = rng.uniform(-0.5, 0.5, size=(dim, 1))
    r2 = ((xs - centre) ** 2).sum(axis=0)
    ds = 0.05 * np.exp(-r2 / 0.1)[None, :] * rng.uniform(0.5, 1.0, size=(dim, 1)) \
        + 0.01 * np.sin(3.0 * xs[::-1]) + rng.uniform(-1e-3, 1e-3, size=(dim, n_s))
    xv = random_points(rng, dim, n_v, scale=1.6)
    dwall = wall_distance(xs, xv)
    return Workload(f"random{seed}_d{dim}_s{n_s}", dim, xs, np.ascontiguousarray(ds), xv, dwall,
                    radius=list(radius), eps=eps, D=D, cap=cap, rho=rho,
                    seeds=seeds if seeds is not None else [[0]])


# --------------------------------------------------------------------------------------------
# Serving mix
# --------------------------------------------------------------------------------------------
@dataclass
class MixGeometry:
    dim: int
    xs: np.ndarray
    xv: np.ndarray
    dwall: np.ndarray
    normals: np.ndarray
    shape: np.ndarray          # [dim, n_s] displacement of the final icing step
    radius: List[float]
    D: float
    cap: int


@dataclass
class MixRequest:
    geom: int                  # index into the geometry list
    step: int                  # icing step 1..steps (amplitude step/steps)
    arrival: float             # seconds after the start
    eps: float
    precision: str


def serving_mix(n_geom: int = 64, steps: int = 4, rate: float = 20.0, frac_2d: float = 0.6,
                scale: float = 1.0, precision: str = "mixed", seed: int = 4, progress=None):
    """Seeded request mix: 2D airfoils (surface log-uniform in [500, 8000] points, O-mesh with
    40-100 layers) and 3D wings (400 x [25, 200] surface grid, 50 layers), each geometry deformed
    in `steps` successive icing steps of growing amplitude (ice horns, or bending plus twist for
    half of the wings), eps drawn from {1e-4, 1e-5}, Poisson arrivals at `rate` per second with
    each geometry's steps in order. `scale` < 1 shrinks every surface and volume (tests, quick
    runs). progress (optional) is called with a line of text after each geometry."""
    rng = np.random.default_rng(SEED_BASE + seed)
    geoms: List[MixGeometry] = []
    n2 = int(round(frac_2d * n_geom))
    for g in range(n_geom):
        if g < n2:
            n_s = int(np.exp(rng.uniform(np.log(500), np.log(8000))) * scale)
            n_s = max(64, n_s - n_s % 2)
            n_r = int(round(40 + 60 * np.log(max(n_s / scale, 500) / 500) / np.log(16)))
            n_r = max(4, int(n_r * min(1.0, scale * 4)))
            xs, xv = airfoil_2d(n_s, n_r, 1e-3)
            nx, ny = contour_normals(xs[0], xs[1])
            s = arc_length_from_te(xs[0], xs[1])
            half = n_s // 2
            amp = np.zeros(n_s)
            for side in (0, 1):
                xc = rng.uniform(0.005, 0.03)
                s_up = upper_arc_length_at(xs[0], s, xc)
                s_c = s_up if side == 0 else 2.0 * s[half] - s_up
                amp += rng.uniform(0.02, 0.05) * _gauss(s, s_c, rng.uniform(0.01, 0.03))
            amp += np.where(xs[0] < 0.1, 0.005, 0.0)
            shape = np.stack([amp * nx, amp * ny])
            geoms.append(MixGeometry(2, xs, xv, wall_distance(xs, xv), np.stack([nx, ny]), shape,
                                     [2.0, 0.5, 0.1], 0.5, 3 * n_s))
        else:
            n_c = max(40, int(400 * scale) - int(400 * scale) % 2)
            n_span = max(6, int(rng.integers(25, 201) * scale))
            n_r = max(4, int(40 * min(1.0, scale * 4)))
            xyz, vol, xc2, zc2, yk = wing_3d(n_c, n_span, n_r, max(4, n_c // 8 - 1))
            n = wing_normals(xyz, n_c, n_span)
            if rng.uniform() < 0.5:
                s = arc_length_from_te(xc2, zc2)
                s0 = upper_arc_length_at(xc2, s, 0.01)
                u = rng.uniform(-1.0, 1.0, size=n_span)
                amp_k = 0.04 * (1.0 - 0.5 * yk / yk[-1]) * (1.0 + 0.1 * u)
                shape = n * (amp_k[:, None] * _gauss(s, s0, 0.02)[None, :]).reshape(-1)[None, :]
            else:
                shape = bend_twist(xyz, yk[-1])
            geoms.append(MixGeometry(3, xyz, vol, wall_distance(xyz, vol), n, np.ascontiguousarray(shape),
                                     [3.0, 0.8, 0.2], 1.0, min(4000, xyz.shape[1])))
        if progress is not None:
            progress(f"serving mix: geometry {g + 1}/{n_geom} built ({geoms[-1].xv.shape[1]} volume points)")
    order = [g for g in range(n_geom) for _ in range(steps)]
    rng.shuffle(order)
    seen = [0] * n_geom
    t = 0.0
    reqs: List[MixRequest] = []
    for g in order:
        t += rng.exponential(1.0 / rate)
        seen[g] += 1
        reqs.append(MixRequest(g, seen[g], t, float(rng.choice([1e-4, 1e-5])), precision))
    return geoms, reqs

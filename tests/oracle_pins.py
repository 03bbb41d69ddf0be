"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each ``pin_*`` function takes an ``oracle.Oracle`` and raises AssertionError when the oracle
disagrees with the fact it checks. ``test_oracle_pins.py`` runs them on the real oracle and
``test_oracle_mutants.py`` runs them on copies of the oracle with a planted mistake, to show
that every plausible slip (dropped term, wrong sign, wrong index, skipped step) fails one pin.
"""
import math

import numpy as np

import synth
from bruteforce import greedy_bruteforce, pairwise_distance, phi_expanded


# ---- basis and weight functions ------------------------------------------------------------
def pin_wendland_dyadic(o):
    """Eq. (2) at dyadic points, where (1-e)^4 (4e+1) is exact in binary floating point."""
    exact = {0.0: 1.0, 0.25: 81.0 / 128.0, 0.5: 3.0 / 16.0, 0.75: 1.0 / 64.0,
             0.875: 4.5 / 4096.0, 0.125: (7.0 / 8.0) ** 4 * 1.5, 1.0: 0.0, 1.5: 0.0, 7.0: 0.0}
    for eta, val in exact.items():
        got = o.wendland_c2(eta)
        assert got == val, (eta, got, val)


def pin_wendland_expansion(o):
    """The factored form equals the expanded quintic 1 - 10e^2 + 20e^3 - 15e^4 + 4e^5 (up to
    the cancellation of the expanded form near eta = 1, a few units of 1e-15)."""
    rng = np.random.default_rng(7)
    for eta in rng.uniform(0.0, 1.0, 200):
        assert abs(o.wendland_c2(eta) - float(phi_expanded(eta))) <= 1e-14, eta


def pin_wendland_c2_cutoff(o):
    """C2 contact at the support edge: phi(1-h) = h^4 (5 - 4h), so phi, phi' and phi'' vanish
    at eta = 1 (checked exactly at dyadic h)."""
    for h in (0.5, 0.25, 0.125, 2.0**-6, 2.0**-10):
        assert o.wendland_c2(1.0 - h) == h**4 * (5.0 - 4.0 * h), h


_TABLE1 = {"c0": (2, 0), "c2": (4, 1), "c4": (6, 2), "c6": (8, 3)}   # (power of 1 - eta, k)


def pin_wendland_table1_values(o):
    """Table 1 at points where the value is exact in binary (C0, C2, C6; C4 has the constant
    35/3 and is checked to a few ulps): phi(0) = 1 for every function, 0 from eta = 1 on."""
    exact = {"c0": {0.5: 0.25, 0.25: 9.0 / 16.0, 0.75: 1.0 / 16.0},
             "c2": {0.5: 3.0 / 16.0, 0.25: 81.0 / 128.0},
             "c6": {0.5: 61.0 / 1024.0, 0.25: 531441.0 / 1048576.0}}
    for b in _TABLE1:
        assert o.wendland(b, 0.0) == 1.0, b
        for eta in (1.0, 1.25, 9.0):
            assert o.wendland(b, eta) == 0.0, (b, eta)
        for eta, val in exact.get(b, {}).items():
            assert o.wendland(b, eta) == val, (b, eta)
    for eta, val in {0.5: 83.0 / 768.0, 0.25: 112995.0 / 196608.0}.items():
        assert abs(o.wendland("c4", eta) - val) <= 4e-16 * val, eta
    for eta in np.linspace(0.0, 0.99, 37):
        assert o.wendland("c2", eta) == o.wendland_c2(eta)


def pin_wendland_table1_smoothness(o):
    """Wendland's construction: the function with (1 - eta)^m as a factor has m - 1 vanishing
    derivatives at eta = 1, and the one of smoothness C^2k has vanishing odd derivatives of
    order < 2k at eta = 0 (it is an even, 2k-times differentiable function of r there). Checked
    on the polynomial through samples of the oracle (exact interpolation, degree m + k)."""
    from numpy.polynomial import polynomial as P

    for b, (m, k) in _TABLE1.items():
        deg = m + k
        nodes = 0.5 - 0.5 * np.cos(np.pi * (np.arange(deg + 1) + 0.5) / (deg + 1))
        vals = np.array([o.wendland(b, e) for e in nodes])
        coef = np.linalg.solve(np.vander(nodes, deg + 1, increasing=True), vals)
        for j in range(m):
            dj = P.polyval(1.0, P.polyder(coef, j)) if j else P.polyval(1.0, coef)
            # rounding scale of the j-th derivative at 1: sum_i |c_i| i! / (i - j)!
            scale = sum(abs(c) * math.factorial(i) / math.factorial(i - j) for i, c in enumerate(coef) if i >= j)
            assert abs(dj) <= 1e-9 * scale, (b, "eta=1", j, dj, scale)
        for j in range(1, 2 * k, 2):
            # phi^(j)(0) = j! c_j, zero up to the fit's rounding (relative to the largest c_i)
            assert abs(coef[j]) <= 1e-10 * np.abs(coef).max(), (b, "eta=0", j, coef[j])
        if k == 0:
            assert abs(P.polyval(0.0, P.polyder(coef, 1)) + 2.0) <= 1e-9   # C0: slope -2 at 0
    # the test itself detects a wrong coefficient: 6 eta -> 5 eta in C4 breaks phi'(0) = 0
    bad = lambda e: (1 - e) ** 6 * (35.0 / 3.0 * e * e + 5.0 * e + 1.0)
    assert abs((bad(1e-6) - bad(0.0)) / 1e-6) > 0.5


def pin_wendland_table1_positive_definite(o):
    """Every function of Table 1 is positive definite on R^3 (Wendland 1995): the matrix on
    random 3D points has positive eigenvalues, and the oracle's weight solve with that basis
    equals LAPACK's."""
    rng = np.random.default_rng(21)
    xc = rng.uniform(-1, 1, (3, 70))
    dsc = rng.uniform(-0.05, 0.05, (3, 70))
    dist = pairwise_distance(xc, xc) / 1.3
    for b in _TABLE1:
        Phi = np.vectorize(lambda e: o.wendland(b, e))(dist)
        assert np.linalg.eigvalsh(Phi).min() > 0.0, b
        st, alpha = o.solve_weights(1.3, xc, dsc, basis=b)
        assert st == 0, b
        ref = np.linalg.solve(Phi, dsc.T).T
        assert np.abs(alpha - ref).max() <= 1e-9 * np.abs(ref).max(), b


def pin_greedy_bruteforce_table1(o):
    """The greedy with the C0, C4 and C6 bases gives the brute-force selection sequence (fresh
    dense solve each iteration, evaluated with the same basis)."""
    w = synth.random_workload(23, 3, 48, 10, [1.2, 0.5], 1e-6)
    for b in ("c0", "c4", "c6"):
        phi = np.vectorize(lambda e, b=b: o.wendland(b, e))
        res = o.greedy(3, w.xs, w.ds, w.radius, w.eps, basis=b)
        levels, alphas, _ = greedy_bruteforce(w.xs, w.ds, w.radius, w.eps, phi=phi)
        got = [list(res.level(l)[0]) for l in range(res.n_levels_used)]
        assert got == [list(c) for c in levels[: res.n_levels_used]], b
        vol = o.volume(w.radius, [0.9, 0.9], res.level_off, w.xs[:, res.ctrl_idx], res.alpha, w.xs[:, :5],
                       np.zeros(5), basis=b)
        surf = sum(o.evaluate(w.radius[l], w.xs[:, res.level(l)[0]], res.level(l)[1], w.xs[:, :5], basis=b)
                   for l in range(res.n_levels_used))
        assert np.abs(vol - surf).max() <= 1e-15 * max(1.0, np.abs(surf).max()), b


def pin_psi(o):
    """Wall-distance function of Section 4: 1 - xi on [0, 1), zero from xi = 1 on."""
    for xi, val in {0.0: 1.0, 0.25: 0.75, 0.5: 0.5, 0.75: 0.25, 1.0: 0.0, 2.0: 0.0}.items():
        assert o.psi(xi) == val, xi


# ---- weights ---------------------------------------------------------------------------------
def pin_solve_matches_lapack(o):
    """Phi_cc alpha = dS_c (eq. (9) on a point set) equals LAPACK's dense solve."""
    rng = np.random.default_rng(11)
    for dim, n, R in ((2, 60, 1.5), (3, 120, 2.0), (3, 17, 0.7)):
        xc = rng.uniform(-1, 1, (dim, n))
        dsc = rng.uniform(-0.05, 0.05, (dim, n))
        st, alpha = o.solve_weights(R, xc, dsc)
        assert st == 0
        Phi = phi_expanded(pairwise_distance(xc, xc) / R)
        ref = np.linalg.solve(Phi, dsc.T).T
        scale = np.abs(ref).max()
        assert np.abs(alpha - ref).max() <= 1e-9 * scale, (dim, n)
        assert np.abs(alpha @ Phi - dsc).max() <= 1e-12


def pin_one_and_two_points(o):
    """Closed forms: one control point gives alpha = dS (phi(0) = 1); two points at distance
    r give alpha = (dS_0 - p dS_1, dS_1 - p dS_0) / (1 - p^2) with p = phi(r/R)."""
    xc = np.array([[0.3], [0.2]])
    st, a = o.solve_weights(1.0, xc, np.array([[0.01], [-0.02]]))
    assert st == 0 and np.array_equal(a, np.array([[0.01], [-0.02]]))
    xc = np.array([[0.0, 0.5], [0.0, 0.0]])
    ds = np.array([[1.0, 2.0], [0.0, -1.0]])
    st, a = o.solve_weights(1.0, xc, ds)
    p = 3.0 / 16.0
    ref = np.stack([(ds[:, 0] - p * ds[:, 1]), (ds[:, 1] - p * ds[:, 0])], axis=1) / (1 - p * p)
    assert st == 0 and np.abs(a - ref).max() <= 1e-15


def pin_not_spd_on_duplicates(o):
    """A repeated point makes Phi_cc singular; the solve reports it instead of returning junk."""
    xc = np.array([[0.0, 0.3, 0.3], [0.0, 0.1, 0.1]])
    st, _ = o.solve_weights(1.0, xc, np.zeros((2, 3)))
    assert st == -3


# ---- greedy ----------------------------------------------------------------------------------
def _tiny_cases():
    cases = []
    for seed, dim, n, radius, eps in ((1, 2, 40, [1.5], 1e-6), (2, 3, 48, [2.0], 1e-5),
                                      (3, 2, 64, [2.0, 0.5], 1e-7), (4, 3, 64, [1.0, 0.4, 0.2], 1e-6)):
        w = synth.random_workload(seed, dim, n, 10, radius, eps)
        cases.append((w.xs, w.ds, radius, eps, [[0]]))
    xs, _ = synth.airfoil_2d(64, 4, 1e-3)
    ds = np.stack([0.02 * np.exp(-((xs[0] - 0.02) / 0.05) ** 2), 0.01 * np.sin(5 * xs[0])])
    cases.append((xs, ds, [2.0, 0.5], 1e-8, [[0, 1]]))
    return cases


def pin_greedy_bruteforce(o):
    """Identical selection to a brute-force greedy that re-solves the dense control-set system
    with LAPACK every iteration (tiny inputs, 2D and 3D, single and multi-level)."""
    for xs, ds, radius, eps, seeds in _tiny_cases():
        dim = xs.shape[0]
        res = o.greedy(dim, xs, ds, radius, eps, seeds=seeds)
        lv, alphas, r = greedy_bruteforce(xs, ds, radius, eps, seeds=seeds)
        got = [list(res.level(l)[0]) for l in range(res.n_levels_used)]
        assert got == lv, (got, lv)
        for l, a in enumerate(alphas):
            ref = res.level(l)[1]
            assert np.abs(ref - a).max() <= 1e-8 * max(1.0, np.abs(a).max())
        assert np.abs(res.e_final - r).max() <= 1e-10


def pin_greedy_reproduction(o):
    """The interpolant reproduces the data at its control points: after a level closes the
    residual there is zero up to rounding (|E_c| <= 1e-12 max|dS|)."""
    w = synth.random_workload(5, 2, 300, 10, [1.0], 1e-6)
    res = o.greedy(2, w.xs, w.ds, w.radius, w.eps)
    c, _ = res.level(0)
    scale = np.sqrt((w.ds**2).sum(0)).max()
    assert np.abs(res.e_final[:, c]).max() <= 1e-12 * scale
    assert res.level_max_err[0] < w.eps


def pin_greedy_all_selected(o):
    """With eps = 0 every point is selected and the greedy interpolant is the full RBF
    interpolant of eq. (9): E is zero everywhere and alpha equals the dense N_s solve."""
    w = synth.random_workload(6, 3, 80, 10, [1.2], 0.0)
    res = o.greedy(3, w.xs, w.ds, [1.2], 0.0, cap=80)
    assert res.level_stop[0] == 2 and len(res.ctrl_idx) == 80
    assert np.abs(res.e_final).max() <= 1e-12 * np.abs(w.ds).max()
    order = res.ctrl_idx
    Phi = phi_expanded(pairwise_distance(w.xs, w.xs) / 1.2)
    full = np.linalg.solve(Phi, w.ds.T).T
    assert np.abs(res.alpha - full[:, order]).max() <= 1e-8 * np.abs(full).max()


def pin_greedy_ties_lowest_index(o):
    """Exact ties (mirror-symmetric points with equal data) go to the lowest index."""
    x = np.array([0.0, -0.3, 0.3, -0.6, 0.6])
    xs = np.stack([x, np.zeros_like(x)])
    ds = np.stack([np.array([0.0, 1.0, 1.0, 0.5, 0.5]), np.zeros(5)])
    res = o.greedy(2, xs, ds, [1.0], 0.0, cap=3, seeds=[[0]])
    assert list(res.ctrl_idx) == [0, 1, 2], res.ctrl_idx


def pin_greedy_native_norm_monotone(o):
    """Each added point is an orthogonal projection onto a larger subspace of the native space,
    so alpha . dS_C (= |s_n|^2 in the native norm) never decreases within a level."""
    w = synth.random_workload(8, 2, 120, 10, [0.8], 1e-9)
    prev = -1.0
    for k in range(1, 40):
        res = o.greedy(2, w.xs, w.ds, [0.8], 1e-9, cap=k)
        c, a = res.level(0)
        nn = float((a * w.ds[:, c]).sum())
        assert nn >= prev * (1 - 1e-12), (k, nn, prev)
        prev = nn


def pin_greedy_telescoping(o):
    """Multi-level: the level interpolants sum to dS minus the final residual (Section 3,
    dS = sum_i Phi_sc^(i) alpha^(i) up to the residual), and each level starts from the last
    level's residual (dS_{l+1} = E)."""
    w = synth.random_workload(9, 3, 200, 10, [2.0, 0.6, 0.25], 1e-7)
    res = o.greedy(3, w.xs, w.ds, w.radius, w.eps)
    assert res.n_levels_used >= 2
    total = np.zeros_like(w.ds)
    for l in range(res.n_levels_used):
        c, a = res.level(l)
        total += o.evaluate(w.radius[l], w.xs[:, c], a, w.xs)
    assert np.abs(total - (w.ds - res.e_final)).max() <= 1e-12 * np.abs(w.ds).max() * 10


def pin_greedy_cap_and_breakdown(o):
    """The cap stops selection; a duplicated surface point breaks the factorization down
    instead of producing a non-finite weight."""
    w = synth.random_workload(10, 2, 100, 10, [1.0, 0.3], 0.0)
    res = o.greedy(2, w.xs, w.ds, [1.0], 0.0, cap=25)
    assert len(res.ctrl_idx) == 25 and res.level_stop[0] == 1 and res.n_levels_used == 1
    res = o.greedy(2, w.xs, w.ds, w.radius, 0.0, cap=25)
    assert res.level_stop[0] == 0 and res.level_stop[1] == 1 and res.level_off[2] == 25
    xs = np.concatenate([w.xs[:, :10], w.xs[:, :1]], axis=1)
    ds = np.concatenate([w.ds[:, :10], w.ds[:, :1]], axis=1)
    res = o.greedy(2, xs, ds, [1.0], 0.0, cap=11)
    assert res.level_stop[0] == 3 and np.all(np.isfinite(res.alpha))


# ---- volume ----------------------------------------------------------------------------------
def _small_volume_case(o, seed=12, dim=3):
    w = synth.random_workload(seed, dim, 150, 400, [1.5, 0.5], 1e-6, D=0.9)
    res = o.greedy(dim, w.xs, w.ds, w.radius, w.eps)
    xc = w.xs[:, res.ctrl_idx]
    return w, res, xc


def pin_volume_zero_beyond_D(o):
    """psi is zero from d = D on, so points at or beyond the support distance get +0.0 exactly."""
    w, res, xc = _small_volume_case(o)
    D = [0.3, 0.2]
    dwall = w.dwall.copy()
    dwall[:50] = 0.3          # exactly at the largest D
    dv = o.volume(w.radius, D, res.level_off, xc, res.alpha, w.xv, dwall)
    far = dwall >= 0.3
    assert far.sum() > 50
    assert np.all(dv[:, far] == 0.0) and not np.any(np.signbit(dv[:, far]))
    assert np.any(dv[:, ~far] != 0.0)


def pin_volume_at_wall(o):
    """At d = 0, psi = 1 and the update is the sum of the level interpolants (eq. (19));
    at the surface points themselves that is dS minus the final residual."""
    w, res, xc = _small_volume_case(o, 13)
    dv = o.volume(w.radius, [1.0, 1.0], res.level_off, xc, res.alpha, w.xs, np.zeros(w.n_s))
    assert np.abs(dv - (w.ds - res.e_final)).max() <= 1e-11 * np.abs(w.ds).max()


def pin_volume_psi_weight(o):
    """With one level, the update at d = D/2 is exactly half of the update at d = 0, and at
    d = 3D/4 a quarter (psi linear on [0, D))."""
    w, res, xc = _small_volume_case(o, 14, dim=2)
    off = np.array([0, res.level_off[1]], dtype=np.int32)
    v0 = o.volume(w.radius[:1], [1.0], off, xc, res.alpha, w.xv, np.zeros(w.n_v))
    vh = o.volume(w.radius[:1], [1.0], off, xc, res.alpha, w.xv, np.full(w.n_v, 0.5))
    vq = o.volume(w.radius[:1], [1.0], off, xc, res.alpha, w.xv, np.full(w.n_v, 0.75))
    assert np.array_equal(vh, 0.5 * v0) and np.array_equal(vq, 0.25 * v0)


def pin_volume_linear(o):
    """For a fixed control set the update is linear in the surface data."""
    rng = np.random.default_rng(15)
    xc = rng.uniform(-1, 1, (3, 50))
    a1 = o.solve_weights(1.0, xc, rng.uniform(-1, 1, (3, 50)))[1]
    a2 = o.solve_weights(1.0, xc, rng.uniform(-1, 1, (3, 50)))[1]
    xv = rng.uniform(-1.5, 1.5, (3, 300))
    d = rng.uniform(0, 1.2, 300)
    off = np.array([0, 50], dtype=np.int32)
    v1 = o.volume([1.0], [1.0], off, xc, a1, xv, d)
    v2 = o.volume([1.0], [1.0], off, xc, a2, xv, d)
    v3 = o.volume([1.0], [1.0], off, xc, 2.0 * a1 - 0.5 * a2, xv, d)
    assert np.abs(v3 - (2.0 * v1 - 0.5 * v2)).max() <= 1e-12 * np.abs(v3).max()


def pin_rigid_motion(o):
    """Translating or rotating the whole problem (points and displacements) moves the result
    with it: same selection, displacements rotated, within rounding of the moved coordinates."""
    w = synth.random_workload(16, 3, 160, 300, [1.5, 0.5], 1e-6, D=0.9)
    base = o.greedy(3, w.xs, w.ds, w.radius, w.eps)
    dv0 = o.volume(w.radius, [w.D] * 2, base.level_off, w.xs[:, base.ctrl_idx], base.alpha, w.xv,
                   w.dwall)
    t = np.array([[1000.0], [-250.0], [400.0]])
    tr = o.greedy(3, w.xs + t, w.ds, w.radius, w.eps)
    assert np.array_equal(tr.ctrl_idx, base.ctrl_idx)
    dvt = o.volume(w.radius, [w.D] * 2, tr.level_off, (w.xs + t)[:, tr.ctrl_idx], tr.alpha,
                   w.xv + t, w.dwall)
    assert np.abs(dvt - dv0).max() <= 1e-8 * np.abs(dv0).max()
    c, s = math.cos(0.7), math.sin(0.7)
    Q = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    rt = o.greedy(3, Q @ w.xs, Q @ w.ds, w.radius, w.eps)
    assert np.array_equal(rt.ctrl_idx, base.ctrl_idx)
    dvr = o.volume(w.radius, [w.D] * 2, rt.level_off, (Q @ w.xs)[:, rt.ctrl_idx], rt.alpha,
                   Q @ w.xv, w.dwall)
    assert np.abs(dvr - Q @ dv0).max() <= 1e-10 * np.abs(dv0).max()


def pin_support_distances(o):
    """Section 4: D_l = k (dS_l)^max. A uniform displacement v gives D_0 = k |v|; later levels
    use the maximum of the error left by the previous level, recomputed here from the level
    interpolants (not from the greedy's own report)."""
    import oracle as orc_mod

    w = synth.random_workload(17, 2, 120, 10, [1.5, 0.4, 0.1], 1e-8)
    v = np.array([[3e-3], [-4e-3]])
    flat = np.repeat(v, w.n_s, axis=1)
    res = o.greedy(2, w.xs, flat, [1.5], 1e-6, cap=20)
    assert orc_mod.support_distances(5.0, flat, res) == [5.0 * 5e-3]
    res = o.greedy(2, w.xs, w.ds, w.radius, w.eps)
    assert res.n_levels_used == 3
    D = orc_mod.support_distances(5.0, w.ds, res)
    r = w.ds.copy()
    for l in range(3):
        want = 5.0 * np.sqrt((r ** 2).sum(axis=0)).max()
        assert abs(D[l] - want) <= 1e-12 * want
        c, a = res.level(l)
        r = r - o.evaluate(w.radius[l], w.xs[:, c], a, w.xs)
    assert D[0] > D[1] > D[2]


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]

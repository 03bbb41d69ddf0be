"""Brute-force greedy selection for tiny inputs: a fresh dense LAPACK solve of the control-set
system every iteration and a numpy argmax. It shares nothing with the oracle except the readings
of the paper (lowest index on ties, per-level targets, selected points excluded) and serves as
the pin for the oracle's greedy: same inputs, identical selection sequence.

The basis is written here in its expanded polynomial form 1 - 10 e^2 + 20 e^3 - 15 e^4 + 4 e^5,
which equals the factored Wendland C2 form of eq. (2) on [0, 1).
"""
import numpy as np


def phi_expanded(eta):
    eta = np.asarray(eta, dtype=np.float64)
    p = 1.0 + eta**2 * (-10.0 + eta * (20.0 + eta * (-15.0 + 4.0 * eta)))
    return np.where(eta < 1.0, p, 0.0)


def pairwise_distance(a, b):
    diff = a[:, :, None] - b[:, None, :]
    return np.sqrt((diff**2).sum(axis=0))


def greedy_bruteforce(xs, ds, radius, eps, rho=0.1, cap=0, seeds=None, phi=phi_expanded):
    """Returns (per-level control lists, per-level alpha [dim, n_l], final residual). ``phi`` is
    the basis as a vectorised function of eta (Wendland C2 by default)."""
    xs = np.asarray(xs, dtype=np.float64)
    r = np.array(ds, dtype=np.float64)
    n = xs.shape[1]
    cap = cap if cap > 0 else n * len(radius)
    seeds = seeds if seeds is not None else [[0]]
    dist = pairwise_distance(xs, xs)
    levels, alphas = [], []
    total = 0
    for l, R in enumerate(radius):
        last = l == len(radius) - 1
        Phi = phi(dist / R)
        rmax = np.sqrt((r**2).sum(axis=0)).max()
        target = eps if last else max(eps, rho * rmax)
        C = []
        for p in (seeds[l] if l < len(seeds) else []):
            if total + len(C) >= cap:
                break
            C.append(int(p))
        while True:
            if C:
                alpha = np.linalg.solve(Phi[np.ix_(C, C)], r[:, C].T).T
                E = r - alpha @ Phi[C, :]
            else:
                alpha = np.zeros((xs.shape[0], 0))
                E = r.copy()
            m2 = (E**2).sum(axis=0)
            m2[C] = -1.0
            if len(C) == n:
                break
            p = int(np.argmax(m2))
            if m2[p] < target * target or total + len(C) >= cap:
                break
            C.append(p)
        levels.append(C)
        alphas.append(alpha)
        total += len(C)
        r = E
        if np.sqrt((E**2).sum(axis=0)).max() < eps or total >= cap:
            break
    return levels, alphas, r

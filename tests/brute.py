"""Brute-force references for tiny graphs (n <= 12): pins of the oracle.

Nothing here calls the oracle's arithmetic.  Reachability is a boolean
transitive closure, spreads are counted vertex by vertex, and the exact IC
spread follows the cascade process of the IC model definition (Sec. 2: each
newly activated vertex tries each incident edge once, succeeding with p_e),
with exact rational probabilities.
"""
from fractions import Fraction
from itertools import combinations

import numpy as np

M64 = (1 << 64) - 1
PHI = 0x9E3779B97F4A7C15


def mix64_np(z):
    """SplitMix64 output function on uint64 numpy arrays (wrap-around arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z ^ (z >> np.uint64(30))
        z = z * np.uint64(0xBF58476D1CE4E5B9)
        z = z ^ (z >> np.uint64(27))
        z = z * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def mix64_int(z):
    return int(mix64_np(np.array([z & M64], dtype=np.uint64))[0])


def key_int(seed, x):
    return mix64_int((seed * PHI + x) & M64)


def live_mask(keys, r, seed, T):
    """Live test of the edges with canonical keys `keys` in sketch r."""
    if T == M64:
        return np.ones(keys.size, dtype=bool)
    K = np.uint64(key_int(seed, r))
    return mix64_np(np.asarray(keys, dtype=np.uint64) ^ K) < np.uint64(T)


def closure_labels(n, edges):
    """Labels (min reachable id) and sizes by boolean transitive closure."""
    A = np.eye(n, dtype=bool)
    for u, v in edges:
        A[u, v] = A[v, u] = True
    # repeated squaring until fixed point
    while True:
        B = (A.astype(np.int64) @ A.astype(np.int64)) > 0
        if (B == A).all():
            break
        A = B
    label = np.array([int(np.nonzero(A[v])[0].min()) for v in range(n)], dtype=np.uint32)
    size = A.sum(axis=1).astype(np.uint32)
    return label, size, A


def spread_in_world(A, S):
    """Number of vertices reachable from S in a world with reachability matrix A."""
    if not S:
        return 0
    return int(np.any(A[list(S)], axis=0).sum())


def brute_greedy(worlds, n, k):
    """Greedy on f(S) = sum over worlds of |reach(S)|, counting spreads directly."""
    S, seeds, gains = [], [], []
    fS = 0
    for _ in range(k):
        best, bestf = None, -1
        for v in range(n):
            if v in S:
                continue
            f = sum(spread_in_world(A, S + [v]) for A in worlds)
            if f > bestf:
                best, bestf = v, f
        seeds.append(best)
        gains.append(bestf - fS)
        S.append(best)
        fS = bestf
    return seeds, gains


def best_k_subset(worlds, n, k):
    best = -1
    for S in combinations(range(n), k):
        f = sum(spread_in_world(A, list(S)) for A in worlds)
        best = max(best, f)
    return best


def exact_ic_spread(n, edges, p, S):
    """E|activated| of the IC cascade started from S, as an exact Fraction.  p: one
    probability for every edge, or a dict {(min, max): probability}."""
    pe = {(min(u, v), max(u, v)): Fraction(p[(min(u, v), max(u, v))] if isinstance(p, dict) else p)
          for u, v in edges}
    adj = {v: [] for v in range(n)}
    for u, v in edges:
        adj[u].append(v)
        adj[v].append(u)

    def rec(active, frontier):
        # every (f, w) with f newly active and w inactive is one independent attempt
        attempts = [(f, w) for f in sorted(frontier) for w in adj[f] if w not in active]
        if not attempts:
            return Fraction(len(active))
        total = Fraction(0)
        m = len(attempts)
        for mask in range(1 << m):
            prob = Fraction(1)
            new = set()
            for i, (f, w) in enumerate(attempts):
                q = pe[(min(f, w), max(f, w))]
                if mask >> i & 1:
                    prob *= q
                    new.add(w)
                else:
                    prob *= 1 - q
            if prob == 0:
                continue
            total += prob * (rec(active | new, frozenset(new)) if new else Fraction(len(active)))
        return total

    S = frozenset(S)
    if not S:
        return Fraction(0)
    return rec(S, S)


def per_edge_p(g, salt=0):
    """A symmetric probability per CSR entry of graph g, from the pair (min, max)."""
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.offsets.astype(np.int64)))
    cols = g.cols.astype(np.int64)
    a, b = np.minimum(rows, cols), np.maximum(rows, cols)
    return np.ascontiguousarray(((a * 7919 + b * 104729 + salt * 31) % 1000) / 1000.0, dtype=np.float64)

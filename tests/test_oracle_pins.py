"""Pins of the oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a published reference output,
exact rational arithmetic, a library routine (scipy connected components),
brute-force reachability / enumeration on tiny graphs, the exact IC cascade
spread, or a closed form.  A plausible slip in the oracle (a dropped term, a
flipped comparison, a wrong index or tie rule) fails at least one of them.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import oracle
from paper_2311_07554_amd import inputs
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M64 = (1 << 64) - 1


# ---------------------------------------------------------------- hash / thresholds

def _golden_streams():
    rows = []
    with open(os.path.join(GOLDEN, "splitmix64_reference.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            rows.append((int(parts[0]), [int(x, 16) for x in parts[1:]]))
    return rows


@pytest.mark.parametrize("state,outs", _golden_streams())
def test_mix64_reproduces_published_splitmix64(state, outs):
    s = state
    for want in outs:
        s = (s + brute.PHI) & M64
        assert oracle.mix64(s) == want
        assert brute.mix64_int(s) == want  # the numpy transcription used by other pins


def test_edge_hash_spec_vectors():
    # Frozen before any implementation: h(u,v,r,seed) = mix64(((min<<32)|max) ^ K(seed, r)),
    # K(seed, r) = mix64(seed * phi + r), evaluated by hand from the published mixer.
    vec = [((0, 1, 0, 1), 0x9E0160293A33AAF7), ((1, 0, 0, 1), 0x9E0160293A33AAF7),
           ((3, 7, 5, 1), 0x76AD6B051034D182), ((999, 0, 63, 1), 0xC63F261867D006FB),
           ((123456, 654321, 255, 42), 0xBB7968C30C90476D)]
    for (u, v, r, seed), h in vec:
        a, b = min(u, v), max(u, v)
        assert oracle.mix64(((a << 32) | b) ^ oracle.key(seed, r)) == h
        # live iff h < T: a threshold just above / at h decides it
        assert oracle.live(u, v, r, seed, h + 1) and not oracle.live(u, v, r, seed, h)


def test_threshold_is_exact_floor_of_p_times_2_64():
    rng = np.random.default_rng(7)
    ps = list(rng.random(2000)) + [0.05, 0.02, 0.1, 0.01, 0.001, 5e-324, 1e-300, 0.5,
                                   math.nextafter(1.0, 0.0)]
    for p in ps:
        assert oracle.threshold(p) == int(Fraction(float(p)) * (1 << 64)), p
    assert oracle.threshold(0.0) == 0 and oracle.threshold(-0.5) == 0
    assert oracle.threshold(1.0) == M64 and oracle.threshold(3.0) == M64
    # values quoted with the workload definitions
    assert oracle.threshold(0.05) == 0x0CCCCCCCCCCCCD00
    assert oracle.threshold(0.02) == 0x051EB851EB851EC0


def test_live_fraction_calibrated():
    # binomial 5-sigma band around p over 200k (edge, sketch) pairs
    rng = np.random.default_rng(3)
    u = rng.integers(0, 1 << 20, 20000)
    v = rng.integers(0, 1 << 20, 20000)
    keys = (np.minimum(u, v).astype(np.uint64) << np.uint64(32)) | np.maximum(u, v).astype(np.uint64)
    for p in (0.5, 0.05, 0.001):
        T = oracle.threshold(p)
        live = sum(int(brute.live_mask(keys, r, 11, T).sum()) for r in range(10))
        N = keys.size * 10
        assert abs(live - N * p) <= 5 * math.sqrt(N * p * (1 - p)) + 1
    # spot-check the numpy transcription against the oracle's own live test
    T = oracle.threshold(0.3)
    mask = brute.live_mask(keys[:200], 4, 9, T)
    for i in range(200):
        assert bool(mask[i]) == oracle.live(int(u[i]), int(v[i]), 4, 9, T)


def test_trivalency_classes():
    rng = np.random.default_rng(5)
    cnt = {oracle.threshold(0.1): 0, oracle.threshold(0.01): 0, oracle.threshold(0.001): 0}
    for _ in range(3000):
        a, b = (int(x) for x in rng.integers(0, 1 << 30, 2))
        if a == b:
            continue
        T = oracle.edge_threshold(1, 0.0, a, b)
        assert T in cnt
        assert T == oracle.edge_threshold(1, 0.7, b, a)  # symmetric, ignores p
        cnt[T] += 1
    tot = sum(cnt.values())
    for c in cnt.values():
        assert abs(c - tot / 3) <= 5 * math.sqrt(tot * (1 / 3) * (2 / 3))
    # class = mix64(key ^ mix64(SALT_TRIV)) mod 3, checked with the numpy transcription
    key = (12 << 32) | 345
    cls = int(brute.mix64_np(np.array([key ^ brute.key_int(0, oracle.SALT_TRIV)], dtype=np.uint64))[0]) % 3
    assert oracle.edge_threshold(1, 0.0, 345, 12) == oracle.threshold((0.1, 0.01, 0.001)[cls])


# ---------------------------------------------------------------- sketches (labels, sizes)

def _edge_keys(g):
    rows = np.repeat(np.arange(g.n, dtype=np.uint64), np.diff(g.offsets.astype(np.int64)))
    cols = g.cols.astype(np.uint64)
    sel = rows < cols
    return (rows[sel] << np.uint64(32)) | cols[sel]


def _scipy_labels(n, keys, live):
    k = keys[live]
    u = (k >> np.uint64(32)).astype(np.int64)
    v = (k & np.uint64(0xFFFFFFFF)).astype(np.int64)
    A = sp.coo_matrix((np.ones(u.size), (u, v)), shape=(n, n))
    ncc, comp = connected_components(A, directed=False)
    mins = np.full(ncc, n, dtype=np.int64)
    np.minimum.at(mins, comp, np.arange(n))
    sizes = np.bincount(comp, minlength=ncc)
    return mins[comp].astype(np.uint32), sizes[comp].astype(np.uint32), ncc


@pytest.mark.parametrize("which", ["er", "rmat"])
def test_sketch_labels_match_library_connected_components(which):
    if which == "er":
        g, kind, p = inputs.er_graph(1000, 5000, seed=1), 0, 0.05
    else:
        g, kind, p = inputs.rmat_graph(12, 16 << 12, seed=9), 1, 0.0
    keys = _edge_keys(g)
    if kind == 0:
        T = np.full(keys.size, oracle.threshold(p), dtype=np.uint64)
    else:
        cls = brute.mix64_np(keys ^ np.uint64(brute.key_int(0, oracle.SALT_TRIV))) % np.uint64(3)
        tri = np.array([oracle.threshold(x) for x in (0.1, 0.01, 0.001)], dtype=np.uint64)
        T = tri[cls.astype(np.int64)]
    for r in (0, 1, 17, 63):
        K = np.uint64(brute.key_int(1, r))
        live = brute.mix64_np(keys ^ K) < T
        want_l, want_s, ncc = _scipy_labels(g.n, keys, live)
        lab, siz = oracle.sketch(g, kind, p, 1, r)
        assert np.array_equal(lab, want_l)
        assert np.array_equal(siz, want_s)
        # invariant: component sizes over the roots sum to n
        roots = lab == np.arange(g.n)
        assert int(siz[roots].sum()) == g.n and int(roots.sum()) == ncc


def _tiny_graphs():
    rng = np.random.default_rng(2024)
    out = []
    for t in range(6):
        n = int(rng.integers(4, 13))
        pairs = {(int(a), int(b)) for a, b in rng.integers(0, n, (int(rng.integers(n, 2 * n + 3)), 2)) if a != b}
        out.append(inputs.csr_from_pairs(n, pairs))
    return out


def _threshold_spelled_out(kind, p, u, w, du, dw):
    # the models' thresholds in Python integers from the published mixer, not the oracle
    if kind == 0:
        return oracle.threshold(p)
    if kind == 1:
        cls = brute.mix64_int(((u << 32) | w) ^ brute.key_int(0, oracle.SALT_TRIV)) % 3
        return oracle.threshold((0.1, 0.01, 0.001)[cls])
    if kind == 2:
        lo, hi = oracle.threshold(p[0]), oracle.threshold(p[1])
        h = brute.mix64_int(((min(u, w) << 32) | max(u, w)) ^ brute.key_int(0, oracle.SALT_RANGE))
        return lo + (((hi - lo) * h) >> 64)
    s_ = du + dw
    return M64 if s_ <= 2 else (1 << 65) // s_


def _live_edges(g, kind, p, seed, r):
    res = []
    deg = np.diff(g.offsets.astype(np.int64))
    for u in range(g.n):
        for j in range(int(g.offsets[u]), int(g.offsets[u + 1])):
            w = int(g.cols[j])
            if u < w:
                if kind == 4:
                    T = oracle.threshold(float(p[j]))
                else:
                    T = _threshold_spelled_out(kind, p, u, w, int(deg[u]), int(deg[w]))
                if T == M64 or brute.mix64_int(((u << 32) | w) ^ brute.key_int(seed, r)) < T:
                    res.append((u, w))
    return res


@pytest.mark.parametrize("gi", range(6))
@pytest.mark.parametrize("kind,p", [(0, 0.45), (1, 0.0), (2, (0.2, 0.7)), (3, 0.0), (4, None)])
def test_sketch_labels_match_transitive_closure(gi, kind, p):
    g = _tiny_graphs()[gi]
    if kind == 4:
        p = brute.per_edge_p(g, gi)
    for r in range(8):
        edges = _live_edges(g, kind, p, 3, r)
        lab_b, siz_b, _ = brute.closure_labels(g.n, edges)
        lab, siz = oracle.sketch(g, kind, p, 3, r)
        assert np.array_equal(lab, lab_b) and np.array_equal(siz, siz_b)


def test_uniform_range_thresholds():
    # Uniform model (appendix on edge-probability distributions): one p_e per edge,
    # uniform over [lo, hi), the same for every sketch and sampling seed
    rng = np.random.default_rng(8)
    lo, hi = 0.1, 0.3
    TL, TH = oracle.threshold(lo), oracle.threshold(hi)
    ts = []
    for _ in range(20000):
        a, b = (int(x) for x in rng.integers(0, 1 << 30, 2))
        if a == b:
            continue
        T = oracle.edge_threshold(oracle.RANGE, (lo, hi), a, b)
        assert T == oracle.edge_threshold(oracle.RANGE, (lo, hi), b, a)
        assert TL <= T < TH
        ts.append(T)
    N = len(ts)
    frac = np.array([t / 2.0**64 for t in ts])
    # mean and every tenth of the range within 5 sigma of uniform
    assert abs(frac.mean() - (lo + hi) / 2) <= 5 * (hi - lo) / math.sqrt(12 * N)
    counts = np.histogram(frac, bins=10, range=(lo, hi))[0]
    assert np.all(np.abs(counts - N / 10) <= 5 * math.sqrt(N * 0.1 * 0.9))
    # lo == hi is the Consistent model
    for a, b in [(1, 2), (5, 900), (77, 3)]:
        assert oracle.edge_threshold(oracle.RANGE, (0.05, 0.05), a, b) == oracle.threshold(0.05)


def test_wic_thresholds_are_exact_floors():
    # WIC (same appendix): p_e = 2 / (d_u + d_v); T = floor(p_e * 2^64) exactly
    for du in range(1, 60):
        for dv in range(1, 60):
            s_ = du + dv
            T = oracle.edge_threshold(oracle.WIC, 0.0, 3, 9, du, dv)
            if s_ == 2:
                assert T == M64
            else:
                assert T * s_ <= 1 << 65 < (T + 1) * s_
    for s_ in (3, 1000, 123457, (1 << 32) + 5):
        T = oracle.edge_threshold(oracle.WIC, 0.0, 0, 1, s_ - 1, 1)
        assert Fraction(T, 1 << 64) <= Fraction(2, s_) < Fraction(T + 1, 1 << 64)


def test_wic_live_fraction_on_stars():
    # star K_{1,d}: every edge has d_u + d_v = d + 1, so it is live with p = 2/(d+1);
    # with d = 1 (a single edge) always
    for d in (1, 3, 9):
        g = inputs.csr_from_pairs(d + 1, [(0, i) for i in range(1, d + 1)])
        R = 4000
        lab, siz = oracle.sketches(g, oracle.WIC, 0.0, 17, R)
        live = int((lab[:, 1:] == 0).sum())  # leaf i joined the center's component
        N = R * d
        pe = 2 / (d + 1)
        assert abs(live - N * pe) <= 5 * math.sqrt(N * pe * (1 - pe)) + 1e-9, d


# ---------------------------------------------------------------- greedy

@pytest.mark.parametrize("gi", range(6))
def test_greedy_matches_brute_force_and_bounds(gi):
    g = _tiny_graphs()[gi]
    R, p, seed = 6, 0.4, 5
    k = min(3, g.n)
    worlds = [brute.closure_labels(g.n, _live_edges(g, 0, p, seed, r))[2] for r in range(R)]
    lab, siz = oracle.sketches(g, 0, p, seed, R)
    seeds, gains = oracle.greedy(lab, siz, k)
    bs, bg = brute.brute_greedy(worlds, g.n, k)
    assert list(seeds) == bs and list(gains) == bg
    # gains non-increasing (submodularity), total = f(S_k) <= R*n
    assert all(gains[i] >= gains[i + 1] for i in range(k - 1))
    fk = sum(brute.spread_in_world(A, list(map(int, seeds))) for A in worlds)
    assert int(gains.sum()) == fk <= R * g.n
    # (1 - 1/e) guarantee of greedy against the exhaustive optimum
    assert fk >= (1 - 1 / math.e) * brute.best_k_subset(worlds, g.n, k) - 1e-9


def test_greedy_on_all_worlds_equals_exact_ic_spread():
    # With the sketch set = every live-edge world of a tiny graph at p = 1/2, the
    # coverage f(S) equals 2^m * sigma(S), sigma from the IC cascade definition.
    n = 6
    edges = [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (4, 5), (1, 5)]
    m = len(edges)
    labs, sizs = [], []
    for mask in range(1 << m):
        live = [e for i, e in enumerate(edges) if mask >> i & 1]
        l, s, _ = brute.closure_labels(n, live)
        labs.append(l)
        sizs.append(s)
    lab, siz = np.array(labs), np.array(sizs)
    k = 3
    seeds, gains = oracle.greedy(lab, siz, k)
    S = []
    prev = Fraction(0)
    for i in range(k):
        sig = {v: brute.exact_ic_spread(n, edges, Fraction(1, 2), S + [v]) for v in range(n) if v not in S}
        best = max(sig.values())
        want = min(v for v in sig if sig[v] == best)
        assert seeds[i] == want
        assert Fraction(int(gains[i]), 1 << m) == best - prev
        S.append(want)
        prev = best


def test_closed_form_p0_and_cliques():
    # p = 0: every CC is a singleton, so seeds are 0..k-1 with gain R each
    g = inputs.er_graph(200, 600, seed=4)
    lab, siz = oracle.sketches(g, 0, 0.0, 1, 8)
    seeds, gains = oracle.greedy(lab, siz, 5)
    assert list(seeds) == [0, 1, 2, 3, 4] and list(gains) == [8] * 5
    # p = 1 on disjoint cliques: components in decreasing size (ties -> smaller min id),
    # the seed is the component's smallest id, gain R*|C|; then zero gains, smallest unused ids
    comps = [[7, 8, 9], [0, 1], [2, 3, 4, 5, 6], [10, 11, 12], [13]]
    pairs = [(a, b) for c in comps for i, a in enumerate(c) for b in c[i + 1:]]
    g = inputs.csr_from_pairs(14, pairs)
    R = 4
    lab, siz = oracle.sketches(g, 0, 1.0, 9, R)
    seeds, gains = oracle.greedy(lab, siz, 8)
    assert list(seeds) == [2, 7, 10, 0, 13, 1, 3, 4]
    assert list(gains) == [5 * R, 3 * R, 3 * R, 2 * R, 1 * R, 0, 0, 0]


def test_celf_equals_plain_greedy():
    g = inputs.rmat_graph(11, 16 << 11, seed=3)
    lab, siz = oracle.sketches(g, 1, 0.0, 2, 16)
    s1, g1 = oracle.greedy(lab, siz, 12)
    s2, g2, ev = oracle.celf(lab, siz, 12)
    assert np.array_equal(s1, s2) and np.array_equal(g1, g2)
    assert ev.min() >= 1


def _celf_cases():
    with open(os.path.join(os.path.dirname(__file__), "golden", "celf_worked_examples.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _celf_cases(), ids=lambda c: c["name"])
def test_celf_worked_examples(case):
    # Algorithm 2 run by hand: with the queue in a total order (score, then smaller id)
    # every pop is determined, so each round's evaluation count is unique
    lab = np.array(case["labels"], dtype=np.uint32)
    siz = np.array(case["sizes"], dtype=np.uint32)
    s, g, ev = oracle.celf(lab, siz, case["k"])
    assert list(s) == case["seeds"] and list(g) == case["gains"] and list(ev) == case["evals"]
    s1, g1 = oracle.greedy(lab, siz, case["k"])
    assert list(s1) == case["seeds"] and list(g1) == case["gains"]


# ---------------------------------------------------------------- CompactSketch

def test_centers_are_hashed_bernoulli():
    n, seed = 20000, 3
    for alpha in (0.1, 0.5):
        c = oracle.centers(n, seed, alpha)
        assert np.all(np.diff(c.astype(np.int64)) > 0)
        K = brute.key_int(seed, oracle.SALT_CENTER)
        want = np.nonzero(brute.mix64_np(np.arange(n, dtype=np.uint64) ^ np.uint64(K))
                          < np.uint64(oracle.threshold(alpha)))[0]
        assert np.array_equal(c, want)
        assert abs(c.size - n * alpha) <= 5 * math.sqrt(n * alpha * (1 - alpha))
    assert np.array_equal(oracle.centers(50, 1, 1.0), np.arange(50))
    assert oracle.centers(50, 1, 0.0).size == 0


@pytest.mark.parametrize("gi", range(6))
def test_compact_triple_matches_definition(gi):
    g = _tiny_graphs()[gi]
    cents = oracle.centers(g.n, 5, 0.5)
    for r in range(5):
        edges = _live_edges(g, 0, 0.45, 5, r)
        _, _, A = brute.closure_labels(g.n, edges)
        lab, siz = oracle.sketch(g, 0, 0.45, 5, r)
        lc, sc = oracle.compact(lab, siz, cents)
        for i, c in enumerate(cents):
            j = min(jj for jj, cc in enumerate(cents) if A[c, cc])
            assert lc[i] == j
            assert sc[i] == (int(A[c].sum()) if j == i else 0)


@pytest.mark.parametrize("alpha", [0.05, 0.3, 1.0])
def test_compact_greedy_equals_full_greedy(alpha):
    # alpha-equivalence (Sec. 3): the GetCenter route reaches the full-label result
    g = inputs.rmat_graph(9, 8 << 9, seed=6)
    R, k, seed = 12, 8, 4
    lab, siz = oracle.sketches(g, 1, 0.0, seed, R)
    s_full, g_full = oracle.greedy(lab, siz, k)
    cents = oracle.centers(g.n, seed, alpha)
    lc, sc = oracle.compact_all(lab, siz, cents)
    s_c, g_c, _ = oracle.compact_greedy(g, 1, 0.0, seed, cents, lc, sc, k)
    assert np.array_equal(s_full, s_c) and np.array_equal(g_full, g_c)


def test_getcenter_cases_and_visit_bound():
    g = inputs.er_graph(3000, 9000, seed=8)
    p, seed, alpha = 0.3, 2, 0.1
    R = 4
    lab, siz = oracle.sketches(g, 0, p, seed, R)
    cents = oracle.centers(g.n, seed, alpha)
    lc, sc = oracle.compact_all(lab, siz, cents)
    in_s = np.zeros(g.n, dtype=np.uint8)
    tot_vis, calls = 0, 0
    for r in range(R):
        for v in range(0, g.n, 7):
            d, l, vis = oracle.getcenter(g, 0, p, seed, r, cents, lc[r], sc[r], in_s, v)
            assert d == siz[r, v]               # no seeds yet: influence = CC size
            has_center = bool(np.any(lab[r, cents] == lab[r, v]))
            assert (l != oracle.NONE) == has_center
            tot_vis += vis
            calls += 1
    # Theorem 3.1: expected visits per call <= min(1/alpha, T); allow sampling slack
    assert tot_vis / calls <= 1.5 / alpha
    # a seed in a center-less CC zeroes the gain of every vertex of that CC
    r = 0
    nocenter = [v for v in range(g.n) if siz[r, v] > 1 and not np.any(lab[r, cents] == lab[r, v])]
    if nocenter:
        v = nocenter[0]
        other = [w for w in range(g.n) if lab[r, w] == lab[r, v] and w != v][0]
        in_s[other] = 1
        d, l, _ = oracle.getcenter(g, 0, p, seed, r, cents, lc[r], sc[r], in_s, v)
        assert d == 0 and l == oracle.NONE


# ---------------------------------------------------------------- inputs

def test_generators_are_deterministic_and_simple():
    a = inputs.rmat_keys(12, 4000, 0.57, 0.19, 0.19, 5)
    b = inputs.rmat_keys(12, 4000, 0.57, 0.19, 0.19, 5)
    assert np.array_equal(a, b) and a.size == 4000
    assert np.all(np.diff(a.astype(np.int64)) > 0)
    g = inputs.csr_from_keys(1 << 12, a)
    off = g.offsets.astype(np.int64)
    rows = np.repeat(np.arange(g.n), np.diff(off))
    assert np.all(rows != g.cols)
    fwd = set(zip(rows.tolist(), g.cols.tolist()))
    assert all((v, u) in fwd for (u, v) in fwd)
    for u in range(g.n):
        seg = g.cols[off[u]:off[u + 1]]
        assert np.all(np.diff(seg.astype(np.int64)) > 0)
    c = inputs.chunglu_keys(5000, 12.0, 2.2, 9)
    assert 0 < c.size <= 30000
    e = inputs.er_keys(1000, 5000, 1)
    assert e.size == 5000


# ---------------------------------------------------------------- NextSeed by prefix doubling (Algorithm 4)

def _ptree_cases():
    with open(os.path.join(os.path.dirname(__file__), "golden", "ptree_worked_examples.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _ptree_cases(), ids=lambda c: c["name"])
def test_ptree_worked_examples(case):
    lab = np.array([case["labels"]], dtype=np.uint32)
    siz = np.array([case["sizes"]], dtype=np.uint32)
    s, g, ev = oracle.ptree(lab, siz, case["k"])
    assert list(s) == case["seeds"] and list(g) == case["gains"] and list(ev) == case["evals"]


@pytest.mark.parametrize("seed", [3, 4, 5, 6])
def test_ptree_selects_the_greedy_seeds_within_twice_celf(seed):
    # Theorem 4.1: the seed of every round is the plain greedy's (largest marginal
    # gain, smallest id on ties); Theorem 4.2: at most twice CELF's evaluations.
    g = inputs.rmat_graph(11, 16 << 11, seed=seed)
    lab, siz = oracle.sketches(g, 1, 0.0, seed, 16)
    k = 40
    s1, g1 = oracle.greedy(lab, siz, k)
    s2, g2, ev = oracle.ptree(lab, siz, k)
    _, _, ev_celf = oracle.celf(lab, siz, k)
    assert np.array_equal(s1, s2) and np.array_equal(g1, g2)
    assert int(ev.sum()) <= 2 * int(ev_celf.sum())
    assert ev[0] == 1 and ev_celf[0] == 1


def test_ptree_round_sizes_are_whole_doubling_prefixes():
    # a round takes whole batches 1, 2, 4, ..., so it evaluates 2^(j+1) - 1 vertices,
    # unless the queue ran out: then exactly every unselected vertex
    g = inputs.rmat_graph(10, 8 << 10, seed=9)
    lab, siz = oracle.sketches(g, 1, 0.0, 9, 8)
    n = g.n
    k = n
    s, gn, ev = oracle.ptree(lab, siz, k)
    s1, g1 = oracle.greedy(lab, siz, k)
    assert np.array_equal(s, s1) and np.array_equal(gn, g1)
    assert sorted(s.tolist()) == list(range(n))
    for i, e in enumerate(ev.tolist()):
        left = n - i
        assert e == left or (e & (e + 1)) == 0, (i, e, left)
        assert 1 <= e <= left


def test_ptree_ties_everywhere():
    # no live edge: every vertex scores R in every round, so each round evaluates only
    # the first entry of the queue and the seeds come out in id order
    g = inputs.rmat_graph(9, 4 << 9, seed=2)
    lab, siz = oracle.sketches(g, 0, 0.0, 1, 4)
    s, gn, ev = oracle.ptree(lab, siz, 20)
    assert list(s) == list(range(20)) and set(gn.tolist()) == {4} and set(ev.tolist()) == {1}


def test_ptree_matches_greedy_with_many_ties():
    # small R on small graphs: equal scores at the top of the queue are common, so a
    # wrong tie rule in s* or in the stop test shows up as a different seed order
    for seed in range(1, 13):
        g = inputs.rmat_graph(7, 3 << 7, seed=seed)
        for R in (1, 2, 3):
            lab, siz = oracle.sketches(g, 0, 0.3, seed, R)
            s, gn, _ = oracle.ptree(lab, siz, g.n)
            s1, g1 = oracle.greedy(lab, siz, g.n)
            assert np.array_equal(s, s1) and np.array_equal(gn, g1), (seed, R)


# ---------------------------------------------------------------- influence by simulation

@pytest.mark.parametrize("gi", range(6))
@pytest.mark.parametrize("kind,p", [(0, 0.35), (1, 0.0), (2, (0.2, 0.7)), (3, 0.0), (4, None)])
def test_influence_equals_reach_in_each_world(gi, kind, p):
    # simulation w is live-edge world w: the sum of the seeds' reach over the worlds,
    # with worlds spelled out from the published mixer and reach from closures
    g = _tiny_graphs()[gi]
    if kind == 4:
        p = brute.per_edge_p(g, gi)
    S = [0, g.n - 1, 0]
    sims, sseed = 40, 77
    want = 0
    for w in range(5, 5 + sims):
        A = brute.closure_labels(g.n, _live_edges(g, kind, p, sseed, w))[2]
        want += brute.spread_in_world(A, sorted(set(S)))
    assert oracle.influence(g, kind, p, S, sseed, 5, sims) == want


def test_influence_matches_the_cascade_in_expectation():
    # the IC cascade's exact expected spread (its definition, enumerated over coin
    # flips) against the simulation mean, within 5 standard errors
    n = 6
    edges = [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (4, 5), (1, 5)]
    g = inputs.csr_from_pairs(n, edges)
    deg = np.diff(g.offsets.astype(np.int64))
    sims = 20000
    cases = [(0, 0.5, None), (3, 0.0, {(min(u, v), max(u, v)): Fraction(2, int(deg[u] + deg[v])) for u, v in edges})]
    for kind, p, pe in cases:
        for S in ([0], [3, 5]):
            exact = brute.exact_ic_spread(n, edges, pe if pe is not None else Fraction(1, 2), S)
            est = Fraction(oracle.influence(g, kind, p, S, 123, 0, sims), sims)
            assert abs(float(est - exact)) <= 5 * (n / 2) / math.sqrt(sims), (kind, S, float(est), float(exact))


def test_influence_closed_forms():
    comps = [[0, 1, 2], [3, 4], [5]]
    g = inputs.csr_from_pairs(6, [(a, b) for c in comps for i, a in enumerate(c) for b in c[i + 1:]])
    assert oracle.influence(g, 0, 0.0, [1, 4, 1], 5, 0, 30) == 30 * 2      # p = 0: the distinct seeds
    assert oracle.influence(g, 0, 1.0, [1, 4, 1], 5, 0, 30) == 30 * 5      # p = 1: their components
    assert oracle.influence(g, 0, 1.0, [5], 5, 0, 7) == 7


def test_per_edge_model_reduces_to_constant_and_matches_cascade():
    # the same p on every entry is the Consistent model, sketch for sketch
    g = inputs.rmat_graph(9, 4 << 9, seed=12)
    const = np.full(g.cols.size, 0.13)
    la, sa = oracle.sketches(g, oracle.PER_EDGE, const, 5, 6)
    lb, sb = oracle.sketches(g, oracle.CONSTANT, 0.13, 5, 6)
    assert np.array_equal(la, lb) and np.array_equal(sa, sb)
    # per-edge probabilities against the cascade's exact expected spread
    n = 6
    edges = [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (4, 5), (1, 5)]
    t = inputs.csr_from_pairs(n, edges)
    pe = brute.per_edge_p(t, 3)
    rows = np.repeat(np.arange(n), np.diff(t.offsets.astype(np.int64)))
    exact_p = {(min(int(u), int(w)), max(int(u), int(w))): Fraction(float(x))
               for u, w, x in zip(rows, t.cols, pe)}
    sims = 20000
    for S in ([0], [2, 4]):
        exact = brute.exact_ic_spread(n, edges, exact_p, S)
        est = oracle.influence(t, oracle.PER_EDGE, pe, S, 321, 0, sims) / sims
        assert abs(est - float(exact)) <= 5 * (n / 2) / math.sqrt(sims), (S, est, float(exact))

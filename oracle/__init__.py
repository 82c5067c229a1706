"""The oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.

ctypes wrapper over ``pacim_oracle.c`` (built to ``liboracle.so`` here), the
plain single-threaded CPU statement of the sketch-based greedy influence
maximization of PaC-IM under the IC model on undirected graphs.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark import this
package; the GPU library and its Python binding never do.

Each wrapper names the passage it follows; the C file holds the readings of
points the paper leaves open.  ``sketches(..., threads=T)`` only spreads
independent calls of the single-threaded ``orc_sketch`` (one per sketch r) over
T host threads; the arithmetic is unchanged.
"""
from __future__ import annotations

import ctypes
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

NONE = 0xFFFFFFFF
ALL_LIVE = 0xFFFFFFFFFFFFFFFF
SALT_CENTER = 0xC000000000000001
SALT_TRIV = 0xC000000000000002
SALT_RANGE = 0xC000000000000003

# edge-probability models (kind): Consistent p, trivalency, Uniform U(lo, hi) per edge, WIC 2 / (d_u + d_v),
# per-edge p given for every CSR entry
CONSTANT, TRIVALENCY, RANGE, WIC, PER_EDGE = 0, 1, 2, 3, 4

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_dblp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"oracle not built: {_LIB_PATH} (run __graft_entry__.build())")
        lib = ctypes.CDLL(_LIB_PATH)
        u32, u64, dbl, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
        lib.orc_mix64.restype = u64
        lib.orc_mix64.argtypes = [u64]
        lib.orc_key.restype = u64
        lib.orc_key.argtypes = [u64, u64]
        lib.orc_threshold.restype = u64
        lib.orc_threshold.argtypes = [dbl]
        lib.orc_edge_threshold.restype = u64
        lib.orc_edge_threshold.argtypes = [i32, dbl, dbl, u32, u32, u64, u64]
        lib.orc_live.restype = i32
        lib.orc_live.argtypes = [u32, u32, u32, u64, u64]
        lib.orc_sketch.restype = ctypes.c_int64
        lib.orc_sketch.argtypes = [u32, _u64p, _u32p, i32, dbl, dbl, _dblp, u64, u32, _u32p, _u32p]
        lib.orc_marginals.restype = None
        lib.orc_marginals.argtypes = [u32, u32, _u32p, _u32p, _u8p, u32, u32, _u64p]
        lib.orc_cover.restype = None
        lib.orc_cover.argtypes = [u32, u32, _u32p, _u8p, u32]
        lib.orc_greedy.restype = i32
        lib.orc_greedy.argtypes = [u32, u32, _u32p, _u32p, u32, _u32p, _u64p]
        lib.orc_centers.restype = u32
        lib.orc_centers.argtypes = [u32, u64, dbl, _u32p]
        lib.orc_compact.restype = None
        lib.orc_compact.argtypes = [u32, u32, _u32p, _u32p, _u32p, _u32p, _u32p]
        lib.orc_getcenter.restype = u64
        lib.orc_getcenter.argtypes = [u32, _u64p, _u32p, i32, dbl, dbl, _dblp, u64, u32, _u32p, _u32p, _u32p, _u8p,
                                      u32, _u32p, _u8p, _u32p, _u64p]
        lib.orc_compact_greedy.restype = i32
        lib.orc_compact_greedy.argtypes = [u32, _u64p, _u32p, i32, dbl, dbl, _dblp, u64, u32, u32, _u32p, _u32p, _u32p,
                                           u32, _u32p, _u64p, _u64p]
        lib.orc_celf_evaluations.restype = i32
        lib.orc_celf_evaluations.argtypes = [u32, u32, _u32p, _u32p, u32, _u32p, _u64p, _u64p]
        lib.orc_influence.restype = u64
        lib.orc_influence.argtypes = [u32, _u64p, _u32p, i32, dbl, dbl, _dblp, _u32p, u32, u64, u32, u32]
        lib.orc_ptree.restype = i32
        lib.orc_ptree.argtypes = [u32, u32, _u32p, _u32p, u32, _u32p, _u64p, _u64p]
        _lib = lib
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def mix64(z: int) -> int:
    """SplitMix64 output function."""
    return int(_load().orc_mix64(z & ALL_LIVE))


def key(seed: int, x: int) -> int:
    return int(_load().orc_key(seed & ALL_LIVE, x & ALL_LIVE))


def threshold(p: float) -> int:
    return int(_load().orc_threshold(float(p)))


def _pp(p):
    """p of a model as (p, p_hi, p_edge): a float; (lo, hi) for the Uniform range model;
    or an array with one probability per CSR entry for the per-edge model (the
    array must outlive the call)."""
    if isinstance(p, np.ndarray):
        assert p.dtype == np.float64 and p.flags.c_contiguous
        return 0.0, 0.0, _p(p, _dblp)
    if isinstance(p, (tuple, list)):
        return float(p[0]), float(p[1]), None
    return float(p), 0.0, None


def edge_threshold(kind: int, p, u: int, v: int, du: int = 0, dv: int = 0) -> int:
    lo, hi, _ = _pp(p)
    return int(_load().orc_edge_threshold(kind, lo, hi, u, v, du, dv))


def live(u: int, v: int, r: int, seed: int, T: int) -> bool:
    """Sample(e, r) of Sec. 3."""
    return bool(_load().orc_live(u, v, r, seed & ALL_LIVE, T & ALL_LIVE))


def sketch(g, kind: int, p: float, seed: int, r: int):
    """Sketch(r) with full labels: (label[n], size[n]) by BFS."""
    lab = np.empty(max(g.n, 1), dtype=np.uint32)
    siz = np.empty(max(g.n, 1), dtype=np.uint32)
    _load().orc_sketch(g.n, _p(g.offsets, _u64p), _p(g.cols, _u32p), kind, *_pp(p), seed & ALL_LIVE, r,
                       _p(lab, _u32p), _p(siz, _u32p))
    return lab[: g.n], siz[: g.n]


def sketches(g, kind: int, p: float, seed: int, R: int, threads: int = 1, rs=None):
    """Full labels and sizes for sketches rs (default 0..R-1): arrays [len(rs)][n]."""
    rs = list(range(R)) if rs is None else list(rs)
    lab = np.empty((len(rs), max(g.n, 1)), dtype=np.uint32)
    siz = np.empty((len(rs), max(g.n, 1)), dtype=np.uint32)
    lib = _load()

    def one(i):
        lib.orc_sketch(g.n, _p(g.offsets, _u64p), _p(g.cols, _u32p), kind, *_pp(p), seed & ALL_LIVE, rs[i],
                       _p(lab[i], _u32p), _p(siz[i], _u32p))

    if threads <= 1:
        for i in range(len(rs)):
            one(i)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, range(len(rs))))
    return lab[:, : g.n], siz[:, : g.n]


def greedy(label: np.ndarray, size: np.ndarray, k: int):
    """Plain greedy (full recomputation each round, smallest id on ties)."""
    R, n = label.shape
    label = np.ascontiguousarray(label, dtype=np.uint32)
    size = np.ascontiguousarray(size, dtype=np.uint32)
    seeds = np.empty(max(k, 1), dtype=np.uint32)
    gains = np.empty(max(k, 1), dtype=np.uint64)
    rc = _load().orc_greedy(n, R, _p(label, _u32p), _p(size, _u32p), k, _p(seeds, _u32p), _p(gains, _u64p))
    if rc != 0:
        raise ValueError("k > n")
    return seeds[:k], gains[:k]


class Coverage:
    """Covered-CC state of the full-label greedy, for range-parallel checks of big cases."""

    def __init__(self, label: np.ndarray, size: np.ndarray):
        self.label = np.ascontiguousarray(label, dtype=np.uint32)
        self.size = np.ascontiguousarray(size, dtype=np.uint32)
        self.R, self.n = self.label.shape
        self.covered = np.zeros(self.R * self.n + 1, dtype=np.uint8)

    def marginals(self, lo: int, hi: int) -> np.ndarray:
        out = np.empty(max(hi - lo, 1), dtype=np.uint64)
        _load().orc_marginals(self.n, self.R, _p(self.label, _u32p), _p(self.size, _u32p),
                              _p(self.covered, _u8p), lo, hi, _p(out, _u64p))
        return out[: hi - lo]

    def all_marginals(self, threads: int = 1) -> np.ndarray:
        if threads <= 1:
            return self.marginals(0, self.n)
        step = (self.n + threads - 1) // threads
        parts = [(lo, min(self.n, lo + step)) for lo in range(0, self.n, step)]
        with ThreadPoolExecutor(threads) as ex:
            res = list(ex.map(lambda ab: self.marginals(*ab), parts))
        return np.concatenate(res)

    def cover(self, s: int):
        _load().orc_cover(self.n, self.R, _p(self.label, _u32p), _p(self.covered, _u8p), s)


def centers(n: int, seed: int, alpha: float) -> np.ndarray:
    lib = _load()
    rho = lib.orc_centers(n, seed & ALL_LIVE, float(alpha), None)
    c = np.empty(max(rho, 1), dtype=np.uint32)
    lib.orc_centers(n, seed & ALL_LIVE, float(alpha), _p(c, _u32p))
    return c[:rho]


def compact(label_r: np.ndarray, size_r: np.ndarray, cents: np.ndarray):
    """Sketch triple of one sketch from its full labels: (label_c[rho], size_c[rho])."""
    n = label_r.size
    rho = cents.size
    label_r = np.ascontiguousarray(label_r, dtype=np.uint32)
    size_r = np.ascontiguousarray(size_r, dtype=np.uint32)
    cents = np.ascontiguousarray(cents, dtype=np.uint32)
    lc = np.empty(max(rho, 1), dtype=np.uint32)
    sc = np.empty(max(rho, 1), dtype=np.uint32)
    _load().orc_compact(n, rho, _p(cents, _u32p), _p(label_r, _u32p), _p(size_r, _u32p), _p(lc, _u32p),
                        _p(sc, _u32p))
    return lc[:rho], sc[:rho]


def compact_all(label: np.ndarray, size: np.ndarray, cents: np.ndarray):
    R = label.shape[0]
    rho = cents.size
    lc = np.empty((R, rho), dtype=np.uint32)
    sc = np.empty((R, rho), dtype=np.uint32)
    for r in range(R):
        lc[r], sc[r] = compact(label[r], size[r], cents)
    return lc, sc


def compact_greedy(g, kind: int, p: float, seed: int, cents: np.ndarray, label_c: np.ndarray,
                   size_c: np.ndarray, k: int):
    """Algorithm 1 with Sec. 3's GetCenter-based Marginal and MarkSeed.
    Returns (seeds, gains, total vertices dequeued by GetCenter)."""
    R, rho = label_c.shape
    cents = np.ascontiguousarray(cents, dtype=np.uint32)
    lc = np.ascontiguousarray(label_c, dtype=np.uint32)
    sc = np.array(size_c, dtype=np.uint32, copy=True, order="C")
    seeds = np.empty(max(k, 1), dtype=np.uint32)
    gains = np.empty(max(k, 1), dtype=np.uint64)
    visits = np.zeros(1, dtype=np.uint64)
    rc = _load().orc_compact_greedy(g.n, _p(g.offsets, _u64p), _p(g.cols, _u32p), kind, *_pp(p),
                                    seed & ALL_LIVE, R, rho, _p(cents, _u32p), _p(lc, _u32p), _p(sc, _u32p), k,
                                    _p(seeds, _u32p), _p(gains, _u64p), _p(visits, _u64p))
    if rc != 0:
        raise ValueError("k > n")
    return seeds[:k], gains[:k], int(visits[0])


def getcenter(g, kind, p, seed, r, cents, label_c_r, size_c_r, in_s, v):
    """One GetCenter(Phi_r, v, S) call: (delta, label or NONE, vertices dequeued)."""
    n = g.n
    rank = np.full(max(n, 1), NONE, dtype=np.uint32)
    rank[cents] = np.arange(cents.size, dtype=np.uint32)
    seen = np.zeros(n + 1, dtype=np.uint8)
    queue = np.empty(max(n, 1), dtype=np.uint32)
    l = np.zeros(1, dtype=np.uint32)
    vis = np.zeros(1, dtype=np.uint64)
    ins = np.ascontiguousarray(in_s, dtype=np.uint8)
    lc = np.ascontiguousarray(label_c_r, dtype=np.uint32)
    sc = np.ascontiguousarray(size_c_r, dtype=np.uint32)
    d = _load().orc_getcenter(n, _p(g.offsets, _u64p), _p(g.cols, _u32p), kind, *_pp(p), seed & ALL_LIVE, r,
                              _p(rank, _u32p), _p(lc, _u32p), _p(sc, _u32p), _p(ins, _u8p), v, _p(l, _u32p),
                              _p(seen, _u8p), _p(queue, _u32p), _p(vis, _u64p))
    return int(d), int(l[0]), int(vis[0])


def celf(label: np.ndarray, size: np.ndarray, k: int):
    """Sequential CELF (Algorithm 2): (seeds, gains, evaluations per round)."""
    R, n = label.shape
    label = np.ascontiguousarray(label, dtype=np.uint32)
    size = np.ascontiguousarray(size, dtype=np.uint32)
    seeds = np.empty(max(k, 1), dtype=np.uint32)
    gains = np.empty(max(k, 1), dtype=np.uint64)
    ev = np.empty(max(k, 1), dtype=np.uint64)
    rc = _load().orc_celf_evaluations(n, R, _p(label, _u32p), _p(size, _u32p), k, _p(seeds, _u32p),
                                      _p(gains, _u64p), _p(ev, _u64p))
    if rc != 0:
        raise ValueError("bad k")
    return seeds[:k], gains[:k], ev[:k]


def ptree(label: np.ndarray, size: np.ndarray, k: int):
    """NextSeed by prefix doubling over a totally ordered queue (Algorithm 4, Sec. 4):
    (seeds, gains, evaluations per round)."""
    R, n = label.shape
    label = np.ascontiguousarray(label, dtype=np.uint32)
    size = np.ascontiguousarray(size, dtype=np.uint32)
    seeds = np.empty(max(k, 1), dtype=np.uint32)
    gains = np.empty(max(k, 1), dtype=np.uint64)
    ev = np.empty(max(k, 1), dtype=np.uint64)
    rc = _load().orc_ptree(n, R, _p(label, _u32p), _p(size, _u32p), k, _p(seeds, _u32p), _p(gains, _u64p),
                           _p(ev, _u64p))
    if rc != 0:
        raise ValueError("bad k")
    return seeds[:k], gains[:k], ev[:k]


def influence(g, kind: int, p, seeds, sim_seed: int, w0: int, sims: int, threads: int = 1) -> int:
    """Sum over simulations w in [w0, w0 + sims) of the vertices the IC cascade from
    `seeds` activates in live-edge world w (worlds keyed like sketches, under
    sim_seed).  ``threads`` only splits the world range over host threads."""
    seeds = np.ascontiguousarray(seeds, dtype=np.uint32)
    lib = _load()

    def part(ab):
        a, b = ab
        return int(lib.orc_influence(g.n, _p(g.offsets, _u64p), _p(g.cols, _u32p), kind, *_pp(p),
                                     _p(seeds, _u32p), seeds.size, sim_seed & ALL_LIVE, a, b - a))
    if threads <= 1 or sims < 2:
        return part((w0, w0 + sims))
    step = (sims + threads - 1) // threads
    parts = [(a, min(w0 + sims, a + step)) for a in range(w0, w0 + sims, step)]
    with ThreadPoolExecutor(threads) as ex:
        return sum(ex.map(part, parts))


def select_seeds(g, kind: int, p: float, R: int, k: int, seed: int, threads: int = 1):
    """The whole path on the CPU: R full sketches, then the plain greedy."""
    lab, siz = sketches(g, kind, p, seed, R, threads=threads)
    return greedy(lab, siz, k)

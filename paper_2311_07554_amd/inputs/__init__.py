"""Seeded synthetic inputs shared by the library's tests, its benchmark and the oracle.

Nothing here computes any part of the influence-maximization method: the module
only builds simple undirected graphs (symmetric CSR, no self-loops, no duplicate
pairs) and the workload descriptions that go with them.  The generators are in
``graphgen.c`` (compiled to ``libpacim_gen.so`` next to this file).

Workloads, shaped like the paper's inputs (Sec. 5: social and web graphs with
IC p = 0.02, R = 256 sketches, k = 100 seeds):

* ``er_small``      Erdos-Renyi, n = 1,000, 5,000 pairs (avg degree 10), uniform p = 0.05,
                    R = 64, k = 10, full labels.
* ``rmat20``        R-MAT scale 20 (2^20 vertices), 2^24 undirected pairs, a=0.57 b=c=0.19,
                    trivalency p in {0.1, 0.01, 0.001}, R = 256, k = 100, full and compact.
* ``rmat24``        R-MAT scale 24, 2^28 pairs, uniform p = 0.02, R = 256, k = 200,
                    CompactSketch with alpha = 0.1.
* ``batched``       64 Chung-Lu power-law graphs (exponent 2.2), n log-uniform in
                    [2^12, 2^18], avg degree U[8, 32], p U[0.01, 0.1], R = 128, k = 50.
* ``serving``       16 resident R-MAT graphs (scales 16..22, avg degree 16) and a Poisson
                    stream of queries with p in {0.01, 0.02, 0.05}, R in {64, 256},
                    k in {10, 50, 100}.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libpacim_gen.so")
_lib = None

PROB_UNIFORM = 0
PROB_TRIVALENCY = 1
PROB_RANGE = 2
PROB_WIC = 3


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"graph generator library not built: {_LIB_PATH} (run __graft_entry__.build())")
        lib = ctypes.CDLL(_LIB_PATH)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.gg_er.restype = ctypes.c_int64
        lib.gg_er.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, u64p, ctypes.c_uint64]
        lib.gg_rmat.restype = ctypes.c_int64
        lib.gg_rmat.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_uint64, ctypes.c_int, u64p, ctypes.c_uint64]
        lib.gg_chunglu.restype = ctypes.c_int64
        lib.gg_chunglu.argtypes = [ctypes.c_uint32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                   u64p, ctypes.c_uint64]
        lib.gg_csr_from_keys.restype = ctypes.c_int
        lib.gg_csr_from_keys.argtypes = [ctypes.c_uint32, u64p, ctypes.c_uint64, u64p, u32p]
        _lib = lib
    return _lib


def _p64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def er_keys(n: int, m: int, seed: int) -> np.ndarray:
    keys = np.empty(max(m, 1), dtype=np.uint64)
    got = _load().gg_er(n, m, seed, _p64(keys), keys.size)
    if got != m:
        raise ValueError(f"gg_er failed ({got})")
    return keys[:m]


def rmat_keys(scale: int, m: int, a: float, b: float, c: float, seed: int, permute: bool = True) -> np.ndarray:
    keys = np.empty(max(m, 1), dtype=np.uint64)
    got = _load().gg_rmat(scale, m, a, b, c, seed, int(permute), _p64(keys), keys.size)
    if got != m:
        raise ValueError(f"gg_rmat failed ({got})")
    return keys[:m]


def chunglu_keys(n: int, avg_deg: float, gamma: float, seed: int) -> np.ndarray:
    cap = max(int(n * avg_deg / 2.0) + 1, 1)
    keys = np.empty(cap, dtype=np.uint64)
    got = _load().gg_chunglu(n, avg_deg, gamma, seed, _p64(keys), cap)
    if got < 0:
        raise ValueError(f"gg_chunglu failed ({got})")
    return keys[:got]


@dataclass
class Graph:
    """A simple undirected graph as a symmetric CSR."""
    n: int
    offsets: np.ndarray  # uint64[n+1]
    cols: np.ndarray     # uint32[2m]
    name: str = ""

    @property
    def m_dir(self) -> int:
        return int(self.cols.size)

    @property
    def m_und(self) -> int:
        return int(self.cols.size) // 2


def csr_from_keys(n: int, keys: np.ndarray, name: str = "") -> Graph:
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    offsets = np.empty(n + 1, dtype=np.uint64)
    cols = np.empty(max(2 * keys.size, 1), dtype=np.uint32)
    rc = _load().gg_csr_from_keys(n, _p64(keys), keys.size, _p64(offsets), _p32(cols))
    if rc != 0:
        raise ValueError("invalid edge keys")
    return Graph(n=n, offsets=offsets, cols=cols[: 2 * keys.size], name=name)


def csr_from_pairs(n: int, pairs) -> Graph:
    """Small hand-written graphs: pairs is an iterable of (u, v), u != v."""
    ks = sorted({(min(u, v) << 32) | max(u, v) for (u, v) in pairs if u != v})
    return csr_from_keys(n, np.array(ks, dtype=np.uint64))


def er_graph(n: int, m: int, seed: int) -> Graph:
    return csr_from_keys(n, er_keys(n, m, seed), name=f"er_n{n}_m{m}_s{seed}")


def rmat_graph(scale: int, m: int, seed: int, a=0.57, b=0.19, c=0.19) -> Graph:
    return csr_from_keys(1 << scale, rmat_keys(scale, m, a, b, c, seed), name=f"rmat{scale}_m{m}_s{seed}")


def chunglu_graph(n: int, avg_deg: float, gamma: float, seed: int) -> Graph:
    return csr_from_keys(n, chunglu_keys(n, avg_deg, gamma, seed), name=f"cl_n{n}_d{avg_deg:.2f}_s{seed}")


@dataclass
class Query:
    """One influence-maximization request: graph, probability model, R, k, seed, alpha."""
    graph: Graph
    prob_kind: int
    p: float
    R: int
    k: int
    seed: int = 1
    alpha: float = 1.0
    tag: str = ""


@dataclass
class Workload:
    name: str
    queries: list = field(default_factory=list)
    note: str = ""


# --- SplitMix64 stream for workload parameters (independent of the method's hash use) ---
_PHI = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def _mix(z: int) -> int:
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


class _Stream:
    def __init__(self, seed: int):
        self.state = seed & _M64

    def next(self) -> int:
        self.state = (self.state + _PHI) & _M64
        return _mix(self.state)

    def unit(self) -> float:
        return (self.next() >> 11) * (1.0 / 9007199254740992.0)


def er_small(R: int = 64, k: int = 10) -> Workload:
    g = er_graph(1000, 5000, seed=1)
    return Workload("er_small", [Query(g, PROB_UNIFORM, 0.05, R, k, seed=1, alpha=1.0, tag="er_small")],
                    note="Erdos-Renyi n=1000, 5000 pairs, uniform p=0.05, R=64, k=10, full labels")


def rmat20(R: int = 256, k: int = 100, alpha: float = 1.0, scale: int = 20, seed: int = 2) -> Workload:
    m = 16 << scale
    g = rmat_graph(scale, m, seed=seed)
    return Workload(f"rmat{scale}", [Query(g, PROB_TRIVALENCY, 0.0, R, k, seed=1, alpha=alpha,
                                          tag=f"rmat{scale}_trivalency")],
                    note=f"R-MAT scale {scale}, {m} pairs, trivalency, R={R}, k={k}, alpha={alpha}")


def rmat24(R: int = 256, k: int = 200, alpha: float = 0.1, scale: int = 24, seed: int = 3) -> Workload:
    m = 16 << scale
    g = rmat_graph(scale, m, seed=seed)
    return Workload(f"rmat{scale}", [Query(g, PROB_UNIFORM, 0.02, R, k, seed=1, alpha=alpha,
                                          tag=f"rmat{scale}_p0.02")],
                    note=f"R-MAT scale {scale}, {m} pairs, uniform p=0.02, R={R}, k={k}, alpha={alpha}")


def batched(count: int = 64, R: int = 128, k: int = 50, seed: int = 4, max_log2n: int = 18,
            min_log2n: int = 12) -> Workload:
    s = _Stream(seed)
    qs = []
    for q in range(count):
        n = int(round(2.0 ** (min_log2n + (max_log2n - min_log2n) * s.unit())))
        d = 8.0 + 24.0 * s.unit()
        p = 0.01 + 0.09 * s.unit()
        gseed = s.next()
        g = chunglu_graph(n, d, 2.2, gseed)
        qs.append(Query(g, PROB_UNIFORM, p, R, min(k, n), seed=q + 1, alpha=1.0, tag=f"cl{q}"))
    return Workload("batched", qs, note=f"{count} Chung-Lu graphs, gamma 2.2, R={R}, k={k}")


SERVING_SCALES = (16, 16, 17, 17, 18, 18, 18, 19, 19, 20, 20, 20, 21, 21, 22, 22)


def serving_graphs(scales=SERVING_SCALES, seed: int = 5):
    return [rmat_graph(sc, 8 << sc, seed=seed * 1000 + i) for i, sc in enumerate(scales)]


def serving_queries(num_graphs: int, count: int = 2000, seed: int = 5):
    """(graph index, p, R, k, sample seed) for each request, drawn from one stream."""
    s = _Stream(seed ^ 0x5EED)
    out = []
    for i in range(count):
        gi = s.next() % num_graphs
        p = (0.01, 0.02, 0.05)[s.next() % 3]
        R = (64, 256)[s.next() % 2]
        k = (10, 50, 100)[s.next() % 3]
        out.append((int(gi), p, R, k, i + 1))
    return out


def poisson_arrivals(count: int, qps: float, seed: int = 5):
    """Arrival times (seconds from start) of a Poisson stream at rate qps."""
    s = _Stream(seed ^ 0xA77)
    t, out = 0.0, []
    for _ in range(count):
        u = s.unit()
        t += -math.log(1.0 - u) / qps
        out.append(t)
    return out


# The served mix of the serving parity test: the first seven graphs of the serving
# workload (R-MAT scales 16, 16, 17, 17, 18, 18, 18), requests with their own
# sampling seeds and label kinds.  Seeds repeat across requests so that sketch sets
# are shared, and two requests differ only in their Uniform-model interval.
SERVING_MIX_GRAPHS = 7


def serving_mix(count: int = 24, seed: int = 55):
    """(graph index, model kind, p, p_hi, R, k, sampling seed, alpha) per request."""
    s = _Stream(seed)
    out = []
    for i in range(count):
        gi = s.next() % SERVING_MIX_GRAPHS
        p = (0.01, 0.02, 0.05)[s.next() % 3]
        R = (64, 256)[s.next() % 2]
        k = (10, 50, 100)[s.next() % 3]
        sseed = (5, 6, 7 + i)[s.next() % 3]
        alpha = (1.0, 0.1)[s.next() % 2]
        out.append((int(gi), PROB_UNIFORM, p, 0.0, R, k, sseed, alpha))
    # the same graph, R and seed under two Uniform U(lo, hi) intervals, and again under the first
    out.append((4, PROB_RANGE, 0.0, 0.05, 64, 50, 9, 1.0))
    out.append((4, PROB_RANGE, 0.02, 0.1, 64, 50, 9, 1.0))
    out.append((4, PROB_RANGE, 0.0, 0.05, 64, 10, 9, 0.1))
    out.append((4, PROB_UNIFORM, 0.05, 0.0, 64, 50, 9, 1.0))
    return out

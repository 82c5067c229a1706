"""Thin ctypes binding of ``libpacim.so`` (the C-ABI declared in include/pacim.h).

Argument marshalling only: every step of the influence-maximization path runs in
the library's HIP kernels.  The module-level ``im_*`` functions mirror the C
entry points one to one; ``Context``, ``Graph`` and ``Sketches`` wrap them with
numpy / torch arguments.  torch, when given, only supplies device memory and the
HIP stream.

The binding refuses to work without the compiled library: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpacim.so")

IM_OK, IM_EINVAL, IM_ENOMEM, IM_EDEVICE, IM_EBUSY, IM_EINTERNAL = range(6)
IM_PROB_UNIFORM, IM_PROB_TRIVALENCY, IM_PROB_RANGE, IM_PROB_WIC, IM_PROB_PER_EDGE = 0, 1, 2, 3, 4
_STATUS = {0: "IM_OK", 1: "IM_EINVAL", 2: "IM_ENOMEM", 3: "IM_EDEVICE", 4: "IM_EBUSY", 5: "IM_EINTERNAL"}


class ImError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class im_prob(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("p", ctypes.c_double), ("p_hi", ctypes.c_double),
                ("p_edge", ctypes.c_void_p)]


class im_sketch_stats(ctypes.Structure):
    _fields_ = [("seeds_chosen", ctypes.c_uint32), ("rho", ctypes.c_uint32), ("evaluations", ctypes.c_uint64),
                ("bfs_overflow", ctypes.c_uint64), ("bfs_visits", ctypes.c_uint64), ("build_ms", ctypes.c_double),
                ("select_ms", ctypes.c_double),
                ("sketches_per_pass", ctypes.c_uint32), ("sketch_bytes", ctypes.c_uint64),
                ("bulk_rounds", ctypes.c_uint32), ("bulk_resampled", ctypes.c_uint32)]


_vp = ctypes.c_void_p
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


class im_query(ctypes.Structure):
    _fields_ = [("graph", _vp), ("prob", im_prob), ("R", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("alpha", ctypes.c_double)]


class im_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_active", ctypes.c_uint32), ("rounds_per_step", ctypes.c_uint32),
                ("max_R", ctypes.c_uint32), ("max_k", ctypes.c_uint32), ("compact_budget", ctypes.c_size_t)]


class im_server_counters(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("steps", ctypes.c_uint64),
                ("builds", ctypes.c_uint64), ("cache_hits", ctypes.c_uint64), ("evictions", ctypes.c_uint64),
                ("compact_completed", ctypes.c_uint64), ("bytes_in_use", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t), ("cached_sets", ctypes.c_uint32),
                ("admit_ms", ctypes.c_double), ("build_wait_ms", ctypes.c_double), ("step_ms", ctypes.c_double),
                ("busy_steps_ms", ctypes.c_double)]


class im_batch_config(ctypes.Structure):
    _fields_ = [("hook_block", ctypes.c_uint32), ("hook_grid", ctypes.c_uint32), ("select_block", ctypes.c_uint32),
                ("select_grid", ctypes.c_uint32)]

# name -> (restype, argtypes); the names and order follow include/pacim.h
_SIGS = {
    "im_ctx_create": (ctypes.c_int, [ctypes.c_int, _vp, ctypes.c_size_t, ctypes.POINTER(_vp)]),
    "im_ctx_destroy": (ctypes.c_int, [_vp]),
    "im_last_error": (ctypes.c_char_p, [_vp]),
    "im_ctx_memory": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "im_ctx_set_profiling": (ctypes.c_int, [_vp, ctypes.c_int]),
    "im_kernel_time": (ctypes.c_int, [_vp, ctypes.c_char_p, _u64p, ctypes.POINTER(ctypes.c_double)]),
    "im_graph_upload": (ctypes.c_int, [_vp, ctypes.c_uint32, ctypes.c_uint64, _vp, _vp, ctypes.c_int,
                                       ctypes.POINTER(_vp)]),
    "im_graph_free": (ctypes.c_int, [_vp]),
    "im_build_sketches": (ctypes.c_int, [_vp, _vp, im_prob, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double,
                                         ctypes.POINTER(_vp)]),
    "im_sketches_free": (ctypes.c_int, [_vp]),
    "im_select_seeds_from": (ctypes.c_int, [_vp, _vp, ctypes.c_uint32, _u32p, _u64p]),
    "im_select_seeds_ptree": (ctypes.c_int, [_vp, _vp, ctypes.c_uint32, _u32p, _u64p]),
    "im_influence": (ctypes.c_int, [_vp, _vp, im_prob, _u32p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
                                    ctypes.c_uint32, _u64p]),
    "im_influence_noalloc": (ctypes.c_int, [_vp, _vp, im_prob, _u32p, ctypes.c_uint32, ctypes.c_uint64,
                                            ctypes.c_uint32, ctypes.c_uint32, _u64p]),
    "im_influence_static_scratch": (ctypes.c_int, [ctypes.POINTER(ctypes.c_size_t)]),
    "im_select_seeds": (ctypes.c_int, [_vp, _vp, im_prob, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                       _u32p, _u64p]),
    "im_sketches_dump": (ctypes.c_int, [_vp, _vp, ctypes.c_uint32, _u32p, _u32p]),
    "im_centers": (ctypes.c_int, [_vp, _vp, _u32p, _u32p]),
    "im_initial_gains": (ctypes.c_int, [_vp, _vp, _u64p]),
    "im_sketches_stats": (ctypes.c_int, [_vp, ctypes.POINTER(im_sketch_stats)]),
    "im_select_trace": (ctypes.c_int, [_vp, _vp, _u32p, ctypes.c_uint32]),
    "im_probe_device": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "im_probe_random": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double)]),
    "im_server_create": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.c_uint32, ctypes.POINTER(im_server_config),
                                        ctypes.POINTER(_vp)]),
    "im_server_submit": (ctypes.c_int, [_vp, ctypes.POINTER(im_query), ctypes.POINTER(ctypes.c_uint64)]),
    "im_server_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]),
    "im_server_wait": (ctypes.c_int, [_vp, ctypes.c_uint64, _u32p, _u64p, ctypes.POINTER(ctypes.c_double)]),
    "im_server_stats": (ctypes.c_int, [_vp, ctypes.POINTER(im_server_counters)]),
    "im_server_destroy": (ctypes.c_int, [_vp]),
    "im_select_seeds_batched": (ctypes.c_int, [_vp, ctypes.c_uint32, ctypes.POINTER(im_query),
                                               ctypes.POINTER(im_batch_config), ctypes.POINTER(_u32p),
                                               ctypes.POINTER(_u64p), ctypes.POINTER(ctypes.c_double)]),
}

_lib = None


def load():
    """The compiled library; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} -- run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_symbols():
    lib = load()
    return [n for n in _SIGS if hasattr(lib, n)]


def _u32(a):
    return a.ctypes.data_as(_u32p)


def _u64(a):
    return a.ctypes.data_as(_u64p)


# ---- module-level mirrors of the C entry points --------------------------------

def im_ctx_create(device: int = 0, hip_stream: int | None = None, hbm_cap: int = 0) -> int:
    h = _vp()
    rc = load().im_ctx_create(device, hip_stream, hbm_cap, ctypes.byref(h))
    if rc != IM_OK:
        raise ImError(rc, "im_ctx_create failed (no usable HIP device?)")
    return h.value


def im_last_error(ctx) -> str:
    s = load().im_last_error(ctx)
    return s.decode() if s else ""


def _check(ctx, rc):
    if rc != IM_OK:
        raise ImError(rc, im_last_error(ctx))


def im_ctx_destroy(ctx):
    _check(ctx, load().im_ctx_destroy(ctx))


def im_ctx_memory(ctx):
    used, cap = ctypes.c_size_t(), ctypes.c_size_t()
    _check(ctx, load().im_ctx_memory(ctx, ctypes.byref(used), ctypes.byref(cap)))
    return used.value, cap.value


def im_ctx_set_profiling(ctx, on: bool):
    _check(ctx, load().im_ctx_set_profiling(ctx, int(bool(on))))


def im_kernel_time(ctx, name: str):
    n, ms = ctypes.c_uint64(), ctypes.c_double()
    _check(ctx, load().im_kernel_time(ctx, name.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def im_graph_upload(ctx, n: int, offsets, cols) -> int:
    """offsets/cols: numpy arrays (host) or torch tensors (device or host)."""
    dev = 0
    if hasattr(offsets, "data_ptr"):
        dev = int(offsets.is_cuda)
        po, pc = offsets.data_ptr(), cols.data_ptr()
        m_dir = int(cols.numel())
        keep = (offsets, cols)
    else:
        offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        cols = np.ascontiguousarray(cols, dtype=np.uint32)
        po, pc = offsets.ctypes.data, cols.ctypes.data
        m_dir = int(cols.size)
        keep = (offsets, cols)
    h = _vp()
    _check(ctx, load().im_graph_upload(ctx, n, m_dir, po, pc if m_dir else None, dev, ctypes.byref(h)))
    del keep
    return h.value


def im_graph_free(g):
    rc = load().im_graph_free(g)
    if rc != IM_OK:
        raise ImError(rc, "im_graph_free")


def _prob(kind: int, p):
    """p: a float; (lo, hi) for IM_PROB_RANGE; a float64 array with one probability per
    CSR entry for IM_PROB_PER_EDGE (the caller keeps it alive for the call)."""
    if isinstance(p, np.ndarray):
        if p.dtype != np.float64 or not p.flags.c_contiguous:
            raise ValueError("per-edge probabilities must be a contiguous float64 array")
        return im_prob(int(kind), 0.0, 0.0, p.ctypes.data)
    if isinstance(p, (tuple, list)):
        return im_prob(int(kind), float(p[0]), float(p[1]), None)
    return im_prob(int(kind), float(p), 0.0, None)


def im_build_sketches(ctx, g, kind: int, p: float, R: int, seed: int, alpha: float = 1.0) -> int:
    h = _vp()
    _check(ctx, load().im_build_sketches(ctx, g, _prob(kind, p), R, seed & ((1 << 64) - 1), float(alpha),
                                         ctypes.byref(h)))
    return h.value


def im_sketches_free(s):
    rc = load().im_sketches_free(s)
    if rc != IM_OK:
        raise ImError(rc, "im_sketches_free")


def im_select_seeds_from(ctx, s, k: int):
    seeds = np.empty(max(k, 1), dtype=np.uint32)
    gains = np.empty(max(k, 1), dtype=np.uint64)
    _check(ctx, load().im_select_seeds_from(ctx, s, k, _u32(seeds), _u64(gains)))
    return seeds[:k], gains[:k]


def im_select_seeds_ptree(ctx, s, k: int):
    seeds = np.empty(max(k, 1), dtype=np.uint32)
    gains = np.empty(max(k, 1), dtype=np.uint64)
    _check(ctx, load().im_select_seeds_ptree(ctx, s, k, _u32(seeds), _u64(gains)))
    return seeds[:k], gains[:k]


def im_influence(ctx, g, kind: int, p, seeds, sim_seed: int, w0: int, sims: int) -> int:
    sd = np.ascontiguousarray(seeds, dtype=np.uint32)
    tot = np.zeros(1, dtype=np.uint64)
    _check(ctx, load().im_influence(ctx, g, _prob(kind, p), _u32(sd if sd.size else np.zeros(1, np.uint32)),
                                    int(sd.size), sim_seed & ((1 << 64) - 1), int(w0), int(sims), _u64(tot)))
    return int(tot[0])


def im_influence_noalloc(ctx, g, kind: int, p, seeds, sim_seed: int, w0: int, sims: int) -> int:
    sd = np.ascontiguousarray(seeds, dtype=np.uint32)
    tot = np.zeros(1, dtype=np.uint64)
    _check(ctx, load().im_influence_noalloc(ctx, g, _prob(kind, p), _u32(sd if sd.size else np.zeros(1, np.uint32)),
                                            int(sd.size), sim_seed & ((1 << 64) - 1), int(w0), int(sims),
                                            _u64(tot)))
    return int(tot[0])


def im_influence_static_scratch() -> int:
    v = ctypes.c_size_t(0)
    rc = load().im_influence_static_scratch(ctypes.byref(v))
    if rc != IM_OK:
        raise ImError(rc, "im_influence_static_scratch")
    return int(v.value)


def im_select_seeds(ctx, g, kind: int, p: float, R: int, k: int, seed: int):
    seeds = np.empty(max(k, 1), dtype=np.uint32)
    gains = np.empty(max(k, 1), dtype=np.uint64)
    _check(ctx, load().im_select_seeds(ctx, g, _prob(kind, p), R, k, seed & ((1 << 64) - 1), _u32(seeds),
                                       _u64(gains)))
    return seeds[:k], gains[:k]


def im_centers(ctx, s):
    rho = ctypes.c_uint32()
    _check(ctx, load().im_centers(ctx, s, None, ctypes.byref(rho)))
    c = np.empty(max(rho.value, 1), dtype=np.uint32)
    _check(ctx, load().im_centers(ctx, s, _u32(c), ctypes.byref(rho)))
    return c[: rho.value]


def im_sketches_dump(ctx, s, r: int, count: int):
    lab = np.empty(max(count, 1), dtype=np.uint32)
    siz = np.empty(max(count, 1), dtype=np.uint32)
    _check(ctx, load().im_sketches_dump(ctx, s, r, _u32(lab), _u32(siz)))
    return lab[:count], siz[:count]


def im_initial_gains(ctx, s, n: int):
    g = np.empty(max(n, 1), dtype=np.uint64)
    _check(ctx, load().im_initial_gains(ctx, s, _u64(g)))
    return g[:n]


def im_select_trace(ctx, s, count: int):
    ev = np.empty(max(count, 1), dtype=np.uint32)
    _check(ctx, load().im_select_trace(ctx, s, _u32(ev), count))
    return ev[:count]


def im_probe_device(ctx):
    """(hash tests per second, copy bytes per second) measured on the device."""
    h, c = ctypes.c_double(), ctypes.c_double()
    _check(ctx, load().im_probe_device(ctx, ctypes.byref(h), ctypes.byref(c)))
    return h.value, c.value


def im_select_seeds_batched(ctx, queries, cfg=None):
    """queries: iterable of (graph handle, kind, p, R, k, seed[, alpha]).  cfg: dict with any
    of hook_block, hook_grid, select_block, select_grid.  Returns ([(seeds, gains)], device_ms)."""
    queries = [tuple(q) + ((1.0,) if len(q) == 6 else ()) for q in queries]
    nq = len(queries)
    arr = (im_query * max(nq, 1))()
    outs = []
    for i, (g, kind, p, R, k, seed, alpha) in enumerate(queries):
        arr[i] = im_query(g, _prob(kind, p), R, k, seed & ((1 << 64) - 1), float(alpha))
        outs.append((np.empty(max(k, 1), dtype=np.uint32), np.empty(max(k, 1), dtype=np.uint64)))
    sp = (_u32p * max(nq, 1))(*[_u32(a) for a, _ in outs])
    gp = (_u64p * max(nq, 1))(*[_u64(b) for _, b in outs])
    c = None
    if cfg:
        c = im_batch_config(int(cfg.get("hook_block", 0)), int(cfg.get("hook_grid", 0)),
                            int(cfg.get("select_block", 0)), int(cfg.get("select_grid", 0)))
    ms = ctypes.c_double()
    _check(ctx, load().im_select_seeds_batched(ctx, nq, arr, ctypes.byref(c) if c else None, sp, gp,
                                               ctypes.byref(ms)))
    return [(a[:q[4]], b[:q[4]]) for (a, b), q in zip(outs, queries)], ms.value


def im_server_create(ctx, graph_handles, hbm_budget=0, max_active=0, rounds_per_step=0, max_R=0, max_k=0,
                     compact_budget=0):
    arr = (_vp * len(graph_handles))(*graph_handles)
    cfg = im_server_config(hbm_budget, max_active, rounds_per_step, max_R, max_k, compact_budget)
    h = _vp()
    _check(ctx, load().im_server_create(ctx, arr, len(graph_handles), ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def _srv_check(rc, what):
    if rc != IM_OK:
        raise ImError(rc, what)


def im_server_submit(srv, graph, kind: int, p, R: int, k: int, seed: int, alpha: float = 1.0) -> int:
    """graph: the handle of one of the server's graphs."""
    t = ctypes.c_uint64()
    q = im_query(graph, _prob(kind, p), R, k, seed & ((1 << 64) - 1), float(alpha))
    _srv_check(load().im_server_submit(srv, ctypes.byref(q), ctypes.byref(t)), "im_server_submit")
    return t.value


def im_server_poll(srv, ticket: int) -> bool:
    d = ctypes.c_int()
    _srv_check(load().im_server_poll(srv, ticket, ctypes.byref(d)), "im_server_poll")
    return bool(d.value)


def im_server_wait(srv, ticket: int, k: int):
    seeds = np.empty(max(k, 1), dtype=np.uint32)
    gains = np.empty(max(k, 1), dtype=np.uint64)
    lat = ctypes.c_double()
    _srv_check(load().im_server_wait(srv, ticket, _u32(seeds), _u64(gains), ctypes.byref(lat)), "im_server_wait")
    return seeds[:k], gains[:k], lat.value


def im_server_stats(srv) -> dict:
    c = im_server_counters()
    _srv_check(load().im_server_stats(srv, ctypes.byref(c)), "im_server_stats")
    return {f: getattr(c, f) for f, _ in im_server_counters._fields_}


def im_server_destroy(srv):
    _srv_check(load().im_server_destroy(srv), "im_server_destroy")


def im_sketches_stats(s) -> dict:
    st = im_sketch_stats()
    rc = load().im_sketches_stats(s, ctypes.byref(st))
    if rc != IM_OK:
        raise ImError(rc, "im_sketches_stats")
    return {f: getattr(st, f) for f, _ in im_sketch_stats._fields_}


# ---- convenience wrappers ------------------------------------------------------

class Context:
    """An im_ctx on one device.  stream: a torch.cuda.Stream (or raw hipStream_t int) or None."""

    def __init__(self, device: int = 0, stream=None, hbm_cap: int = 0):
        raw = None
        if stream is not None:
            raw = getattr(stream, "cuda_stream", stream)
        self.h = im_ctx_create(device, raw, hbm_cap)

    def close(self):
        if self.h:
            im_ctx_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def graph(self, n, offsets, cols):
        return Graph(self, n, offsets, cols)

    def profiling(self, on=True):
        im_ctx_set_profiling(self.h, on)

    def kernel_time(self, name):
        return im_kernel_time(self.h, name)

    def memory(self):
        return im_ctx_memory(self.h)

    def probe(self):
        return im_probe_device(self.h)

    def probe_random(self):
        """Independent random 4-byte reads per second (4 GiB buffer)."""
        v = ctypes.c_double(0)
        _check(self.h, load().im_probe_random(self.h, ctypes.byref(v)))
        return v.value

    def select_batched(self, queries, cfg=None):
        """queries: list of (Graph, kind, p, R, k, seed[, alpha])."""
        return im_select_seeds_batched(self.h, [(q[0].h,) + tuple(q[1:]) for q in queries], cfg)


class Graph:
    def __init__(self, ctx: Context, n, offsets, cols):
        self.ctx = ctx
        self.n = int(n)
        self.h = im_graph_upload(ctx.h, self.n, offsets, cols)

    def close(self):
        if self.h:
            im_graph_free(self.h)
            self.h = None

    def sketches(self, kind, p, R, seed, alpha=1.0):
        return Sketches(self, kind, p, R, seed, alpha)

    def select_seeds(self, kind, p, R, k, seed):
        return im_select_seeds(self.ctx.h, self.h, kind, p, R, k, seed)

    def influence(self, kind, p, seeds, sim_seed, w0=0, sims=20000):
        """Sum over simulated worlds [w0, w0 + sims) of the seeds' activated vertices."""
        return im_influence(self.ctx.h, self.h, kind, p, seeds, sim_seed, w0, sims)

    def influence_noalloc(self, kind, p, seeds, sim_seed, w0=0, sims=20000):
        """influence() through the allocation-free entry point (static device scratch)."""
        return im_influence_noalloc(self.ctx.h, self.h, kind, p, seeds, sim_seed, w0, sims)


class Sketches:
    def __init__(self, graph: Graph, kind, p, R, seed, alpha=1.0):
        self.graph = graph
        self.ctx = graph.ctx
        self.R = int(R)
        self.alpha = float(alpha)
        self.h = im_build_sketches(self.ctx.h, graph.h, kind, p, R, seed, alpha)

    def close(self):
        if self.h:
            im_sketches_free(self.h)
            self.h = None

    def select(self, k):
        return im_select_seeds_from(self.ctx.h, self.h, k)

    def select_ptree(self, k):
        return im_select_seeds_ptree(self.ctx.h, self.h, k)

    def centers(self):
        return im_centers(self.ctx.h, self.h)

    def dump(self, r):
        count = self.graph.n if self.alpha >= 1.0 else int(self.stats()["rho"])
        return im_sketches_dump(self.ctx.h, self.h, r, count)

    def initial_gains(self):
        return im_initial_gains(self.ctx.h, self.h, self.graph.n)

    def stats(self):
        return im_sketches_stats(self.h)

    def trace(self):
        return im_select_trace(self.ctx.h, self.h, int(self.stats()["seeds_chosen"]))


class Server:
    """Request server over resident graphs (continuous batching in the library)."""

    def __init__(self, ctx: Context, graphs, **cfg):
        self.ctx = ctx
        self.graphs = list(graphs)
        self.h = im_server_create(ctx.h, [g.h for g in self.graphs], **cfg)
        self._k = {}

    def submit(self, graph: int, kind: int, p, R: int, k: int, seed: int, alpha: float = 1.0) -> int:
        """graph: index into the server's graphs; seed: the request's sampling seed;
        alpha: 1 for full labels, below 1 for CompactSketch."""
        t = im_server_submit(self.h, self.graphs[graph].h, kind, p, R, k, seed, alpha)
        self._k[t] = k
        return t

    def poll(self, ticket: int) -> bool:
        return im_server_poll(self.h, ticket)

    def wait(self, ticket: int):
        return im_server_wait(self.h, ticket, self._k.pop(ticket))

    def stats(self):
        return im_server_stats(self.h)

    def close(self):
        if self.h:
            im_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def select_seeds(offsets, cols, kind: int, p, R: int, k: int, seed: int, alpha: float = 1.0, stream=None):
    """One query on the current torch device: upload the CSR (torch tensors -- int64
    offsets, int32 cols, on the device or the host -- or numpy arrays), build R sketches
    (full labels for alpha = 1, CompactSketch below), select k seeds, free everything.
    Work is issued on `stream` (default: torch's current stream); torch only supplies
    the memory and the stream.  Returns (seeds uint32[k], gains uint64[k])."""
    import torch
    dev = torch.cuda.current_device()
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    n = int(offsets.numel() if hasattr(offsets, "numel") else len(offsets)) - 1
    with Context(dev, stream) as ctx:
        g = ctx.graph(n, offsets, cols)
        try:
            sk = g.sketches(kind, p, R, seed, alpha)
            try:
                return sk.select(k)
            finally:
                sk.close()
        finally:
            g.close()

"""Autotuner of the batched launch shapes (im_batch_config).

The batched path runs every query's sketch build as one flattened pass over
(query, pass, edge) items and every query's selection in one workgroup.  The
best launch shapes depend on the mix of graph sizes, so they are measured on the
batch itself, one axis at a time with the others at their best so far: the
sampling pass's block size, then its grid (0: one item per thread; else that
many workgroups striding over the items), then the selection workgroup size,
then the number of selection workgroups (0: one per query, at most 256; fewer
take several queries each from the shared counter).  Each candidate is timed by
the graph launch's own device time (best of `repeats`); a tie keeps the earlier
candidate.  Results are cached in a JSON file keyed by device name and a
signature of the batch (sizes, R, k), so a repeated batch shape costs no tuning.
"""
from __future__ import annotations

import hashlib
import json
import os

HOOK_BLOCKS = (128, 256, 512, 1024)
HOOK_GRIDS = (0, 1024, 4096, 16384)
SELECT_BLOCKS = (256, 512, 1024)
SELECT_GRIDS = (0, 16, 32)
# search order and starting point of every axis
AXES = (("hook_block", HOOK_BLOCKS), ("hook_grid", HOOK_GRIDS), ("select_block", SELECT_BLOCKS),
        ("select_grid", SELECT_GRIDS))
START = {"hook_block": 128, "hook_grid": 0, "select_block": 1024, "select_grid": 0}


def _cache_path():
    base = os.environ.get("PACIM_AUTOTUNE_CACHE")
    if base:
        return base
    root = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(root, "pacim", "autotune.json")


def signature(queries) -> str:
    """queries: list of (Graph, kind, p, R, k, seed) with Graph.n and an m_und attribute or None."""
    h = hashlib.sha1()
    for (g, kind, p, R, k, _seed) in queries:
        h.update(f"{g.n}:{getattr(g, 'm_und', 0)}:{kind}:{p:.6g}:{R}:{k};".encode())
    return h.hexdigest()[:16]


def _load():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(data):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def tune(ctx, queries, device_name: str = "gpu", repeats: int = 2, use_cache: bool = True):
    """Returns (best config dict, table of measured candidates)."""
    key = f"{device_name}/{signature(queries)}"
    cache = _load() if use_cache else {}
    if key in cache:
        return cache[key]["config"], cache[key].get("table", [])
    table = []

    def run(cfg):
        best = None
        for _ in range(repeats):
            _, ms = ctx.select_batched(queries, cfg)
            best = ms if best is None else min(best, ms)
        table.append({"config": dict(cfg), "device_ms": best})
        return best

    cfg = dict(START)
    best_t = run(cfg)
    for axis, cands in AXES:
        start = cfg[axis]  # measured already, with the other axes as they are now
        for v in cands:
            if v == start:
                continue
            trial = dict(cfg, **{axis: v})
            t = run(trial)
            if t < best_t:
                cfg, best_t = trial, t
    if use_cache:
        cache = _load()
        cache[key] = {"config": cfg, "table": table}
        _store(cache)
    return cfg, table

"""Autotuner of the batched launch shapes (im_batch_config).

The batched path runs every query's sketch build as one flattened pass over
(query, pass, edge) items and every query's selection in one workgroup.  The
best block sizes depend on the mix of graph sizes, so they are measured on the
batch itself: the sampling block size first (selection fixed), then the
selection workgroup size, each candidate timed by the graph launch's own device
time (best of `repeats`).  Results are cached in a JSON file keyed by device
name and a signature of the batch (sizes, R, k), so a repeated batch shape
costs no tuning.
"""
from __future__ import annotations

import hashlib
import json
import os

HOOK_BLOCKS = (128, 256, 512, 1024)
SELECT_BLOCKS = (256, 512, 1024)


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

    best_hook, best_t = None, None
    for hb in HOOK_BLOCKS:
        t = run({"hook_block": hb, "select_block": 1024})
        if best_t is None or t < best_t:
            best_hook, best_t = hb, t
    best_sel, best_t2 = 1024, best_t
    for sb in SELECT_BLOCKS:
        if sb == 1024:
            continue
        t = run({"hook_block": best_hook, "select_block": sb})
        if t < best_t2:
            best_sel, best_t2 = sb, t
    cfg = {"hook_block": best_hook, "select_block": best_sel}
    if use_cache:
        cache = _load()
        cache[key] = {"config": cfg, "table": table}
        _store(cache)
    return cfg, table

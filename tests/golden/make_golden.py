#!/usr/bin/env python3
"""Writes the stored expected results of the full-size parity tests.

Every value written here comes from the oracle (``oracle/``, the plain CPU
statement of the method) run on the seeded synthetic inputs
(``paper_2311_07554_amd.inputs``); nothing is read from the GPU library.  For each
query the oracle labels the R sampled graphs by BFS (``oracle.sketches``, one
single-threaded call per sketch, spread over host threads) and then selects the
seeds with NextSeed by prefix doubling over those labels (``oracle.ptree``,
Algorithm 4), whose seeds and gains equal the plain greedy's (Theorem 4.1; pinned
in tests/test_oracle_pins.py against the plain greedy and brute force).  The
R-MAT cases also record CELF's evaluation count (Algorithm 2,
``oracle.celf``) as the reference figure for the winning tree's evaluations
(Sec. 5, the table of evaluation counts).

Each entry is keyed by a digest of its graph (n, offsets and columns) and of the
query's parameters, so a test that regenerates the graph checks that it is the
graph the expected values belong to.

    python tests/golden/make_golden.py rmat24 rmat20 batched serving [--threads 8]

Files (JSON): rmat24_p0.02_R256_k200.json, rmat20_trivalency_R256_k100.json,
batched_chunglu64_R128_k50.json, serving_mix.json.  rmat24 needs about 40 GiB of host memory (labels and sizes of
256 sketches of 2^24 vertices) and 15-30 minutes on 8 cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FILES = {
    "rmat24": "rmat24_p0.02_R256_k200.json",
    "rmat20": "rmat20_trivalency_R256_k100.json",
    "batched": "batched_chunglu64_R128_k50.json",
    "serving": "serving_mix.json",
}


def graph_digest(g) -> str:
    """sha256 of the graph's vertex count, CSR offsets and columns."""
    h = hashlib.sha256()
    h.update(np.uint64(g.n).tobytes())
    h.update(np.ascontiguousarray(g.offsets, dtype=np.uint64).tobytes())
    h.update(np.ascontiguousarray(g.cols, dtype=np.uint32).tobytes())
    return h.hexdigest()


def query_id(digest: str, kind: int, p: float, p_hi: float, R: int, seed: int) -> str:
    """Key of one sketch set: graph digest, model (kind, p, p_hi as exact hex floats), R, sampling seed."""
    s = f"{digest}|{kind}|{float(p).hex()}|{float(p_hi).hex()}|{R}|{seed}"
    return hashlib.sha256(s.encode()).hexdigest()[:24]


def path_of(name: str) -> str:
    return os.path.join(HERE, FILES[name])


def load(name: str) -> dict:
    """{query id: entry} of a stored file."""
    with open(path_of(name)) as f:
        doc = json.load(f)
    return {e["id"]: e for e in doc["entries"]}


def _say(*a):
    print(*a, flush=True)


def oracle_entry(g, digest, kind, p, p_hi, R, k, seed, threads, celf=False):
    import oracle
    pm = (p, p_hi) if kind == 2 else p
    t0 = time.time()
    lab, siz = oracle.sketches(g, kind, pm, seed, R, threads=threads)
    t1 = time.time()
    seeds, gains, ev = oracle.ptree(lab, siz, k)
    t2 = time.time()
    e = {"id": query_id(digest, kind, p, p_hi, R, seed), "graph": digest, "n": g.n, "m_und": g.m_und,
         "kind": kind, "p": p, "p_hi": p_hi, "R": R, "k": k, "seed": seed,
         "seeds": [int(x) for x in seeds], "gains": [int(x) for x in gains],
         "ptree_evaluations": [int(x) for x in ev]}
    if celf:
        cs, cg, cev = oracle.celf(lab, siz, k)
        assert np.array_equal(cs, seeds) and np.array_equal(cg, gains), "CELF and prefix doubling disagree"
        e["celf_evaluations"] = [int(x) for x in cev]
    _say(f"  n={g.n} kind={kind} p={p} p_hi={p_hi} R={R} k={k} seed={seed}: sketches {t1 - t0:.1f}s, "
         f"selection {t2 - t1:.1f}s{' + CELF ' + f'{time.time() - t2:.1f}s' if celf else ''}")
    del lab, siz
    return e


def write(name: str, config: dict, entries: list):
    doc = {"source": "oracle/ (BFS sketches + Algorithm 4 over them), written by tests/golden/make_golden.py",
           "config": config, "entries": entries}
    tmp = path_of(name) + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, separators=(",", ":"))
        f.write("\n")
    os.replace(tmp, path_of(name))
    _say(f"wrote {path_of(name)} ({len(entries)} entries)")


def make_rmat24(threads):
    from paper_2311_07554_amd import inputs
    q = inputs.rmat24().queries[0]
    g = q.graph
    d = graph_digest(g)
    _say(f"rmat24: n={g.n} m_und={g.m_und} digest {d[:16]}")
    e = oracle_entry(g, d, q.prob_kind, q.p, 0.0, q.R, q.k, q.seed, threads, celf=True)
    write("rmat24", {"workload": "R-MAT scale 24, 2^28 pairs, graph seed 3; uniform p = 0.02; R = 256; k = 200; "
                                 "sampling seed 1"}, [e])


def make_rmat20(threads):
    from paper_2311_07554_amd import inputs
    q = inputs.rmat20().queries[0]
    g = q.graph
    d = graph_digest(g)
    _say(f"rmat20: n={g.n} m_und={g.m_und} digest {d[:16]}")
    e = oracle_entry(g, d, q.prob_kind, q.p, 0.0, q.R, q.k, q.seed, threads, celf=True)
    write("rmat20", {"workload": "R-MAT scale 20, 2^24 pairs, graph seed 2; trivalency; R = 256; k = 100; "
                                 "sampling seed 1"}, [e])


def make_batched(threads):
    from paper_2311_07554_amd import inputs
    w = inputs.batched()
    entries = []
    _say(f"batched: {len(w.queries)} queries")
    for q in w.queries:
        d = graph_digest(q.graph)
        entries.append(oracle_entry(q.graph, d, q.prob_kind, q.p, 0.0, q.R, q.k, q.seed, threads))
    write("batched", {"workload": "64 Chung-Lu graphs (inputs.batched()), R = 128, k = 50, seed q + 1"}, entries)


def make_serving(threads):
    from paper_2311_07554_amd import inputs
    graphs = inputs.serving_graphs(scales=inputs.SERVING_SCALES[:inputs.SERVING_MIX_GRAPHS])
    digests = [graph_digest(g) for g in graphs]
    mix = inputs.serving_mix()
    # one oracle run per sketch set, up to the largest k asked of it (the greedy's
    # first k1 seeds of a k2-seed run are the k1-seed run)
    sets = {}
    for (gi, kind, p, p_hi, R, k, seed, _alpha) in mix:
        key = (gi, kind, p, p_hi, R, seed)
        sets[key] = max(sets.get(key, 0), k)
    _say(f"serving: {len(mix)} requests over {len(sets)} sketch sets")
    entries = []
    for (gi, kind, p, p_hi, R, seed), k in sorted(sets.items()):
        entries.append(oracle_entry(graphs[gi], digests[gi], kind, p, p_hi, R, k, seed, threads))
    write("serving", {"workload": "inputs.serving_mix() over the first 7 serving graphs (R-MAT scales 16-18)"},
          entries)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="+", choices=sorted(FILES))
    ap.add_argument("--threads", type=int, default=max(1, min(16, os.cpu_count() or 1)))
    a = ap.parse_args()
    for w in a.which:
        {"rmat24": make_rmat24, "rmat20": make_rmat20, "batched": make_batched,
         "serving": make_serving}[w](a.threads)


if __name__ == "__main__":
    main()

"""GPU parity at full size: the R-MAT scale-20 workload and the scale-24 one.

R-MAT scale 20: 2^20 vertices, 2^24 undirected pairs, trivalency probabilities,
R = 256, k = 100; full labels and CompactSketch (alpha = 0.1), in the
configuration the benchmark times.  The oracle labels all 256 sketches (threaded
BFS) and selects the 100 seeds over them with Algorithm 4 (equal to the plain
greedy, Theorem 4.1).  Checked: sampled sketches' labels, sizes and compact
triples, every vertex's initial gain, and the whole seed and gain sequence of
the winning tree (full labels and CompactSketch) and of prefix doubling, with
prefix doubling's per-round evaluation counts.

R-MAT scale 24: 2^24 vertices, 2^28 pairs, uniform p = 0.02, R = 256, k = 200.
The oracle's seeds and gains are stored (tests/golden/rmat24_p0.02_R256_k200.json,
written by tests/golden/make_golden.py from the oracle alone: 40 GiB of host
memory and half an hour on 8 cores); the test checks that the graph it
generates is the stored one, labels two sampled sketches with the oracle, and
compares the CompactSketch (alpha = 0.1) and full-label sequences with the stored
ones element by element.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2311_07554_amd import inputs, pacim
from tests.golden import make_golden
from tests.gpu_util import upload

pytestmark = pytest.mark.gpu

SAMPLED_SKETCHES = (0, 77, 131, 255)


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = pacim.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def workload():
    q = inputs.rmat20().queries[0]
    threads = max(1, min(16, os.cpu_count() or 1))
    _say(f"case rmat20 full size: oracle labels of {q.R} sketches on {threads} threads")
    lab, siz = oracle.sketches(q.graph, q.prob_kind, q.p, q.seed, q.R, threads=threads)
    _say("  oracle: Algorithm 4 over the 256 sketches")
    ref = oracle.ptree(lab, siz, q.k)
    return q, lab, siz, threads, ref


def test_rmat20_full_labels_parity(ctx, workload):
    q, lab, siz, threads, (ws, wg, _) = workload
    g = q.graph
    gr = upload(ctx, g)
    sk = gr.sketches(q.prob_kind, q.p, q.R, q.seed, 1.0)
    for r in SAMPLED_SKETCHES:
        gl, gs = sk.dump(r)
        assert np.array_equal(gl, lab[r]), r
        assert np.array_equal(gs, siz[r]), r
    assert np.array_equal(sk.initial_gains(), siz.astype(np.uint64).sum(axis=0))
    seeds, gains = sk.select(q.k)
    sk.close()
    gr.close()
    _say("  seeds", seeds[:8], "gains", gains[:8])
    # the whole sequence, every round
    assert np.array_equal(seeds, ws) and np.array_equal(gains, wg)


def test_rmat20_compact_parity(ctx, workload):
    q, lab, siz, _, (ws, wg, _) = workload
    g = q.graph
    alpha = 0.1
    cents = oracle.centers(g.n, q.seed, alpha)
    gr = upload(ctx, g)
    sk = gr.sketches(q.prob_kind, q.p, q.R, q.seed, alpha)
    assert np.array_equal(sk.centers(), cents)
    for r in SAMPLED_SKETCHES:
        lc, sc = oracle.compact(lab[r], siz[r], cents)
        gl, gs = sk.dump(r)
        assert np.array_equal(gl, lc) and np.array_equal(gs, sc), r
    assert np.array_equal(sk.initial_gains(), siz.astype(np.uint64).sum(axis=0))
    seeds, gains = sk.select(q.k)
    st = sk.stats()
    sk.close()
    gr.close()
    _say("  compact: bulk rounds", st["bulk_rounds"], "re-derived", st["bulk_resampled"], "evaluations",
         st["evaluations"])
    assert np.array_equal(seeds, ws) and np.array_equal(gains, wg)


@pytest.mark.parametrize("alpha", [1.0, 0.1])
def test_rmat20_prefix_doubling_full_size(ctx, workload, alpha):
    # NextSeed by prefix doubling (Algorithm 4) on the benchmark's sketches: seeds, gains
    # and every round's evaluation count against the oracle run whole (its round 1
    # re-evaluates all but a few of the 2^20 vertices)
    q, lab, siz, _, (ws, wg, wev) = workload
    gr = upload(ctx, q.graph)
    sk = gr.sketches(q.prob_kind, q.p, q.R, q.seed, alpha)
    s, gn = sk.select_ptree(q.k)
    ev = sk.trace()
    sk.close()
    gr.close()
    _say(f"  prefix doubling alpha={alpha}: evaluations {int(ev.sum())}, largest round {int(ev.max())}")
    assert np.array_equal(s, ws) and np.array_equal(gn, wg)
    assert np.array_equal(ev.astype(np.uint64), wev)


def test_rmat24_full_size_matches_stored_oracle(ctx):
    """R-MAT scale 24 (2^24 vertices, 2^28 pairs), uniform p = 0.02, R = 256,
    k = 200: CompactSketch alpha = 0.1 and full labels (34 GB of E) against the
    oracle's stored sequence."""
    q = inputs.rmat24().queries[0]
    g = q.graph
    _say(f"case rmat24 full size: n={g.n} m={g.m_und}")
    digest = make_golden.graph_digest(g)
    stored = make_golden.load("rmat24")
    e = stored[make_golden.query_id(digest, q.prob_kind, q.p, 0.0, q.R, q.seed)]
    assert e["graph"] == digest and e["k"] == q.k
    cents = oracle.centers(g.n, q.seed, q.alpha)
    gr = upload(ctx, g)
    sk = gr.sketches(q.prob_kind, q.p, q.R, q.seed, q.alpha)
    assert np.array_equal(sk.centers(), cents)
    sampled = {}
    for r in (0, 255):
        lab_r, siz_r = oracle.sketch(g, q.prob_kind, q.p, q.seed, r)
        sampled[r] = (lab_r, siz_r)
        lc, sc = oracle.compact(lab_r, siz_r, cents)
        gl, gs = sk.dump(r)
        assert np.array_equal(gl, lc) and np.array_equal(gs, sc), r
    seeds, gains = sk.select(q.k)
    st = sk.stats()
    sk.close()
    _say("  compact: seeds", seeds[:6], "gains", gains[:6], "bulk rounds", st["bulk_rounds"], "re-derived",
         st["bulk_resampled"])
    assert seeds.tolist() == e["seeds"] and gains.tolist() == e["gains"]

    fk = gr.sketches(q.prob_kind, q.p, q.R, q.seed, 1.0)
    for r, (lab_r, siz_r) in sampled.items():
        gl, gs = fk.dump(r)
        assert np.array_equal(gl, lab_r) and np.array_equal(gs, siz_r), r
    s2, g2 = fk.select(q.k)
    fk.close()
    gr.close()
    assert s2.tolist() == e["seeds"] and g2.tolist() == e["gains"]

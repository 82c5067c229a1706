"""GPU parity of NextSeed by prefix doubling (Sec. 4, Algorithm 4) against the oracle.

The queue's order is total (larger stale gain, then smaller id), so the batches
a round takes are unique: seeds, gains and the per-round evaluation counts are
all compared bit-exactly with ``oracle.ptree``.  With CompactSketch the GPU
evaluates by GetCenter, whose Marginal equals the full-label one (pinned by the
oracle's own tests), so the full-label oracle fixes the same counts.  Sizes span
several 4096-key sort tiles and merge passes, rounds that re-evaluate nearly
every vertex, the queue running empty (k = n), and ties everywhere (p = 0).
"""
import numpy as np
import pytest

import oracle
from paper_2311_07554_amd import inputs, pacim
from tests.gpu_util import upload

pytestmark = pytest.mark.gpu

U, TRI = pacim.IM_PROB_UNIFORM, pacim.IM_PROB_TRIVALENCY


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = pacim.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)


def _ptree_gpu(ctx, g, kind, p, R, k, seed, alpha, chunks=None):
    gr = upload(ctx, g)
    try:
        sk = gr.sketches(kind, p, R, seed, alpha)
        try:
            parts = [sk.select_ptree(c) for c in (chunks or [k])]
            s = np.concatenate([a for a, _ in parts])
            gn = np.concatenate([b for _, b in parts])
            return s, gn, sk.trace(), sk.stats()
        finally:
            sk.close()
    finally:
        gr.close()


@pytest.mark.parametrize("scale,kind,p,R,k,seed", [
    (12, TRI, 0.0, 40, 40, 3),
    (13, U, 0.05, 64, 30, 4),
    (14, U, 0.3, 16, 20, 5),     # a giant component: round 1 re-evaluates most of 2^14 vertices
    (9, U, 0.02, 8, 512, 6),     # k = n: the queue runs empty
    (15, U, 0.3, 8, 10, 12),     # batches of 2^14 vertices: the label-caching evaluation
])
@pytest.mark.parametrize("alpha", [1.0, 0.25])
def test_ptree_matches_oracle(ctx, scale, kind, p, R, k, seed, alpha):
    g = inputs.rmat_graph(scale, 8 << scale, seed=seed)
    k = min(k, g.n)
    _say(f"case ptree scale={scale} kind={kind} p={p} R={R} k={k} alpha={alpha}")
    lab, siz = oracle.sketches(g, kind, p, seed, R, threads=8)
    ws, wg, wev = oracle.ptree(lab, siz, k)
    s, gn, ev, st = _ptree_gpu(ctx, g, kind, p, R, k, seed, alpha)
    assert np.array_equal(s, ws) and np.array_equal(gn, wg)
    assert np.array_equal(ev.astype(np.uint64), wev)
    assert st["evaluations"] == int(wev.sum())


def test_ptree_ties_everywhere(ctx):
    g = inputs.rmat_graph(10, 8 << 10, seed=2)
    _say("case ptree ties p=0")
    s, gn, ev, _ = _ptree_gpu(ctx, g, U, 0.0, 8, 100, 1, 1.0)
    assert list(s) == list(range(100)) and set(gn.tolist()) == {8} and set(ev.tolist()) == {1}


@pytest.mark.parametrize("alpha", [1.0, 0.25])
def test_ptree_continues_across_calls(ctx, alpha):
    g = inputs.rmat_graph(12, 8 << 12, seed=7)
    _say(f"case ptree chunks alpha={alpha}")
    lab, siz = oracle.sketches(g, TRI, 0.0, 7, 32, threads=8)
    ws, wg, wev = oracle.ptree(lab, siz, 24)
    s, gn, ev, _ = _ptree_gpu(ctx, g, TRI, 0.0, 32, 24, 7, alpha, chunks=[1, 7, 16])
    assert np.array_equal(s, ws) and np.array_equal(gn, wg)
    assert np.array_equal(ev.astype(np.uint64), wev)


@pytest.mark.parametrize("alpha", [1.0, 0.25])
def test_ptree_and_winning_tree_mixed(ctx, alpha):
    # each selection rebuilds its structure from the keys the other left: the seeds
    # stay the plain greedy's
    g = inputs.rmat_graph(12, 8 << 12, seed=8)
    _say(f"case mixed selections alpha={alpha}")
    lab, siz = oracle.sketches(g, U, 0.05, 8, 32, threads=8)
    ws, wg = oracle.greedy(lab, siz, 30)
    gr = upload(ctx, g)
    sk = gr.sketches(U, 0.05, 32, 8, alpha)
    parts = [sk.select(5), sk.select_ptree(8), sk.select(9), sk.select_ptree(8)]
    sk.close()
    gr.close()
    s = np.concatenate([a for a, _ in parts])
    gn = np.concatenate([b for _, b in parts])
    assert np.array_equal(s, ws) and np.array_equal(gn, wg)


def test_ptree_within_twice_celf(ctx):
    # Theorem 4.2 on the GPU's own counts
    g = inputs.rmat_graph(13, 8 << 13, seed=9)
    _say("case ptree vs celf")
    lab, siz = oracle.sketches(g, TRI, 0.0, 9, 64, threads=8)
    _, _, cev = oracle.celf(lab, siz, 50)
    _, _, ev, _ = _ptree_gpu(ctx, g, TRI, 0.0, 64, 50, 9, 1.0)
    assert int(ev.sum()) <= 2 * int(cev.sum())


@pytest.mark.parametrize("bulk,cap", [("0", None), ("1", None), ("64", None), ("1", "1"), ("64", "1")])
def test_ptree_compact_bulk_evaluation(ctx, bulk, cap, monkeypatch):
    # CompactSketch rounds may evaluate a large batch from every vertex's fresh key
    # (bitmaps, or re-derived components past the search cap): same counts as the
    # per-vertex GetCenter evaluation.  A giant component makes round 1 take
    # batches of thousands of vertices.
    monkeypatch.setenv("PACIM_PTREE_BULK", bulk)
    if cap is not None:
        monkeypatch.setenv("PACIM_BULK_SEARCH_CAP", cap)
    g = inputs.rmat_graph(14, 8 << 14, seed=5)
    k = 20
    _say(f"case ptree compact bulk={bulk} cap={cap}")
    lab, siz = oracle.sketches(g, U, 0.3, 5, 16, threads=8)
    ws, wg, wev = oracle.ptree(lab, siz, k)
    s, gn, ev, st = _ptree_gpu(ctx, g, U, 0.3, 16, k, 5, 0.2)
    assert np.array_equal(s, ws) and np.array_equal(gn, wg)
    assert np.array_equal(ev.astype(np.uint64), wev)
    if bulk == "0":
        assert st["bulk_rounds"] == 0
    elif bulk == "1":
        assert st["bulk_rounds"] == k
    else:
        assert st["bulk_rounds"] >= 1
    # rounds whose seeds all lie in the largest components need no search, so
    # they use the bitmaps even with the cap
    if cap is None:
        assert st["bulk_resampled"] == 0
    elif bulk == "1":
        assert 1 <= st["bulk_resampled"] <= st["bulk_rounds"]


@pytest.mark.parametrize("scale,kind,p,R,k,seed", [(12, TRI, 0.0, 40, 40, 3), (14, U, 0.3, 16, 20, 5)])
def test_ptree_host_driven_rounds(ctx, scale, kind, p, R, k, seed, monkeypatch):
    # full labels run whole rounds on the device by default; the host-driven rounds
    # (every batch a launch and a read-back) must give the same
    monkeypatch.setenv("PACIM_PTREE_DEVICE", "0")
    g = inputs.rmat_graph(scale, 8 << scale, seed=seed)
    _say(f"case ptree host-driven scale={scale}")
    lab, siz = oracle.sketches(g, kind, p, seed, R, threads=8)
    ws, wg, wev = oracle.ptree(lab, siz, k)
    s, gn, ev, _ = _ptree_gpu(ctx, g, kind, p, R, k, seed, 1.0)
    assert np.array_equal(s, ws) and np.array_equal(gn, wg)
    assert np.array_equal(ev.astype(np.uint64), wev)

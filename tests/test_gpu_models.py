"""GPU parity of the per-edge probability models of the appendix on edge-probability
distributions: "Uniform" (p_e drawn from U(lo, hi) once per edge) and WIC
(p_e = 2 / (d_u + d_v)), against the oracle, bit-exact.

The models change only which edges are live (the sampling pass, GetCenter's
searches, the bulk rounds' re-derived components), so every sketch of a build is
compared entry by entry -- full labels and sizes, or the CompactSketch triple --
and the seeds and gains after it.  Cases: both label kinds, the CompactSketch
bulk round re-deriving its sketches, the batched launch with mixed models, and
the models' argument checks.
"""
import numpy as np
import pytest

import oracle
from paper_2311_07554_amd import inputs, pacim
from tests import brute
from tests.gpu_util import run_select, upload

pytestmark = pytest.mark.gpu

RANGE, WIC = pacim.IM_PROB_RANGE, pacim.IM_PROB_WIC

MODELS = [(RANGE, (0.0, 0.1)), (RANGE, (0.1, 0.3)), (WIC, 0.0)]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = pacim.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("kind,p", MODELS, ids=["U(0,0.1)", "U(0.1,0.3)", "WIC"])
@pytest.mark.parametrize("alpha", [1.0, 0.2])
def test_models_match_oracle(ctx, kind, p, alpha):
    scale, R, k, seed = 12, 40, 25, 9
    g = inputs.rmat_graph(scale, 16 << scale, seed=41)
    _say(f"case model kind={kind} p={p} alpha={alpha}")
    lab, siz = oracle.sketches(g, kind, p, seed, R, threads=8)
    gr = upload(ctx, g)
    sk = gr.sketches(kind, p, R, seed, alpha)
    if alpha == 1.0:
        for r in range(R):
            gl, gs = sk.dump(r)
            assert np.array_equal(gl, lab[r]) and np.array_equal(gs, siz[r]), r
    else:
        cents = oracle.centers(g.n, seed, alpha)
        lc, sc = oracle.compact_all(lab, siz, cents)
        for r in range(R):
            gl, gs = sk.dump(r)
            assert np.array_equal(gl, lc[r]) and np.array_equal(gs, sc[r]), r
    assert np.array_equal(sk.initial_gains(), siz.astype(np.uint64).sum(axis=0))
    s, gn = sk.select(k)
    ws, wg = oracle.greedy(lab, siz, k)
    assert np.array_equal(s, ws) and np.array_equal(gn, wg)
    sk.close()
    gr.close()


@pytest.mark.parametrize("kind,p", [(RANGE, (0.1, 0.3)), (WIC, 0.0)], ids=["U(0.1,0.3)", "WIC"])
def test_models_bulk_rounds_rederive(ctx, kind, p, monkeypatch):
    # every CompactSketch round after the first in bulk, past the search cap: the
    # sampled graphs are re-derived under the model
    monkeypatch.setenv("PACIM_BULK", "always")
    monkeypatch.setenv("PACIM_BULK_SEARCH_CAP", "1")
    g = inputs.rmat_graph(11, 16 << 11, seed=42)
    R, k, seed = 24, 12, 4
    _say(f"case model bulk kind={kind}")
    lab, siz = oracle.sketches(g, kind, p, seed, R, threads=8)
    ws, wg = oracle.greedy(lab, siz, k)
    s, gn, st = run_select(ctx, g, kind, p, R, k, seed, alpha=0.1)
    assert np.array_equal(s, ws) and np.array_equal(gn, wg)
    assert st["bulk_rounds"] == k - 1


def test_models_in_one_batched_launch(ctx):
    specs = [(1500, 10.0, WIC, 0.0, 40, 12), (1200, 14.0, RANGE, (0.0, 0.1), 64, 9),
             (900, 8.0, pacim.IM_PROB_TRIVALENCY, 0.0, 20, 5), (2000, 6.0, RANGE, (0.1, 0.3), 33, 7)]
    _say("case models batched")
    graphs, want = [], []
    for i, (n, d, kind, p, R, k) in enumerate(specs):
        g = inputs.chunglu_graph(n, d, 2.2, seed=300 + i)
        lab, siz = oracle.sketches(g, kind, p, i + 1, R, threads=8)
        want.append(oracle.greedy(lab, siz, k))
        graphs.append(ctx.graph(g.n, g.offsets, g.cols))
    try:
        qs = [(gr, kind, p, R, k, i + 1) for i, (gr, (n, d, kind, p, R, k)) in enumerate(zip(graphs, specs))]
        res, _ = ctx.select_batched(qs, None)
        for (s, gn), (ws, wg) in zip(res, want):
            assert np.array_equal(s, ws) and np.array_equal(gn, wg)
    finally:
        for gr in graphs:
            gr.close()


def test_model_arguments(ctx):
    g = inputs.er_graph(50, 100, seed=2)
    gr = upload(ctx, g)
    for kind, p in [(RANGE, (0.3, 0.1)), (RANGE, (0.1, 1.0)), (RANGE, (-0.1, 0.2)), (7, 0.1)]:
        with pytest.raises(pacim.ImError) as e:
            gr.sketches(kind, p, 4, 1)
        assert e.value.status == pacim.IM_EINVAL
    sk = gr.sketches(RANGE, (0.2, 0.2), 4, 1)   # lo == hi: the Consistent model
    s1, g1 = sk.select(10)
    sk.close()
    sk = gr.sketches(pacim.IM_PROB_UNIFORM, 0.2, 4, 1)
    s2, g2 = sk.select(10)
    sk.close()
    gr.close()
    assert np.array_equal(s1, s2) and np.array_equal(g1, g2)


PER_EDGE = pacim.IM_PROB_PER_EDGE


@pytest.mark.parametrize("alpha", [1.0, 0.2])
def test_per_edge_model_matches_oracle(ctx, alpha):
    # the caller's probability for every CSR entry (symmetric), converted once to thresholds
    scale, R, k, seed = 12, 36, 20, 6
    g = inputs.rmat_graph(scale, 16 << scale, seed=43)
    pe = brute.per_edge_p(g, 5) * 0.2  # p_e in [0, 0.2)
    _say(f"case per-edge alpha={alpha}")
    lab, siz = oracle.sketches(g, oracle.PER_EDGE, pe, seed, R, threads=8)
    gr = upload(ctx, g)
    sk = gr.sketches(PER_EDGE, pe, R, seed, alpha)
    if alpha == 1.0:
        for r in range(0, R, 5):
            gl, gs = sk.dump(r)
            assert np.array_equal(gl, lab[r]) and np.array_equal(gs, siz[r]), r
    else:
        cents = oracle.centers(g.n, seed, alpha)
        lc, sc = oracle.compact_all(lab, siz, cents)
        for r in range(0, R, 5):
            gl, gs = sk.dump(r)
            assert np.array_equal(gl, lc[r]) and np.array_equal(gs, sc[r]), r
    assert np.array_equal(sk.initial_gains(), siz.astype(np.uint64).sum(axis=0))
    s, gn = sk.select(k)
    sk.close()
    ws, wg = oracle.greedy(lab, siz, k)
    assert np.array_equal(s, ws) and np.array_equal(gn, wg)
    got = gr.influence(PER_EDGE, pe, s, 11, 100, 70)
    gr.close()
    assert got == oracle.influence(g, oracle.PER_EDGE, pe, s, 11, 100, 70, threads=8)


def test_per_edge_model_arguments(ctx):
    g = inputs.er_graph(60, 150, seed=3)
    gr = upload(ctx, g)
    pe = brute.per_edge_p(g, 1)
    bad = pe.copy()
    bad[0] = 1.5
    asym = pe.copy()
    asym[0] = (asym[0] + 0.5) % 1.0   # one direction of an edge only
    for p in (bad, asym):
        with pytest.raises(pacim.ImError) as e:
            gr.sketches(PER_EDGE, p, 4, 1)
        assert e.value.status == pacim.IM_EINVAL
    with pytest.raises(pacim.ImError) as e:
        ctx.select_batched([(gr, PER_EDGE, pe, 4, 3, 1)], None)
    assert e.value.status == pacim.IM_EINVAL
    sk = gr.sketches(PER_EDGE, np.full(g.cols.size, 0.3), 8, 2)   # constant: the Consistent model
    s1, g1 = sk.select(6)
    sk.close()
    sk = gr.sketches(pacim.IM_PROB_UNIFORM, 0.3, 8, 2)
    s2, g2 = sk.select(6)
    sk.close()
    gr.close()
    assert np.array_equal(s1, s2) and np.array_equal(g1, g2)

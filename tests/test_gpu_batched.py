"""Batched selection (one hipGraph of persistent kernels) against each query
alone and against the oracle: bit-exact seeds and gains for every query, under
several launch shapes."""
import numpy as np
import pytest

import oracle
from paper_2311_07554_amd import inputs, pacim
from tests.gpu_util import run_select

pytestmark = pytest.mark.gpu
U, TRI = pacim.IM_PROB_UNIFORM, pacim.IM_PROB_TRIVALENCY


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = pacim.Context(0)
    yield c
    c.close()


# (n, avg degree, kind, p, R, k): uneven sizes, R below / at / above one 64-sketch pass
SPECS = [(500, 8.0, U, 0.05, 5, 3), (2000, 12.0, U, 0.02, 64, 10), (4097, 20.0, U, 0.08, 70, 15),
         (1000, 30.0, TRI, 0.0, 128, 20), (64, 4.0, U, 0.5, 8, 64), (3000, 9.0, U, 0.03, 33, 7),
         (1500, 16.0, U, 1.0, 3, 4)]


@pytest.fixture(scope="module")
def batch():
    out = []
    for i, (n, d, kind, p, R, k) in enumerate(SPECS):
        g = inputs.chunglu_graph(n, d, 2.2, seed=100 + i)
        lab, siz = oracle.sketches(g, kind, p, i + 1, R, threads=8)
        ws, wg = oracle.greedy(lab, siz, k)
        out.append((g, kind, p, R, k, i + 1, ws, wg))
    return out


@pytest.mark.parametrize("cfg", [None, {"hook_block": 64, "select_block": 64},
                                 {"hook_block": 1024, "select_block": 256, "select_grid": 3}])
def test_batched_matches_oracle_and_standalone(ctx, batch, cfg):
    print("case batched cfg", cfg, flush=True)
    graphs = [ctx.graph(g.n, g.offsets, g.cols) for (g, *_rest) in batch]
    try:
        qs = [(gr, kind, p, R, k, seed) for gr, (g, kind, p, R, k, seed, ws, wg) in zip(graphs, batch)]
        res, ms = ctx.select_batched(qs, cfg)
        assert ms > 0
        for (s, gn), (g, kind, p, R, k, seed, ws, wg) in zip(res, batch):
            assert np.array_equal(s, ws) and np.array_equal(gn, wg), (g.n, R, k)
    finally:
        for gr in graphs:
            gr.close()


def test_batched_equals_one_query_per_launch(ctx, batch):
    graphs = [ctx.graph(g.n, g.offsets, g.cols) for (g, *_rest) in batch]
    try:
        qs = [(gr, kind, p, R, k, seed) for gr, (g, kind, p, R, k, seed, ws, wg) in zip(graphs, batch)]
        res, _ = ctx.select_batched(qs)
        for (gr, kind, p, R, k, seed), (s, gn) in zip(qs, res):
            s1, g1 = gr.select_seeds(kind, p, R, k, seed)
            assert np.array_equal(s, s1) and np.array_equal(gn, g1)
    finally:
        for gr in graphs:
            gr.close()


def test_batched_rejects_bad_queries(ctx):
    g = inputs.er_graph(50, 100, seed=3)
    gr = ctx.graph(g.n, g.offsets, g.cols)
    try:
        with pytest.raises(pacim.ImError):
            ctx.select_batched([(gr, U, 0.1, 4, 51, 1)])
        with pytest.raises(pacim.ImError):
            ctx.select_batched([(gr, U, 0.1, 4, 5, 1)], {"hook_block": 100})
        res, _ = ctx.select_batched([(gr, U, 0.1, 4, 50, 1)])
        assert len(set(res[0][0].tolist())) == 50
    finally:
        gr.close()

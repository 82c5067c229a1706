"""The allocation-free influence entry point (im_influence_noalloc, static device
scratch) against im_influence, which allocates its scratch: the same summed
spread, bit-exact, on calls in a row with shrinking inputs (the static array
keeps the previous call's contents), with fewer than 64 worlds per pass on a
larger graph, and the rejections of inputs beyond the array."""
import numpy as np
import pytest

import oracle
from paper_2311_07554_amd import inputs, pacim
from tests.gpu_util import upload

pytestmark = pytest.mark.gpu

U, TRI, WIC = pacim.IM_PROB_UNIFORM, pacim.IM_PROB_TRIVALENCY, pacim.IM_PROB_WIC


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = pacim.Context(0)
    yield c
    c.close()


def test_noalloc_equals_allocating_call_twice_in_a_row(ctx):
    assert pacim.im_influence_static_scratch() == 64 << 20
    big = inputs.rmat_graph(14, 16 << 14, seed=61)
    small = inputs.er_graph(1000, 5000, seed=1)
    rng = np.random.default_rng(7)
    cases = [(big, U, 0.05, rng.integers(0, big.n, 60).astype(np.uint32), 0x51D, 17, 300),
             (small, U, 0.05, rng.integers(0, small.n, 9).astype(np.uint32), 3, 0, 70)]
    for g, kind, p, seeds, sim_seed, w0, sims in cases:
        _say(f"case noalloc n={g.n} k={seeds.size} worlds [{w0}, {w0 + sims})")
        gr = upload(ctx, g)
        got = gr.influence_noalloc(kind, p, seeds, sim_seed, w0, sims)
        want = gr.influence(kind, p, seeds, sim_seed, w0, sims)
        gr.close()
        assert got == want, (g.n, got, want)
    # the smaller case against the oracle as well
    g, kind, p, seeds, sim_seed, w0, sims = cases[1]
    assert got == oracle.influence(g, kind, p, seeds, sim_seed, w0, sims)


def test_noalloc_few_worlds_per_pass_and_models(ctx):
    # 2^18 vertices: 12 bytes per vertex per world leave room for 20 worlds per pass
    g = inputs.rmat_graph(18, 8 << 18, seed=62)
    gr = upload(ctx, g)
    rng = np.random.default_rng(8)
    seeds = rng.integers(0, g.n, 25).astype(np.uint32)
    for kind, p, sims in [(TRI, 0.0, 50), (WIC, 0.0, 41)]:
        _say(f"case noalloc rmat18 kind={kind} sims={sims}")
        got = gr.influence_noalloc(kind, p, seeds, 5, 100, sims)
        want = gr.influence(kind, p, seeds, 5, 100, sims)
        assert got == want, (kind, got, want)
    gr.close()


def test_noalloc_rejects_what_the_array_cannot_hold(ctx):
    small = inputs.er_graph(1000, 5000, seed=1)
    gr = upload(ctx, small)
    assert gr.influence_noalloc(U, 0.5, [], 1, 0, 70) == 0
    assert gr.influence_noalloc(U, 0.5, [2], 1, 0, 0) == 0
    with pytest.raises(pacim.ImError) as e:
        pacim.im_influence_noalloc(ctx.h, gr.h, pacim.IM_PROB_PER_EDGE,
                                   np.full(small.m_dir, 0.1), [1], 1, 0, 10)
    assert e.value.status == pacim.IM_EINVAL
    with pytest.raises(pacim.ImError) as e:
        gr.influence_noalloc(U, 0.5, [small.n], 1, 0, 10)
    assert e.value.status == pacim.IM_EINVAL
    gr.close()
    # 6,000,000 isolated vertices: one world needs 72 MB of forests, beyond the 64 MiB array
    n = 6_000_000
    huge = inputs.Graph(n, np.zeros(n + 1, dtype=np.uint64), np.zeros(0, dtype=np.uint32))
    gh = upload(ctx, huge)
    with pytest.raises(pacim.ImError) as e:
        gh.influence_noalloc(U, 0.5, [0, 5], 1, 0, 10)
    assert e.value.status == pacim.IM_EINVAL
    assert gh.influence(U, 0.5, [0, 5], 1, 0, 10) == 20
    gh.close()

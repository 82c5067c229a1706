"""GPU parity: the HIP path, called through the C-ABI, against the oracle.

Integer results, so the bar is bit-exact: labels, sizes, compact triples,
initial gains, seed sequences and gains.  Sizes span several tiles, ragged
tails (n not a multiple of 64, R not a multiple of the sketches per pass) and
the degenerate cases (p = 0, p = 1, k = n, tiny n).
"""
import os

import numpy as np
import pytest

import oracle
from paper_2311_07554_amd import inputs, pacim
from tests.gpu_util import run_select, upload

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


def test_er_small_full_labels_and_seeds(ctx):
    g = inputs.er_graph(1000, 5000, seed=1)
    R, k, seed, p = 64, 10, 1, 0.05
    _say("case er_small n=1000 R=64 k=10")
    lab, siz = oracle.sketches(g, 0, p, seed, R)
    gr = upload(ctx, g)
    sk = gr.sketches(U, p, R, seed, 1.0)
    for r in range(R):
        gl, gs = sk.dump(r)
        assert np.array_equal(gl, lab[r]), r
        assert np.array_equal(gs, siz[r]), r
    assert np.array_equal(sk.initial_gains(), siz.astype(np.uint64).sum(axis=0))
    s, gn = sk.select(k)
    ws, wg = oracle.greedy(lab, siz, k)
    assert np.array_equal(s, ws) and np.array_equal(gn, wg)
    sk.close()
    gr.close()


@pytest.mark.parametrize("scale,kind,p,R,k", [
    (12, TRI, 0.0, 40, 25),      # R below one pass
    (13, U, 0.05, 70, 30),       # R above one pass with a ragged last pass (B forced to 32)
    (14, TRI, 0.0, 64, 40),
])
def test_rmat_full_matches_oracle(ctx, scale, kind, p, R, k, monkeypatch):
    monkeypatch.setenv("PACIM_SKETCHES_PER_PASS", "32")
    g = inputs.rmat_graph(scale, 16 << scale, seed=scale)
    seed = 7
    _say(f"case rmat{scale} kind={kind} R={R} k={k}")
    lab, siz = oracle.sketches(g, kind, p, seed, R, threads=8)
    ws, wg = oracle.greedy(lab, siz, k)
    s, gn, st = run_select(ctx, g, kind, p, R, k, seed)
    assert np.array_equal(s, ws) and np.array_equal(gn, wg)
    assert st["sketches_per_pass"] == min(32, R)


@pytest.mark.parametrize("alpha", [0.1, 0.3, 0.02])
def test_rmat_compact_matches_oracle(ctx, alpha):
    scale, R, k, seed = 12, 32, 20, 3
    g = inputs.rmat_graph(scale, 16 << scale, seed=21)
    _say(f"case compact rmat{scale} alpha={alpha}")
    lab, siz = oracle.sketches(g, TRI, 0.0, seed, R, threads=8)
    cents = oracle.centers(g.n, seed, alpha)
    lc, sc = oracle.compact_all(lab, siz, cents)
    gr = upload(ctx, g)
    sk = gr.sketches(TRI, 0.0, R, seed, alpha)
    assert np.array_equal(sk.centers(), cents)
    for r in range(R):
        gl, gs = sk.dump(r)
        assert np.array_equal(gl, lc[r]) and np.array_equal(gs, sc[r]), r
    assert np.array_equal(sk.initial_gains(), siz.astype(np.uint64).sum(axis=0))
    s, gn = sk.select(k)
    ws, wg = oracle.greedy(lab, siz, k)   # alpha-equivalence: compact result = full result
    assert np.array_equal(s, ws) and np.array_equal(gn, wg)
    st = sk.stats()
    _say("  evaluations", st["evaluations"], "overflow", st["bfs_overflow"])
    sk.close()
    gr.close()


@pytest.mark.parametrize("width", ["6", "8"])
def test_pass_width_matches_oracle(ctx, width, monkeypatch):
    # scratch rows of 6 and 8 entries: the set-up writes a row in 16-byte pieces only
    # when the width is a multiple of 4 (8), entry by entry otherwise (6); 20
    # sketches in passes of 6, 6, 6, 2 or 8, 8, 4; full labels, CompactSketch, and
    # simulated influence over 7 worlds (rows of 6, or of 7 where passes hold 8)
    monkeypatch.setenv("PACIM_SKETCHES_PER_PASS", width)
    g = inputs.rmat_graph(11, 8 << 11, seed=41)
    R, k, seed, p = 20, 10, 9, 0.1
    _say(f"case pass width {width}")
    lab, siz = oracle.sketches(g, U, p, seed, R, threads=8)
    ws, wg = oracle.greedy(lab, siz, k)
    gr = upload(ctx, g)
    try:
        sk = gr.sketches(U, p, R, seed, 1.0)
        assert sk.stats()["sketches_per_pass"] == int(width)
        for r in range(R):
            gl, gs = sk.dump(r)
            assert np.array_equal(gl, lab[r]) and np.array_equal(gs, siz[r]), r
        s, gn = sk.select(k)
        sk.close()
        assert np.array_equal(s, ws) and np.array_equal(gn, wg)
        cents = oracle.centers(g.n, seed, 0.3)
        lc, sc = oracle.compact_all(lab, siz, cents)
        sk = gr.sketches(U, p, R, seed, 0.3)
        for r in range(R):
            cl, cz = sk.dump(r)
            assert np.array_equal(cl, lc[r]) and np.array_equal(cz, sc[r]), r
        s, gn = sk.select(k)
        sk.close()
        assert np.array_equal(s, ws) and np.array_equal(gn, wg)
        assert gr.influence(U, p, [int(x) for x in ws[:3]], 3, 5, 7) == \
            oracle.influence(g, U, p, [int(x) for x in ws[:3]], 3, 5, 7, threads=8)
    finally:
        gr.close()


@pytest.mark.parametrize("policy,cap", [("always", None), ("never", None), ("auto", None), ("always", "1"),
                                        ("auto", "1")])
def test_compact_bulk_rounds_match_oracle(ctx, policy, cap, monkeypatch):
    # uniform p = 0.1 on R-MAT gives a giant component, so the first seed covers a
    # large share of every sketch and "auto" switches the next round to bulk.
    # cap "1": a seed's component outside its sketch's largest one makes the bulk
    # round re-derive the sketches instead of using the build's bitmaps.
    monkeypatch.setenv("PACIM_BULK", policy)
    if cap is not None:
        monkeypatch.setenv("PACIM_BULK_SEARCH_CAP", cap)
    g = inputs.rmat_graph(12, 16 << 12, seed=31)
    R, k, seed, alpha = 32, 25, 5, 0.1
    _say(f"case compact bulk={policy} cap={cap}")
    lab, siz = oracle.sketches(g, U, 0.1, seed, R, threads=8)
    ws, wg = oracle.greedy(lab, siz, k)
    s, gn, st = run_select(ctx, g, U, 0.1, R, k, seed, alpha=alpha)
    assert np.array_equal(s, ws) and np.array_equal(gn, wg)
    _say("  bulk rounds", st["bulk_rounds"], "re-derived", st["bulk_resampled"])
    if policy == "always" and cap == "1":
        assert st["bulk_resampled"] >= 1
    if policy == "always":
        assert st["bulk_rounds"] == k - 1
    elif policy == "never":
        assert st["bulk_rounds"] == 0
    else:
        assert st["bulk_rounds"] >= 1
    s2, g2, _ = run_select(ctx, g, U, 0.1, R, k, seed, alpha=alpha, chunks=[1, 3, 21])
    assert np.array_equal(s2, ws) and np.array_equal(g2, wg)


def test_compact_overflow_path_exact(ctx):
    # p = 1 on a long path: one component of 3000 vertices and a tiny alpha, so
    # GetCenter searches outgrow the on-chip queue and take the global-memory path.
    n = 3000
    g = inputs.csr_from_pairs(n, [(i, i + 1) for i in range(n - 1)] + [(5000 % n, 17)])
    R, k, seed, alpha = 4, 3, 2, 0.0005
    lab, siz = oracle.sketches(g, U, 1.0, seed, R)
    ws, wg = oracle.greedy(lab, siz, k)
    s, gn, st = run_select(ctx, g, U, 1.0, R, k, seed, alpha=alpha)
    assert np.array_equal(s, ws) and np.array_equal(gn, wg)
    assert st["bfs_overflow"] > 0


def test_degenerate_probabilities(ctx):
    g = inputs.er_graph(300, 900, seed=4)
    s, gn, _ = run_select(ctx, g, U, 0.0, 8, 5, 1)          # no live edge
    assert list(s) == [0, 1, 2, 3, 4] and list(gn) == [8] * 5
    comps = [[7, 8, 9], [0, 1], [2, 3, 4, 5, 6], [10, 11, 12], [13]]
    pairs = [(a, b) for c in comps for i, a in enumerate(c) for b in c[i + 1:]]
    g = inputs.csr_from_pairs(14, pairs)
    for alpha in (1.0, 0.5):
        s, gn, _ = run_select(ctx, g, U, 1.0, 4, 14, 9, alpha=alpha)   # k = n: every vertex
        assert list(s) == [2, 7, 10, 0, 13, 1, 3, 4, 5, 6, 8, 9, 11, 12]
        assert list(gn) == [20, 12, 12, 8, 4] + [0] * 9


def test_tiny_graphs(ctx):
    for n in (1, 2, 5, 63, 64, 65, 4097):
        pairs = [(i, (i * 7 + 3) % n) for i in range(n) if n > 1 and i != (i * 7 + 3) % n]
        g = inputs.csr_from_pairs(n, pairs)
        k = min(n, 4)
        lab, siz = oracle.sketches(g, U, 0.5, 3, 5)
        ws, wg = oracle.greedy(lab, siz, k)
        s, gn, _ = run_select(ctx, g, U, 0.5, 5, k, 3)
        assert np.array_equal(s, ws) and np.array_equal(gn, wg), n


def test_edgeless_graph(ctx):
    # every vertex isolated: no linked vertex, every component a singleton
    g = inputs.csr_from_pairs(70, [])
    lab, siz = oracle.sketches(g, U, 0.5, 2, 6)
    ws, wg = oracle.greedy(lab, siz, 10)
    for alpha in (1.0, 0.3):
        s, gn, _ = run_select(ctx, g, U, 0.5, 6, 10, 2, alpha=alpha)
        assert np.array_equal(s, ws) and np.array_equal(gn, wg), alpha
    assert list(ws) == list(range(10)) and set(wg.tolist()) == {6}


def test_resume_equals_one_shot(ctx):
    g = inputs.rmat_graph(12, 16 << 12, seed=5)
    a = run_select(ctx, g, TRI, 0.0, 24, 30, 11)
    b = run_select(ctx, g, TRI, 0.0, 24, 30, 11, chunks=[7, 1, 22])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    c = run_select(ctx, g, TRI, 0.0, 24, 30, 11, alpha=0.2, chunks=[10, 20])
    assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])


@pytest.mark.parametrize("step", ["1", "3", "200"])
def test_persistent_handoff_matches_oracle(ctx, step, monkeypatch):
    # The persistent selection kernel hands a round to the per-level kernels when an
    # evaluation step exceeds its limit; lowering the limit forces hand-overs at
    # every level (step 1), at some levels (3), or only for CompactSketch (200).
    monkeypatch.setenv("PACIM_PERSIST_STEP", step)
    g = inputs.rmat_graph(12, 16 << 12, seed=17)
    R, k, seed = 24, 30, 6
    _say(f"case persistent hand-off step={step}")
    lab, siz = oracle.sketches(g, TRI, 0.0, seed, R)
    ws, wg = oracle.greedy(lab, siz, k)
    for alpha in (1.0, 0.2):
        s, gn, _ = run_select(ctx, g, TRI, 0.0, R, k, seed, alpha=alpha, chunks=[5, 25])
        assert np.array_equal(s, ws) and np.array_equal(gn, wg), alpha


def test_per_level_rounds_match_oracle(ctx, monkeypatch):
    # without the persistent kernel (where a cooperative launch is refused) every
    # lazy round runs as per-level kernels
    monkeypatch.setenv("PACIM_PERSIST", "0")
    g = inputs.rmat_graph(12, 16 << 12, seed=19)
    R, k, seed = 24, 20, 8
    _say("case per-level rounds")
    lab, siz = oracle.sketches(g, TRI, 0.0, seed, R)
    ws, wg = oracle.greedy(lab, siz, k)
    for alpha in (1.0, 0.2):
        s, gn, _ = run_select(ctx, g, TRI, 0.0, R, k, seed, alpha=alpha, chunks=[3, 17])
        assert np.array_equal(s, ws) and np.array_equal(gn, wg), alpha


def test_deterministic_repeats(ctx):
    g = inputs.rmat_graph(13, 16 << 13, seed=8)
    ref = run_select(ctx, g, TRI, 0.0, 48, 20, 2)
    for _ in range(4):
        got = run_select(ctx, g, TRI, 0.0, 48, 20, 2)
        assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])


def test_invalid_arguments(ctx):
    lib = pacim
    g = inputs.er_graph(50, 100, seed=2)
    with pytest.raises(pacim.ImError) as e:
        bad = g.cols.copy()
        bad[0] = 999
        ctx.graph(g.n, g.offsets, bad)
    assert e.value.status == pacim.IM_EINVAL
    with pytest.raises(pacim.ImError):
        loop = inputs.csr_from_pairs(3, [(0, 1)])
        cols = loop.cols.copy()
        cols[0] = 0
        ctx.graph(3, loop.offsets, cols)
    asym = (np.array([0, 1, 1], dtype=np.uint64), np.array([1], dtype=np.uint32))
    with pytest.raises(pacim.ImError):
        ctx.graph(2, *asym)
    gr = upload(ctx, g)
    with pytest.raises(pacim.ImError):
        gr.sketches(U, 1.5, 4, 1)
    with pytest.raises(pacim.ImError):
        gr.sketches(U, 0.1, 0, 1)
    with pytest.raises(pacim.ImError):
        gr.sketches(U, 0.1, 4, 1, alpha=0.0)
    sk = gr.sketches(U, 0.1, 4, 1)
    with pytest.raises(pacim.ImError) as e:
        sk.select(51)
    assert e.value.status == pacim.IM_EINVAL
    sk.select(50)
    sk.close()
    gr.close()
    assert lib.im_ctx_memory(ctx.h)[0] == 0


def test_size_limits_rejected_before_device_work(ctx):
    # the build's size limits (keys of ceil(log2(R*n+2)) + ceil(log2 n) <= 64 bits;
    # CompactSketch: R*n < 2^40 and R < 2^24) are refused with EINVAL before any
    # allocation, on an edgeless graph of 2^20 vertices and a small one
    big = inputs.csr_from_pairs(1 << 20, [])
    gr = upload(ctx, big)
    small = upload(ctx, inputs.er_graph(50, 100, seed=2))
    try:
        for g_, R, alpha in [(gr, (1 << 32) - 1, 1.0), (gr, 1 << 20, 0.5), (small, 1 << 24, 0.5)]:
            with pytest.raises(pacim.ImError) as e:
                g_.sketches(U, 0.1, R, 1, alpha)
            assert e.value.status == pacim.IM_EINVAL, (R, alpha)
        assert pacim.im_ctx_memory(ctx.h)[0] > 0  # the two graphs only
    finally:
        gr.close()
        small.close()
    assert pacim.im_ctx_memory(ctx.h)[0] == 0


def test_zero_seed_requests(ctx):
    # k = 0 is a valid request on every path: nothing is selected and the handle's
    # state is unchanged (the next k seeds are the oracle's first k)
    g = inputs.er_graph(300, 1200, seed=5)
    R, k, seed, p = 16, 6, 3, 0.2
    _say("case k = 0 requests")
    lab, siz = oracle.sketches(g, U, p, seed, R)
    ws, wg = oracle.greedy(lab, siz, k)
    gr = upload(ctx, g)
    try:
        for alpha in (1.0, 0.3):
            sk = gr.sketches(U, p, R, seed, alpha)
            for sel in (sk.select, sk.select_ptree):
                s0, g0 = sel(0)
                assert s0.size == 0 and g0.size == 0
            s, gn = sk.select(k)
            assert np.array_equal(s, ws) and np.array_equal(gn, wg), alpha
            s0, g0 = sk.select_ptree(0)
            assert s0.size == 0 and g0.size == 0
            sk.close()
        res, _ = ctx.select_batched([(gr, U, p, R, 0, seed), (gr, U, p, R, k, seed), (gr, U, p, R, 0, seed, 0.3)])
        assert res[0][0].size == 0 and res[0][1].size == 0 and res[2][0].size == 0
        assert np.array_equal(res[1][0], ws) and np.array_equal(res[1][1], wg)
        assert ctx.select_batched([])[0] == []
    finally:
        gr.close()


def test_module_level_select_from_torch_tensors():
    # CSR handed over as device tensors on torch's current stream; full labels and CompactSketch
    import torch
    g = inputs.rmat_graph(11, 16 << 11, seed=44)
    off = torch.from_numpy(g.offsets.view(np.int64)).cuda()
    cols = torch.from_numpy(g.cols.view(np.int32)).cuda()
    lab, siz = oracle.sketches(g, TRI, 0.0, 3, 24, threads=8)
    ws, wg = oracle.greedy(lab, siz, 12)
    for alpha in (1.0, 0.25):
        s, gn = pacim.select_seeds(off, cols, TRI, 0.0, 24, 12, 3, alpha=alpha)
        assert np.array_equal(s, ws) and np.array_equal(gn, wg), alpha


@pytest.mark.parametrize("hubs", ["0", "1", "300", "1000000"])
def test_labelling_order_does_not_change_results(ctx, hubs, monkeypatch):
    # the union-find passes number vertices hubs-first, then linked, then isolated;
    # labels (smallest id), sizes, triples, seeds and gains must not depend on it:
    # no hubs, one, some, and every linked vertex a hub
    # three passes of 32, 32 and 6 sketches: isolated vertices are set up by the first only
    monkeypatch.setenv("PACIM_HUBS", hubs)
    monkeypatch.setenv("PACIM_SKETCHES_PER_PASS", "32")
    g = inputs.rmat_graph(12, 8 << 12, seed=31)
    assert (np.diff(g.offsets.astype(np.int64)) == 0).any()  # isolated vertices present
    R, k, seed, p = 70, 15, 5, 0.08
    _say(f"case labelling order hubs={hubs}")
    lab, siz = oracle.sketches(g, U, p, seed, R, threads=8)
    ws, wg = oracle.greedy(lab, siz, k)
    gr = upload(ctx, g)
    try:
        sk = gr.sketches(U, p, R, seed, 1.0)
        for r in (0, 11, 40, R - 1):
            gl, gs = sk.dump(r)
            assert np.array_equal(gl, lab[r]) and np.array_equal(gs, siz[r]), r
        s, gn = sk.select(k)
        sk.close()
        assert np.array_equal(s, ws) and np.array_equal(gn, wg)
        cents = oracle.centers(g.n, seed, 0.2)
        lc, sc = oracle.compact_all(lab, siz, cents)
        sk = gr.sketches(U, p, R, seed, 0.2)
        for r in (0, 33, R - 1):
            cl, cz = sk.dump(r)
            assert np.array_equal(cl, lc[r]) and np.array_equal(cz, sc[r]), r
        s, gn = sk.select(k)
        sk.close()
        assert np.array_equal(s, ws) and np.array_equal(gn, wg)
    finally:
        gr.close()

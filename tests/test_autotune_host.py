"""Host logic of the batched-launch autotuner, with a stand-in context whose
launch times are given: the search order, the chosen shape and the cache."""
from types import SimpleNamespace

import pytest

from paper_2311_07554_amd import autotune


class FakeCtx:
    """select_batched returns a device time that is lowest at hook block 512,
    selection block 256 and sampling grid 4096 (the selection grid does not
    matter); records every configuration it was asked for."""

    def __init__(self, forbid=False):
        self.calls = []
        self.forbid = forbid

    def select_batched(self, queries, cfg):
        if self.forbid:
            raise AssertionError("a cached shape must not be measured again")
        self.calls.append(dict(cfg))
        hb, sb, hg = cfg["hook_block"], cfg["select_block"], cfg.get("hook_grid", 0)
        return None, abs(hb - 512) / 64.0 + abs(sb - 256) / 256.0 + (0.0 if hg == 4096 else 0.5) + 1.0


def _queries(n=1000):
    g = SimpleNamespace(n=n, m_und=4 * n)
    return [(g, 1, 0.0, 64, 10, 1), (g, 0, 0.05, 32, 5, 2)]


def test_search_picks_the_fastest_shape():
    ctx = FakeCtx()
    cfg, table = autotune.tune(ctx, _queries(), repeats=2, use_cache=False)
    # the selection grid is a tie everywhere: its first candidate stays
    assert cfg == {"hook_block": 512, "hook_grid": 4096, "select_block": 256, "select_grid": 0}
    # one axis at a time, in order, from the starting shape: the sampling blocks first
    firsts = [c["hook_block"] for c in ctx.calls[::2][:len(autotune.HOOK_BLOCKS)]]
    assert firsts == list(autotune.HOOK_BLOCKS)
    assert table[0]["config"] == autotune.START
    # every candidate differs from the best shape so far in one axis, visited in order
    axes = [name for name, _ in autotune.AXES]
    best, best_t, seen = dict(table[0]["config"]), table[0]["device_ms"], []
    for t in table[1:]:
        diff = [k for k in axes if t["config"][k] != best[k]]
        assert len(diff) == 1, (t, best)
        seen.append(axes.index(diff[0]))
        if t["device_ms"] < best_t:
            best, best_t = dict(t["config"]), t["device_ms"]
    assert seen == sorted(seen) and best == cfg
    assert len(table) == 1 + sum(len(c) - 1 for _, c in autotune.AXES)
    assert len(ctx.calls) == 2 * len(table)  # best of `repeats` per candidate


def test_cache_keyed_by_device_and_batch(tmp_path, monkeypatch):
    monkeypatch.setenv("PACIM_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    cfg1, _ = autotune.tune(FakeCtx(), _queries(), device_name="dev0")
    cfg2, table2 = autotune.tune(FakeCtx(forbid=True), _queries(), device_name="dev0")
    assert cfg1 == cfg2 and table2
    with pytest.raises(AssertionError):  # another batch shape is measured
        autotune.tune(FakeCtx(forbid=True), _queries(n=2000), device_name="dev0")
    with pytest.raises(AssertionError):  # and so is another device
        autotune.tune(FakeCtx(forbid=True), _queries(), device_name="dev1")


def test_signature_depends_on_every_query_field():
    base = autotune.signature(_queries())
    g = SimpleNamespace(n=1000, m_und=4000)
    variants = [
        [(g, 1, 0.0, 64, 10, 1), (g, 0, 0.05, 32, 6, 2)],   # k
        [(g, 1, 0.0, 64, 10, 1), (g, 0, 0.06, 32, 5, 2)],   # p
        [(g, 1, 0.0, 128, 10, 1), (g, 0, 0.05, 32, 5, 2)],  # R
        [(g, 0, 0.0, 64, 10, 1), (g, 0, 0.05, 32, 5, 2)],   # model
    ]
    sigs = {autotune.signature(v) for v in variants}
    assert base not in sigs and len(sigs) == len(variants)
    # the sampling seed does not change the launch shape
    assert autotune.signature([(g, 1, 0.0, 64, 10, 9), (g, 0, 0.05, 32, 5, 7)]) == base

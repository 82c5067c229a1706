"""Host logic of the batched-launch autotuner, with a stand-in context whose
launch times are given: the search order, the chosen shape and the cache."""
from types import SimpleNamespace

import pytest

from paper_2311_07554_amd import autotune


class FakeCtx:
    """select_batched returns a device time that is lowest at hook block 512 and
    selection block 256; records every configuration it was asked for."""

    def __init__(self, forbid=False):
        self.calls = []
        self.forbid = forbid

    def select_batched(self, queries, cfg):
        if self.forbid:
            raise AssertionError("a cached shape must not be measured again")
        self.calls.append(dict(cfg))
        hb, sb = cfg["hook_block"], cfg["select_block"]
        return None, abs(hb - 512) / 64.0 + abs(sb - 256) / 256.0 + 1.0


def _queries(n=1000):
    g = SimpleNamespace(n=n, m_und=4 * n)
    return [(g, 1, 0.0, 64, 10, 1), (g, 0, 0.05, 32, 5, 2)]


def test_search_picks_the_fastest_shape():
    ctx = FakeCtx()
    cfg, table = autotune.tune(ctx, _queries(), repeats=2, use_cache=False)
    assert cfg == {"hook_block": 512, "select_block": 256}
    # sampling blocks first with the selection block fixed, then the other selection blocks
    firsts = [c["hook_block"] for c in ctx.calls[::2][:len(autotune.HOOK_BLOCKS)]]
    assert firsts == list(autotune.HOOK_BLOCKS)
    assert len(table) == len(autotune.HOOK_BLOCKS) + len(autotune.SELECT_BLOCKS) - 1
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

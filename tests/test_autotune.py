"""The launch-shape autotuner's selection and cache (host logic, no GPU), and
the tuning entry point's argument checks."""
import pytest

from paper_2405_19994_amd import autotune
from paper_2405_19994_amd import hsdc as H


class _FakeContext:
    """Stands in for a context: a step costs what the candidate's table says."""
    cost = {}
    clock = [0.0]

    def __init__(self):
        self.setting = None

    def tune(self, blocks, margin):
        self.setting = (blocks, margin)

    def advance(self, n):
        _FakeContext.clock[0] += n * _FakeContext.cost[self.setting]

    def destroy(self):
        pass


def test_tuner_picks_fastest_and_caches(tmp_path, monkeypatch):
    monkeypatch.setenv("HSDC_TUNE_CACHE", str(tmp_path / "t.json"))
    monkeypatch.setattr(autotune.time, "perf_counter", lambda: _FakeContext.clock[0])
    _FakeContext.cost = {(b, m): 1.0 + 0.01 * abs(b - 256) + 0.1 * m
                         for b in autotune.CG_BLOCKS for m in autotune.CG_MARGINS}
    p = H.make_problem((64, 48), 0.025)
    m = H.make_method(M=6, max_iter=6)
    key = autotune.shape_key(p, m)
    best, timings = autotune.tune(_FakeContext, key, sync=lambda: None)
    assert best == {"cg_blocks": 256, "cg_margin": -1}
    # within the noise margin of the default, the default is kept
    d = (autotune.DEFAULT["cg_blocks"], autotune.DEFAULT["cg_margin"])
    _FakeContext.cost[d] = 0.99 * _FakeContext.cost[(256, -1)]
    _FakeContext.cost[(256, -1)] = 0.985 * _FakeContext.cost[d]
    kept, _ = autotune.tune(_FakeContext, key + "b", sync=lambda: None, use_cache=False)
    assert kept == autotune.DEFAULT
    assert len(timings) == len(autotune.CG_BLOCKS) * len(autotune.CG_MARGINS)
    # a second call is served from the cache without timing
    again, t2 = autotune.tune(_FakeContext, key, sync=lambda: None)
    assert again == best and t2 is None
    ctx = _FakeContext()
    assert autotune.apply(ctx, key) == best and ctx.setting == (256, -1)
    # another shape has its own entry (defaults until tuned)
    other = autotune.shape_key(H.make_problem((64, 50), 0.025), m)
    assert other != key and autotune.lookup(other) is None
    assert autotune.apply(_FakeContext(), other) == autotune.DEFAULT


def test_tune_entry_point_rejects_null_context():
    assert H.lib().hsdc_tune(None, 256, 2) == -1

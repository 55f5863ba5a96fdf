"""The launch-shape autotuner's selection and cache (host logic, no GPU), and
the tuning entry points' argument checks."""
import ctypes

import pytest

from paper_2405_19994_amd import autotune
from paper_2405_19994_amd import hsdc as H


class _FakeContext:
    """Stands in for a context: a step costs what the cost function says of
    the launch setting applied to it."""
    cost = staticmethod(lambda s: 1.0)
    clock = [0.0]

    def __init__(self):
        self.setting = dict(autotune.DEFAULT)

    def tune(self, blocks, margin):
        self.setting.update(cg_blocks=blocks, cg_margin=margin)

    def tune_shapes(self, node_block, cg_tile, prolong_tile):
        self.setting.update(node_block=node_block, cg_tile=cg_tile, prolong_tile=prolong_tile)

    def advance(self, n):
        _FakeContext.clock[0] += n * _FakeContext.cost(self.setting)

    def destroy(self):
        pass


def _cost(s):
    return (1.0 + 0.03 * abs(s["cg_blocks"] - 256) / 128 + 0.1 * (s["cg_margin"] + 1)
            + {64: 0.0, 128: 0.05, 256: 0.08, 512: 0.2}[s["node_block"]]
            + (0.0 if s["cg_tile"] == 3 else 0.06) + 0.001 * s["prolong_tile"])


def test_tuner_picks_fastest_per_axis_and_caches(tmp_path, monkeypatch):
    monkeypatch.setenv("HSDC_TUNE_CACHE", str(tmp_path / "t.json"))
    monkeypatch.setattr(autotune.time, "perf_counter", lambda: _FakeContext.clock[0])
    _FakeContext.cost = staticmethod(_cost)
    p = H.make_problem((64, 48), 0.025)
    m = H.make_method(M=6, max_iter=6)
    key = autotune.shape_key(p, m)
    axes = autotune.relevant_axes(p, m)
    assert axes == ("cg", "node_block", "cg_tile")  # 2D, one level: no correction tile
    best, timings = autotune.tune(_FakeContext, key, axes=axes, sync=lambda: None)
    assert best == dict(autotune.DEFAULT, cg_blocks=256, node_block=64, cg_tile=3)
    # one timing per distinct setting: the CG grid, then each shape axis (the
    # default start tile, -1, is the library's choice for the mesh, which the
    # explicit tiles 0..8 are timed against)
    n_cg = len(autotune.CG_BLOCKS) * len(autotune.CG_MARGINS)
    assert autotune.DEFAULT["cg_tile"] == -1
    assert len(timings) == n_cg + (len(autotune.NODE_BLOCKS) - 1) + len(autotune.CG_TILES)
    # a second call is served from the cache without timing
    again, t2 = autotune.tune(_FakeContext, key, axes=axes, sync=lambda: None)
    assert again == best and t2 is None
    ctx = _FakeContext()
    assert autotune.apply(ctx, key) == best and ctx.setting == best
    # another shape has its own entry (defaults until tuned)
    other = autotune.shape_key(H.make_problem((64, 50), 0.025), m)
    assert other != key and autotune.lookup(other) is None
    assert autotune.apply(_FakeContext(), other) == autotune.DEFAULT


def test_tuner_keeps_the_default_within_the_noise_margin(monkeypatch):
    monkeypatch.setattr(autotune.time, "perf_counter", lambda: _FakeContext.clock[0])
    d = autotune.DEFAULT
    # every other setting 1.5% faster than the default: not enough to switch
    _FakeContext.cost = staticmethod(lambda s: 1.0 if s == d else 0.985)
    kept, _ = autotune.tune(_FakeContext, "k", use_cache=False, sync=lambda: None)
    assert kept == d


def test_relevant_axes_by_problem_shape():
    m3 = H.make_method(M=(6, 3), levels=2, space_coarsen=2, P=4)
    assert autotune.relevant_axes(H.make_problem((8, 6, 4), 0.025), m3) == \
        ("cg", "node_block", "prolong_tile")
    assert autotune.relevant_axes(H.make_problem((16, 12), 0.025), H.make_method(M=4, solver=2)) \
        == ("cg", "node_block")


def test_tune_entry_points_reject_bad_arguments():
    L = H.lib()
    assert L.hsdc_tune(None, 256, 2) == -1
    assert L.hsdc_tune_shapes(None, 256, 0, 0) == -1
    assert b"NULL" in L.hsdc_last_error(None)

"""Launch-shape autotuner for libhsdc.

The CG kernels are latency bound on small meshes and bandwidth bound on large
ones, the spare iterations of a predicted CG budget trade a no-op launch
against the risk of recomputing a step, and the block and tile shapes of the
node update, the one-launch CG start and the coarse-to-fine correction decide
how many compute units a small mesh fills and how much halo a tile re-reads.
For one problem shape the tuner times a few steps per candidate on fresh
contexts, one launch parameter at a time with the others at the best found so
far (CG block cap and budget margin together, then the node-update block, the
CG-start tile, the correction tile), keeps a candidate only when it beats the
current setting by more than the noise margin, and caches the result per
shape key, so that later runs of the same shape apply it without timing
anything.  Tuning changes launch shapes only: results agree up to the order of
the reductions over blocks and tiles.

The cache is a JSON file, by default ~/.cache/paper_2405_19994_amd/tuning.json
(HSDC_TUNE_CACHE overrides the path).
"""
import json
import os
import time

CG_BLOCKS = (128, 256, 512, 1024)
# -1: the library's default margin (none after the tiled CG start, one otherwise)
CG_MARGINS = (-1, 1, 2)
NODE_BLOCKS = (64, 128, 256, 512)
CG_TILES = (0, 1, 2, 3, 4, 5, 6, 7, 8)  # include/hsdc.h, hsdc_tune_shapes: 64x16 .. 48x32
PROLONG_TILES = (0, 1, 2, 3)
# cg_tile -1: the library's default tile for the mesh (hsdc_tune_shapes keeps it)
DEFAULT = {"cg_blocks": 512, "cg_margin": -1, "node_block": 256, "cg_tile": -1, "prolong_tile": 0}
# the order in which launch parameters are tuned; each group is timed with the
# others at the best setting found so far
AXES = ("cg", "node_block", "cg_tile", "prolong_tile")


def cache_path():
    return os.environ.get("HSDC_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_2405_19994_amd", "tuning.json")


def shape_key(problems, method):
    """Mesh sizes, per-node sigma, stepping and level structure: what decides
    the launch shapes of a context."""
    probs = problems if isinstance(problems, (list, tuple)) else [problems]
    dims = sorted((p.nx, p.ny, p.nz) for p in probs)
    pernode = bool(probs[0].sigma_node)
    return json.dumps({"dims": dims if len(dims) <= 4 else [len(dims), dims[0], dims[-1]],
                       "pernode": pernode, "levels": method.levels, "M": list(method.M),
                       "P": method.P, "sweeps": method.max_iter,
                       "coarsen": method.space_coarsen, "fp32": method.coarse_fp32},
                      sort_keys=True)


def _load():
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(table):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(key):
    """Cached setting for key, or None."""
    return _load().get(key)


def relevant_axes(problems, method):
    """The launch parameters that matter for a context of this shape: the
    CG-start tile on 2D meshes with CG from its Chebyshev start, the
    correction tile with a space-coarsened second level."""
    probs = problems if isinstance(problems, (list, tuple)) else [problems]
    axes = ["cg", "node_block"]
    if probs[0].dim == 2 and method.solver == 0:
        axes.append("cg_tile")
    if method.levels == 2 and method.space_coarsen == 2:
        axes.append("prolong_tile")
    return tuple(axes)


def _candidates(axis, cur):
    if axis == "cg":
        return [dict(cur, cg_blocks=b, cg_margin=m) for b in CG_BLOCKS for m in CG_MARGINS]
    values = {"node_block": NODE_BLOCKS, "cg_tile": CG_TILES, "prolong_tile": PROLONG_TILES}[axis]
    return [dict(cur, **{axis: v}) for v in values]


def _apply(ctx, s):
    s = dict(DEFAULT, **s)
    ctx.tune(s["cg_blocks"], s["cg_margin"])
    ctx.tune_shapes(s["node_block"], s["cg_tile"], s["prolong_tile"])
    return s


def tune(make_context, key, steps=6, warm=2, axes=AXES, use_cache=True, sync=None,
         min_gain=0.02):
    """For each launch parameter of `axes` in turn, time `steps` steps after
    `warm` untimed ones on a fresh context from make_context() for every
    candidate value; return (best setting, timings).  A candidate replaces the
    current setting only when it is faster by more than min_gain (relative),
    so timing noise does not pick the launch shapes.

    sync: callable that waits for the device (torch.cuda.synchronize)."""
    if use_cache:
        hit = lookup(key)
        if hit is not None:
            return dict(DEFAULT, **hit), None
    if sync is None:
        import torch
        sync = torch.cuda.synchronize
    timings = []
    cache = {}

    def time_setting(s):
        k = json.dumps(s, sort_keys=True)
        if k not in cache:
            ctx = make_context()
            _apply(ctx, s)
            ctx.advance(warm)
            sync()
            t0 = time.perf_counter()
            ctx.advance(steps)
            sync()
            dt = time.perf_counter() - t0
            ctx.destroy()
            cache[k] = dt / steps
            timings.append(dict(s, s_per_step=cache[k]))
        return cache[k]

    best = dict(DEFAULT)
    for axis in axes:
        t_best = time_setting(best)
        for cand in _candidates(axis, best):
            t = time_setting(cand)
            if t < (1.0 - min_gain) * t_best:
                best, t_best = cand, t
    if use_cache:
        table = _load()
        table[key] = best
        _store(table)
    return best, timings


def apply(ctx, key):
    """Apply the cached setting for key to ctx (the defaults when none)."""
    return _apply(ctx, lookup(key) or DEFAULT)

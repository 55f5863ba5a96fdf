"""Helpers shared by the parity tests: build matching oracle and library
problems from one workload description, move arrays, compare fields."""
import numpy as np

from oracle import ttp06
from oracle.hsdc import Level
from oracle.pfasst import Hierarchy
from oracle.problems import Monodomain
from oracle.tissue import coarse_dims, prolong_space, restrict_space


def oracle_problem(w, dims=None, dx=None):
    dims = tuple(dims or w["dims"])
    stim = w["stim_w"] if dims == tuple(w["dims"]) else restrict_space(w["stim_w"], w["dims"])
    return Monodomain(dims, dx or w["dx"], w["sigma"], w.get("sigma_node"), w["chi"], w["Cm"], stim,
                      w["stim_amp"], w["stim_t0"], w["stim_dur"], g_scale=w.get("g_scale", (1, 1, 1)),
                      dt_ref=w["dt"], fd_order=w.get("fd_order", 2))


def oracle_hierarchy(w, Mf, Mc, coarsen):
    pf = oracle_problem(w)
    fine = Level(pf, Mf, w["dt"])
    if coarsen == 2:
        pc = oracle_problem(w, coarse_dims(w["dims"]), 2 * w["dx"])
        dims = tuple(w["dims"])
        return Hierarchy([fine, Level(pc, Mc, w["dt"])],
                         space_restrict=[lambda u: restrict_space(u, dims)],
                         space_prolong=[lambda u: prolong_space(u, dims)])
    return Hierarchy([fine, Level(pf, Mc, w["dt"])])


def oracle_hierarchy_levels(w, Ms, coarsen):
    """Any number of levels: level l has Ms[l] nodes, on the mesh coarsened
    coarsen**l (coarsen 1: time only)."""
    dims = [tuple(w["dims"])]
    for _ in Ms[1:]:
        dims.append(coarse_dims(dims[-1]) if coarsen == 2 else dims[-1])
    levels, rs, ps = [], [], []
    stim = w["stim_w"]
    for l, M in enumerate(Ms):
        ww = dict(w)
        ww["dims"], ww["stim_w"] = dims[l], stim
        levels.append(Level(oracle_problem(ww, dims[l], w["dx"] * coarsen ** l), M, w["dt"]))
        if l + 1 < len(Ms) and coarsen == 2:
            d = dims[l]
            rs.append(lambda u, d=d: restrict_space(u, d))
            ps.append(lambda u, d=d: prolong_space(u, d))
            stim = restrict_space(stim, d)
    if coarsen == 2:
        return Hierarchy(levels, space_restrict=rs, space_prolong=ps)
    return Hierarchy(levels)


def rest(N):
    return np.repeat(ttp06.rest_state()[:, None], N, axis=1)


def field_errors(a, b):
    """Per field: max |a - b| / max |b| (relative to the field's magnitude)."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    scale = np.max(np.abs(b), axis=-1)
    scale = np.where(scale > 0, scale, 1.0)
    return np.max(np.abs(a - b), axis=-1) / scale

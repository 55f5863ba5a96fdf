"""Benchmark: SDC node-updates/s of serial hybrid SDC on the 2D slab workload.

Workload (512 x 512 nodes, dx 0.025 cm, 5-point Laplacian, sigma 1 mS/cm,
TTP06 epicardial rest state, 50 uA/cm^2 corner stimulus for 1 ms; 6 Radau IIA
nodes, 6 sweeps per step, dt 0.05 ms, CG to 1e-12).  One benchmark step is one
HSDC time step: 6 sweeps, each a forward substitution over the 6 collocation
nodes (fused cell-model / exponential-gating kernel + implicit diffusion CG
solve per node), the collocation-integral assembly, and the spread to the next
step.  node-updates = nodes x M x sweeps x steps.  Inputs are resident in HBM
before the timed region; the timed region starts at t = 0; the median of
--runs timed runs is reported.  The line also carries the fused cell-model
kernel's roofline (FP64 vector bound, with its HBM side), the diffusion
operator measured out of cache (8192 x 8192) against the HBM peak, and the
FP64 oracle timed on the host cores (a bounded sample; see cpu_baseline).

    python bench.py [--gpus 1] [--steps 400] [--warmup 20] [--runs 5]

With --workload slab3d: two-level PFASST (Algorithm 1) on the 192 x 96 x 48
slab (7-point, sigma (3, 1, 1), planar-face stimulus; 16 slices of dt 0.1 ms;
fine M 6 in FP64, coarse M 3 in FP32 on the 2x coarser mesh unless --coarse
fp64 / --coarsen 1), timed over --blocks blocks at a fixed per-field error
--eps against serial hybrid SDC swept to its collocation solution (K = 40),
beside serial hybrid SDC in FP64 at the fewest sweeps per step that reach the
same error.  The metric is simulated ms per wall second.

    python bench.py --workload slab3d [--blocks 2] [--coarsen 2] [--eps 1e-8]

With --workload batch2d: 64 independent 2D tissues (sides uniform in 64..512,
per-node lognormal sigma, an 8 x 8 stimulus patch each; M 4, K 4, dt 0.05 ms)
advanced as one ragged batch, every launch covering every tissue; reported
beside the same tissues stepped one context at a time.

    python bench.py --workload batch2d [--steps 50]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--runs", type=int, default=5,
                    help="slab2d: timed runs of --steps steps; the median run is reported")
    ap.add_argument("--no-spmv", action="store_true",
                    help="slab2d: skip the out-of-cache diffusion-operator measurement")
    ap.add_argument("--graph", action="store_true",
                    help="slab2d: replay each step from a captured HIP graph")
    ap.add_argument("--solver", choices=tuple(SOLVER_NAMES), default="cg",
                    help="diffusion solver (the slab workloads name CG): cg starts from "
                         "Chebyshev steps, cg_plain from the warm start; slab2d also times "
                         "the other solvers beside its line as an option study")
    ap.add_argument("--no-solver-option", action="store_true",
                    help="slab2d: skip timing the other diffusion solvers")
    ap.add_argument("--no-autotune", action="store_true",
                    help="slab2d: keep the default CG launch shapes instead of tuning them first")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 512 MiB device copy (counter calibration)")
    ap.add_argument("--workload", choices=("slab2d", "slab3d", "batch2d", "cable1d", "adjoint",
                                           "slab2d_fd4"),
                    default="slab2d")
    ap.add_argument("--tissues", type=int, default=64, help="batch2d: tissues in the batch")
    ap.add_argument("--side", type=int, default=512,
                    help="slab2d: mesh side (the metric is quoted on 512; other sides show how "
                         "the kernels scale with the mesh, without the CPU baseline and counters)")
    ap.add_argument("--summarize-valu", metavar="COUNTER_CSV",
                    help="write the VALU instruction counters (SQ_WAVES, SQ_INSTS_VALU and its "
                         "FP64 FMA/ADD/MUL/TRANS parts) of a rocprofv3 --pmc run into "
                         "profiles/valu_slab2d.json")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter_collection.csv files (FETCH_SIZE, "
                         "WRITE_SIZE) of a --calibrate-copy run into profiles/hbm_traffic_slab2d.json")
    ap.add_argument("--blocks", type=int, default=2, help="slab3d: PFASST blocks timed")
    ap.add_argument("--coarsen", type=int, choices=(1, 2), default=2,
                    help="slab3d: space coarsening factor of the coarse level")
    ap.add_argument("--eps", type=float, default=1e-8,
                    help="slab3d: per-field error both contenders are held to")
    ap.add_argument("--tols", type=float, nargs="+", default=[1e-8, 3e-9, 1e-9, 3e-10, 1e-10],
                    help="slab3d: per-field PFASST residual tolerances tried, loosest first")
    ap.add_argument("--max-iter", type=int, default=80, help="slab3d: PFASST iterations cap")
    ap.add_argument("--prefix-stop", action="store_true",
                    help="slab3d: slices whose residual, and every earlier slice's, is below tol "
                         "stop iterating (two levels)")
    ap.add_argument("--pfasst-only", action="store_true",
                    help="slab3d: time the PFASST blocks alone (no reference runs; for profilers)")
    ap.add_argument("--levels", type=int, choices=(2, 3), default=2,
                    help="slab3d: PFASST levels (3: M 6/3/1, FP64)")
    ap.add_argument("--coarse", choices=("fp32", "fp64"), default="fp32",
                    help="slab3d: precision of the coarse level's cell model, reaction terms and "
                         "CG vectors (the fine level, residual and tau stay FP64)")
    return ap.parse_args()


def _oracle_tile(args):
    """One worker of the CPU baseline: the oracle's serial HSDC on one tile of
    the slab (no-flux tile edges), single-threaded.  Returns (node-updates,
    seconds of its own compute)."""
    side, stimulated, nsteps = args
    import synthetic_inputs as si
    from oracle import ttp06
    from oracle.hsdc import Level, run_serial
    from oracle.problems import Monodomain

    ws = si.workload("slab2d", dims=(side, side))
    stim = ws["stim_w"] if stimulated else np.zeros(side * side)
    p = Monodomain(ws["dims"], ws["dx"], ws["sigma"], None, ws["chi"], ws["Cm"], stim,
                   ws["stim_amp"], ws["stim_t0"], ws["stim_dur"], dt_ref=ws["dt"])
    lev = Level(p, ws["M"], ws["dt"])
    y0 = np.repeat(ttp06.rest_state()[:, None], p.N, axis=1)
    t0 = time.perf_counter()
    run_serial(lev, y0, nsteps, ws["K"])
    return p.N * ws["M"] * ws["K"] * nsteps, time.perf_counter() - t0


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(nsteps=2, side=128):
    """The FP64 oracle on the host cores, on a bounded sample of the slab
    workload: the 512 x 512 slab cut into independent side x side tiles, one
    single-threaded oracle process per core (the corner tile carries the
    stimulus), first nsteps steps of M 6, K 6, dt 0.05 ms.  The rate is the
    node-updates of all tiles over the longest worker's compute time (the
    workers run at once).  Run before the GPU is touched: the workers are
    fresh interpreters started as child processes."""
    import multiprocessing as mp

    ncpu = os.cpu_count() or 1
    share = os.environ.get("OMP_NUM_THREADS")
    workers = max(1, min(ncpu, int(share) if share and share.isdigit() else ncpu, 16))
    keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                           "MKL_NUM_THREADS")}
    for k in keep:
        os.environ[k] = "1"  # one thread per worker process
    try:
        with mp.get_context("spawn").Pool(workers) as pool:
            res = pool.map(_oracle_tile, [(side, k == 0, nsteps) for k in range(workers)])
    finally:
        for k, v in keep.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    updates = sum(r[0] for r in res)
    secs = max(r[1] for r in res)
    return {"value": updates / secs, "unit": "node-updates/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} independent {side}x{side} tiles of the 512x512 slab (no-flux tile "
                      f"edges, the corner tile with the stimulus), one single-threaded oracle process "
                      f"per core, first {nsteps} steps (M 6, K 6, dt 0.05 ms), {secs:.1f} s",
            "nproc": ncpu, "cpu_model": _cpu_model()}


def _kernel_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in ("hsdc_kernels.hip", "hsdc_device.h", "ttp06_device.h", "hsdc_internal.h"):
        with open(os.path.join(ROOT, "paper_2405_19994_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel, path="hbm_traffic_slab2d.json"):
    """HBM bytes per launch of `kernel` measured with rocprofv3 counters
    (FETCH_SIZE + WRITE_SIZE, each scaled by the ratio the same counter gives
    for a plain copy of known size), from profiles/<path>; None when absent or
    taken on kernel sources other than the current ones."""
    path = os.path.join(ROOT, "profiles", path)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("sources_digest") != _kernel_sources_digest():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


# FP64 work of one node update of the fused cell-model kernel (TTP06 currents,
# gates and their exponential update, the explicit auxiliary update and the
# diffusion right-hand side), counted with rocprofv3 instruction counters on
# the 512 x 512 slab: 64 lanes x (2 FMA + ADD + MUL + transcendental) per wave
# instruction, per node.
FLOP_PER_NODE_UPDATE = 2391.0
# the minimum HBM traffic of a node update: read one stage, write one stage
FLOOR_BYTES_PER_NODE_UPDATE = 2 * 19 * 8.0


def _valu_issue(kernel, avg_us):
    """Fraction of VALU issue slots the kernel used (all VALU instructions of a
    launch, four cycles each on a 16-lane SIMD, 1024 SIMDs at 2.4 GHz, over its
    duration), from profiles/valu_slab2d.json taken on the current sources."""
    path = os.path.join(ROOT, "profiles", "valu_slab2d.json")
    if not os.path.exists(path) or not avg_us:
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("sources_digest") != _kernel_sources_digest():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["valu"] * 4.0 / (1024 * 2.4e9 * avg_us * 1e-6)


def _roofline(name, k, N, counters=True):
    """Roofline object of the dominant kernel from its event-timed average
    launch duration.  The fused cell-model kernel (node_update) is judged
    against the FP64 vector peak (algorithmic FLOP = FLOP_PER_NODE_UPDATE x the
    launch's nodes); its HBM side is given beside it (bytes per launch counted
    from the sizes, against the 8 TB/s peak) with the ceiling its arithmetic
    intensity allows (an HBM-bound kernel reaches at most intensity x 8 TB/s).
    Other kernels are judged against the HBM peak.  counters=False (another
    mesh than the counters' 512 x 512): no counter-based figures."""
    traffic = _traffic(name) if counters else None
    gbps = k["GBps"]
    if name != "node_update":
        return {"kernel": name, "bound": "hbm", "achieved": gbps, "peak": 8000.0, "unit": "GB/s",
                "frac": gbps / 8000.0, "traffic": traffic}
    t = k["avg_us"] * 1e-6
    flop = FLOP_PER_NODE_UPDATE * N
    tf = flop / t / 1e12
    intensity = flop / k["bytes_per_launch"]
    return {"kernel": name, "bound": "alu", "achieved": tf, "peak": 78.6, "unit": "TFLOP/s",
            "frac": tf / 78.6, "traffic": traffic, "flop_per_launch": flop,
            "flop_per_node_update": FLOP_PER_NODE_UPDATE,
            "intensity_flop_per_byte": intensity,
            "attainable_frac": min(1.0, intensity * 8.0 / 78.6),
            "valu_issue_frac": _valu_issue(name, k["avg_us"]) if counters else None,
            "hbm": {"achieved": gbps, "peak": 8000.0, "unit": "GB/s", "frac": gbps / 8000.0,
                    "bytes_per_launch": k["bytes_per_launch"],
                    "bytes_per_node_update": k["bytes_per_launch"] / N,
                    "floor_bytes_per_node_update": FLOOR_BYTES_PER_NODE_UPDATE,
                    "floor_frac": FLOOR_BYTES_PER_NODE_UPDATE * N / t / 8.0e12}}


def _kernel_table(kp, overrides=None):
    """Per-class launches, average duration, achieved GB/s and share of the
    profiled kernel time from the library's event profile."""
    kernels = {}
    for k, v in kp.items():
        b = (overrides or {}).get(k, v["bytes"])
        kernels[k] = {"launches": v["launches"], "avg_us": 1e3 * v["ms"] / v["launches"],
                      "time_share": 0.0, "GBps": b / (v["ms"] * 1e-3) / 1e9 if v["ms"] > 0 else 0.0,
                      "bytes_per_launch": b / v["launches"]}
    tot_ms = sum(v["ms"] for v in kp.values())
    for k, v in kp.items():
        kernels[k]["time_share"] = v["ms"] / tot_ms
    return kernels


def _field_error(y, ref):
    """max over fields of max_x |y - ref| / max_x |ref|."""
    d = (y - ref).abs().amax(dim=1)
    s = ref.abs().amax(dim=1).clamp_min(1e-300)
    return float((d / s).max())


def bench_slab3d(a):
    """Two-level PFASST on the 3D slab at a fixed error: the error of a run is
    its per-field distance at the block end from serial hybrid SDC swept to its
    collocation solution (40 sweeps a step, CG to 1e-13).  PFASST (stop test on
    the per-field relative residual) is timed at the loosest tolerance of
    --tols whose error is <= --eps; serial hybrid SDC in FP64 at the fewest
    sweeps per step whose error is <= --eps.  Each is timed --runs times after
    a warm-up and the median run is reported."""
    import torch

    import synthetic_inputs as si
    from paper_2405_19994_amd import hsdc as H

    w = si.workload("slab3d")
    N = int(np.prod(w["dims"]))
    P, dt = w["P"], w["dt"]
    nsteps = a.blocks * P
    T = nsteps * dt
    fp32 = a.coarse != "fp64"
    dev = torch.device("cuda:0")
    stim = torch.tensor(w["stim_w"], dtype=torch.float64, device=dev)
    prob = H.make_problem(w["dims"], w["dx"], w["sigma"], None, w["chi"], w["Cm"], (1, 1, 1), stim,
                          w["stim_amp"], w["stim_t0"], w["stim_dur"])

    Ms = (w["M"], w["Mc"], 1) if a.levels == 3 else (w["M"], w["Mc"])
    if a.levels == 3:
        fp32 = False  # three levels run in FP64

    def pfasst_method(tol):
        return H.make_method(M=Ms, levels=a.levels, space_coarsen=a.coarsen, P=P, dt=dt,
                             max_iter=a.max_iter, tol=tol, burn_in=1, cg_rtol=w["cg_rtol"],
                             cg_maxit=500, coarse_fp32=fp32, solver=a.solver,
                             residual_norm="per_field", prefix_stop=a.prefix_stop)

    def serial_method(K, rtol):
        return H.make_method(M=(w["M"], 1), dt=dt, max_iter=K, cg_rtol=rtol, cg_maxit=500,
                             solver=a.solver)

    stream = torch.cuda.Stream()

    def run(method, n, graph=a.graph):
        ctx = H.Context(prob, method, None, stream)
        if graph and method.levels == 2:
            ctx.use_graph(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.advance(n)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        y = ctx.get_state(0, 0, 0).clone()
        st = ctx.stats()
        ctx.destroy()
        return y, wall, st

    def median_run(method, n):
        res = [run(method, n) for _ in range(max(1, a.runs))]
        res.sort(key=lambda r: r[1])
        return res[len(res) // 2]

    if a.pfasst_only:
        # the PFASST blocks alone, at the first tolerance of --tols (for profilers)
        run(pfasst_method(a.tols[0]), 1)  # warm-up
        y, wall, st = run(pfasst_method(a.tols[0]), a.blocks)
        print(json.dumps({"workload": "slab3d PFASST blocks only", "levels": a.levels,
                          "M": list(Ms), "coarse_fp32": fp32, "tol_per_field": a.tols[0],
                          "blocks": a.blocks, "wall_s": wall,
                          "pfasst_iters": st["pfasst_iters"], "sim_ms_per_wall_s": T / wall}))
        return
    # the error reference: serial hybrid SDC swept to its collocation solution
    ref, wall_ref, _ = run(serial_method(40, 1e-13), nsteps)
    tries = []
    chosen = None
    for tol in a.tols:
        y, wall, st = run(pfasst_method(tol), a.blocks)  # also the warm-up
        e = _field_error(y, ref)
        tries.append({"tol": tol, "error": e, "iters_per_block": st["pfasst_iters"] / a.blocks,
                      "wall_s": wall})
        if e <= a.eps:
            chosen = tol
            break
    if chosen is None:
        chosen = a.tols[-1]
    y_pf, wall_pf, st_pf = median_run(pfasst_method(chosen), a.blocks)
    err_pf = _field_error(y_pf, ref)
    # the other launch mode once: the coarse part of each iteration from a
    # captured graph, or eagerly
    other_mode = None
    if a.levels == 2:
        y_o, wall_o, st_o = run(pfasst_method(chosen), a.blocks, graph=not a.graph)
        other_mode = {"graph_replay": not a.graph, "wall_s": wall_o,
                      "sim_ms_per_wall_s": T / wall_o, "pfasst_iters": st_o["pfasst_iters"],
                      "same_result": bool(torch.equal(y_o, y_pf))}
    serial = None
    for K in range(2, 21):
        y_s, wall_s, _ = run(serial_method(K, w["cg_rtol"]), nsteps)
        e = _field_error(y_s, ref)
        if e <= a.eps or K == 20:
            y_s, wall_s, _ = median_run(serial_method(K, w["cg_rtol"]), nsteps)
            serial = {"sweeps_per_step": K, "error": _field_error(y_s, ref), "wall_s": wall_s,
                      "sim_ms_per_wall_s": T / wall_s,
                      "node_updates_per_s": N * w["M"] * K * nsteps / wall_s,
                      "reached_error": e <= a.eps}
            break

    # profiled pass over one block: per-class kernel durations (HIP events on
    # the library's stream)
    ctx = H.Context(prob, pfasst_method(chosen), None)
    ctx.profile(True)
    ctx.advance(1)
    torch.cuda.synchronize()
    kp = ctx.profile_read()
    pst = ctx.stats()
    ctx.destroy()
    kernels = _kernel_table(kp)
    if "cg_iter" in kernels:
        # coarse and fine solves share the class and their iteration counts are
        # not split by level: no byte figure for it here
        kernels["cg_iter"]["GBps"] = None
        kernels["cg_iter"]["bytes_per_launch"] = None
    cands = {k: v for k, v in kernels.items() if v["GBps"] is not None}
    dom = max(cands, key=lambda k: cands[k]["time_share"])
    roofline = {"kernel": dom, "bound": "hbm", "achieved": kernels[dom]["GBps"], "peak": 8000.0,
                "unit": "GB/s", "frac": kernels[dom]["GBps"] / 8000.0, "traffic": None}
    value = T / wall_pf
    out = {
        "metric": "simulated ms per wall-s at fixed error ("
                  + ("three-level PFASST, FP64)" if a.levels == 3 else
                     "two-level PFASST, " + ("FP32 coarse level)" if fp32 else "FP64)")),
        "value": value,
        "unit": "sim-ms/s",
        "n_gpus": 1,
        "steps": nsteps,
        "warmup": 1,
        "ms_per_step": 1e3 * wall_pf / nsteps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": "slab3d 192x96x48, 7-point sigma (3,1,1), TTP06, PFASST P16 "
                               f"M {'/'.join(str(x) for x in Ms)}, coarse mesh /{a.coarsen} per "
                               f"level, dt 0.1 ms, per-field error <= {a.eps:g}",
                   "nodes": N, "P": P, "M": list(Ms), "space_coarsen": a.coarsen,
                   "coarse_fp32": fp32, "solver": a.solver, "blocks": a.blocks,
                   "prefix_stop": bool(a.prefix_stop),
                   "t_simulated_ms": T, "eps": a.eps, "tol_per_field": chosen},
        "tol_search": tries,
        "pfasst_iters_per_block": st_pf["pfasst_iters"] / a.blocks,
        "error_vs_collocation": err_pf,
        "fine_node_updates_per_s": N * w["M"] * st_pf["sweeps"] / wall_pf,
        "serial_same_error": serial,
        "vs_serial_same_error": None if serial is None else value / serial["sim_ms_per_wall_s"],
        "reference_wall_s": wall_ref,
        "median_of": max(1, a.runs),
        "graph_replay": bool(a.graph),
        "other_launch_mode": other_mode,
        "coarse_redo": st_pf["cg_redo_steps"],
        "profiled_block": {"pfasst_iters": pst["pfasst_iters"], "cg_iters": pst["cg_iters"],
                           "cg_solves": pst["cg_solves"], "cg_redo_steps": pst["cg_redo_steps"]},
        "roofline": roofline,
        "kernels": kernels,
    }
    print(json.dumps(out))


def bench_slab2d_fd4(a):
    """The paper's own spatial setup on the 512 x 512 slab: the fourth-order
    stencil with direct DCT-II solves of every diffusion system (M 6, K 6, dt
    0.05 ms), beside the second-order stencil with the same DCT-II solver and
    with CG from its Chebyshev start.  Median of --runs runs of --steps steps
    (default 100) after a warm-up; a profiled pass gives the kernel classes,
    the DCT-II solves against the HBM peak on their algorithmic bytes."""
    import torch

    import synthetic_inputs as si
    from paper_2405_19994_amd import hsdc as H

    w = si.workload("slab2d")
    steps = a.steps if a.steps != 400 else 100
    dev = torch.device("cuda:0")
    stim = torch.tensor(w["stim_w"], dtype=torch.float64, device=dev)
    N = int(np.prod(w["dims"]))

    def problem(order):
        return H.make_problem(w["dims"], w["dx"], w["sigma"], None, w["chi"], w["Cm"], (1, 1, 1),
                              stim, w["stim_amp"], w["stim_t0"], w["stim_dur"], fd_order=order)

    def method(solver):
        return H.make_method(M=w["M"], dt=w["dt"], max_iter=w["K"], cg_rtol=w["cg_rtol"],
                             cg_maxit=500, solver=solver)

    def timed(order, solver, nsteps, runs):
        res = []
        for _ in range(max(1, runs)):
            ctx = H.Context(problem(order), method(solver))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.advance(nsteps)
            torch.cuda.synchronize()
            res.append(time.perf_counter() - t0)
            ctx.destroy()
        res.sort()
        return res[len(res) // 2]

    upd = N * w["M"] * w["K"]
    timed(4, "dct", min(a.warmup, 10) or 1, 1)  # warm-up
    wall = timed(4, "dct", steps, a.runs)
    others = {}
    for order, solver in ((2, "dct"), (2, "cg")):
        wl = timed(order, solver, steps, 1)
        others[f"order{order}_{solver}"] = {"node_updates_per_s": upd * steps / wl,
                                           "ms_per_step": 1e3 * wl / steps}
    ctx = H.Context(problem(4), method("dct"))
    ctx.profile(True)
    ctx.advance(min(steps, 20))
    torch.cuda.synchronize()
    kp = ctx.profile_read()
    ctx.destroy()
    kernels = _kernel_table(kp)
    dct = None
    if "dct_solve" in kernels:
        # 512 x 512: the fast transforms (three launches a solve, each reading
        # and writing 8 B per node: 48 B per node); latency-bound at this size
        kd = kernels["dct_solve"]
        dct = {"kernel": "dct_solve (three launches)", "bound": "hbm", "achieved": kd["GBps"],
               "peak": 8000.0, "unit": "GB/s", "frac": kd["GBps"] / 8000.0,
               "traffic": None}
    nu = kernels.get("node_update")
    roof = None
    if nu:
        ach = FLOP_PER_NODE_UPDATE * N / (nu["avg_us"] * 1e-6) / 1e12
        roof = {"kernel": "node_update", "bound": "alu", "achieved": ach, "peak": 78.6,
                "unit": "TFLOP/s", "frac": ach / 78.6, "traffic": None}
    out = {
        "metric": "SDC node-updates/s (serial hybrid SDC, FP64, fourth-order stencil, DCT-II solves)",
        "value": upd * steps / wall,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * wall / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "slab2d 512x512, fourth-order stencil, TTP06, M6 K6, dt 0.05 ms, "
                               "DCT-II direct solves", "nodes": N, "M": w["M"], "sweeps": w["K"],
                   "dt_ms": w["dt"]},
        "median_of": max(1, a.runs),
        "other_configurations": others,
        "roofline": roof,
        "dct_roofline": dct,
        "kernels": kernels,
    }
    print(json.dumps(out))


def bench_batch2d(a):
    """64 independent 2D tissues (sides uniform in 64..512, per-node lognormal
    sigma, an 8 x 8 stimulus patch each; M 4, K 4, dt 0.05 ms) advanced by
    serial hybrid SDC as one batch (every launch covers every tissue), against
    the same tissues stepped one context at a time."""
    import torch

    import synthetic_inputs as si
    from paper_2405_19994_amd import hsdc as H

    ws = si.batch2d_tissues(a.tissues, seed=0)
    steps = a.steps if a.steps != 400 else 50
    dev = torch.device("cuda:0")

    def t(x):
        return torch.tensor(x, dtype=torch.float64, device=dev)

    probs = [H.make_problem(w["dims"], w["dx"], w["sigma"], t(w["sigma_node"]), w["chi"], w["Cm"],
                            (1, 1, 1), t(w["stim_w"]), w["stim_amp"], w["stim_t0"], w["stim_dur"])
             for w in ws]
    m = H.make_method(M=ws[0]["M"], dt=ws[0]["dt"], max_iter=ws[0]["K"], cg_rtol=ws[0]["cg_rtol"],
                      cg_maxit=500, solver=a.solver)
    Ns = [p.N for p in probs]
    upd_per_step = sum(Ns) * ws[0]["M"] * ws[0]["K"]
    # block and tile shapes tuned for this batch (cached per shape)
    tuning = None
    if not a.no_autotune:
        from paper_2405_19994_amd import autotune
        setting, timings = autotune.tune(lambda: H.BatchContext(probs, m), "batch", steps=4,
                                         warm=2, axes=("node_block", "cg_tile"), use_cache=False)
        tuning = {"setting": setting, "candidates": timings}

    def new_batch():
        c = H.BatchContext(probs, m)
        if tuning:
            autotune._apply(c, tuning["setting"])
        return c

    if a.warmup > 0:
        ctx = new_batch()
        ctx.advance(min(a.warmup, 5))
        torch.cuda.synchronize()
        ctx.destroy()
    ctx = new_batch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.advance(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = ctx.stats()
    ctx.destroy()
    # the same tissues one context at a time (each context's launches cover one tissue)
    loop_steps = max(1, steps // 5)
    t0 = time.perf_counter()
    for p in probs:
        c1 = H.Context(p, m)
        c1.advance(loop_steps)
        c1.destroy()
    torch.cuda.synchronize()
    wall_loop = time.perf_counter() - t0
    # profiled pass: per-class kernel durations of the batch
    ctx = new_batch()
    ctx.profile(True)
    ctx.advance(min(steps, 20))
    torch.cuda.synchronize()
    kp = ctx.profile_read()
    pst = ctx.stats()
    ctx.destroy()
    b_cg = (pst["cg_iters"] - pst["cg_solves"]) * 80.0 * sum(Ns) / len(Ns) \
        + pst["cg_solves"] * 64.0 * sum(Ns) / len(Ns)
    kernels = _kernel_table(kp, {"cg_iter": b_cg})
    dom = max(kernels, key=lambda k: kernels[k]["time_share"])
    value = upd_per_step * steps / wall
    loop_value = upd_per_step * loop_steps / wall_loop
    out = {
        "metric": "SDC node-updates/s (serial hybrid SDC, FP64, ragged batch of tissues)",
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * wall / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batch2d {a.tissues} tissues, sides 64..512, lognormal sigma, "
                               "8x8 patch, TTP06, M4 K4, dt 0.05 ms, "
                               + SOLVER_NAMES[a.solver] + " 1e-12",
                   "tissues": a.tissues, "nodes_total": int(sum(Ns)), "nodes_min": int(min(Ns)),
                   "nodes_max": int(max(Ns)), "M": ws[0]["M"], "sweeps": ws[0]["K"],
                   "dt_ms": ws[0]["dt"]},
        "one_context_per_tissue": {"node_updates_per_s": loop_value, "steps": loop_steps,
                                   "wall_s": wall_loop},
        "vs_one_context_per_tissue": value / loop_value,
        "tuning": tuning,
        "cg_iters_per_solve": st["cg_iters"] / max(1, st["cg_solves"]),
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": kernels[dom]["GBps"],
                     "peak": 8000.0, "unit": "GB/s", "frac": kernels[dom]["GBps"] / 8000.0,
                     "traffic": None},
        "kernels": kernels,
    }
    print(json.dumps(out))


_KERNEL_CLASS = (("k_node_update", "node_update"), ("k_cg_iter", "cg_iter"),
                 ("k_cg_init", "cg_init"), ("k_assemble", "assemble"),
                 ("k_eval_stages", "eval_stages"), ("k_spmv_stages", "spmv"),
                 ("k_copy_fields", "copy"), ("k_copy_V_to_stages", "copy"),
                 ("k_cheb_iter", "cheb_iter"), ("k_cg_start", "cg_start"),
                 ("k_cg_log", "cg_log"), ("k_apply_K", "apply_K"))


def summarize_counters(fetch_csv, write_csv):
    """Per kernel class: average FETCH_SIZE and WRITE_SIZE per dispatch (KiB),
    each scaled by the ratio the same counter reads for the calibration copy
    (the largest device copy of the run: 512 MiB from a cache-cold source), and
    their sum in bytes per launch."""
    import csv

    def load(path):
        per, calib = {}, 0.0
        for r in csv.DictReader(open(path)):
            name, v = r["Kernel_Name"], float(r["Counter_Value"])
            if "copyBuffer" in name:
                calib = max(calib, v)
                continue
            for key, cls in _KERNEL_CLASS:
                if key in name:
                    per.setdefault(cls, []).append(v)
                    break
        return per, calib

    fetch, cf = load(fetch_csv)
    write, cw = load(write_csv)
    copy_bytes = 512 * 1024 * 1024
    ff, fw = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    kernels = {}
    for cls in fetch:
        if cls not in write:
            continue
        f = sum(fetch[cls]) / len(fetch[cls])
        w = sum(write[cls]) / len(write[cls])
        kernels[cls] = {"fetch_KiB": f, "write_KiB": w, "dispatches": len(fetch[cls]),
                        "bytes_per_launch": 1024.0 * (f * ff + w * fw)}
    rec = {"workload": "slab2d 512x512, M 6, K 6, dt 0.05 ms",
           "sources_digest": _kernel_sources_digest(),
           "calibration": {"copy_bytes": copy_bytes, "FETCH_SIZE_KiB": cf, "WRITE_SIZE_KiB": cw,
                           "fetch_factor": ff, "write_factor": fw},
           "kernels": kernels}
    path = os.path.join(ROOT, "profiles", "hbm_traffic_slab2d.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def summarize_valu(csv_path):
    """Per kernel class: average per dispatch of the VALU instruction counters
    (all VALU, FP64 FMA, ADD, MUL and transcendental, waves) and the FP64 FLOP
    they make, into profiles/valu_slab2d.json."""
    import csv

    per = {}
    for r in csv.DictReader(open(csv_path)):
        name = r["Kernel_Name"]
        for key, cls in _KERNEL_CLASS:
            if key in name:
                d = per.setdefault(cls, {})
                d.setdefault((r["Dispatch_Id"], r["Counter_Name"]), 0.0)
                d[(r["Dispatch_Id"], r["Counter_Name"])] += float(r["Counter_Value"])
                break
    kernels = {}
    for cls, d in per.items():
        disp = sorted({k[0] for k in d})
        avg = {}
        for cn in ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64",
                   "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_TRANS_F64"):
            avg[cn] = sum(d.get((i, cn), 0.0) for i in disp) / len(disp)
        flop = 64.0 * (2.0 * avg["SQ_INSTS_VALU_FMA_F64"] + avg["SQ_INSTS_VALU_ADD_F64"]
                       + avg["SQ_INSTS_VALU_MUL_F64"] + avg["SQ_INSTS_VALU_TRANS_F64"])
        kernels[cls] = {"dispatches": len(disp), "waves": avg["SQ_WAVES"],
                        "valu": avg["SQ_INSTS_VALU"], "fma_f64": avg["SQ_INSTS_VALU_FMA_F64"],
                        "add_f64": avg["SQ_INSTS_VALU_ADD_F64"],
                        "mul_f64": avg["SQ_INSTS_VALU_MUL_F64"],
                        "trans_f64": avg["SQ_INSTS_VALU_TRANS_F64"], "flop_f64": flop}
    rec = {"workload": "slab2d 512x512, M 6, K 6, dt 0.05 ms",
           "sources_digest": _kernel_sources_digest(), "kernels": kernels}
    path = os.path.join(ROOT, "profiles", "valu_slab2d.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def bench_cable1d(a):
    """The 1D cable (128 nodes, M 4, K 4, dt 0.05 ms, T 10 ms): a latency-bound
    serial run, timed as one single-workgroup launch for all steps (the
    default for such meshes), on the per-launch kernels with eager launches,
    and with each step replayed from a captured HIP graph."""
    import torch

    import synthetic_inputs as si
    from paper_2405_19994_amd import hsdc as H

    w = si.workload("cable1d")
    N = int(np.prod(w["dims"]))
    steps = a.steps if a.steps != 400 else int(round(w["t_end"] / w["dt"]))
    dev = torch.device("cuda:0")
    stim = torch.tensor(w["stim_w"], dtype=torch.float64, device=dev)
    prob = H.make_problem(w["dims"], w["dx"], w["sigma"], None, w["chi"], w["Cm"], (1, 1, 1), stim,
                          w["stim_amp"], w["stim_t0"], w["stim_dur"])
    meth = H.make_method(M=w["M"], dt=w["dt"], max_iter=w["K"], cg_rtol=w["cg_rtol"], cg_maxit=300,
                         solver=a.solver)
    stream = torch.cuda.Stream()
    res, ends = {}, {}
    for mode in ("single_block", "eager", "graph"):
        for rep in range(2):  # the first pass warms up
            ctx = H.Context(prob, meth, None, stream)
            if mode != "single_block":
                ctx.single_block(False)
            if mode == "graph":
                ctx.use_graph(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.advance(steps)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            st = ctx.stats()
            ends[mode] = ctx.get_state(0, 0, 0).clone()
            ctx.destroy()
        res[mode] = {"wall_s": wall, "ms_per_step": 1e3 * wall / steps,
                     "node_updates_per_s": N * w["M"] * w["K"] * steps / wall,
                     "cg_redo_steps": st["cg_redo_steps"]}
    # the direct solves against CG to cg_rtol: per-field distance at T
    ref = ends["eager"]
    scale = ref.abs().amax(dim=1).clamp_min(1e-300)
    diff = float(((ends["single_block"] - ref).abs().amax(dim=1) / scale).max())
    value = res["single_block"]["node_updates_per_s"]
    print(json.dumps({
        "metric": "SDC node-updates/s (serial hybrid SDC, FP64, all steps in one single-workgroup "
                  "launch)",
        "value": value, "unit": "node-updates/s", "n_gpus": 1, "steps": steps, "warmup": steps,
        "ms_per_step": res["single_block"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "cable1d 128 nodes, dx 0.01 cm, TTP06, M4 K4, dt 0.05 ms, T 10 ms",
                   "nodes": N, "M": w["M"], "sweeps": w["K"], "dt_ms": w["dt"], "solver": a.solver},
        "single_block": res["single_block"], "eager": res["eager"], "graph": res["graph"],
        "speedup_over_graph": res["graph"]["wall_s"] / res["single_block"]["wall_s"],
        "single_block_vs_eager_max_field_rel_diff": diff}))


def spmv_out_of_cache(dims=(8192, 8192), reps=10):
    """The diffusion operator K v on a mesh far larger than the 256 MB
    last-level cache (8192 x 8192: v and K v are 537 MB each), timed with HIP
    events around reps back-to-back launches on one stream; algorithmic bytes
    16 per node (v read once, K v written once; the neighbours' reuse comes
    from the caches)."""
    import torch

    from paper_2405_19994_amd import hsdc as H

    N = int(np.prod(dims))
    prob = H.make_problem(dims, 0.025, (1.0, 1.0, 1.0))
    v = torch.rand(N, dtype=torch.float64, device="cuda")
    out = torch.empty_like(v)
    stream = torch.cuda.current_stream()
    H.apply_diffusion(prob, v, out=out)  # warm-up (code object load)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        H.apply_diffusion(prob, v, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / reps
    gbps = 16.0 * N / (us * 1e-6) / 1e9
    traffic = _traffic("apply_K")
    return {"kernel": "apply_K", "bound": "hbm", "dims": list(dims), "nodes": N,
            "bytes_per_launch": 16.0 * N, "avg_us": us, "achieved": gbps, "peak": 8000.0,
            "unit": "GB/s", "frac": gbps / 8000.0, "traffic": traffic, "launches": reps}


def bench_adjoint(a):
    """The adjoint workload at full size: 256 x 256 slab, per-node lognormal
    sigma, a 16 x 16 corner stimulus, TTP06, M 4, K 4, dt 0.05 ms, T = 10 ms
    (200 steps); 64 probes sampled every 0.5 ms; targets from a run at perturbed
    parameters (sigma x exp(0.1 N(0,1)), g_Na x 1.1, g_CaL x 0.9, g_Kr x 1.2).
    Times the forward run with its per-step checkpoints and the backward run
    (recompute and transposed sweep of every step), and checks the scaling
    gradient against central differences (h = 1e-6) of the library's own
    forward."""
    import torch

    import synthetic_inputs as si
    from paper_2405_19994_amd import hsdc as H

    dims, dx, M, K, dt, nsteps, every = (256, 256), 0.025, 4, 4, 0.05, 200, 10
    N = dims[0] * dims[1]
    rng = np.random.default_rng(0)
    sigma0 = np.exp(0.3 * rng.standard_normal(N))
    truth = sigma0 * np.exp(0.1 * rng.standard_normal(N))
    probes = np.sort(rng.choice(N, 64, replace=False))
    dev = torch.device("cuda:0")

    def t(x, dtype=torch.float64):
        return torch.tensor(x, dtype=dtype, device=dev)

    stim = t(si.corner_weights(dims, (16, 16)))
    meth = H.make_method(M=(M, 1), dt=dt, max_iter=K, cg_rtol=1e-13, cg_maxit=500)

    def problem(sig, gs):
        return H.make_problem(dims, dx, (1.0, 1.0, 1.0), t(sig), 1400.0, 1.0, gs, stim, 50.0,
                              0.0, 1.0)

    # targets: V at the probes of a forward run at the perturbed parameters
    ctx = H.Context(problem(truth, (1.1, 0.9, 1.2)), meth)
    targets = []
    for _ in range(nsteps // every):
        ctx.advance(every)
        targets.append(ctx.get_state(0, 0, 0)[0][t(probes, torch.int64)].clone())
    ctx.destroy()
    targets = torch.stack(targets).contiguous()
    pr = t(probes, torch.int64)

    def misfit(sig, gs):
        return H.Misfit(problem(sig, gs), meth, pr, targets, nsteps, every)

    misfit(sigma0, (1.0, 1.0, 1.0)).destroy()  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m = misfit(sigma0, (1.0, 1.0, 1.0))
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    ds, dg, _ = m.backward(sigma=True)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    loss = m.loss
    m.destroy()
    h = 1e-6
    fd = []
    for q in range(3):
        gp = [1.0, 1.0, 1.0]
        gm = [1.0, 1.0, 1.0]
        gp[q] += h
        gm[q] -= h
        mp, mm = misfit(sigma0, tuple(gp)), misfit(sigma0, tuple(gm))
        fd.append((mp.loss - mm.loss) / (2 * h))
        mp.destroy()
        mm.destroy()
    rel = [abs(fd[q] - dg[q]) / max(abs(fd[q]), 1e-300) for q in range(3)]
    updates = N * M * K * nsteps
    out = {
        "metric": "SDC node-updates/s of the forward and backward runs of the misfit gradient "
                  "(serial hybrid SDC, FP64)",
        "value": 2 * updates / (t_fwd + t_bwd),
        "unit": "node-updates/s",
        "n_gpus": 1, "steps": nsteps, "warmup": 1, "ms_per_step": 1e3 * (t_fwd + t_bwd) / nsteps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "adjoint 256x256, per-node lognormal sigma, TTP06, M4 K4, dt 0.05 ms, "
                               "T 10 ms, 64 probes every 0.5 ms", "nodes": N},
        "loss": loss, "forward_s": t_fwd, "backward_s": t_bwd,
        "backward_over_forward": t_bwd / t_fwd,
        "checkpoint_bytes": (nsteps + 1) * 19 * 8 * N,
        "grad_gscale": list(dg), "fd_gscale_library_forward": fd, "fd_rel_error": rel,
        "grad_sigma_norm": float(torch.linalg.vector_norm(ds)),
    }
    print(json.dumps(out))


def main():
    a = _args()
    if a.summarize_counters:
        summarize_counters(*a.summarize_counters)
        return
    if a.summarize_valu:
        summarize_valu(a.summarize_valu)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU (a single-GPU box); --gpus must be 1"}))
        sys.exit(2)
    if a.workload == "slab3d":
        bench_slab3d(a)
        return
    if a.workload == "batch2d":
        bench_batch2d(a)
        return
    if a.workload == "cable1d":
        bench_cable1d(a)
        return
    if a.workload == "adjoint":
        bench_adjoint(a)
        return
    if a.workload == "slab2d_fd4":
        bench_slab2d_fd4(a)
        return
    # the oracle's worker processes run before anything touches the GPU (the
    # baseline is of the 512 x 512 slab the metric is quoted on)
    cpu = None if (a.no_cpu_baseline or a.side != 512) else cpu_baseline()

    import torch

    import synthetic_inputs as si
    from paper_2405_19994_amd import hsdc as H

    w = si.workload("slab2d", dims=(a.side, a.side))
    N = int(np.prod(w["dims"]))
    dev = torch.device("cuda:0")
    stim = torch.tensor(w["stim_w"], dtype=torch.float64, device=dev)
    prob = H.make_problem(w["dims"], w["dx"], w["sigma"], None, w["chi"], w["Cm"], (1, 1, 1), stim,
                          w["stim_amp"], w["stim_t0"], w["stim_dur"])

    def method(solver):
        return H.make_method(M=(w["M"], 1), dt=w["dt"], max_iter=w["K"], cg_rtol=w["cg_rtol"],
                             cg_maxit=500, solver=solver)

    meth = method(a.solver)
    # graph replay needs a stream other than the null stream
    stream = torch.cuda.Stream() if a.graph else torch.cuda.current_stream()

    # launch-shape tuning before the timed region (cached per shape)
    tuning = None
    if not a.no_autotune:
        from paper_2405_19994_amd import autotune
        key = autotune.shape_key(prob, meth)
        setting, timings = autotune.tune(lambda: H.Context(prob, meth, None, stream), key,
                                         axes=autotune.relevant_axes(prob, meth), use_cache=False)
        tuning = {"setting": setting, "candidates": timings}

    def new_context(m=None):
        c = H.Context(prob, m or meth, None, stream)
        if tuning:
            s = tuning["setting"]
            c.tune(s["cg_blocks"], s["cg_margin"])
            c.tune_shapes(s["node_block"], s["cg_tile"], s["prolong_tile"])
        if a.graph:
            c.use_graph(True)
        return c

    # warm-up on its own context (code objects, allocator, CG predictors)
    if a.warmup > 0:
        ctx_w = new_context()
        ctx_w.advance(a.warmup)
        torch.cuda.synchronize()
        ctx_w.destroy()

    # a.runs timed runs of a.steps steps, each on a fresh context from t = 0;
    # the reported figures are the median run's
    runs = []
    for _ in range(max(1, a.runs)):
        ctx = new_context()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        ctx.advance(a.steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = ctx.stats()
        Vmax = float(ctx.get_state(0, 0, 0)[0].max())
        ctx.destroy()
        runs.append({"wall_s": wall, "gpu_event_ms": ev0.elapsed_time(ev1), "stats": st,
                     "V_max_end_mV": Vmax})
    order = sorted(range(len(runs)), key=lambda k: runs[k]["wall_s"])
    med = runs[order[len(runs) // 2]]
    wall, st = med["wall_s"], med["stats"]

    # second pass, same workload and launch configuration, with every kernel
    # bracketed by HIP events on the library's stream: per-class durations
    prof_steps = min(a.steps, 100)
    ctx = new_context()
    ctx.profile(True)
    ctx.advance(prof_steps)
    torch.cuda.synchronize()
    kp = ctx.profile_read()
    pst = ctx.stats()
    ctx.destroy()
    kernels = _kernel_table(kp, _solver_bytes(pst, N))
    dom = max(kernels, key=lambda k: kernels[k]["time_share"])
    roofline = _roofline(dom, kernels[dom], N, counters=a.side == 512)

    updates = N * w["M"] * w["K"] * a.steps
    value = updates / wall
    out = {
        "metric": "SDC node-updates/s (serial hybrid SDC, FP64)",
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * wall / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"slab2d {a.side}x{a.side}, 5-point, TTP06, M6 K6, dt 0.05 ms, "
                               + SOLVER_NAMES[a.solver] + " 1e-12",
                   "nodes": N, "M": w["M"], "sweeps": w["K"], "dt_ms": w["dt"],
                   "t_simulated_ms": a.steps * w["dt"]},
        "sim_ms_per_wall_s": a.steps * w["dt"] / wall,
        "timed_runs": [{"wall_s": r["wall_s"], "gpu_event_ms": r["gpu_event_ms"]} for r in runs],
        "median_of": len(runs),
        "graph_replay": bool(a.graph),
        "gpu_event_ms": med["gpu_event_ms"],
        "cg_iters_per_solve": st["cg_iters"] / max(1, st["cg_solves"]),
        "cg_unconverged": st["cg_unconverged"],
        "cg_redo_steps": st["cg_redo_steps"],
        "V_max_end_mV": med["V_max_end_mV"],
        "roofline": roofline,
        "kernels": kernels,
        "tuning": tuning,
    }
    if not a.no_spmv:
        out["spmv_out_of_cache"] = spmv_out_of_cache()
    if a.calibrate_copy:
        # a plain copy of known size whose source is not cache resident: the
        # 2 GiB written in between exceeds the 256 MB last-level cache
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device=dev)
        evict = torch.empty(4 * 64 * 1024 * 1024, dtype=torch.float64, device=dev)
        evict.fill_(2.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel() * 8
        del evict
    # option study: the same workload and tolerance with the other solvers
    for other in ([] if a.no_solver_option else [o for o in SOLVER_NAMES if o != a.solver]):
        m2 = method(other)
        if a.warmup > 0:
            cw = new_context(m2)
            cw.advance(a.warmup)
            torch.cuda.synchronize()
            cw.destroy()
        c2 = new_context(m2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c2.advance(a.steps)
        torch.cuda.synchronize()
        wall2 = time.perf_counter() - t0
        st2 = c2.stats()
        V2 = c2.get_state(0, 0, 0)
        c2.destroy()
        c2 = new_context(m2)
        c2.profile(True)
        c2.advance(prof_steps)
        torch.cuda.synchronize()
        kp2, pst2 = c2.profile_read(), c2.stats()
        c2.destroy()
        out.setdefault("solver_options", []).append({
            "solver": other, "value": updates / wall2, "ms_per_step": 1e3 * wall2 / a.steps,
            "iters_per_solve": st2["cg_iters"] / max(1, st2["cg_solves"]),
            "unconverged": st2["cg_unconverged"], "redo_steps": st2["cg_redo_steps"],
            "V_max_end_mV": float(V2[0].max()),
            "kernels": _kernel_table(kp2, _solver_bytes(pst2, N)),
        })
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


SOLVER_NAMES = {"cg": "CG from a Chebyshev start", "chebyshev": "Chebyshev",
                "cg_plain": "CG from the warm start"}


def _solver_bytes(pst, N):
    """Algorithmic bytes of the diffusion-solver classes of a profiled serial run
    on N nodes.  CG iterations that did work move 80 B/node (r, w, s, p, x read
    and written); the first of a solve reads neither s nor p (64 B); early-exit
    launches move nothing.  After a Chebyshev start most solves need no CG
    iteration, so the first iterations are counted as min(iterations, solves).
    A Chebyshev iterate beyond x_1 (which the node update forms) reads x_k,
    x_{k-1} and b and writes x_{k+1}: 32 B/node.  Only the class the run used
    appears in its table."""
    iters, solves = pst["cg_iters"], pst["cg_solves"]
    first = min(iters, solves)
    return {"cg_iter": (iters - first) * 80.0 * N + first * 64.0 * N,
            "cheb_iter": max(0, iters - solves) * 32.0 * N}


if __name__ == "__main__":
    main()

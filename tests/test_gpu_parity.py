"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

Tolerances: building blocks 1e-13 relative (rounding order only); runs of the
method 1e-10 relative per field (max |gpu - oracle| / max |oracle|), the FP64
bar of the hot path, with CG solves at 1e-14 relative residual."""
import numpy as np
import pytest
import torch

import synthetic_inputs as si
from oracle import coeffs, ttp06
from oracle.hsdc import Level, collocation_solve, run_serial, serial_step
from oracle.pfasst import pfasst_block
from oracle.tissue import ImplicitSolver, laplacian
from tests._parity import field_errors, oracle_hierarchy, oracle_problem, rest

pytestmark = pytest.mark.gpu

H = pytest.importorskip("paper_2405_19994_amd.hsdc")


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def lib_problem(w, dims=None):
    dims = tuple(dims or w["dims"])
    sn = None if w.get("sigma_node") is None else dev(w["sigma_node"])
    return H.make_problem(dims, w["dx"], w["sigma"], sn, w["chi"], w["Cm"], w.get("g_scale", (1, 1, 1)),
                          dev(w["stim_w"]), w["stim_amp"], w["stim_t0"], w["stim_dur"],
                          fd_order=w.get("fd_order", 2))


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("gs", [(1.0, 1.0, 1.0), (1.1, 0.9, 1.2)])
def test_ionic_eval_parity(gs):
    y = si.random_states(100_003, seed=11)
    I, ha, lam, winf = (host(t) for t in H.ionic_eval(dev(y), gs))
    I_o, ha_o, lam_o, winf_o = ttp06.evaluate(y, gs)
    assert np.max(field_errors(I[None], I_o[None])) < 1e-13
    assert np.max(field_errors(ha, ha_o)) < 1e-13
    assert np.max(np.abs(lam - lam_o) / np.abs(lam_o)) < 1e-13
    assert np.max(field_errors(winf, winf_o)) < 1e-13


def test_ionic_eval_full_slab_size():
    """One cell-model evaluation per node of the 512 x 512 slab, every node compared."""
    y = si.random_states(512 * 512, seed=12)
    I, ha, lam, winf = (host(t) for t in H.ionic_eval(dev(y)))
    I_o, ha_o, lam_o, winf_o = ttp06.evaluate(y)
    assert np.max(field_errors(I[None], I_o[None])) < 1e-13
    assert np.max(field_errors(ha, ha_o)) < 1e-13
    assert np.max(np.abs(lam - lam_o) / np.abs(lam_o)) < 1e-13


@pytest.mark.parametrize("kmax", [1, 3, 4, 6, 8])
def test_phi_parity(kmax):
    x = np.concatenate([-np.logspace(-12, 3.6, 3001), np.linspace(-12.0, 12.0, 1201), [0.0]])
    got = host(H.phi(dev(x), kmax))
    for k in range(1, kmax + 1):
        ref = coeffs.phi(k, x)
        err = np.abs(got[k - 1] - ref) / np.abs(ref)
        assert np.max(err) < 5e-14, (k, x[np.argmax(err)], np.max(err))


@pytest.mark.parametrize("M", [2, 3, 4, 6, 8])
def test_colloc_coefficients_parity(M):
    z = np.concatenate([[0.0], -np.logspace(-9, 3.3, 400)])
    a, c = H.colloc_coefficients(M, dev(z))
    a = host(a)
    assert np.max(np.abs(c - coeffs.radau_iia_nodes(M))) < 1e-15
    ref = coeffs.exp_colloc_matrix(z, coeffs.radau_iia_nodes(M))
    tol = 2e-13 if M <= 6 else 2e-12
    assert np.max(np.abs(a - ref)) < tol


@pytest.mark.parametrize("case", ["1d", "2d", "3d_aniso", "2d_pernode"])
def test_apply_diffusion_parity(case):
    rng = np.random.default_rng(3)
    dims, sigma, sn = {"1d": ((37,), (1.0, 1, 1), None), "2d": ((13, 11), (1.0, 1, 1), None),
                       "3d_aniso": ((9, 7, 5), (3.0, 1.0, 0.5), None),
                       "2d_pernode": ((13, 11), (1.0, 1, 1), np.exp(0.3 * rng.standard_normal(143)))}[case]
    N = int(np.prod(dims))
    v = rng.standard_normal(N)
    K = laplacian(dims, 0.025, sigma, sn) / (1400.0 * 1.0)
    p = H.make_problem(dims, 0.025, sigma, None if sn is None else dev(sn))
    got = host(H.apply_diffusion(p, dev(v)))
    ref = K @ v
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("dims,sigma", [((14, 11), (1.0, 1.0)), ((1030, 37), (3.0, 1.0)),
                                        ((2, 5), (1.0, 2.0)), ((512, 16), (1.0, 1.0))])
def test_apply_diffusion_streamed_2d(dims, sigma):
    """The column-streamed operator of 2D meshes with uniform sigma and even nx
    (two nodes per lane, 16-byte accesses; partial blocks in x and y, a mesh
    two nodes wide) equals the oracle's K v and, to rounding (the compiler may
    fuse a product into an add differently), the node-per-thread kernel (taken
    for vectors that are not 16-byte aligned)."""
    rng = np.random.default_rng(5)
    N = int(np.prod(dims))
    v = rng.standard_normal(N)
    p = H.make_problem(dims, 0.025, sigma + (1.0,))
    got = host(H.apply_diffusion(p, dev(v)))
    ref = (laplacian(dims, 0.025, sigma + (1.0,)) / 1400.0) @ v
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))
    vb = torch.zeros(N + 1, dtype=torch.float64, device="cuda")
    vb[1:] = dev(v)
    ob = torch.zeros(N + 1, dtype=torch.float64, device="cuda")
    H.apply_diffusion(p, vb[1:], out=ob[1:])
    assert np.max(np.abs(host(ob[1:]) - got)) <= 4e-16 * np.max(np.abs(got))


@pytest.mark.parametrize("case", ["2d", "3d_aniso", "2d_pernode"])
def test_diffusion_solve_parity(case):
    rng = np.random.default_rng(4)
    dims, sigma, sn = {"2d": ((33, 21), (1.0, 1, 1), None),
                       "3d_aniso": ((12, 10, 6), (3.0, 1.0, 1.0), None),
                       "2d_pernode": ((33, 21), (1.0, 1, 1), np.exp(0.3 * rng.standard_normal(693)))}[case]
    N = int(np.prod(dims))
    b = -85.0 + rng.standard_normal(N)
    a = 0.05 * 0.26
    K = laplacian(dims, 0.025, sigma, sn) / 1400.0
    ref = ImplicitSolver(K).solve(b, a)
    p = H.make_problem(dims, 0.025, sigma, None if sn is None else dev(sn))
    x, it = H.diffusion_solve(p, a, dev(b), rtol=1e-14, maxit=200)
    assert 1 <= it < 200
    assert np.max(np.abs(host(x) - ref)) < 1e-12 * np.max(np.abs(ref))


# ---------------------------------------------------------------------------
# serial HSDC runs
# ---------------------------------------------------------------------------

def _serial_parity(w, nsteps, every, M, K, y0=None, tol=1e-10, solver="cg"):
    po = oracle_problem(w)
    lev = Level(po, M, w["dt"])
    N = po.N
    y0 = rest(N) if y0 is None else y0
    ctx = H.Context(lib_problem(w), H.make_method(M=(M, 1), dt=w["dt"], max_iter=K, cg_rtol=1e-14,
                                                  cg_maxit=300, solver=solver), dev(y0))
    y = y0.copy()
    worst = 0.0
    for n0 in range(0, nsteps, every):
        y = run_serial(lev, y, every, K, step0=n0)
        ctx.advance(every)
        g = host(ctx.get_state(0, 0, 0))
        e = field_errors(g, y)
        worst = max(worst, float(np.max(e)))
        assert np.max(e) < tol, (n0 + every, ttp06.FIELD_NAMES[int(np.argmax(e))], np.max(e))
    st = ctx.stats()
    assert st["steps"] == nsteps and st["cg_unconverged"] == 0
    ctx.destroy()
    return y, worst


def test_cable1d_full_run_parity():
    """The 1D cable workload in full: 128 nodes, M 4, K 4, dt 0.05, T 10 ms."""
    w = si.workload("cable1d")
    y, _ = _serial_parity(w, 200, 20, 4, 4)
    assert y[0].max() > 0.0  # the stimulus launched a propagating action potential


def test_serial_convergence_order_in_dt():
    """Sec. 5.1: hybrid SDC with K sweeps converges in dt with order min(K, M + 1)
    (or higher).  A 24-node cable through its upstroke (stimulus on [0, 0.5]
    ms, T = 1 ms, M 4): the library's error against the oracle's reference
    (64 steps, 8 sweeps) falls between the two finest step sizes at least like
    dt^(K - 0.3), for K = 1..4."""
    dims = (24,)
    w = dict(si.workload("cable1d", dims=dims))
    w["stim_w"], w["stim_t0"], w["stim_dur"] = si.corner_weights(dims, (4,)), 0.0, 0.5
    T = 1.0
    w["dt"] = T / 64
    ref = run_serial(Level(oracle_problem(w), 4, T / 64), rest(24), 64, 8)
    for K in (1, 2, 3, 4):
        errs = []
        for n in (16, 32):
            w["dt"] = T / n
            ctx = H.Context(lib_problem(w), H.make_method(M=4, dt=T / n, max_iter=K, cg_rtol=1e-14,
                                                          cg_maxit=300))
            ctx.advance(n)
            y = host(ctx.get_state(0, 0, 0))
            ctx.destroy()
            errs.append(np.max(np.abs(y[0] - ref[0])) / np.max(np.abs(ref[0])))
        order = np.log2(errs[0] / errs[1])
        assert order > K - 0.3, (K, errs, order)


def test_slab2d_reduced_parity():
    """The 2D slab workload at a reduced, ragged mesh (31 x 23), M 6, K 6."""
    w = si.workload("slab2d", dims=(31, 23))
    _serial_parity(w, 30, 10, 6, 6)


def test_narrow_slab_parity():
    """A long, narrow 2D mesh (700 x 3): the tiled CG start has more tiles (22)
    than the node update has blocks (16 with the XCD padding), so the CG
    partial buffers must be sized for the tiles."""
    w = si.workload("slab2d", dims=(700, 3))
    _serial_parity(w, 12, 6, 4, 4)


def test_pernode_sigma_parity():
    """Per-node lognormal conductivity (the batched-tissue workload's field)."""
    t = si.batch2d_tissues(1, seed=3, lo=20, hi=40)[0]
    _serial_parity(t, 24, 8, 4, 4)


def test_slab3d_serial_parity():
    w = si.workload("slab3d", dims=(10, 8, 6))
    _serial_parity(w, 12, 4, 3, 3)


@pytest.mark.parametrize("case", ["cable1d", "slab2d", "pernode", "slab3d"])
def test_chebyshev_solver_serial_parity(case):
    """The Chebyshev diffusion solver (Gershgorin interval, count from the
    residual bound, no inner products) on every stencil and on per-node sigma:
    serial runs match the oracle's exact solves to 1e-10."""
    if case == "cable1d":
        _serial_parity(si.workload("cable1d"), 60, 20, 4, 4, solver="chebyshev")
    elif case == "slab2d":
        _serial_parity(si.workload("slab2d", dims=(31, 23)), 30, 10, 6, 6, solver="chebyshev")
    elif case == "pernode":
        t = si.batch2d_tissues(1, seed=3, lo=20, hi=40)[0]
        _serial_parity(t, 24, 8, 4, 4, solver="chebyshev")
    else:
        _serial_parity(si.workload("slab3d", dims=(10, 8, 6)), 12, 4, 3, 3, solver="chebyshev")


@pytest.mark.parametrize("case", ["cable1d", "slab2d", "pernode", "slab3d"])
def test_plain_cg_serial_parity(case):
    """CG from the warm start alone (no Chebyshev steps first) on every stencil
    and on per-node sigma: serial runs match the oracle's exact solves to
    1e-10."""
    if case == "cable1d":
        _serial_parity(si.workload("cable1d"), 60, 20, 4, 4, solver="cg_plain")
    elif case == "slab2d":
        _serial_parity(si.workload("slab2d", dims=(31, 23)), 30, 10, 6, 6, solver="cg_plain")
    elif case == "pernode":
        t = si.batch2d_tissues(1, seed=3, lo=20, hi=40)[0]
        _serial_parity(t, 24, 8, 4, 4, solver="cg_plain")
    else:
        _serial_parity(si.workload("slab3d", dims=(10, 8, 6)), 12, 4, 3, 3, solver="cg_plain")


@pytest.mark.parametrize("solver", ["cg", "chebyshev", "cg_plain"])
def test_solver_iteration_cap_reports_enoconv(solver):
    """A solve that cannot reach cg_rtol within cg_maxit (2 iterations to 1e-16,
    through the stimulus) ends in HSDC_ENOCONV after the step, counted in
    cg_unconverged, with the state advanced and finite.  The status describes
    the call that returns it: with a uniform state after the stimulus (a
    constant residual, which one CG iteration removes exactly) a later call
    returns OK."""
    w = dict(si.workload("slab2d", dims=(31, 23)))
    w["stim_dur"] = 0.15  # the first three steps
    ctx = H.Context(lib_problem(w), H.make_method(M=(4, 1), dt=w["dt"], max_iter=2, cg_rtol=1e-16,
                                                  cg_maxit=2, solver=solver))
    with pytest.raises(H.HsdcError) as e:
        ctx.advance(3)
    assert e.value.code == -4
    st = ctx.stats()
    assert st["cg_unconverged"] > 0 and st["steps"] == 3
    assert np.all(np.isfinite(host(ctx.get_state(0, 0, 0))))
    if solver != "chebyshev":  # a Chebyshev degree of 2 does not remove a constant residual
        ctx.set_state(dev(rest(31 * 23)))
        ctx.advance(2)
        assert ctx.stats()["cg_unconverged"] == st["cg_unconverged"]
    ctx.destroy()


@pytest.mark.parametrize("solver", ["cg", "chebyshev", "cg_plain"])
def test_nonfinite_state_reports_enonfinite(solver):
    """A NaN in the state: hsdc_residual returns HSDC_ENONFINITE, and stepping
    stops with HSDC_ENONFINITE after the step that met it (every solve ends at
    once on a NaN residual instead of running to cg_maxit)."""
    w = si.workload("slab2d", dims=(31, 23))
    y0 = rest(31 * 23)
    y0[0, 100] = np.nan
    m = H.make_method(M=(4, 1), dt=w["dt"], max_iter=4, cg_rtol=1e-12, cg_maxit=400, solver=solver)
    ctx = H.Context(lib_problem(w), m, dev(y0))
    with pytest.raises(H.HsdcError) as e:
        ctx.residual()
    assert e.value.code == -5
    with pytest.raises(H.HsdcError) as e:
        ctx.advance(5)
    assert e.value.code == -5
    st = ctx.stats()
    assert st["steps"] == 1
    assert st["cg_iters"] <= 4 * st["cg_solves"]
    ctx.destroy()


def test_sweep_and_residual_parity():
    """hsdc_sdc_sweep applies eq. prec_picard sweeps to the current step;
    hsdc_residual returns ||C(y_n) - 1 (x) y_n||_inf / ||y_n||_inf."""
    w = si.workload("slab2d", dims=(17, 13))
    po = oracle_problem(w)
    lev = Level(po, 6, w["dt"])
    y0 = rest(po.N)
    ctx = H.Context(lib_problem(w), H.make_method(M=(6, 1), dt=w["dt"], max_iter=6, cg_rtol=1e-14),
                    dev(y0))
    # the initial guess is the spread 1 (x) y_n (eq. prec_picard)
    for j in range(7):
        assert np.array_equal(host(ctx.get_state(0, 0, j)), y0)
    for K in (1, 2, 3):
        ctx.sdc_sweep(1)
        Y = serial_step(lev, 0, y0, K)
        for j in range(7):
            assert np.max(field_errors(host(ctx.get_state(0, 0, j)), Y[j])) < 1e-10
        _, rel = lev.residual(0, Y, y0)
        assert abs(ctx.residual()[0] - rel) < 1e-12


# ---------------------------------------------------------------------------
# PFASST
# ---------------------------------------------------------------------------

def _pfasst_case(dims, Mf, Mc, coarsen, P, dt, seed_state=False, solver="cg"):
    kind = {1: "cable1d", 2: "slab2d", 3: "slab3d"}[len(dims)]
    w = dict(si.workload(kind, dims=dims))
    w["dt"] = dt
    if len(dims) == 1:
        w["stim_w"] = si.corner_weights(dims, (2,))
    h = oracle_hierarchy(w, Mf, Mc, coarsen)
    y0 = rest(h.levels[0].prob.N)
    m = H.make_method(M=(Mf, Mc), levels=2, space_coarsen=coarsen, P=P, dt=dt, max_iter=50,
                      tol=0.0, burn_in=1, cg_rtol=1e-14, cg_maxit=300, solver=solver)
    return w, h, y0, m


@pytest.mark.parametrize("dims,coarsen,solver", [((8, 6, 4), 2, "cg"), ((16,), 1, "cg"),
                                                ((8, 6, 4), 2, "chebyshev"),
                                                ((8, 6, 4), 2, "cg_plain"),
                                                ((36, 18), 2, "cg")])
def test_pfasst_iterates_parity(dims, coarsen, solver):
    """Every iterate of Algorithm 1 (burn-in, tau, Q^seq coarse sweep, coarse
    grid correction, Q^par fine sweep) matches the oracle, slice by slice (with
    every diffusion solver on both levels; the 2D case runs the tiled CG start
    over several slices, with tiles cut by the mesh edge)."""
    P = 4
    w, h, y0, m = _pfasst_case(dims, 6 if coarsen == 2 else 4, 3 if coarsen == 2 else 2,
                                coarsen, P, 0.1, solver=solver)
    ctx = H.Context(lib_problem(w), m, dev(y0))
    for k in (1, 2, 3):
        res, _ = ctx.pfasst_iter()
        z, hist, _ = pfasst_block(h, y0, P, k, tol=0.0)
        for n in range(P):
            for j in (0, h.levels[0].M):
                e = field_errors(host(ctx.get_state(0, n, j)), z[n][j])
                assert np.max(e) < 1e-10, (k, n, j, np.max(e))
        assert np.max(np.abs(np.array(hist[-1]) - res)) < 1e-9 * max(1.0, np.max(hist[-1]))


@pytest.mark.parametrize("solver", ["cg", "cg_plain"])
def test_pfasst_sixteen_slices_every_stage_parity(solver):
    """Algorithm 1 at 16 slices (8 x 6 x 4 slab, coarse level M 3 on the 2x
    coarser mesh, dt 0.1 ms, staggered burn-in): after each of three iterations
    every stage 0..M of every slice equals the oracle's, on the fine level and
    on the coarse level (its iterate after the Q^seq sweep), and so does the
    residual of every slice."""
    P = 16
    w, h, y0, m = _pfasst_case((8, 6, 4), 6, 3, 2, P, 0.1, solver=solver)
    ctx = H.Context(lib_problem(w), m, dev(y0))
    seen = []

    def check(k, z, zc):
        res, _ = ctx.pfasst_iter()
        for n in range(P):
            for j in range(7):
                e = field_errors(host(ctx.get_state(0, n, j)), z[n][j])
                assert np.max(e) < 1e-10, ("fine", k, n, j, np.max(e))
            for j in range(4):
                e = field_errors(host(ctx.get_state(1, n, j)), zc[n][j])
                assert np.max(e) < 1e-10, ("coarse", k, n, j, np.max(e))
        seen.append(res)

    _, hist, _ = pfasst_block(h, y0, P, 3, tol=0.0, callback=check)
    assert len(seen) == 3
    for k in range(3):
        assert np.max(np.abs(np.array(hist[k]) - seen[k])) < 1e-9 * max(1.0, np.max(hist[k]))


@pytest.mark.parametrize("dims,coarsen,P", [((8, 8, 4), 2, 4), ((36, 20), 2, 4), ((16,), 1, 4),
                                           ((24, 16), 2, 1)])
def test_three_level_pfasst_iterates_parity(dims, coarsen, P):
    """Algorithm 1 with three levels, M 6, 3, 1 (Sec. 5.1): after each of three
    iterations every stage of every slice on the fine level, the coarsest
    level's iterate after its Q^seq sweep, and every slice's residual equal
    the oracle's.  Space coarsening twice (3D, 2D) or time only (1D); P = 1 is
    the serial multilevel case of the paper's convergence runs."""
    from tests._parity import oracle_hierarchy_levels
    kind = {1: "cable1d", 2: "slab2d", 3: "slab3d"}[len(dims)]
    w = dict(si.workload(kind, dims=dims))
    w["dt"] = 0.1
    if len(dims) == 1:
        w["stim_w"] = si.corner_weights(dims, (2,))
    h = oracle_hierarchy_levels(w, (6, 3, 1), coarsen)
    y0 = rest(h.levels[0].prob.N)
    m = H.make_method(M=(6, 3, 1), levels=3, space_coarsen=coarsen, P=P, dt=0.1, max_iter=50,
                      tol=0.0, burn_in=1, cg_rtol=1e-14, cg_maxit=300)
    ctx = H.Context(lib_problem(w), m, dev(y0))
    seen = []

    def check(k, z, zc):
        res, _ = ctx.pfasst_iter()
        for n in range(P):
            for j in range(7):
                e = field_errors(host(ctx.get_state(0, n, j)), z[n][j])
                assert np.max(e) < 1e-10, ("fine", k, n, j, np.max(e))
            for j in range(2):
                e = field_errors(host(ctx.get_state(2, n, j)), zc[n][j])
                assert np.max(e) < 1e-10, ("coarsest", k, n, j, np.max(e))
        seen.append(res)

    _, hist, _ = pfasst_block(h, y0, P, 3, tol=0.0, callback=check)
    assert len(seen) == 3
    for k in range(3):
        assert np.max(np.abs(np.array(hist[k]) - seen[k])) < 1e-9 * max(1.0, np.max(hist[k]))
    ctx.destroy()


def test_three_level_pfasst_converges_to_serial_collocation():
    """Iterated to convergence, three-level PFASST reaches the fine level's
    serial collocation solution (the fixed point of Algorithm 1) on every slice."""
    P = 4
    w = dict(si.workload("slab2d", dims=(16, 12)))
    w["dt"] = 0.1
    from tests._parity import oracle_hierarchy_levels
    h = oracle_hierarchy_levels(w, (6, 3, 1), 2)
    y0 = rest(h.levels[0].prob.N)
    m = H.make_method(M=(6, 3, 1), levels=3, space_coarsen=2, P=P, dt=0.1, max_iter=60,
                      tol=1e-12, burn_in=1, cg_rtol=1e-14, cg_maxit=300)
    ctx = H.Context(lib_problem(w), m, dev(y0))
    ctx.advance(1)
    y = y0
    for n in range(P):
        Y, _ = collocation_solve(h.levels[0], n, y, tol=1e-14)
        y = Y[-1]
    e = field_errors(host(ctx.get_state(0, 0, 0)), y)
    assert np.max(e) < 1e-9, np.max(e)
    assert ctx.stats()["pfasst_iters"] < 60
    ctx.destroy()


def test_pfasst_sixteen_slices_fp32_coarse_converges_to_collocation():
    """The same 16 slices with the coarse level in FP32, iterated to a per-field
    residual of 5e-11: the end value of every slice equals the serial
    collocation solution (oracle) to 1e-8 per field."""
    P = 16
    w, h, y0, m = _pfasst_case((8, 6, 4), 6, 3, 2, P, 0.1)
    m.coarse_fp32, m.tol, m.max_iter, m.residual_norm = 1, 5e-11, 120, 1
    ctx = H.Context(lib_problem(w), m, dev(y0))
    hist = []
    for _ in range(120):
        res, conv = ctx.pfasst_iter()
        hist.append(float(np.max(res)))
        if conv:
            break
    assert conv, (len(hist), hist[-6:])
    y = y0
    for n in range(P):
        Y, _ = collocation_solve(h.levels[0], n, y, tol=1e-14)
        y = Y[-1]
        e = field_errors(host(ctx.get_state(0, n, 6)), y)
        assert np.max(e) < 1e-8, (n, np.max(e), hist)


def test_residual_per_field_norm():
    """residual_norm = per field: the largest ratio ||r_{n,f}||_inf /
    ||y_{n,f}||_inf over the fields, as the oracle computes it."""
    w = si.workload("slab2d", dims=(17, 13))
    po = oracle_problem(w)
    lev = Level(po, 4, w["dt"])
    y0 = rest(po.N)
    ctx = H.Context(lib_problem(w), H.make_method(M=(4, 1), dt=w["dt"], max_iter=4,
                                                  cg_rtol=1e-14, residual_norm="per_field"),
                    dev(y0))
    ctx.sdc_sweep(2)
    Y = serial_step(lev, 0, y0, 2)
    r = lev.C(0, Y) - y0[None]
    ref = np.max(np.max(np.abs(r), axis=(0, 2)) / np.max(np.abs(Y), axis=(0, 2)))
    got = ctx.residual()[0]
    assert abs(got - ref) < 1e-9 * ref, (got, ref)


@pytest.mark.parametrize("solver", ["cg", "chebyshev"])
def test_pfasst_converges_to_serial_collocation(solver):
    P = 4
    w, h, y0, m = _pfasst_case((8, 6, 4), 6, 3, 2, P, 0.1, solver=solver)
    m.tol, m.max_iter = 1e-13, 60
    ctx = H.Context(lib_problem(w), m, dev(y0))
    conv = False
    for _ in range(60):
        res, conv = ctx.pfasst_iter()
        if conv:
            break
    assert conv
    y = y0
    for n in range(P):
        Y, _ = collocation_solve(h.levels[0], n, y, tol=1e-14)
        y = Y[-1]
    g = host(ctx.get_state(0, P - 1, h.levels[0].M))
    assert np.max(np.abs(g - y)) < 1e-11 * np.max(np.abs(y))


@pytest.mark.parametrize("dims,coarsen", [((8, 6, 4), 2), ((16,), 1)])
def test_pfasst_fp32_coarse_converges_to_serial_collocation(dims, coarsen):
    """Coarse level in FP32 (cell model, sweep, CG vectors): the fixed point is
    still the FP64 fine collocation solution.  PFASST iterated to stagnation
    matches serial collocation (oracle) to 1e-8 per field, and reaches a
    residual of 1e-7 in at most three iterations more than with an FP64 coarse
    level."""
    P = 4
    Mf, Mc = (6, 3) if coarsen == 2 else (4, 2)
    w, h, y0, m = _pfasst_case(dims, Mf, Mc, coarsen, P, 0.1)

    def run(fp32):
        m.coarse_fp32 = int(fp32)
        m.tol, m.max_iter = 1e-10, 80
        ctx = H.Context(lib_problem(w), m, dev(y0))
        hist = []
        for _ in range(80):
            res, conv = ctx.pfasst_iter()
            hist.append(float(np.max(res)))
            if conv or (len(hist) > 8 and hist[-1] >= 0.9 * hist[-4]):
                break
        g = host(ctx.get_state(0, P - 1, Mf))
        ctx.destroy()
        return g, hist

    g32, h32 = run(True)
    _, h64 = run(False)
    assert np.all(np.isfinite(g32))
    y = y0
    for n in range(P):
        Y, _ = collocation_solve(h.levels[0], n, y, tol=1e-14)
        y = Y[-1]
    assert np.max(field_errors(g32, y)) < 1e-8, (np.max(field_errors(g32, y)), h32)
    k32 = next(k for k, r in enumerate(h32) if r < 1e-7)
    k64 = next(k for k, r in enumerate(h64) if r < 1e-7)
    assert k32 <= k64 + 3, (h32, h64)


def test_pfasst_advance_blocks():
    """hsdc_advance in PFASST mode: two blocks iterated to tol, chained."""
    from oracle.pfasst import run_pfasst
    P = 2
    w, h, y0, m = _pfasst_case((16,), 4, 2, 1, P, 0.1)
    m.tol, m.max_iter = 1e-12, 40
    ctx = H.Context(lib_problem(w), m, dev(y0))
    ctx.advance(2)
    y_ref, _ = run_pfasst(h, y0, 2, P, 40, 1e-12)
    g = host(ctx.get_state(0, 0, 0))
    assert ctx.step == 2 * P
    assert np.max(field_errors(g, y_ref)) < 1e-10


# ---------------------------------------------------------------------------
# ragged batch of independent tissues in one set of launches
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("solver", ["cg", "chebyshev"])
def test_batch_matches_oracle_per_tissue(solver):
    """Three ragged tissues (per-node lognormal sigma, an 8 x 8 stimulus patch
    each) stepped together through the stimulus (24 steps of dt 0.05 ms, M 4,
    K 4): every tissue equals the oracle's serial HSDC run of that tissue alone."""
    ws = si.batch2d_tissues(3, seed=3, lo=12, hi=28)
    m = H.make_method(M=4, dt=ws[0]["dt"], max_iter=4, cg_rtol=1e-14, cg_maxit=300, solver=solver)
    ctx = H.BatchContext([lib_problem(w) for w in ws], m)
    nsteps = 24
    ctx.advance(nsteps)
    assert ctx.step == nsteps
    for n, w in enumerate(ws):
        po = oracle_problem(w)
        y = run_serial(Level(po, 4, w["dt"]), rest(po.N), nsteps, 4)
        g = host(ctx.get_state(0, n, 0))
        assert np.max(field_errors(g, y)) < 1e-10, (n, w["dims"], np.max(field_errors(g, y)))


@pytest.mark.parametrize("solver", ["cg", "chebyshev", "cg_plain", "cg_register_tiles"])
def test_batch_matches_single_contexts(solver):
    """Five ragged tissues (20..60 nodes a side): the batch equals five separate
    contexts bitwise (every reduction adds the same partials in the same order,
    and a Chebyshev solve takes its tissue's own spectral bound and count),
    including set_state on one tissue and a sweep applied to all; also with
    the CG start's register-resident tiles (48 x 16) on both sides."""
    ws = si.batch2d_tissues(5, seed=7, lo=20, hi=60)
    tile = 5 if solver == "cg_register_tiles" else -1
    solver = "cg" if tile >= 0 else solver
    m = H.make_method(M=4, dt=ws[0]["dt"], max_iter=4, cg_rtol=1e-14, cg_maxit=300, solver=solver)
    probs = [lib_problem(w) for w in ws]
    y0 = [None] * 5
    y0[2] = dev(si.random_states(ws[2]["dims"][0] * ws[2]["dims"][1], seed=5))
    ctx = H.BatchContext(probs, m, y0)
    ctx.tune_shapes(0, tile, -1)
    ctx.advance(10)
    ctx.sdc_sweep(2)
    for n, w in enumerate(ws):
        single = H.Context(probs[n], m, y0[n])
        single.tune_shapes(0, tile, -1)
        single.advance(10)
        single.sdc_sweep(2)
        for j in (0, 4):
            a = host(ctx.get_state(0, n, j))
            b = host(single.get_state(0, 0, j))
            assert np.array_equal(a, b), (n, j, np.max(field_errors(a, b)))
        single.destroy()
    with pytest.raises(H.HsdcError):
        ctx.sdc_sweep(1, slice=1)


def test_tuned_launch_shapes_give_the_same_run():
    """CG block cap and budget margin change launch shapes only: a context tuned
    to 128 blocks and margin 3 matches an untuned one up to the order of the CG
    reductions; out-of-range values are rejected."""
    w = si.workload("slab2d", dims=(61, 47))
    m = H.make_method(M=6, dt=w["dt"], max_iter=6, cg_rtol=1e-13, cg_maxit=300)
    a = H.Context(lib_problem(w), m)
    b = H.Context(lib_problem(w), m)
    b.tune(128, 3)
    with pytest.raises(H.HsdcError):
        b.tune(4096, 0)
    with pytest.raises(H.HsdcError):
        b.tune(0, 100)
    a.advance(12)
    b.advance(12)
    e = field_errors(host(b.get_state(0, 0, 0)), host(a.get_state(0, 0, 0)))
    assert np.max(e) < 1e-11


def test_cg_start_tiles_agree_bitwise_on_the_full_slab():
    """On the 512 x 512 slab of the benchmark (M 6, K 6, solves to 1e-12) the
    one-launch start of degree 7 meets the tolerance by itself, so the state
    depends on the start kernel alone (no CG iteration updates it): the LDS
    tile and every register tile (blocks of 48 x 8 .. 48 x 32 nodes, the
    mesh's edges cutting them) give the same state bit for bit."""
    w = si.workload("slab2d", dims=(512, 512))
    prob = lib_problem(w)
    m = H.make_method(M=w["M"], dt=w["dt"], max_iter=w["K"], cg_rtol=w["cg_rtol"], cg_maxit=500)
    ref = None
    for tile in (0, 5, 6, 7, 8):
        c = H.Context(prob, m)
        c.tune_shapes(0, tile, -1)
        c.advance(6)
        y = host(c.get_state(0, 0, 0))
        st = c.stats()
        c.destroy()
        assert st["cg_iters"] == 0 and st["cg_unconverged"] == 0, (tile, st)
        if ref is None:
            ref = y
        assert np.array_equal(y, ref), (tile, np.max(field_errors(y, ref)))


@pytest.mark.parametrize("pernode", [False, True])
def test_tuned_block_and_tile_shapes_give_the_same_run(pernode):
    """Every node-update block size and every CG-start tile (uniform and
    per-node sigma, a mesh whose edges cut the tiles) gives the default run up
    to the order of the reductions over blocks and tiles; bad shapes are
    rejected before any work."""
    # a tissue with per-node lognormal sigma, or the uniform slab, 61 x 47
    w = si.batch2d_tissues(1, seed=3, lo=61, hi=61)[0] if pernode else si.workload("slab2d",
                                                                                   dims=(61, 47))
    prob = lib_problem(w)
    m = H.make_method(M=6, dt=w["dt"], max_iter=6, cg_rtol=1e-13, cg_maxit=300)
    ref = H.Context(prob, m)
    ref.advance(8)
    y_ref = host(ref.get_state(0, 0, 0))
    ref.destroy()
    shapes = ([(nb, 0) for nb in (64, 128, 512)] + [(256, t) for t in (1, 2, 3, 4, 5, 6, 7, 8)]
              + [(64, 4), (128, 5)])
    for nb, tile in shapes:
        c = H.Context(prob, m)
        c.tune_shapes(nb, tile, -1)
        c.advance(8)
        e = field_errors(host(c.get_state(0, 0, 0)), y_ref)
        st = c.stats()
        c.destroy()
        assert np.max(e) < 1e-11, (nb, tile, np.max(e))
        assert st["cg_unconverged"] == 0
    c = H.Context(prob, m)
    for bad in ((96, -1, -1), (0, 9, -1), (0, -1, 4), (1024, 0, 0)):
        with pytest.raises(H.HsdcError):
            c.tune_shapes(*bad)
    c.destroy()


@pytest.mark.parametrize("dims", [(8, 6, 4), (36, 18)])
def test_tuned_correction_tiles_give_the_same_iterates(dims):
    """Every tile of the coarse-to-fine correction (3D and 2D) and a smaller
    node-update block give the default PFASST iterates, and those match the
    oracle's Algorithm 1 iterate by iterate."""
    P = 4
    w, h, y0, m = _pfasst_case(dims, 6, 3, 2, P, 0.1)
    z, _, _ = pfasst_block(h, y0, P, 3, tol=0.0)
    for tile in range(4):
        ctx = H.Context(lib_problem(w), m, dev(y0))
        ctx.tune_shapes(128 if tile == 3 else 0, -1, tile)
        for _ in range(3):
            ctx.pfasst_iter()
        for n in range(P):
            for j in (0, h.levels[0].M):
                e = field_errors(host(ctx.get_state(0, n, j)), z[n][j])
                assert np.max(e) < 1e-10, (tile, n, j, np.max(e))
        ctx.destroy()


def test_pfasst_prefix_stop_iterates_parity():
    """prefix_stop (leading converged slices stop iterating, Sec. 3.2): every
    iterate of every slice and every residual equal the oracle's, through the
    iterations at which slices stop, and a stopped slice is left unchanged;
    the coarse part replayed from a graph gives the same iterates."""
    P = 8
    w, h, y0, m = _pfasst_case((8, 6, 4), 6, 3, 2, P, 0.1)
    m.tol, m.max_iter, m.prefix_stop = 1e-9, 60, 1
    stream = torch.cuda.Stream()
    ctx = H.Context(lib_problem(w), m, dev(y0), stream)
    ctg = H.Context(lib_problem(w), m, dev(y0), stream)
    ctg.use_graph(True)
    seen = []

    def check(k, z, zc):
        res, conv = ctx.pfasst_iter()
        resg, _ = ctg.pfasst_iter()
        assert np.array_equal(res, resg), (k, res, resg)
        for n in range(P):
            for j in (0, 6):
                g = host(ctx.get_state(0, n, j))
                e = field_errors(g, z[n][j])
                assert np.max(e) < 1e-10, (k, n, j, np.max(e))
                assert np.array_equal(g, host(ctg.get_state(0, n, j))), (k, n, j)
        seen.append((res, conv))

    _, hist, k = pfasst_block(h, y0, P, 60, tol=1e-9, prefix_stop=True, callback=check)
    assert len(seen) == k and seen[-1][1]
    stopped = [sum(1 for x in r if x < 1e-9) for r in hist]
    assert 0 < stopped[-2] < P  # some slices stopped before the last iteration
    for q in range(k):
        assert np.max(np.abs(np.array(hist[q]) - seen[q][0])) < 1e-9 * max(1.0, np.max(hist[q]))
    assert ctx.stats()["pfasst_iters"] == k
    ctx.destroy()
    ctg.destroy()


@pytest.mark.parametrize("coarse_fp32", [False, True])
def test_pfasst_graph_replay_equals_eager_iterations(coarse_fp32):
    """PFASST with the coarse part of each iteration (FAS restriction, coarse
    evaluations, the Q^seq chain with budgeted solves) replayed from a captured
    HIP graph gives the eager iterates exactly: budgets change only how many
    no-op CG launches follow convergence, and a missed budget reruns the part
    with every solve checked.  Whole blocks with the stop test too."""
    stream = torch.cuda.Stream()
    P = 4
    w, h, y0, m = _pfasst_case((8, 6, 4), 6, 3, 2, P, 0.1)
    m.coarse_fp32 = int(coarse_fp32)
    a = H.Context(lib_problem(w), m, dev(y0), stream)
    b = H.Context(lib_problem(w), m, dev(y0), stream)
    b.use_graph(True)
    for k in range(12):
        ra, _ = a.pfasst_iter()
        rb, _ = b.pfasst_iter()
        assert np.array_equal(ra, rb), (k, ra, rb)
    for n in range(P):
        for j in (0, 3, 6):
            e = field_errors(host(b.get_state(0, n, j)), host(a.get_state(0, n, j)))
            assert np.max(e) == 0.0, (n, j, np.max(e))
    sa, sb = a.stats(), b.stats()
    assert sa["pfasst_iters"] == sb["pfasst_iters"] == 12
    assert sa["coarse_sweeps"] == sb["coarse_sweeps"]
    assert sa["cg_unconverged"] == sb["cg_unconverged"] == 0
    a.destroy()
    b.destroy()
    m.tol, m.max_iter = 1e-9, 60
    a = H.Context(lib_problem(w), m, dev(y0), stream)
    b = H.Context(lib_problem(w), m, dev(y0), stream)
    b.use_graph(True)
    a.advance(2)
    b.advance(2)
    e = field_errors(host(b.get_state(0, 0, 0)), host(a.get_state(0, 0, 0)))
    assert np.max(e) == 0.0
    assert a.stats()["pfasst_iters"] == b.stats()["pfasst_iters"]
    a.destroy()
    b.destroy()


@pytest.mark.parametrize("solver", ["cg", "chebyshev", "cg_plain"])
def test_graph_replay_equals_eager_steps(solver):
    """Serial steps replayed from a captured HIP graph (device step counter,
    budgeted solves verified per replay) give the same states as eager steps,
    through the stimulus, for a slab and for a ragged batch; a graph needs a
    non-null stream."""
    stream = torch.cuda.Stream()
    w = si.workload("slab2d", dims=(61, 47))
    m = H.make_method(M=6, dt=w["dt"], max_iter=6, cg_rtol=1e-13, cg_maxit=300, solver=solver)
    a = H.Context(lib_problem(w), m, None, stream)
    b = H.Context(lib_problem(w), m, None, stream)
    b.use_graph(True)
    for _ in range(4):
        a.advance(10)
        b.advance(10)
        for j in (0, 3):
            e = field_errors(host(b.get_state(0, 0, j)), host(a.get_state(0, 0, j)))
            assert np.max(e) < 1e-12, (b.step, j, np.max(e))
    assert a.step == b.step == 40
    sa, sb = a.stats(), b.stats()
    # every step sweeps 6 times, a recomputed step (a missed solve budget) again
    for st in (sa, sb):
        assert st["steps"] == 40 and st["sweeps"] == 6 * (40 + st["cg_redo_steps"]), st
    ws = si.batch2d_tissues(3, seed=3, lo=12, hi=28)
    mb = H.make_method(M=4, dt=ws[0]["dt"], max_iter=4, cg_rtol=1e-13, cg_maxit=300, solver=solver)
    ba = H.BatchContext([lib_problem(x) for x in ws], mb, None, stream)
    bb = H.BatchContext([lib_problem(x) for x in ws], mb, None, stream)
    bb.use_graph(True)
    ba.advance(24)
    bb.advance(24)
    for n in range(3):
        e = field_errors(host(bb.get_state(0, n, 0)), host(ba.get_state(0, n, 0)))
        assert np.max(e) < 1e-12, (n, np.max(e))
    c = H.Context(lib_problem(w), m)  # null stream
    with pytest.raises(H.HsdcError):
        c.use_graph(True)


# ---------------------------------------------------------------------------
# full size: the 512 x 512 slab in the benchmark's launch configuration
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("solver", ["cg", "chebyshev", "cg_plain"])
def test_slab2d_full_size_sweep_equation_at_sampled_nodes(solver):
    """At full size, after 30 steps (through the stimulus), two more sweeps of
    the 31st step; the oracle evaluates eq. prec_picard at 3000 sampled nodes
    (plus corners and stimulus edges) from the library's whole stage vectors.
    Bound on V: the node-to-node form accumulates the solve residuals of nodes
    1..i, so |defect_i| <= i * cg_rtol * max ||b||_2; other fields: rounding."""
    from oracle.sampled import sweep_defect
    w = si.workload("slab2d")
    po = oracle_problem(w)
    N = po.N
    ctx = H.Context(lib_problem(w), H.make_method(M=(6, 1), dt=w["dt"], max_iter=6,
                                                  cg_rtol=w["cg_rtol"], cg_maxit=500,
                                                  solver=solver))
    ctx.advance(30)
    ctx.sdc_sweep(1)
    Yk = np.stack([host(ctx.get_state(0, 0, j)) for j in range(7)])
    ctx.sdc_sweep(1)
    Yn = np.stack([host(ctx.get_state(0, 0, j)) for j in range(7)])
    assert ctx.stats()["cg_unconverged"] == 0
    ctx.destroy()
    rng = np.random.default_rng(7)
    rows = np.unique(np.concatenate([rng.choice(N, 3000, replace=False),
                                     [0, 511, N - 512, N - 1, 15, 16, 15 * 512, 16 * 512 + 16]]))
    D = sweep_defect(po, 6, w["dt"], 30, Yk, Yn, Yk[0], rows)
    bnorm = np.sqrt(np.sum(Yn[:, 0] ** 2, axis=1)).max()
    for i in range(7):
        assert np.max(np.abs(D[i, 0])) <= 2 * max(i, 1) * w["cg_rtol"] * bnorm, (i, np.max(np.abs(D[i, 0])))
    scale = np.max(np.abs(Yn[:, 1:, rows]), axis=(0, 2))
    assert np.max(np.max(np.abs(D[:, 1:]), axis=(0, 2)) / scale) < 1e-12
    # the stimulated corner has fired and the wave is moving through the slab
    assert Yn[-1, 0].max() > 0.0 and Yn[-1, 0].min() < -80.0


def test_slab2d_full_size_uniform_state_is_a_single_cell():
    """Property at any size: without stimulus a uniform state stays uniform (the
    no-flux Laplacian of a constant is exactly 0) and equals the single-cell run."""
    w = dict(si.workload("slab2d"))
    w["stim_amp"] = 0.0
    N = 512 * 512
    y1 = ttp06.rest_state()
    y1[0] = -55.0  # above threshold: an action potential starts everywhere
    ctx = H.Context(lib_problem(w), H.make_method(M=(6, 1), dt=w["dt"], max_iter=6,
                                                  cg_rtol=w["cg_rtol"], cg_maxit=500),
                    dev(np.repeat(y1[:, None], N, axis=1)))
    ctx.advance(20)
    g = host(ctx.get_state(0, 0, 0))
    ctx.destroy()
    assert np.all(g == g[:, :1])
    cell = oracle_problem(dict(w, dims=(1,), stim_w=np.zeros(1)))
    ref = run_serial(Level(cell, 6, w["dt"]), y1[:, None], 20, 6)
    assert np.max(field_errors(g[:, :1], ref)) < 1e-10


# ---------------------------------------------------------------------------
# full size: the 3D PFASST workload and the 64-tissue batch
# ---------------------------------------------------------------------------

def test_slab3d_full_size_pfasst_reaches_serial_collocation():
    """At full size in the benchmark's configuration (192 x 96 x 48, 16 slices,
    fine M 6 in FP64, coarse M 3 in FP32 on the 2x coarser mesh, dt 0.1 ms) one
    block iterated to a per-field residual of 1e-10: (a) the oracle evaluates
    the collocation equations C(y_n) = 1 (x) y_{n-1,M} (eq. def_C) of slices 0,
    7 and 15 at 400 sampled nodes on the library's stage vectors and finds them
    satisfied; (b) the block end equals serial HSDC swept to its collocation
    solution (40 sweeps a step) to 1e-8 per field: the fixed point of
    Algorithm 1 is the serial collocation solution at any size."""
    from oracle.sampled import collocation_defect
    w = si.workload("slab3d")
    prob = lib_problem(w)
    m = H.make_method(M=(6, 3), levels=2, space_coarsen=2, P=16, dt=w["dt"], max_iter=150,
                      tol=1e-10, burn_in=1, cg_rtol=1e-13, cg_maxit=500, coarse_fp32=True,
                      residual_norm="per_field")
    ctx = H.Context(prob, m)
    conv = False
    for _ in range(150):
        res, conv = ctx.pfasst_iter()
        if conv:
            break
    assert conv, (ctx.stats()["pfasst_iters"], np.max(res))
    po = oracle_problem(w)
    rng = np.random.default_rng(11)
    rows = np.unique(np.concatenate([rng.choice(po.N, 400, replace=False), [0, 1, 2, po.N - 1]]))
    y0 = rest(po.N)
    for n in (0, 7, 15):
        Y = np.stack([host(ctx.get_state(0, n, j)) for j in range(7)])
        u = y0 if n == 0 else host(ctx.get_state(0, n - 1, 6))
        D = collocation_defect(po, 6, w["dt"], n, Y, u, rows)
        scale = np.max(np.abs(Y[:, :, rows]), axis=(0, 2))
        assert np.max(np.max(np.abs(D), axis=(0, 2)) / scale) < 1e-9, n
    y_pf = host(ctx.get_state(0, 15, 6))
    ctx.destroy()
    ref = H.Context(prob, H.make_method(M=6, dt=w["dt"], max_iter=40, cg_rtol=1e-13, cg_maxit=500))
    ref.advance(16)
    y_ref = host(ref.get_state(0, 0, 0))
    ref.destroy()
    assert np.all(np.isfinite(y_pf))
    assert np.max(field_errors(y_pf, y_ref)) < 1e-8, np.max(field_errors(y_pf, y_ref))
    assert y_ref[0].max() > 0.0  # the face stimulus started an action potential


@pytest.mark.parametrize("solver", ["cg", "chebyshev", "cg_plain"])
def test_batch2d_full_size_tissues_equal_single_contexts(solver):
    """The 64-tissue batch at full size (sides 64..512, 6.05M nodes, M 4, K 4):
    after 4 steps through the stimulus onset, sampled tissues (the smallest, the
    largest and two others) equal their own single contexts bitwise."""
    ws = si.batch2d_tissues(64, seed=0)
    m = H.make_method(M=4, dt=ws[0]["dt"], max_iter=4, cg_rtol=1e-12, cg_maxit=500, solver=solver)
    probs = [lib_problem(w) for w in ws]
    ctx = H.BatchContext(probs, m)
    ctx.advance(4)
    sizes = [p.N for p in probs]
    picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 17, 42})
    for n in picks:
        single = H.Context(probs[n], m)
        single.advance(4)
        a = host(ctx.get_state(0, n, 0))
        b = host(single.get_state(0, 0, 0))
        single.destroy()
        assert np.array_equal(a, b), (n, ws[n]["dims"])


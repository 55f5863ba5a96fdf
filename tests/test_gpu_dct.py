"""The paper's own spatial setup on the GPU: the fourth-order stencil (Sec. 2.2)
and the direct DCT-II solves of (I - a K) x = b (Sec. 5, computational setup),
against the oracle's sparse operator and LU solves.

Tolerances: the operator and single solves 1e-12 relative (a dense transform
sums n products per entry: rounding grows like n eps); runs of the method
1e-10 per field, the FP64 bar of the other solvers."""
import numpy as np
import pytest
import torch

import synthetic_inputs as si
from oracle.hsdc import Level, run_serial
from oracle.pfasst import pfasst_block
from oracle.tissue import ImplicitSolver, dct_solve_uniform, laplacian
from tests._parity import field_errors, oracle_hierarchy, oracle_problem, rest

pytestmark = pytest.mark.gpu

H = pytest.importorskip("paper_2405_19994_amd.hsdc")


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def lib_problem(w):
    return H.make_problem(tuple(w["dims"]), w["dx"], w["sigma"], None, w["chi"], w["Cm"],
                          w.get("g_scale", (1, 1, 1)), dev(w["stim_w"]), w["stim_amp"],
                          w["stim_t0"], w["stim_dur"], fd_order=w.get("fd_order", 2))


# lengths that are not powers of two take the dense transforms, the others
# (every transformed axis a power of two) the fast ones
CASES = {"1d": ((37,), (1.0, 1, 1)), "2d": ((33, 21), (1.0, 2.0, 1)),
         "3d_aniso": ((12, 10, 6), (3.0, 1.0, 0.5)), "2d_odd_small": ((5, 3), (1.0, 1, 1)),
         "1d_pow2": ((128,), (1.0, 1, 1)), "2d_pow2": ((64, 32), (1.0, 2.0, 1)),
         "3d_pow2_aniso": ((16, 8, 4), (3.0, 1.0, 0.5)), "2d_pow2_tiny": ((2, 4), (1.0, 1, 1)),
         "2d_pow2_long": ((2048, 2), (1.0, 1.5, 1))}


@pytest.mark.parametrize("case", sorted(CASES))
def test_fourth_order_operator_parity(case):
    dims, sigma = CASES[case]
    rng = np.random.default_rng(3)
    v = rng.standard_normal(int(np.prod(dims)))
    K = laplacian(dims, 0.025, sigma, order=4) / 1400.0
    p = H.make_problem(dims, 0.025, sigma, fd_order=4)
    got = host(H.apply_diffusion(p, dev(v)))
    ref = K @ v
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("case", sorted(CASES))
def test_dct_solve_parity(case):
    """One solve of (I - a K) x = b with the fourth-order K against the
    oracle's LU solve and its scipy DCT-II solve."""
    dims, sigma = CASES[case]
    rng = np.random.default_rng(4)
    N = int(np.prod(dims))
    b = -85.0 + rng.standard_normal(N)
    a = 0.05 * 0.26
    K = laplacian(dims, 0.025, sigma, order=4) / 1400.0
    ref = ImplicitSolver(K).solve(b, a)
    ref2 = dct_solve_uniform(dims, 0.025, sigma, a / 1400.0, b, order=4)
    assert np.max(np.abs(ref - ref2)) < 1e-12 * np.max(np.abs(ref))
    p = H.make_problem(dims, 0.025, sigma, fd_order=4)
    x, it = H.diffusion_solve(p, a, dev(b), rtol=1e-14, maxit=10)
    assert it == 0
    assert np.max(np.abs(host(x) - ref)) < 1e-12 * np.max(np.abs(ref))


def test_dct_solve_full_slab_size():
    """The 512 x 512 slab's mesh: a rough right-hand side (all modes present)."""
    dims, sigma = (512, 512), (1.0, 1.0, 1.0)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(512 * 512)
    a = 0.05 * 0.26
    ref = dct_solve_uniform(dims, 0.025, sigma, a / 1400.0, b, order=4)
    p = H.make_problem(dims, 0.025, sigma, fd_order=4)
    x, _ = H.diffusion_solve(p, a, dev(b), rtol=1e-14, maxit=10)
    assert np.max(np.abs(host(x) - ref)) < 1e-12 * np.max(np.abs(ref))


def _serial(w, nsteps, every, M, K, tol=1e-10):
    po = oracle_problem(w)
    lev = Level(po, M, w["dt"])
    y = rest(po.N)
    ctx = H.Context(lib_problem(w), H.make_method(M=(M, 1), dt=w["dt"], max_iter=K,
                                                  cg_rtol=1e-14, cg_maxit=300, solver="dct"))
    for n0 in range(0, nsteps, every):
        y = run_serial(lev, y, every, K, step0=n0)
        ctx.advance(every)
        e = field_errors(host(ctx.get_state(0, 0, 0)), y)
        assert np.max(e) < tol, (n0 + every, np.max(e))
    st = ctx.stats()
    assert st["steps"] == nsteps and st["cg_iters"] == 0
    ctx.destroy()
    return y


@pytest.mark.parametrize("kind,dims,order", [("cable1d", (64,), 4), ("slab2d", (31, 23), 4),
                                             ("slab3d", (10, 8, 6), 4), ("slab2d", (31, 23), 2),
                                             ("slab2d", (32, 16), 4), ("slab3d", (8, 4, 4), 4)])
def test_dct_serial_parity(kind, dims, order):
    """Serial hybrid SDC with the DCT-II solver, fourth-order stencil (and the
    second-order one), 1D/2D/3D, against the oracle's LU solves."""
    w = dict(si.workload(kind, dims=dims))
    w["fd_order"] = order
    y = _serial(w, 20, 10, 4, 4)
    assert np.all(np.isfinite(y))


@pytest.mark.parametrize("dims", [(8, 6, 4), (36, 18), (16, 8), (8, 4, 4), (64,)])
def test_dct_pfasst_iterates_parity(dims):
    """Two-level PFASST (space-coarsened, the coarse level fourth order on its
    own mesh) with DCT-II solves on both levels: every iterate of Algorithm 1
    matches the oracle slice by slice."""
    P = 4
    kind = {1: "cable1d", 2: "slab2d", 3: "slab3d"}[len(dims)]
    w = dict(si.workload(kind, dims=dims))
    w["dt"] = 0.1
    w["fd_order"] = 4
    h = oracle_hierarchy(w, 6, 3, 2)
    y0 = rest(h.levels[0].prob.N)
    m = H.make_method(M=(6, 3), levels=2, space_coarsen=2, P=P, dt=0.1, max_iter=50, tol=0.0,
                      burn_in=1, cg_rtol=1e-14, cg_maxit=300, solver="dct")
    ctx = H.Context(lib_problem(w), m, dev(y0))
    for k in (1, 2, 3):
        ctx.pfasst_iter()
        z, _, _ = pfasst_block(h, y0, P, k, tol=0.0)
        for n in range(P):
            for j in (0, 6):
                e = field_errors(host(ctx.get_state(0, n, j)), z[n][j])
                assert np.max(e) < 1e-10, (k, n, j, np.max(e))
    ctx.destroy()


@pytest.mark.parametrize("dims", [(16, 8), (36, 20)])
def test_dct_three_level_pfasst_iterates_parity(dims):
    """The paper's spatial setup with three levels (Sec. 5.1: M 6, 3, 1): the
    fourth-order stencil and DCT-II solves on every level, each level on a mesh
    coarsened twice in space; after each of three iterations every stage of
    every slice on the fine level and the coarsest level's two stages equal the
    oracle's.  16 x 8 takes the fast transforms on all three levels (16 x 8,
    8 x 4, 4 x 2), 36 x 20 the dense ones (36 x 20, 18 x 10, 9 x 5)."""
    from tests._parity import oracle_hierarchy_levels
    P = 4
    w = dict(si.workload("slab2d", dims=dims))
    w["dt"] = 0.1
    w["fd_order"] = 4
    h = oracle_hierarchy_levels(w, (6, 3, 1), 2)
    y0 = rest(h.levels[0].prob.N)
    m = H.make_method(M=(6, 3, 1), levels=3, space_coarsen=2, P=P, dt=0.1, max_iter=50, tol=0.0,
                      burn_in=1, cg_rtol=1e-14, cg_maxit=300, solver="dct")
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

"""Pins of the oracle's tissue operator (exact DCT-II diagonalisation), the
space transfers and the TTP06 restatement's structural properties (no GPU)."""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle import ttp06
from oracle.tissue import (ImplicitSolver, coarse_dims, dct_solve_uniform, laplacian,
                           prolong_space, restrict_space)


@pytest.mark.parametrize("dims,sigma", [((37,), (1.0,)), ((12, 9), (1.0, 1.0)),
                                        ((8, 6, 5), (3.0, 1.0, 0.5))])
def test_laplacian_solve_matches_dct(dims, sigma):
    dx = 0.025
    A = laplacian(dims, dx, tuple(sigma) + (1.0,) * (3 - len(sigma)))
    assert abs(A - A.T).max() == 0.0
    assert np.max(np.abs(A @ np.ones(A.shape[0]))) < 1e-9
    rng = np.random.default_rng(1)
    b = rng.standard_normal(A.shape[0])
    a = 0.05 * 0.2 / 1400.0
    x = ImplicitSolver(A).solve(b, a)
    x_dct = dct_solve_uniform(dims, dx, tuple(sigma) + (1.0,) * (3 - len(sigma)), a, b)
    assert np.max(np.abs(x - x_dct)) < 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("dims,sigma", [((37,), (1.0,)), ((12, 9), (1.0, 2.0)),
                                        ((8, 6, 5), (3.0, 1.0, 0.5)), ((3,), (1.0,))])
def test_fourth_order_laplacian_solve_matches_dct(dims, sigma):
    """The fourth-order operator is symmetric, annihilates constants, and its
    LU solve equals the DCT-II solve with the eigenvalues of its symbol."""
    dx = 0.025
    sg = tuple(sigma) + (1.0,) * (3 - len(sigma))
    A = laplacian(dims, dx, sg, order=4)
    assert abs(A - A.T).max() < 1e-9 * abs(A).max()
    assert np.max(np.abs(A @ np.ones(A.shape[0]))) < 1e-9
    rng = np.random.default_rng(1)
    b = rng.standard_normal(A.shape[0])
    a = 0.05 * 0.2 / 1400.0
    x = ImplicitSolver(A).solve(b, a)
    x_dct = dct_solve_uniform(dims, dx, sg, a, b, order=4)
    assert np.max(np.abs(x - x_dct)) < 1e-12 * np.max(np.abs(b))


def test_fourth_order_eigenvalues_and_rows():
    """The dense spectrum of the 1D mirrored operator equals its symbol at
    theta = pi k / n (so the DCT-II basis diagonalises it); an interior row is
    the five-point stencil and the first rows fold the mirror in."""
    from oracle.tissue import dct_eigenvalues, second_difference_4
    for n in (1, 2, 5, 12):
        ev = np.sort(np.linalg.eigvalsh(second_difference_4(n)))
        assert np.max(np.abs(ev - np.sort(dct_eigenvalues(n, 4)))) < 1e-12
    D = 12.0 * second_difference_4(7)
    assert np.allclose(D[3], [0, -1, 16, -30, 16, -1, 0], atol=0)
    assert np.allclose(D[0], [-14, 15, -1, 0, 0, 0, 0], atol=0)   # V_-1 = V_0, V_-2 = V_1
    assert np.allclose(D[1], [15, -30, 16, -1, 0, 0, 0], atol=0)
    assert np.allclose(D[6], D[0][::-1], atol=0)


@pytest.mark.parametrize("order,rate", [(2, 2.0), (4, 4.0)])
def test_laplacian_order_of_accuracy_on_a_no_flux_field(order, rate):
    """On V = cos(pi x / L) cos(2 pi y / L), whose odd derivatives vanish at the
    walls (so the mirrored field is smooth), the error of A V against the
    exact Laplacian falls with dx^order."""
    L = 1.0
    errs = []
    for n in (16, 32, 64):
        dx = L / n
        x = (np.arange(n) + 0.5) * dx
        X, Y = np.meshgrid(x, x)
        V = np.cos(np.pi * X / L) * np.cos(2 * np.pi * Y / L)
        exact = -((np.pi / L) ** 2 + (2 * np.pi / L) ** 2) * V
        AV = laplacian((n, n), dx, order=order) @ V.ravel()
        errs.append(np.max(np.abs(AV - exact.ravel())))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - rate) < 0.15), rates


def test_laplacian_stencil_rows():
    """Interior row of the 5-point stencil and a no-flux corner row."""
    dx = 0.5
    A = laplacian((4, 3), dx).toarray()
    k = 1.0 / dx ** 2
    p = 1 + 4 * 1  # (ix=1, iy=1)
    row = np.zeros(12)
    row[[0 + 4, 2 + 4, 1, 1 + 8]] = k
    row[p] = -4 * k
    assert np.array_equal(A[p], row)
    corner = np.zeros(12)
    corner[[1, 4]] = k
    corner[0] = -2 * k
    assert np.array_equal(A[0], corner)


def test_per_node_sigma_harmonic_faces():
    dims = (6, 5)
    s = np.exp(0.3 * np.random.default_rng(2).standard_normal(30))
    A = laplacian(dims, 0.1, sigma_node=s).toarray()
    # face between (0,0) and (1,0)
    assert A[0, 1] == pytest.approx(2 * s[0] * s[1] / (s[0] + s[1]) / 0.01, rel=1e-15)
    # constant field reduces to the uniform operator
    B = laplacian(dims, 0.1, sigma_node=np.full(30, 2.0)).toarray()
    C = laplacian(dims, 0.1, sigma=(2.0, 2.0, 2.0)).toarray()
    assert np.max(np.abs(B - C)) < 1e-12


@pytest.mark.parametrize("dims", [(8,), (6, 4), (4, 6, 2)])
def test_space_transfer(dims):
    nx, ny, nz = (tuple(dims) + (1, 1, 1))[:3]
    N = nx * ny * nz
    rng = np.random.default_rng(3)
    u = rng.standard_normal((2, N))
    cu = restrict_space(u, dims)
    cd = coarse_dims(dims)
    cx, cy, cz = (cd + (1, 1, 1))[:3]
    # brute-force average of the children
    U = u.reshape(2, nz, ny, nx)
    for iz in range(cz):
        for iy in range(cy):
            for ix in range(cx):
                zs = [2 * iz, 2 * iz + 1] if nz > 1 else [0]
                ys = [2 * iy, 2 * iy + 1] if ny > 1 else [0]
                xs = [2 * ix, 2 * ix + 1] if nx > 1 else [0]
                ref = U[:, zs][:, :, ys][:, :, :, xs].mean(axis=(1, 2, 3))
                assert np.allclose(cu.reshape(2, cz, cy, cx)[:, iz, iy, ix], ref, rtol=0, atol=1e-15)
    # prolongation: constants exact; restriction after prolongation is a (1/8, 3/4, 1/8) smoother
    c = np.full((1, cx * cy * cz), 3.5)
    assert np.max(np.abs(prolong_space(c, dims) - 3.5)) < 1e-15
    v = rng.standard_normal((1, cx * cy * cz))
    assert np.max(np.abs(restrict_space(prolong_space(v, dims), dims)
                         - _smooth_reference(v, cd))) < 1e-14
    # linear field in x is reproduced away from the walls
    xc = (np.arange(cx) + 0.5) * 2.0
    lin_c = np.tile(xc, cy * cz)[None]
    pf = prolong_space(lin_c, dims).reshape(nz, ny, nx)
    xf = np.arange(nx) + 0.5
    assert np.allclose(pf[..., 1:-1], np.broadcast_to(xf[1:-1], pf[..., 1:-1].shape), atol=1e-14)


def _smooth_reference(v, cd):
    """R P v = (1/8, 3/4, 1/8) smoothing per axis with mirror walls."""
    cx, cy, cz = (tuple(cd) + (1, 1, 1))[:3]
    w = v.reshape(cz, cy, cx).copy()
    for ax, n in ((2, cx), (1, cy), (0, cz)):
        if n > 1:
            lo = np.concatenate([np.take(w, [0], ax), np.take(w, np.arange(n - 1), ax)], ax)
            hi = np.concatenate([np.take(w, np.arange(1, n), ax), np.take(w, [n - 1], ax)], ax)
            w = 0.125 * lo + 0.75 * w + 0.125 * hi
    return w.reshape(1, -1)


def test_ttp06_rest_state_is_near_equilibrium():
    y = ttp06.rest_state()[:, None]
    I_ion, ha, L, inf = ttp06.evaluate(y)
    assert abs(I_ion[0]) < 0.01          # |dV/dt| < 0.01 mV/ms
    assert np.max(np.abs(ha)) < 1e-3
    assert np.all(L < 0)


def test_ttp06_fast_gates_of_the_published_state_are_at_steady_state():
    """The model publication's epicardial end-diastolic state (its table of
    initial values, `rest_state`) was taken after long pacing; the fast gates
    m, h, d, r and s relax within a few ms, so their tabulated values are the
    steady states w_inf(V) at the tabulated V = -85.23 mV.  The steady-state
    curves come from the publication's gating equations, a separate source:
    a wrong half-activation voltage or slope in one of them (a shift of 0.5 mV
    moves m_inf by 11%) fails here; the five agree to 0.3%.  The slow gates (j, xr1, xs, f, f2, fCass)
    are still relaxing at end-diastole and are not compared."""
    y = ttp06.rest_state()
    inf, tau = ttp06.gates(np.array([y[0]]), np.array([y[3]]))
    for g, field in ((0, 7), (1, 8), (6, 13), (7, 14), (8, 15)):  # m h r s d
        assert abs(inf[g, 0] - y[field]) < 0.01 * y[field], (ttp06.FIELD_NAMES[field],
                                                            inf[g, 0], y[field])
        assert tau[g, 0] < 10.0  # fast: relaxed long before the end of diastole


def test_ttp06_gate_ranges_and_cal_limit():
    y = si.random_states(20000, seed=5)
    I_ion, ha, L, inf = ttp06.evaluate(y)
    assert np.all(np.isfinite(I_ion)) and np.all(np.isfinite(ha))
    assert np.all((inf >= 0) & (inf <= 1)) and np.all(L < 0)
    # removable singularity of I_CaL at V = 15 mV: continuous through it
    yy = np.repeat(ttp06.rest_state()[:, None], 3, axis=1)
    yy[0] = [15.0 - 1e-7, 15.0, 15.0 + 1e-7]
    yy[15] = 0.5
    cal = ttp06.currents(yy)["CaL"]
    assert abs(cal[1] - cal[0]) < 1e-5 * abs(cal[1]) and abs(cal[2] - cal[1]) < 1e-5 * abs(cal[1])


def test_ttp06_conductance_scalings():
    y = si.random_states(100, seed=6)
    base = ttp06.currents(y)
    sc = ttp06.currents(y, (1.1, 0.9, 1.2))
    assert np.allclose(sc["Na"], 1.1 * base["Na"], rtol=1e-14)
    assert np.allclose(sc["CaL"], 0.9 * base["CaL"], rtol=1e-14)
    assert np.allclose(sc["Kr"], 1.2 * base["Kr"], rtol=1e-14)
    assert np.allclose(sc["K1"], base["K1"], rtol=0)


def test_ttp06_jacobian_spectral_radius_is_of_order_1000():
    """Sec. 5 (model setup) gives the spectral radius of the Jacobian of the
    ionic right-hand side f_E + f_e of the TTP06 model as about 1000 (1/ms) for
    states away from equilibrium.  Along a stimulated single-cell action
    potential (0..400 ms) the largest spectral radius of the central-difference
    Jacobian of the oracle's 19-state right-hand side must be of that order
    (within a factor 2); a rate constant of the fastest gate written wrong by a
    factor of ten, or an ionic current with a wrong sign, fails this."""
    from scipy.integrate import solve_ivp

    from oracle.problems import Monodomain

    p = Monodomain((1,), 0.01, stim_w=np.ones(1), stim_amp=50.0, stim_t0=0.0, stim_dur=1.0)

    def rhs(t, y):
        y = y.reshape(19, 1)
        return (p.f_E(t, y) + p.lam(y) * (y - p.y_inf(y))).ravel()

    sol = solve_ivp(rhs, (0.0, 400.0), ttp06.rest_state(), method="LSODA", rtol=1e-8,
                    atol=1e-10, dense_output=True, max_step=0.5)
    assert sol.y[0].max() > 20.0  # the stimulus triggered an action potential

    def rho(y):
        J = np.empty((19, 19))
        for m in range(19):
            h = 1e-6 * max(1.0, abs(y[m]))
            e = np.zeros(19)
            e[m] = h
            J[:, m] = (rhs(5.0, y + e) - rhs(5.0, y - e)) / (2.0 * h)  # t = 5: no stimulus
        return np.max(np.abs(np.linalg.eigvals(J)))

    times = np.concatenate([np.linspace(0.25, 20.0, 40), np.linspace(25.0, 400.0, 76)])
    rhos = np.array([rho(sol.sol(t)) for t in times])
    Vs = np.array([sol.sol(t)[0] for t in times])
    off_eq = Vs > -84.0  # away from the rest potential (-85.2 mV)
    assert off_eq.sum() > 50
    assert 500.0 < rhos[off_eq].max() < 2000.0

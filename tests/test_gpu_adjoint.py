"""The discrete adjoint of serial hybrid SDC (hsdc_misfit_forward/backward,
through the C ABI and torch.autograd) against central finite differences of
the FP64 oracle's forward run.

Reduced adjoint workload: 16 x 16 slab, per-node lognormal sigma, a 4 x 4
corner stimulus, TTP06, M 4, K 4, dt 0.05 ms, 2 ms (40 steps), 8 probes
sampled every 0.5 ms; targets from the oracle run at perturbed parameters
(sigma x exp(0.1 N(0,1)), g_Na x 1.1, g_CaL x 0.9, g_Kr x 1.2)."""
import numpy as np
import pytest
import torch

import synthetic_inputs as si
from oracle import ttp06
from oracle.hsdc import Level, run_serial
from oracle.problems import Monodomain

pytestmark = pytest.mark.gpu

H = pytest.importorskip("paper_2405_19994_amd.hsdc")

DIMS, DX, M, K, DT = (16, 16), 0.025, 4, 4, 0.05
NSTEPS, EVERY = 40, 10


def _case():
    N = DIMS[0] * DIMS[1]
    rng = np.random.default_rng(21)
    sigma0 = np.exp(0.3 * rng.standard_normal(N))
    truth = sigma0 * np.exp(0.1 * rng.standard_normal(N))
    probes = np.sort(rng.choice(N, 8, replace=False))
    stim = si.corner_weights(DIMS, (4, 4))
    return N, rng, sigma0, truth, probes, stim


def _oracle_V(sigma, g, probes, stim):
    """V at the probes every EVERY steps of the oracle's serial HSDC run."""
    N = DIMS[0] * DIMS[1]
    po = Monodomain(DIMS, DX, (1.0, 1.0, 1.0), sigma, 1400.0, 1.0, stim, 50.0, 0.0, 1.0,
                    g_scale=g, dt_ref=DT)
    Vs = []
    run_serial(Level(po, M, DT), np.repeat(ttp06.rest_state()[:, None], N, 1), NSTEPS, K,
               callback=lambda n, Y: Vs.append(Y[-1, 0, probes].copy()) if (n + 1) % EVERY == 0
               else None)
    return np.array(Vs)


def test_adjoint_gradient_matches_oracle_central_differences():
    """Loss equal to the oracle's (1e-9 relative); the gradient along two
    random directions of the conductivity field and along each conductance
    scaling equal to the oracle's central difference with h = 1e-6.  The
    tolerance, 1e-5 relative to the derivative, covers the difference
    quotient's truncation (h^2 terms, about 1e-12) and its rounding (the
    loss's rounding of about 1e-12 relative divided by h, about 1e-6 of the
    derivative), and the solves of the device run (1e-14 relative)."""
    from paper_2405_19994_amd.adjoint import probe_misfit
    N, rng, sigma0, truth, probes, stim = _case()
    targets = _oracle_V(truth, (1.1, 0.9, 1.2), probes, stim)

    def oracle_loss(sig, g):
        return float(np.sum((_oracle_V(sig, g, probes, stim) - targets) ** 2))

    spec = dict(dims=DIMS, dx=DX, chi=1400.0, Cm=1.0,
                stim_w=torch.tensor(stim, dtype=torch.float64, device="cuda"),
                stim_amp=50.0, stim_t0=0.0, stim_dur=1.0,
                method=H.make_method(M=(M, 1), dt=DT, max_iter=K, cg_rtol=1e-14, cg_maxit=400),
                probes=torch.tensor(probes, dtype=torch.int64, device="cuda"),
                targets=torch.tensor(targets, dtype=torch.float64, device="cuda"),
                nsteps=NSTEPS, sample_every=EVERY)
    sig_t = torch.tensor(sigma0, dtype=torch.float64, device="cuda", requires_grad=True)
    g_t = torch.tensor([1.0, 1.0, 1.0], dtype=torch.float64, requires_grad=True)
    L = probe_misfit(sig_t, g_t, spec)
    L.backward()
    gsig = sig_t.grad.detach().cpu().numpy()
    gg = g_t.grad.detach().cpu().numpy()
    L0 = oracle_loss(sigma0, (1.0, 1.0, 1.0))
    assert abs(float(L.detach()) - L0) < 1e-9 * L0, (float(L.detach()), L0)
    h = 1e-6
    dirs = [("sigma", sigma0 * rng.standard_normal(N)) for _ in range(2)]
    dirs += [("g", np.eye(3)[q]) for q in range(3)]
    for kind, v in dirs:
        if kind == "sigma":
            fd = (oracle_loss(sigma0 + h * v, (1.0, 1.0, 1.0))
                  - oracle_loss(sigma0 - h * v, (1.0, 1.0, 1.0))) / (2 * h)
            ad = float(gsig @ v)
        else:
            fd = (oracle_loss(sigma0, tuple(1.0 + h * v)) - oracle_loss(sigma0, tuple(1.0 - h * v))) / (2 * h)
            ad = float(gg @ v)
        assert abs(fd - ad) <= 1e-5 * abs(fd), (kind, v[:3], fd, ad)


def test_adjoint_gradient_of_initial_state_and_repeat():
    """The same run's gradient with respect to the initial state along a random
    direction of V against the oracle's central difference, and a second
    backward call on the same handle gives the same gradients."""
    N, rng, sigma0, truth, probes, stim = _case()
    targets = _oracle_V(truth, (1.1, 0.9, 1.2), probes, stim)
    prob = H.make_problem(DIMS, DX, (1.0, 1.0, 1.0), torch.tensor(sigma0, dtype=torch.float64,
                                                                   device="cuda"),
                          1400.0, 1.0, (1.0, 1.0, 1.0),
                          torch.tensor(stim, dtype=torch.float64, device="cuda"), 50.0, 0.0, 1.0)
    m = H.Misfit(prob, H.make_method(M=(M, 1), dt=DT, max_iter=K, cg_rtol=1e-14, cg_maxit=400),
                 torch.tensor(probes, dtype=torch.int64, device="cuda"),
                 torch.tensor(targets, dtype=torch.float64, device="cuda"), NSTEPS, EVERY)
    ds1, dg1, dy1 = m.backward(sigma=True, y0=True)
    ds2, dg2, dy2 = m.backward(sigma=True, y0=True)
    m.destroy()
    assert torch.equal(ds1, ds2) and np.array_equal(dg1, dg2) and torch.equal(dy1, dy2)
    v = rng.standard_normal(N)
    y0 = np.repeat(ttp06.rest_state()[:, None], N, 1)

    def loss_from(y):
        po = Monodomain(DIMS, DX, (1.0, 1.0, 1.0), sigma0, 1400.0, 1.0, stim, 50.0, 0.0, 1.0,
                        dt_ref=DT)
        Vs = []
        run_serial(Level(po, M, DT), y, NSTEPS, K,
                   callback=lambda n, Y: Vs.append(Y[-1, 0, probes].copy())
                   if (n + 1) % EVERY == 0 else None)
        return float(np.sum((np.array(Vs) - targets) ** 2))

    h = 1e-6
    yp, ym = y0.copy(), y0.copy()
    yp[0] += h * v
    ym[0] -= h * v
    fd = (loss_from(yp) - loss_from(ym)) / (2 * h)
    ad = float(dy1[0].cpu().numpy() @ v)
    assert abs(fd - ad) <= 1e-5 * abs(fd), (fd, ad)


@pytest.mark.parametrize("solver", ["chebyshev", "cg_plain"])
def test_adjoint_solver_options_agree(solver):
    """The adjoint's diffusion solves start from Chebyshev steps when the
    forward solves have Chebyshev tables (solvers "cg" and "chebyshev") and
    run plain CG otherwise ("cg_plain"); every solve converges to 1e-14, so
    the gradients of the three options agree to rounding (1e-8 relative),
    also on a 1D cable (the other stencil)."""
    N, rng, sigma0, truth, probes, stim = _case()
    targets = _oracle_V(truth, (1.1, 0.9, 1.2), probes, stim)

    def grads(dims, sig, st, pr, tg, solv):
        prob = H.make_problem(dims, DX, (1.0, 1.0, 1.0),
                              torch.tensor(sig, dtype=torch.float64, device="cuda"), 1400.0, 1.0,
                              (1.0, 1.0, 1.0), torch.tensor(st, dtype=torch.float64, device="cuda"),
                              50.0, 0.0, 1.0)
        m = H.Misfit(prob, H.make_method(M=(M, 1), dt=DT, max_iter=K, cg_rtol=1e-14, cg_maxit=400,
                                         solver=solv),
                     torch.tensor(pr, dtype=torch.int64, device="cuda"),
                     torch.tensor(tg, dtype=torch.float64, device="cuda"), NSTEPS, EVERY)
        ds, dg, dy = m.backward(sigma=True, y0=True)
        m.destroy()
        return ds.cpu().numpy(), np.asarray(dg), dy.cpu().numpy()

    def close(a, b):
        return np.max(np.abs(a - b)) <= 1e-8 * np.max(np.abs(b))

    ref = grads(DIMS, sigma0, stim, probes, targets, "cg")
    got = grads(DIMS, sigma0, stim, probes, targets, solver)
    for a, b in zip(got, ref):
        assert close(a, b), (np.max(np.abs(a - b)), np.max(np.abs(b)))
    # 1D: 64 cells, the first 4 stimulated, 4 probes, random targets
    n1 = 64
    s1 = np.exp(0.3 * rng.standard_normal(n1))
    st1 = np.zeros(n1)
    st1[:4] = 1.0
    pr1 = np.array([5, 20, 40, 60])
    tg1 = -80.0 + 10.0 * rng.standard_normal((NSTEPS // EVERY, 4))
    ref1 = grads((n1,), s1, st1, pr1, tg1, "cg")
    got1 = grads((n1,), s1, st1, pr1, tg1, solver)
    for a, b in zip(got1, ref1):
        assert close(a, b), (np.max(np.abs(a - b)), np.max(np.abs(b)))

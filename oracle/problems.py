"""ODE problems in the split form y' = f_I(t,y) + f_E(t,y) + f_e(t,y),
f_e = Lambda(y)(y - y_inf(y)) (eqs. def_ode, def_fe) (TEST INFRASTRUCTURE ONLY).

A problem exposes, for states y of shape (nf, N):
    f_I(t, y), solve_I(t, b, a)      (x - a f_I(t, x) = b, f_I linear)
    f_E(t, y), lam(y), y_inf(y)      (Lambda diagonal: same shape as y)
"""
import numpy as np

from . import ttp06
from .tissue import ImplicitSolver, laplacian


class ScalarTest:
    """The linear scalar test equation y' = lam_I y + lam_E y + lam_e y (eq. test),
    vectorised over independent (lam_I, lam_E, lam_e) triples: nf = 1, N triples."""

    def __init__(self, lam_I, lam_E, lam_e):
        self.lI = np.atleast_1d(np.asarray(lam_I, float))
        self.lE = np.atleast_1d(np.asarray(lam_E, float))
        self.le = np.atleast_1d(np.asarray(lam_e, float))
        self.nf = 1
        self.N = max(len(self.lI), len(self.lE), len(self.le))

    def f_I(self, t, y):
        return self.lI * y

    def solve_I(self, t, b, a):
        return b / (1.0 - a * self.lI)

    def f_E(self, t, y):
        return self.lE * y

    def lam(self, y):
        return np.broadcast_to(self.le, y.shape).copy()

    def y_inf(self, y):
        return np.zeros_like(y)


class Monodomain:
    """Semi-discrete monodomain equation with the TTP06 cell model (eqs. sd_sys,
    def_f_IE, def_Lambda):

        f_I = ((chi Cm)^-1 A V, 0, 0)
        f_E = (Cm^-1 (I_stim(t) - Cm I_TTP(y)), h_a(y), 0)
        f_e = (0, 0, Lambda_g (w_g - w_g,inf))

    Units: ms, mV, cm, mS/cm, uF/cm^2, uA/cm^2.  The TTP06 currents are per unit
    capacitance (pA/pF), so the membrane current density is Cm * I_TTP.
    The stimulus is I_stim(t, x) = stim_amp * stim_w(x) while
    stim_t0 < t <= stim_t0 + stim_dur, else 0 (both ends shifted by 1e-9 dt so
    that the decision does not depend on the rounding of t_{n,j}).  The window
    is open on the left and closed on the right because the collocation
    polynomial interpolates the nodes c_1..c_M in (0, 1]: a window made of
    whole steps is then reproduced exactly by every step it covers."""

    nf = ttp06.NF

    def __init__(self, dims, dx, sigma=(1.0, 1.0, 1.0), sigma_node=None, chi=1400.0,
                 Cm=1.0, stim_w=None, stim_amp=0.0, stim_t0=0.0, stim_dur=0.0,
                 g_scale=(1.0, 1.0, 1.0), dt_ref=0.05, fd_order=2):
        self.dims = tuple(int(n) for n in dims)
        self.N = int(np.prod(self.dims))
        self.dx = float(dx)
        self.sigma = tuple(float(s) for s in (tuple(sigma) + (1.0, 1.0, 1.0))[:3])
        self.sigma_node = None if sigma_node is None else np.asarray(sigma_node, float).ravel()
        self.chi, self.Cm = float(chi), float(Cm)
        self.stim_w = np.zeros(self.N) if stim_w is None else np.asarray(stim_w, float).ravel()
        self.stim_amp, self.stim_t0, self.stim_dur = float(stim_amp), float(stim_t0), float(stim_dur)
        self.g_scale = tuple(float(g) for g in g_scale)
        self.eps_t = 1e-9 * dt_ref
        self.fd_order = int(fd_order)
        A = laplacian(self.dims, self.dx, self.sigma, self.sigma_node, self.fd_order)
        self.K = A / (self.chi * self.Cm)
        self.solver = ImplicitSolver(self.K)

    def stim_on(self, t):
        return (self.stim_t0 + self.eps_t < t) and (t <= self.stim_t0 + self.stim_dur + self.eps_t)

    def f_I(self, t, y):
        out = np.zeros_like(y)
        out[0] = self.K @ y[0]
        return out

    def solve_I(self, t, b, a):
        x = np.array(b, float, copy=True)
        x[0] = self.solver.solve(b[0], a)
        return x

    def _ionic(self, y):
        # memo: f_E, lam and y_inf of the same state share one evaluation
        key = (y.shape, hash(np.ascontiguousarray(y).tobytes()))
        memo = self.__dict__.setdefault("_memo", {})
        if key not in memo:
            if len(memo) >= 32:
                memo.pop(next(iter(memo)))
            memo[key] = ttp06.evaluate(y, self.g_scale)
        return memo[key]

    def f_E(self, t, y):
        I_ion, ha, _, _ = self._ionic(y)
        out = np.zeros_like(y)
        I_stim = self.stim_amp * self.stim_w if self.stim_on(t) else 0.0
        out[0] = (I_stim - self.Cm * I_ion) / self.Cm
        out[ttp06.AUX] = ha
        return out

    def lam(self, y):
        _, _, L, _ = self._ionic(y)
        out = np.zeros_like(y)
        out[ttp06.GATES] = L
        return out

    def y_inf(self, y):
        _, _, _, inf = self._ionic(y)
        out = np.zeros_like(y)
        out[ttp06.GATES] = inf
        return out

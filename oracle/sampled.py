"""The HSDC operators at a subset of mesh nodes (TEST INFRASTRUCTURE ONLY,
see package doc).

Everything in P and C (eqs. def_P, def_C) is node-local except f_I = K V, whose
value at a node needs its stencil neighbours.  Given whole stage vectors, the
values of K V_j at the sampled nodes are computed once per stage (a sparse
row-block product) and the rest of the operators is evaluated at the sampled
nodes only, so a sweep of a large mesh can be checked node by node.
"""
import numpy as np

from .hsdc import Level
from .problems import Monodomain


class FrozenDiffusion:
    """Monodomain terms at `rows` of `full`, with f_I(t, .) = KV[t] supplied per
    stage time t_{n,j}."""

    def __init__(self, full, rows, kv_by_stage, times):
        self.rows = np.asarray(rows)
        self.N = len(self.rows)
        self.nf = full.nf
        self.cell = Monodomain((self.N,), full.dx, (0.0, 0.0, 0.0), None, full.chi, full.Cm,
                               full.stim_w[self.rows], full.stim_amp, full.stim_t0, full.stim_dur,
                               full.g_scale)
        self.cell.eps_t = full.eps_t
        self._kv = {round(float(t), 9): kv for t, kv in zip(times, kv_by_stage)}

    def f_I(self, t, y):
        out = np.zeros_like(y)
        out[0] = self._kv[round(float(t), 9)]
        return out

    def f_E(self, t, y):
        return self.cell.f_E(t, y)

    def lam(self, y):
        return self.cell.lam(y)

    def y_inf(self, y):
        return self.cell.y_inf(y)

    def solve_I(self, t, b, a):
        raise NotImplementedError("sampled operators are for evaluation only")


def sweep_defect(full, M, dt, step, Yk, Ynew, yn, rows):
    """P(Y^{k+1}) - [(P - C)(Y^k) + 1 (x) y_n] at the nodes `rows` (eq. prec_picard,
    Y^k with its start value replaced by y_n as in Level.sweep), for whole stage
    vectors Yk, Ynew of shape (M+1, nf, N).  Returns (M+1, nf, len(rows))."""
    times = [(step + c) * dt for c in np.concatenate([[0.0], Level(full, M, dt).c])]

    def level_for(Y):
        kv = [full.K[rows] @ Y[j, 0] for j in range(M + 1)]
        return Level(FrozenDiffusion(full, rows, kv, times), M, dt)

    Yk = np.array(Yk, float, copy=True)
    Yk[0] = yn                      # the right-hand side takes the new start value
    lev_new, lev_old = level_for(Ynew), level_for(Yk)
    Yn = Ynew[:, :, rows]
    Yo = Yk[:, :, rows]
    rhs = lev_old.P(step, Yo) - lev_old.C(step, Yo) + yn[None][:, :, rows]
    return lev_new.P(step, Yn) - rhs


def collocation_defect(full, M, dt, step, Y, u, rows):
    """C(Y) - 1 (x) u at the nodes `rows` (eq. def_C; row 0 is the start-value
    jump Y_0 - u), for a whole stage vector Y of shape (M+1, nf, N) and start
    value u of shape (nf, N).  Returns (M+1, nf, len(rows))."""
    times = [(step + c) * dt for c in np.concatenate([[0.0], Level(full, M, dt).c])]
    kv = [full.K[rows] @ Y[j, 0] for j in range(M + 1)]
    lev = Level(FrozenDiffusion(full, rows, kv, times), M, dt)
    return lev.C(step, Y[:, :, rows]) - np.asarray(u, float)[None][:, :, rows]

"""Hybrid SDC on one time step (TEST INFRASTRUCTURE ONLY, see package doc).

Notation follows Sec. 3.1.  A stage vector Y has shape (M+1, nf, N):
Y[0] = y_{n,0}, ..., Y[M] = y_{n,M}, at times t_{n,j} = (n + c_j) dt.

Readings of the paper used here (the full list is in the design notes):
* Lambda_n = Lambda(y_{n,0}) (text after eq. def_A_matrix: y_n is replaced by
  y_{n,0} in g and in A(dt Lambda)).
* In the preconditioned Picard iteration (eq. prec_picard) the right-hand side
  (P - C)(y^k) is evaluated at y^k with its start value replaced by the start
  value u of the new iterate (row 0 of the sweep gives y^{k+1}_{n,0} = u), so
  that P, C, Lambda_n and g_n of both sides belong to the same step, as in
  Sec. 3.1.3 where y^k_{n,0} = y_n for every k.  For a single step nothing is
  replaced; in PFASST the start values move between iterations, and evaluating
  the right-hand side at the old start value makes the two-level iteration
  unstable in the stiff regime that Sec. 4.1 reports stable (L = 2, P = 4, K = 2).
* f_E(y_{n,j-1}) in P is taken at time t_{n,j-1}; g(y_{n,j}) at t_{n,j}.
* f_I(y_{n,j}) inside P is evaluated by applying the operator to the stage
  (never recovered from the implicit solve's right-hand side).
"""
import numpy as np

from .coeffs import (exp_colloc_matrix, lagrange_derivatives_at_zero, node_spacings, phi,
                     radau_iia_nodes)


class Level:
    """One collocation level: a problem, M Radau IIA nodes and the step size."""

    def __init__(self, problem, M, dt, exponential=True):
        self.prob = problem
        self.M = int(M)
        self.dt = float(dt)
        # exponential=False gives the naive SDC of Sec. 4.2: Lambda_n replaced by 0
        self.exponential = bool(exponential)
        self.c = radau_iia_nodes(self.M)
        self.c0 = np.concatenate([[0.0], self.c])
        self.d = node_spacings(self.c)
        self.w = lagrange_derivatives_at_zero(self.c)

    def t(self, step, j):
        """t_{n,j} = (n + c_j) dt."""
        return (step + self.c0[j]) * self.dt

    def spread(self, y):
        """1 (x) y: every stage equal to y (initial guess y^0, eq. prec_picard)."""
        return np.repeat(np.asarray(y, float)[None], self.M + 1, axis=0)

    def coefficients(self, y0):
        """Lambda_n = Lambda(y_{n,0}), a_ij(dt Lambda_n) with shape (nf, N, M, M)
        and phi_1(d_j dt Lambda_n) with shape (M, nf, N).

        Entries with Lambda_n = 0 take a(0) = Q.  Results are memoised per
        y_{n,0} (the same start value serves every sweep of a step)."""
        key = (y0.shape, hash(np.ascontiguousarray(y0).tobytes()))
        cache = self.__dict__.setdefault("_coef_cache", {})
        if key in cache:
            return cache[key]
        L0 = self.prob.lam(y0) if self.exponential else np.zeros_like(y0)
        z = self.dt * L0
        nz = z != 0.0
        A = np.empty(z.shape + (self.M, self.M))
        A[...] = exp_colloc_matrix(np.zeros(()), self.c, self.w)
        A[nz] = exp_colloc_matrix(z[nz], self.c, self.w)
        phi1 = np.stack([phi(1, self.d[j] * z) for j in range(self.M)])
        if len(cache) >= 8:
            cache.pop(next(iter(cache)))
        cache[key] = (L0, A, phi1)
        return cache[key]

    def f_e(self, y):
        return self.prob.lam(y) * (y - self.prob.y_inf(y))

    def g(self, step, j, y, y0, L0):
        """g_n(y) = f_I + f_E + f_e + Lambda_n (y_{n,0} - y) (eq. def_g) at t_{n,j}."""
        t = self.t(step, j)
        return self.prob.f_I(t, y) + self.prob.f_E(t, y) + self.f_e(y) + L0 * (y0 - y)

    def integrals(self, step, Y, coef=None):
        """I_i = sum_{j=1..M} a_ij(dt Lambda_n) g_n(y_{n,j}), i = 1..M (rows of
        A(dt Lambda) G in eq. def_C); returns shape (M, nf, N)."""
        L0, A, _ = self.coefficients(Y[0]) if coef is None else coef
        G = np.stack([self.g(step, j, Y[j], Y[0], L0) for j in range(1, self.M + 1)])
        I = np.zeros_like(G)
        for i in range(self.M):
            for j in range(self.M):
                I[i] += A[..., i, j] * G[j]
        return I

    def C(self, step, Y, coef=None):
        """C(y_n) = (I - dt A(dt Lambda(y_{n,0})) G)(y_n) (eqs. def_C, def_A_matrix)."""
        out = np.array(Y, float, copy=True)
        out[1:] -= self.dt * self.integrals(step, Y, coef)
        return out

    def Phi(self, step, Y, j, L0, phi1):
        """Summand of P_i (eq. def_P):
        f_I(y_j) + f_E(y_{j-1}) + phi_1(d_j dt Lambda_n)(f_e(y_{j-1}) + Lambda_n (y_{n,0} - y_{j-1}))."""
        p = self.prob
        return (p.f_I(self.t(step, j), Y[j]) + p.f_E(self.t(step, j - 1), Y[j - 1])
                + phi1[j - 1] * (self.f_e(Y[j - 1]) + L0 * (Y[0] - Y[j - 1])))

    def P(self, step, Y, coef=None):
        """Preconditioner P_i(y_n) = y_{n,i} - dt sum_{j<=i} d_j Phi_j (eq. def_P)."""
        L0, _, phi1 = self.coefficients(Y[0]) if coef is None else coef
        out = np.array(Y, float, copy=True)
        acc = np.zeros_like(Y[0])
        for i in range(1, self.M + 1):
            acc = acc + self.d[i - 1] * self.Phi(step, Y, i, L0, phi1)
            out[i] -= self.dt * acc
        return out

    def solve_P(self, step, rhs):
        """Solve P(Y) = rhs by forward substitution over the nodes: implicit in
        f_I (one linear solve per node), explicit in f_E, exponential Euler in
        f_e (Sec. 3.1.3)."""
        p = self.prob
        Y = np.empty_like(rhs)
        Y[0] = rhs[0]
        L0, _, phi1 = self.coefficients(Y[0])
        acc = np.zeros_like(Y[0])       # sum_{j<i} d_j Phi_j(Y)
        for i in range(1, self.M + 1):
            ti, tim1 = self.t(step, i), self.t(step, i - 1)
            expl = p.f_E(tim1, Y[i - 1]) + phi1[i - 1] * (self.f_e(Y[i - 1]) + L0 * (Y[0] - Y[i - 1]))
            a = self.dt * self.d[i - 1]
            b = rhs[i] + self.dt * acc + a * expl
            Y[i] = p.solve_I(ti, b, a)
            acc = acc + self.d[i - 1] * (p.f_I(ti, Y[i]) + expl)
        return Y

    def sweep(self, step, Yk, shift):
        """One preconditioned Picard iteration (eq. prec_picard):
        P(Y^{k+1}) = (P - C)(Y^k) + shift, where shift is 1 (x) y_n for a single
        step, or the block right-hand side b_n + tau_n + H y_{n-1} of PFASST.
        Row 0 of shift is the start value u of the new iterate; Y^k enters with
        its start value replaced by u (reading in the module doc)."""
        Y = np.array(Yk, float, copy=True)
        Y[0] = shift[0]
        coef = self.coefficients(Y[0])
        rhs = self.P(step, Y, coef) - self.C(step, Y, coef) + shift
        return self.solve_P(step, rhs)

    def residual(self, step, Y, u):
        """r_n = C(y_n) - 1 (x) u (the rows of D(z) - b, Alg. 1) and the relative
        residual ||r_n||_inf / ||y_n||_inf over all stages, fields and nodes."""
        r = self.C(step, Y) - u[None]
        return r, float(np.max(np.abs(r)) / np.max(np.abs(Y)))


def serial_step(lev, step, yn, K):
    """One HSDC step: y^0 = 1 (x) y_n, exactly K sweeps, y_{n+1} = y^K_{n,M}."""
    Y = lev.spread(yn)
    shift = lev.spread(yn)
    for _ in range(K):
        Y = lev.sweep(step, Y, shift)
    return Y


def run_serial(lev, y0, nsteps, K, step0=0, callback=None):
    """nsteps serial HSDC steps of K sweeps each from y0; returns y_{nsteps}."""
    y = np.asarray(y0, float)
    for n in range(step0, step0 + nsteps):
        Y = serial_step(lev, n, y, K)
        if callback is not None:
            callback(n, Y)
        y = Y[-1]
    return y


def collocation_solve(lev, step, yn, tol=1e-14, maxit=200):
    """Iterate sweeps until the relative residual is below tol: the fixed point
    of eq. prec_picard, i.e. the solution of eq. def_C."""
    Y = lev.spread(yn)
    shift = lev.spread(yn)
    for k in range(maxit):
        Y = lev.sweep(step, Y, shift)
        _, rel = lev.residual(step, Y, yn)
        if rel < tol:
            return Y, k + 1
    return Y, maxit

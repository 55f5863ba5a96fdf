"""Multilevel, parallel-in-time HSDC: Algorithm 1 of Sec. 3.2 (TEST
INFRASTRUCTURE ONLY, see package doc).

A block z is a list of P stage vectors (one per time slice, eq. erk_sys); slice n
of the block starting at global step `step0` is step step0 + n.  Levels are
ordered fine (index 0, the paper's l = 1) to coarse.

Readings of the paper used here:
* Burn-in (cited, not defined, by the paper): the staggered coarse predictor.
  Spread y_0 on every slice and restrict to the coarsest level; for stage
  s = 0..P-1 every slice n >= s does one coarsest-level sweep (tau = 0) whose
  start value is the coarsest end value that slice n-1 held at the end of stage
  s-1 (y_0 restricted for n = 0); then the difference to the restricted spread is
  prolonged level by level.  Skipped for P = 1, as the paper states.
* Exactly one sweep per level per iteration, in the order of Algorithm 1.
* Stop when every slice has ||r_n||_inf < tol ||y_n||_inf, or after K
  iterations (Algorithm 1); tol <= 0 runs exactly K iterations.
* prefix_stop (two levels): the variant Sec. 3.2 describes beside Algorithm 1,
  where the slices whose residual, and that of every earlier slice, is below
  tol stop iterating.  A stopped slice keeps its fine and coarse iterates; the
  first active slice takes its start value from the stopped slice before it,
  on each level from that level's iterate (the coarse one from its last Q^seq
  sweep).
* L = 1 runs Q^seq sweeps on the single level (tau = 0).
"""
import numpy as np

from .coeffs import prolongation_matrix, restriction_matrix


class Hierarchy:
    """Levels plus the transfer operators S (restriction R in time composed with
    the space restriction) and U (prolongation T in time composed with the space
    prolongation) between consecutive levels."""

    def __init__(self, levels, space_restrict=None, space_prolong=None):
        self.levels = list(levels)
        L = len(self.levels)
        ident = lambda u: u
        self.rs = list(space_restrict) if space_restrict else [ident] * (L - 1)
        self.ps = list(space_prolong) if space_prolong else [ident] * (L - 1)
        self.R = [restriction_matrix(self.levels[l].c, self.levels[l + 1].c) for l in range(L - 1)]
        self.T = [prolongation_matrix(self.levels[l + 1].c, self.levels[l].c) for l in range(L - 1)]

    def S(self, l, Y):
        """Restriction of one stage vector from level l to level l+1."""
        return np.tensordot(self.R[l], self.rs[l](Y), axes=(1, 0))

    def U(self, l, Y):
        """Prolongation of one stage vector from level l+1 to level l."""
        return np.tensordot(self.T[l], self.ps[l](Y), axes=(1, 0))

    def D(self, l, step0, z):
        """D(z) = (C_P - E (x) H)(z) (eq. def_D) at level l."""
        lev = self.levels[l]
        out = []
        for n, Y in enumerate(z):
            r = lev.C(step0 + n, Y)
            if n > 0:
                r = r - z[n - 1][-1][None]
            out.append(r)
        return out

    def solve_Q(self, l, step0, X, rhs_extra, seq):
        """Solve Q(z) = (Q - D)(X) + rhs_extra with Q = Q^seq or Q^par (eq. def_Q).

        Slice by slice this is one sweep P(y_n) = (P - C)(x_n) + rhs_extra_n + 1 (x) u_n
        with u_n the new (Q^seq) or the given (Q^par) end value of slice n-1."""
        lev = self.levels[l]
        out = []
        for n, Xn in enumerate(X):
            shift = np.array(rhs_extra[n], float, copy=True)
            if n > 0:
                prev_end = out[n - 1][-1] if seq else X[n - 1][-1]
                shift = shift + prev_end[None]
            out.append(lev.sweep(step0 + n, Xn, shift))
        return out


def _zeros_like_block(z):
    return [np.zeros_like(Y) for Y in z]


def block_rhs(h, y0, P):
    """b_1 = (1 (x) y_0, 0, ..., 0) and b_l = S b_{l-1} (Algorithm 1)."""
    fine = h.levels[0]
    b = [[fine.spread(y0)] + [np.zeros_like(fine.spread(y0)) for _ in range(P - 1)]]
    for l in range(len(h.levels) - 1):
        b.append([h.S(l, Y) for Y in b[l]])
    return b


def burn_in(h, y0, P, step0, b):
    """Initial block iterate on the finest level (reading stated in the module doc)."""
    L = len(h.levels)
    z = [[h.levels[0].spread(y0) for _ in range(P)]]
    if P == 1 or L == 1:
        return z[0]
    for l in range(L - 1):
        z.append([h.S(l, Y) for Y in z[l]])
    spread_restricted = [list(zl) for zl in z]
    Lc = L - 1
    lev = h.levels[Lc]
    X = z[Lc]
    for s in range(P):
        ends = [Y[-1].copy() for Y in X]
        for n in range(s, P):
            shift = np.array(b[Lc][n], float, copy=True)
            if n > 0:
                shift = shift + ends[n - 1][None]
            X[n] = lev.sweep(step0 + n, X[n], shift)
    for l in range(Lc - 1, -1, -1):
        for n in range(P):
            z[l][n] = spread_restricted[l][n] + h.U(l, z[l + 1][n] - h.S(l, spread_restricted[l][n]))
    return z[0]


def _iterate_prefix(h, z, zc_store, a0, step0, b):
    """One iteration of the two-level algorithm over the active slices a0..P-1
    (prefix_stop); z and zc_store (the coarse iterates) are updated in place.
    tau is formed without the previous-slice terms of D, which cancel in it."""
    P = len(z)
    lf, lc = h.levels
    act = range(a0, P)
    Sz = {n: h.S(0, z[n]) for n in act}
    tau = {n: lc.C(step0 + n, Sz[n]) - h.S(0, lf.C(step0 + n, z[n])) for n in act}
    for n in act:  # Q^seq on the coarse level
        shift = b[1][n] + tau[n]
        if n > 0:
            shift = shift + zc_store[n - 1][-1][None]
        zc_store[n] = lc.sweep(step0 + n, Sz[n], shift)
    X = {n: z[n] + h.U(0, zc_store[n] - Sz[n]) for n in act}
    shifts = {}
    for n in act:  # Q^par on the fine level from the corrected iterate
        shifts[n] = np.array(b[0][n], float, copy=True)
        if n > 0:
            shifts[n] = shifts[n] + (X[n - 1] if n - 1 >= a0 else z[n - 1])[-1][None]
    for n in act:
        z[n] = lf.sweep(step0 + n, X[n], shifts[n])


def pfasst_block(h, y0, P, K, tol, step0=0, use_burn_in=True, z_init=None, callback=None,
                 prefix_stop=False):
    """Algorithm 1: P steps from y0.  Returns (z_fine, residual history, k).

    residual history: list over iterations of the P relative residuals.
    callback(k, z_fine, z_coarsest), if given, sees every iterate k = 1, 2, ...
    (z_coarsest: the coarsest level's iterate after its Q^seq sweep, or None
    for one level)."""
    L = len(h.levels)
    b = block_rhs(h, y0, P)
    if z_init is not None:
        z = [np.array(Y, float, copy=True) for Y in z_init]
    elif use_burn_in:
        z = burn_in(h, y0, P, step0, b)
    else:
        z = [h.levels[0].spread(y0) for _ in range(P)]
    hist = []
    k = 0
    converged = False
    if prefix_stop and L != 2:
        raise ValueError("prefix_stop is for two levels")
    a0 = 0
    zc_store = [None] * P
    rel = None
    while not converged and k < K:
        zc = None
        if prefix_stop:
            _iterate_prefix(h, z, zc_store, a0, step0, b)
            zc = zc_store
            k += 1
            r = h.D(0, step0, z)
            new = []
            for n in range(P):
                rn = r[n] - b[0][n]
                new.append(float(np.max(np.abs(rn)) / np.max(np.abs(z[n]))))
            rel = [rel[n] if (rel is not None and n < a0) else new[n] for n in range(P)]
            hist.append(rel)
            if callback is not None:
                callback(k, z, zc)
            while tol > 0 and a0 < P and rel[a0] < tol:
                a0 += 1
            converged = a0 == P
            continue
        if L == 1:
            z = h.solve_Q(0, step0, z, b[0], seq=True)
        else:
            zh = [None] * L
            tau = [None] * L
            zh[0] = z
            tau[0] = _zeros_like_block(z)
            for l in range(1, L):
                Sz = [h.S(l - 1, Y) for Y in zh[l - 1]]
                Dc = h.D(l, step0, Sz)
                Df = h.D(l - 1, step0, zh[l - 1])
                tau[l] = [Dc[n] - h.S(l - 1, Df[n]) + h.S(l - 1, tau[l - 1][n]) for n in range(P)]
                extra = [b[l][n] + tau[l][n] for n in range(P)]
                zh[l] = h.solve_Q(l, step0, Sz, extra, seq=(l == L - 1))
            znew = zh[L - 1]
            zc = znew
            for l in range(L - 2, -1, -1):
                corr = [h.U(l, znew[n] - h.S(l, zh[l][n])) for n in range(P)]
                X = [zh[l][n] + corr[n] for n in range(P)]
                extra = [b[l][n] + tau[l][n] for n in range(P)]
                znew = h.solve_Q(l, step0, X, extra, seq=False)
            z = znew
        k += 1
        r = h.D(0, step0, z)
        rel = []
        for n in range(P):
            rn = r[n] - b[0][n]
            rel.append(float(np.max(np.abs(rn)) / np.max(np.abs(z[n]))))
        hist.append(rel)
        if callback is not None:
            callback(k, z, zc)
        converged = tol > 0 and all(x < tol for x in rel)
    return z, hist, k


def run_pfasst(h, y0, nblocks, P, K, tol, use_burn_in=True, callback=None):
    """nblocks consecutive blocks of P steps; the next block starts from y_{P-1,M}."""
    y = np.asarray(y0, float)
    iters = []
    for blk in range(nblocks):
        z, hist, k = pfasst_block(h, y, P, K, tol, step0=blk * P, use_burn_in=use_burn_in)
        iters.append(k)
        if callback is not None:
            callback(blk, z, hist)
        y = z[-1][-1]
    return y, iters

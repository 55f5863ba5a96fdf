"""Collocation coefficients of hybrid SDC (TEST INFRASTRUCTURE ONLY, see package doc).

* Radau IIA nodes c_1 < ... < c_M = 1 with c_0 = 0 (Sec. 3.1.2, eq. piN).
  Pinned by the textbook Radau IIA tableaux (tests/golden/radau_iia.txt).
* Lagrange derivative weights w_j^k = l_j^{(k)}(0) (Appendix A, eqs. fornberg,
  fornberg_ell).  Pinned by the moment identity sum_j w_j^k c_j^m = k! delta_km.
* phi_k(z) (Appendix A, eq. def_phik).  Pinned against mpmath quadrature of the
  defining integral, phi_k(0) = 1/k! and the expm identity.
* a_ij(z) (eq. def_aij, computed with eq. def_aij_computable).  Pinned against
  mpmath quadrature of eq. def_aij and the row-sum / moment identities.
* Lagrange time transfer R (restriction) and T (prolongation) (Sec. 3.2).
  Pinned by exact reproduction of polynomials of degree < M.
"""
import math

import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly

_LD = np.longdouble
if np.finfo(_LD).eps > 1e-18:  # x86 80-bit extended precision is required
    raise RuntimeError("oracle.coeffs needs an extended-precision long double")


def radau_iia_nodes(M):
    """Right Radau nodes on [0, 1]: the roots of P_M(2c-1) - P_{M-1}(2c-1),
    c_M = 1 (Sec. 3.1.2: Radau IIA collocation nodes with c_M = 1)."""
    if M < 1:
        raise ValueError("M >= 1")
    if M == 1:
        return np.array([1.0])
    coef = np.zeros(M + 1)
    coef[M] = 1.0
    coef[M - 1] = -1.0
    x = np.sort(npleg.legroots(coef).real)
    dcoef = npleg.legder(coef)
    for _ in range(3):  # Newton polish in the Legendre basis
        x = x - npleg.legval(x, coef) / npleg.legval(x, dcoef)
    c = (x + 1.0) / 2.0
    c[-1] = 1.0
    return c


def node_spacings(c):
    """d_j = c_j - c_{j-1}, j = 1..M, with c_0 = 0 (text after eq. deriv_P_a)."""
    return np.diff(np.concatenate([[0.0], c]))


def lagrange_derivatives_at_zero(c):
    """w[k, j] = l_j^{(k)}(0), k = 0..M-1, j = 1..M (Appendix A, eq. fornberg).

    Written from the definition: expand each Lagrange basis polynomial l_j in
    the power basis and read its Taylor coefficients at 0."""
    c = np.asarray(c, float)
    M = len(c)
    w = np.empty((M, M))
    for j in range(M):
        others = np.delete(c, j)
        coeffs = nppoly.polyfromroots(others) / np.prod(c[j] - others)
        coeffs = np.concatenate([coeffs, np.zeros(M - len(coeffs))])
        for k in range(M):
            w[k, j] = math.factorial(k) * coeffs[k]
    return w


def phi(k, x):
    """phi_k(x) = 1/(k-1)! * int_0^1 e^{(1-r) x} r^{k-1} dr for k >= 1 and
    phi_0(x) = e^x (Appendix A, eq. def_phik).

    Evaluated in 80-bit extended precision from two exact expressions of the
    same function: the Taylor series sum_m x^m/(m+k)! for |x| < 2 and the closed
    form (e^x - sum_{m<k} x^m/m!) / x^k for |x| >= 2; the result is rounded to
    FP64."""
    x = np.asarray(x, dtype=float)
    xl = x.astype(_LD)
    out = np.empty(x.shape, dtype=_LD)
    small = np.abs(x) < 2.0
    xs = xl[small]
    term = np.full(xs.shape, _LD(1) / _LD(math.factorial(k)))
    acc = term.copy()
    for m in range(1, 40):
        term = term * xs / _LD(m + k)
        acc = acc + term
    out[small] = acc
    xb = xl[~small]
    partial = np.zeros(xb.shape, dtype=_LD)
    p = np.ones(xb.shape, dtype=_LD)
    for m in range(k):
        partial = partial + p
        p = p * xb / _LD(m + 1)
    out[~small] = (np.exp(xb) - partial) / xb ** k
    return out.astype(float)


def exp_colloc_matrix(z, c, w=None):
    """a_ij(z) = int_0^{c_i} e^{(c_i - s) z} l_j(s) ds for every entry of z
    (eq. def_aij), computed as sum_k c_i^k w_j^{k-1} phi_k(c_i z)
    (eq. def_aij_computable).  Returns an array of shape z.shape + (M, M)."""
    c = np.asarray(c, float)
    M = len(c)
    if w is None:
        w = lagrange_derivatives_at_zero(c)
    z = np.asarray(z, float)
    A = np.zeros(z.shape + (M, M))
    for i in range(M):
        x = c[i] * z
        for k in range(1, M + 1):
            pk = phi(k, x) * c[i] ** k
            A[..., i, :] += pk[..., None] * w[k - 1, :]
    return A


def collocation_matrix(c):
    """Q = a(0): the standard collocation weights q_ij = int_0^{c_i} l_j(s) ds
    (text after eq. def_A_matrix: z = 0 gives standard collocation)."""
    return exp_colloc_matrix(np.zeros(()), c)


def lagrange_basis_values(c_nodes, s):
    """L[a, j] = l_j(s_a) for the Lagrange basis through c_nodes (eq. piN)."""
    c_nodes = np.asarray(c_nodes, float)
    s = np.asarray(s, float)
    M = len(c_nodes)
    L = np.ones((len(s), M))
    for j in range(M):
        for m in range(M):
            if m != j:
                L[:, j] *= (s - c_nodes[m]) / (c_nodes[j] - c_nodes[m])
    return L


def restriction_matrix(c_fine, c_coarse):
    """Matrix of R_l^{l+1} (Sec. 3.2): row 0 copies y_{n,0}; row i interpolates
    the fine nodes c_1..c_Mf at the coarse node c_i (y_{n,0} is not used)."""
    Mf, Mc = len(c_fine), len(c_coarse)
    R = np.zeros((Mc + 1, Mf + 1))
    R[0, 0] = 1.0
    R[1:, 1:] = lagrange_basis_values(c_fine, c_coarse)
    return R


def prolongation_matrix(c_coarse, c_fine):
    """Matrix of T_{l+1}^l (Sec. 3.2): same construction with the roles of the
    coarse and fine nodes exchanged."""
    return restriction_matrix(c_coarse, c_fine)

"""Pins of the oracle's collocation coefficients against textbook values,
closed forms, identities and brute-force quadrature (no GPU)."""
import math
import os

import mpmath
import numpy as np
import pytest
import scipy.linalg

from oracle.coeffs import (collocation_matrix, exp_colloc_matrix, lagrange_derivatives_at_zero,
                           node_spacings, phi, prolongation_matrix, radau_iia_nodes,
                           restriction_matrix)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _expr(s):
    return float(eval(s.strip(), {"__builtins__": {}}, {"sqrt": math.sqrt}))


def _load_radau():
    out = {}
    with open(os.path.join(GOLDEN, "radau_iia.txt")) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            M, c, q = line.split(";")
            out[int(M)] = (np.array([_expr(x) for x in c.split(",")]),
                           np.array([[_expr(x) for x in row.split(",")] for row in q.split("|")]))
    return out


@pytest.mark.parametrize("M", [1, 2, 3])
def test_radau_textbook(M):
    c_ref, q_ref = _load_radau()[M]
    c = radau_iia_nodes(M)
    assert np.max(np.abs(c - c_ref)) < 1e-15
    assert np.max(np.abs(collocation_matrix(c) - q_ref)) < 1e-15


@pytest.mark.parametrize("M", [2, 3, 4, 5, 6, 8])
def test_radau_order_conditions(M):
    """Collocation condition C(M) and the Radau quadrature order 2M-1."""
    c = radau_iia_nodes(M)
    Q = collocation_matrix(c)
    # a(0) from the Appendix formula carries the cancellation of the large w_j^k
    tol = 1e-13 if M <= 6 else 2e-12
    for m in range(M):
        assert np.max(np.abs(Q @ c ** m - c ** (m + 1) / (m + 1))) < tol
    b = Q[-1]
    for m in range(2 * M - 1):
        assert abs(b @ c ** m - 1.0 / (m + 1)) < tol
    assert abs(b @ c ** (2 * M - 1) - 1.0 / (2 * M)) > 1e-10  # not exact beyond
    assert np.all(np.diff(c) > 0) and c[-1] == 1.0 and c[0] > 0
    assert np.allclose(node_spacings(c).sum(), 1.0)


@pytest.mark.parametrize("M", [2, 3, 4, 6, 8])
def test_fornberg_moments(M):
    """sum_j w_j^k c_j^m = k! delta_km (derivatives at 0 of the monomials)."""
    c = radau_iia_nodes(M)
    w = lagrange_derivatives_at_zero(c)
    for k in range(M):
        for m in range(M):
            expect = math.factorial(k) if k == m else 0.0
            assert abs(w[k] @ c ** m - expect) < 1e-9 * max(1.0, np.abs(w[k]).sum())


def _phi_mp(k, x):
    mpmath.mp.dps = 40
    x = mpmath.mpf(x)
    if k == 0:
        return mpmath.e ** x
    f = lambda r: mpmath.e ** ((1 - r) * x) * r ** (k - 1)
    pts = [0, 1] if abs(x) < 10 else [0, 1 - 30 / abs(x), 1 - 3 / abs(x), 1]
    return mpmath.quad(f, pts) / mpmath.factorial(k - 1)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6, 8])
def test_phi_against_quadrature(k):
    xs = [-1e-9, -1e-3, -0.37, -1.99, -2.0, -2.01, -3.7, -9.5, -40.0, -250.0, -1800.0, 0.8, 3.0]
    got = phi(k, np.array(xs))
    for x, v in zip(xs, got):
        ref = float(_phi_mp(k, x))
        assert abs(v - ref) <= 2e-15 * abs(ref), (k, x, v, ref)


def test_phi_identities():
    x = np.concatenate([-np.logspace(-8, 3.5, 200), np.linspace(-5, 5, 101)])
    for k in range(0, 8):
        assert phi(k, np.zeros(1))[0] == pytest.approx(1.0 / math.factorial(k), rel=1e-16)
        lhs = phi(k, x)
        rhs = 1.0 / math.factorial(k) + x * phi(k + 1, x)
        scale = np.maximum(np.abs(lhs), 1.0 / math.factorial(k))
        assert np.max(np.abs(lhs - rhs) / scale) < 1e-12
    # [expm(B)]_{0,k} = phi_k(x) with B = x e_0 e_0^T + superdiagonal ones
    for xv in (-0.01, -1.5, -12.0, -120.0):
        B = np.diag(np.ones(6), 1)
        B[0, 0] = xv
        E = scipy.linalg.expm(B)
        for k in range(7):
            assert abs(E[0, k] - phi(k, np.array([xv]))[0]) < 1e-13 * abs(E[0, k])


def _aij_mp(c, i, j, z):
    mpmath.mp.dps = 40
    M = len(c)
    cm = [mpmath.mpf(v) for v in c]

    def ell(s):
        p = mpmath.mpf(1)
        for m in range(M):
            if m != j:
                p *= (s - cm[m]) / (cm[j] - cm[m])
        return p

    ci = cm[i]
    f = lambda s: mpmath.e ** ((ci - s) * z) * ell(s)
    if abs(z) * ci > 20:
        pts = [0, ci - 20 / abs(z), ci - 2 / abs(z), ci]
    else:
        pts = [0, ci]
    return mpmath.quad(f, pts)


@pytest.mark.parametrize("M", [2, 4, 6])
def test_aij_against_definition(M):
    """eq. def_aij by brute-force quadrature vs eq. def_aij_computable."""
    c = radau_iia_nodes(M)
    zs = np.array([-1e-6, -0.3, -5.0, -50.0, -500.0])
    A = exp_colloc_matrix(zs, c)
    for zi, z in enumerate(zs):
        for i in range(M):
            for j in range(M):
                ref = float(_aij_mp(c, i, j, z))
                tol = 2e-13 if M <= 4 else 5e-13
                assert abs(A[zi, i, j] - ref) < tol * max(1.0, abs(ref)), (M, z, i, j)


@pytest.mark.parametrize("M", [3, 4, 6])
def test_aij_row_sums_and_moments(M):
    """sum_j a_ij = c_i phi_1(c_i z);  sum_j a_ij c_j^m = m! c_i^{m+1} phi_{m+1}(c_i z)."""
    c = radau_iia_nodes(M)
    zs = -np.logspace(-4, 2.7, 25)
    A = exp_colloc_matrix(zs, c)
    for m in range(M):
        lhs = A @ c ** m
        rhs = math.factorial(m) * c[None] ** (m + 1) * np.stack(
            [phi(m + 1, c[i] * zs) for i in range(M)], axis=1)
        assert np.max(np.abs(lhs - rhs)) < 1e-12


def test_aij_zero_is_collocation():
    for M in (2, 3, 4, 6):
        c = radau_iia_nodes(M)
        A0 = exp_colloc_matrix(np.zeros(1), c)[0]
        assert np.max(np.abs(A0 - collocation_matrix(c))) == 0.0


@pytest.mark.parametrize("Mf,Mc", [(6, 3), (4, 2), (8, 4), (3, 1)])
def test_transfer_matrices(Mf, Mc):
    """R and T reproduce polynomials of degree < M_from and copy row 0."""
    cf, cc = radau_iia_nodes(Mf), radau_iia_nodes(Mc)
    R = restriction_matrix(cf, cc)
    T = prolongation_matrix(cc, cf)
    assert R.shape == (Mc + 1, Mf + 1) and T.shape == (Mf + 1, Mc + 1)
    assert R[0, 0] == 1.0 and np.all(R[0, 1:] == 0) and np.all(R[1:, 0] == 0)
    assert T[0, 0] == 1.0 and np.all(T[0, 1:] == 0) and np.all(T[1:, 0] == 0)
    for m in range(Mf):
        yf = np.concatenate([[7.0], cf ** m])
        assert np.max(np.abs((R @ yf)[1:] - cc ** m)) < 1e-12
    for m in range(Mc):
        yc = np.concatenate([[7.0], cc ** m])
        assert np.max(np.abs((T @ yc)[1:] - cf ** m)) < 1e-12
    # c_M = 1 on both levels: the last coarse node picks the last fine node
    assert R[-1, -1] == 1.0 and np.all(R[-1, :-1] == 0.0)

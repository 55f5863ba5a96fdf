"""Tissue discretisation (TEST INFRASTRUCTURE ONLY, see package doc).

The paper discretises the diffusion term of eq. monodomain_pde with finite
differences on rectangular domains and keeps A symmetric (Sec. 2.2).  The
workloads use the second-order 3/5/7-point stencil on a cell-centred uniform
mesh: node p sits at x_p = (p + 1/2) dx and the no-flux condition is a mirror
ghost, so the face between a node and the wall carries no flux.  Row p of
A V is  sum over the faces (p, q) of  k_pq (V_q - V_p),  k_pq = sigma_face/dx^2,
with sigma_face the per-axis conductivity (uniform or anisotropic tensor) or the
harmonic mean 2 s_p s_q/(s_p + s_q) of a per-node field.

Node ordering is x fastest, then y, then z: p = ix + nx (iy + ny iz).

Space transfer between a mesh and the mesh coarsened 2x per axis (used by the
space-coarsened PFASST level; the paper coarsens in time only): restriction is
the average of the 2^d children, prolongation is cell-centred multilinear
interpolation with weights 3/4 and 1/4 per axis and a mirror at the walls.

The paper's own discretisation is fourth order (Sec. 2.2) with DCT-II solves
(Sec. 5, computational setup); order = 4 builds it for uniform sigma: per axis
the centred five-point second difference (-1, 16, -30, 16, -1)/(12 dx^2), with
the no-flux wall as the same even mirror (V_{-1} = V_0, V_{-2} = V_1 on the
cell-centred mesh).  That mirror makes the operator symmetric and diagonal in
the DCT-II basis, which is what the paper's DCT solves need.

The Laplacian is pinned by its exact DCT-II diagonalisation for uniform sigma
(both orders) and by its order of accuracy on smooth no-flux fields; the
transfers by exactness on constants and linear fields.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def second_difference_4(n):
    """The 1D fourth-order second difference on n cell-centred nodes with the
    even mirror at both walls, times dx^2 (dense n x n)."""
    c = {-2: -1.0 / 12.0, -1: 16.0 / 12.0, 0: -30.0 / 12.0, 1: 16.0 / 12.0, 2: -1.0 / 12.0}
    D = np.zeros((n, n))
    for p in range(n):
        for m, w in c.items():
            q = p + m
            while q < 0 or q >= n:  # mirror about the walls at -1/2 and n - 1/2
                q = -1 - q if q < 0 else 2 * n - 1 - q
            D[p, q] += w
    return D


def laplacian(dims, dx, sigma=(1.0, 1.0, 1.0), sigma_node=None, order=2):
    """Sparse symmetric A (CSR) with (A V)_p = sum_faces k_pq (V_q - V_p)
    (order 2), or the fourth-order stencil above (order 4, uniform sigma)."""
    if order == 4:
        if sigma_node is not None:
            raise ValueError("the fourth-order stencil takes a uniform sigma")
        dims = tuple(int(n) for n in dims)
        nx, ny, nz = (dims + (1, 1, 1))[:3]
        A = sp.csr_matrix((nx * ny * nz, nx * ny * nz))
        for axis, n in enumerate((nx, ny, nz)):
            if n < 2:
                continue
            ops = [sp.identity(m, format="csr") for m in (nz, ny, nx)]
            ops[2 - axis] = sp.csr_matrix(second_difference_4(n))
            A = A + (float(sigma[axis]) / dx ** 2) * sp.kron(sp.kron(ops[0], ops[1]), ops[2])
        return A.tocsr()
    if order != 2:
        raise ValueError("order must be 2 or 4")
    dims = tuple(int(n) for n in dims)
    nx, ny, nz = (dims + (1, 1, 1))[:3]
    N = nx * ny * nz
    idx = np.arange(N).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []
    for axis, n_axis in ((2, nx), (1, ny), (0, nz)):
        if n_axis < 2:
            continue
        lo = np.take(idx, np.arange(n_axis - 1), axis=axis).ravel()
        hi = np.take(idx, np.arange(1, n_axis), axis=axis).ravel()
        if sigma_node is None:
            s_face = np.full(lo.shape, float(sigma[2 - axis]))
        else:
            s = np.asarray(sigma_node, float).ravel()
            s_face = 2.0 * s[lo] * s[hi] / (s[lo] + s[hi])
        k = s_face / dx ** 2
        rows += [lo, hi, lo, hi]
        cols += [hi, lo, lo, hi]
        vals += [k, k, -k, -k]
    if not rows:
        return sp.csr_matrix((N, N))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return A.tocsr()


class ImplicitSolver:
    """Direct solves of (I - a K) x = b with K = A/(chi Cm), one sparse LU
    factorisation per distinct factor a (cached)."""

    def __init__(self, K):
        self.K = K.tocsc()
        self.N = K.shape[0]
        self._lu = {}

    def solve(self, b, a):
        key = float(a)
        if key not in self._lu:
            M = sp.identity(self.N, format="csc") - key * self.K
            self._lu[key] = spla.splu(M)
        return self._lu[key].solve(np.asarray(b, float))


def dct_eigenvalues(n, order=2):
    """Eigenvalues (times dx^2) of the 1D no-flux second difference for the
    DCT-II mode k = 0..n-1, theta = pi k / n: the stencil's symbol at theta,
    2 cos(theta) - 2 = -4 sin^2(theta / 2) (order 2) and
    (-30 + 32 cos(theta) - 2 cos(2 theta)) / 12 (order 4)."""
    th = np.pi * np.arange(n) / n
    if order == 2:
        return -4.0 * np.sin(th / 2.0) ** 2
    return (-30.0 + 32.0 * np.cos(th) - 2.0 * np.cos(2.0 * th)) / 12.0


def dct_solve_uniform(dims, dx, sigma, a, b, order=2):
    """Exact solve of (I - a A) x = b for uniform diagonal sigma through the
    DCT-II eigenbasis of the no-flux cell-centred stencil (the solver family
    the paper uses for its Laplacian solves, Sec. 5 computational setup).
    Eigenvalues per axis: sigma/dx^2 times dct_eigenvalues(n, order)."""
    import scipy.fft as sfft
    dims = tuple(int(n) for n in dims)
    shape = tuple(reversed(dims))  # (nz, ny, nx)
    bb = np.asarray(b, float).reshape(shape)
    lam = np.zeros(shape)
    for ax_arr, n in enumerate(shape):
        s = sigma[len(shape) - 1 - ax_arr]
        ev = (s / dx ** 2) * dct_eigenvalues(n, order)
        sh = [1] * len(shape)
        sh[ax_arr] = n
        lam = lam + ev.reshape(sh)
    bh = sfft.dctn(bb, type=2, norm="ortho")
    xh = bh / (1.0 - a * lam)
    return sfft.idctn(xh, type=2, norm="ortho").ravel()


def coarse_dims(dims):
    """Dims of the mesh coarsened by 2 along every axis with more than 1 node."""
    out = []
    for n in dims:
        if n > 1:
            if n % 2:
                raise ValueError("space coarsening needs even dims")
            out.append(n // 2)
        else:
            out.append(1)
    return tuple(out)


def restrict_space(u, dims):
    """Average of the children: u has shape (..., N_fine) -> (..., N_coarse)."""
    dims = tuple(int(n) for n in dims)
    nx, ny, nz = (dims + (1, 1, 1))[:3]
    lead = u.shape[:-1]
    v = u.reshape(lead + (nz, ny, nx))
    for ax, n in ((-1, nx), (-2, ny), (-3, nz)):
        if n > 1:
            sh = list(v.shape)
            sh[ax] = n // 2
            sh.insert(len(sh) + ax + 1, 2)
            v = v.reshape(sh).mean(axis=len(sh) + ax)
    return v.reshape(lead + (-1,))


def _prolong_axis(v, ax):
    n = v.shape[ax]
    lo = np.concatenate([np.take(v, [0], axis=ax), np.take(v, np.arange(n - 1), axis=ax)], axis=ax)
    hi = np.concatenate([np.take(v, np.arange(1, n), axis=ax), np.take(v, [n - 1], axis=ax)], axis=ax)
    even = 0.75 * v + 0.25 * lo    # child 2I sits a quarter cell left of I
    odd = 0.75 * v + 0.25 * hi     # child 2I+1 sits a quarter cell right of I
    out = np.stack([even, odd], axis=ax + 1 if ax >= 0 else ax)
    sh = list(v.shape)
    sh[ax] = 2 * n
    return out.reshape(sh)


def prolong_space(u, dims_fine):
    """Cell-centred multilinear interpolation from the coarse mesh to dims_fine."""
    dims = tuple(int(n) for n in dims_fine)
    nx, ny, nz = (dims + (1, 1, 1))[:3]
    cx, cy, cz = (coarse_dims(dims) + (1, 1, 1))[:3]
    lead = u.shape[:-1]
    v = u.reshape(lead + (cz, cy, cx))
    for ax, n in ((-1, nx), (-2, ny), (-3, nz)):
        if n > 1:
            v = _prolong_axis(v, ax)
    return v.reshape(lead + (-1,))

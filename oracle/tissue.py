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

The Laplacian is pinned by its exact DCT-II diagonalisation for uniform sigma;
the transfers by exactness on constants and linear fields.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def laplacian(dims, dx, sigma=(1.0, 1.0, 1.0), sigma_node=None):
    """Sparse symmetric A (CSR) with (A V)_p = sum_faces k_pq (V_q - V_p)."""
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


def dct_solve_uniform(dims, dx, sigma, a, b):
    """Exact solve of (I - a A) x = b for uniform diagonal sigma through the
    DCT-II eigenbasis of the no-flux cell-centred stencil (the solver family
    the paper uses for its Laplacian solves, Sec. 5 computational setup).
    Eigenvalues per axis: -(4 sigma/dx^2) sin^2(pi k / (2 n))."""
    import scipy.fft as sfft
    dims = tuple(int(n) for n in dims)
    shape = tuple(reversed(dims))  # (nz, ny, nx)
    bb = np.asarray(b, float).reshape(shape)
    lam = np.zeros(shape)
    for ax_arr, n in enumerate(shape):
        s = sigma[len(shape) - 1 - ax_arr]
        k = np.arange(n)
        ev = -(4.0 * s / dx ** 2) * np.sin(np.pi * k / (2.0 * n)) ** 2
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

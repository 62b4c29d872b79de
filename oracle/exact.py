"""Quadrature-free assembly of the mass, Laplace and elasticity matrices -- TEST
INFRASTRUCTURE ONLY.

A brute-force pin for the oracle: every basis function is expanded into a polynomial in
the barycentric coordinates lambda_0..lambda_d (Silvester product, multiplied out), the
physical gradient uses grad(lambda_i) from solving the cell's barycentric system, and
every product is integrated exactly (rational arithmetic) with the Dirichlet formula
    int_T lambda^g dx = |T| d! g! / (|g| + d)!.
No quadrature rule, no tabulation and no Jacobian inverse of the oracle proper is used,
so the assembled matrix times u checks the action's quadrature, tabulation, geometry,
form and scatter at once (mass and elasticity integrands are polynomials, so the
quadrature-based action equals this exactly up to rounding).
"""
from __future__ import annotations

import math
from collections import defaultdict
from fractions import Fraction

import numpy as np

from .basis import lattice


def _poly_mul(p, q):
    r = defaultdict(Fraction)
    for e1, c1 in p.items():
        for e2, c2 in q.items():
            r[tuple(a + b for a, b in zip(e1, e2))] += c1 * c2
    return dict(r)


def _poly_diff(p, i):
    r = {}
    for e, c in p.items():
        if e[i] > 0:
            e2 = list(e)
            e2[i] -= 1
            r[tuple(e2)] = r.get(tuple(e2), Fraction(0)) + c * e[i]
    return r


def _basis_polys(dim: int, k: int):
    """Each basis function as {exponent tuple over (lambda_0..lambda_d): coefficient}."""
    nb = dim + 1
    polys = []
    for alpha in lattice(dim, k):
        b = [k - sum(alpha)] + list(alpha)
        p = {tuple([0] * nb): Fraction(1)}
        for i in range(nb):
            for j in range(b[i]):
                e = [0] * nb
                e[i] = 1
                lin = {tuple(e): Fraction(k, j + 1)}
                lin[tuple([0] * nb)] = lin.get(tuple([0] * nb), Fraction(0)) - Fraction(j, j + 1)
                p = _poly_mul(p, lin)
        polys.append(p)
    return polys


def _integrate_ref(p, dim):
    """int over T of p divided by |T| (cell-independent), in exact rational arithmetic."""
    s = Fraction(0)
    for e, c in p.items():
        s += c * Fraction(math.factorial(dim) * math.prod(math.factorial(x) for x in e),
                          math.factorial(sum(e) + dim))
    return s


def basis_polys(dim: int, k: int):
    return _basis_polys(dim, k)


def eval_poly(p, lam):
    return sum(float(c) * math.prod(l ** x for l, x in zip(lam, e)) for e, c in p.items())


class _RefIntegrals:
    def __init__(self, dim: int, k: int):
        polys = _basis_polys(dim, k)
        nb = dim + 1
        n = len(polys)
        self.n = n
        self.mass = np.zeros((n, n))
        self.grad = np.zeros((n, nb, n, nb))     # int dphi_a/dlam_i dphi_b/dlam_j / |T|
        dp = [[_poly_diff(p, i) for i in range(nb)] for p in polys]
        for a in range(n):
            for b in range(n):
                self.mass[a, b] = float(_integrate_ref(_poly_mul(polys[a], polys[b]), dim))
                for i in range(nb):
                    for j in range(nb):
                        self.grad[a, i, b, j] = float(
                            _integrate_ref(_poly_mul(dp[a][i], dp[b][j]), dim))


_cache: dict = {}


def _ref(dim, k):
    if (dim, k) not in _cache:
        _cache[(dim, k)] = _RefIntegrals(dim, k)
    return _cache[(dim, k)]


def _cell_bary(coords_cell: np.ndarray):
    """|T| and grad(lambda_i) [d+1, d] from the barycentric system [1; x] lambda = [1; x]."""
    d = coords_cell.shape[1]
    A = np.ones((d + 1, d + 1))
    A[1:, :] = coords_cell.T
    Ainv = np.linalg.inv(A)
    vol = abs(np.linalg.det(A)) / math.factorial(d)
    return vol, Ainv[:, 1:]


def assemble_mass(mesh) -> np.ndarray:
    R = _ref(mesh.dim, mesh.k)
    M = np.zeros((mesh.n_node, mesh.n_node))
    for cell in range(mesh.n_cell):
        vol, _ = _cell_bary(mesh.coords[mesh.cell_verts[cell]])
        nodes = mesh.cell_nodes[cell]
        M[np.ix_(nodes, nodes)] += vol * R.mass
    return M


def assemble_elasticity(mesh, lam: float, mu: float) -> np.ndarray:
    """K[(a,c),(b,e)] = int lam d_e phi_b d_c phi_a + mu (delta_ce grad phi_b . grad phi_a
    + d_c phi_b d_e phi_a), DoF (node, c) at node*d + c."""
    d = mesh.dim
    R = _ref(d, mesh.k)
    n = R.n
    K = np.zeros((mesh.n_node * d, mesh.n_node * d))
    for cell in range(mesh.n_cell):
        vol, gl = _cell_bary(mesh.coords[mesh.cell_verts[cell]])
        # D[a, j, b, l] = int d_j phi_a d_l phi_b
        D = vol * np.einsum("aibk,ij,kl->ajbl", R.grad, gl, gl)
        Ke = np.zeros((n, d, n, d))
        for c in range(d):
            for e in range(d):
                Ke[:, c, :, e] += lam * D[:, c, :, e] + mu * D[:, e, :, c]
                if c == e:
                    Ke[:, c, :, e] += mu * np.einsum("ajbj->ab", D)
        idx = (mesh.cell_nodes[cell][:, None] * d + np.arange(d)[None, :]).ravel()
        K[np.ix_(idx, idx)] += Ke.reshape(n * d, n * d)
    return K


def assemble_laplace(mesh) -> np.ndarray:
    """L[a, b] = int grad phi_a . grad phi_b."""
    d = mesh.dim
    R = _ref(d, mesh.k)
    L = np.zeros((mesh.n_node, mesh.n_node))
    for cell in range(mesh.n_cell):
        vol, gl = _cell_bary(mesh.coords[mesh.cell_verts[cell]])
        D = vol * np.einsum("aibk,ij,kl->ajbl", R.grad, gl, gl)
        nodes = mesh.cell_nodes[cell]
        L[np.ix_(nodes, nodes)] += np.einsum("ajbj->ab", D)
    return L

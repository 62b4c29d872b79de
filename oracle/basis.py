"""Oracle P_k Lagrange basis on the reference simplex (test infrastructure only).

Equispaced Lagrange nodes xi = alpha/k (|alpha| <= k), in the local order of the cell-to-
node map: first coordinate fastest.  The paper leaves the element family at "P_k
Lagrange" (table of kernel parameters, Sec. 4) and never fixes node placement; the
equispaced family is the reading adopted here.

Basis by the Silvester product formula in barycentric coordinates
lambda_0 = 1 - sum(xi), lambda_r = xi_r, with full index b = (k-|alpha|, alpha_1..alpha_d):
    phi_b(lambda) = prod_i prod_{j < b_i} (k lambda_i - j) / (j + 1).
The reference derivatives d phi / d xi_r = d phi/d lambda_r - d phi/d lambda_0 are the
tabulations Phi of Sec. 2.2 (tabulated-values equation).
"""
from __future__ import annotations

import numpy as np


def lattice(dim: int, k: int) -> list[tuple[int, ...]]:
    pts = []
    if dim == 2:
        for j in range(k + 1):
            for i in range(k + 1 - j):
                pts.append((i, j))
    elif dim == 3:
        for l in range(k + 1):
            for j in range(k + 1 - l):
                for i in range(k + 1 - j - l):
                    pts.append((i, j, l))
    else:
        raise ValueError("dim must be 2 or 3")
    return pts


def _factor_product(k: int, lam: float, b: int) -> tuple[float, float]:
    """prod_{j<b} (k lam - j)/(j+1) and its derivative in lam."""
    val = 1.0
    for j in range(b):
        val *= (k * lam - j) / (j + 1)
    der = 0.0
    for m in range(b):
        p = k / (m + 1)
        for j in range(b):
            if j != m:
                p *= (k * lam - j) / (j + 1)
        der += p
    return val, der


def eval_basis(dim: int, k: int, xi: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Values [nloc] and reference gradients [nloc, dim] at one reference point."""
    nodes = lattice(dim, k)
    lam = [1.0 - float(sum(xi))] + [float(x) for x in xi]
    vals = np.zeros(len(nodes))
    grads = np.zeros((len(nodes), dim))
    for a, alpha in enumerate(nodes):
        b = [k - sum(alpha)] + list(alpha)
        f = [_factor_product(k, lam[i], b[i]) for i in range(dim + 1)]
        v = 1.0
        for i in range(dim + 1):
            v *= f[i][0]
        dlam = []
        for i in range(dim + 1):
            p = f[i][1]
            for i2 in range(dim + 1):
                if i2 != i:
                    p *= f[i2][0]
            dlam.append(p)
        vals[a] = v
        for r in range(dim):
            grads[a, r] = dlam[r + 1] - dlam[0]
    return vals, grads


def tabulate(dim: int, k: int, points: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """phi [Q, nloc] and dphi [Q, nloc, dim] at the quadrature points."""
    vals, grads = [], []
    for x in points:
        v, g = eval_basis(dim, k, x)
        vals.append(v)
        grads.append(g)
    return np.asarray(vals), np.asarray(grads)

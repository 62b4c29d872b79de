"""Oracle quadrature on the reference simplex (test infrastructure only).

The paper replaces each cell integral by a weighted sum over Q nodes (Sec. 2.2, the
quadrature-replacement equation) but never states which rule; only Q per case appears
(table of kernel parameters, Sec. 4).  The reading adopted here: the Stroud conical
product rule -- Gauss-Jacobi rules in collapsed coordinates -- with ceil((m+1)/2)
points per direction, exact for every polynomial of total degree <= m.

Reference simplex: {xi >= 0, sum xi <= 1}, measure 1/d!.
  2D: xi2 = t (weight (1-t)),  xi1 = s (1-t).
  3D: xi3 = w (weight (1-w)^2), xi2 = t (1-w) (weight (1-t)), xi1 = s (1-t)(1-w).
Point order: the innermost direction (s) fastest.

The 1D rules come from ``scipy.special.roots_jacobi`` (a library primitive).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import roots_jacobi


def gauss_jacobi_01(npts: int, alpha: int) -> tuple[np.ndarray, np.ndarray]:
    """Nodes/weights on [0,1] for the weight (1-t)^alpha."""
    x, w = roots_jacobi(npts, float(alpha), 0.0)     # weight (1-x)^a (1+x)^0 on [-1,1]
    t = 0.5 * (1.0 + x)
    return t, w / 2.0 ** (alpha + 1)


def points_per_direction(degree: int) -> int:
    return max(1, math.ceil((degree + 1) / 2))


def stroud(dim: int, degree: int) -> tuple[np.ndarray, np.ndarray]:
    """Stroud conical-product rule: (points [Q, dim], weights [Q])."""
    n = points_per_direction(degree)
    s, ws = gauss_jacobi_01(n, 0)
    if dim == 2:
        t, wt = gauss_jacobi_01(n, 1)
        pts, wts = [], []
        for j in range(n):
            for i in range(n):
                pts.append((s[i] * (1.0 - t[j]), t[j]))
                wts.append(ws[i] * wt[j])
        return np.asarray(pts), np.asarray(wts)
    if dim == 3:
        t, wt = gauss_jacobi_01(n, 1)
        z, wz = gauss_jacobi_01(n, 2)
        pts, wts = [], []
        for l in range(n):
            for j in range(n):
                for i in range(n):
                    pts.append((s[i] * (1.0 - t[j]) * (1.0 - z[l]),
                                t[j] * (1.0 - z[l]),
                                z[l]))
                    wts.append(ws[i] * wt[j] * wz[l])
        return np.asarray(pts), np.asarray(wts)
    raise ValueError("dim must be 2 or 3")

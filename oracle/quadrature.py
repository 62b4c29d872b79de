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

The second family, ``symmetric``: fully symmetric rules, whose points lie on orbits of the
simplex's symmetry group with one weight per orbit, with as many unknowns as there are
independent symmetric moment conditions up to the degree (so each rule is an isolated root
of its moment equations).  The paper's table of kernel parameters lists point counts that
match rules of this kind; it prints no rule.  Here each rule is the root of the moment
equations nearest to a few-digit approximation of its orbit parameters, found by scipy's
least-squares solver (a library primitive) and accepted only if it integrates every
monomial up to the degree exactly (to rounding), has positive weights and points inside.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy.optimize import least_squares
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


# --------------------------------------------------------------------- symmetric rules
# Orbits in barycentric coordinates.  Triangle: "c" centroid, "aab" = perms of (a, a, 1-2a),
# "abc" = perms of (a, b, 1-a-b).  Tetrahedron: "c", "aaab" = perms of (a, a, a, 1-3a),
# "aabb" = perms of (a, a, 1/2-a, 1/2-a), "aabc" = perms of (a, a, b, 1-2a-b).
# Each entry: (orbit, approximate parameters, approximate weight); weights sum to 1/d!.
SYMMETRIC_APPROX = {
    (2, 4): [("aab", (0.445948,), 0.111691), ("aab", (0.0915762,), 0.0549759)],
    (2, 6): [("aab", (0.249287,), 0.0583931), ("aab", (0.0630890,), 0.0254225),
             ("abc", (0.310352, 0.0531450), 0.0414255)],
    (2, 8): [("c", (), 0.0721578), ("aab", (0.0505472,), 0.0162292),
             ("aab", (0.459293,), 0.0475458), ("aab", (0.170569,), 0.0516087),
             ("abc", (0.263113, 0.00839478), 0.0136152)],
    (2, 10): [("c", (), 0.0416099), ("aab", (0.0285035,), 0.00547564),
              ("aab", (0.162913,), 0.0263260), ("abc", (0.153303, 0.0336857), 0.0146614),
              ("abc", (0.363363, 0.607330), 0.0176975), ("abc", (0.336696, 0.146812), 0.0281386)],
    (2, 12): [("aab", (0.271463,), 0.0312706), ("aab", (0.488204,), 0.0121334),
              ("aab", (0.440112,), 0.0249592), ("aab", (0.109258,), 0.0142430),
              ("aab", (0.0246464,), 0.00396582), ("abc", (0.255454, 0.116296), 0.0216137),
              ("abc", (0.127280, 0.851338), 0.00754184), ("abc", (0.291656, 0.0230342), 0.0108918)],
    (3, 5): [("aaab", (0.310886,), 0.0187813), ("aaab", (0.0927353,), 0.0122488),
             ("aabb", (0.0455037,), 0.00709100)],
    (3, 6): [("aaab", (0.214603,), 0.00665379), ("aaab", (0.0406740,), 0.00167954),
             ("aaab", (0.322338,), 0.00922620), ("aabc", (0.0636610, 0.269672), 0.00803571)],
    (3, 8): [("aaab", (0.0834534,), 0.00200563), ("aaab", (0.0100916,), 0.000209000),
             ("aabb", (0.449481,), 0.00454683), ("aabc", (0.0368078, 0.734271), 0.00214781),
             ("aabc", (0.222840, 0.430062), 0.00428064), ("aabc", (0.229785, 0.513039), 0.00444881)],
}


def _orbit(dim: int, kind: str, prm) -> list[tuple]:
    """Barycentric points of one orbit: the distinct arrangements of its symbol pattern."""
    if kind == "c":
        return [tuple([np.longdouble(1) / (dim + 1)] * (dim + 1))]
    if dim == 2 and kind == "aab":
        value = {"a": prm[0], "b": 1.0 - 2.0 * prm[0]}
    elif dim == 2 and kind == "abc":
        value = {"a": prm[0], "b": prm[1], "c": 1.0 - prm[0] - prm[1]}
    elif dim == 3 and kind == "aaab":
        value = {"a": prm[0], "b": 1.0 - 3.0 * prm[0]}
    elif dim == 3 and kind == "aabb":
        value = {"a": prm[0], "b": 0.5 - prm[0]}
    elif dim == 3 and kind == "aabc":
        value = {"a": prm[0], "b": prm[1], "c": 1.0 - 2.0 * prm[0] - prm[1]}
    else:
        raise ValueError(kind)
    return [tuple(value[ch] for ch in arr) for arr in sorted(set(itertools.permutations(kind)))]


def _rule_degree(dim: int, degree: int):
    """The smallest tabulated symmetric degree >= degree, or None."""
    cands = [m for (d, m) in SYMMETRIC_APPROX if d == dim and m >= degree]
    return min(cands) if cands else None


def _expand(dim: int, structure, x):
    pts, wts, i = [], [], 0
    for kind, prm0, _ in structure:
        k = len(prm0)
        prm, w = x[i:i + k], x[i + k]
        i += k + 1
        for lam in _orbit(dim, kind, prm):
            pts.append(lam[1:])
            wts.append(w)
    return np.asarray(pts), np.asarray(wts)


def _monomial_exponents(dim: int, m: int):
    return [e for e in itertools.product(range(m + 1), repeat=dim) if sum(e) <= m]


def _monomial_integral(e) -> float:
    """Exact integral of prod xi_r^e_r over the reference simplex: prod e_r! / (|e| + d)!."""
    return math.prod(math.factorial(k) for k in e) / math.factorial(sum(e) + len(e))


def has_symmetric(dim: int, degree: int) -> bool:
    return degree <= 2 or _rule_degree(dim, degree) is not None


def symmetric(dim: int, degree: int) -> tuple[np.ndarray, np.ndarray]:
    """Fully symmetric rule exact to `degree`: (points [Q, dim], weights [Q])."""
    vol = 1.0 / math.factorial(dim)
    if degree <= 1:
        return np.full((1, dim), 1.0 / (dim + 1)), np.array([vol])
    if degree == 2:
        # orbit of (1 - d b, b, ..., b); the second moment of a barycentric coordinate,
        # int lambda^2 = 2 vol / ((d + 1)(d + 2)), fixes b:
        #   triangle: 6 b^2 - 4 b + 1/2 = 0 -> b = 1/6;  tet: 12 b^2 - 6 b + 3/5 = 0
        b = 1.0 / 6.0 if dim == 2 else (5.0 - math.sqrt(5.0)) / 20.0
        a = 1.0 - dim * b
        pts = [tuple(a if r + 1 == k else b for r in range(dim)) for k in range(dim + 1)]
        return np.asarray(pts), np.full(dim + 1, vol / (dim + 1))
    m = _rule_degree(dim, degree)
    if m is None:
        raise ValueError(f"no symmetric rule of degree {degree} in {dim}D")
    structure = SYMMETRIC_APPROX[(dim, m)]
    mons = np.array(_monomial_exponents(dim, m))
    exact = np.array([_monomial_integral(e) for e in mons])

    def residual(x):
        pts, wts = _expand(dim, structure, x)
        vals = np.prod(pts[:, None, :] ** mons[None, :, :], axis=2)
        return (wts @ vals - exact) / exact

    x0 = []
    for _, prm, w in structure:
        x0 += list(prm) + [w]
    sol = least_squares(residual, np.asarray(x0), xtol=1e-15, ftol=1e-15, gtol=1e-15)
    # polish in extended precision (numpy long double): Gauss-Newton with a central-
    # difference Jacobian, so the root is resolved below double rounding even where the
    # moment equations are ill-conditioned
    exact_ld = np.array([np.longdouble(math.prod(math.factorial(k) for k in e))
                         / np.longdouble(math.factorial(int(sum(e)) + dim)) for e in mons])

    def residual_ld(x):
        pts, wts = _expand(dim, structure, x)
        vals = np.prod(pts.astype(np.longdouble)[:, None, :] ** mons[None, :, :], axis=2)
        return (wts.astype(np.longdouble) @ vals - exact_ld) / exact_ld

    x = sol.x.astype(np.longdouble)
    for _ in range(30):
        r = residual_ld(x)
        if np.max(np.abs(r)) < 1e-18:
            break
        J = np.empty((len(r), len(x)))
        for k in range(len(x)):
            h = np.longdouble(1e-8) * max(np.longdouble(1e-2), abs(x[k]))
            xp, xm = x.copy(), x.copy()
            xp[k] += h
            xm[k] -= h
            J[:, k] = ((residual_ld(xp) - residual_ld(xm)) / (2 * h)).astype(np.float64)
        dx = np.linalg.lstsq(J, -r.astype(np.float64), rcond=None)[0]
        x = x + dx.astype(np.longdouble)
    pts, wts = _expand(dim, structure, x)
    pts, wts = pts.astype(np.float64), wts.astype(np.float64)
    sol_x = x.astype(np.float64)
    if np.max(np.abs(residual(sol_x))) > 1e-14 or np.any(wts <= 0):
        raise RuntimeError(f"symmetric rule {dim}D degree {m} did not converge")
    lam0 = 1.0 - pts.sum(axis=1)
    if np.any(pts < -1e-15) or np.any(lam0 < -1e-15):
        raise RuntimeError(f"symmetric rule {dim}D degree {m} has a point outside")
    return pts, wts

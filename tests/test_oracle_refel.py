"""Pins for the oracle's quadrature and basis (CPU only).

Quadrature: exact integration of every monomial up to the rule's degree against the
Dirichlet closed form  int_{ref simplex} xi^b = b! / (|b| + d)!.
Basis: Kronecker property at the lattice nodes and agreement, in values and derivatives,
with an independent construction (inverse of the monomial Vandermonde matrix).
"""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import basis, quadrature

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def monomials(dim, deg):
    for b in itertools.product(range(deg + 1), repeat=dim):
        if sum(b) <= deg:
            yield b


def dirichlet(b):
    return math.prod(math.factorial(x) for x in b) / math.factorial(sum(b) + len(b))


@pytest.mark.parametrize("dim,degree", [(2, m) for m in range(0, 15)] + [(3, m) for m in range(0, 11)])
def test_stroud_exactness(dim, degree):
    pts, w = quadrature.stroud(dim, degree)
    n = quadrature.points_per_direction(degree)
    assert len(w) == n ** dim
    assert np.all(w > 0)
    assert np.all(pts >= 0) and np.all(pts.sum(1) <= 1)
    assert abs(w.sum() - 1.0 / math.factorial(dim)) < 1e-15
    for b in monomials(dim, degree):
        val = np.sum(w * np.prod(pts ** np.asarray(b), axis=1))
        assert abs(val - dirichlet(b)) <= 1e-13 * dirichlet(b), b


@pytest.mark.parametrize("dim,degree", [(2, 3), (2, 7), (3, 3), (3, 5)])
def test_stroud_not_exact_beyond_degree(dim, degree):
    # the rule with ceil((m+1)/2) points per direction is exact up to 2n-1 and no further
    pts, w = quadrature.stroud(dim, degree)
    n = quadrature.points_per_direction(degree)
    errs = [abs(np.sum(w * np.prod(pts ** np.asarray(b), axis=1)) - dirichlet(b))
            for b in monomials(dim, 2 * n) if sum(b) == 2 * n]
    assert max(errs) > 1e-8


SYM = [(2, m) for m in range(0, 13)] + [(3, m) for m in range(0, 9)]


@pytest.mark.parametrize("dim,degree", SYM)
def test_symmetric_exactness_and_orbits(dim, degree):
    """Pin of the symmetric rules: exact on every monomial up to the degree against the
    closed-form simplex moments, positive weights, points inside, total weight 1/d!, and
    the point set (with its weights) invariant under every permutation of the barycentric
    coordinates -- what makes the rule fully symmetric."""
    pts, w = quadrature.symmetric(dim, degree)
    assert np.all(w > 0)
    lam = np.c_[1.0 - pts.sum(1), pts]
    assert np.all(lam > 0)
    assert abs(w.sum() - 1.0 / math.factorial(dim)) < 1e-15
    for b in monomials(dim, degree):
        val = np.sum(w * np.prod(pts ** np.asarray(b), axis=1))
        assert abs(val - dirichlet(b)) <= 2e-14 * dirichlet(b), b
    key = sorted(tuple(np.round(np.r_[l, wq], 12)) for l, wq in zip(lam, w))
    for perm in itertools.permutations(range(dim + 1)):
        key_p = sorted(tuple(np.round(np.r_[l[list(perm)], wq], 12)) for l, wq in zip(lam, w))
        assert key_p == key, perm


@pytest.mark.parametrize("dim,degree", [(2, 4), (2, 8), (3, 5)])
def test_symmetric_not_exact_beyond_degree(dim, degree):
    pts, w = quadrature.symmetric(dim, degree)
    errs = [abs(np.sum(w * np.prod(pts ** np.asarray(b), axis=1)) - dirichlet(b))
            for b in monomials(dim, degree + 2) if sum(b) > degree]
    assert max(errs) > 1e-10


def test_symmetric_point_counts():
    # fewer points than the conical rule of the same degree, as the paper's tables suggest
    counts = {(2, 4): 6, (2, 6): 12, (2, 8): 16, (2, 10): 25, (2, 12): 33, (3, 2): 4, (3, 5): 14, (3, 6): 24, (3, 8): 50}
    for (dim, deg), n in counts.items():
        assert len(quadrature.symmetric(dim, deg)[1]) == n
        assert n < len(quadrature.stroud(dim, deg)[1])


def _vandermonde_basis(dim, k):
    nodes = np.asarray(basis.lattice(dim, k), dtype=float) / k
    mons = [b for b in monomials(dim, k)]
    V = np.array([[np.prod(x ** np.asarray(b)) for b in mons] for x in nodes])
    C = np.linalg.inv(V)          # column a: monomial coefficients of phi_a

    def evaluate(x):
        m = np.array([np.prod(x ** np.asarray(b)) for b in mons])
        dm = np.zeros((len(mons), dim))
        for i, b in enumerate(mons):
            for r in range(dim):
                if b[r] > 0:
                    b2 = list(b)
                    b2[r] -= 1
                    dm[i, r] = b[r] * np.prod(x ** np.asarray(b2))
        return m @ C, (dm.T @ C).T
    return evaluate


@pytest.mark.parametrize("dim,k", [(2, k) for k in range(1, 9)] + [(3, k) for k in range(1, 7)])
def test_basis_against_vandermonde(dim, k):
    rng = np.random.default_rng(k + 10 * dim)
    ref = _vandermonde_basis(dim, k)
    nodes = np.asarray(basis.lattice(dim, k), dtype=float) / k
    # Kronecker property
    for a, x in enumerate(nodes):
        v, _ = basis.eval_basis(dim, k, x)
        e = np.zeros(len(nodes))
        e[a] = 1
        assert np.max(np.abs(v - e)) < 1e-12
    for _ in range(5):
        x = rng.dirichlet(np.ones(dim + 1))[1:]
        v, g = basis.eval_basis(dim, k, x)
        vr, gr = ref(x)
        assert np.max(np.abs(v - vr)) < 1e-9
        assert np.max(np.abs(g - gr)) < 1e-8 * k
        assert abs(v.sum() - 1.0) < 1e-13
        assert np.max(np.abs(g.sum(0))) < 1e-11


def test_local_counts_match_paper_table():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "param_space.txt"))
            if l.strip() and not l.startswith("#")]
    for dim, op, k, n_trial, n_test, *_ in rows:
        n = len(basis.lattice(int(dim), int(k)))
        assert n == int(n_trial) == int(n_test), (op, dim, k)


def test_lattice_order_matches_meshgen():
    import meshgen
    for dim in (2, 3):
        for k in range(1, 7):
            assert np.array_equal(np.asarray(basis.lattice(dim, k)), meshgen.local_lattice(dim, k))

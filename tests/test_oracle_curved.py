"""Pins for the oracle on curved (non-affine, P2-geometry) cells (CPU only).

On a P2 geometry the Jacobian of the cell map varies over the cell and is evaluated at
every quadrature point (paper Sec. 2.4).  The pins, fixed by the mathematics:
  straight P2 geometry (edge nodes at the edge centres) describes the affine cells, so
      every form's action equals the affine one;
  the curved meshes keep the unit square / cube (boundary nodes do not move), so
      sum(M 1) = |Omega| = 1 and, on isoparametric P2 cells (whose nodes are the geometry
      nodes), sum(M x_0) = int x_0 = 1/2; both integrands are polynomials in xi that the
      rule integrates exactly (|det J| has degree d(1) -> 2 in 2D, 3 in 3D);
  isoparametric P2 cells hold every function linear in x exactly (u = a + b.x has
      grad u = b at every point), so the Laplace and elasticity patch tests hold: zero
      residual at interior nodes (|det J| K^T is the adjugate, a polynomial), rigid modes
      in the elasticity kernel, and a finite rotation gives a zero hyperelastic residual;
  the hyperelastic residual is the gradient of the discrete energy and the VJP the
      transpose of its Jacobian (central differences), on curved cells.
"""
import numpy as np
import pytest

import meshgen
import oracle

F_MASS, F_EL, F_NH, F_SVK = oracle.FORM_MASS, oracle.FORM_ELAST, oracle.FORM_NH, oracle.FORM_SVK
F_LAP, F_HELM = oracle.FORM_LAPLACE, oracle.FORM_HELMHOLTZ
LAME = (1.0, 0.5)
NH = (10.0, 1.0)
HYPER = pytest.mark.parametrize("form", [F_NH, F_SVK], ids=["nh", "svk"])


def curved_mesh(dim, n, k, amp=0.08, seed=0):
    m = meshgen.make_mesh(dim, n, k, None, np.random.default_rng(seed))
    return meshgen.curved(m, amp)


def node_positions(mc):
    """Positions of the solution nodes of an isoparametric (k = 2) curved mesh."""
    assert mc.k == 2 and np.array_equal(mc.cell_nodes, mc.cell_gnodes)
    return mc.gcoords


def test_curved_meshes_are_curved():
    for dim in (2, 3):
        m = meshgen.make_mesh(dim, 3 if dim == 2 else 2, 2, None, np.random.default_rng(0))
        mc = meshgen.curved(m, 0.08)
        straight = meshgen.curved(m, 0.0)
        moved = np.max(np.linalg.norm(mc.gcoords - straight.gcoords, axis=1))
        assert moved > 0.02
        # vertices of the straight P2 geometry are the mesh vertices
        corners = (0, 2, 5) if dim == 2 else (0, 2, 5, 9)
        assert np.array_equal(straight.gcoords[straight.cell_gnodes[:, corners]],
                              m.coords[m.cell_verts])


CASES = [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2)]
FORMS = [F_MASS, F_EL, F_NH, F_SVK, F_LAP, F_HELM]


@pytest.mark.parametrize("dim,k", CASES)
@pytest.mark.parametrize("form", FORMS)
def test_straight_p2_geometry_equals_affine(form, dim, k):
    m = meshgen.make_mesh(dim, 3 if dim == 2 else 2, k, None, np.random.default_rng(3))
    ms = meshgen.curved(m, 0.0)
    ncomp = 1 if form in oracle.SCALAR_FORMS else dim
    rng = np.random.default_rng(1)
    if form in (F_NH, F_SVK):
        u = meshgen.nh_displacement(rng, m, 0.05)
    else:
        u = rng.uniform(-1, 1, m.n_node * ncomp)
    qd = 2 * k
    prm = () if form in oracle.SCALAR_FORMS else NH
    a = oracle.action(form, m, u, qd, prm)
    c = oracle.action(form, ms, u, qd, prm)
    assert np.max(np.abs(a - c)) < 1e-12 * np.max(np.abs(a))
    if form in (F_NH, F_SVK):
        v = rng.uniform(-1, 1, m.n_node * ncomp)
        ga = oracle.vjp(form, m, u, v, qd, prm)
        gc = oracle.vjp(form, ms, u, v, qd, prm)
        assert np.max(np.abs(ga - gc)) < 1e-12 * np.max(np.abs(ga))


@pytest.mark.parametrize("dim,qd", [(2, 4), (3, 5)])
def test_curved_mass_moments(dim, qd):
    mc = curved_mesh(dim, 3 if dim == 2 else 2, 2, seed=4)
    one = oracle.action(F_MASS, mc, np.ones(mc.n_node), qd)
    assert abs(one.sum() - 1.0) < 1e-13
    X = node_positions(mc)
    for j in range(dim):
        mx = oracle.action(F_MASS, mc, X[:, j].copy(), qd)
        assert abs(mx.sum() - 0.5) < 1e-13
    # a rule too weak for |det J| misses the area (the cells really are curved)
    one1 = oracle.action(F_MASS, mc, np.ones(mc.n_node), 1)
    assert abs(one1.sum() - 1.0) > 1e-6


@pytest.mark.parametrize("dim,qd", [(2, 2), (3, 3)])
def test_curved_laplace_patch_test(dim, qd):
    mc = curved_mesh(dim, 3 if dim == 2 else 2, 2, seed=5)
    y1 = oracle.action(F_LAP, mc, np.ones(mc.n_node), qd)
    assert np.max(np.abs(y1)) < 1e-13
    X = node_positions(mc)
    u = 0.3 + X @ np.arange(1.0, dim + 1.0)
    y = oracle.action(F_LAP, mc, u, qd)
    interior = np.all((X > 1e-12) & (X < 1 - 1e-12), axis=1)
    assert np.max(np.abs(y[interior])) < 1e-12 * max(1.0, np.max(np.abs(y)))
    assert np.max(np.abs(y[~interior])) > 1e-3          # the boundary flux is not zero
    # symmetry of the curved operator
    rng = np.random.default_rng(13)
    a, b = rng.uniform(-1, 1, (2, mc.n_node))
    La, Lb = oracle.action(F_LAP, mc, a, qd), oracle.action(F_LAP, mc, b, qd)
    assert abs(b @ La - a @ Lb) < 1e-12 * abs(b @ La)


def rigid_modes(X):
    n, d = X.shape
    modes = []
    for c in range(d):
        r = np.zeros((n, d))
        r[:, c] = 1
        modes.append(r.ravel())
    for i, j in ([(0, 1)] if d == 2 else [(0, 1), (1, 2), (0, 2)]):
        r = np.zeros((n, d))
        r[:, i] = -X[:, j]
        r[:, j] = X[:, i]
        modes.append(r.ravel())
    return modes


@pytest.mark.parametrize("dim,qd", [(2, 2), (3, 3)])
def test_curved_elasticity_rigid_modes_and_patch_test(dim, qd):
    mc = curved_mesh(dim, 3 if dim == 2 else 2, 2, seed=6)
    X = node_positions(mc)
    for r in rigid_modes(X):
        assert np.max(np.abs(oracle.action(F_EL, mc, r, qd, LAME))) < 1e-12
    B = np.random.default_rng(0).normal(size=(dim, dim))
    y = oracle.action(F_EL, mc, (X @ B.T).ravel(), qd, LAME).reshape(-1, dim)
    interior = np.all((X > 1e-12) & (X < 1 - 1e-12), axis=1)
    assert np.max(np.abs(y[interior])) < 1e-12 * np.max(np.abs(y))


@pytest.mark.parametrize("dim", [2, 3])
@HYPER
def test_curved_hyper_finite_rotation(form, dim):
    mc = curved_mesh(dim, 3 if dim == 2 else 2, 2, seed=7)
    X = node_positions(mc)
    th = 0.7
    if dim == 2:
        R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    else:
        a = np.array([1.0, 2.0, 2.0]) / 3
        Kx = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
        R = np.eye(3) + np.sin(th) * Kx + (1 - np.cos(th)) * Kx @ Kx
    uR = (X @ (R - np.eye(dim)).T).ravel()
    assert np.max(np.abs(oracle.action(form, mc, uR, 4, NH))) < 1e-12


@pytest.mark.parametrize("dim,n,k", [(2, 2, 2), (2, 1, 3), (3, 1, 2)])
@HYPER
def test_curved_hyper_energy_gradient_and_vjp(form, dim, n, k):
    mc = curved_mesh(dim, n, k, amp=0.1, seed=8)
    qd = 2 * k
    rng = np.random.default_rng(9)
    u = meshgen.nh_displacement(rng, mc, 0.05)
    assert oracle.min_det_f(mc, u, qd) > 0.5
    r = oracle.action(form, mc, u, qd, NH)
    v = rng.uniform(-1, 1, len(u))
    g = oracle.vjp(form, mc, u, v, qd, NH)
    h = 1e-6
    fd = np.zeros_like(u)
    Jcols = np.zeros((len(u), len(u)))
    for i in range(len(u)):
        e = np.zeros_like(u)
        e[i] = h
        fd[i] = (oracle.energy(form, mc, u + e, qd, NH) - oracle.energy(form, mc, u - e, qd, NH)) / (2 * h)
        Jcols[:, i] = (oracle.action(form, mc, u + e, qd, NH) - oracle.action(form, mc, u - e, qd, NH)) / (2 * h)
    assert np.max(np.abs(fd - r)) < 1e-6 * np.max(np.abs(r)) + 1e-9
    assert np.max(np.abs(Jcols.T @ v - g)) < 1e-6 * np.max(np.abs(g))

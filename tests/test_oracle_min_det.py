"""Pins of the oracle's admissibility check min det F (F = I + grad u_h, minimum over cells
and quadrature points), against values fixed by the deformation itself:

- u = 0 gives F = I, so the minimum is exactly 1;
- an affine displacement u = (A - I) x lies in P_k (k >= 1), and on isoparametric P2 cells
  in P_2, so F = A at every point and the minimum is det A;
- u = alpha x_j^2 e_j (in P_k for k >= 2 on affine cells) gives F = I + 2 alpha x_j e_j e_j^T,
  det F = 1 + 2 alpha x_j, so the minimum is 1 + 2 alpha times the extreme x_j over the
  physical quadrature points x_q = x_0 + J xi_q, computed here from the rule's reference
  points and the vertices (no finite element arithmetic): this pins the per-point
  evaluation, the minimum and the rule family passed in.
"""
import numpy as np
import pytest

import meshgen
import oracle

FAMILIES = ["conical", "symmetric"]


def lattice_positions(mesh):
    X = np.zeros((mesh.n_node, mesh.dim))
    lat = np.asarray(meshgen.local_lattice(mesh.dim, mesh.k), dtype=float) / mesh.k
    for c in range(mesh.n_cell):
        x = mesh.coords[mesh.cell_verts[c]]
        X[mesh.cell_nodes[c]] = x[0] + lat @ (x[1:] - x[0])
    return X


def mesh_for(dim, k, seed):
    return meshgen.make_mesh(dim, 3 if dim == 2 else 2, k, None, np.random.default_rng(seed))


def rule_degree(dim, k, family):
    # a degree with a symmetric rule in both dimensions
    return 4 if dim == 2 else 5


@pytest.mark.parametrize("family", FAMILIES)
@pytest.mark.parametrize("dim,k", [(2, 1), (2, 4), (3, 1), (3, 3)])
def test_zero_displacement_gives_one(dim, k, family):
    m = mesh_for(dim, k, 1)
    u = np.zeros(m.n_node * dim)
    assert oracle.min_det_f(m, u, rule_degree(dim, k, family), family=family) == 1.0


@pytest.mark.parametrize("family", FAMILIES)
@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 5), (3, 1), (3, 2), (3, 4)])
def test_affine_displacement_gives_det_a(dim, k, family):
    m = mesh_for(dim, k, 2)
    rng = np.random.default_rng(3)
    A = np.eye(dim) + 0.3 * rng.uniform(-1, 1, (dim, dim))
    X = lattice_positions(m)
    u = (X @ (A - np.eye(dim)).T).ravel()
    got = oracle.min_det_f(m, u, rule_degree(dim, k, family), family=family)
    assert abs(got - np.linalg.det(A)) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_affine_displacement_on_curved_cells(dim):
    m = meshgen.make_mesh(dim, 3 if dim == 2 else 2, 2, None, np.random.default_rng(4))
    mc = meshgen.curved(m, 0.08)
    rng = np.random.default_rng(5)
    A = np.eye(dim) + 0.3 * rng.uniform(-1, 1, (dim, dim))
    # isoparametric P2: the solution nodes are the geometry nodes
    assert np.array_equal(mc.cell_nodes, mc.cell_gnodes)
    u = (mc.gcoords @ (A - np.eye(dim)).T).ravel()
    for family in FAMILIES:
        got = oracle.min_det_f(mc, u, 4, family=family)
        assert abs(got - np.linalg.det(A)) < 1e-12


@pytest.mark.parametrize("family", FAMILIES)
@pytest.mark.parametrize("alpha", [0.3, -0.2])
@pytest.mark.parametrize("dim,k,j", [(2, 2, 0), (2, 3, 1), (3, 2, 2), (3, 3, 0)])
def test_quadratic_displacement_extreme_point(dim, k, j, alpha, family):
    m = mesh_for(dim, k, 6)
    X = lattice_positions(m)
    U = np.zeros((m.n_node, dim))
    U[:, j] = alpha * X[:, j] ** 2
    qd = rule_degree(dim, k, family)
    t = oracle.tables(dim, k, qd, family)
    xq = []
    for c in range(m.n_cell):
        x = m.coords[m.cell_verts[c]]
        xq.append(x[0] + t.points @ (x[1:] - x[0]))
    xj = np.concatenate(xq)[:, j]
    expect = 1.0 + 2.0 * alpha * (xj.min() if alpha > 0 else xj.max())
    got = oracle.min_det_f(m, U.ravel(), qd, family=family)
    assert abs(got - expect) < 1e-13


def test_family_changes_the_points():
    """The quadratic case distinguishes the two rules' points, so a family argument that
    were ignored would fail one of the two comparisons above; check they differ here."""
    m = mesh_for(2, 2, 6)
    X = lattice_positions(m)
    U = np.zeros((m.n_node, 2))
    U[:, 0] = 0.3 * X[:, 0] ** 2
    a = oracle.min_det_f(m, U.ravel(), 4, family="conical")
    b = oracle.min_det_f(m, U.ravel(), 4, family="symmetric")
    assert a != b

"""Pins for the oracle's action, VJP, energy and colouring (CPU only).

Each pin is fixed by the mathematics, not by the oracle itself:
  mass         partition of unity (sum of M 1 = |Omega| = 1); P2 closed form of M 1;
               P1 element matrix |T| (1 + delta_ab) / ((d+1)(d+2));
               equality with the quadrature-free exact assembly (brute force);
  Laplace      constants in the kernel; affine patch test; symmetry; the P1 reference
               element matrix; exact assembly (brute force);
  Helmholtz    equals exact Laplace plus exact mass assembly;
  elasticity   rigid modes in the kernel; affine patch test; symmetry;
               lambda = 0, mu = 1/2 gives sigma = eps; exact assembly (brute force);
  neo-Hookean and St Venant-Kirchhoff
               r(0) = 0, r(u + c) = r(u), r(finite rotation) = 0 (frame indifference);
               r = grad of the discrete energy (central differences);
               VJP at u = 0 equals the elasticity action with the same (lambda, mu);
               VJP against central differences of r and the transpose identity;
               SVK stretch and simple shear on one P1 cell against hand-worked stresses;
  colouring    validity and greedy first-fit minimality.
"""
import math

import numpy as np
import pytest

import meshgen
import oracle
from oracle import exact

F_MASS, F_EL, F_NH, F_SVK = oracle.FORM_MASS, oracle.FORM_ELAST, oracle.FORM_NH, oracle.FORM_SVK
F_LAP, F_HELM = oracle.FORM_LAPLACE, oracle.FORM_HELMHOLTZ
HYPER = pytest.mark.parametrize("form", [F_NH, F_SVK], ids=["nh", "svk"])


def small_mesh(dim, n, k, seed=0, jitter=None):
    return meshgen.make_mesh(dim, n, k, jitter, np.random.default_rng(seed))


def lattice_positions(mesh):
    """Physical coordinates of every global node (affine image of the reference lattice)."""
    X = np.zeros((mesh.n_node, mesh.dim))
    lat = np.asarray(meshgen.local_lattice(mesh.dim, mesh.k), dtype=float) / mesh.k
    for c in range(mesh.n_cell):
        x = mesh.coords[mesh.cell_verts[c]]
        X[mesh.cell_nodes[c]] = x[0] + lat @ (x[1:] - x[0])
    return X


# ----------------------------------------------------------------------------- mass
@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 3), (2, 5), (2, 8), (3, 1), (3, 2), (3, 3),
                                   (3, 6)])
def test_mass_partition_of_unity(dim, k):
    m = small_mesh(dim, 3 if dim == 2 else 2, k)
    y = oracle.action(F_MASS, m, np.ones(m.n_node), 2 * k)
    assert abs(y.sum() - 1.0) < 1e-13


def test_mass_p2_closed_form():
    # int_T lambda_i (2 lambda_i - 1) = 0 and int_T 4 lambda_i lambda_j = |T| / 3:
    # (M 1) vanishes at vertex nodes and equals sum of |T|/3 over cells holding an edge node
    m = small_mesh(2, 4, 2, seed=3)
    y = oracle.action(F_MASS, m, np.ones(m.n_node), 4)
    expect = np.zeros(m.n_node)
    for c in range(m.n_cell):
        x = m.coords[m.cell_verts[c]]
        area = 0.5 * abs(np.linalg.det(x[1:] - x[0]))
        for a, alpha in enumerate(meshgen.local_lattice(2, 2)):
            if max(list(alpha) + [2 - sum(alpha)]) < 2:      # edge midpoint node
                expect[m.cell_nodes[c, a]] += area / 3
    assert np.max(np.abs(y - expect)) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_p1_element_matrix(dim):
    m = small_mesh(dim, 1, 1, jitter=0.0)
    M = exact.assemble_mass(m)
    # on one cell the element matrix is |T| (1 + delta_ab) / ((d+1)(d+2))
    m1 = meshgen.Mesh(dim, 1, 1, m.coords, m.cell_verts[:1], m.cell_verts[:1], m.n_vert, 1.0)
    M1 = exact.assemble_mass(m1)
    vol = 1.0 / math.factorial(dim)
    idx = m.cell_verts[0]
    E = vol * (np.ones((dim + 1, dim + 1)) + np.eye(dim + 1)) / ((dim + 1) * (dim + 2))
    assert np.allclose(M1[np.ix_(idx, idx)], E, atol=1e-15, rtol=0)
    assert abs(M.sum() - 1.0) < 1e-14


@pytest.mark.parametrize("dim,n,k", [(2, 1, 1), (2, 2, 2), (2, 2, 4), (2, 2, 6), (3, 1, 1),
                                      (3, 1, 2), (3, 1, 3), (3, 1, 4)])
def test_mass_equals_exact_assembly(dim, n, k):
    m = small_mesh(dim, n, k, seed=7, jitter=0.2 if dim == 2 else 0.1)
    rng = np.random.default_rng(1)
    u = rng.uniform(-1, 1, m.n_node)
    y = oracle.action(F_MASS, m, u, 2 * k)
    M = exact.assemble_mass(m)
    assert np.max(np.abs(y - M @ u)) < 1e-14 * max(1, np.max(np.abs(M @ u))) * 10


# ------------------------------------------------------------------- Laplace and Helmholtz
@pytest.mark.parametrize("dim,k", [(2, 1), (2, 3), (2, 6), (2, 8), (3, 1), (3, 2), (3, 4), (3, 6)])
def test_laplace_kernel_patch_test_symmetry(dim, k):
    m = small_mesh(dim, 3 if dim == 2 else 2, k, seed=12, jitter=0.2 if dim == 2 else 0.1)
    qd = 2 * (k - 1)
    y1 = oracle.action(F_LAP, m, np.ones(m.n_node), qd)
    assert np.max(np.abs(y1)) < 1e-13
    # affine u: the residual vanishes at every interior node (divergence theorem)
    X = lattice_positions(m)
    u = 0.3 + X @ np.arange(1.0, dim + 1.0)
    y = oracle.action(F_LAP, m, u, qd)
    interior = np.all((X > 1e-9) & (X < 1 - 1e-9), axis=1)
    assert np.max(np.abs(y[interior])) < 1e-12 * max(1.0, np.max(np.abs(y)))
    rng = np.random.default_rng(13)
    a, b = rng.uniform(-1, 1, (2, m.n_node))
    La, Lb = oracle.action(F_LAP, m, a, qd), oracle.action(F_LAP, m, b, qd)
    assert abs(b @ La - a @ Lb) < 1e-12 * abs(b @ La)


def test_laplace_p1_reference_element():
    """Textbook P1 stiffness of the reference triangle: [[1,-1/2,-1/2],[-1/2,1/2,0],[-1/2,0,1/2]]."""
    m = meshgen.Mesh(2, 1, 1, np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]),
                     np.array([[0, 1, 2]], dtype=np.int32), np.array([[0, 1, 2]], dtype=np.int32),
                     3, 1.0)
    Kref = np.array([[1.0, -0.5, -0.5], [-0.5, 0.5, 0.0], [-0.5, 0.0, 0.5]])
    cols = np.array([oracle.action(F_LAP, m, e, 0) for e in np.eye(3)]).T
    assert np.max(np.abs(cols - Kref)) < 1e-15


@pytest.mark.parametrize("dim,n,k", [(2, 2, 2), (2, 2, 4), (3, 1, 2), (3, 1, 3)])
def test_laplace_helmholtz_equal_exact_assembly(dim, n, k):
    m = small_mesh(dim, n, k, seed=14, jitter=0.2 if dim == 2 else 0.1)
    rng = np.random.default_rng(15)
    u = rng.uniform(-1, 1, m.n_node)
    L = exact.assemble_laplace(m)
    M = exact.assemble_mass(m)
    yl = oracle.action(F_LAP, m, u, 2 * (k - 1))
    yh = oracle.action(F_HELM, m, u, 2 * k)
    assert np.max(np.abs(yl - L @ u)) < 1e-13 * np.max(np.abs(L @ u))
    assert np.max(np.abs(yh - (L + M) @ u)) < 1e-13 * np.max(np.abs((L + M) @ u))


# ----------------------------------------------------------------------------- elasticity
LAME = meshgen.lame_from_young(1.0, 0.3)


def rigid_modes(X):
    n, d = X.shape
    modes = []
    for c in range(d):
        r = np.zeros((n, d))
        r[:, c] = 1
        modes.append(r.ravel())
    pairs = [(0, 1)] if d == 2 else [(0, 1), (1, 2), (0, 2)]
    for i, j in pairs:
        r = np.zeros((n, d))
        r[:, i] = -X[:, j]
        r[:, j] = X[:, i]
        modes.append(r.ravel())
    return modes


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 4), (3, 1), (3, 2), (3, 3)])
def test_elasticity_rigid_modes(dim, k):
    m = small_mesh(dim, 3 if dim == 2 else 2, k, seed=2)
    X = lattice_positions(m)
    for r in rigid_modes(X):
        y = oracle.action(F_EL, m, r, 2 * (k - 1), LAME)
        assert np.max(np.abs(y)) < 1e-12


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (3, 2)])
def test_elasticity_patch_test_and_symmetry(dim, k):
    m = small_mesh(dim, 3 if dim == 2 else 2, k, seed=5)
    X = lattice_positions(m)
    rng = np.random.default_rng(0)
    B = rng.normal(size=(dim, dim))
    u_aff = (X @ B.T).ravel()
    y = oracle.action(F_EL, m, u_aff, 2 * (k - 1), LAME)
    interior = np.all((X > 1e-12) & (X < 1 - 1e-12), axis=1)
    # a boundary node may be interior to the domain; vertex jitter moves only interior
    # vertices so nodes on the boundary lines stay on them
    yi = y.reshape(-1, dim)[interior]
    assert np.max(np.abs(yi)) < 1e-12
    u = rng.uniform(-1, 1, m.n_node * dim)
    v = rng.uniform(-1, 1, m.n_node * dim)
    Au = oracle.action(F_EL, m, u, 2 * (k - 1), LAME)
    Av = oracle.action(F_EL, m, v, 2 * (k - 1), LAME)
    assert abs(v @ Au - u @ Av) < 1e-12 * abs(v @ Au)


@pytest.mark.parametrize("dim,n,k,lm", [(2, 2, 1, LAME), (2, 2, 2, LAME), (2, 2, 4, (0.0, 0.5)),
                                         (2, 1, 3, (10.0, 1.0)), (3, 1, 1, LAME), (3, 1, 2, LAME),
                                         (3, 1, 3, (0.0, 0.5))])
def test_elasticity_equals_exact_assembly(dim, n, k, lm):
    m = small_mesh(dim, n, k, seed=11, jitter=0.2 if dim == 2 else 0.1)
    rng = np.random.default_rng(2)
    u = rng.uniform(-1, 1, m.n_node * dim)
    y = oracle.action(F_EL, m, u, 2 * (k - 1), lm)
    K = exact.assemble_elasticity(m, *lm)
    ref = K @ u
    assert np.max(np.abs(y - ref)) < 1e-13 * np.max(np.abs(ref))


def test_elasticity_paper_constants_sigma_is_eps():
    # lambda = 0, mu = 1/2: sigma = eps, so the action is int eps(u) : eps(v)
    m = small_mesh(2, 2, 2, seed=4)
    rng = np.random.default_rng(3)
    u = rng.uniform(-1, 1, m.n_node * 2)
    y = oracle.action(F_EL, m, u, 2, (0.0, 0.5))
    y2 = oracle.action(F_EL, m, u, 2, (0.0, 1.0))
    assert np.allclose(2 * y, y2, rtol=0, atol=1e-13)


# ------------------------------------------------------------ hyperelastic (NH and SVK)
NH = (10.0, 1.0)


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 4), (3, 2)])
@HYPER
def test_hyper_invariances(form, dim, k):
    m = small_mesh(dim, 3 if dim == 2 else 2, k, seed=6)
    qd = 2 * k
    r0 = oracle.action(form, m, np.zeros(m.n_node * dim), qd, NH)
    assert np.max(np.abs(r0)) == 0.0
    rng = np.random.default_rng(4)
    u = meshgen.nh_displacement(rng, m, 0.05)
    assert oracle.min_det_f(m, u, qd) > 0.5
    r = oracle.action(form, m, u, qd, NH)
    c = np.tile(rng.normal(size=dim), m.n_node)
    rc = oracle.action(form, m, u + c, qd, NH)
    assert np.max(np.abs(rc - r)) < 1e-12 * np.max(np.abs(r))
    # finite rotation: u_R = (R - I) x is in P_k and P(R) = 0
    X = lattice_positions(m)
    th = 0.7
    if dim == 2:
        R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    else:
        a = np.array([1.0, 2.0, 2.0]) / 3
        Kx = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
        R = np.eye(3) + np.sin(th) * Kx + (1 - np.cos(th)) * Kx @ Kx
    uR = (X @ (R - np.eye(dim)).T).ravel()
    rR = oracle.action(form, m, uR, qd, NH)
    assert np.max(np.abs(rR)) < 1e-12


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 4), (3, 2)])
@HYPER
def test_hyper_residual_is_energy_gradient(form, dim, k):
    m = small_mesh(dim, 2 if dim == 2 else 1, k, seed=8)
    qd = 2 * k
    rng = np.random.default_rng(5)
    u = meshgen.nh_displacement(rng, m, 0.05)
    assert oracle.min_det_f(m, u, qd) > 0.5
    r = oracle.action(form, m, u, qd, NH)
    h = 1e-6
    fd = np.zeros_like(u)
    for i in range(len(u)):
        e = np.zeros_like(u)
        e[i] = h
        fd[i] = (oracle.energy(form, m, u + e, qd, NH) - oracle.energy(form, m, u - e, qd, NH)) / (2 * h)
    assert np.max(np.abs(fd - r)) < 1e-6 * np.max(np.abs(r)) + 1e-9


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 4), (3, 2)])
@HYPER
def test_hyper_vjp_at_zero_is_elasticity(form, dim, k):
    m = small_mesh(dim, 2, k, seed=9)
    qd = 2 * k
    rng = np.random.default_rng(6)
    v = rng.uniform(-1, 1, m.n_node * dim)
    g = oracle.vjp(form, m, np.zeros(m.n_node * dim), v, qd, NH)
    a = oracle.action(F_EL, m, v, qd, NH)
    assert np.max(np.abs(g - a)) < 1e-12 * np.max(np.abs(a))
    # and the linearisation of r at 0 along v is the same operator (central differences)
    h = 1e-6
    fd = (oracle.action(form, m, h * v, qd, NH) - oracle.action(form, m, -h * v, qd, NH)) / (2 * h)
    assert np.max(np.abs(fd - a)) < 1e-6 * np.max(np.abs(a))


@pytest.mark.parametrize("dim,k,n", [(2, 2, 2), (2, 4, 2), (3, 2, 1)])
@HYPER
def test_hyper_vjp_against_finite_differences(form, dim, k, n):
    m = small_mesh(dim, n, k, seed=10)
    qd = 2 * k
    rng = np.random.default_rng(7)
    u = meshgen.nh_displacement(rng, m, 0.05)
    assert oracle.min_det_f(m, u, qd) > 0.5
    v = rng.uniform(-1, 1, m.n_node * dim)
    w = rng.uniform(-1, 1, m.n_node * dim)
    g = oracle.vjp(form, m, u, v, qd, NH)
    # Jacobian columns by central differences; J^T v compared entrywise
    h = 1e-6
    Jcols = np.zeros((len(u), len(u)))
    for i in range(len(u)):
        e = np.zeros_like(u)
        e[i] = h
        Jcols[:, i] = (oracle.action(form, m, u + e, qd, NH)
                       - oracle.action(form, m, u - e, qd, NH)) / (2 * h)
    assert np.max(np.abs(Jcols.T @ v - g)) < 1e-6 * np.max(np.abs(g))
    # transpose identity <v, J w> = <J^T v, w>, J w by central differences
    Jw = (oracle.action(form, m, u + h * w, qd, NH) - oracle.action(form, m, u - h * w, qd, NH)) / (2 * h)
    assert abs(v @ Jw - g @ w) < 1e-6 * abs(g @ w)


@pytest.mark.parametrize("case", ["stretch", "shear"])
def test_svk_homogeneous_one_cell(case):
    """One reference triangle, P1, u = (F - I) x, so F is constant and the residual is
    r_(a, c) = |T| sum_j P_cj d_j phi_a with grad phi = (-1,-1), (1,0), (0,1).  Closed forms of
    the SVK stress P = F S worked out by hand:
      uniaxial stretch F = diag(s, 1): E = diag(e, 0), e = (s^2 - 1)/2,
        P = diag(s (lam + 2 mu) e, lam e);
      simple shear F = [[1, g], [0, 1]]: E = [[0, g/2], [g/2, g^2/2]], tr E = g^2/2,
        S = [[lam g^2/2, mu g], [mu g, lam g^2/2 + mu g^2]],
        P = [[lam g^2/2 + mu g^2, mu g + g (lam g^2/2 + mu g^2)], [mu g, lam g^2/2 + mu g^2]]."""
    lam, mu = 10.0, 1.0
    m = meshgen.Mesh(2, 1, 1, np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]),
                     np.array([[0, 1, 2]], dtype=np.int32), np.array([[0, 1, 2]], dtype=np.int32),
                     3, 1.0)
    if case == "stretch":
        s_ = 1.3
        F = np.diag([s_, 1.0])
        e = (s_ * s_ - 1.0) / 2.0
        P = np.diag([s_ * (lam + 2 * mu) * e, lam * e])
    else:
        g = 0.4
        F = np.array([[1.0, g], [0.0, 1.0]])
        t = lam * g * g / 2
        P = np.array([[t + mu * g * g, mu * g + g * (t + mu * g * g)], [mu * g, t + mu * g * g]])
    X = m.coords
    u = ((X @ F.T) - X).ravel()
    r = oracle.action(F_SVK, m, u, 2, (lam, mu)).reshape(3, 2)
    grads = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
    ref = 0.5 * grads @ P.T
    assert np.max(np.abs(r - ref)) < 1e-13 * np.max(np.abs(ref))


# ----------------------------------------------------------------------------- colouring
@pytest.mark.parametrize("dim,n,k", [(2, 6, 1), (2, 5, 3), (3, 3, 1), (3, 2, 2)])
def test_colouring_valid_and_greedy(dim, n, k):
    m = small_mesh(dim, n, k)
    col, nc = oracle.colouring(m.cell_nodes, m.n_node)
    assert col.max() + 1 == nc
    node_cells = [[] for _ in range(m.n_node)]
    for c in range(m.n_cell):
        for nd in m.cell_nodes[c]:
            node_cells[nd].append(c)
    for c in range(m.n_cell):
        nbrs = {c2 for nd in m.cell_nodes[c] for c2 in node_cells[nd] if c2 != c}
        assert all(col[c2] != col[c] for c2 in nbrs)
        earlier = {col[c2] for c2 in nbrs if c2 < c}
        assert all(cc in earlier for cc in range(col[c]))      # first fit


# ----------------------------------------------------------------------------- generator
@pytest.mark.parametrize("dim,n,k", [(2, 64, 2), (2, 8, 4), (3, 4, 2), (3, 3, 4)])
def test_generator_counts_and_orientation(dim, n, k):
    m = small_mesh(dim, n, k)
    assert m.n_node == (k * n + 1) ** dim
    assert m.n_cell == (2 if dim == 2 else 6) * n ** dim
    assert np.array_equal(np.unique(m.cell_nodes), np.arange(m.n_node))
    x = m.coords[m.cell_verts]
    dets = np.linalg.det(np.swapaxes(x[:, 1:] - x[:, :1], 1, 2))
    if dim == 2:
        assert dets.min() > 0
    assert np.abs(dets).min() > 0.3 * (1.0 / n) ** dim
    vol = np.abs(dets).sum() / math.factorial(dim)
    assert abs(vol - 1.0) < 1e-12
    # vertex nodes of the P_k map sit on the fine lattice at k * vertex
    lat = meshgen.local_lattice(dim, k)
    for r in range(dim + 1):
        alpha = np.zeros(dim, dtype=int)
        if r > 0:
            alpha[r - 1] = k
        a = int(np.where((lat == alpha).all(1))[0][0])
        v = m.cell_verts[:, r]
        nv1, nn1 = n + 1, k * n + 1
        if dim == 2:
            vx, vy = v % nv1, v // nv1
            node = k * vx + nn1 * k * vy
        else:
            vx, vy, vz = v % nv1, (v // nv1) % nv1, v // (nv1 * nv1)
            node = k * vx + nn1 * (k * vy + nn1 * k * vz)
        assert np.array_equal(m.cell_nodes[:, a], node)


def test_workload_sizes():
    w = meshgen.workload("mass_p2_2d")
    assert (w.mesh.n_cell, w.n_dof) == (8192, 16641)
    assert w.mesh.cell_nodes.shape[1] == 6

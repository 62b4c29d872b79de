"""C-ABI checks that need no GPU: exported symbols, the host-side steps of the plan
(reference tabulation and quadrature, colouring) against the oracle, and error paths."""
import ctypes
import itertools
import math
import os
import re

import numpy as np
import pytest

import meshgen
import oracle
import paper_2506_17471_amd as fx
from oracle import basis, quadrature

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "fem_action.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(fem_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert {"fem_action", "fem_action_vjp", "fem_plan_create"} <= set(names)
    L = fx.lib()
    for n in names:
        assert hasattr(L, n), n
    assert fx.lib().fem_version() >= 100


@pytest.mark.parametrize("dim,k,qd", [(2, 1, 2), (2, 2, 4), (2, 3, 6), (2, 4, 8), (2, 6, 12),
                                      (2, 7, 14), (2, 8, 16), (3, 1, 2), (3, 2, 2), (3, 2, 4),
                                      (3, 4, 6), (3, 5, 10), (3, 6, 12)])
def test_reference_tables_match_oracle(dim, k, qd):
    pts, w, phi, dphi = fx.reference_tables(dim, k, qd)
    opts, ow = quadrature.stroud(dim, qd)
    ophi, odphi = basis.tabulate(dim, k, opts)
    assert pts.shape == opts.shape
    assert np.max(np.abs(pts - opts)) < 1e-15
    # individual Gauss-Jacobi weights from two independent computations agree to ~4e-14 at
    # 8-9 points per direction; what the rule must do -- integrate every monomial up to its
    # degree exactly -- both do to rounding
    assert np.max(np.abs(w - ow) / ow) < 1e-13
    for P, W in ((pts, w), (opts, ow)):
        for e in itertools.product(range(qd + 1), repeat=dim):
            if sum(e) <= qd:
                exact = math.prod(math.factorial(a) for a in e) / math.factorial(sum(e) + dim)
                assert abs(np.sum(W * np.prod(P ** np.array(e), axis=1)) - exact) < 5e-14 * exact
    assert np.max(np.abs(phi - ophi)) < 1e-13 * max(1.0, np.max(np.abs(ophi)))
    assert np.max(np.abs(dphi - odphi)) < 1e-13 * max(10.0, np.max(np.abs(odphi)))


@pytest.mark.parametrize("dim,n,k", [(2, 16, 2), (2, 7, 4), (3, 4, 2), (3, 3, 3)])
def test_colouring_bit_exact_with_oracle(dim, n, k):
    m = meshgen.make_mesh(dim, n, k, None, np.random.default_rng(0))
    col, nc = fx.colouring(m.cell_nodes, m.n_node)
    ocol, onc = oracle.colouring(m.cell_nodes, m.n_node)
    assert nc == onc
    assert np.array_equal(col, ocol)


def test_colouring_full_size_valid():
    # at full size: the property (no two cells of one colour share a node), checked
    # vectorised per colour, plus the colour count of the oracle on the same mesh
    w = meshgen.workload("nh_p4_2d", n=128)
    col, nc = fx.colouring(w.mesh.cell_nodes, w.mesh.n_node)
    for c in range(nc):
        nodes = w.mesh.cell_nodes[col == c].ravel()
        assert len(np.unique(nodes)) == len(nodes)
    _, onc = oracle.colouring(w.mesh.cell_nodes, w.mesh.n_node)
    assert nc == onc


def _create(form=0, dim=2, degree=2, qd=4, mesh=None, params=(), **over):
    L = fx.lib()
    m = mesh or meshgen.unit_square(2, degree)
    coords = np.ascontiguousarray(over.get("coords", m.coords), dtype=np.float64)
    cv = np.ascontiguousarray(over.get("cell_verts", m.cell_verts), dtype=np.int32)
    cn = np.ascontiguousarray(over.get("cell_nodes", m.cell_nodes), dtype=np.int32)
    prm = np.asarray(params, dtype=np.float64)
    h = ctypes.c_void_p()
    st = L.fem_plan_create(ctypes.byref(h), form, dim, degree, qd, coords.shape[0],
                           coords.ctypes.data if over.get("null_coords") is None else None,
                           cv.shape[0], cv.ctypes.data, cn.ctypes.data,
                           over.get("n_node", m.n_node),
                           prm.ctypes.data if prm.size else None, prm.size)
    if st == 0:
        L.fem_plan_destroy(h)
    return st, L.fem_last_error().decode()


def test_error_paths_from_host():
    assert _create(form=7)[0] == -2
    assert _create(dim=4)[0] == -2
    assert _create(degree=9)[0] == -2
    assert _create(dim=3, degree=7, mesh=meshgen.unit_cube(1, 1))[0] == -2
    # curved cells and batches are built up to P6 (2D): a curved P7 plan is refused on the host
    mc = meshgen.curved(meshgen.unit_square(2, 7), 0.05)
    assert _create_curved(mc, degree=7, qd=14)[0] == -2
    assert _create(qd=50)[0] == -2
    assert _create(null_coords=True)[0] == -1
    assert _create(form=1, params=())[0] == -1                     # vector form, no params
    m = meshgen.unit_square(2, 2)
    bad = m.cell_nodes.copy()
    bad[3, 2] = m.n_node
    assert _create(cell_nodes=bad)[0] == -3
    badv = m.cell_verts.copy()
    badv[0, 0] = -1
    assert _create(cell_verts=badv)[0] == -3
    inv = m.cell_verts.copy()
    inv[1, [1, 2]] = inv[1, [2, 1]]                                 # clockwise triangle
    st, msg = _create(cell_verts=inv)
    assert st == -4 and "cell 1" in msg
    L = fx.lib()
    assert L.fem_action(None, None, None, None) == -1
    assert L.fem_action_vjp(None, None, None, None, None) == -1
    assert L.fem_plan_info(None, None, None, None, None, None) == -1
    # the one-shot entry fails in plan creation, before touching the vectors
    st1 = L.fem_action_once(7, 2, 2, 4, 0, None, 0, None, None, 0, None, 0, None, None, None)
    assert st1 == -2
    assert L.fem_plan_set_timing(None, 1) == -1
    assert L.fem_plan_get_timing(None, None, None) == -1
    assert L.fem_plan_destroy(None) == 0
    # measurement aids: argument checks before any launch
    assert L.fem_stream_copy(None, None, 4, None) == -1
    assert L.fem_stream_copy(None, None, 0, None) == 0
    assert L.fem_stream_copy(16, 24, 4, None) == -1 and "aligned" in L.fem_last_error().decode()
    assert L.fem_stream_copy(16, 32, 4, None) == -1 and "overlap" in L.fem_last_error().decode()
    assert L.fem_stream_read(None, 4, None, 0, None) == -1
    assert L.fem_stream_read(16, 4, 32, fx.STREAM_SINK - 1, None) == -1


def _create_curved(mesh, gcoords=None, cell_gnodes=None, form=0, degree=2, qd=4):
    L = fx.lib()
    gc = np.ascontiguousarray(mesh.gcoords if gcoords is None else gcoords, dtype=np.float64)
    cg = np.ascontiguousarray(mesh.cell_gnodes if cell_gnodes is None else cell_gnodes,
                              dtype=np.int32)
    cn = np.ascontiguousarray(mesh.cell_nodes, dtype=np.int32)
    h = ctypes.c_void_p()
    st = L.fem_plan_create_curved(ctypes.byref(h), form, mesh.dim, degree, qd, gc.shape[0],
                                  gc.ctypes.data, cg.shape[0], cg.ctypes.data, cn.ctypes.data,
                                  mesh.n_node, None, 0)
    if st == 0:
        L.fem_plan_destroy(h)
    return st, L.fem_last_error().decode()


def test_curved_plan_validation_from_host():
    m = meshgen.curved(meshgen.unit_square(3, 2), 0.05)
    # a valid curved mesh passes validation (and then needs a device)
    st, _ = _create_curved(m)
    try:
        import torch
        has_dev = torch.cuda.is_available()
    except ImportError:
        has_dev = False
    assert st == (0 if has_dev else -5)
    bad = m.cell_gnodes.copy()
    bad[2, 3] = m.gcoords.shape[0]
    assert _create_curved(m, cell_gnodes=bad)[0] == -3
    # an edge node of cell 4 dragged across its cell folds the map: det J changes sign
    gc = m.gcoords.copy()
    c = 4
    mid, opp = m.cell_gnodes[c, 1], m.cell_gnodes[c, 5]     # edge (v0, v1) and vertex v2
    gc[mid] = gc[mid] + 1.5 * (gc[opp] - gc[mid])
    st, msg = _create_curved(m, gcoords=gc)
    assert st == -4 and "curved cell" in msg


def test_plan_without_device_reports_hip_error():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a device is present")
    except ImportError:
        pass
    st, msg = _create()
    assert st == -5 and "hipGetDevice" in msg


@pytest.mark.parametrize("form,dim,n,k,P", [(0, 2, 9, 2, 64), (2, 2, 12, 4, 128), (2, 2, 16, 4, 256),
                                            (1, 3, 3, 2, 64), (1, 3, 4, 2, 256), (0, 3, 3, 4, 64),
                                            (2, 2, 7, 6, 0), (1, 3, 2, 3, 0), (0, 2, 1, 1, 64),
                                            (1, 3, 3, 4, 63), (2, 3, 3, 2, 21), (1, 3, 4, 2, 84)])
def test_patch_layout_valid(form, dim, n, k, P):
    m = meshgen.make_mesh(dim, n, k, None, np.random.default_rng(n))
    st = fx.check_patch_layout(form, m, P)
    assert st["n_patch"] == -(-m.n_cell // st["patch_cells"])
    assert st["max_patch_nodes"] <= st["patch_cells"] * m.cell_nodes.shape[1]
    assert st["lds_bytes"] <= 160 * 1024
    # every node held by some patch; shared nodes have one partial per holding patch
    assert st["patch_node_pairs"] == m.n_node + st["partial_slots"] - st["shared_nodes"]


def test_tetrahedral_patch_sub_colours_near_vertex_bound():
    # the 24 tetrahedra around an interior vertex of the structured cube mesh need 24 colours;
    # first-fit in Morton order takes up to 31 on 256-cell patches, and with DSatur's colouring
    # kept where it saves two or more no patch of this mesh needs more than 26; the layout
    # check also validates the colouring (no node twice within a colour)
    m = meshgen.make_mesh(3, 16, 2, None, np.random.default_rng(16))
    st = fx.check_patch_layout(1, m, 256)
    assert 24 <= st["max_colours"] <= 26


def test_patch_layout_rejects_bad_size():
    m = meshgen.unit_square(4, 2)
    with pytest.raises(fx.FemError):
        fx.check_patch_layout(0, m, 300)


SYM_DEGREES = [(2, d) for d in range(0, 13)] + [(3, d) for d in range(0, 9)]


@pytest.mark.parametrize("dim,deg", SYM_DEGREES)
def test_symmetric_rules_exact(dim, deg):
    """The library's symmetric rules: exact on every monomial up to the degree, positive
    weights, points inside, and the same point set as the oracle's independently solved
    rule (both solve the moment equations; the NH operator depends on the rule)."""
    import itertools
    import math
    pts, w, phi, dphi = fx.reference_tables(dim, 2, deg, fx.QUAD_SYMMETRIC)
    assert np.all(w > 0) and np.all(pts > 0) and np.all(pts.sum(1) < 1)
    for b in itertools.product(range(deg + 1), repeat=dim):
        if sum(b) > deg:
            continue
        ref = math.prod(math.factorial(x) for x in b) / math.factorial(sum(b) + dim)
        assert abs(np.sum(w * np.prod(pts ** np.asarray(b), axis=1)) - ref) <= 2e-14 * ref
    opts, ow = quadrature.symmetric(dim, deg)
    assert len(ow) == len(w)
    ka, kb = np.lexsort(np.c_[pts, w].T[::-1]), np.lexsort(np.c_[opts, ow].T[::-1])
    # the same root to the conditioning of the moment equations (~1e-13 at degree 10)
    assert np.max(np.abs(pts[ka] - opts[kb])) < 5e-13 and np.max(np.abs(w[ka] - ow[kb])) < 5e-14
    # tabulation at the symmetric points agrees with the oracle's basis at the same points
    ophi, odphi = basis.tabulate(dim, 2, pts)
    assert np.max(np.abs(phi - ophi)) < 1e-14 and np.max(np.abs(dphi - odphi)) < 1e-13


@pytest.mark.parametrize("dim,deg", [(2, 30), (3, 30)])
def test_symmetric_rule_missing_degree_is_unsupported(dim, deg):
    with pytest.raises(fx.FemError):
        fx.reference_tables(dim, 2, deg, fx.QUAD_SYMMETRIC)

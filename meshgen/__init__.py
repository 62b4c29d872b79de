"""Seeded synthetic inputs: structured simplex meshes, P_k node numbering, random vectors.

This module is the only code shared by the CPU oracle and the GPU library's tests and
benchmark. It builds *inputs* only (vertex coordinates, cell-to-vertex map, cell-to-node
map, nodal vectors); it holds none of the finite element arithmetic (no basis, no
quadrature, no geometry, no forms).

Mesh recipe (the paper benchmarks on the unit square and the unit cube, Sec. 6.2.1;
the split into simplices is not stated there, so it is fixed here):

* 2D: an n x n grid of squares; square (i, j) is cut along its (i,j)-(i+1,j+1) diagonal
  into triangles t=0: (v00, v10, v11) and t=1: (v00, v11, v01), both counter-clockwise.
  Cell id = 2 (i + n j) + t.  Vertex id = x + (n+1) y on the integer vertex lattice.
* 3D: an n^3 grid of cubes; cube (i, j, l) is cut into the six Kuhn tetrahedra, one per
  permutation s of the axes in lexicographic order, v_0 = cube corner,
  v_{r+1} = v_r + e_{s_r}.  Cell id = 6 (i + n (j + n l)) + perm index.
  Vertex id = x + (n+1) (y + (n+1) z).  Odd permutations give det J < 0; the action uses
  |det J| so these cells are valid as they stand.

Local node order of a P_k cell (the interface convention shared by every consumer of
``cell_nodes``): the reference lattice points xi = alpha / k with alpha in N^d,
|alpha| <= k, enumerated with the first coordinate fastest:
``for a_d ... for a_2: for a_1`` (e.g. 2D: for j in 0..k: for i in 0..k-j: (i, j)).
The global node of local point alpha in a cell with vertex lattice points v_0..v_d is
the fine-lattice point  L = k v_0 + sum_r alpha_r (v_r - v_0), numbered
L_x + (kn+1) L_y (+ (kn+1)^2 L_z); this yields exactly (kn+1)^d nodes.

Jitter: interior vertices only are moved, by U[-a h, a h] per coordinate, so the domain
measure stays exactly 1.  Random draws use numpy PCG64 (``default_rng(seed)``) in the
fixed order: jitter [n_vert, d], then u, then v.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Mesh", "local_lattice", "unit_square", "unit_cube", "make_mesh", "n_local",
    "Workload", "workload", "batch_workloads", "nh_displacement", "curved",
]


def n_local(dim: int, k: int) -> int:
    """Number of P_k Lagrange nodes on a d-simplex: C(k+d, d)."""
    return math.comb(k + dim, dim)


def local_lattice(dim: int, k: int) -> np.ndarray:
    """Reference lattice multi-indices alpha (|alpha| <= k), first coordinate fastest."""
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
    return np.asarray(pts, dtype=np.int64)


@dataclass
class Mesh:
    dim: int
    n: int                      # grid cells per side
    k: int                      # polynomial degree of the node map
    coords: np.ndarray          # float64 [n_vert, dim]
    cell_verts: np.ndarray      # int32 [n_cell, dim+1]
    cell_nodes: np.ndarray      # int32 [n_cell, C(k+d,d)]
    n_node: int
    h: float = field(default=0.0)
    # curved meshes only (see ``curved``): P2 geometry nodes and each cell's 6 / 10 of them
    gcoords: np.ndarray | None = None       # float64 [n_gnode, dim]
    cell_gnodes: np.ndarray | None = None   # int32 [n_cell, C(2+d,d)], local P2 lattice order

    @property
    def n_cell(self) -> int:
        return int(self.cell_verts.shape[0])

    @property
    def n_vert(self) -> int:
        return int(self.coords.shape[0])


def _jitter(rng, lattice_xyz: np.ndarray, n: int, h: float, amp: float) -> np.ndarray:
    nv, d = lattice_xyz.shape
    draw = rng.uniform(-1.0, 1.0, size=(nv, d))
    interior = np.all((lattice_xyz > 0) & (lattice_xyz < n), axis=1)
    coords = lattice_xyz.astype(np.float64) * h
    coords[interior] += amp * h * draw[interior]
    return coords


def unit_square(n: int, k: int, jitter: float = 0.1, rng=None) -> Mesh:
    """Unit square, n x n squares, 2 triangles each; P_k node numbering."""
    if rng is None:
        rng = np.random.default_rng(0)
    h = 1.0 / n
    nv1 = n + 1
    jj, ii = np.meshgrid(np.arange(nv1), np.arange(nv1), indexing="ij")
    lat = np.stack([ii.ravel(), jj.ravel()], axis=1)          # vertex id = x + (n+1) y
    coords = _jitter(rng, lat, n, h, jitter)

    sj, si = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    si = si.ravel()
    sj = sj.ravel()                                            # square id = i + n j
    c00 = np.stack([si, sj], 1)
    off = {
        0: [(0, 0), (1, 0), (1, 1)],
        1: [(0, 0), (1, 1), (0, 1)],
    }
    nsq = n * n
    vl = np.empty((nsq, 2, 3, 2), dtype=np.int64)              # [square, t, vertex, xy]
    for t in (0, 1):
        for r, (dx, dy) in enumerate(off[t]):
            vl[:, t, r, 0] = c00[:, 0] + dx
            vl[:, t, r, 1] = c00[:, 1] + dy
    vl = vl.reshape(2 * nsq, 3, 2)
    cell_verts = (vl[:, :, 0] + nv1 * vl[:, :, 1]).astype(np.int32)

    alpha = local_lattice(2, k)                                # [nloc, 2]
    e = vl[:, 1:, :] - vl[:, :1, :]                            # [cell, r, xy]
    L = k * vl[:, None, 0, :] + np.einsum("ar,crx->cax", alpha, e)
    nn1 = k * n + 1
    cell_nodes = (L[..., 0] + nn1 * L[..., 1]).astype(np.int32)
    return Mesh(2, n, k, coords, cell_verts, cell_nodes, nn1 * nn1, h)


def unit_cube(n: int, k: int, jitter: float = 0.05, rng=None) -> Mesh:
    """Unit cube, n^3 cubes, 6 Kuhn tetrahedra each; P_k node numbering."""
    if rng is None:
        rng = np.random.default_rng(0)
    h = 1.0 / n
    nv1 = n + 1
    zz, yy, xx = np.meshgrid(np.arange(nv1), np.arange(nv1), np.arange(nv1), indexing="ij")
    lat = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    coords = _jitter(rng, lat, n, h, jitter)

    cz, cy, cx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    corner = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], 1)  # cube id = i + n (j + n l)
    ncube = n ** 3
    perms = list(itertools.permutations(range(3)))              # lexicographic order
    vl = np.empty((ncube, 6, 4, 3), dtype=np.int64)
    for p, s in enumerate(perms):
        cur = corner.copy()
        vl[:, p, 0] = cur
        for r in range(3):
            cur = cur.copy()
            cur[:, s[r]] += 1
            vl[:, p, r + 1] = cur
    vl = vl.reshape(6 * ncube, 4, 3)
    cell_verts = (vl[..., 0] + nv1 * (vl[..., 1] + nv1 * vl[..., 2])).astype(np.int32)

    alpha = local_lattice(3, k)
    e = vl[:, 1:, :] - vl[:, :1, :]
    L = k * vl[:, None, 0, :] + np.einsum("ar,crx->cax", alpha, e)
    nn1 = k * n + 1
    cell_nodes = (L[..., 0] + nn1 * (L[..., 1] + nn1 * L[..., 2])).astype(np.int32)
    return Mesh(3, n, k, coords, cell_verts, cell_nodes, nn1 ** 3, h)


def make_mesh(dim: int, n: int, k: int, jitter: float | None = None, rng=None) -> Mesh:
    if dim == 2:
        return unit_square(n, k, 0.1 if jitter is None else jitter, rng)
    if dim == 3:
        return unit_cube(n, k, 0.05 if jitter is None else jitter, rng)
    raise ValueError("dim must be 2 or 3")


def _warp(x: np.ndarray) -> np.ndarray:
    """Smooth displacement field vanishing on the boundary of the unit square / cube:
    prod_j sin(pi x_j) times (cos pi x_1, cos pi x_0) in 2D, (cos pi x_1, cos pi x_2,
    cos pi x_0) in 3D."""
    d = x.shape[1]
    s = np.prod(np.sin(np.pi * x), axis=1)
    return s[:, None] * np.cos(np.pi * x[:, [(i + 1) % d for i in range(d)]])


def curved(mesh: Mesh, amp: float = 0.05) -> Mesh:
    """The same mesh with curved (non-affine) cells: a P2 geometry per cell.

    Geometry nodes: the P2 lattice of the mesh, numbered like P2 solution nodes
    (L = 2 v_0 + sum_r alpha_r (v_r - v_0) on the (2n+1)^d lattice), each placed at the
    barycentric point (alpha_0, alpha_1, ..)/2 of its cell's (jittered) vertices and then
    moved by ``amp * _warp(x)``.  Nodes on the boundary do not move, so the domain stays the
    unit square / cube and every boundary edge straight; inside, each cell is the P2
    interpolant of a smooth nonlinear map.  ``amp = 0`` gives straight P2 geometry, which
    describes the affine cells exactly.  The solution nodes (``cell_nodes``) are unchanged.
    """
    d, n = mesh.dim, mesh.n
    nv1, nn1 = n + 1, 2 * n + 1
    vid = mesh.cell_verts.astype(np.int64)
    if d == 2:
        vl = np.stack([vid % nv1, vid // nv1], axis=-1)
    else:
        vl = np.stack([vid % nv1, (vid // nv1) % nv1, vid // (nv1 * nv1)], axis=-1)
    alpha = local_lattice(d, 2)                                  # [ng, d]
    e = vl[:, 1:, :] - vl[:, :1, :]
    L = 2 * vl[:, None, 0, :] + np.einsum("ar,crx->cax", alpha, e)
    gid = L[..., 0] + nn1 * L[..., 1] + (nn1 * nn1 * L[..., 2] if d == 3 else 0)
    bary = np.concatenate([2 - alpha.sum(axis=1, keepdims=True), alpha], axis=1) / 2.0
    X = mesh.coords[mesh.cell_verts]                             # [cell, d+1, d]
    pts = np.einsum("gv,cvx->cgx", bary, X)
    gcoords = np.zeros((nn1 ** d, d))
    gcoords[gid.reshape(-1)] = pts.reshape(-1, d)
    lat = np.zeros((nn1 ** d, d), dtype=np.int64)
    lat[gid.reshape(-1)] = L.reshape(-1, d)
    interior = np.all((lat > 0) & (lat < 2 * n), axis=1)
    gcoords[interior] += amp * _warp(gcoords[interior])
    return Mesh(d, n, mesh.k, mesh.coords, mesh.cell_verts, mesh.cell_nodes, mesh.n_node,
                mesh.h, gcoords, gid.astype(np.int32))


def nh_displacement(rng, mesh: Mesh, amplitude: float = 0.01) -> np.ndarray:
    """Displacement for the hyperelastic forms: amplitude * (h/k) * U[-1,1] per DoF.

    Nodal values of size O(1) would make grad u ~ k/h and fold the cells (det F <= 0);
    scaling by h/k keeps |grad u| ~ amplitude.
    """
    return amplitude * (mesh.h / mesh.k) * rng.uniform(-1.0, 1.0, size=mesh.n_node * mesh.dim)


# ---------------------------------------------------------------------------
# The named workloads.  Form ids: 0 mass, 1 linear elasticity, 2 neo-Hookean.
# ---------------------------------------------------------------------------
FORM_MASS, FORM_ELAST, FORM_NH, FORM_SVK, FORM_LAPLACE, FORM_HELMHOLTZ = 0, 1, 2, 3, 4, 5


def lame_from_young(E: float, nu: float) -> tuple[float, float]:
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


@dataclass
class Workload:
    name: str
    form: int
    mesh: Mesh
    quad_degree: int
    params: tuple          # (lambda, mu) for elasticity / NH, () for mass
    u: np.ndarray
    v: np.ndarray | None = None

    @property
    def ncomp(self) -> int:
        return 1 if self.form in (FORM_MASS, FORM_LAPLACE, FORM_HELMHOLTZ) else self.mesh.dim

    @property
    def n_dof(self) -> int:
        return self.mesh.n_node * self.ncomp


# name -> (form, dim, n, k, quad_degree, jitter, seed, params)
_SPECS = {
    # 2D P2 mass, 64^2 squares (8192 cells, 16641 DoFs), quadrature degree 4
    "mass_p2_2d": (FORM_MASS, 2, 64, 2, 4, 0.1, 0, ()),
    # same form at 1024^2: large enough to be bound by HBM rather than launch latency
    "mass_p2_2d_1024": (FORM_MASS, 2, 1024, 2, 4, 0.1, 0, ()),
    # 2D vector P4 neo-Hookean residual, 512^2 squares, mu=1, lambda=10, degree 8
    "nh_p4_2d": (FORM_NH, 2, 512, 4, 8, 0.1, 1, (10.0, 1.0)),
    # 3D vector P2 linear elasticity, 64^3 cubes x 6 tets, E=1, nu=0.3, degree 2
    "elast_p2_3d": (FORM_ELAST, 3, 64, 2, 2, 0.05, 2, lame_from_young(1.0, 0.3)),
    # VJP of the neo-Hookean residual on the 512^2 P4 mesh
    "nh_vjp_p4_2d": (FORM_NH, 2, 512, 4, 8, 0.1, 3, (10.0, 1.0)),
    # St Venant-Kirchhoff residual and tangent on the same mesh and rule degree (the
    # paper's hyperelastic law; its benchmark times the tangent action)
    "svk_p4_2d": (FORM_SVK, 2, 512, 4, 8, 0.1, 5, (10.0, 1.0)),
    # curved (P2-geometry) cells: the neo-Hookean P4 residual and the P2 mass action on
    # the meshes above with every cell bent by ``curved(mesh, 0.05)``
    "nh_p4_2d_curved": (FORM_NH, 2, 512, 4, 8, 0.1, 1, (10.0, 1.0)),
    "mass_p2_2d_1024_curved": (FORM_MASS, 2, 1024, 2, 4, 0.1, 0, ()),
    # high degree at the paper's smaller sizes (about 2e5 cells): 3D P4 elasticity (32^3
    # cubes x 6 tets, degree 6) and the 2D P6 neo-Hookean residual (316^2 squares, degree 12)
    "elast_p4_3d": (FORM_ELAST, 3, 32, 4, 6, 0.05, 6, lame_from_young(1.0, 0.3)),
    "nh_p6_2d": (FORM_NH, 2, 316, 6, 12, 0.1, 7, (10.0, 1.0)),
}
_CURVED_AMP = {"nh_p4_2d_curved": 0.05, "mass_p2_2d_1024_curved": 0.05}


def workload(name: str, n: int | None = None, seed: int | None = None,
             with_v: bool = False) -> Workload:
    """Build a named workload; ``n`` overrides the grid size (same recipe otherwise)."""
    form, dim, n0, k, qdeg, jit, seed0, params = _SPECS[name]
    n = n0 if n is None else n
    rng = np.random.default_rng(seed0 if seed is None else seed)
    mesh = make_mesh(dim, n, k, jit, rng)
    if name in _CURVED_AMP:
        mesh = curved(mesh, _CURVED_AMP[name])
    ncomp = 1 if form in (FORM_MASS, FORM_LAPLACE, FORM_HELMHOLTZ) else dim
    if form in (FORM_NH, FORM_SVK):
        u = nh_displacement(rng, mesh)
    else:
        u = rng.uniform(-1.0, 1.0, size=mesh.n_node * ncomp)
    v = None
    if with_v or name.startswith("nh_vjp"):
        v = rng.uniform(-1.0, 1.0, size=mesh.n_node * ncomp)
    return Workload(name, form, mesh, qdeg, tuple(params), u, v)


def batch_workloads(n_mesh: int = 64, seed: int = 4, lo: float = 1e3, hi: float = 2e5,
                    scale: float = 1.0) -> list[Workload]:
    """Uneven batch: mesh i has form i mod 3 (2D P3 mass, 2D P6 neo-Hookean,
    3D P4 elasticity), cell counts log-uniform in [lo, hi] (times ``scale``)."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_mesh)) * scale
    out = []
    for i in range(n_mesh):
        kind = i % 3
        if kind == 0:
            n = max(1, int(round(math.sqrt(sizes[i] / 2))))
            mesh = unit_square(n, 3, 0.1, rng)
            out.append(Workload(f"batch{i}_mass_p3_2d", FORM_MASS, mesh, 6, (),
                                rng.uniform(-1, 1, size=mesh.n_node)))
        elif kind == 1:
            n = max(1, int(round(math.sqrt(sizes[i] / 2))))
            mesh = unit_square(n, 6, 0.1, rng)
            out.append(Workload(f"batch{i}_nh_p6_2d", FORM_NH, mesh, 12, (10.0, 1.0),
                                nh_displacement(rng, mesh)))
        else:
            n = max(1, int(round((sizes[i] / 6) ** (1.0 / 3.0))))
            mesh = unit_cube(n, 4, 0.05, rng)
            out.append(Workload(f"batch{i}_elast_p4_3d", FORM_ELAST, mesh, 6,
                                lame_from_young(1.0, 0.3),
                                rng.uniform(-1, 1, size=mesh.n_node * 3)))
    return out

"""CPU oracle for the matrix-free finite element action -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct FP64 code that the GPU library is checked against.
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it; the GPU library never does, and the two share no code (basis, quadrature,
geometry, forms, colouring are all written separately here).

Pieces:
* ``quadrature.stroud``  -- conical-product rule (scipy Gauss-Jacobi roots);
* ``quadrature.symmetric`` -- fully symmetric rules (moment equations, scipy least squares);
* ``basis.tabulate``     -- Silvester-formula P_k Lagrange values and reference gradients;
* ``fem_oracle.c``       -- the per-cell loop of the paper's generic action kernel
  (Sec. 2.3) for the mass, Laplace, Helmholtz, linear elasticity, neo-Hookean and
  St Venant-Kirchhoff forms (App. A), the hyperelastic VJPs written as the literal
  transpose of the tangent, the discrete energies, and greedy first-fit colouring; the
  Jacobian of the cell map is evaluated at every quadrature point from a geometry basis
  (P1 on the vertices for affine cells, P2 for curved cells, Sec. 2.4);
* ``exact``              -- quadrature-free assembly of mass, elasticity and Laplace
  matrices by exact integration of barycentric monomials (the brute-force pin).

Parity pins: every function here is checked in ``tests/test_oracle_*.py`` against closed
forms, invariants and brute force; none is pinned by re-running itself.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import basis, quadrature

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fem_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

FORM_MASS, FORM_ELAST, FORM_NH, FORM_SVK, FORM_LAPLACE, FORM_HELMHOLTZ = 0, 1, 2, 3, 4, 5
SCALAR_FORMS = (FORM_MASS, FORM_LAPLACE, FORM_HELMHOLTZ)


def build() -> str:
    """Compile the C oracle with gcc (plain -O2, no fast-math)."""
    # build beside the target and rename, so that concurrent test workers never load a
    # half-written library
    tmp = f"{_LIB}.{os.getpid()}.tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


class using_library:
    """Temporarily route the oracle through another build of fem_oracle.c (the mutation
    tests compile deliberately broken copies to check that the pins catch them)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _load()
        _lib = _bind(ctypes.CDLL(self.path))
        return _lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _bind(lib):
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_double
    lib.oracle_action.argtypes = [i32, i32, i32, i32, P, P, P, i32, P, i64, P, P, P, f64, f64, P,
                                  P, i64]
    lib.oracle_action.restype = None
    lib.oracle_vjp.argtypes = [i32, i32, i32, i32, P, P, P, i32, P, i64, P, P, P, f64, f64, P, P,
                               P, i64]
    lib.oracle_vjp.restype = None
    lib.oracle_energy.argtypes = [i32, i32, i32, i32, P, P, i32, P, i64, P, P, P, f64, f64, P]
    lib.oracle_energy.restype = f64
    lib.oracle_min_det_f.argtypes = [i32, i32, i32, P, i32, P, i64, P, P, P, P]
    lib.oracle_min_det_f.restype = f64
    lib.oracle_colouring.argtypes = [i64, i32, P, i32, P, P]
    lib.oracle_colouring.restype = i32
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Tables:
    """Quadrature rule and tabulation for (dim, k, quadrature degree, rule family)."""

    def __init__(self, dim: int, k: int, quad_degree: int, family: str = "conical"):
        self.dim, self.k, self.quad_degree, self.family = dim, k, quad_degree, family
        if family == "conical":
            self.points, self.weights = quadrature.stroud(dim, quad_degree)
        elif family == "symmetric":
            self.points, self.weights = quadrature.symmetric(dim, quad_degree)
        else:
            raise ValueError(family)
        phi, dphi = basis.tabulate(dim, k, self.points)
        self.phi = np.ascontiguousarray(phi, dtype=np.float64)
        self.dphi = np.ascontiguousarray(dphi, dtype=np.float64)
        self.weights = np.ascontiguousarray(self.weights, dtype=np.float64)
        self.nq = len(self.weights)
        self.nloc = self.phi.shape[1]
        self._geometry = {}

    def geometry(self, degree: int) -> np.ndarray:
        """Reference gradients [nq, ng, dim] of the degree-1 (vertices) or degree-2 (curved
        cells) geometry basis at the rule's points: the cell map is x(xi) = sum_g x_g phiG_g."""
        if degree not in self._geometry:
            _, g = basis.tabulate(self.dim, degree, self.points)
            self._geometry[degree] = np.ascontiguousarray(g, dtype=np.float64)
        return self._geometry[degree]


_tables_cache: dict = {}


def tables(dim: int, k: int, quad_degree: int, family: str = "conical") -> Tables:
    key = (dim, k, quad_degree, family)
    if key not in _tables_cache:
        _tables_cache[key] = Tables(dim, k, quad_degree, family)
    return _tables_cache[key]


def _mesh_arrays(mesh, t: Tables):
    """(cell geometry nodes, cell nodes, geometry coordinates, ng, geometry gradients): the
    vertices and P1 geometry, or a curved mesh's P2 geometry nodes (``mesh.cell_gnodes``)."""
    curved = getattr(mesh, "cell_gnodes", None) is not None
    cv = np.ascontiguousarray(mesh.cell_gnodes if curved else mesh.cell_verts, dtype=np.int32)
    cn = np.ascontiguousarray(mesh.cell_nodes, dtype=np.int32)
    xy = np.ascontiguousarray(mesh.gcoords if curved else mesh.coords, dtype=np.float64)
    g = t.geometry(2 if curved else 1)
    assert g.shape[1] == cv.shape[1]
    return cv, cn, xy, g.shape[1], g


def _lam_mu(params):
    if len(params) == 0:
        return 0.0, 0.0
    return float(params[0]), float(params[1])


def action(form: int, mesh, u: np.ndarray, quad_degree: int, params=(),
           family: str = "conical") -> np.ndarray:
    """y = A(u) by the plain per-cell loop."""
    lib = _load()
    t = tables(mesh.dim, mesh.k, quad_degree, family)
    cv, cn, xy, ng, g = _mesh_arrays(mesh, t)
    ncomp = 1 if form in SCALAR_FORMS else mesh.dim
    n_dof = mesh.n_node * ncomp
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert u.shape == (n_dof,)
    y = np.empty(n_dof)
    lam, mu = _lam_mu(params)
    lib.oracle_action(form, mesh.dim, t.nloc, t.nq, _ptr(t.phi), _ptr(t.dphi), _ptr(t.weights),
                      ng, _ptr(g), cv.shape[0], _ptr(cv), _ptr(xy), _ptr(cn), lam, mu, _ptr(u),
                      _ptr(y), n_dof)
    return y


def vjp(form: int, mesh, u: np.ndarray, v: np.ndarray, quad_degree: int, params=(),
        family: str = "conical") -> np.ndarray:
    """g = (dA/du)^T v."""
    lib = _load()
    t = tables(mesh.dim, mesh.k, quad_degree, family)
    cv, cn, xy, ng, gd = _mesh_arrays(mesh, t)
    ncomp = 1 if form in SCALAR_FORMS else mesh.dim
    n_dof = mesh.n_node * ncomp
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert u.shape == (n_dof,) and v.shape == (n_dof,)
    g = np.empty(n_dof)
    lam, mu = _lam_mu(params)
    lib.oracle_vjp(form, mesh.dim, t.nloc, t.nq, _ptr(t.phi), _ptr(t.dphi), _ptr(t.weights),
                   ng, _ptr(gd), cv.shape[0], _ptr(cv), _ptr(xy), _ptr(cn), lam, mu, _ptr(u),
                   _ptr(v), _ptr(g), n_dof)
    return g


def energy(form: int, mesh, u: np.ndarray, quad_degree: int, params,
           family: str = "conical") -> float:
    """Discrete energy Pi_h(u) of a hyperelastic form (neo-Hookean or St Venant-Kirchhoff)."""
    lib = _load()
    t = tables(mesh.dim, mesh.k, quad_degree, family)
    cv, cn, xy, ng, g = _mesh_arrays(mesh, t)
    u = np.ascontiguousarray(u, dtype=np.float64)
    lam, mu = _lam_mu(params)
    return lib.oracle_energy(form, mesh.dim, t.nloc, t.nq, _ptr(t.dphi), _ptr(t.weights), ng,
                             _ptr(g), cv.shape[0], _ptr(cv), _ptr(xy), _ptr(cn), lam, mu, _ptr(u))


def nh_energy(mesh, u: np.ndarray, quad_degree: int, params, family: str = "conical") -> float:
    """Discrete neo-Hookean energy Pi_h(u)."""
    return energy(FORM_NH, mesh, u, quad_degree, params, family)


def min_det_f(mesh, u: np.ndarray, quad_degree: int, family: str = "conical") -> float:
    lib = _load()
    t = tables(mesh.dim, mesh.k, quad_degree, family)
    cv, cn, xy, ng, g = _mesh_arrays(mesh, t)
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib.oracle_min_det_f(mesh.dim, t.nloc, t.nq, _ptr(t.dphi), ng, _ptr(g), cv.shape[0],
                                _ptr(cv), _ptr(xy), _ptr(cn), _ptr(u))


def colouring(cell_nodes: np.ndarray, n_node: int, nwords: int = 2) -> tuple[np.ndarray, int]:
    """Greedy first-fit colouring by shared nodes, cells in ascending id."""
    lib = _load()
    cn = np.ascontiguousarray(cell_nodes, dtype=np.int32)
    colour = np.empty(cn.shape[0], dtype=np.int32)
    masks = np.zeros(n_node * nwords, dtype=np.uint64)
    nc = lib.oracle_colouring(cn.shape[0], cn.shape[1], _ptr(cn), nwords, _ptr(colour), _ptr(masks))
    if nc < 0:
        raise RuntimeError("more colours than the mask holds")
    return colour, nc

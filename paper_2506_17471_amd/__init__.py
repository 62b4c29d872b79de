"""femx: matrix-free FP64 finite element actions on MI355X (gfx950).

A thin ctypes binding over the C ABI in ``include/fem_action.h`` (``libfemx.so``).
PyTorch supplies device memory and the current HIP stream; every step of the action runs
in the library's HIP kernels.  There is no CPU fallback: if the library is missing the
import of :func:`lib` raises.

    plan = Plan(FORM_NEOHOOKEAN, dim=2, degree=4, quad_degree=8, coords=..., cell_verts=...,
                cell_nodes=..., n_node=..., params=(lam, mu))
    y = plan.action(u)                 # u: float64 CUDA tensor [n_node * ncomp]
    g = plan.vjp(u, v)                 # (dA/du)^T v
    y = FemAction.apply(u, plan)       # autograd: backward calls the VJP kernel
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

__all__ = ["FORM_MASS", "FORM_ELASTICITY", "FORM_NEOHOOKEAN", "FemError", "Plan", "FemAction",
           "lib", "reference_tables", "colouring", "check_patch_layout", "LIB_PATH", "Batch",
           "SCATTER_COLOUR", "SCATTER_PATCH"]

FORM_MASS, FORM_ELASTICITY, FORM_NEOHOOKEAN, FORM_SVK, FORM_LAPLACE, FORM_HELMHOLTZ = 0, 1, 2, 3, 4, 5
SCALAR_FORMS = (FORM_MASS, FORM_LAPLACE, FORM_HELMHOLTZ)
QUAD_CONICAL, QUAD_SYMMETRIC = 0, 1
SCATTER_COLOUR, SCATTER_PATCH = 0, 1
SUM_ELEMENT, SUM_COLOURED = 1, 2
OK, E_ARG, E_UNSUPPORTED, E_INDEX, E_INVERTED, E_HIP, E_NOMEM = 0, -1, -2, -3, -4, -5, -6
LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfemx.so")

_STATUS = {0: "FEM_OK", -1: "FEM_E_ARG", -2: "FEM_E_UNSUPPORTED", -3: "FEM_E_INDEX",
           -4: "FEM_E_INVERTED", -5: "FEM_E_HIP", -6: "FEM_E_NOMEM"}

_lib = None


class FemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def lib() -> ctypes.CDLL:
    """Load libfemx.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        import torch  # noqa: F401  (loads the HIP runtime the library binds to)
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2506_17471_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    L.fem_plan_create.argtypes = [ctypes.POINTER(P), i32, i32, i32, i32, i64, P, i64, P, P, i64, P, i32]
    L.fem_plan_create.restype = i32
    L.fem_plan_create_curved.argtypes = L.fem_plan_create.argtypes
    L.fem_plan_create_curved.restype = i32
    L.fem_plan_destroy.argtypes = [P]
    L.fem_plan_destroy.restype = i32
    L.fem_action.argtypes = [P, P, P, P]
    L.fem_action.restype = i32
    L.fem_action_vjp.argtypes = [P, P, P, P, P]
    L.fem_action_vjp.restype = i32
    L.fem_plan_info.argtypes = [P, P, P, P, P, P]
    L.fem_plan_info.restype = i32
    L.fem_plan_colouring.argtypes = [P, P]
    L.fem_plan_colouring.restype = i32
    L.fem_reference_tables.argtypes = [i32, i32, i32, i32, P, P, P, P, P, P]
    L.fem_plan_set_quadrature.argtypes = [P, i32]
    L.fem_plan_set_quadrature.restype = i32
    L.fem_reference_tables.restype = i32
    L.fem_plan_set_block.argtypes = [P, i32]
    L.fem_plan_set_block.restype = i32
    L.fem_action_jvp.argtypes = [P, P, P, P, P]
    L.fem_action_jvp.restype = i32
    L.fem_action_once.argtypes = [i32, i32, i32, i32, i64, P, i64, P, P, i64, P, i32, P, P, P]
    L.fem_action_once.restype = i32
    L.fem_plan_get_quadrature.argtypes = [P, P, P]
    L.fem_plan_get_quadrature.restype = i32
    L.fem_plan_set_timing.argtypes = [P, i32]
    L.fem_plan_set_timing.restype = i32
    L.fem_plan_get_timing.argtypes = [P, P, P]
    L.fem_plan_get_timing.restype = i32
    L.fem_plan_set_strategy.argtypes = [P, i32, i32, i32, i32]
    L.fem_plan_set_strategy.restype = i32
    L.fem_plan_get_strategy.argtypes = [P, P, P, P, P]
    L.fem_plan_get_strategy.restype = i32
    L.fem_tune.argtypes = [P, P, P, P, i32, ctypes.c_char_p, P, P, i32, P, i32]
    L.fem_tune.restype = i32
    L.fem_tune_predict.argtypes = [P, i32, P, i32, P]
    L.fem_tune_predict.restype = i32
    L.fem_check_patch_layout.argtypes = [i32, i32, i32, i64, P, i64, P, P, i64, i32, P]
    L.fem_check_patch_layout.restype = i32
    L.fem_batch_create.argtypes = [ctypes.POINTER(P), i32, P, P, P]
    L.fem_batch_create.restype = i32
    L.fem_batch_set_vectors.argtypes = [P, P, P]
    L.fem_batch_set_vectors.restype = i32
    L.fem_batch_run.argtypes = [P, P, i32]
    L.fem_batch_run.restype = i32
    L.fem_batch_info.argtypes = [P, P, P, P, P]
    L.fem_batch_info.restype = i32
    L.fem_batch_destroy.argtypes = [P]
    L.fem_batch_destroy.restype = None
    L.fem_colouring.argtypes = [i64, i32, P, i64, P, P]
    L.fem_colouring.restype = i32
    L.fem_last_error.argtypes = []
    L.fem_last_error.restype = ctypes.c_char_p
    L.fem_version.argtypes = []
    L.fem_version.restype = i32
    L.fem_action_noalloc.argtypes = [P, P, P, P]
    L.fem_action_noalloc.restype = i32
    L.fem_plan_kernel_info.argtypes = [P, i32, P, P, P]
    L.fem_plan_kernel_info.restype = i32
    L.fem_stream_copy.argtypes = [P, P, i64, P]
    L.fem_stream_copy.restype = i32
    L.fem_stream_read.argtypes = [P, i64, P, i64, P]
    L.fem_stream_read.restype = i32
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        raise FemError(status, lib().fem_last_error().decode())


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def reference_tables(dim: int, degree: int, quad_degree: int, family: int = 0):
    """The library's quadrature rule and tabulation: (points, weights, phi, dphi)."""
    L = lib()
    nq, nl = ctypes.c_int(), ctypes.c_int()
    _check(L.fem_reference_tables(dim, degree, quad_degree, family, ctypes.byref(nq),
                                  ctypes.byref(nl), None, None, None, None))
    pts = np.empty((nq.value, dim))
    w = np.empty(nq.value)
    phi = np.empty((nq.value, nl.value))
    dphi = np.empty((nq.value, nl.value, dim))
    _check(L.fem_reference_tables(dim, degree, quad_degree, family, None, None, _np_ptr(pts),
                                  _np_ptr(w), _np_ptr(phi), _np_ptr(dphi)))
    return pts, w, phi, dphi


def colouring(cell_nodes, n_node: int):
    """The library's host colouring: (colour [n_cell] int32, n_colours)."""
    L = lib()
    cn = np.ascontiguousarray(cell_nodes, dtype=np.int32)
    out = np.empty(cn.shape[0], dtype=np.int32)
    nc = ctypes.c_int32()
    _check(L.fem_colouring(cn.shape[0], cn.shape[1], _np_ptr(cn), int(n_node), _np_ptr(out),
                           ctypes.byref(nc)))
    return out, nc.value


def check_patch_layout(form: int, mesh, patch_cells: int = 0) -> dict:
    """Host-only validation of the patch layout for `mesh` (raises FemError on a violation)."""
    L = lib()
    xy = np.ascontiguousarray(mesh.coords, dtype=np.float64)
    cv = np.ascontiguousarray(mesh.cell_verts, dtype=np.int32)
    cn = np.ascontiguousarray(mesh.cell_nodes, dtype=np.int32)
    st = np.zeros(8, dtype=np.int64)
    _check(L.fem_check_patch_layout(form, mesh.dim, mesh.k, xy.shape[0], _np_ptr(xy), cv.shape[0],
                                    _np_ptr(cv), _np_ptr(cn), int(mesh.n_node), patch_cells,
                                    _np_ptr(st)))
    keys = ["patch_cells", "n_patch", "max_patch_nodes", "patch_node_pairs", "shared_nodes",
            "partial_slots", "lds_bytes", "max_colours"]
    return dict(zip(keys, (int(x) for x in st)))


def _stream_handle(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _dev_ptr(t, n: int, name: str) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be contiguous with {n} entries")
    return t.data_ptr()


STREAM_SINK = 65536
NOALLOC_SCRATCH_DOUBLES = 2097152   # the static buffer behind fem_action_noalloc


def stream_copy(src, dst, stream=None):
    """dst <- src through the library's STREAM-style copy kernel (float64 CUDA tensors)."""
    n = src.numel()
    _check(lib().fem_stream_copy(_dev_ptr(src, n, "src"), _dev_ptr(dst, n, "dst"), n,
                                 _stream_handle(stream)))


def stream_read(src, sink, stream=None):
    """Read src once (a cache-evicting pass with no dirty lines); per-workgroup sums land
    in sink (a float64 CUDA tensor of at least STREAM_SINK entries)."""
    _check(lib().fem_stream_read(_dev_ptr(src, src.numel(), "src"), src.numel(),
                                 _dev_ptr(sink, sink.numel(), "sink"), sink.numel(),
                                 _stream_handle(stream)))


class Plan:
    """A mesh + form + quadrature, validated, coloured and resident on the current device."""

    def __init__(self, form: int, dim: int, degree: int, quad_degree: int, coords, cell_verts,
                 cell_nodes, n_node: int, params=(), geometry: int = 1):
        """geometry=1: ``cell_verts`` [n_cell, dim+1] vertices of affine cells (fem_plan_create);
        geometry=2: curved cells, ``coords`` the geometry nodes and ``cell_verts`` each cell's
        [n_cell, 6 or 10] P2 geometry nodes in the local lattice order (fem_plan_create_curved)."""
        L = lib()
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        cell_verts = np.ascontiguousarray(cell_verts, dtype=np.int32)
        cell_nodes = np.ascontiguousarray(cell_nodes, dtype=np.int32)
        prm = np.ascontiguousarray(params, dtype=np.float64)
        if coords.ndim != 2 or coords.shape[1] != dim:
            raise ValueError("coords must be [n_vert, dim]")
        if geometry not in (1, 2):
            raise ValueError("geometry must be 1 (affine) or 2 (P2 curved cells)")
        nv = dim + 1 if geometry == 1 else math.comb(dim + 2, dim)
        if cell_verts.ndim != 2 or cell_verts.shape[1] != nv:
            raise ValueError(f"cell geometry nodes must be [n_cell, {nv}]")
        n_loc = math.comb(degree + dim, dim) if degree >= 0 and dim >= 0 else -1
        if cell_nodes.ndim != 2 or cell_nodes.shape != (cell_verts.shape[0], n_loc):
            raise ValueError(f"cell_nodes must be [n_cell, {n_loc}] for degree {degree}")
        h = ctypes.c_void_p()
        self._h = None
        create = L.fem_plan_create if geometry == 1 else L.fem_plan_create_curved
        _check(create(ctypes.byref(h), form, dim, degree, quad_degree,
                                 coords.shape[0], _np_ptr(coords), cell_verts.shape[0],
                                 _np_ptr(cell_verts), _np_ptr(cell_nodes), int(n_node),
                                 _np_ptr(prm) if prm.size else None, int(prm.size)))
        self._h = h
        self.form, self.dim, self.degree, self.quad_degree = form, dim, degree, quad_degree
        self.geometry = geometry
        self.n_cell = cell_verts.shape[0]
        nl, nc, nq, ncol, nd = (ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int(),
                                ctypes.c_int64())
        _check(L.fem_plan_info(h, ctypes.byref(nl), ctypes.byref(nc), ctypes.byref(nq),
                               ctypes.byref(ncol), ctypes.byref(nd)))
        self.n_loc, self.ncomp, self.n_quad, self.n_colours, self.n_dof = (
            nl.value, nc.value, nq.value, ncol.value, nd.value)
        self._read_quadrature()

    def _read_quadrature(self):
        fam, nq = ctypes.c_int(), ctypes.c_int()
        _check(lib().fem_plan_get_quadrature(self.handle, ctypes.byref(fam), ctypes.byref(nq)))
        self.quad_family, self.n_quad = fam.value, nq.value

    @property
    def quad_family_name(self) -> str:
        """'symmetric' or 'conical' (the oracle's names for the two rule families)."""
        return "symmetric" if self.quad_family == QUAD_SYMMETRIC else "conical"

    @classmethod
    def from_mesh(cls, form: int, mesh, quad_degree: int, params=()):
        """A plan on a generated mesh; curved meshes (``mesh.cell_gnodes`` set) give P2 cells."""
        if getattr(mesh, "cell_gnodes", None) is not None:
            return cls(form, mesh.dim, mesh.k, quad_degree, mesh.gcoords, mesh.cell_gnodes,
                       mesh.cell_nodes, mesh.n_node, params, geometry=2)
        return cls(form, mesh.dim, mesh.k, quad_degree, mesh.coords, mesh.cell_verts,
                   mesh.cell_nodes, mesh.n_node, params)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan is closed")
        return self._h

    def kernel_info(self, vjp: bool = False) -> dict:
        """Registers, scratch bytes per lane and wave-priority flag of the main kernel the
        current configuration launches."""
        r, sc, pr = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().fem_plan_kernel_info(self.handle, int(vjp), ctypes.byref(r), ctypes.byref(sc),
                                          ctypes.byref(pr)))
        return {"registers": r.value, "scratch_bytes": sc.value, "wave_priority": bool(pr.value)}

    def close(self):
        if getattr(self, "_h", None) is not None:
            _check(lib().fem_plan_destroy(self._h))   # refused while a batch holds the plan
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_quadrature(self, family: int):
        _check(lib().fem_plan_set_quadrature(self.handle, family))
        self._read_quadrature()

    def set_block(self, cells_per_block: int):
        _check(lib().fem_plan_set_block(self.handle, cells_per_block))

    def set_strategy(self, strategy: int, patch_cells: int = 0, lanes_per_cell: int = 0,
                     sum_mode: int = 0):
        _check(lib().fem_plan_set_strategy(self.handle, strategy, patch_cells, lanes_per_cell,
                                           sum_mode))

    def set_timing(self, enable: bool = True):
        """Bracket the main kernel of every later call with HIP events (resets totals)."""
        _check(lib().fem_plan_set_timing(self.handle, int(bool(enable))))

    def timing(self):
        """(summed kernel milliseconds, bracketed calls) since timing was last switched."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().fem_plan_get_timing(self.handle, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def strategy(self):
        st, pc, ln, sm = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().fem_plan_get_strategy(self.handle, ctypes.byref(st), ctypes.byref(pc),
                                           ctypes.byref(ln), ctypes.byref(sm)))
        return st.value, pc.value, ln.value, sm.value

    def tune(self, u, y=None, v=None, cache_path: str | None = None, stream=None,
             max_timed: int = 0):
        """Time the launch configurations on (u[, v]) and keep the fastest (all of them, or
        the cost model's `max_timed` best plus the current one).

        Returns a list of (strategy, cells_per_patch, lanes_per_cell, block, sum_mode, ms)."""
        import torch
        if y is None:
            y = torch.empty_like(u)
        res = np.zeros((64, 6))
        nres = ctypes.c_int()
        vjp = v is not None
        _check(lib().fem_tune(self.handle, _dev_ptr(u, self.n_dof, "u"),
                              _dev_ptr(v, self.n_dof, "v") if vjp else None,
                              _dev_ptr(y, self.n_dof, "y"), int(vjp),
                              cache_path.encode() if cache_path else None, _stream_handle(stream),
                              _np_ptr(res), 64, ctypes.byref(nres), int(max_timed)))
        return [tuple(r) for r in res[:nres.value]]

    def tune_predict(self, vjp: bool = False):
        """The cost model's predicted ms for every tuner candidate (no launch), as rows
        (strategy, cells_per_patch, lanes_per_cell, block, sum_mode, predicted_ms)."""
        res = np.zeros((64, 6))
        nres = ctypes.c_int()
        _check(lib().fem_tune_predict(self.handle, int(vjp), _np_ptr(res), 64, ctypes.byref(nres)))
        return [tuple(r) for r in res[:nres.value]]

    def colouring(self) -> np.ndarray:
        out = np.empty(self.n_cell, dtype=np.int32)
        _check(lib().fem_plan_colouring(self.handle, _np_ptr(out)))
        return out

    def action(self, u, out=None, stream=None):
        """y = A(u) on the current stream (asynchronous)."""
        import torch
        if out is None:
            out = torch.empty_like(u)
        _check(lib().fem_action(self.handle, _dev_ptr(u, self.n_dof, "u"),
                                _dev_ptr(out, self.n_dof, "y"), _stream_handle(stream)))
        return out

    def jvp(self, u, w, out=None, stream=None):
        """(dA/du) w, the tangent action at u, on the current stream (asynchronous)."""
        import torch
        if out is None:
            out = torch.empty_like(w)
        _check(lib().fem_action_jvp(self.handle, _dev_ptr(u, self.n_dof, "u"),
                                    _dev_ptr(w, self.n_dof, "w"),
                                    _dev_ptr(out, self.n_dof, "out"), _stream_handle(stream)))
        return out

    def vjp(self, u, v, out=None, stream=None):
        """g = (dA/du)^T v on the current stream (asynchronous)."""
        import torch
        if out is None:
            out = torch.empty_like(v)
        _check(lib().fem_action_vjp(self.handle, _dev_ptr(u, self.n_dof, "u"),
                                    _dev_ptr(v, self.n_dof, "v"),
                                    _dev_ptr(out, self.n_dof, "g"), _stream_handle(stream)))
        return out


def action_once(form: int, dim: int, degree: int, quad_degree: int, coords, cell_verts,
                cell_nodes, n_node: int, params, u, out=None, stream=None):
    """y = A(u) straight from the mesh arrays (a temporary plan; synchronous, slow)."""
    import torch
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    cell_verts = np.ascontiguousarray(cell_verts, dtype=np.int32)
    cell_nodes = np.ascontiguousarray(cell_nodes, dtype=np.int32)
    prm = np.ascontiguousarray(params, dtype=np.float64)
    n = int(n_node) * (1 if form in SCALAR_FORMS else dim)
    if out is None:
        out = torch.empty_like(u)
    _check(lib().fem_action_once(form, dim, degree, quad_degree, coords.shape[0],
                                 _np_ptr(coords), cell_verts.shape[0], _np_ptr(cell_verts),
                                 _np_ptr(cell_nodes), int(n_node),
                                 _np_ptr(prm) if prm.size else None, int(prm.size),
                                 _dev_ptr(u, n, "u"), _dev_ptr(out, n, "y"),
                                 _stream_handle(stream)))
    return out


class Batch:
    """Many plans' actions in a few launches recorded into one HIP graph.

    `us` and `ys` are float64 CUDA tensors (one per plan), bound at creation; keep them
    alive (and the plans) as long as the batch."""

    def __init__(self, plans, us, ys):
        L = lib()
        n = len(plans)
        if not (len(us) == len(ys) == n) or n == 0:
            raise ValueError("need one input and one output per plan")
        self.plans, self.us, self.ys = list(plans), list(us), list(ys)
        ph = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
        up = (ctypes.c_void_p * n)(*[_dev_ptr(u, p.n_dof, "u") for u, p in zip(us, plans)])
        yp = (ctypes.c_void_p * n)(*[_dev_ptr(y, p.n_dof, "y") for y, p in zip(ys, plans)])
        h = ctypes.c_void_p()
        self._h = None
        _check(L.fem_batch_create(ctypes.byref(h), n, ph, up, yp))
        self._h = h
        nm, ng, npat, nsh = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64(), ctypes.c_int64()
        _check(L.fem_batch_info(h, ctypes.byref(nm), ctypes.byref(ng), ctypes.byref(npat),
                                ctypes.byref(nsh)))
        self.n_groups, self.n_patches, self.n_shared = ng.value, npat.value, nsh.value

    def run(self, graph: bool = True, stream=None):
        _check(lib().fem_batch_run(self._h, _stream_handle(stream), int(graph)))

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().fem_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autograd_function():
    import torch

    class _FemAction(torch.autograd.Function):
        """y = A(u); backward g = (dA/du)^T grad_y, recomputing quadrature states from u."""

        @staticmethod
        def forward(ctx, u, plan):
            ctx.plan = plan
            ctx.save_for_backward(u)
            return plan.action(u.contiguous())

        @staticmethod
        def backward(ctx, gy):
            (u,) = ctx.saved_tensors
            return ctx.plan.vjp(u.contiguous(), gy.contiguous()), None

    return _FemAction


class _LazyFemAction:
    _fn = None

    def __getattr__(self, name):
        if _LazyFemAction._fn is None:
            _LazyFemAction._fn = _autograd_function()
        return getattr(_LazyFemAction._fn, name)


FemAction = _LazyFemAction()

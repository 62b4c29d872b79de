// Plan construction and the C ABI entry points.
//
// A plan validates the mesh once, tabulates the reference element, colours the cells so
// that no two cells of one colour share a node (the scatter of the action is then free
// of write conflicts inside a colour and runs colour by colour, deterministically), and
// stores colour-sorted, structure-of-arrays copies of the maps on the device so that the
// per-cell map reads of a wavefront are contiguous.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace {
thread_local std::string g_last_error;

int fail(const femx::Error &e)
{
    g_last_error = e.what();
    return e.code;
}

template <class F>
int guarded(F &&f)
{
    try {
        f();
        g_last_error.clear();
        return FEM_OK;
    } catch (const femx::Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return FEM_E_NOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return FEM_E_ARG;
    } catch (...) {
        g_last_error = "unknown failure";
        return FEM_E_ARG;
    }
}

template <class T>
T *device_upload(const std::vector<T> &h, const char *what)
{
    T *d = nullptr;
    if (h.empty()) return nullptr;
    hipError_t e = hipMalloc((void **)&d, h.size() * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw femx::Error(e == hipErrorOutOfMemory ? FEM_E_NOMEM : FEM_E_HIP,
                          std::string("hipMalloc for ") + what + ": " + hipGetErrorString(e));
    }
    e = hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        throw femx::Error(FEM_E_HIP, std::string("hipMemcpy for ") + what + ": " +
                                          hipGetErrorString(e));
    }
    return d;
}

void free_plan_memory(fem_plan *p)
{
    if (!p) return;
    (void)hipFree(p->d_coords);
    (void)hipFree(p->d_verts);
    (void)hipFree(p->d_nodes);
    (void)hipFree(p->d_first);
    (void)hipFree(p->d_tab);
    (void)hipFree(p->d_untouched);
}

// Greedy first-fit colouring, cells in ascending id; conflict = a shared node.
int greedy_colouring(int64_t n_cell, int nloc, const int32_t *cell_nodes, int64_t n_node,
                     std::vector<int32_t> &colour)
{
    for (int nwords = 1; nwords <= 16; nwords *= 4) {
        std::vector<uint64_t> used((size_t)n_node * nwords, 0);
        colour.assign((size_t)n_cell, 0);
        int ncol = 0;
        bool overflow = false;
        std::vector<uint64_t> forbidden(nwords);
        for (int64_t c = 0; c < n_cell && !overflow; ++c) {
            std::fill(forbidden.begin(), forbidden.end(), 0);
            const int32_t *cn = cell_nodes + c * nloc;
            for (int a = 0; a < nloc; ++a)
                for (int w = 0; w < nwords; ++w) forbidden[w] |= used[(size_t)cn[a] * nwords + w];
            int col = -1;
            for (int w = 0; w < nwords; ++w)
                if (~forbidden[w]) {
                    col = 64 * w + __builtin_ctzll(~forbidden[w]);
                    break;
                }
            if (col < 0) {
                overflow = true;
                break;
            }
            colour[c] = col;
            for (int a = 0; a < nloc; ++a)
                used[(size_t)cn[a] * nwords + col / 64] |= uint64_t(1) << (col % 64);
            ncol = std::max(ncol, col + 1);
        }
        if (!overflow) return ncol;
    }
    throw femx::Error(FEM_E_UNSUPPORTED, "colouring needs more than 1024 colours");
}

// Host-side validation of the mesh; runs before any HIP call.
void validate_mesh(fem_plan *p, const double *coords, const int32_t *cell_verts,
                   const int32_t *cell_nodes, const double *params, int n_params)
{
    using femx::Error;
    const int d = p->dim, nv = d + 1, nloc = p->nloc;
    if (p->form != FEM_MASS) {
        if (n_params < 2 || !params) throw Error(FEM_E_ARG, "vector forms need params {lambda, mu}");
        p->lam = params[0];
        p->mu = params[1];
        if (!std::isfinite(p->lam) || !std::isfinite(p->mu)) throw Error(FEM_E_ARG, "non-finite params");
    }
    for (int64_t i = 0; i < p->n_vert * d; ++i)
        if (!std::isfinite(coords[i])) throw Error(FEM_E_ARG, "non-finite vertex coordinate");
    for (int64_t i = 0; i < p->n_cell * nv; ++i)
        if (cell_verts[i] < 0 || cell_verts[i] >= p->n_vert)
            throw Error(FEM_E_INDEX, "cell_verts entry " + std::to_string(i) + " out of range");
    for (int64_t i = 0; i < p->n_cell * nloc; ++i)
        if (cell_nodes[i] < 0 || cell_nodes[i] >= p->n_node)
            throw Error(FEM_E_INDEX, "cell_nodes entry " + std::to_string(i) + " out of range");
    for (int64_t c = 0; c < p->n_cell; ++c) {
        double e[3][3];
        const double *x0 = coords + (int64_t)cell_verts[c * nv] * d;
        for (int r = 0; r < d; ++r) {
            const double *xr = coords + (int64_t)cell_verts[c * nv + r + 1] * d;
            for (int i = 0; i < d; ++i) e[i][r] = xr[i] - x0[i];
        }
        double det = d == 2 ? e[0][0] * e[1][1] - e[0][1] * e[1][0]
                            : e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                                  e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                                  e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
        if (det == 0.0 || (d == 2 && det < 0.0))
            throw Error(FEM_E_INVERTED, "cell " + std::to_string(c) + " has det J = " +
                                            std::to_string(det));
    }
}

void build_plan(fem_plan *p, const double *coords, const int32_t *cell_verts,
                const int32_t *cell_nodes)
{
    const int d = p->dim, nv = d + 1, nloc = p->nloc;
    // --- reference tables
    femx::RefTables t = femx::reference_tables(d, p->degree, p->quad_degree);
    p->nq = t.nq;
    std::vector<double> tab = femx::kernel_table(p->form, t);

    // --- colouring and colour-sorted structure-of-arrays maps
    p->n_colours = p->n_cell ? greedy_colouring(p->n_cell, nloc, cell_nodes, p->n_node, p->colour) : 0;
    p->colour_off.assign(p->n_colours + 1, 0);
    for (int64_t c = 0; c < p->n_cell; ++c) p->colour_off[p->colour[c] + 1]++;
    for (int k = 0; k < p->n_colours; ++k) p->colour_off[k + 1] += p->colour_off[k];
    std::vector<int64_t> perm((size_t)p->n_cell), fill(p->colour_off.begin(), p->colour_off.end() - 1);
    for (int64_t c = 0; c < p->n_cell; ++c) perm[fill[p->colour[c]]++] = c;

    p->stride = std::max<int64_t>(64, (p->n_cell + 63) / 64 * 64);
    std::vector<int32_t> verts((size_t)nv * p->stride, 0), nodes((size_t)nloc * p->stride, 0);
    std::vector<uint64_t> first((size_t)p->stride, 0);
    std::vector<uint8_t> seen((size_t)p->n_node, 0);
    for (int64_t s = 0; s < p->n_cell; ++s) {
        const int64_t c = perm[s];
        for (int j = 0; j < nv; ++j) verts[(size_t)j * p->stride + s] = cell_verts[c * nv + j];
        uint64_t m = 0;
        for (int a = 0; a < nloc; ++a) {
            const int32_t nd = cell_nodes[c * nloc + a];
            nodes[(size_t)a * p->stride + s] = nd;
            if (!seen[nd]) {
                seen[nd] = 1;
                m |= uint64_t(1) << a;
            }
        }
        first[s] = m;
    }
    std::vector<int32_t> untouched;
    for (int64_t n = 0; n < p->n_node; ++n)
        if (!seen[n]) untouched.push_back((int32_t)n);
    p->n_untouched = (int64_t)untouched.size();

    std::vector<double> xy(coords, coords + p->n_vert * d);
    p->d_coords = device_upload(xy, "coords");
    p->d_verts = device_upload(verts, "cell_verts");
    p->d_nodes = device_upload(nodes, "cell_nodes");
    p->d_first = device_upload(first, "first-touch masks");
    p->d_tab = device_upload(tab, "tables");
    p->d_untouched = device_upload(untouched, "untouched nodes");
}

void check_plan(const fem_plan *p)
{
    if (!p) throw femx::Error(FEM_E_ARG, "null plan");
}

void run(const fem_plan *p, const double *u, const double *v, double *y, void *stream, bool vjp)
{
    using femx::Error;
    check_plan(p);
    if (p->n_dof > 0 && (!u || !y || (vjp && !v))) throw Error(FEM_E_ARG, "null vector");
    if (p->n_dof == 0) return;
    if (y == u || (vjp && y == v)) throw Error(FEM_E_ARG, "output aliases an input");
    hipStream_t s = (hipStream_t)stream;
    int dev = -1;
    femx::check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (dev != p->device) throw Error(FEM_E_ARG, "plan was built on another device");
    if (p->n_untouched > 0)
        femx::check_hip(femx::launch_zero_nodes(p->d_untouched, p->n_untouched, p->ncomp, y, s),
                        "zero untouched nodes");
    femx::LaunchArgs a{};
    a.verts = p->d_verts;
    a.nodes = p->d_nodes;
    a.first = p->d_first;
    a.coords = p->d_coords;
    a.tab = p->d_tab;
    a.stride = p->stride;
    a.nq = p->nq;
    a.lam = p->lam;
    a.mu = p->mu;
    a.y = y;
    // the linear forms are symmetric: their VJP is the action applied to v
    const bool nl_vjp = vjp && p->form == FEM_NEOHOOKEAN;
    a.u = (vjp && !nl_vjp) ? v : u;
    a.v = nl_vjp ? v : nullptr;
    for (int c = 0; c < p->n_colours; ++c) {
        a.begin = p->colour_off[c];
        a.count = p->colour_off[c + 1] - p->colour_off[c];
        if (a.count == 0) continue;
        femx::check_hip(femx::launch_action(*p, a, p->block, nl_vjp, s), "action launch");
    }
}

}  // namespace

namespace femx {
void check_hip(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(e == hipErrorOutOfMemory ? FEM_E_NOMEM : FEM_E_HIP,
                    std::string(what) + ": " + hipGetErrorString(e));
    }
}
}  // namespace femx

extern "C" {

int fem_plan_create(fem_plan **out, int form, int dim, int degree, int quad_degree,
                    int64_t n_vert, const double *coords, int64_t n_cell,
                    const int32_t *cell_verts, const int32_t *cell_nodes, int64_t n_node,
                    const double *params, int n_params)
{
    if (out) *out = nullptr;
    fem_plan *p = nullptr;
    const int st = guarded([&] {
        using femx::Error;
        if (!out) throw Error(FEM_E_ARG, "null output pointer");
        if (form < FEM_MASS || form > FEM_NEOHOOKEAN) throw Error(FEM_E_UNSUPPORTED, "unknown form");
        if (dim != 2 && dim != 3) throw Error(FEM_E_UNSUPPORTED, "dim must be 2 or 3");
        if (degree < 1 || degree > (dim == 2 ? 6 : 4) || !femx::kernel_available(form, dim, degree))
            throw Error(FEM_E_UNSUPPORTED, "degree " + std::to_string(degree) + " not built for dim " +
                                               std::to_string(dim));
        if (quad_degree < 0 || quad_degree > 20) throw Error(FEM_E_UNSUPPORTED, "quad_degree must be 0..20");
        if (n_vert < 0 || n_cell < 0 || n_node < 0) throw Error(FEM_E_ARG, "negative size");
        if (n_node > INT32_MAX || n_vert > INT32_MAX) throw Error(FEM_E_ARG, "more than 2^31 nodes");
        if ((n_vert > 0 && !coords) || (n_cell > 0 && (!cell_verts || !cell_nodes)))
            throw Error(FEM_E_ARG, "null mesh array");
        p = new fem_plan();
        p->form = form;
        p->dim = dim;
        p->degree = degree;
        p->quad_degree = quad_degree;
        p->nloc = femx::n_local(dim, degree);
        p->ncomp = form == FEM_MASS ? 1 : dim;
        p->n_vert = n_vert;
        p->n_cell = n_cell;
        p->n_node = n_node;
        p->n_dof = n_node * p->ncomp;
        validate_mesh(p, coords, cell_verts, cell_nodes, params, n_params);
        femx::check_hip(hipGetDevice(&p->device), "hipGetDevice");
        build_plan(p, coords, cell_verts, cell_nodes);
    });
    if (st != FEM_OK) {
        free_plan_memory(p);
        delete p;
        return st;
    }
    *out = p;
    return FEM_OK;
}

void fem_plan_destroy(fem_plan *plan)
{
    if (!plan) return;
    (void)hipDeviceSynchronize();
    free_plan_memory(plan);
    delete plan;
}

int fem_action(const fem_plan *plan, const double *u, double *y, void *stream)
{
    return guarded([&] { run(plan, u, nullptr, y, stream, false); });
}

int fem_action_vjp(const fem_plan *plan, const double *u, const double *v, double *g, void *stream)
{
    return guarded([&] { run(plan, u, v, g, stream, true); });
}

int fem_plan_info(const fem_plan *plan, int *n_loc, int *ncomp, int *n_quad, int *n_colours,
                  int64_t *n_dof)
{
    return guarded([&] {
        check_plan(plan);
        if (n_loc) *n_loc = plan->nloc;
        if (ncomp) *ncomp = plan->ncomp;
        if (n_quad) *n_quad = plan->nq;
        if (n_colours) *n_colours = plan->n_colours;
        if (n_dof) *n_dof = plan->n_dof;
    });
}

int fem_plan_colouring(const fem_plan *plan, int32_t *colour)
{
    return guarded([&] {
        check_plan(plan);
        if (!colour && plan->n_cell > 0) throw femx::Error(FEM_E_ARG, "null output");
        std::memcpy(colour, plan->colour.data(), plan->colour.size() * sizeof(int32_t));
    });
}

int fem_reference_tables(int dim, int degree, int quad_degree, int *n_quad, int *n_loc,
                         double *points, double *weights, double *phi, double *dphi)
{
    return guarded([&] {
        femx::RefTables t = femx::reference_tables(dim, degree, quad_degree);
        if (n_quad) *n_quad = t.nq;
        if (n_loc) *n_loc = t.nloc;
        if (!points) return;
        if (!weights || !phi || !dphi) throw femx::Error(FEM_E_ARG, "null output");
        std::memcpy(points, t.points.data(), t.points.size() * sizeof(double));
        std::memcpy(weights, t.weights.data(), t.weights.size() * sizeof(double));
        std::memcpy(phi, t.phi.data(), t.phi.size() * sizeof(double));
        std::memcpy(dphi, t.dphi.data(), t.dphi.size() * sizeof(double));
    });
}

int fem_plan_set_block(fem_plan *plan, int cells_per_block)
{
    return guarded([&] {
        check_plan(plan);
        if (cells_per_block != 0 && cells_per_block != 64 && cells_per_block != 128 &&
            cells_per_block != 256)
            throw femx::Error(FEM_E_ARG, "cells_per_block must be 0, 64, 128 or 256");
        plan->block = cells_per_block;
    });
}

int fem_colouring(int64_t n_cell, int n_loc, const int32_t *cell_nodes, int64_t n_node,
                  int32_t *colour, int32_t *n_colours)
{
    return guarded([&] {
        using femx::Error;
        if (n_cell < 0 || n_node < 0 || n_loc < 1 || n_loc > 64) throw Error(FEM_E_ARG, "bad size");
        if (n_cell > 0 && (!cell_nodes || !colour)) throw Error(FEM_E_ARG, "null array");
        for (int64_t i = 0; i < n_cell * n_loc; ++i)
            if (cell_nodes[i] < 0 || cell_nodes[i] >= n_node)
                throw Error(FEM_E_INDEX, "cell_nodes entry " + std::to_string(i) + " out of range");
        std::vector<int32_t> col;
        const int nc = n_cell ? greedy_colouring(n_cell, n_loc, cell_nodes, n_node, col) : 0;
        if (n_cell) std::memcpy(colour, col.data(), col.size() * sizeof(int32_t));
        if (n_colours) *n_colours = nc;
    });
}

const char *fem_last_error(void) { return g_last_error.c_str(); }

int fem_version(void) { return 100; }

}  // extern "C"

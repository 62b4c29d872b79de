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
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace femx {
std::string &last_error()
{
    static thread_local std::string msg;
    return msg;
}
}  // namespace femx

namespace {
#define g_last_error femx::last_error()

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

void free_patch_memory(fem_plan *p)
{
    (void)hipFree(p->d_pverts);
    (void)hipFree(p->d_lidx);
    (void)hipFree(p->d_patch_off);
    (void)hipFree(p->d_patch_nodes);
    (void)hipFree(p->d_patch_nint);
    (void)hipFree(p->d_patch_pbase);
    (void)hipFree(p->d_patch_ncol);
    (void)hipFree(p->d_colour);
    (void)hipFree(p->d_pdest);
    (void)hipFree(p->d_csr_off);
    (void)hipFree(p->d_csr_slots);
    (void)hipFree(p->d_fix_node);
    (void)hipFree(p->d_fix_off);
    (void)hipFree(p->d_partial);
    p->d_pverts = nullptr;
    p->d_lidx = nullptr;
    p->d_patch_off = p->d_patch_nodes = p->d_patch_nint = p->d_patch_pbase = p->d_csr_off = nullptr;
    p->d_patch_ncol = nullptr;
    p->d_colour = nullptr;
    p->d_pdest = nullptr;
    p->d_csr_slots = nullptr;
    p->d_fix_node = p->d_fix_off = nullptr;
    p->d_partial = nullptr;
    p->patch = 0;
}

// Wait for every recorded timing pair, add its time up and keep the events for reuse.
void drain_timing(const fem_plan *p)
{
    for (auto &ev : p->timing_pending) {
        femx::check_hip(hipEventSynchronize(ev.second), "hipEventSynchronize");
        float ms = 0.f;
        femx::check_hip(hipEventElapsedTime(&ms, ev.first, ev.second), "hipEventElapsedTime");
        p->timing_ms += ms;
        p->timing_calls += 1;
        p->timing_free.push_back(ev);
    }
    p->timing_pending.clear();
}

std::pair<hipEvent_t, hipEvent_t> timing_pair(const fem_plan *p)
{
    if (p->timing_pending.size() >= 1024) drain_timing(p);
    if (!p->timing_free.empty()) {
        auto ev = p->timing_free.back();
        p->timing_free.pop_back();
        return ev;
    }
    // timing-only events: no system-scope fence (cache write-back) when they are recorded,
    // so they read the kernel's own duration
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    femx::check_hip(hipEventCreateWithFlags(&ev.first, hipEventDisableSystemFence),
                    "hipEventCreateWithFlags");
    if (hipEventCreateWithFlags(&ev.second, hipEventDisableSystemFence) != hipSuccess) {
        (void)hipEventDestroy(ev.first);
        femx::check_hip(hipErrorOutOfMemory, "hipEventCreate");
    }
    return ev;
}

void destroy_timing_events(fem_plan *p)
{
    for (auto *v : {&p->timing_pending, &p->timing_free})
        for (auto &ev : *v) {
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
    p->timing_pending.clear();
    p->timing_free.clear();
}

void free_plan_memory(fem_plan *p)
{
    if (!p) return;
    destroy_timing_events(p);
    (void)hipFree(p->d_coords);
    (void)hipFree(p->d_verts);
    (void)hipFree(p->d_nodes);
    (void)hipFree(p->d_first);
    (void)hipFree(p->d_tab);
    (void)hipFree(p->d_mtab);
    (void)hipFree(p->d_untouched);
    free_patch_memory(p);
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

void build_patches(fem_plan *p, const double *coords, const int32_t *cell_verts,
                   const int32_t *cell_nodes, int P);
int default_patch(const fem_plan *p);
int default_lanes(const fem_plan *p);
int default_lanes_vector(const fem_plan *p);
int default_sum_mode(const fem_plan *p);

// Curved cells: det J (J = sum_g x_g (x) grad_xi phiG_g) at every point of the rule must be
// finite, nonzero and of one sign over the cell, positive in 2D.  Only the points are
// checked: they are where the action evaluates the map.
void check_curved(const fem_plan *p, const double *coords, const int32_t *cell_gnodes,
                  const femx::RefTables &g)
{
    const int d = p->dim, ng = g.nloc;
    for (int64_t c = 0; c < p->n_cell; ++c) {
        double sign0 = 0.0;
        for (int q = 0; q < g.nq; ++q) {
            double J[3][3] = {};
            for (int k = 0; k < ng; ++k) {
                const double *x = coords + (int64_t)cell_gnodes[c * ng + k] * d;
                for (int i = 0; i < d; ++i)
                    for (int r = 0; r < d; ++r) J[i][r] += x[i] * g.dphi[((size_t)q * ng + k) * d + r];
            }
            const double det = d == 2 ? J[0][0] * J[1][1] - J[0][1] * J[1][0]
                                      : J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                            J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                            J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
            if (q == 0) sign0 = det;
            if (!std::isfinite(det) || det == 0.0 || (d == 2 && det < 0.0) || det * sign0 <= 0.0)
                throw femx::Error(FEM_E_INVERTED, "curved cell " + std::to_string(c) +
                                                      " has det J = " + std::to_string(det) +
                                                      " at quadrature point " + std::to_string(q));
        }
    }
}

// the rule family a plan starts with: the fully symmetric rule (fewest points) wherever one
// is built for the degree, else the conical rule
int default_family(const fem_plan *p)
{
    return femx::has_symmetric_rule(p->dim, p->quad_degree) ? FEM_QUAD_SYMMETRIC : FEM_QUAD_CONICAL;
}

// Kernel tables of the plan's form on the rule of `family`; curved plans append the P2
// geometry gradients (and, with `check`, have det J checked at the rule's points).
std::vector<double> plan_tables(const fem_plan *p, int family, const double *coords,
                                const int32_t *cell_verts, bool check, int *nq)
{
    femx::RefTables t = femx::reference_tables(p->dim, p->degree, p->quad_degree, family);
    *nq = t.nq;
    if (p->geom == 1) return femx::kernel_table(p->form, t);
    femx::RefTables g = femx::reference_tables(p->dim, 2, p->quad_degree, family);
    if (check) check_curved(p, coords, cell_verts, g);
    return femx::kernel_table(p->form, t, &g);
}

// The matrix-core kernels' tabulation on the rule of `family` (affine cells whose kernel is
// built; empty otherwise).
std::vector<double> plan_mfma_table(const fem_plan *p, int family, int *n_tiles)
{
    *n_tiles = 0;
    if (p->geom != 1 || !femx::mfma_available(p->form, p->dim, p->degree)) return {};
    femx::RefTables t = femx::reference_tables(p->dim, p->degree, p->quad_degree, family);
    return femx::mfma_table(p->form, t, n_tiles);
}

// Host-side validation of the mesh; runs before any HIP call.
void validate_mesh(fem_plan *p, const double *coords, const int32_t *cell_verts,
                   const int32_t *cell_nodes, const double *params, int n_params)
{
    using femx::Error;
    const int d = p->dim, nv = femx::cell_geom_nodes(d, p->geom), nloc = p->nloc;
    if (!femx::scalar_form(p->form)) {
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
    // curved cells: det J varies over the cell and is checked at the points of the rule the
    // plan starts with
    if (p->geom == 2) {
        const femx::RefTables g =
            femx::reference_tables(d, 2, p->quad_degree, default_family(p));
        check_curved(p, coords, cell_verts, g);
    }
    for (int64_t c = 0; p->geom == 1 && c < p->n_cell; ++c) {
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
    const int d = p->dim, nv = femx::cell_geom_nodes(d, p->geom), nloc = p->nloc;
    // --- reference tables
    // for the linear forms on affine cells both rule families give the same operator; the
    // hyperelastic integrands (and curved cells) are not polynomial of the rule's degree,
    // and their operator depends on the rule
    p->quad_family = default_family(p);
    std::vector<double> tab = plan_tables(p, p->quad_family, coords, cell_verts, false, &p->nq);

    // --- colouring and colour-sorted structure-of-arrays maps
    p->n_colours = p->n_cell ? greedy_colouring(p->n_cell, nloc, cell_nodes, p->n_node, p->colour) : 0;
    p->colour_off.assign(p->n_colours + 1, 0);
    for (int64_t c = 0; c < p->n_cell; ++c) p->colour_off[p->colour[c] + 1]++;
    for (int k = 0; k < p->n_colours; ++k) p->colour_off[k + 1] += p->colour_off[k];
    std::vector<int64_t> perm((size_t)p->n_cell), fill(p->colour_off.begin(), p->colour_off.end() - 1);
    for (int64_t c = 0; c < p->n_cell; ++c) perm[fill[p->colour[c]]++] = c;

    p->stride = std::max<int64_t>(64, (p->n_cell + 63) / 64 * 64);
    std::vector<int32_t> verts((size_t)nv * p->stride, 0), nodes((size_t)nloc * p->stride, 0);
    const int nwf = (nloc + 63) / 64;        // first-touch words per cell
    std::vector<uint64_t> first((size_t)nwf * p->stride, 0);
    std::vector<uint8_t> seen((size_t)p->n_node, 0);
    for (int64_t s = 0; s < p->n_cell; ++s) {
        const int64_t c = perm[s];
        for (int j = 0; j < nv; ++j) verts[(size_t)j * p->stride + s] = cell_verts[c * nv + j];
        for (int a = 0; a < nloc; ++a) {
            const int32_t nd = cell_nodes[c * nloc + a];
            nodes[(size_t)a * p->stride + s] = nd;
            if (!seen[nd]) {
                seen[nd] = 1;
                first[(size_t)(a >> 6) * p->stride + s] |= uint64_t(1) << (a & 63);
            }
        }
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
    p->d_mtab = device_upload(plan_mfma_table(p, p->quad_family, &p->nqt), "matrix-core tables");
    p->d_untouched = device_upload(untouched, "untouched nodes");
    p->lanes = default_lanes(p);
    p->sum_mode = default_sum_mode(p);
    if (p->n_cell > 0) build_patches(p, coords, cell_verts, cell_nodes, default_patch(p));
    else p->strategy = femx::STRAT_COLOUR;
}


// Morton key of a cell's centroid on a 2^21 (3D) or 2^31 (2D) lattice over the bounding box.
uint64_t spread2(uint64_t v)
{
    v &= 0x7fffffffULL;
    v = (v | (v << 16)) & 0x0000ffff0000ffffULL;
    v = (v | (v << 8)) & 0x00ff00ff00ff00ffULL;
    v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0fULL;
    v = (v | (v << 2)) & 0x3333333333333333ULL;
    v = (v | (v << 1)) & 0x5555555555555555ULL;
    return v;
}

uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffULL;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

std::vector<int64_t> morton_order(const fem_plan *p, const double *coords, const int32_t *cell_verts)
{
    const int d = p->dim, nv = femx::cell_geom_nodes(d, p->geom);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < p->n_vert; ++v)
        for (int i = 0; i < d; ++i) {
            lo[i] = std::min(lo[i], coords[v * d + i]);
            hi[i] = std::max(hi[i], coords[v * d + i]);
        }
    const double levels = d == 2 ? 2147483647.0 : 2097151.0;
    std::vector<std::pair<uint64_t, int64_t>> key((size_t)p->n_cell);
    for (int64_t c = 0; c < p->n_cell; ++c) {
        uint64_t k = 0;
        for (int i = 0; i < d; ++i) {
            double x = 0.0;
            for (int j = 0; j < nv; ++j) x += coords[(int64_t)cell_verts[c * nv + j] * d + i];
            x /= nv;
            const double span = hi[i] - lo[i];
            const double t = span > 0 ? (x - lo[i]) / span : 0.0;
            const uint64_t q = (uint64_t)std::min(levels, std::max(0.0, t * levels));
            k |= d == 2 ? spread2(q) << i : spread3(q) << i;
        }
        key[c] = {k, c};
    }
    std::sort(key.begin(), key.end());
    std::vector<int64_t> order((size_t)p->n_cell);
    for (int64_t c = 0; c < p->n_cell; ++c) order[c] = key[c].second;
    return order;
}

// Patch strategy data: cells along the Morton curve cut into patches of P cells.  Per patch
// its distinct nodes -- first those no other patch holds (interior, ascending id), then the
// shared ones (ascending id) -- and per cell the patch-local index of each of its nodes.
// A shared node's sum leaves the patch as a partial.  Partial slots are node-major: the
// holders of shared node k fill slots fix_off[k] .. fix_off[k+1] in patch order, so the
// fixup kernel reads each node's partials contiguously; the patch finds the slot of its
// j-th shared node in pdest[base + j].
// Two ways to sum inside a patch:
//   element buffer: every cell vector goes to LDS and each node sums its slots (the CSR
//     lists below, in ascending (cell, local node));
//   coloured: cells are greedily coloured inside the patch (conflict = a shared node) and
//     accumulate into one LDS node buffer colour by colour, barriers in between.
struct PatchLayout {
    int P = 0, max_nodes = 0, max_colours = 0;
    int64_t n_patch = 0, stride = 0;
    std::vector<int64_t> order;
    std::vector<int32_t> pverts, patch_off, patch_nodes, patch_nint, patch_pbase, csr_off;
    std::vector<int32_t> fix_node, fix_off, pdest;
    std::vector<uint16_t> lidx, csr_slots;
    std::vector<uint8_t> colour, patch_ncol;
};

// DSatur colouring (Brelaz 1979) of the n <= 256 cells of one patch, two cells conflicting
// when they share one of the U local nodes (node(i, a): local node a of cell i): the next cell
// is the uncoloured one whose neighbours hold the most distinct colours (ties: more
// neighbours, then the earlier cell), given the smallest colour its neighbours leave free.
// Returns the number of colours, or 65 when 64 do not suffice.
template <class NodeOf>
int dsatur_colours(int n, int U, int nloc, NodeOf node, int *cols)
{
    constexpr int W = 4;                              // 256 cells as four 64-bit words
    std::vector<uint64_t> at((size_t)U * W, 0);       // cells holding each local node
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < nloc; ++a) at[(size_t)node(i, a) * W + (i >> 6)] |= uint64_t(1) << (i & 63);
    std::vector<uint64_t> adj((size_t)n * W, 0);
    std::vector<int> deg((size_t)n, 0);
    for (int i = 0; i < n; ++i) {
        uint64_t *r = &adj[(size_t)i * W];
        for (int a = 0; a < nloc; ++a)
            for (int w = 0; w < W; ++w) r[w] |= at[(size_t)node(i, a) * W + w];
        r[i >> 6] &= ~(uint64_t(1) << (i & 63));
        for (int w = 0; w < W; ++w) deg[i] += __builtin_popcountll(r[w]);
    }
    std::vector<uint64_t> sat((size_t)n, 0);          // colours held by a cell's neighbours
    for (int i = 0; i < n; ++i) cols[i] = -1;
    int ncol = 0;
    for (int step = 0; step < n; ++step) {
        int best = -1, bs = -1, bd = -1;
        for (int i = 0; i < n; ++i) {
            if (cols[i] >= 0) continue;
            const int si = __builtin_popcountll(sat[i]);
            if (si > bs || (si == bs && deg[i] > bd)) { best = i; bs = si; bd = deg[i]; }
        }
        if (sat[best] == ~uint64_t(0)) return 65;
        const int c = __builtin_ctzll(~sat[best]);
        cols[best] = c;
        ncol = std::max(ncol, c + 1);
        const uint64_t *r = &adj[(size_t)best * W];
        for (int w = 0; w < W; ++w)
            for (uint64_t m = r[w]; m; m &= m - 1) sat[(w << 6) + __builtin_ctzll(m)] |= uint64_t(1) << c;
    }
    return ncol;
}

PatchLayout make_patch_layout(const fem_plan *p, const double *coords, const int32_t *cell_verts,
                              const int32_t *cell_nodes, int P)
{
    using femx::Error;
    const int nv = femx::cell_geom_nodes(p->dim, p->geom), nloc = p->nloc;
    if (P < 1 || P > 256) throw Error(FEM_E_ARG, "patch size must be 1..256");
    if (nloc > 255) throw Error(FEM_E_UNSUPPORTED, "more than 255 nodes per cell");
    PatchLayout L;
    L.P = P;
    L.order = morton_order(p, coords, cell_verts);
    L.n_patch = (p->n_cell + P - 1) / P;
    L.stride = std::max<int64_t>(P, L.n_patch * P);
    // pass 1: how many patches hold each node
    std::vector<int32_t> node_count((size_t)p->n_node, 0);
    std::vector<int32_t> nodes;
    for (int64_t pt = 0; pt < L.n_patch; ++pt) {
        const int64_t c0 = pt * P, c1 = std::min<int64_t>(p->n_cell, c0 + P);
        nodes.clear();
        for (int64_t s = c0; s < c1; ++s)
            for (int a = 0; a < nloc; ++a) nodes.push_back(cell_nodes[L.order[s] * nloc + a]);
        std::sort(nodes.begin(), nodes.end());
        nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
        for (int32_t nd : nodes) node_count[nd]++;
    }
    // shared nodes: partial ranges in patch order
    std::vector<int32_t> fix_index((size_t)p->n_node, -1);
    L.fix_off.assign(1, 0);
    for (int64_t n = 0; n < p->n_node; ++n)
        if (node_count[n] > 1) {
            fix_index[n] = (int32_t)L.fix_node.size();
            L.fix_node.push_back((int32_t)n);
            L.fix_off.push_back(L.fix_off.back() + node_count[n]);
        }
    L.pdest.assign((size_t)L.fix_off.back(), -1);
    std::vector<int32_t> fix_fill(L.fix_node.size(), 0);

    // pass 2: per patch node order, local indices, CSR, sub-colours
    L.pverts.assign((size_t)nv * L.stride, 0);
    L.lidx.assign((size_t)nloc * L.stride, 0);
    L.colour.assign((size_t)L.stride, 0);
    L.patch_off.assign((size_t)L.n_patch + 1, 0);
    L.patch_nint.assign((size_t)L.n_patch, 0);
    L.patch_pbase.assign((size_t)L.n_patch, 0);
    L.patch_ncol.assign((size_t)L.n_patch, 0);
    L.csr_off.assign(1, 0);
    L.patch_nodes.reserve((size_t)(p->n_cell * nloc / 2 + 16));
    L.csr_slots.reserve((size_t)(p->n_cell * nloc));
    std::vector<std::pair<int64_t, int32_t>> pairs;   // ((rank*P + cl)*nloc + a, slot)
    std::vector<uint64_t> used;                        // colours held per local node
    int32_t pbase = 0;
    for (int64_t pt = 0; pt < L.n_patch; ++pt) {
        const int64_t c0 = pt * P, c1 = std::min<int64_t>(p->n_cell, c0 + P);
        nodes.clear();
        for (int64_t s = c0; s < c1; ++s)
            for (int a = 0; a < nloc; ++a) nodes.push_back(cell_nodes[L.order[s] * nloc + a]);
        std::sort(nodes.begin(), nodes.end());
        nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
        // interior nodes first, then shared, each ascending
        std::stable_partition(nodes.begin(), nodes.end(),
                              [&](int32_t nd) { return node_count[nd] == 1; });
        int nint = 0;
        while (nint < (int)nodes.size() && node_count[nodes[nint]] == 1) ++nint;
        const int U = (int)nodes.size();
        L.patch_nint[pt] = nint;
        L.patch_pbase[pt] = pbase;
        for (int j = nint; j < U; ++j) {
            const int32_t k = fix_index[nodes[j]];
            L.pdest[pbase + (j - nint)] = L.fix_off[k] + fix_fill[k]++;
        }
        pbase += U - nint;
        // local index of every (cell, a)
        auto local = [&](int32_t nd) -> int {
            // nodes is sorted within its two groups
            auto lo = node_count[nd] == 1 ? nodes.begin() : nodes.begin() + nint;
            auto hi = node_count[nd] == 1 ? nodes.begin() + nint : nodes.end();
            return (int)(std::lower_bound(lo, hi, nd) - nodes.begin());
        };
        // sub-colours: greedy first-fit over the patch's cells in Morton order, replaced by
        // DSatur's colouring of the same cells where that needs at least two colours fewer.
        // Each colour is a barrier-separated accumulation phase; on the 256-cell patches of
        // the structured tetrahedral meshes first-fit takes 26-31 colours and DSatur the 24
        // that the 24 cells around a vertex force, while a saving of one colour measured
        // neutral. The cells are then stably sorted by colour, so that the lanes of a
        // wavefront share one or two colours and skip the other colours' accumulation
        // phases (the node sums still run in colour order, so the result does not depend
        // on this permutation)
        used.assign((size_t)U, 0);
        int ncol = 0;
        int cols[256], perm[256];
        const int n_in = (int)(c1 - c0);
        bool ff_ok = true;
        for (int64_t s = c0; s < c1 && ff_ok; ++s) {
            const int64_t c = L.order[s];
            uint64_t forbid = 0;
            int lids[256];
            for (int a = 0; a < nloc; ++a) {
                lids[a] = local(cell_nodes[c * nloc + a]);
                forbid |= used[lids[a]];
            }
            if (forbid == ~uint64_t(0)) { ff_ok = false; break; }
            const int col = __builtin_ctzll(~forbid);
            cols[s - c0] = col;
            ncol = std::max(ncol, col + 1);
            for (int a = 0; a < nloc; ++a) used[lids[a]] |= uint64_t(1) << col;
        }
        {
            int dcols[256];
            const int dn = dsatur_colours(n_in, U, nloc, [&](int i, int a) {
                return local(cell_nodes[L.order[c0 + i] * nloc + a]);
            }, dcols);
            if (dn <= 64 && (!ff_ok || dn + 2 <= ncol)) {
                ncol = dn;
                for (int i = 0; i < n_in; ++i) cols[i] = dcols[i];
                ff_ok = true;
            }
        }
        if (!ff_ok) throw Error(FEM_E_UNSUPPORTED, "a patch needs more than 64 colours");
        for (int i = 0; i < n_in; ++i) perm[i] = i;
        std::stable_sort(perm, perm + n_in, [&](int x, int y) { return cols[x] < cols[y]; });
        {
            int64_t sorted[256];
            for (int i = 0; i < n_in; ++i) sorted[i] = L.order[c0 + perm[i]];
            for (int i = 0; i < n_in; ++i) L.order[c0 + i] = sorted[i];
        }
        pairs.clear();
        for (int64_t s = c0; s < c1; ++s) {
            const int64_t c = L.order[s];
            const int cl = (int)(s - c0);
            for (int j = 0; j < nv; ++j) L.pverts[(size_t)j * L.stride + s] = cell_verts[c * nv + j];
            for (int a = 0; a < nloc; ++a) {
                const int l = local(cell_nodes[c * nloc + a]);
                L.lidx[(size_t)a * L.stride + s] = (uint16_t)l;
                pairs.push_back({((int64_t)l * P + cl) * nloc + a, (a << 8) | cl});
            }
            L.colour[s] = (uint8_t)cols[perm[cl]];
        }
        L.patch_ncol[pt] = (uint8_t)ncol;
        L.max_colours = std::max(L.max_colours, ncol);
        std::sort(pairs.begin(), pairs.end());
        for (int j = 0; j < U; ++j) L.patch_nodes.push_back(nodes[j]);
        size_t k = 0;
        for (int j = 0; j < U; ++j) {
            while (k < pairs.size() && pairs[k].first / ((int64_t)P * nloc) == j) {
                L.csr_slots.push_back((uint16_t)pairs[k].second);
                ++k;
            }
            L.csr_off.push_back((int32_t)L.csr_slots.size());
        }
        L.patch_off[pt + 1] = (int32_t)L.patch_nodes.size();
        L.max_nodes = std::max(L.max_nodes, U);
    }
    return L;
}

// Check every index the patch and fixup kernels will follow, on the host: each (cell, a)
// slot is summed exactly once, into the node the map gives it; every local index points at
// its node; interior nodes are held by one patch only; every partial slot is written by
// exactly one (patch, node) and read by that node's fixup; sub-colours separate every two
// cells of a patch that share a node; all indices fall inside their buffers.  Throws on
// the first violation.
void validate_patch_layout(const fem_plan *p, const PatchLayout &L, const int32_t *cell_nodes)
{
    using femx::Error;
    const int P = L.P, nloc = p->nloc;
    auto bad = [](const std::string &m) { throw Error(FEM_E_ARG, "patch layout: " + m); };
    if ((int64_t)L.patch_off.size() != L.n_patch + 1 || L.patch_off[0] != 0) bad("patch offsets");
    if (L.csr_off.size() != L.patch_nodes.size() + 1) bad("csr offsets size");
    if ((int64_t)L.csr_slots.size() != p->n_cell * nloc) bad("slot count");
    std::vector<uint8_t> slot_seen((size_t)L.n_patch * P * nloc, 0);
    std::vector<int32_t> partial_writer((size_t)L.fix_off.back(), -1);
    std::vector<int32_t> holders((size_t)p->n_node, 0);
    for (int64_t pt = 0; pt < L.n_patch; ++pt) {
        const int nb = L.patch_off[pt], U = L.patch_off[pt + 1] - nb, nint = L.patch_nint[pt];
        if (U < 0 || U > L.max_nodes || nint < 0 || nint > U) bad("node counts");
        const int64_t c0 = pt * P, c1 = std::min<int64_t>(p->n_cell, c0 + P);
        for (int j = 0; j < U; ++j) {
            const int32_t nd = L.patch_nodes[nb + j];
            if (nd < 0 || nd >= p->n_node) bad("node id");
            holders[nd]++;
            const int e0 = L.csr_off[nb + j], e1 = L.csr_off[nb + j + 1];
            if (e0 < 0 || e1 < e0 || e1 > (int)L.csr_slots.size()) bad("csr range");
            for (int e = e0; e < e1; ++e) {
                const int sl = L.csr_slots[e], a = sl >> 8, cl = sl & 255;
                if (a >= nloc || cl >= P) bad("slot index");
                const int64_t s = c0 + cl;
                if (s >= c1) bad("slot of an absent cell");
                if (cell_nodes[L.order[s] * nloc + a] != nd) bad("slot sums into the wrong node");
                if (L.lidx[(size_t)a * L.stride + s] != j) bad("local index");
                uint8_t &seen = slot_seen[(size_t)(pt * P + cl) * nloc + a];
                if (seen) bad("slot summed twice");
                seen = 1;
            }
            if (j >= nint) {
                const int64_t e = (int64_t)L.patch_pbase[pt] + (j - nint);
                if (e >= (int64_t)L.pdest.size()) bad("partial entry range");
                const int64_t dest = L.pdest[e];
                if (dest < 0 || dest >= (int64_t)partial_writer.size()) bad("partial slot range");
                if (partial_writer[dest] >= 0) bad("partial slot written twice");
                partial_writer[dest] = nd;
            }
        }
        // sub-colours: no node twice within a colour of the patch
        std::vector<uint64_t> held((size_t)U, 0);
        for (int64_t s = c0; s < c1; ++s) {
            const int col = L.colour[s];
            if (col >= L.patch_ncol[pt]) bad("colour beyond the patch's count");
            for (int a = 0; a < nloc; ++a) {
                const int l = L.lidx[(size_t)a * L.stride + s];
                if (l >= U) bad("local index range");
                if ((held[l] >> col) & 1) bad("two cells of one colour share a node");
            }
            for (int a = 0; a < nloc; ++a) held[L.lidx[(size_t)a * L.stride + s]] |= uint64_t(1) << col;
        }
        for (int j = 0; j < nint; ++j)
            if (j > 0 && L.patch_nodes[nb + j - 1] >= L.patch_nodes[nb + j]) bad("interior order");
    }
    for (int64_t s = 0; s < p->n_cell; ++s)
        for (int a = 0; a < nloc; ++a)
            if (!slot_seen[(size_t)s * nloc + a]) bad("slot never summed");
    // every node with several holders is a fixup node whose slots are exactly its writers
    for (size_t k = 0; k < L.fix_node.size(); ++k) {
        const int32_t nd = L.fix_node[k];
        if (holders[nd] != L.fix_off[k + 1] - L.fix_off[k]) bad("fixup count");
        for (int o = L.fix_off[k]; o < L.fix_off[k + 1]; ++o)
            if (partial_writer[o] != nd) bad("fixup reads a foreign partial");
    }
    for (int32_t w : partial_writer)
        if (w < 0) bad("partial slot never written");
    for (int64_t pt = 0; pt < L.n_patch; ++pt) {
        const int nb = L.patch_off[pt];
        for (int j = 0; j < L.patch_nint[pt]; ++j)
            if (holders[L.patch_nodes[nb + j]] != 1) bad("interior node held twice");
    }
}

void build_patches(fem_plan *p, const double *coords, const int32_t *cell_verts,
                   const int32_t *cell_nodes, int P)
{
    using femx::Error;
    PatchLayout L = make_patch_layout(p, coords, cell_verts, cell_nodes, P);
    const char *chk = std::getenv("FEM_CHECK");
    if (chk && chk[0] == '1') validate_patch_layout(p, L, cell_nodes);
    // the action's need decides whether the layout is usable; the hyperelastic VJP, which
    // stages two vectors, is checked when it is called
    const size_t lds = femx::patch_lds_bytes(p->form, p->dim, p->degree, false, P, L.max_nodes,
                                             p->sum_mode);
    if (lds > 160 * 1024)
        throw Error(FEM_E_UNSUPPORTED, "patch of " + std::to_string(P) + " cells needs " +
                                           std::to_string(lds) + " bytes of LDS");
    free_patch_memory(p);
    p->patch = P;
    p->n_patch = L.n_patch;
    p->n_pn = (int64_t)L.patch_nodes.size();
    p->n_partial = L.fix_off.back();
    p->n_shared = (int64_t)L.fix_node.size();
    p->max_patch_nodes = L.max_nodes;
    p->max_colours = L.max_colours;
    p->pstride = L.stride;
    p->d_pverts = device_upload(L.pverts, "patch cell_verts");
    p->d_lidx = device_upload(L.lidx, "patch local indices");
    p->d_colour = device_upload(L.colour, "patch colours");
    p->d_patch_off = device_upload(L.patch_off, "patch offsets");
    p->d_patch_nodes = device_upload(L.patch_nodes, "patch nodes");
    p->d_patch_nint = device_upload(L.patch_nint, "patch interior counts");
    p->d_patch_pbase = device_upload(L.patch_pbase, "patch partial bases");
    p->d_patch_ncol = device_upload(L.patch_ncol, "patch colour counts");
    p->d_csr_off = device_upload(L.csr_off, "patch csr offsets");
    p->d_csr_slots = device_upload(L.csr_slots, "patch csr slots");
    p->d_fix_node = device_upload(L.fix_node, "shared nodes");
    p->d_fix_off = device_upload(L.fix_off, "shared offsets");
    p->d_pdest = device_upload(L.pdest, "partial destinations");
    if (p->n_partial > 0) {
        std::vector<double> zeros((size_t)p->n_partial * p->ncomp, 0.0);
        p->d_partial = device_upload(zeros, "partials");
    }
}

// Coloured sums everywhere: with the patch's cells sorted by colour a wavefront runs the
// adds of one or two colours only, and the smaller LDS need keeps more workgroups resident;
// measured faster than the element buffer on every 2D case and on P1/P2 tetrahedra for
// all six forms (about 24 colours there).
int default_sum_mode(const fem_plan *)
{
    return femx::SUM_COLOURED;
}

// One lane per cell in 2D up to P4: with coloured sums the lane-pair split no longer pays for its
// shuffles (measured on the P4 neo-Hookean action and VJP); lane triples in 3D from P3 on,
// where one lane's cell vector would not fit its registers.
int default_lanes(const fem_plan *p)
{
    if (p->geom == 2) {
        // curved cells: one lane, or lane triples (3D vector forms) -- for elasticity from P4,
        // where one lane spills (per 1.6e5 curved tetrahedra: 552 against 807 us), and for the
        // hyperelastic forms where one lane's tangent spills (P3, P4), so that the default
        // can take its VJP (their action is slower on triples there: neo-Hookean P3 322
        // against 246 us, St Venant-Kirchhoff P4 1068 against 984)
        if (!femx::curved_triple_available(p->form, p->dim, p->degree)) return 1;
        if (p->form == FEM_ELASTICITY) return p->degree >= 4 ? 3 : 1;
        if (femx::nonlinear_form(p->form) &&
            femx::vjp_kernel_spills(p->form, p->dim, p->degree, false, 1, femx::SUM_COLOURED, 2))
            return 3;
        return 1;
    }
    const bool mfma = femx::mfma_available(p->form, p->dim, p->degree) && p->nqt > 0;
    // the matrix-core kernel from P4 on tetrahedra, from P6 on triangles for the hyperelastic
    // forms and from P7 for elasticity, where it measured faster than the lane splits (per 2e5
    // cells: elasticity 3D P4 222 / 400 us; neo-Hookean 3D P4 392 / 874 us, its VJP 851 / 1953
    // us; neo-Hookean 2D P6 136 / 144 us, its VJP 184 / 391 us; elasticity 2D P8 346 / 716
    // us); below, the vector path wins (neo-Hookean 2D P4 110 / 104 us per 5e5 cells,
    // elasticity 2D P4 96 / 77 us, 3D P2 467 / 171 us at 1.6e6 cells).  The scalar forms
    // from P5 on tetrahedra and P7 on triangles (per 2e5 tets / 5e5 triangles, one lane
    // against matrix cores: Helmholtz 3D P5 3928 / 769 us, Laplace 3D P5 719 / 377, mass 3D
    // P6 2537 / 1031, Helmholtz 2D P8 1878 / 1205, mass 2D P7 314 / 264; one lane wins up to
    // 3D P4 and 2D P6, e.g. mass 3D P4 66 / 99 us, Laplace 2D P6 161 / 183)
    const int from2d = femx::nonlinear_form(p->form) ? 6 : 7;
    const int from3d = femx::scalar_form(p->form) ? 5 : 4;
    if (mfma && ((p->dim == 3 && p->degree >= from3d) || (p->dim == 2 && p->degree >= from2d)))
        return femx::kMfmaLanes;
    // the hyperelastic forms whose lane kernel's tangent would spill: the matrix-core kernel,
    // which holds the cell in fewer registers
    if (femx::nonlinear_form(p->form) && mfma) {
        const int l = default_lanes_vector(p);
        if (femx::vjp_kernel_spills(p->form, p->dim, p->degree, false, l, femx::SUM_COLOURED, 1))
            return femx::kMfmaLanes;
        return l;
    }
    return default_lanes_vector(p);
}

int default_lanes_vector(const fem_plan *p)
{
    if (femx::triple_available(p->form, p->dim, p->degree) && p->degree >= 3) return 3;
    // 2D vector forms from P6 on (P5 for elasticity and St Venant-Kirchhoff): a lane's half
    // of the cell (one component) fits its registers at three waves per SIMD, the whole
    // cell does not (per 5e5 cells, pairs against one lane: P6 neo-Hookean 362 / 543 us,
    // SVK 384 / 470, elasticity 298 / 317; P5 elasticity 125 / 161, SVK 180 / 196, but
    // neo-Hookean 232 / 210; from P7 one lane spills)
    if (femx::pair_available(p->form, p->dim, p->degree) &&
        (p->degree >= 6 || (p->degree == 5 && p->form != FEM_NEOHOOKEAN)))
        return 2;
    return 1;
}

// Patch sizes a lane split allows: powers of two up to 256 lanes for one or two lanes per
// cell; multiples of 21 cells (one wavefront of 21 lane triples) for three.
bool patch_allowed(int P, int lanes)
{
    if (lanes == 3) return P == 21 || P == 42 || P == 63 || P == 84;
    if (lanes == femx::kMfmaLanes) return P == 64;
    return (P == 64 || P == 128 || P == 256) && P * lanes <= 256;
}

int default_patch_for(const fem_plan *p, int lanes, int sum_mode)
{
    if (lanes == femx::kMfmaLanes) return 64;   // four wavefronts of 16 cells
    // lane triples with coloured sums: two wavefronts per patch measured best (P4 elasticity)
    if (lanes == 3 && sum_mode == femx::SUM_COLOURED) return 42;
    // the largest allowed patch whose element buffer (the larger LDS need) fits 64 KB
    static const int sizes12[] = {256, 128, 64};
    static const int sizes3[] = {84, 63, 42, 21};
    const int *sz = lanes == 3 ? sizes3 : sizes12;
    const int n = lanes == 3 ? 4 : 3;
    for (int i = 0; i < n; ++i)
        if (patch_allowed(sz[i], lanes) && (size_t)sz[i] * p->nloc * p->ncomp * 8 <= 64 * 1024)
            return sz[i];
    return sz[n - 1];
}

int default_patch(const fem_plan *p) { return default_patch_for(p, p->lanes, p->sum_mode); }

void check_plan(const fem_plan *p)
{
    if (!p) throw femx::Error(FEM_E_ARG, "null plan");
}

// A batch keeps device pointers into its plans (tables, patch arrays, partial sums) in its
// descriptors and its recorded graph: calls that replace those arrays are refused while one
// holds the plan.
void check_unbatched(const fem_plan *p)
{
    check_plan(p);
    if (p->batch_refs > 0)
        throw femx::Error(FEM_E_ARG, "the plan is held by a batch; destroy the batch first");
}

// partial: the shared nodes' partial sums (the plan's own buffer unless given); timed: the
// plan's kernel timing applies (off for the allocation-free entry point)
void run(const fem_plan *p, const double *u, const double *v, double *y, void *stream, bool vjp,
         double *partial = nullptr, bool timed = true)
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
    // the linear forms are symmetric: their VJP is the action applied to v
    const bool nl_vjp = vjp && femx::nonlinear_form(p->form);
    const double *in = (vjp && !nl_vjp) ? v : u;
    const bool colour = !(p->strategy == femx::STRAT_PATCH && p->patch > 0);
    if (nl_vjp && femx::vjp_kernel_spills(p->form, p->dim, p->degree, colour, p->lanes,
                                          p->sum_mode, p->geom))
        throw Error(FEM_E_UNSUPPORTED,
                    "the tangent kernel of this configuration spills registers to scratch memory "
                    "and is not run; use a configuration whose kernel fits its registers (the "
                    "matrix-core kernel, lanes_per_cell 4, or the lane splits)");
    if (nl_vjp && !colour) {
        const size_t need = femx::patch_lds_bytes(p->form, p->dim, p->degree, true, p->patch,
                                                  p->max_patch_nodes, p->sum_mode, p->lanes);
        if (need > 160 * 1024)
            throw Error(FEM_E_UNSUPPORTED,
                        "the tangent kernel of this configuration stages u and v and needs " +
                            std::to_string(need) + " bytes of LDS per workgroup, more than "
                            "160 KB; a smaller patch may fit");
    }
    if (p->n_untouched > 0)
        femx::check_hip(femx::launch_zero_nodes(p->d_untouched, p->n_untouched, p->ncomp, y, s),
                        "zero untouched nodes");
    if (p->strategy == femx::STRAT_PATCH && p->patch > 0) {
        femx::PatchArgs a{};
        a.verts = p->d_pverts;
        a.lidx = p->d_lidx;
        a.colour = p->d_colour;
        a.patch_off = p->d_patch_off;
        a.patch_nodes = p->d_patch_nodes;
        a.patch_nint = p->d_patch_nint;
        a.patch_pbase = p->d_patch_pbase;
        a.pdest = p->d_pdest;
        a.patch_ncol = p->d_patch_ncol;
        a.csr_off = p->d_csr_off;
        a.csr_slots = p->d_csr_slots;
        a.coords = p->d_coords;
        a.tab = p->d_tab;
        a.u = in;
        a.v = nl_vjp ? v : nullptr;
        a.y = y;
        a.partial = partial ? partial : p->d_partial;
        a.mtab = p->d_mtab;
        a.nqt = p->nqt;
        a.stride = p->pstride;
        a.n_cell = p->n_cell;
        a.nq = p->nq;
        a.lds_a = (int)femx::patch_lds_a(p->form, p->dim, p->degree, nl_vjp, p->patch,
                                         p->max_patch_nodes, p->sum_mode, p->lanes);
        a.lam = p->lam;
        a.mu = p->mu;
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        const bool timing = timed && p->timing;
        if (timing) ev = timing_pair(p);
        femx::check_hip(femx::launch_patch(*p, a, nl_vjp, s, ev.first, ev.second), "patch launch");
        if (timing) p->timing_pending.push_back(ev);
        if (p->n_shared > 0)
            femx::check_hip(femx::launch_fixup(p->d_fix_node, p->d_fix_off,
                                               p->n_shared, a.partial, p->ncomp, y, s),
                            "fixup launch");
        return;
    }
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
    a.u = in;
    a.v = nl_vjp ? v : nullptr;
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    const bool timing = timed && p->timing;
    if (timing) {
        ev = timing_pair(p);
        femx::check_hip(hipEventRecord(ev.first, s), "hipEventRecord");
    }
    for (int c = 0; c < p->n_colours; ++c) {
        a.begin = p->colour_off[c];
        a.count = p->colour_off[c + 1] - p->colour_off[c];
        if (a.count == 0) continue;
        femx::check_hip(femx::launch_action(*p, a, p->block, nl_vjp, s), "action launch");
    }
    if (timing) {
        femx::check_hip(hipEventRecord(ev.second, s), "hipEventRecord");
        p->timing_pending.push_back(ev);
    }
}

}  // namespace

namespace femx {
void set_strategy(fem_plan *plan, int strategy, int patch_cells, int lanes_per_cell, int sum_mode)
{
    check_plan(plan);
    if (strategy == FEM_SCATTER_COLOUR) {
        if (patch_cells != 0 || lanes_per_cell > 1 || sum_mode != 0)
            throw Error(FEM_E_ARG, "the colour strategy takes no patch size, lane split or sum mode");
        plan->strategy = STRAT_COLOUR;
        return;
    }
    if (strategy != FEM_SCATTER_PATCH) throw Error(FEM_E_ARG, "unknown strategy");
    if (plan->n_cell == 0) throw Error(FEM_E_ARG, "empty mesh has no patches");
    // with a patch size but no lane split: the default split if it allows that size, else one
    int lanes = lanes_per_cell;
    if (lanes == 0) {
        lanes = default_lanes(plan);
        // the matrix-core kernel sums by sub-colours only: with element sums, the lane split
        if (lanes == kMfmaLanes && sum_mode == SUM_ELEMENT) lanes = default_lanes_vector(plan);
        if (patch_cells != 0 && !patch_allowed(patch_cells, lanes)) lanes = 1;
    }
    if (lanes < 1 || lanes > kMfmaLanes)
        throw Error(FEM_E_ARG, "lanes_per_cell must be 0, 1, 2, 3 or 4");
    if (lanes == kMfmaLanes && (plan->geom != 1 || !mfma_available(plan->form, plan->dim, plan->degree)))
        throw Error(FEM_E_UNSUPPORTED,
                    "the matrix-core kernel (four lanes per cell) exists for affine cells only");
    if (lanes > 1 && plan->geom == 2 &&
        !(lanes == 3 && curved_triple_available(plan->form, plan->dim, plan->degree)))
        throw Error(FEM_E_UNSUPPORTED, "curved cells run one lane per cell, or lane triples for "
                                       "the 3D vector forms");
    if (lanes == 2 && !pair_available(plan->form, plan->dim, plan->degree))
        throw Error(FEM_E_UNSUPPORTED, "two lanes per cell exist for the 2D vector forms only");
    if (lanes == 3 && !triple_available(plan->form, plan->dim, plan->degree))
        throw Error(FEM_E_UNSUPPORTED, "three lanes per cell exist for the 3D vector forms only");
    const int mode = sum_mode == 0 ? default_sum_mode(plan) : sum_mode;
    if (mode != SUM_ELEMENT && mode != SUM_COLOURED) throw Error(FEM_E_ARG, "unknown sum mode");
    if (lanes == kMfmaLanes && mode != SUM_COLOURED)
        throw Error(FEM_E_UNSUPPORTED, "the matrix-core kernel sums by sub-colours only");
    const int P = patch_cells == 0 ? default_patch_for(plan, lanes, mode) : patch_cells;
    if (!patch_allowed(P, lanes))
        throw Error(FEM_E_ARG, "patch_cells must be 64, 128 or 256 (at most 256 lanes) for one or "
                               "two lanes per cell, 21, 42, 63 or 84 for three, and 64 for four");
    const size_t lds = patch_lds_bytes(plan->form, plan->dim, plan->degree, false, P,
                                       P == plan->patch ? plan->max_patch_nodes : 0, mode, lanes);
    if (P == plan->patch && lds > 160 * 1024)
        throw Error(FEM_E_UNSUPPORTED, "this configuration needs more than 160 KB of LDS");
    const int old_mode = plan->sum_mode;
    plan->sum_mode = mode;
    if (P != plan->patch) {
        if (plan->h_cell_verts.empty()) throw Error(FEM_E_ARG, "plan keeps no host mesh");
        check_hip(hipDeviceSynchronize(), "synchronise before rebuilding patches");
        const int old_patch = plan->patch;
        try {
            build_patches(plan, plan->h_coords.data(), plan->h_cell_verts.data(),
                          plan->h_cell_nodes.data(), P);
        } catch (...) {
            plan->sum_mode = old_mode;
            throw;
        }
        // the new layout's largest patch decides the action's LDS need of this lane split;
        // past 160 KB, back to the old layout
        const size_t need = patch_lds_bytes(plan->form, plan->dim, plan->degree, false, P,
                                            plan->max_patch_nodes, mode, lanes);
        if (need > 160 * 1024) {
            plan->sum_mode = old_mode;
            if (old_patch > 0)
                build_patches(plan, plan->h_coords.data(), plan->h_cell_verts.data(),
                              plan->h_cell_nodes.data(), old_patch);
            throw Error(FEM_E_UNSUPPORTED, "this configuration needs " + std::to_string(need) +
                                               " bytes of LDS per workgroup, more than 160 KB");
        }
    }
    plan->lanes = lanes;
    plan->strategy = STRAT_PATCH;
}

void run_action(const fem_plan *p, const double *u, const double *v, double *y, hipStream_t s,
                bool vjp)
{
    run(p, u, v, y, (void *)s, vjp);
}

void check_hip(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(e == hipErrorOutOfMemory ? FEM_E_NOMEM : FEM_E_HIP,
                    std::string(what) + ": " + hipGetErrorString(e));
    }
}
}  // namespace femx

namespace {
int create_plan(fem_plan **out, int form, int dim, int degree, int quad_degree, int geom,
                int64_t n_vert, const double *coords, int64_t n_cell, const int32_t *cell_verts,
                const int32_t *cell_nodes, int64_t n_node, const double *params, int n_params)
{
    if (out) *out = nullptr;
    fem_plan *p = nullptr;
    const int st = guarded([&] {
        using femx::Error;
        if (!out) throw Error(FEM_E_ARG, "null output pointer");
        if (form < FEM_MASS || form > FEM_HELMHOLTZ) throw Error(FEM_E_UNSUPPORTED, "unknown form");
        if (dim != 2 && dim != 3) throw Error(FEM_E_UNSUPPORTED, "dim must be 2 or 3");
        if (degree < 1 || degree > (dim == 2 ? 8 : 6) || !femx::kernel_available(form, dim, degree))
            throw Error(FEM_E_UNSUPPORTED, "degree " + std::to_string(degree) + " not built for dim " +
                                               std::to_string(dim));
        if (geom == 2 && !femx::curved_available(form, dim, degree))
            throw Error(FEM_E_UNSUPPORTED, "curved cells are built up to degree " +
                                               std::string(dim == 2 ? "6" : "4") + " in " +
                                               std::to_string(dim) + "D");
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
        p->geom = geom;
        p->nloc = femx::n_local(dim, degree);
        p->ncomp = femx::ncomp_of(form, dim);
        p->n_vert = n_vert;
        p->n_cell = n_cell;
        p->n_node = n_node;
        p->n_dof = n_node * p->ncomp;
        validate_mesh(p, coords, cell_verts, cell_nodes, params, n_params);
        p->h_coords.assign(coords, coords + n_vert * dim);
        p->h_cell_verts.assign(cell_verts, cell_verts + n_cell * femx::cell_geom_nodes(dim, geom));
        p->h_cell_nodes.assign(cell_nodes, cell_nodes + n_cell * p->nloc);
        femx::check_hip(hipGetDevice(&p->device), "hipGetDevice");
        build_plan(p, coords, cell_verts, cell_nodes);
        femx::apply_tuning_cache(p);
    });
    if (st != FEM_OK) {
        free_plan_memory(p);
        delete p;
        return st;
    }
    *out = p;
    return FEM_OK;
}
}  // namespace

extern "C" {

int fem_plan_create(fem_plan **out, int form, int dim, int degree, int quad_degree,
                    int64_t n_vert, const double *coords, int64_t n_cell,
                    const int32_t *cell_verts, const int32_t *cell_nodes, int64_t n_node,
                    const double *params, int n_params)
{
    return create_plan(out, form, dim, degree, quad_degree, 1, n_vert, coords, n_cell,
                       cell_verts, cell_nodes, n_node, params, n_params);
}

int fem_plan_create_curved(fem_plan **out, int form, int dim, int degree, int quad_degree,
                           int64_t n_gnode, const double *gcoords, int64_t n_cell,
                           const int32_t *cell_gnodes, const int32_t *cell_nodes, int64_t n_node,
                           const double *params, int n_params)
{
    return create_plan(out, form, dim, degree, quad_degree, 2, n_gnode, gcoords, n_cell,
                       cell_gnodes, cell_nodes, n_node, params, n_params);
}

int fem_plan_destroy(fem_plan *plan)
{
    if (!plan) return FEM_OK;
    if (plan->batch_refs > 0)
        return fail(femx::Error(FEM_E_ARG, "the plan is held by a batch; destroy the batch first"));
    (void)hipDeviceSynchronize();
    free_plan_memory(plan);
    delete plan;
    femx::last_error().clear();
    return FEM_OK;
}

int fem_action_jvp(const fem_plan *plan, const double *u, const double *w, double *out,
                   void *stream)
{
    // the tangent of a hyperelastic residual has major symmetry, so (dA/du) w equals
    // (dA/du)^T w and the VJP kernels compute it; the linear forms give A w
    return guarded([&] { run(plan, u, w, out, stream, true); });
}

int fem_action_once(int form, int dim, int degree, int quad_degree, int64_t n_vert,
                    const double *coords, int64_t n_cell, const int32_t *cell_verts,
                    const int32_t *cell_nodes, int64_t n_node, const double *params,
                    int n_params, const double *u, double *y, void *stream)
{
    fem_plan *p = nullptr;
    int st = fem_plan_create(&p, form, dim, degree, quad_degree, n_vert, coords, n_cell,
                             cell_verts, cell_nodes, n_node, params, n_params);
    if (st != FEM_OK) return st;
    st = guarded([&] {
        run(p, u, nullptr, y, stream, false);
        femx::check_hip(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
    });
    fem_plan_destroy(p);
    return st;
}

int fem_plan_get_quadrature(const fem_plan *plan, int *family, int *n_points)
{
    return guarded([&] {
        check_plan(plan);
        if (family) *family = plan->quad_family;
        if (n_points) *n_points = plan->nq;
    });
}

int fem_plan_set_timing(fem_plan *plan, int enable)
{
    return guarded([&] {
        check_plan(plan);
        drain_timing(plan);
        plan->timing = enable != 0;
        plan->timing_ms = 0.0;
        plan->timing_calls = 0;
    });
}

int fem_plan_get_timing(fem_plan *plan, double *kernel_ms, int64_t *calls)
{
    return guarded([&] {
        check_plan(plan);
        drain_timing(plan);
        if (kernel_ms) *kernel_ms = plan->timing_ms;
        if (calls) *calls = plan->timing_calls;
    });
}

int fem_action(const fem_plan *plan, const double *u, double *y, void *stream)
{
    return guarded([&] { run(plan, u, nullptr, y, stream, false); });
}

int fem_action_noalloc(const fem_plan *plan, const double *u, double *y, void *stream)
{
    return guarded([&] {
        check_plan(plan);
        double *partial = nullptr;
        if (plan->strategy == femx::STRAT_PATCH && plan->patch > 0 && plan->n_shared > 0) {
            int dev = -1;
            femx::check_hip(hipGetDevice(&dev), "hipGetDevice");
            if (dev != plan->device) throw femx::Error(FEM_E_ARG, "plan was built on another device");
            const size_t need = (size_t)plan->n_partial * plan->ncomp;
            if (need > (size_t)FEM_NOALLOC_SCRATCH_DOUBLES)
                throw femx::Error(FEM_E_UNSUPPORTED,
                                  "the plan's shared-node partial sums need " + std::to_string(need) +
                                      " doubles, more than the " +
                                      std::to_string((long long)FEM_NOALLOC_SCRATCH_DOUBLES) +
                                      " of the static scratch buffer");
            partial = femx::static_scratch(dev);
        }
        run(plan, u, nullptr, y, stream, false, partial, false);
    });
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

int fem_reference_tables(int dim, int degree, int quad_degree, int family, int *n_quad,
                         int *n_loc, double *points, double *weights, double *phi, double *dphi)
{
    return guarded([&] {
        femx::RefTables t = femx::reference_tables(dim, degree, quad_degree, family);
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
        if (n_cell < 0 || n_node < 0 || n_loc < 1 || n_loc > 255) throw Error(FEM_E_ARG, "bad size");
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

int fem_check_patch_layout(int form, int dim, int degree, int64_t n_vert, const double *coords,
                           int64_t n_cell, const int32_t *cell_verts, const int32_t *cell_nodes,
                           int64_t n_node, int patch_cells, int64_t *stats)
{
    return guarded([&] {
        using femx::Error;
        if (form < FEM_MASS || form > FEM_HELMHOLTZ || (dim != 2 && dim != 3) || degree < 1 ||
            degree > 8)
            throw Error(FEM_E_UNSUPPORTED, "unsupported form/dim/degree");
        if (n_vert < 0 || n_cell < 1 || n_node < 0) throw Error(FEM_E_ARG, "bad size");
        if (!coords || !cell_verts || !cell_nodes) throw Error(FEM_E_ARG, "null mesh array");
        fem_plan p;
        p.form = form;
        p.dim = dim;
        p.degree = degree;
        p.nloc = femx::n_local(dim, degree);
        p.ncomp = femx::ncomp_of(form, dim);
        p.n_vert = n_vert;
        p.n_cell = n_cell;
        p.n_node = n_node;
        const double lm[2] = {1.0, 1.0};
        validate_mesh(&p, coords, cell_verts, cell_nodes, lm, 2);
        p.lanes = default_lanes(&p);
        p.sum_mode = default_sum_mode(&p);
        const int P = patch_cells == 0 ? default_patch(&p) : patch_cells;
        PatchLayout L = make_patch_layout(&p, coords, cell_verts, cell_nodes, P);
        validate_patch_layout(&p, L, cell_nodes);
        if (stats) {
            stats[0] = L.P;
            stats[1] = L.n_patch;
            stats[2] = L.max_nodes;
            stats[3] = (int64_t)L.patch_nodes.size();
            stats[4] = (int64_t)L.fix_node.size();
            stats[5] = L.fix_off.back();
            stats[6] = (int64_t)femx::patch_lds_bytes(form, dim, degree, femx::nonlinear_form(form), P,
                                                      L.max_nodes, p.sum_mode);
            stats[7] = L.max_colours;
        }
    });
}

int fem_plan_set_quadrature(fem_plan *plan, int family)
{
    return guarded([&] {
        check_unbatched(plan);
        int nq = 0;
        std::vector<double> tab = plan_tables(plan, family, plan->h_coords.data(),
                                              plan->h_cell_verts.data(), true, &nq);
        int nqt = 0;
        std::vector<double> mtab = plan_mfma_table(plan, family, &nqt);
        double *d = device_upload(tab, "tables");
        double *dm = nullptr;
        try {
            dm = device_upload(mtab, "matrix-core tables");
        } catch (...) {
            (void)hipFree(d);
            throw;
        }
        femx::check_hip(hipDeviceSynchronize(), "synchronise before replacing tables");
        (void)hipFree(plan->d_tab);
        (void)hipFree(plan->d_mtab);
        plan->d_tab = d;
        plan->d_mtab = dm;
        plan->nq = nq;
        plan->nqt = nqt;
        plan->quad_family = family;
    });
}

int fem_plan_set_strategy(fem_plan *plan, int strategy, int patch_cells, int lanes_per_cell,
                          int sum_mode)
{
    return guarded([&] {
        check_unbatched(plan);
        femx::set_strategy(plan, strategy, patch_cells, lanes_per_cell, sum_mode);
    });
}

int fem_tune(fem_plan *plan, const double *u, const double *v, double *y, int vjp,
             const char *cache_path, void *stream, double *results, int max_results,
             int *n_results, int max_timed)
{
    return guarded([&] {
        check_unbatched(plan);
        if (plan->n_cell == 0) throw femx::Error(FEM_E_ARG, "nothing to tune on an empty mesh");
        if (!u || !y || (vjp && !v)) throw femx::Error(FEM_E_ARG, "null vector");
        if (max_results < 0 || max_timed < 0) throw femx::Error(FEM_E_ARG, "negative count");
        femx::tune(plan, u, v, y, vjp != 0, cache_path, (hipStream_t)stream, results, max_results,
                   n_results, max_timed);
    });
}

int fem_tune_predict(const fem_plan *plan, int vjp, double *results, int max_results,
                     int *n_results)
{
    return guarded([&] {
        check_plan(plan);
        if (max_results < 0) throw femx::Error(FEM_E_ARG, "negative max_results");
        femx::tune_predict(plan, vjp != 0, results, max_results, n_results);
    });
}

int fem_plan_get_strategy(const fem_plan *plan, int *strategy, int *patch_cells,
                          int *lanes_per_cell, int *sum_mode)
{
    return guarded([&] {
        check_plan(plan);
        const bool patch = plan->strategy == femx::STRAT_PATCH;
        if (strategy) *strategy = patch ? FEM_SCATTER_PATCH : FEM_SCATTER_COLOUR;
        if (patch_cells) *patch_cells = patch ? plan->patch : 0;
        if (lanes_per_cell) *lanes_per_cell = patch ? plan->lanes : 1;
        if (sum_mode) *sum_mode = patch ? plan->sum_mode : 0;
    });
}

int fem_plan_kernel_info(const fem_plan *plan, int vjp, int *regs, int *scratch_bytes,
                         int *wave_priority)
{
    return guarded([&] {
        check_plan(plan);
        const bool nl_vjp = vjp && femx::nonlinear_form(plan->form);
        const bool colour = plan->strategy == femx::STRAT_COLOUR || plan->patch == 0;
        if (!colour && femx::mass_pipe_used(*plan, nl_vjp)) {
            if (femx::mass_pipe_info(*plan, regs, scratch_bytes) != 0)
                throw femx::Error(FEM_E_HIP, "kernel attributes unavailable");
            if (wave_priority) *wave_priority = 0;
            return;
        }
        if (femx::kernel_info(plan->form, plan->dim, plan->degree, nl_vjp, colour, plan->lanes,
                              plan->sum_mode, plan->geom, regs, scratch_bytes, wave_priority) != 0)
            throw femx::Error(FEM_E_HIP, "kernel attributes unavailable");
    });
}

int fem_stream_copy(const double *src, double *dst, int64_t n, void *stream)
{
    return guarded([&] {
        if (n < 0) throw femx::Error(FEM_E_ARG, "negative length");
        if (n == 0) return;
        if (!src || !dst) throw femx::Error(FEM_E_ARG, "null buffer");
        if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15)
            throw femx::Error(FEM_E_ARG, "buffers must be 16-byte aligned");
        if (src < dst + n && dst < src + n) throw femx::Error(FEM_E_ARG, "buffers overlap");
        femx::check_hip(femx::launch_stream_copy(src, dst, n, (hipStream_t)stream), "stream copy");
    });
}

int fem_stream_read(const double *src, int64_t n, double *sink, int64_t n_sink, void *stream)
{
    return guarded([&] {
        if (n < 0) throw femx::Error(FEM_E_ARG, "negative length");
        if (!src || !sink) throw femx::Error(FEM_E_ARG, "null buffer");
        if (n_sink < femx::stream_sink_size())
            throw femx::Error(FEM_E_ARG, "the sink needs FEM_STREAM_SINK doubles");
        if (reinterpret_cast<uintptr_t>(src) & 15)
            throw femx::Error(FEM_E_ARG, "src must be 16-byte aligned");
        femx::check_hip(femx::launch_stream_read(src, n, sink, (hipStream_t)stream), "stream read");
    });
}

const char *fem_last_error(void) { return g_last_error.c_str(); }

int fem_version(void) { return 200; }

}  // extern "C"

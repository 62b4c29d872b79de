// Batched actions over many meshes: the plans are grouped by kernel variant (form,
// dimension, degree, lanes per cell, cells per patch); every group runs as one launch whose
// workgroups walk all patches of all its meshes through a device table of per-mesh
// arguments, and one more launch sums the shared nodes of every mesh.  The sequence is
// captured once into a HIP graph on a private stream and replayed on the caller's stream.
// In the graph the groups are parallel branches (they write disjoint meshes), so a
// memory-bound group's launch overlaps a compute-bound one's and each fills the others' tail;
// the fixup and the zeroing of untouched nodes join after all of them.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

struct fem_batch {
    struct Group {
        int form, dim, degree, lanes, patch, sum_mode;
        size_t lds = 0;
        int64_t n_patch = 0;
        std::vector<int> members;
        std::vector<size_t> members_lds_a;
        std::vector<femx::BatchDesc> desc;
        femx::BatchDesc *d_desc = nullptr;
        int32_t *d_patch_mesh = nullptr;
    };
    int device = 0;
    std::vector<fem_plan *> plans;
    std::vector<Group> groups;
    std::vector<femx::FixDesc> fix;
    std::vector<int> fix_member;          // plan index of each fix entry
    femx::FixDesc *d_fix = nullptr;
    int64_t n_fix = 0;
    std::vector<double *> y;              // each mesh's output vector
    hipStream_t capture = nullptr;
    std::vector<hipStream_t> branch;      // one per group after the first (graph capture)
    std::vector<hipEvent_t> branch_ev;    // fork event, then one join event per branch
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

template <class F>
int guarded(F &&f)
{
    try {
        f();
        femx::last_error().clear();
        return FEM_OK;
    } catch (const femx::Error &e) {
        femx::last_error() = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        femx::last_error() = "host allocation failed";
        return FEM_E_NOMEM;
    } catch (const std::exception &e) {
        femx::last_error() = e.what();
        return FEM_E_ARG;
    }
}

template <class T>
T *upload(const std::vector<T> &h, const char *what)
{
    T *d = nullptr;
    if (h.empty()) return nullptr;
    femx::check_hip(hipMalloc((void **)&d, h.size() * sizeof(T)), what);
    hipError_t e = hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        femx::check_hip(e, what);
    }
    return d;
}

femx::PatchArgs patch_args(const fem_plan *p, const double *u, double *y)
{
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
    a.u = u;
    a.v = nullptr;
    a.y = y;
    a.partial = p->d_partial;
    a.mtab = p->d_mtab;
    a.nqt = p->nqt;
    a.stride = p->pstride;
    a.n_cell = p->n_cell;
    a.nq = p->nq;
    a.lam = p->lam;
    a.mu = p->mu;
    return a;
}

void free_batch(fem_batch *b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    for (hipStream_t t : b->branch) (void)hipStreamDestroy(t);
    for (hipEvent_t e : b->branch_ev) (void)hipEventDestroy(e);
    for (auto &g : b->groups) {
        (void)hipFree(g.d_desc);
        (void)hipFree(g.d_patch_mesh);
    }
    (void)hipFree(b->d_fix);
}

void set_vectors(fem_batch *b, const double *const *u, double *const *y)
{
    using femx::Error;
    const int n = (int)b->plans.size();
    for (int i = 0; i < n; ++i)
        if (!u || !y || !u[i] || !y[i]) throw Error(FEM_E_ARG, "null vector for mesh " + std::to_string(i));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (y[i] == y[j] && i != j) throw Error(FEM_E_ARG, "two meshes share an output vector");
    femx::check_hip(hipDeviceSynchronize(), "synchronise before rebinding the batch");
    for (auto &g : b->groups) {
        for (size_t k = 0; k < g.members.size(); ++k) {
            g.desc[k].args.u = u[g.members[k]];
            g.desc[k].args.y = y[g.members[k]];
        }
        femx::check_hip(hipMemcpy(g.d_desc, g.desc.data(), g.desc.size() * sizeof(femx::BatchDesc),
                                  hipMemcpyHostToDevice),
                        "batch descriptors");
    }
    for (size_t k = 0; k < b->fix.size(); ++k) b->fix[k].y = y[b->fix_member[k]];
    if (!b->fix.empty())
        femx::check_hip(hipMemcpy(b->d_fix, b->fix.data(), b->fix.size() * sizeof(femx::FixDesc),
                                  hipMemcpyHostToDevice),
                        "batch fixup descriptors");
    // untouched nodes are zeroed by launches whose arguments the graph holds by value
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
    }
    b->y.assign(y, y + n);
}

void launch_group(const fem_batch::Group &g, hipStream_t s)
{
    femx::check_hip(femx::launch_batch_patch(g.form, g.dim, g.degree, g.lanes, g.patch,
                                             g.sum_mode, g.d_desc, g.d_patch_mesh, g.n_patch,
                                             g.lds, s),
                    "batched patch launch");
}

// parallel: groups after the first on the branch streams, forked from and joined back to s
// by events (used while capturing the graph, where this becomes parallel graph branches)
void enqueue(fem_batch *b, hipStream_t s, bool parallel = false)
{
    const size_t ng = b->groups.size();
    if (parallel && ng > 1) {
        femx::check_hip(hipEventRecord(b->branch_ev[0], s), "fork event");
        for (size_t i = 1; i < ng; ++i) {
            femx::check_hip(hipStreamWaitEvent(b->branch[i - 1], b->branch_ev[0], 0), "fork wait");
            launch_group(b->groups[i], b->branch[i - 1]);
            femx::check_hip(hipEventRecord(b->branch_ev[i], b->branch[i - 1]), "join event");
        }
        launch_group(b->groups[0], s);
        for (size_t i = 1; i < ng; ++i)
            femx::check_hip(hipStreamWaitEvent(s, b->branch_ev[i], 0), "join wait");
    } else {
        for (auto &g : b->groups) launch_group(g, s);
    }
    if (b->n_fix > 0)
        femx::check_hip(femx::launch_batch_fixup(b->d_fix, (int)b->fix.size(), b->n_fix, s),
                        "batched fixup launch");
    for (size_t i = 0; i < b->plans.size(); ++i) {
        const fem_plan *p = b->plans[i];
        if (p->n_untouched > 0)
            femx::check_hip(femx::launch_zero_nodes(p->d_untouched, p->n_untouched, p->ncomp,
                                                    b->y[i], s),
                            "zero untouched nodes");
    }
}

}  // namespace

extern "C" {

int fem_batch_create(fem_batch **out, int n, fem_plan *const *plans, const double *const *u,
                     double *const *y)
{
    if (out) *out = nullptr;
    fem_batch *b = nullptr;
    const int st = guarded([&] {
        using femx::Error;
        if (!out || n < 1 || !plans) throw Error(FEM_E_ARG, "need at least one plan");
        b = new fem_batch();
        femx::check_hip(hipGetDevice(&b->device), "hipGetDevice");
        for (int i = 0; i < n; ++i) {
            fem_plan *p = plans[i];
            if (!p) throw Error(FEM_E_ARG, "null plan " + std::to_string(i));
            if (p->device != b->device) throw Error(FEM_E_ARG, "plans on different devices");
            for (int j = 0; j < i; ++j)
                if (plans[j] == p) throw Error(FEM_E_ARG, "a plan appears twice in the batch");
            if (p->geom != 1)
                throw Error(FEM_E_UNSUPPORTED, "batches take plans of affine cells only");
            if (p->n_cell > 0 && !femx::batch_available(p->form, p->dim, p->degree, 1, femx::SUM_COLOURED))
                throw Error(FEM_E_UNSUPPORTED, "batch kernels are built up to P6 (2D) / P4 (3D)");
            if (p->n_cell > 0 && (p->strategy != femx::STRAT_PATCH || p->patch == 0))
                femx::set_strategy(p, FEM_SCATTER_PATCH, 0, 0, 0);
            b->plans.push_back(p);
        }
        // group by kernel variant
        std::map<std::tuple<int, int, int, int, int, int>, int> gid;
        for (int i = 0; i < n; ++i) {
            fem_plan *p = b->plans[i];
            if (p->n_cell == 0) continue;
            const auto key =
                std::make_tuple(p->form, p->dim, p->degree, p->lanes, p->patch, p->sum_mode);
            auto it = gid.find(key);
            if (it == gid.end()) {
                it = gid.emplace(key, (int)b->groups.size()).first;
                fem_batch::Group g;
                g.form = p->form;
                g.dim = p->dim;
                g.degree = p->degree;
                g.lanes = p->lanes;
                g.patch = p->patch;
                g.sum_mode = p->sum_mode;
                b->groups.push_back(g);
            }
            fem_batch::Group &g = b->groups[it->second];
            g.members.push_back(i);
            femx::BatchDesc d{};
            d.args = patch_args(p, nullptr, nullptr);
            d.first_patch = g.n_patch;
            g.desc.push_back(d);
            g.n_patch += p->n_patch;
            g.members_lds_a.push_back(femx::patch_lds_a(p->form, p->dim, p->degree, false, p->patch,
                                                        p->max_patch_nodes, p->sum_mode, p->lanes));
            if (p->n_shared > 0) {
                femx::FixDesc f{};
                f.fix_node = p->d_fix_node;
                f.fix_off = p->d_fix_off;
                f.partial = p->d_partial;
                f.first = b->n_fix;
                f.ncomp = p->ncomp;
                b->fix.push_back(f);
                b->fix_member.push_back(i);
                b->n_fix += p->n_shared * p->ncomp;   // (node, component) items
            }
        }
        for (auto &g : b->groups) {
            // every mesh of the group shares one dynamic LDS size: region A takes the
            // group's largest, region B follows it
            size_t a_max = 0;
            for (size_t v : g.members_lds_a) a_max = std::max(a_max, v);
            size_t b_max = 0;
            for (size_t k = 0; k < g.members.size(); ++k) {
                const fem_plan *p = b->plans[g.members[k]];
                const size_t bb = femx::patch_lds_bytes(p->form, p->dim, p->degree, false, p->patch,
                                                        p->max_patch_nodes, p->sum_mode, p->lanes) -
                                  8 * g.members_lds_a[k];
                b_max = std::max(b_max, bb);
                g.desc[k].args.lds_a = (int)a_max;
            }
            g.lds = 8 * a_max + b_max;
            if (g.lds > 160 * 1024)
                throw Error(FEM_E_UNSUPPORTED, "a batch group needs more than 160 KB of LDS");
            std::vector<int32_t> pm((size_t)g.n_patch);
            for (size_t k = 0; k < g.members.size(); ++k) {
                const fem_plan *p = b->plans[g.members[k]];
                std::fill(pm.begin() + g.desc[k].first_patch,
                          pm.begin() + g.desc[k].first_patch + p->n_patch, (int32_t)k);
            }
            g.d_patch_mesh = upload(pm, "batch patch map");
            g.d_desc = upload(g.desc, "batch descriptors");
        }
        b->d_fix = upload(b->fix, "batch fixup descriptors");
        femx::check_hip(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking),
                        "capture stream");
        // branch streams (default priority) and their fork / join events for the graph
        for (size_t i = 1; i < b->groups.size(); ++i) {
            hipStream_t t = nullptr;
            femx::check_hip(hipStreamCreateWithFlags(&t, hipStreamNonBlocking), "branch stream");
            b->branch.push_back(t);
        }
        for (size_t i = 0; i < b->groups.size(); ++i) {
            hipEvent_t e = nullptr;
            femx::check_hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "branch event");
            b->branch_ev.push_back(e);
        }
        set_vectors(b, u, y);
    });
    if (st != FEM_OK) {
        free_batch(b);
        delete b;
        return st;
    }
    for (fem_plan *p : b->plans) ++p->batch_refs;
    *out = b;
    return FEM_OK;
}

int fem_batch_set_vectors(fem_batch *batch, const double *const *u, double *const *y)
{
    return guarded([&] {
        if (!batch) throw femx::Error(FEM_E_ARG, "null batch");
        set_vectors(batch, u, y);
    });
}

int fem_batch_run(fem_batch *batch, void *stream, int use_graph)
{
    return guarded([&] {
        using femx::Error;
        if (!batch) throw Error(FEM_E_ARG, "null batch");
        int dev = -1;
        femx::check_hip(hipGetDevice(&dev), "hipGetDevice");
        if (dev != batch->device) throw Error(FEM_E_ARG, "batch was built on another device");
        hipStream_t s = (hipStream_t)stream;
        if (!use_graph) {
            enqueue(batch, s);
            return;
        }
        if (!batch->exec) {
            femx::check_hip(hipStreamBeginCapture(batch->capture, hipStreamCaptureModeThreadLocal),
                            "hipStreamBeginCapture");
            try {
                enqueue(batch, batch->capture, true);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(batch->capture, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            femx::check_hip(hipStreamEndCapture(batch->capture, &batch->graph), "hipStreamEndCapture");
            femx::check_hip(hipGraphInstantiate(&batch->exec, batch->graph, nullptr, nullptr, 0),
                            "hipGraphInstantiate");
        }
        femx::check_hip(hipGraphLaunch(batch->exec, s), "hipGraphLaunch");
    });
}

int fem_batch_info(const fem_batch *batch, int *n_mesh, int *n_groups, int64_t *n_patches,
                   int64_t *n_shared)
{
    return guarded([&] {
        if (!batch) throw femx::Error(FEM_E_ARG, "null batch");
        if (n_mesh) *n_mesh = (int)batch->plans.size();
        if (n_groups) *n_groups = (int)batch->groups.size();
        if (n_patches) {
            int64_t t = 0;
            for (const auto &g : batch->groups) t += g.n_patch;
            *n_patches = t;
        }
        if (n_shared) *n_shared = batch->n_fix;
    });
}

void fem_batch_destroy(fem_batch *batch)
{
    if (!batch) return;
    (void)hipDeviceSynchronize();
    for (fem_plan *p : batch->plans) --p->batch_refs;
    free_batch(batch);
    delete batch;
}

}  // extern "C"

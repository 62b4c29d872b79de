// Launchers of the matrix-free action kernels for gfx950 (CDNA4); the kernel templates
// live in kernel_templates.h and are instantiated per form in kernels_<form>.hip.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <set>

#include "kernel_templates.h"

namespace femx {
namespace {

// Shared-node sums of many meshes: thread i sums shared node i - fix[m].first of the mesh m
// whose range holds i (binary search over the meshes' first indices).
// (`first` counts (node, component) items, so meshes of different ncomp mix freely)
__global__ void batch_fixup_kernel(const FixDesc *__restrict__ fix, int n_mesh, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = n_mesh - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (fix[mid].first <= i) lo = mid; else hi = mid - 1;
    }
    const FixDesc &f = fix[lo];
    const int64_t item = i - f.first;
    const int64_t k = item / f.ncomp;
    const int c = (int)(item - k * f.ncomp);
    const int64_t nd = f.fix_node[k];
    const int o0 = f.fix_off[k], o1 = f.fix_off[k + 1];
    double s = 0.0;
    for (int o = o0; o < o1; ++o) s += f.partial[(int64_t)o * f.ncomp + c];
    f.y[nd * f.ncomp + c] = s;
}

// thread i sums component i % ncomp of shared node i / ncomp over its partials, which lie
// contiguously in node-major order (one per holding patch, in patch order)
__global__ void fixup_kernel(const int32_t *__restrict__ fix_node, const int32_t *__restrict__ fix_off,
                             int64_t n, const double *__restrict__ partial, int ncomp,
                             double *__restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * ncomp) return;
    const int64_t k = i / ncomp;
    const int c = (int)(i - k * ncomp);
    const int64_t nd = fix_node[k];
    const int o0 = fix_off[k], o1 = fix_off[k + 1];
    double s = 0.0;
    for (int o = o0; o < o1; ++o) s += partial[(int64_t)o * ncomp + c];
    y[nd * ncomp + c] = s;
}

__global__ void zero_nodes_kernel(const int32_t *__restrict__ nodes, int64_t n, int ncomp,
                                  double *__restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t nd = nodes[i];
    for (int c = 0; c < ncomp; ++c) y[nd * ncomp + c] = 0.0;
}

Kernels lookup(int form, int dim, int degree, bool vjp)
{
    switch (form) {
    case FEM_MASS: return lookup_mass(dim, degree, vjp);
    case FEM_ELASTICITY: return lookup_elasticity(dim, degree, vjp);
    case FEM_NEOHOOKEAN: return lookup_neohookean(dim, degree, vjp);
    case FEM_SVK: return lookup_svk(dim, degree, vjp);
    case FEM_LAPLACE: return lookup_laplace(dim, degree, vjp);
    case FEM_HELMHOLTZ: return lookup_helmholtz(dim, degree, vjp);
    default: return Kernels{};
    }
}

}  // namespace

bool kernel_available(int form, int dim, int degree)
{
    return lookup(form, dim, degree, false).colour != nullptr;
}

hipError_t launch_action(const fem_plan &p, const LaunchArgs &a, int block, bool vjp,
                         hipStream_t s)
{
    const Kernels ks = lookup(p.form, p.dim, p.degree, vjp);
    ColourFn fn = p.geom == 2 ? ks.colour_p2 : ks.colour;
    if (!fn) return hipErrorInvalidDeviceFunction;
    if (block <= 0) block = 64;
    if (block > kMaxBlock) return hipErrorInvalidConfiguration;
    const int64_t grid = (a.count + block - 1) / block;
    if (grid > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(block), 0, s, a);
    return hipGetLastError();
}

// LDS region A (doubles): the staged nodal values, then the element buffer (SUM_ELEMENT)
// or the node accumulator (SUM_COLOURED), which fits in the staging space.
size_t patch_lds_a(int form, int dim, int degree, bool vjp, int patch, int max_nodes, int sum_mode)
{
    const int nloc = nloc_of(dim, degree);
    const int nc = ncomp_of(form, dim);
    const size_t stage = (size_t)max_nodes * nc * (vjp ? 2 : 1);
    if (sum_mode == SUM_COLOURED) return stage;
    const size_t elem = (size_t)patch * nloc * nc;
    return stage > elem ? stage : elem;
}

// Region B (bytes): node ids, plus for the element buffer the relative sum offsets and slots.
size_t patch_lds_bytes(int form, int dim, int degree, bool vjp, int patch, int max_nodes,
                       int sum_mode)
{
    const int nloc = nloc_of(dim, degree);
    size_t b = 4 * (size_t)max_nodes;
    if (sum_mode == SUM_ELEMENT) b += 4 * ((size_t)max_nodes + 1) + 2 * (size_t)patch * nloc;
    return 8 * patch_lds_a(form, dim, degree, vjp, patch, max_nodes, sum_mode) +
           ((b + 7) & ~(size_t)7);
}

// curved (P2-geometry) and batch kernels exist up to P6 (2D) / P4 (3D)
bool curved_available(int form, int dim, int degree)
{
    return lookup(form, dim, degree, false).colour_p2 != nullptr;
}

bool batch_available(int form, int dim, int degree, int lanes, int sum_mode)
{
    if (lanes < 1 || lanes > 3 || sum_mode < 1 || sum_mode > 2) return false;
    return lookup(form, dim, degree, false).batch[lanes][sum_mode] != nullptr;
}

bool pair_available(int form, int dim, int degree)
{
    return lookup(form, dim, degree, false).patch[2][SUM_ELEMENT] != nullptr;
}

bool triple_available(int form, int dim, int degree)
{
    return lookup(form, dim, degree, false).patch[3][SUM_ELEMENT] != nullptr;
}

// Registers per lane of the kernel a launch configuration runs (the compiled kernel's
// attributes), 0 if that kernel is not built.
int kernel_registers(int form, int dim, int degree, bool vjp, bool colour, int lanes,
                     int sum_mode, int geom)
{
    const Kernels ks = lookup(form, dim, degree, vjp);
    const bool ok = lanes >= 1 && lanes <= 3 && sum_mode >= 1 && sum_mode <= 2;
    const void *fn = nullptr;
    if (geom == 2)
        fn = colour ? (const void *)ks.colour_p2
                    : (ok && lanes == 1 ? (const void *)ks.patch_p2[sum_mode] : nullptr);
    else
        fn = colour ? (const void *)ks.colour : (ok ? (const void *)ks.patch[lanes][sum_mode] : nullptr);
    if (!fn) return 0;
    hipFuncAttributes attr{};
    if (hipFuncGetAttributes(&attr, fn) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return attr.numRegs;
}

// threads of a patch workgroup: P * lanes, or 64 per 21 cells for lane triples
int patch_threads(int P, int lanes)
{
    return lanes == 3 ? 64 * ((P + 20) / 21) : P * lanes;
}

hipError_t allow_lds(const void *fn, size_t lds)
{
    if (lds <= 64 * 1024) return hipSuccess;
    static std::mutex mu;
    static std::set<const void *> raised;
    std::lock_guard<std::mutex> g(mu);
    if (raised.count(fn)) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e == hipSuccess) raised.insert(fn);
    return e;
}

hipError_t launch_batch_patch(int form, int dim, int degree, int lanes, int patch, int sum_mode,
                              const BatchDesc *desc, const int32_t *patch_mesh, int64_t n_patch,
                              size_t lds, hipStream_t s)
{
    if (lanes < 1 || lanes > 3 || (sum_mode != SUM_ELEMENT && sum_mode != SUM_COLOURED))
        return hipErrorInvalidConfiguration;
    const Kernels ks = lookup(form, dim, degree, false);
    BatchFn fn = ks.batch[lanes][sum_mode];
    if (!fn) return hipErrorInvalidDeviceFunction;
    const int threads = patch_threads(patch, lanes);
    if (patch < 1 || patch > 256 || threads > kMaxBlock || lds > 160 * 1024 || n_patch > 0x7fffffff)
        return hipErrorInvalidConfiguration;
    hipError_t e = allow_lds((const void *)fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3((unsigned)n_patch), dim3(threads), lds, s, desc, patch_mesh, patch);
    return hipGetLastError();
}

hipError_t launch_batch_fixup(const FixDesc *fix, int n_mesh, int64_t n, hipStream_t s)
{
    const int block = 256;
    const int64_t grid = (n + block - 1) / block;
    hipLaunchKernelGGL(batch_fixup_kernel, dim3((unsigned)grid), dim3(block), 0, s, fix, n_mesh, n);
    return hipGetLastError();
}

hipError_t launch_patch(const fem_plan &p, const PatchArgs &a, bool vjp, hipStream_t s,
                        hipEvent_t start, hipEvent_t stop)
{
    if (p.lanes < 1 || p.lanes > 3 || (p.sum_mode != SUM_ELEMENT && p.sum_mode != SUM_COLOURED))
        return hipErrorInvalidConfiguration;
    const Kernels ks = lookup(p.form, p.dim, p.degree, vjp);
    // curved cells run the one-lane kernels only
    PatchFn fn = p.geom == 2 ? (p.lanes == 1 ? ks.patch_p2[p.sum_mode] : nullptr)
                             : ks.patch[p.lanes][p.sum_mode];
    if (!fn) return hipErrorInvalidDeviceFunction;
    const int threads = patch_threads(p.patch, p.lanes);
    if (p.patch < 1 || p.patch > 256 || threads > kMaxBlock) return hipErrorInvalidConfiguration;
    const size_t lds = patch_lds_bytes(p.form, p.dim, p.degree, vjp, p.patch, p.max_patch_nodes,
                                       p.sum_mode);
    if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
    hipError_t e = allow_lds((const void *)fn, lds);
    if (e != hipSuccess) return e;
    if (p.n_patch > 0x7fffffff) return hipErrorInvalidConfiguration;
    if (start || stop) {
        // timed: the events are stamped by the dispatch at the kernel's own start and end
        PatchArgs args = a;
        int P = p.patch;
        void *kargs[] = {(void *)&args, (void *)&P};
        return hipExtLaunchKernel((const void *)fn, dim3((unsigned)p.n_patch), dim3(threads), kargs,
                                  lds, s, start, stop, 0);
    }
    hipLaunchKernelGGL(fn, dim3((unsigned)p.n_patch), dim3(threads), lds, s, a, p.patch);
    return hipGetLastError();
}

hipError_t launch_fixup(const int32_t *fix_node, const int32_t *fix_off, int64_t n_shared,
                        const double *partial, int ncomp, double *y, hipStream_t s)
{
    const int block = 256;
    const int64_t grid = (n_shared * ncomp + block - 1) / block;
    hipLaunchKernelGGL(fixup_kernel, dim3((unsigned)grid), dim3(block), 0, s, fix_node, fix_off,
                       n_shared, partial, ncomp, y);
    return hipGetLastError();
}

hipError_t launch_zero_nodes(const int32_t *nodes, int64_t n, int ncomp, double *y,
                             hipStream_t s)
{
    const int block = 256;
    const int64_t grid = (n + block - 1) / block;
    hipLaunchKernelGGL(zero_nodes_kernel, dim3((unsigned)grid), dim3(block), 0, s, nodes, n,
                       ncomp, y);
    return hipGetLastError();
}

}  // namespace femx

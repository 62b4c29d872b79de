// FP64 matrix-free action kernels for gfx950 (CDNA4).
//
// One lane owns one cell: the per-cell body of the paper's generic action kernel (Sec.
// 2.3) runs in registers, its tabulation operands arriving through scalar loads
// (forms.h).  Two deterministic ways to sum the cell vectors into the global vector:
//
// colour strategy: cells are greedily coloured so that no two cells of a colour share a
//   node; one launch per colour, each lane writing (first holder of a node in colour
//   order) or read-add-writing its nodes.  The colour-sorted structure-of-arrays maps
//   make every map read of a wavefront contiguous.
//
// patch strategy: cells are ordered along a Morton curve and cut into patches of P cells
//   (one workgroup each, one launch for the whole mesh).  The workgroup stages the
//   patch's distinct nodes' values in LDS, every lane reads its cell's values from there,
//   computes its cell vector, and writes it to an element buffer in the same LDS (the two
//   live ranges do not overlap).  Then each distinct node of the patch is summed by one
//   lane over its contributions in a fixed order (ascending local cell, local node) and
//   stored: straight into y when no other patch holds the node, otherwise into a partial
//   slot that a small fixup kernel adds up in patch order.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <set>

#include "forms.h"
#include "internal.h"

namespace femx {
namespace {

constexpr int kMaxBlock = 256;

template <int DIM>
__device__ __forceinline__ double gather_geometry(const int32_t *__restrict__ verts,
                                                  int64_t stride, int64_t s,
                                                  const double *__restrict__ coords,
                                                  double (&K)[DIM][DIM])
{
    double x[DIM + 1][DIM];
#pragma unroll
    for (int j = 0; j <= DIM; ++j) {
        const int64_t vj = verts[j * stride + s];
#pragma unroll
        for (int i = 0; i < DIM; ++i) x[j][i] = coords[vj * DIM + i];
    }
    return affine_geometry<DIM>(x, K);
}

// ------------------------------------------------------------------ colour strategy
template <int FORM, int DIM, int K, bool VJP>
__global__ void __launch_bounds__(kMaxBlock) colour_kernel(const LaunchArgs a)
{
    constexpr int NLOC = nloc_of(DIM, K);
    constexpr int NC = FORM == FEM_MASS ? 1 : DIM;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.count) return;
    const int64_t s = a.begin + i;
    double Kinv[DIM][DIM];
    const double adet = gather_geometry<DIM>(a.verts, a.stride, s, a.coords, Kinv);
    double ul[NLOC][NC], vl[VJP ? NLOC : 1][NC], yl[NLOC][NC];
#pragma unroll
    for (int n = 0; n < NLOC; ++n) {
        const int64_t nd = a.nodes[n * a.stride + s];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            ul[n][c] = a.u[nd * NC + c];
            if constexpr (VJP) vl[n][c] = a.v[nd * NC + c];
        }
    }
    cell_quadrature<FORM, DIM, K, VJP>(ul, vl, Kinv, adet, a.tab, a.nq, a.lam, a.mu, yl);
    const uint64_t first = a.first[s];
#pragma unroll
    for (int n = 0; n < NLOC; ++n) {
        const int64_t nd = a.nodes[n * a.stride + s];
        double *dst = a.y + nd * NC;
        if ((first >> n) & 1) {
#pragma unroll
            for (int c = 0; c < NC; ++c) dst[c] = yl[n][c];
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) dst[c] += yl[n][c];
        }
    }
}

// ------------------------------------------------------------------- patch strategy
template <int FORM, int DIM, int K, bool VJP>
__global__ void __launch_bounds__(kMaxBlock) patch_kernel(const PatchArgs a, int logp)
{
    constexpr int NLOC = nloc_of(DIM, K);
    constexpr int NC = FORM == FEM_MASS ? 1 : DIM;
    extern __shared__ double lds[];
    const int P = 1 << logp;
    const int tid = threadIdx.x;
    const int64_t p = blockIdx.x;
    const int nb = a.patch_off[p];
    const int U = a.patch_off[p + 1] - nb;

    // 1. stage the values of the patch's distinct nodes
    for (int j = tid; j < U; j += P) {
        const int64_t nd = a.patch_nodes[nb + j];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            lds[j * NC + c] = a.u[nd * NC + c];
            if constexpr (VJP) lds[(U + j) * NC + c] = a.v[nd * NC + c];
        }
    }
    __syncthreads();

    // 2. gather the cell's values from LDS and its geometry from global memory
    const int64_t s = (p << logp) + tid;
    const bool active = s < a.n_cell;
    double Kinv[DIM][DIM], adet = 0.0;
    double ul[NLOC][NC], vl[VJP ? NLOC : 1][NC], yl[NLOC][NC];
    if (active) {
        adet = gather_geometry<DIM>(a.verts, a.stride, s, a.coords, Kinv);
#pragma unroll
        for (int n = 0; n < NLOC; ++n) {
            const int l = a.lidx[n * a.stride + s];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                ul[n][c] = lds[l * NC + c];
                if constexpr (VJP) vl[n][c] = lds[(U + l) * NC + c];
            }
        }
    }
    __syncthreads();   // the staged values are dead from here on; LDS becomes the element buffer

    // 3. the cell's quadrature loop; its vector goes to the element buffer
    if (active) {
        cell_quadrature<FORM, DIM, K, VJP>(ul, vl, Kinv, adet, a.tab, a.nq, a.lam, a.mu, yl);
#pragma unroll
        for (int n = 0; n < NLOC; ++n)
#pragma unroll
            for (int c = 0; c < NC; ++c) lds[(n * NC + c) * P + tid] = yl[n][c];
    }
    __syncthreads();

    // 4. each distinct node summed by one lane in a fixed order
    for (int j = tid; j < U; j += P) {
        const int e0 = a.csr_off[nb + j], e1 = a.csr_off[nb + j + 1];
        double sum[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) sum[c] = 0.0;
        for (int e = e0; e < e1; ++e) {
            const int sl = a.csr_slots[e];
            const int an = sl >> logp, cl = sl & (P - 1);
#pragma unroll
            for (int c = 0; c < NC; ++c) sum[c] += lds[(an * NC + c) * P + cl];
        }
        const int dest = a.patch_dest[nb + j];
        if (dest < 0) {
            const int64_t nd = a.patch_nodes[nb + j];
#pragma unroll
            for (int c = 0; c < NC; ++c) a.y[nd * NC + c] = sum[c];
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) a.partial[(int64_t)dest * NC + c] = sum[c];
        }
    }
}

__global__ void fixup_kernel(const int32_t *__restrict__ fix_node, const int32_t *__restrict__ fix_off,
                             int64_t n, const double *__restrict__ partial, int ncomp,
                             double *__restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t nd = fix_node[i];
    const int o0 = fix_off[i], o1 = fix_off[i + 1];
    for (int c = 0; c < ncomp; ++c) {
        double s = 0.0;
        for (int o = o0; o < o1; ++o) s += partial[(int64_t)o * ncomp + c];
        y[nd * ncomp + c] = s;
    }
}

__global__ void zero_nodes_kernel(const int32_t *__restrict__ nodes, int64_t n, int ncomp,
                                  double *__restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t nd = nodes[i];
    for (int c = 0; c < ncomp; ++c) y[nd * ncomp + c] = 0.0;
}

// ----------------------------------------------------------------------- dispatch
using ColourFn = void (*)(const LaunchArgs);
using PatchFn = void (*)(const PatchArgs, int);

struct Kernels {
    ColourFn colour;
    PatchFn patch;
};

template <int FORM, int DIM, int K, bool VJP>
Kernels entry()
{
    return {colour_kernel<FORM, DIM, K, VJP>, patch_kernel<FORM, DIM, K, VJP>};
}

template <int DIM, int K>
Kernels pick(int form, bool vjp)
{
    if (form == FEM_MASS) return entry<FEM_MASS, DIM, K, false>();
    if (form == FEM_ELASTICITY) return entry<FEM_ELASTICITY, DIM, K, false>();
    if (vjp) return entry<FEM_NEOHOOKEAN, DIM, K, true>();
    return entry<FEM_NEOHOOKEAN, DIM, K, false>();
}

Kernels lookup(int form, int dim, int degree, bool vjp)
{
    if (form < FEM_MASS || form > FEM_NEOHOOKEAN) return {nullptr, nullptr};
    if (dim == 2) {
        switch (degree) {
        case 1: return pick<2, 1>(form, vjp);
        case 2: return pick<2, 2>(form, vjp);
        case 3: return pick<2, 3>(form, vjp);
        case 4: return pick<2, 4>(form, vjp);
        case 5: return pick<2, 5>(form, vjp);
        case 6: return pick<2, 6>(form, vjp);
        default: break;
        }
    } else if (dim == 3) {
        switch (degree) {
        case 1: return pick<3, 1>(form, vjp);
        case 2: return pick<3, 2>(form, vjp);
        case 3: return pick<3, 3>(form, vjp);
        case 4: return pick<3, 4>(form, vjp);
        default: break;
        }
    }
    return {nullptr, nullptr};
}

int log2_exact(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return (1 << l) == v ? l : -1;
}

}  // namespace

bool kernel_available(int form, int dim, int degree)
{
    return lookup(form, dim, degree, false).colour != nullptr;
}

hipError_t launch_action(const fem_plan &p, const LaunchArgs &a, int block, bool vjp,
                         hipStream_t s)
{
    ColourFn fn = lookup(p.form, p.dim, p.degree, vjp).colour;
    if (!fn) return hipErrorInvalidDeviceFunction;
    if (block <= 0) block = 64;
    if (block > kMaxBlock) return hipErrorInvalidConfiguration;
    const int64_t grid = (a.count + block - 1) / block;
    if (grid > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(block), 0, s, a);
    return hipGetLastError();
}

size_t patch_lds_bytes(int form, int dim, int degree, bool vjp, int patch, int max_nodes)
{
    const int nloc = nloc_of(dim, degree);
    const int nc = form == FEM_MASS ? 1 : dim;
    const size_t stage = (size_t)max_nodes * nc * (vjp ? 2 : 1);
    const size_t elem = (size_t)patch * nloc * nc;
    return 8 * (stage > elem ? stage : elem);
}

hipError_t launch_patch(const fem_plan &p, const PatchArgs &a, bool vjp, hipStream_t s)
{
    PatchFn fn = lookup(p.form, p.dim, p.degree, vjp).patch;
    if (!fn) return hipErrorInvalidDeviceFunction;
    const int logp = log2_exact(p.patch);
    if (logp < 0 || p.patch > kMaxBlock) return hipErrorInvalidConfiguration;
    const size_t lds = patch_lds_bytes(p.form, p.dim, p.degree, vjp, p.patch, p.max_patch_nodes);
    if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
    if (lds > 64 * 1024) {
        static std::mutex mu;
        static std::set<const void *> raised;
        std::lock_guard<std::mutex> g(mu);
        if (!raised.count((const void *)fn)) {
            hipError_t e = hipFuncSetAttribute((const void *)fn,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               160 * 1024);
            if (e != hipSuccess) return e;
            raised.insert((const void *)fn);
        }
    }
    if (p.n_patch > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(fn, dim3((unsigned)p.n_patch), dim3(p.patch), lds, s, a, logp);
    return hipGetLastError();
}

hipError_t launch_fixup(const int32_t *fix_node, const int32_t *fix_off, int64_t n_shared,
                        const double *partial, int ncomp, double *y, hipStream_t s)
{
    const int block = 256;
    const int64_t grid = (n_shared + block - 1) / block;
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

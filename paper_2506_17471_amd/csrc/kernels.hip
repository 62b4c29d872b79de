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

// Waves per SIMD the register allocator is asked to leave room for (occupancy target):
// the lane-pair kernels and the one-lane low-degree 2D kernels fit without spilling in
// the loop; everything else keeps the allocator's default.
constexpr int waves_target(int form, int dim, int k, bool vjp, int lpc)
{
    if (lpc == 3) return 1;
    if (lpc == 2) return vjp ? (k <= 4 ? 3 : 1) : 4;
    return (!vjp && dim == 2 && k <= 4 && form != FEM_MASS) ? 3 : 1;
}

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
// Stage the patch's node ids (region B) and nodal values (region A) in LDS.  Each thread
// takes B nodes per round and issues all their id loads, then all their value loads,
// before the first wait: a few memory round trips per workgroup instead of one per node a
// thread stages.  Indices past the end are clamped to the last node (U >= 1 for every
// patch), so the loads need no branches; only the LDS stores are guarded.  B = 8, or 4
// for the mass form, whose patches hold about 2.5 nodes per lane and whose occupancy is
// set by registers.

template <int NC, bool VJP, int B>
__device__ __forceinline__ void stage_nodes(const PatchArgs &a, int nb, int U, int tid,
                                            int nthreads, double *lds, int32_t *b_node)
{
    for (int j0 = tid; j0 < U; j0 += B * nthreads) {
        int32_t nd[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int j = min(j0 + b * nthreads, U - 1);
            nd[b] = a.patch_nodes[nb + j];
        }
        double uv[B][NC], vv[VJP ? B : 1][NC];
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                uv[b][c] = a.u[(int64_t)nd[b] * NC + c];
                if constexpr (VJP) vv[b][c] = a.v[(int64_t)nd[b] * NC + c];
            }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int j = j0 + b * nthreads;
            if (j < U) {
                b_node[j] = nd[b];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    lds[j * NC + c] = uv[b][c];
                    if constexpr (VJP) lds[(U + j) * NC + c] = vv[b][c];
                }
            }
        }
    }
}

// Copy n consecutive elements from global memory to LDS, kStageBatch loads in flight per
// thread (indices clamped as in stage_nodes; n >= 1).
constexpr int kStageBatch = 8;

template <typename T>
__device__ __forceinline__ void stage_copy(const T *__restrict__ src, int n, int tid,
                                           int nthreads, T *dst)
{
    for (int j0 = tid; j0 < n; j0 += kStageBatch * nthreads) {
        T val[kStageBatch];
#pragma unroll
        for (int b = 0; b < kStageBatch; ++b) val[b] = src[min(j0 + b * nthreads, n - 1)];
#pragma unroll
        for (int b = 0; b < kStageBatch; ++b) {
            const int j = j0 + b * nthreads;
            if (j < n) dst[j] = val[b];
        }
    }
}

// LPC lanes per cell: 1; 2 for the 2D vector forms (lane c of a pair owns component c);
// 3 for the 3D vector forms (lane c of a triple owns component c; a wavefront holds 21
// triples and leaves its last lane idle).  SUM: SUM_ELEMENT (LDS element buffer and fixed-
// order node sums) or SUM_COLOURED (sub-colour phases accumulating into an LDS node buffer).
template <int FORM, int DIM, int K, bool VJP, int LPC, int SUM>
__device__ __forceinline__ void patch_body(const PatchArgs &a, int64_t p, int P)
{
    constexpr int NLOC = nloc_of(DIM, K);
    constexpr int NC = FORM == FEM_MASS ? 1 : DIM;
    static_assert(LPC == 1 || (LPC == 2 && DIM == 2 && FORM != FEM_MASS) ||
                      (LPC == 3 && DIM == 3 && FORM != FEM_MASS),
                  "lane split");
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int nthreads = blockDim.x;
    int cl, comp, base = 0;                   // local cell, component, first lane of the triple
    if constexpr (LPC == 1) {
        cl = tid;
        comp = 0;
    } else if constexpr (LPC == 2) {
        cl = tid >> 1;
        comp = tid & 1;
    } else {
        const int lane = tid & 63, wave = tid >> 6;
        cl = lane < 63 ? wave * 21 + lane / 3 : P;    // the idle lane owns no cell
        comp = lane < 63 ? lane % 3 : 0;
        base = lane < 63 ? lane - comp : 0;
    }
    const int nb = a.patch_off[p];
    const int U = a.patch_off[p + 1] - nb;
    const int nint = a.patch_nint[p];
    const int pbase = a.patch_pbase[p];

    // 1. the cell's own loads (geometry, local node indices) go out first, then the patch's
    //    distinct nodal values are staged in LDS (region A) and its node ids (and, for the
    //    element buffer, its sum lists) in region B
    const int64_t s = p * P + cl;
    const bool active = cl < P && s < a.n_cell;
    constexpr int CW = LPC == 1 ? NC : 1;     // components a lane holds
    double Kinv[DIM][DIM], adet = 0.0;
    int lid[NLOC];
    if (active) {
        adet = gather_geometry<DIM>(a.verts, a.stride, s, a.coords, Kinv);
#pragma unroll
        for (int n = 0; n < NLOC; ++n) lid[n] = a.lidx[n * a.stride + s];
    }
    int32_t *b_node = reinterpret_cast<int32_t *>(lds + a.lds_a);
    int32_t *b_off = b_node + U;              // element buffer only
    uint16_t *b_slot = reinterpret_cast<uint16_t *>(b_off + U + 1);
    int e_base = 0;
    if constexpr (SUM == SUM_ELEMENT) {
        // slot lists: b_off holds global CSR offsets, rebased by e_base when read
        e_base = a.csr_off[nb];
        const int n_slots = a.csr_off[nb + U] - e_base;
        stage_copy(a.csr_off + nb, U + 1, tid, nthreads, b_off);
        stage_copy(a.csr_slots + e_base, n_slots, tid, nthreads, b_slot);
    }
    stage_nodes<NC, VJP, FORM == FEM_MASS ? 4 : 8>(a, nb, U, tid, nthreads, lds, b_node);
    __syncthreads();

    // 2. the cell's values from LDS
    double ul[NLOC][CW], vl[VJP ? NLOC : 1][CW], yl[NLOC][CW];
    if (active) {
#pragma unroll
        for (int n = 0; n < NLOC; ++n) {
            const int l = lid[n];
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                ul[n][c] = lds[l * NC + c + comp];
                if constexpr (VJP) vl[n][c] = lds[(U + l) * NC + c + comp];
            }
        }
    }
    __syncthreads();   // the staged values are dead from here on; region A is reused

    if constexpr (SUM == SUM_COLOURED) {
        for (int j = tid; j < U * NC; j += nthreads) lds[j] = 0.0;   // the node accumulator
    }

    // 3. the cell's quadrature loop
    if (active) {
        if constexpr (LPC == 1) {
            cell_quadrature<FORM, DIM, K, VJP>(ul, vl, Kinv, adet, a.tab, a.nq, a.lam, a.mu, yl);
        } else if constexpr (LPC == 3) {
            double u1[NLOC], v1[VJP ? NLOC : 1], y1[NLOC];
#pragma unroll
            for (int n = 0; n < NLOC; ++n) {
                u1[n] = ul[n][0];
                if constexpr (VJP) v1[n] = vl[n][0];
            }
            cell_quadrature_triple<FORM, K, VJP>(u1, v1, comp, base, Kinv, adet, a.tab, a.nq,
                                                 a.lam, a.mu, y1);
#pragma unroll
            for (int n = 0; n < NLOC; ++n) yl[n][0] = y1[n];
        } else {
            double u1[NLOC], v1[VJP ? NLOC : 1], y1[NLOC];
#pragma unroll
            for (int n = 0; n < NLOC; ++n) {
                u1[n] = ul[n][0];
                if constexpr (VJP) v1[n] = vl[n][0];
            }
            cell_quadrature_pair<FORM, K, VJP>(u1, v1, comp, Kinv, adet, a.tab, a.nq, a.lam, a.mu,
                                               y1);
#pragma unroll
            for (int n = 0; n < NLOC; ++n) yl[n][0] = y1[n];
        }
    }

    // 4. sum the cell vectors into the patch's nodes
    if constexpr (SUM == SUM_ELEMENT) {
        if (active) {
#pragma unroll
            for (int n = 0; n < NLOC; ++n)
#pragma unroll
                for (int c = 0; c < CW; ++c) lds[(n * NC + c + comp) * P + cl] = yl[n][c];
        }
        __syncthreads();
    } else {
        // reloaded after the barriers rather than kept live through the quadrature loop
        const int col = active ? a.colour[s] : -1;
        int lid2[NLOC];
        if (active) {
#pragma unroll
            for (int n = 0; n < NLOC; ++n) lid2[n] = a.lidx[n * a.stride + s];
        }
        const int ncol = a.patch_ncol[p];
        __syncthreads();                      // the accumulator is zero everywhere
        // no two cells of a colour share a node, so within a phase each address has one
        // writer: the LDS atomic add (no return) is only a read-modify-write without the
        // round trip, and the sum order stays fixed (colour order)
        for (int k = 0; k < ncol; ++k) {
            if (col == k) {
#pragma unroll
                for (int n = 0; n < NLOC; ++n)
#pragma unroll
                    for (int c = 0; c < CW; ++c)
                        __hip_atomic_fetch_add(&lds[lid2[n] * NC + c + comp], yl[n][c],
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            __syncthreads();
        }
    }

    // 5. each distinct node stored once: interior nodes into y, shared ones as partials
    for (int j = tid; j < U; j += nthreads) {
        double sum[NC];
        if constexpr (SUM == SUM_ELEMENT) {
            const int e0 = b_off[j] - e_base, e1 = b_off[j + 1] - e_base;
#pragma unroll
            for (int c = 0; c < NC; ++c) sum[c] = 0.0;
            for (int e = e0; e < e1; ++e) {
                const int sl = b_slot[e];
                const int an = sl >> 8, sc = sl & 255;
#pragma unroll
                for (int c = 0; c < NC; ++c) sum[c] += lds[(an * NC + c) * P + sc];
            }
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) sum[c] = lds[j * NC + c];
        }
        if (j < nint) {
            const int64_t nd = b_node[j];
#pragma unroll
            for (int c = 0; c < NC; ++c) a.y[nd * NC + c] = sum[c];
        } else {
            const int64_t dest = a.pdest[pbase + (j - nint)];
#pragma unroll
            for (int c = 0; c < NC; ++c) a.partial[dest * NC + c] = sum[c];
        }
    }
}

// The dispatcher deals workgroups to the 8 XCDs in turn (workgroup b to XCD b mod 8), and
// each XCD has its own L2.  Renumbering so that XCD x works through one contiguous run of
// the n patches -- runs of n/8 patches, the first n mod 8 runs one longer -- keeps Morton
// neighbours, which share nodes and vertices, in one L2.  A bijection of [0, n) whatever
// the dispatch order, so only locality depends on the dealing rule.
constexpr int kXcds = 8;

__device__ __forceinline__ int64_t xcd_order(int64_t b, int64_t n)
{
    const int64_t q = n / kXcds, r = n % kXcds;
    const int64_t x = b % kXcds, i = b / kXcds;
    return x * q + (x < r ? x : r) + i;
}

template <int FORM, int DIM, int K, bool VJP, int LPC, int SUM>
__global__ void __launch_bounds__(kMaxBlock)
    __attribute__((amdgpu_waves_per_eu(waves_target(FORM, DIM, K, VJP, LPC))))
    patch_kernel(const PatchArgs a, int P)
{
    patch_body<FORM, DIM, K, VJP, LPC, SUM>(a, xcd_order(blockIdx.x, gridDim.x), P);
}

// Many meshes of one kernel variant in one launch: workgroup b works on patch
// b - desc[m].first_patch of mesh m = patch_mesh[b].
template <int FORM, int DIM, int K, bool VJP, int LPC, int SUM>
__global__ void __launch_bounds__(kMaxBlock)
    __attribute__((amdgpu_waves_per_eu(waves_target(FORM, DIM, K, VJP, LPC))))
    batch_patch_kernel(const BatchDesc *__restrict__ desc, const int32_t *__restrict__ patch_mesh,
                       int P)
{
    const int64_t b = xcd_order(blockIdx.x, gridDim.x);
    const int m = patch_mesh[b];
    const BatchDesc &d = desc[m];
    patch_body<FORM, DIM, K, VJP, LPC, SUM>(d.args, b - d.first_patch, P);
}

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

// ----------------------------------------------------------------------- dispatch
using ColourFn = void (*)(const LaunchArgs);
using PatchFn = void (*)(const PatchArgs, int);   // (arguments, cells per patch)
using BatchFn = void (*)(const BatchDesc *, const int32_t *, int);

struct Kernels {
    ColourFn colour;
    PatchFn patch[4][3];  // [lanes per cell 1..3][sum mode 1..2], null where absent
    BatchFn batch[4][3];
};

template <int FORM, int DIM, int K, bool VJP, int LPC>
void fill_lanes(Kernels &k)
{
    k.patch[LPC][SUM_ELEMENT] = patch_kernel<FORM, DIM, K, VJP, LPC, SUM_ELEMENT>;
    k.patch[LPC][SUM_COLOURED] = patch_kernel<FORM, DIM, K, VJP, LPC, SUM_COLOURED>;
    k.batch[LPC][SUM_ELEMENT] = batch_patch_kernel<FORM, DIM, K, VJP, LPC, SUM_ELEMENT>;
    k.batch[LPC][SUM_COLOURED] = batch_patch_kernel<FORM, DIM, K, VJP, LPC, SUM_COLOURED>;
}

template <int FORM, int DIM, int K, bool VJP>
Kernels entry()
{
    Kernels k{};
    k.colour = colour_kernel<FORM, DIM, K, VJP>;
    fill_lanes<FORM, DIM, K, VJP, 1>(k);
    if constexpr (DIM == 2 && FORM != FEM_MASS) fill_lanes<FORM, DIM, K, VJP, 2>(k);
    if constexpr (DIM == 3 && FORM != FEM_MASS) fill_lanes<FORM, DIM, K, VJP, 3>(k);
    return k;
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
    if (form < FEM_MASS || form > FEM_NEOHOOKEAN) return Kernels{};
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
    return Kernels{};
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

// LDS region A (doubles): the staged nodal values, then the element buffer (SUM_ELEMENT)
// or the node accumulator (SUM_COLOURED), which fits in the staging space.
size_t patch_lds_a(int form, int dim, int degree, bool vjp, int patch, int max_nodes, int sum_mode)
{
    const int nloc = nloc_of(dim, degree);
    const int nc = form == FEM_MASS ? 1 : dim;
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

bool pair_available(int form, int dim, int degree)
{
    return lookup(form, dim, degree, false).patch[2][SUM_ELEMENT] != nullptr;
}

bool triple_available(int form, int dim, int degree)
{
    return lookup(form, dim, degree, false).patch[3][SUM_ELEMENT] != nullptr;
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

hipError_t launch_patch(const fem_plan &p, const PatchArgs &a, bool vjp, hipStream_t s)
{
    if (p.lanes < 1 || p.lanes > 3 || (p.sum_mode != SUM_ELEMENT && p.sum_mode != SUM_COLOURED))
        return hipErrorInvalidConfiguration;
    const Kernels ks = lookup(p.form, p.dim, p.degree, vjp);
    PatchFn fn = ks.patch[p.lanes][p.sum_mode];
    if (!fn) return hipErrorInvalidDeviceFunction;
    const int threads = patch_threads(p.patch, p.lanes);
    if (p.patch < 1 || p.patch > 256 || threads > kMaxBlock) return hipErrorInvalidConfiguration;
    const size_t lds = patch_lds_bytes(p.form, p.dim, p.degree, vjp, p.patch, p.max_patch_nodes,
                                       p.sum_mode);
    if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
    hipError_t e = allow_lds((const void *)fn, lds);
    if (e != hipSuccess) return e;
    if (p.n_patch > 0x7fffffff) return hipErrorInvalidConfiguration;
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

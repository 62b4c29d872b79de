// Kernel templates of the matrix-free action (included by the per-form translation
// units, which instantiate them; kernels.hip holds the launchers).
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
//   patch's distinct nodes' values in LDS, every lane reads its cell's values from there
//   and computes its cell vector; the cell vectors are summed into the patch's nodes in a
//   fixed order, either through an LDS element buffer (each node adds its slots in
//   ascending (cell, local node)) or colour by colour into an LDS node buffer.  A node no
//   other patch holds is stored straight into y; a shared one leaves as a partial sum that
//   a small fixup kernel adds up in patch order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "forms.h"
#include "internal.h"

namespace femx {

using ColourFn = void (*)(const LaunchArgs);
using PatchFn = void (*)(const PatchArgs, int);   // (arguments, cells per patch)
using BatchFn = void (*)(const BatchDesc *, const int32_t *, int);

struct Kernels {
    ColourFn colour;
    PatchFn patch[5][3];  // [lanes per cell 1..4][sum mode 1..2], null where absent; four
    BatchFn batch[5][3];  //   lanes: the matrix-core kernel (coloured sums only)
    PatchFn patch_prio[5];  // coloured sums with wave-priority hints, [lanes per cell]
    BatchFn batch_prio[5];
    ColourFn colour_p2;   // P2-geometry cells: colour kernel and one-lane patch kernels
    PatchFn patch_p2[3];  // [sum mode 1..2]
    PatchFn patch_p2_3[3];  // P2-geometry lane triples (3D vector forms), [sum mode 1..2]
};

// one per form, each in its own translation unit (they compile in parallel)
Kernels lookup_mass(int dim, int degree, bool vjp);
Kernels lookup_elasticity(int dim, int degree, bool vjp);
Kernels lookup_neohookean(int dim, int degree, bool vjp);
Kernels lookup_svk(int dim, int degree, bool vjp);
Kernels lookup_laplace(int dim, int degree, bool vjp);
Kernels lookup_helmholtz(int dim, int degree, bool vjp);

constexpr int kMaxBlock = 256;

namespace {


// Waves per SIMD the register allocator is asked to leave room for (occupancy target):
// the lane-pair kernels and the one-lane low-degree 2D kernels fit without spilling in
// the loop; everything else keeps the allocator's default.
constexpr int waves_target(int form, int dim, int k, bool vjp, int lpc, int geo = 1)
{
    if (lpc == 3) return 1;
    // lane pairs, forward: four waves up to P4; three at P5/P6, where four spill ~45
    // registers (P6 neo-Hookean 412 -> 149 us per 2e5 cells at three)
    if (lpc == 2) return vjp ? (k <= 4 ? 3 : 1) : (k <= 4 ? 4 : (k <= 6 ? 3 : 1));
    // affine P1/P2 tetrahedra, linear elasticity: a short loop between long memory and
    // accumulation phases, where a third wave per SIMD pays (the compiler otherwise takes
    // 183 VGPRs; the hyperelastic forms would spill at this bound)
    if (form == FEM_ELASTICITY && !vjp && dim == 3 && k <= 2 && geo == 1) return 3;
    // P4 tetrahedra, scalar forms: 174 VGPRs would leave two waves per SIMD; at three (4
    // spilled) Laplace 165 -> 114 us and Helmholtz 393 -> 227 us per 2e5 cells (the same
    // bound on the 2D P8 scalar kernels spills 24-44 registers and doubles their time)
    if (scalar_form(form) && dim == 3 && k == 4 && geo == 1) return 3;
    // curved cells hold their geometry nodes through the loop: two waves, not three
    return (!vjp && dim == 2 && k <= 4 && !scalar_form(form)) ? (geo == 2 ? 2 : 3) : 1;
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

// The cell's geometry: its affine K and |det J| (GEO = 1, vertices), or the coordinates of
// its P2 geometry nodes for per-point evaluation (GEO = 2; K and |det J| then unused).
template <int DIM, int GEO>
__device__ __forceinline__ double gather_cell_geometry(const int32_t *__restrict__ verts,
                                                       int64_t stride, int64_t s,
                                                       const double *__restrict__ coords,
                                                       double (&K)[DIM][DIM],
                                                       double (&gx)[geom_nodes(DIM, GEO)][DIM])
{
    if constexpr (GEO == 1) {
        return gather_geometry<DIM>(verts, stride, s, coords, K);
    } else {
#pragma unroll
        for (int g = 0; g < geom_nodes(DIM, GEO); ++g) {
            const int64_t vg = verts[g * stride + s];
#pragma unroll
            for (int i = 0; i < DIM; ++i) gx[g][i] = coords[vg * DIM + i];
        }
        return 0.0;
    }
}

// ------------------------------------------------------------------ colour strategy
template <int FORM, int DIM, int K, bool VJP, int GEO>
__global__ void __launch_bounds__(kMaxBlock) colour_kernel(const LaunchArgs a)
{
    constexpr int NLOC = nloc_of(DIM, K);
    constexpr int NC = ncomp_of(FORM, DIM);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.count) return;
    const int64_t s = a.begin + i;
    double Kinv[DIM][DIM], gx[geom_nodes(DIM, GEO)][DIM];
    const double adet = gather_cell_geometry<DIM, GEO>(a.verts, a.stride, s, a.coords, Kinv, gx);
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
    cell_quadrature<FORM, DIM, K, VJP, GEO>(ul, vl, Kinv, adet, gx, a.tab, a.nq, a.lam, a.mu, yl);
    // first-touch bits, one 64-bit word per 64 local nodes ([word][stride])
    constexpr int NWF = (NLOC + 63) / 64;
    uint64_t first[NWF];
#pragma unroll
    for (int w = 0; w < NWF; ++w) first[w] = a.first[w * a.stride + s];
#pragma unroll
    for (int n = 0; n < NLOC; ++n) {
        const int64_t nd = a.nodes[n * a.stride + s];
        double *dst = a.y + nd * NC;
        if ((first[n >> 6] >> (n & 63)) & 1) {
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
template <int FORM, int DIM, int K, bool VJP, int LPC, int SUM, int GEO, bool PRIO>
__device__ __forceinline__ void patch_body(const PatchArgs &a, int64_t p, int P)
{
    constexpr int NLOC = nloc_of(DIM, K);
    constexpr int NC = ncomp_of(FORM, DIM);
    static_assert(LPC == 1 || (LPC == 2 && DIM == 2 && !scalar_form(FORM)) ||
                      (LPC == 3 && DIM == 3 && !scalar_form(FORM)),
                  "lane split");
    static_assert(GEO == 1 || LPC == 1 || LPC == 3,
                  "P2-geometry cells run one lane per cell, or lane triples (3D vector forms)");
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
    // Wave priorities (PRIO; coloured sums, affine cells): a workgroup's memory phases -- the
    // staging here, the sums and the write-out after its quadrature loop -- take issue
    // precedence over the loops of the other workgroups sharing the SIMD, so they overlap
    // those loops rather than wait behind them.  Both variants are built; the launchers run
    // the hinted one only where the compiled kernel uses no scratch memory (no spills).
    static_assert(!PRIO || (SUM == SUM_COLOURED && GEO == 1), "hints: coloured affine kernels");
    constexpr bool kPrio = PRIO;
    if constexpr (kPrio) __builtin_amdgcn_s_setprio(2);
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
    // curved lane triples: lane c keeps coordinate c of the geometry nodes only
    constexpr bool TRI_GEO = LPC == 3 && GEO == 2;
    double Kinv[DIM][DIM], adet = 0.0, gx[TRI_GEO ? 1 : geom_nodes(DIM, GEO)][DIM];
    double gxc[TRI_GEO ? geom_nodes(DIM, GEO) : 1];
    int lid[NLOC];
    if (active) {
        if constexpr (TRI_GEO) {
#pragma unroll
            for (int g = 0; g < geom_nodes(DIM, GEO); ++g)
                gxc[g] = a.coords[(int64_t)a.verts[g * a.stride + s] * DIM + comp];
        } else {
            adet = gather_cell_geometry<DIM, GEO>(a.verts, a.stride, s, a.coords, Kinv, gx);
        }
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
    stage_nodes<NC, VJP, scalar_form(FORM) ? 4 : 8>(a, nb, U, tid, nthreads, lds, b_node);
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
    if constexpr (kPrio) __builtin_amdgcn_s_setprio(0);
    if (active) {
        if constexpr (LPC == 1) {
            cell_quadrature<FORM, DIM, K, VJP, GEO>(ul, vl, Kinv, adet, gx, a.tab, a.nq, a.lam,
                                                    a.mu, yl);
        } else if constexpr (LPC == 3) {
            double u1[NLOC], v1[VJP ? NLOC : 1], y1[NLOC];
#pragma unroll
            for (int n = 0; n < NLOC; ++n) {
                u1[n] = ul[n][0];
                if constexpr (VJP) v1[n] = vl[n][0];
            }
            cell_quadrature_triple<FORM, K, VJP, GEO>(u1, v1, comp, base, Kinv, adet, gxc, a.tab,
                                                      a.nq, a.lam, a.mu, y1);
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
    if constexpr (kPrio) __builtin_amdgcn_s_setprio(1);
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

template <int FORM, int DIM, int K, bool VJP, int LPC, int SUM, int GEO, bool PRIO = false>
__global__ void __launch_bounds__(kMaxBlock)
    __attribute__((amdgpu_waves_per_eu(waves_target(FORM, DIM, K, VJP, LPC, GEO))))
    patch_kernel(const PatchArgs a, int P)
{
    patch_body<FORM, DIM, K, VJP, LPC, SUM, GEO, PRIO>(a, xcd_order(blockIdx.x, gridDim.x), P);
}

// Many meshes of one kernel variant in one launch: workgroup b works on patch
// b - desc[m].first_patch of mesh m = patch_mesh[b].
template <int FORM, int DIM, int K, bool VJP, int LPC, int SUM, bool PRIO = false>
__global__ void __launch_bounds__(kMaxBlock)
    __attribute__((amdgpu_waves_per_eu(waves_target(FORM, DIM, K, VJP, LPC))))
    batch_patch_kernel(const BatchDesc *__restrict__ desc, const int32_t *__restrict__ patch_mesh,
                       int P)
{
    const int64_t b = xcd_order(blockIdx.x, gridDim.x);
    const int m = patch_mesh[b];
    const BatchDesc &d = desc[m];
    patch_body<FORM, DIM, K, VJP, LPC, SUM, 1, PRIO>(d.args, b - d.first_patch, P);
}

}  // namespace
}  // namespace femx

#include "mfma_patch.h"

namespace femx {
namespace {

template <int FORM, int DIM, int K, bool VJP, int LPC, bool BATCH>
void fill_lanes(Kernels &k)
{
    k.patch[LPC][SUM_ELEMENT] = patch_kernel<FORM, DIM, K, VJP, LPC, SUM_ELEMENT, 1>;
    k.patch[LPC][SUM_COLOURED] = patch_kernel<FORM, DIM, K, VJP, LPC, SUM_COLOURED, 1>;
    k.patch_prio[LPC] = patch_kernel<FORM, DIM, K, VJP, LPC, SUM_COLOURED, 1, true>;
    if constexpr (BATCH) {
        k.batch[LPC][SUM_ELEMENT] = batch_patch_kernel<FORM, DIM, K, VJP, LPC, SUM_ELEMENT>;
        k.batch[LPC][SUM_COLOURED] = batch_patch_kernel<FORM, DIM, K, VJP, LPC, SUM_COLOURED>;
        k.batch_prio[LPC] = batch_patch_kernel<FORM, DIM, K, VJP, LPC, SUM_COLOURED, true>;
    }
}

// Degrees up to P6 (2D) / P4 (3D) get every variant; the higher ones (the rest of the
// degree sweep) the single-mesh kernels on affine cells only: no batch, no P2 geometry.
constexpr bool full_set(int dim, int k) { return dim == 2 ? k <= 6 : k <= 4; }

template <int FORM, int DIM, int K, bool VJP>
Kernels entry()
{
    constexpr bool FULL = full_set(DIM, K);
    Kernels k{};
    k.colour = colour_kernel<FORM, DIM, K, VJP, 1>;
    fill_lanes<FORM, DIM, K, VJP, 1, FULL>(k);
    if constexpr (FULL) {
        k.colour_p2 = colour_kernel<FORM, DIM, K, VJP, 2>;
        k.patch_p2[SUM_ELEMENT] = patch_kernel<FORM, DIM, K, VJP, 1, SUM_ELEMENT, 2>;
        k.patch_p2[SUM_COLOURED] = patch_kernel<FORM, DIM, K, VJP, 1, SUM_COLOURED, 2>;
        if constexpr (DIM == 3 && !scalar_form(FORM)) {
            k.patch_p2_3[SUM_ELEMENT] = patch_kernel<FORM, DIM, K, VJP, 3, SUM_ELEMENT, 2>;
            k.patch_p2_3[SUM_COLOURED] = patch_kernel<FORM, DIM, K, VJP, 3, SUM_COLOURED, 2>;
        }
    }
    if constexpr (DIM == 2 && !scalar_form(FORM)) fill_lanes<FORM, DIM, K, VJP, 2, FULL>(k);
    if constexpr (DIM == 3 && !scalar_form(FORM)) fill_lanes<FORM, DIM, K, VJP, 3, FULL>(k);
    k.patch[kMfmaLanes][SUM_COLOURED] = mfma_patch_kernel<FORM, DIM, K, VJP>;
    if constexpr (FULL) k.batch[kMfmaLanes][SUM_COLOURED] = mfma_batch_kernel<FORM, DIM, K, VJP>;
    return k;
}

// the kernel table of one form for (dim, degree), empty where not built
template <int FORM, int DIM, int K>
Kernels pick(bool vjp)
{
    if constexpr (FORM == FEM_NEOHOOKEAN || FORM == FEM_SVK) {
        if (vjp) return entry<FORM, DIM, K, true>();
    }
    return entry<FORM, DIM, K, false>();
}

template <int FORM>
Kernels lookup_form(int dim, int degree, bool vjp)
{
    if (dim == 2) {
        switch (degree) {
        case 1: return pick<FORM, 2, 1>(vjp);
        case 2: return pick<FORM, 2, 2>(vjp);
        case 3: return pick<FORM, 2, 3>(vjp);
        case 4: return pick<FORM, 2, 4>(vjp);
        case 5: return pick<FORM, 2, 5>(vjp);
        case 6: return pick<FORM, 2, 6>(vjp);
        case 7: return pick<FORM, 2, 7>(vjp);
        case 8: return pick<FORM, 2, 8>(vjp);
        default: break;
        }
    } else if (dim == 3) {
        switch (degree) {
        case 1: return pick<FORM, 3, 1>(vjp);
        case 2: return pick<FORM, 3, 2>(vjp);
        case 3: return pick<FORM, 3, 3>(vjp);
        case 4: return pick<FORM, 3, 4>(vjp);
        case 5: return pick<FORM, 3, 5>(vjp);
        case 6: return pick<FORM, 3, 6>(vjp);
        default: break;
        }
    }
    return Kernels{};
}

}  // namespace
}  // namespace femx

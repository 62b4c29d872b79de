// The patch kernel on the FP64 matrix cores (included by kernel_templates.h).
//
// Both contractions of the quadrature loop (paper Sec. 2.3: evaluation of the reference
// gradients at the points from the nodal values, and the test-function contraction of the
// pointwise result) are small dense products shared by every cell of a patch, so they run
// as v_mfma_f64_16x16x4_f64 tiles with 16 cells per tile; the pointwise form (geometry,
// stress or tangent, weight) runs on the vector ALU between them.  A wavefront takes 16
// cells; lane l works on cell l % 16 and on rows l / 16 + 4 k (k = 0..3, its four result
// registers) of every 16-row result tile (the instruction's output layout), so each cell
// is spread over four lanes ("four lanes per cell").
//
// Shapes for dimension d, n = n_loc nodes, Q points padded to 16 T point tiles, rows D_r of
// the tabulation (r < R: the d reference derivatives for the vector forms and Laplace, the
// values for mass, both for Helmholtz) and C components (d, or 1 for the scalar forms):
//   evaluation, point tile t, row r, component c (R C products per tile and k-step):
//     G_rc[q][cell] = sum_a D_r[q][a] u_c[a][cell]      16 x 16, k-steps of 4 nodes
//   pointwise at each of the lane's 4 points of the tile:  T_cr = W P(G K) K^T (vector
//     forms); T_r = W (K K^T G)_r for the derivative rows, W G for the value row (scalar)
//   contraction, node tile m, component c, row r:
//     y_c[a][cell] += sum_q D_r[q][a] T_cr[q][cell]     16 x 16, k-steps of 4 points
// The evaluation's output register k of lane group g (point 16 t + 4 k + g) is exactly the
// contraction's B operand of k-step (t, k) for that lane (k-step (t, k) sums the points
// 16 t + 4 k .. 16 t + 4 k + 3, lane group g supplying the g-th): no data moves between the
// two products.  The A operands (the tabulation, in the
// instruction's operand order, zero-padded) come from the plan's fragment table, one
// 8-byte load per lane per product; the B operands of the evaluation are the cells' nodal
// values gathered from the patch's LDS staging.  Padded points carry weight 0, padded
// nodes zero tabulation, so neither contributes.
#pragma once

namespace femx {

typedef double dvec4 __attribute__((ext_vector_type(4)));

// The fragment table (mfma_table, internal.h), per point tile of 16 points:
//   eval  [r][ks][64]; con [k][r][m][64]; w [16].

namespace {

// Scheduling fences between a tile's evaluation products, its pointwise step and its
// contraction products (the compiler then keeps each phase's instructions together instead
// of interleaving the pointwise vector work into the matrix products).  Outputs are the
// same bit for bit; the time is not, and the better schedule depends on the case, so it is
// chosen per case from an A/B on MI355X (kernel us, fenced against interleaved; per 3e5
// triangles / 1.5e5 tetrahedra): faster fenced -- mass 3D P6 771 -> 413, Helmholtz 2D P8
// 746 -> 370, 3D P6 4487 -> 2818, Laplace 3D P6 3283 -> 2157, 2D P7 240 -> 191,
// neo-Hookean 2D P8 920 -> 541, its VJP 1546 -> 1219, 3D P4 VJP 722 -> 569, St
// Venant-Kirchhoff alike, elasticity and the hyperelastic forms 3D P5 3-5% -- and slower
// fenced -- Helmholtz 3D P5 583 -> 1810, elasticity 3D P4 180 -> 193, the hyperelastic
// forms 2D P6 and 3D P4 (action) 1-9%, their VJP 2D P7 3-4%; within 1% elsewhere.
constexpr bool mfma_fence(int form, int dim, int k, bool vjp)
{
    if (scalar_form(form))
        return dim == 2 ? k >= 7 : (k >= 5 && !(form == FEM_HELMHOLTZ && k == 5));
    if (vjp) return (dim == 2 && k == 8) || (dim == 3 && k == 4);
    return (dim == 2 && k == 8) || (dim == 3 && k == 5);
}

template <int FORM, int DIM, int K, bool VJP>
__device__ __forceinline__ void mfma_body(const PatchArgs &a, int64_t p, int P)
{
    constexpr int NLOC = nloc_of(DIM, K);
    constexpr int NC = ncomp_of(FORM, DIM);
    constexpr int NR = mfma_rows(FORM, DIM);
    constexpr int KS = mfma_ks(NLOC);
    constexpr int MA = mfma_ma(NLOC);
    constexpr int TILE = mfma_tile_doubles(NR, NLOC);
    static_assert(NR * NC * 4 <= 64, "accumulators");
    constexpr int EVAL = NR * KS * 64;
    constexpr int CON = 4 * NR * MA * 64;
    constexpr bool SCALAR = scalar_form(FORM);
    constexpr bool FENCE = mfma_fence(FORM, DIM, K, VJP);
    // the contraction's fragments one k-step ahead, fenced: the 3D vector forms from P5 (NH
    // P5 2224 -> 1510 us, elasticity P5 527 -> 445 per 1.5e5 tetrahedra; at P4 2-6% slower),
    // but not the 3D P6 tangents, which it would make spill
    constexpr bool CPF = !SCALAR && DIM == 3 && K >= 5 && !(VJP && K >= 6);
    // the evaluation's operand prefetch (below): every vector form but the 2D tangents up to
    // P4 (St Venant-Kirchhoff's spilled with it at P3/P4; the vector kernels are the default
    // there) and the 3D P6 tangents, which it would make spill
    constexpr bool EPF = !SCALAR && !(VJP && ((DIM == 2 && K <= 4) || (DIM == 3 && K >= 6)));
    static_assert(!(SCALAR && VJP), "the scalar forms are linear: their VJP is the action");
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int nthreads = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int j = lane & 15, g = lane >> 4;

    const int nb = a.patch_off[p];
    const int U = a.patch_off[p + 1] - nb;
    const int nint = a.patch_nint[p];
    const int pbase = a.patch_pbase[p];

    // this lane's cell (16 per wavefront) and its local node indices for the evaluation's
    // B operands: node 4 ks + g of the cell
    const int cl = wave * 16 + j;
    const int64_t s = p * P + cl;
    const bool active = cl < P && s < a.n_cell;
    double Kinv[DIM][DIM], adet = 0.0;
    int lid[KS];
    if (active) {
        adet = gather_geometry<DIM>(a.verts, a.stride, s, a.coords, Kinv);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int n = 4 * ks + g;
            lid[ks] = n < NLOC ? (int)a.lidx[n * a.stride + s] : -1;
        }
    } else {
#pragma unroll
        for (int r = 0; r < DIM; ++r)
#pragma unroll
            for (int c = 0; c < DIM; ++c) Kinv[r][c] = r == c ? 1.0 : 0.0;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) lid[ks] = -1;
    }
    // region A: the staged values (u, then v), read through the whole loop, then the node
    // accumulator; region B: the node ids
    int32_t *b_node = reinterpret_cast<int32_t *>(lds + a.lds_a);
    double *acc_nodes = lds;
    stage_nodes<NC, VJP, 8>(a, nb, U, tid, nthreads, lds, b_node);
    __syncthreads();

    // the evaluation's B operands (the cell's value at node 4 ks + g): held in registers
    // when they are few, else gathered from the staged values at every point tile
    constexpr bool HOLD = KS * NC * (VJP ? 2 : 1) <= 24;
    double bu[HOLD ? KS : 1][NC], bv[HOLD && VJP ? KS : 1][NC];
    auto gather = [&](int ks, int c, bool second) {
        const int l = lid[ks];
        return l >= 0 ? lds[((second ? U : 0) + l) * NC + c] : 0.0;
    };
    if constexpr (HOLD) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                bu[ks][c] = gather(ks, c, false);
                if constexpr (VJP) bv[ks][c] = gather(ks, c, true);
            }
    }

    // the scalar forms' flux map K K^T (the cell's constant; inactive lanes: W = 0)
    double KKt[SCALAR ? DIM : 1][SCALAR ? DIM : 1];
    if constexpr (SCALAR) {
#pragma unroll
        for (int r = 0; r < DIM; ++r)
#pragma unroll
            for (int q2 = 0; q2 < DIM; ++q2) {
                double s2 = 0.0;
#pragma unroll
                for (int jj = 0; jj < DIM; ++jj) s2 = fma(Kinv[r][jj], Kinv[q2][jj], s2);
                KKt[r][q2] = s2;
            }
    }

    dvec4 y[NC][MA];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int m = 0; m < MA; ++m) y[c][m] = dvec4{0.0, 0.0, 0.0, 0.0};

    const double *__restrict__ mt = a.mtab;
#pragma unroll 1
    for (int t = 0; t < a.nqt; ++t) {
        if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
        const double *tile = mt + (int64_t)t * TILE;
        // evaluation: G_rc (and the gradient of v for the VJP) on this tile's 16 points
        dvec4 acc[NR][NC], accv[VJP ? NR : 1][NC];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                acc[r][c] = dvec4{0.0, 0.0, 0.0, 0.0};
                if constexpr (VJP) accv[r][c] = dvec4{0.0, 0.0, 0.0, 0.0};
            }
        // the next k-step's operands are loaded before this one's products (EPF: a fence
        // keeps them there, nine products ahead of their use instead of the few the compiler
        // leaves; measured 5-23% faster for the vector forms, bitwise the same; the scalar
        // forms, with one to four products per k-step, keep the compiler's order)
        double afn[NR], b0n[NC], b1n[VJP ? NC : 1];
        auto load_step = [&](int ks) {
#pragma unroll
            for (int r = 0; r < NR; ++r) afn[r] = tile[(r * KS + ks) * 64 + lane];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if constexpr (HOLD) {
                    b0n[c] = bu[ks][c];
                    if constexpr (VJP) b1n[c] = bv[ks][c];
                } else {
                    b0n[c] = gather(ks, c, false);
                    if constexpr (VJP) b1n[c] = gather(ks, c, true);
                }
            }
        };
        load_step(0);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            double b0[NC], b1[VJP ? NC : 1], afc[NR];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                b0[c] = b0n[c];
                if constexpr (VJP) b1[c] = b1n[c];
            }
#pragma unroll
            for (int r = 0; r < NR; ++r) afc[r] = afn[r];
            if (ks + 1 < KS) load_step(ks + 1);
            if constexpr (EPF) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const double af = afc[r];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, b0[c], acc[r][c], 0, 0, 0);
                    if constexpr (VJP)
                        accv[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, b1[c], accv[r][c], 0, 0, 0);
                }
            }
        }
        // the pointwise form at the lane's four points 16 t + 4 k + g of its cell
        if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
        const double *wt = tile + EVAL + CON;
        if constexpr (SCALAR) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double W = wt[4 * k + g] * adet;
                if constexpr (FORM != FEM_MASS) {
                    // flux against the reference test derivatives: W K K^T grad_ref u
                    double gr[DIM];
#pragma unroll
                    for (int r = 0; r < DIM; ++r) gr[r] = acc[r][0][k];
#pragma unroll
                    for (int r = 0; r < DIM; ++r) {
                        double s2 = 0.0;
#pragma unroll
                        for (int q2 = 0; q2 < DIM; ++q2) s2 = fma(KKt[r][q2], gr[q2], s2);
                        acc[r][0][k] = W * s2;
                    }
                }
                if constexpr (FORM == FEM_MASS || FORM == FEM_HELMHOLTZ)
                    acc[NR - 1][0][k] = W * acc[NR - 1][0][k];     // the value row
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double gu[DIM][DIM], gv[DIM][DIM], G[DIM][DIM], H[DIM][DIM], S[DIM][DIM], T[DIM][DIM];
#pragma unroll
                for (int c = 0; c < DIM; ++c)
#pragma unroll
                    for (int r = 0; r < DIM; ++r) {
                        gu[c][r] = acc[r][c][k];
                        if constexpr (VJP) gv[c][r] = accv[r][c][k];
                    }
                to_physical<DIM>(gu, Kinv, G);
                if constexpr (VJP) to_physical<DIM>(gv, Kinv, H);
                pointwise<FORM, DIM, VJP>(G, H, a.lam, a.mu, S);
                pull_back<DIM>(S, Kinv, wt[4 * k + g] * adet, T);
#pragma unroll
                for (int c = 0; c < DIM; ++c)
#pragma unroll
                    for (int r = 0; r < DIM; ++r) acc[r][c][k] = T[c][r];
            }
        }
        // contraction: k-step (t, k) takes register k of every lane as its B operand
        if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
        const double *con = tile + EVAL;
        if constexpr (CPF) {
            // the next k-step's fragments loaded before this one's products (fenced)
            double cfn[NR][MA];
#pragma unroll
            for (int r = 0; r < NR; ++r)
#pragma unroll
                for (int m = 0; m < MA; ++m) cfn[r][m] = con[(r * MA + m) * 64 + lane];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double cf[NR][MA];
#pragma unroll
                for (int r = 0; r < NR; ++r)
#pragma unroll
                    for (int m = 0; m < MA; ++m) cf[r][m] = cfn[r][m];
                if (k + 1 < 4) {
#pragma unroll
                    for (int r = 0; r < NR; ++r)
#pragma unroll
                        for (int m = 0; m < MA; ++m)
                            cfn[r][m] = con[(((k + 1) * NR + r) * MA + m) * 64 + lane];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int r = 0; r < NR; ++r)
#pragma unroll
                    for (int m = 0; m < MA; ++m)
#pragma unroll
                        for (int c = 0; c < NC; ++c)
                            y[c][m] = __builtin_amdgcn_mfma_f64_16x16x4f64(cf[r][m], acc[r][c][k],
                                                                           y[c][m], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int r = 0; r < NR; ++r)
#pragma unroll
                    for (int m = 0; m < MA; ++m) {
                        const double af = con[((k * NR + r) * MA + m) * 64 + lane];
#pragma unroll
                        for (int c = 0; c < NC; ++c)
                            y[c][m] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, acc[r][c][k], y[c][m],
                                                                           0, 0, 0);
                    }
        }
    }

    if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
    // sum the cell vectors into the patch's nodes, sub-colour by sub-colour (no two cells of
    // a colour share a node, and the four lanes of a cell hold different nodes: one writer
    // per address within a phase, so the order is fixed)
    const int col = active ? a.colour[s] : -1;
    int lid2[MA][4];
#pragma unroll
    for (int m = 0; m < MA; ++m)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int n = 16 * m + 4 * k + g;          // result row 4 k + g of node tile m
            lid2[m][k] = (active && n < NLOC) ? (int)a.lidx[n * a.stride + s] : -1;
        }
    const int ncol = a.patch_ncol[p];
    __syncthreads();                          // every wavefront is past its last gather
    for (int jj = tid; jj < U * NC; jj += nthreads) acc_nodes[jj] = 0.0;
    __syncthreads();
    for (int kc = 0; kc < ncol; ++kc) {
        if (col == kc) {
#pragma unroll
            for (int m = 0; m < MA; ++m)
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (lid2[m][k] >= 0) {
#pragma unroll
                        for (int c = 0; c < NC; ++c)
                            __hip_atomic_fetch_add(&acc_nodes[lid2[m][k] * NC + c], y[c][m][k],
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
        }
        __syncthreads();
    }

    // each distinct node stored once: interior nodes into y, shared ones as partials
    for (int jj = tid; jj < U; jj += nthreads) {
        double sum[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) sum[c] = acc_nodes[jj * NC + c];
        if (jj < nint) {
            const int64_t nd = b_node[jj];
#pragma unroll
            for (int c = 0; c < NC; ++c) a.y[nd * NC + c] = sum[c];
        } else {
            const int64_t dest = a.pdest[pbase + (jj - nint)];
#pragma unroll
            for (int c = 0; c < NC; ++c) a.partial[dest * NC + c] = sum[c];
        }
    }
}

// Waves per SIMD the register allocator is asked to leave room for: more resident
// workgroups overlap one another's staging, sums and write-out with the matrix products.
// Set per case from the compiler's resource report so that no bound causes a spill (1: the
// allocator's default, which also uses the accumulation registers).
constexpr int mfma_waves(int form, int dim, int k, bool vjp)
{
    if (scalar_form(form)) return 1;
    if (!vjp) {
        if (dim == 2) {
            if (k <= 4) return 4;
            if (form == FEM_ELASTICITY) return k <= 6 ? 4 : 3;
            return k <= 7 ? 3 : 1;
        }
        if (form == FEM_ELASTICITY) return k <= 2 ? 3 : (k <= 5 ? 2 : 1);
        if (form == FEM_NEOHOOKEAN) return k == 1 ? 3 : ((k == 2 || k == 4) ? 2 : 1);
        return k == 1 ? 3 : (k <= 5 ? 2 : 1);                       // St Venant-Kirchhoff
    }
    if (dim == 2) {
        if (form == FEM_NEOHOOKEAN) return (k <= 3 || k == 6) ? 3 : 1;
        return (k == 1 || k == 3 || k == 4 || k == 6) ? 3 : 1;      // St Venant-Kirchhoff
    }
    return (form == FEM_SVK && k == 1) ? 2 : 1;
}

template <int FORM, int DIM, int K, bool VJP>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(mfma_waves(FORM, DIM, K, VJP))))
    mfma_patch_kernel(const PatchArgs a, int P)
{
    mfma_body<FORM, DIM, K, VJP>(a, xcd_order(blockIdx.x, gridDim.x), P);
}

template <int FORM, int DIM, int K, bool VJP>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(mfma_waves(FORM, DIM, K, VJP))))
    mfma_batch_kernel(const BatchDesc *__restrict__ desc, const int32_t *__restrict__ patch_mesh, int P)
{
    const int64_t b = xcd_order(blockIdx.x, gridDim.x);
    const int m = patch_mesh[b];
    const BatchDesc &d = desc[m];
    mfma_body<FORM, DIM, K, VJP>(d.args, b - d.first_patch, P);
}

}  // namespace
}  // namespace femx

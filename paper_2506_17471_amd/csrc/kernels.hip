// FP64 matrix-free action kernels for gfx950 (CDNA4).
//
// One lane owns one cell (the per-cell loop of the paper's generic action kernel, Sec.
// 2.3, mapped so that a wavefront works on 64 cells of one colour).  Per lane:
//   gather:   the cell's vertex ids and node ids from the colour-sorted structure-of-arrays
//             maps (consecutive lanes read consecutive words), then the coordinates and the
//             nodal values through them;
//   geometry: J = [x_1 - x_0 | ...], |det J| and K = J^{-1}, once per cell (affine cells);
//   per quadrature point:
//     evaluation:  reference gradients of u (or u itself for the mass form) from the
//                  tabulation, a small dense contraction over the cell's nodes;
//     pointwise:   the form's stress (mass: the value), mapped by K and scaled by w |det J|;
//     quadrature:  accumulation against the same tabulation into the cell's output;
//   scatter:  write (first holder of a node in colour order) or read-add-write (later
//             holders).  Cells of one launch share no node, so no atomics are needed and
//             the summation order is fixed.
// The tabulation index is the same for all 64 lanes, so the tables are read through the
// constant address space: the compiler emits scalar loads into SGPRs and every FMA of the
// two contractions takes its table operand from an SGPR.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

#define CONSTANT __attribute__((address_space(4)))

namespace femx {
namespace {

constexpr int kMaxBlock = 256;

__host__ __device__ constexpr int nloc_of(int dim, int k)
{
    return dim == 2 ? (k + 1) * (k + 2) / 2 : (k + 1) * (k + 2) * (k + 3) / 6;
}

__host__ __device__ constexpr int record_of(int form, int dim, int nloc)
{
    return (((form == FEM_MASS ? nloc : dim * nloc) + 1) + 1) & ~1;
}

// K = J^{-1} and |det J| from the vertex coordinates (J[i][r] = x_{r+1,i} - x_{0,i}).
template <int DIM>
__device__ __forceinline__ double affine_geometry(const double (&x)[DIM + 1][DIM],
                                                  double (&K)[DIM][DIM])
{
    double J[DIM][DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int r = 0; r < DIM; ++r) J[i][r] = x[r + 1][i] - x[0][i];
    if constexpr (DIM == 2) {
        const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const double inv = 1.0 / det;
        K[0][0] = J[1][1] * inv;
        K[0][1] = -J[0][1] * inv;
        K[1][0] = -J[1][0] * inv;
        K[1][1] = J[0][0] * inv;
        return fabs(det);
    } else {
        const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        const double inv = 1.0 / det;
        K[0][0] = c00 * inv;
        K[1][0] = c01 * inv;
        K[2][0] = c02 * inv;
        K[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * inv;
        K[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * inv;
        K[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * inv;
        K[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * inv;
        K[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * inv;
        K[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * inv;
        return fabs(det);
    }
}

// A^{-1} and det A for a small matrix.
template <int DIM>
__device__ __forceinline__ double invert(const double (&A)[DIM][DIM], double (&B)[DIM][DIM])
{
    if constexpr (DIM == 2) {
        const double det = A[0][0] * A[1][1] - A[0][1] * A[1][0];
        const double inv = 1.0 / det;
        B[0][0] = A[1][1] * inv;
        B[0][1] = -A[0][1] * inv;
        B[1][0] = -A[1][0] * inv;
        B[1][1] = A[0][0] * inv;
        return det;
    } else {
        const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
        const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
        const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
        const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
        const double inv = 1.0 / det;
        B[0][0] = c00 * inv;
        B[1][0] = c01 * inv;
        B[2][0] = c02 * inv;
        B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * inv;
        B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * inv;
        B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * inv;
        B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * inv;
        B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * inv;
        B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * inv;
        return det;
    }
}

// physical gradient G[c][j] = sum_r gref[c][r] K[r][j]
template <int DIM>
__device__ __forceinline__ void to_physical(const double (&gref)[DIM][DIM],
                                            const double (&K)[DIM][DIM], double (&G)[DIM][DIM])
{
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < DIM; ++r) s = fma(gref[c][r], K[r][j], s);
            G[c][j] = s;
        }
}

// T[c][r] = W sum_j S[c][j] K[r][j]  (stress pulled back to reference derivatives)
template <int DIM>
__device__ __forceinline__ void pull_back(const double (&S)[DIM][DIM], const double (&K)[DIM][DIM],
                                          double W, double (&T)[DIM][DIM])
{
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int r = 0; r < DIM; ++r) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < DIM; ++j) s = fma(S[c][j], K[r][j], s);
            T[c][r] = W * s;
        }
}

template <int DIM>
__device__ __forceinline__ void stress_elasticity(const double (&G)[DIM][DIM], double lam,
                                                  double mu, double (&S)[DIM][DIM])
{
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) tr += G[i][i];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) S[i][j] = mu * (G[i][j] + G[j][i]) + (i == j ? lam * tr : 0.0);
}

// P = mu (F - F^{-T}) + lam ln(det F) F^{-T},  F = I + G
template <int DIM>
__device__ __forceinline__ void stress_neohookean(const double (&G)[DIM][DIM], double lam,
                                                  double mu, double (&S)[DIM][DIM])
{
    double F[DIM][DIM], Fi[DIM][DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) F[i][j] = G[i][j] + (i == j ? 1.0 : 0.0);
    const double detF = invert<DIM>(F, Fi);
    const double c = lam * log(detF) - mu;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) S[i][j] = fma(mu, F[i][j], c * Fi[j][i]);
}

// dP[H] = mu H + (mu - lam ln J) F^{-T} H^T F^{-T} + lam tr(F^{-1} H) F^{-T}
// (the tangent contracted with H; it equals the transpose contraction because the
// tangent of a hyperelastic stress has major symmetry)
template <int DIM>
__device__ __forceinline__ void tangent_neohookean(const double (&G)[DIM][DIM],
                                                   const double (&H)[DIM][DIM], double lam,
                                                   double mu, double (&S)[DIM][DIM])
{
    double F[DIM][DIM], Fi[DIM][DIM], FiH[DIM][DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) F[i][j] = G[i][j] + (i == j ? 1.0 : 0.0);
    const double detF = invert<DIM>(F, Fi);
    const double b = mu - lam * log(detF);
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) s = fma(Fi[i][k], H[k][j], s);
            FiH[i][j] = s;
        }
#pragma unroll
    for (int i = 0; i < DIM; ++i) tr += FiH[i][i];
    const double ct = lam * tr;
    // (F^{-T} H^T F^{-T})[k][l] = (F^{-1} H F^{-1})[l][k] = sum_m FiH[l][m] Fi[m][k]
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int l = 0; l < DIM; ++l) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < DIM; ++m) s = fma(FiH[l][m], Fi[m][k], s);
            S[k][l] = fma(mu, H[k][l], fma(b, s, ct * Fi[l][k]));
        }
}

// The cell's colour-sorted index and the gather of its geometry.
template <int DIM>
__device__ __forceinline__ double gather_geometry(const LaunchArgs &a, int64_t s,
                                                  double (&K)[DIM][DIM])
{
    double x[DIM + 1][DIM];
#pragma unroll
    for (int j = 0; j <= DIM; ++j) {
        const int64_t vj = a.verts[j * a.stride + s];
#pragma unroll
        for (int i = 0; i < DIM; ++i) x[j][i] = a.coords[vj * DIM + i];
    }
    return affine_geometry<DIM>(x, K);
}

template <int NLOC, int NC>
__device__ __forceinline__ void gather_values(const LaunchArgs &a, int64_t s, const double *vec,
                                              double (&loc)[NLOC][NC])
{
#pragma unroll
    for (int n = 0; n < NLOC; ++n) {
        const int64_t nd = a.nodes[n * a.stride + s];
#pragma unroll
        for (int c = 0; c < NC; ++c) loc[n][c] = vec[nd * NC + c];
    }
}

template <int NLOC, int NC>
__device__ __forceinline__ void scatter_values(const LaunchArgs &a, int64_t s,
                                               const double (&loc)[NLOC][NC])
{
    const uint64_t first = a.first[s];
#pragma unroll
    for (int n = 0; n < NLOC; ++n) {
        const int64_t nd = a.nodes[n * a.stride + s];
        double *dst = a.y + nd * NC;
        if ((first >> n) & 1) {
#pragma unroll
            for (int c = 0; c < NC; ++c) dst[c] = loc[n][c];
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) dst[c] += loc[n][c];
        }
    }
}

// ---------------------------------------------------------------------------- mass
template <int DIM, int K>
__global__ void __launch_bounds__(kMaxBlock) mass_kernel(const LaunchArgs a)
{
    constexpr int NLOC = nloc_of(DIM, K);
    constexpr int REC = record_of(FEM_MASS, DIM, NLOC);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.count) return;
    const int64_t s = a.begin + i;
    double Kinv[DIM][DIM];
    const double adet = gather_geometry<DIM>(a, s, Kinv);
    double ul[NLOC][1], yl[NLOC][1];
    gather_values<NLOC, 1>(a, s, a.u, ul);
#pragma unroll
    for (int n = 0; n < NLOC; ++n) yl[n][0] = 0.0;
    const CONSTANT double *tab = (const CONSTANT double *)a.tab;
#pragma unroll 1
    for (int q = 0; q < a.nq; ++q) {
        const CONSTANT double *t = tab + q * REC;
        double uq = 0.0;
#pragma unroll
        for (int n = 0; n < NLOC; ++n) uq = fma(t[n], ul[n][0], uq);
        const double e = t[NLOC] * adet * uq;
#pragma unroll
        for (int n = 0; n < NLOC; ++n) yl[n][0] = fma(t[n], e, yl[n][0]);
    }
    scatter_values<NLOC, 1>(a, s, yl);
}

// ------------------------------------------------------------------ vector forms
// FORM: FEM_ELASTICITY or FEM_NEOHOOKEAN; VJP: neo-Hookean vector-Jacobian product.
template <int FORM, int DIM, int K, bool VJP>
__global__ void __launch_bounds__(kMaxBlock) vector_kernel(const LaunchArgs a)
{
    constexpr int NLOC = nloc_of(DIM, K);
    constexpr int REC = record_of(FORM, DIM, NLOC);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.count) return;
    const int64_t s = a.begin + i;
    double Kinv[DIM][DIM];
    const double adet = gather_geometry<DIM>(a, s, Kinv);
    double ul[NLOC][DIM], vl[VJP ? NLOC : 1][DIM], yl[NLOC][DIM];
    gather_values<NLOC, DIM>(a, s, a.u, ul);
    if constexpr (VJP) gather_values<NLOC, DIM>(a, s, a.v, vl);
#pragma unroll
    for (int n = 0; n < NLOC; ++n)
#pragma unroll
        for (int c = 0; c < DIM; ++c) yl[n][c] = 0.0;
    const CONSTANT double *tab = (const CONSTANT double *)a.tab;
#pragma unroll 1
    for (int q = 0; q < a.nq; ++q) {
        const CONSTANT double *t = tab + q * REC;
        // evaluation: reference gradients at the point
        double gu[DIM][DIM], gv[DIM][DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int r = 0; r < DIM; ++r) {
                gu[c][r] = 0.0;
                gv[c][r] = 0.0;
            }
#pragma unroll
        for (int n = 0; n < NLOC; ++n)
#pragma unroll
            for (int r = 0; r < DIM; ++r) {
                const double tr = t[r * NLOC + n];
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    gu[c][r] = fma(tr, ul[n][c], gu[c][r]);
                    if constexpr (VJP) gv[c][r] = fma(tr, vl[n][c], gv[c][r]);
                }
            }
        // pointwise form
        double G[DIM][DIM], S[DIM][DIM], T[DIM][DIM];
        to_physical<DIM>(gu, Kinv, G);
        if constexpr (VJP) {
            double H[DIM][DIM];
            to_physical<DIM>(gv, Kinv, H);
            tangent_neohookean<DIM>(G, H, a.lam, a.mu, S);
        } else if constexpr (FORM == FEM_ELASTICITY) {
            stress_elasticity<DIM>(G, a.lam, a.mu, S);
        } else {
            stress_neohookean<DIM>(G, a.lam, a.mu, S);
        }
        pull_back<DIM>(S, Kinv, t[DIM * NLOC] * adet, T);
        // quadrature: accumulate against the test-function gradients
#pragma unroll
        for (int n = 0; n < NLOC; ++n)
#pragma unroll
            for (int r = 0; r < DIM; ++r) {
                const double tr = t[r * NLOC + n];
#pragma unroll
                for (int c = 0; c < DIM; ++c) yl[n][c] = fma(tr, T[c][r], yl[n][c]);
            }
    }
    scatter_values<NLOC, DIM>(a, s, yl);
}

__global__ void zero_nodes_kernel(const int32_t *__restrict__ nodes, int64_t n, int ncomp,
                                  double *__restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t nd = nodes[i];
    for (int c = 0; c < ncomp; ++c) y[nd * ncomp + c] = 0.0;
}

using KernelFn = void (*)(const LaunchArgs);

template <int DIM, int K>
KernelFn pick(int form, bool vjp)
{
    if (form == FEM_MASS) return mass_kernel<DIM, K>;
    if (form == FEM_ELASTICITY) return vector_kernel<FEM_ELASTICITY, DIM, K, false>;
    if (vjp) return vector_kernel<FEM_NEOHOOKEAN, DIM, K, true>;
    return vector_kernel<FEM_NEOHOOKEAN, DIM, K, false>;
}

KernelFn lookup(int form, int dim, int degree, bool vjp)
{
    if (dim == 2) {
        switch (degree) {
        case 1: return pick<2, 1>(form, vjp);
        case 2: return pick<2, 2>(form, vjp);
        case 3: return pick<2, 3>(form, vjp);
        case 4: return pick<2, 4>(form, vjp);
        case 5: return pick<2, 5>(form, vjp);
        case 6: return pick<2, 6>(form, vjp);
        default: return nullptr;
        }
    }
    if (dim == 3) {
        switch (degree) {
        case 1: return pick<3, 1>(form, vjp);
        case 2: return pick<3, 2>(form, vjp);
        case 3: return pick<3, 3>(form, vjp);
        case 4: return pick<3, 4>(form, vjp);
        default: return nullptr;
        }
    }
    return nullptr;
}

}  // namespace

bool kernel_available(int form, int dim, int degree)
{
    return lookup(form, dim, degree, false) != nullptr;
}

hipError_t launch_action(const fem_plan &p, const LaunchArgs &a, int block, bool vjp,
                         hipStream_t s)
{
    KernelFn fn = lookup(p.form, p.dim, p.degree, vjp);
    if (!fn) return hipErrorInvalidDeviceFunction;
    if (block <= 0) block = 64;
    if (block > kMaxBlock) return hipErrorInvalidConfiguration;
    const int64_t grid = (a.count + block - 1) / block;
    if (grid > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(block), 0, s, a);
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

// Device-side pieces of the per-cell computation shared by the launch strategies:
// affine geometry, the pointwise forms, and the evaluation -> pointwise -> quadrature loop
// over the quadrature points of one cell (paper Sec. 2.3: the generic action kernel's
// per-cell body; App. A: the forms).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/fem_action.h"
#include "internal.h"

#define FEMX_CONSTANT __attribute__((address_space(4)))

namespace femx {

__host__ __device__ constexpr int nloc_of(int dim, int k)
{
    return dim == 2 ? (k + 1) * (k + 2) / 2 : (k + 1) * (k + 2) * (k + 3) / 6;
}

// doubles per quadrature-point record of the kernel table (see table_record()): values
// phi_a (mass, Helmholtz), reference derivatives (all but mass), the weight; even length
__host__ __device__ constexpr int record_base(int form, int dim, int nloc)
{
    return ((form == FEM_MASS || form == FEM_HELMHOLTZ) ? nloc : 0) +
           (form == FEM_MASS ? 0 : dim * nloc) + 1;
}

// ... then, for P2 geometry (geo = 2), the geometry basis' reference derivatives
__host__ __device__ constexpr int record_of(int form, int dim, int nloc, int geo = 1)
{
    return (record_base(form, dim, nloc) + (geo == 2 ? dim * (dim == 2 ? 6 : 10) : 0) + 1) & ~1;
}

// 1/d: hardware reciprocal estimate refined by two Newton-Raphson steps (each doubles the
// number of correct bits), then one residual correction; within 1 ulp of 1/d for finite
// nonzero normal d.
__device__ __forceinline__ double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    return fma(fma(-d, r, 1.0), r, r);
}

// Natural logarithm of a positive finite double by the classical reduction
//   x = 2^e m,  m in [1/sqrt2, sqrt2),  ln m = 2 atanh(s),  s = (m-1)/(m+1),  |s| <= 0.1716,
// with the Taylor series atanh(s) = s + s^3/3 + s^5/5 + ... summed to s^23 (the first
// omitted term is below 2^-58 relative), and ln 2 split in two parts so that e ln 2 is
// exact to double precision.  Error a few ulp; no special cases for x <= 0, inf or nan
// (the forms only take logarithms of det F > 0).
__device__ __forceinline__ double ln_pos(double x)
{
    int e = __builtin_amdgcn_frexp_exp(x);
    double m = __builtin_amdgcn_frexp_mant(x);          // [0.5, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double num = m - 1.0, den = m + 1.0;
    const double r = recip(den);
    double s = num * r;
    s = fma(fma(-s, den, num), r, s);                    // correct the quotient
    const double z = s * s;
    double p = 1.0 / 23.0;
    p = fma(p, z, 1.0 / 21.0);
    p = fma(p, z, 1.0 / 19.0);
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    const double lnm = fma(2.0 * s * z, p, 2.0 * s);     // 2 s (1 + z p)
    const double fe = (double)e;
    // ln 2 = ln2_hi + ln2_lo: ln2_hi is ln 2 truncated to 36 fraction bits (so e * ln2_hi is
    // exact for any exponent of a double), ln2_lo the rounded remainder.
    constexpr double ln2_hi = 0x1.62e42fefa0000p-1;
    constexpr double ln2_lo = 1.6465949582897082e-12;
    return fma(fe, ln2_hi, fma(fe, ln2_lo, lnm));
}

// K = J^{-1} and |det J| from the vertex coordinates (J[i][r] = x_{r+1,i} - x_{0,i}).
// K = J^{-1} by cofactors; returns |det J|
template <int DIM>
__device__ __forceinline__ double jacobian_inverse(const double (&J)[DIM][DIM], double (&K)[DIM][DIM])
{
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

// affine cell from its vertices: J = [x_1 - x_0 | ... | x_d - x_0], K = J^{-1}, |det J|
template <int DIM>
__device__ __forceinline__ double affine_geometry(const double (&x)[DIM + 1][DIM],
                                                  double (&K)[DIM][DIM])
{
    double J[DIM][DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int r = 0; r < DIM; ++r) J[i][r] = x[r + 1][i] - x[0][i];
    return jacobian_inverse<DIM>(J, K);
}

// geometry nodes a cell carries: the d+1 vertices (affine) or the P2 lattice (GEO = 2)
__host__ __device__ constexpr int geom_nodes(int dim, int geo)
{
    return geo == 2 ? nloc_of(dim, 2) : dim + 1;
}

// Non-affine cells (P2 geometry, paper Sec. 2.4): at quadrature point q,
// J_ir = sum_g x_g,i d phi^G_g / d xi_r from the tabulated geometry gradients tg (r-major,
// NG per direction), K = J^{-1} and |det J| per point.  For affine cells (GEO = 1) the
// cell's constant K and |det J| pass through.
template <int DIM, int GEO>
__device__ __forceinline__ double point_geometry(const FEMX_CONSTANT double *tg,
                                                 const double (&gx)[geom_nodes(DIM, GEO)][DIM],
                                                 const double (&Kc)[DIM][DIM], double adc,
                                                 double (&Kq)[DIM][DIM])
{
    if constexpr (GEO == 1) {
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
            for (int j = 0; j < DIM; ++j) Kq[i][j] = Kc[i][j];
        return adc;
    } else {
        constexpr int NG = geom_nodes(DIM, GEO);
        double J[DIM][DIM];
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
            for (int r = 0; r < DIM; ++r) {
                double acc = 0.0;
#pragma unroll
                for (int g = 0; g < NG; ++g) acc = fma(gx[g][i], tg[r * NG + g], acc);
                J[i][r] = acc;
            }
        return jacobian_inverse<DIM>(J, Kq);
    }
}

template <int DIM>
__device__ __forceinline__ double invert(const double (&A)[DIM][DIM], double (&B)[DIM][DIM])
{
    if constexpr (DIM == 2) {
        const double det = A[0][0] * A[1][1] - A[0][1] * A[1][0];
        const double inv = recip(det);
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
        const double inv = recip(det);
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

// T[c][r] = W sum_j S[c][j] K[r][j]: the stress paired with reference test derivatives
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

// sigma = lam tr(G) I + mu (G + G^T)
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
    const double c = lam * ln_pos(detF) - mu;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) S[i][j] = fma(mu, F[i][j], c * Fi[j][i]);
}

// dP[H] = mu H + (mu - lam ln J) F^{-T} H^T F^{-T} + lam tr(F^{-1} H) F^{-T}: the tangent
// contracted with H; it equals the transposed contraction because the tangent of a
// hyperelastic stress has major symmetry.
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
    const double b = mu - lam * ln_pos(detF);
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

// St Venant-Kirchhoff: E = (F^T F - I)/2, S = lam tr(E) I + 2 mu E, P = F S,  F = I + G
template <int DIM>
__device__ __forceinline__ void stress_svk(const double (&G)[DIM][DIM], double lam, double mu,
                                           double (&P)[DIM][DIM])
{
    double F[DIM][DIM], S[DIM][DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) F[i][j] = G[i][j] + (i == j ? 1.0 : 0.0);
    double trE = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) trE = fma(F[i][j], F[i][j], trE);
    trE = 0.5 * (trE - DIM);
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = i; j < DIM; ++j) {
            double c = 0.0;                          // (F^T F)_ij
#pragma unroll
            for (int k = 0; k < DIM; ++k) c = fma(F[k][i], F[k][j], c);
            const double e = 0.5 * (c - (i == j ? 1.0 : 0.0));
            S[i][j] = 2.0 * mu * e + (i == j ? lam * trE : 0.0);
            S[j][i] = S[i][j];
        }
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) s = fma(F[i][k], S[k][j], s);
            P[i][j] = s;
        }
}

// dP[H] = H S + F dS,  dS = lam tr(dE) I + 2 mu dE,  dE = sym(F^T H): the St Venant-
// Kirchhoff tangent contracted with H (major symmetry: also the transposed contraction)
template <int DIM>
__device__ __forceinline__ void tangent_svk(const double (&G)[DIM][DIM],
                                            const double (&H)[DIM][DIM], double lam, double mu,
                                            double (&dP)[DIM][DIM])
{
    double F[DIM][DIM], S[DIM][DIM], dS[DIM][DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) F[i][j] = G[i][j] + (i == j ? 1.0 : 0.0);
    double trE = 0.0, trdE = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
            trE = fma(F[i][j], F[i][j], trE);
            trdE = fma(F[i][j], H[i][j], trdE);     // tr(F^T H)
        }
    trE = 0.5 * (trE - DIM);
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = i; j < DIM; ++j) {
            double c = 0.0, fh = 0.0, hf = 0.0;     // (F^T F)_ij, (F^T H)_ij, (F^T H)_ji
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                c = fma(F[k][i], F[k][j], c);
                fh = fma(F[k][i], H[k][j], fh);
                hf = fma(F[k][j], H[k][i], hf);
            }
            const double e = 0.5 * (c - (i == j ? 1.0 : 0.0));
            const double de = 0.5 * (fh + hf);
            S[i][j] = 2.0 * mu * e + (i == j ? lam * trE : 0.0);
            dS[i][j] = 2.0 * mu * de + (i == j ? lam * trdE : 0.0);
            S[j][i] = S[i][j];
            dS[j][i] = dS[i][j];
        }
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) s = fma(H[i][k], S[k][j], fma(F[i][k], dS[k][j], s));
            dP[i][j] = s;
        }
}

// The pointwise map of a form at one quadrature point: the stress of G, or with VJP the
// tangent of the stress at G contracted with H.
template <int FORM, int DIM, bool VJP>
__device__ __forceinline__ void pointwise(const double (&G)[DIM][DIM], const double (&H)[DIM][DIM],
                                          double lam, double mu, double (&S)[DIM][DIM])
{
    if constexpr (FORM == FEM_ELASTICITY) {
        stress_elasticity<DIM>(G, lam, mu, S);
    } else if constexpr (FORM == FEM_NEOHOOKEAN) {
        if constexpr (VJP) tangent_neohookean<DIM>(G, H, lam, mu, S);
        else stress_neohookean<DIM>(G, lam, mu, S);
    } else {
        static_assert(FORM == FEM_SVK, "vector form");
        if constexpr (VJP) tangent_svk<DIM>(G, H, lam, mu, S);
        else stress_svk<DIM>(G, lam, mu, S);
    }
}

// The quadrature loop of one cell: evaluation of u (and v) at each point from the
// tabulation, the pointwise form, and accumulation into yl against the test functions.
// The tabulation address is uniform across the wavefront (constant address space), so its
// values arrive through scalar loads.  GEO = 2: P2-geometry cells, whose K and |det J|
// are evaluated at every point from the geometry nodes gx (unused for GEO = 1, where the
// cell's constant Kinv and adet hold).
template <int FORM, int DIM, int K, bool VJP, int GEO = 1>
__device__ __forceinline__ void cell_quadrature(
    const double (&ul)[nloc_of(DIM, K)][ncomp_of(FORM, DIM)],
    const double (&vl)[VJP ? nloc_of(DIM, K) : 1][ncomp_of(FORM, DIM)],
    const double (&Kinv)[DIM][DIM], double adet, const double (&gx)[geom_nodes(DIM, GEO)][DIM],
    const double *table, int nq, double lam, double mu,
    double (&yl)[nloc_of(DIM, K)][ncomp_of(FORM, DIM)])
{
    constexpr int NLOC = nloc_of(DIM, K);
    constexpr int REC = record_of(FORM, DIM, NLOC, GEO);
    constexpr int GOFF = record_base(FORM, DIM, NLOC);      // geometry gradients (GEO = 2)
    const FEMX_CONSTANT double *tab = (const FEMX_CONSTANT double *)table;
    if constexpr (FORM == FEM_MASS) {
#pragma unroll
        for (int n = 0; n < NLOC; ++n) yl[n][0] = 0.0;
#pragma unroll 1
        for (int q = 0; q < nq; ++q) {
            const FEMX_CONSTANT double *t = tab + q * REC;
            double Kq[DIM][DIM];
            const double adq = point_geometry<DIM, GEO>(t + GOFF, gx, Kinv, adet, Kq);
            double uq = 0.0;
#pragma unroll
            for (int n = 0; n < NLOC; ++n) uq = fma(t[n], ul[n][0], uq);
            const double e = t[NLOC] * adq * uq;
#pragma unroll
            for (int n = 0; n < NLOC; ++n) yl[n][0] = fma(t[n], e, yl[n][0]);
        }
    } else if constexpr (FORM == FEM_LAPLACE || FORM == FEM_HELMHOLTZ) {
        // record: [phi_a (Helmholtz only); d phi_a / d xi_r, r-major; w]
        constexpr int D0 = FORM == FEM_HELMHOLTZ ? NLOC : 0;
        // K K^T maps reference derivatives of u to the flux against reference test
        // derivatives: grad phi_a . grad u = sum_rs dref_r phi_a (K K^T)_rs dref_s u
        auto kkt = [](const double (&Km)[DIM][DIM], double (&KKt)[DIM][DIM]) {
#pragma unroll
            for (int r = 0; r < DIM; ++r)
#pragma unroll
                for (int s2 = 0; s2 < DIM; ++s2) {
                    double acc = 0.0;
#pragma unroll
                    for (int j = 0; j < DIM; ++j) acc = fma(Km[r][j], Km[s2][j], acc);
                    KKt[r][s2] = acc;
                }
        };
        double KKc[DIM][DIM];       // the affine cell's constant K K^T
        if constexpr (GEO == 1) kkt(Kinv, KKc);
#pragma unroll
        for (int n = 0; n < NLOC; ++n) yl[n][0] = 0.0;
#pragma unroll 1
        for (int q = 0; q < nq; ++q) {
            const FEMX_CONSTANT double *t = tab + q * REC;
            double Kq[DIM][DIM], KKt[DIM][DIM];
            const double adq = point_geometry<DIM, GEO>(t + GOFF, gx, Kinv, adet, Kq);
            if constexpr (GEO == 2) {
                kkt(Kq, KKt);
            } else {
#pragma unroll
                for (int r = 0; r < DIM; ++r)
#pragma unroll
                    for (int s2 = 0; s2 < DIM; ++s2) KKt[r][s2] = KKc[r][s2];
            }
            double g[DIM];
#pragma unroll
            for (int r = 0; r < DIM; ++r) {
                double acc = 0.0;
#pragma unroll
                for (int n = 0; n < NLOC; ++n) acc = fma(t[D0 + r * NLOC + n], ul[n][0], acc);
                g[r] = acc;
            }
            const double W = t[D0 + DIM * NLOC] * adq;
            double f[DIM];
#pragma unroll
            for (int r = 0; r < DIM; ++r) {
                double acc = 0.0;
#pragma unroll
                for (int s2 = 0; s2 < DIM; ++s2) acc = fma(KKt[r][s2], g[s2], acc);
                f[r] = W * acc;
            }
            double e = 0.0;
            if constexpr (FORM == FEM_HELMHOLTZ) {
                double uq = 0.0;
#pragma unroll
                for (int n = 0; n < NLOC; ++n) uq = fma(t[n], ul[n][0], uq);
                e = W * uq;
            }
#pragma unroll
            for (int n = 0; n < NLOC; ++n) {
                double acc = yl[n][0];
                if constexpr (FORM == FEM_HELMHOLTZ) acc = fma(t[n], e, acc);
#pragma unroll
                for (int r = 0; r < DIM; ++r) acc = fma(t[D0 + r * NLOC + n], f[r], acc);
                yl[n][0] = acc;
            }
        }
    } else {
#pragma unroll
        for (int n = 0; n < NLOC; ++n)
#pragma unroll
            for (int c = 0; c < DIM; ++c) yl[n][c] = 0.0;
        auto point = [&](int q) {
            const FEMX_CONSTANT double *t = tab + q * REC;
            double Kq[DIM][DIM];
            const double adq = point_geometry<DIM, GEO>(t + GOFF, gx, Kinv, adet, Kq);
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
            double G[DIM][DIM], H[DIM][DIM], S[DIM][DIM], T[DIM][DIM];
            to_physical<DIM>(gu, Kq, G);
            if constexpr (VJP) to_physical<DIM>(gv, Kq, H);
            pointwise<FORM, DIM, VJP>(G, H, lam, mu, S);
            pull_back<DIM>(S, Kq, t[DIM * NLOC] * adq, T);
#pragma unroll
            for (int n = 0; n < NLOC; ++n)
#pragma unroll
                for (int r = 0; r < DIM; ++r) {
                    const double tr = t[r * NLOC + n];
#pragma unroll
                    for (int c = 0; c < DIM; ++c) yl[n][c] = fma(tr, T[c][r], yl[n][c]);
                }
        };
        // Two points per trip give the scheduler two independent pointwise chains (the
        // log and reciprocal sequences are long serial dependences) where the cell's
        // values and outputs leave room: affine forward actions with at most 42 of them.
        // Larger cells, curved cells and the VJP run one point per trip, and so does P2
        // tetrahedral elasticity: its linear law is a short chain, and the second point's
        // registers would spill under that kernel's three-wave bound (28 bytes per lane).
        if constexpr (!VJP && GEO == 1 && NLOC * DIM <= 42 &&
                      !(FORM == FEM_ELASTICITY && DIM == 3 && K == 2)) {
#pragma unroll 2
            for (int q = 0; q < nq; ++q) point(q);
        } else {
#pragma unroll 1
            for (int q = 0; q < nq; ++q) point(q);
        }
    }
}

// Exchange a double with the neighbouring lane of the pair (lanes 2i <-> 2i+1) through
// DPP quad permutation [1,0,3,2]; both lanes of a pair must be active.
__device__ __forceinline__ double pair_swap(double x)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0xB1, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0xB1, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// The 2D vector forms with the two components of a cell on a lane pair: lane c holds
// component c of the cell's values and output, evaluates row c of the reference gradient,
// swaps rows with its partner, evaluates the (whole) pointwise form, and accumulates the
// row c of the stress against the test gradients.
template <int FORM, int K, bool VJP>
__device__ __forceinline__ void cell_quadrature_pair(
    const double (&ul)[nloc_of(2, K)], const double (&vl)[VJP ? nloc_of(2, K) : 1], int c,
    const double (&Kinv)[2][2], double adet, const double *table, int nq, double lam,
    double mu, double (&yl)[nloc_of(2, K)])
{
    constexpr int NLOC = nloc_of(2, K);
    constexpr int REC = record_of(FORM, 2, NLOC);
    const FEMX_CONSTANT double *tab = (const FEMX_CONSTANT double *)table;
    const bool odd = c != 0;
#pragma unroll
    for (int n = 0; n < NLOC; ++n) yl[n] = 0.0;
#pragma unroll 1
    for (int q = 0; q < nq; ++q) {
        const FEMX_CONSTANT double *t = tab + q * REC;
        double g0 = 0.0, g1 = 0.0, h0 = 0.0, h1 = 0.0;
#pragma unroll
        for (int n = 0; n < NLOC; ++n) {
            g0 = fma(t[n], ul[n], g0);
            g1 = fma(t[NLOC + n], ul[n], g1);
            if constexpr (VJP) {
                h0 = fma(t[n], vl[n], h0);
                h1 = fma(t[NLOC + n], vl[n], h1);
            }
        }
        // rows of the reference gradient: this lane's row c and the partner's row 1 - c
        const double o0 = pair_swap(g0), o1 = pair_swap(g1);
        double gu[2][2], G[2][2], H[2][2], S[2][2], T[2][2];
        gu[0][0] = odd ? o0 : g0;
        gu[0][1] = odd ? o1 : g1;
        gu[1][0] = odd ? g0 : o0;
        gu[1][1] = odd ? g1 : o1;
        to_physical<2>(gu, Kinv, G);
        if constexpr (VJP) {
            const double p0 = pair_swap(h0), p1 = pair_swap(h1);
            double gv[2][2];
            gv[0][0] = odd ? p0 : h0;
            gv[0][1] = odd ? p1 : h1;
            gv[1][0] = odd ? h0 : p0;
            gv[1][1] = odd ? h1 : p1;
            to_physical<2>(gv, Kinv, H);
        }
        pointwise<FORM, 2, VJP>(G, H, lam, mu, S);
        pull_back<2>(S, Kinv, t[2 * NLOC] * adet, T);
        const double t0 = odd ? T[1][0] : T[0][0];
        const double t1 = odd ? T[1][1] : T[0][1];
#pragma unroll
        for (int n = 0; n < NLOC; ++n) yl[n] = fma(t[n], t0, fma(t[NLOC + n], t1, yl[n]));
    }
}

// The 3D vector forms with the three components of a cell on a lane triple (lanes 3g,
// 3g+1, 3g+2 of a wavefront; `base` = 3g): lane c holds component c, evaluates row c of the
// reference gradient, gathers the three rows from the triple by lane shuffles, evaluates
// the (whole) pointwise form and accumulates row c of the stress.  Curved cells (GEO = 2):
// lane c holds coordinate c of the ten geometry nodes (gxc) and evaluates row c of J at each
// point, the triple exchanging the rows as it does the gradient's; K and |det J| then come
// per point from the whole J on every lane.
template <int FORM, int K, bool VJP, int GEO = 1>
__device__ __forceinline__ void cell_quadrature_triple(
    const double (&ul)[nloc_of(3, K)], const double (&vl)[VJP ? nloc_of(3, K) : 1], int c,
    int base, const double (&Kinv)[3][3], double adet,
    const double (&gxc)[GEO == 2 ? geom_nodes(3, 2) : 1], const double *table, int nq,
    double lam, double mu, double (&yl)[nloc_of(3, K)])
{
    constexpr int NLOC = nloc_of(3, K);
    constexpr int REC = record_of(FORM, 3, NLOC, GEO);
    constexpr int GOFF = record_base(FORM, 3, NLOC);      // geometry gradients (GEO = 2)
    const FEMX_CONSTANT double *tab = (const FEMX_CONSTANT double *)table;
#pragma unroll
    for (int n = 0; n < NLOC; ++n) yl[n] = 0.0;
#pragma unroll 1
    for (int q = 0; q < nq; ++q) {
        const FEMX_CONSTANT double *t = tab + q * REC;
        double g[3] = {0.0, 0.0, 0.0}, h[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int n = 0; n < NLOC; ++n)
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                g[r] = fma(t[r * NLOC + n], ul[n], g[r]);
                if constexpr (VJP) h[r] = fma(t[r * NLOC + n], vl[n], h[r]);
            }
        double gu[3][3], gv[3][3], G[3][3], S[3][3], T[3][3];
#pragma unroll
        for (int row = 0; row < 3; ++row)
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                gu[row][r] = __shfl(g[r], base + row);
                if constexpr (VJP) gv[row][r] = __shfl(h[r], base + row);
            }
        double Kq[3][3], adq = adet;
        if constexpr (GEO == 2) {
            constexpr int NG = geom_nodes(3, 2);
            const FEMX_CONSTANT double *tg = t + GOFF;
            double jr[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                double acc = 0.0;
#pragma unroll
                for (int gn = 0; gn < NG; ++gn) acc = fma(gxc[gn], tg[r * NG + gn], acc);
                jr[r] = acc;
            }
            double J[3][3];
#pragma unroll
            for (int row = 0; row < 3; ++row)
#pragma unroll
                for (int r = 0; r < 3; ++r) J[row][r] = __shfl(jr[r], base + row);
            adq = jacobian_inverse<3>(J, Kq);
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) Kq[i][j] = Kinv[i][j];
        }
        to_physical<3>(gu, Kq, G);
        double H[3][3];
        if constexpr (VJP) to_physical<3>(gv, Kq, H);
        pointwise<FORM, 3, VJP>(G, H, lam, mu, S);
        pull_back<3>(S, Kq, t[3 * NLOC] * adq, T);
        double tc[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) tc[r] = c == 0 ? T[0][r] : (c == 1 ? T[1][r] : T[2][r]);
#pragma unroll
        for (int n = 0; n < NLOC; ++n)
            yl[n] = fma(t[n], tc[0], fma(t[NLOC + n], tc[1], fma(t[2 * NLOC + n], tc[2], yl[n])));
    }
}

}  // namespace femx

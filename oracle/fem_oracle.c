/*
 * Oracle: plain, slow, FP64 CPU loops for the matrix-free finite element action.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load this library.  It shares no code with the GPU library.
 *
 * Structure: the generic action kernel of the paper (Sec. 2.3, the generic action
 * algorithm): for every cell, in index order,
 *   gather the geometry nodes' coordinates and the cell's DoFs through the maps,
 *   for every quadrature point:
 *     Jacobian of the cell map x(xi) = sum_g x_g phiG_g(xi) at the point and its
 *     determinant (affine cells: phiG = P1 on the vertices, J = [x_1 - x_0 | ... | x_d - x_0]
 *     at every point; curved cells: P2 geometry, J varies over the cell, Sec. 2.4),
 *     evaluation: reference derivatives of u at the point from the tabulation,
 *     apply the form's pointwise map and the geometry (J^{-1}, |det J|, weight),
 *     quadrature: accumulate against the test-function tabulation,
 *   scatter-add the cell vector into the global vector.
 * The integrand uses J^{-T} grad_ref and |det J| (Sec. 2.2, substituted-integrand eq.).
 *
 * Forms (App. A): 0 mass  a = int u v;
 *   1 linear elasticity  sigma = lam tr(eps) I + 2 mu eps,  a = int sigma(u) : eps(v);
 *   2 compressible neo-Hookean residual (the paper's hyperelastic residual with the
 *     neo-Hookean energy Psi = mu/2 (tr F^T F - d) - mu ln J + lam/2 (ln J)^2 in place of
 *     St Venant-Kirchhoff, body force 0):  r = int P(F) : grad v,
 *     F = I + grad u,  P = dPsi/dF = mu (F - F^{-T}) + lam ln(det F) F^{-T};
 *   3 St Venant-Kirchhoff residual (the paper's hyperelastic law, App. A): E = (F^T F - I)/2,
 *     S = lam tr(E) I + 2 mu E, P = F S (energy Psi = lam/2 tr(E)^2 + mu E:E);
 *   4 Laplace  a = int grad u . grad v;   5 Helmholtz  a = int grad u . grad v + u v.
 *
 * Layouts: coords [n_vert][d] (geometry nodes); cell_verts [n_cell][ng] (each cell's ng
 * geometry nodes: d+1 vertices, or the P2 lattice); cell_nodes [n_cell][nloc];
 * vectors node-major interleaved, value (node, c) at node*ncomp + c;
 * phi [nq][nloc]; dphi [nq][nloc][d]; w [nq]; gdphi [nq][ng][d] (geometry basis).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

enum { OR_MASS = 0, OR_ELAST = 1, OR_NH = 2, OR_SVK = 3, OR_LAPLACE = 4, OR_HELMHOLTZ = 5 };

/* largest local node count handled (P8 triangle: 45, P6 tetrahedron: 84) */
#define ORACLE_MAX_NLOC 128
/* largest geometry node count (P2 tetrahedron) */
#define ORACLE_MAX_GEOM 10

/* determinant and inverse of a d x d matrix (d = 2, 3) */
static double inverse(int d, const double A[3][3], double B[3][3])
{
    double det;
    if (d == 2) {
        det = A[0][0] * A[1][1] - A[0][1] * A[1][0];
        B[0][0] = A[1][1] / det;
        B[0][1] = -A[0][1] / det;
        B[1][0] = -A[1][0] / det;
        B[1][1] = A[0][0] / det;
    } else {
        det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
            - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
            + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
        B[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
        B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
        B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
        B[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
        B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
        B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
        B[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
        B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
        B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
    }
    return det;
}

/* The cell map's Jacobian at one point, J[i][r] = sum_g x_g,i d phiG_g / d xi_r, from the
 * geometry basis' reference gradients there (gdq [ng][d]); returns det J and writes
 * K = J^{-1} (K[r][i]). */
static double geometry(int d, int ng, const double x[][3], const double *gdq, double J[3][3],
                       double K[3][3])
{
    for (int i = 0; i < d; ++i)
        for (int r = 0; r < d; ++r) {
            J[i][r] = 0.0;
            for (int g = 0; g < ng; ++g)
                J[i][r] += x[g][i] * gdq[g * d + r];
        }
    return inverse(d, J, K);
}

/* physical gradient G[c][j] = sum_a u[a][c] dphi_j(a), with dphi_j = sum_r K[r][j] dref_r */
static void physical_gradient(int d, int nloc, const double *dphi_q, const double K[3][3],
                              const double *uloc, double G[3][3])
{
    double gref[3][3] = {{0}};
    for (int a = 0; a < nloc; ++a)
        for (int c = 0; c < d; ++c)
            for (int r = 0; r < d; ++r)
                gref[c][r] += dphi_q[a * d + r] * uloc[a * d + c];
    for (int c = 0; c < d; ++c)
        for (int j = 0; j < d; ++j) {
            G[c][j] = 0.0;
            for (int r = 0; r < d; ++r)
                G[c][j] += gref[c][r] * K[r][j];
        }
}

/* first Piola-Kirchhoff stress of the forms (elasticity: Cauchy stress sigma) */
static void stress(int form, int d, double lam, double mu, const double G[3][3],
                   double S[3][3])
{
    if (form == OR_ELAST) {
        double tr = 0.0;
        for (int i = 0; i < d; ++i)
            tr += G[i][i];
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                double eps = 0.5 * (G[i][j] + G[j][i]);
                S[i][j] = 2.0 * mu * eps + (i == j ? lam * tr : 0.0);
            }
    } else if (form == OR_NH) {
        double F[3][3], Fi[3][3];
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j)
                F[i][j] = (i == j ? 1.0 : 0.0) + G[i][j];
        double detF = inverse(d, F, Fi);
        double lnJ = log(detF);
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                double FiT = Fi[j][i];
                S[i][j] = mu * (F[i][j] - FiT) + lam * lnJ * FiT;
            }
    } else { /* St Venant-Kirchhoff */
        double F[3][3], E[3][3], S2[3][3], trE = 0.0;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j)
                F[i][j] = (i == j ? 1.0 : 0.0) + G[i][j];
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                double c = 0.0;
                for (int k = 0; k < d; ++k)
                    c += F[k][i] * F[k][j];
                E[i][j] = 0.5 * (c - (i == j ? 1.0 : 0.0));
            }
        for (int i = 0; i < d; ++i)
            trE += E[i][i];
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j)
                S2[i][j] = 2.0 * mu * E[i][j] + (i == j ? lam * trE : 0.0);
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                S[i][j] = 0.0;
                for (int k = 0; k < d; ++k)
                    S[i][j] += F[i][k] * S2[k][j];
            }
    }
}

/* strain energy density of the hyperelastic forms */
static double energy_density(int form, int d, double lam, double mu, const double G[3][3])
{
    double F[3][3], Fi[3][3];
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            F[i][j] = (i == j ? 1.0 : 0.0) + G[i][j];
    if (form == OR_SVK) {
        double E[3][3], trE = 0.0, EE = 0.0;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                double c = 0.0;
                for (int k = 0; k < d; ++k)
                    c += F[k][i] * F[k][j];
                E[i][j] = 0.5 * (c - (i == j ? 1.0 : 0.0));
            }
        for (int i = 0; i < d; ++i) {
            trE += E[i][i];
            for (int j = 0; j < d; ++j)
                EE += E[i][j] * E[i][j];
        }
        return 0.5 * lam * trE * trE + mu * EE;
    }
    double detF = inverse(d, F, Fi);
    double lnJ = log(detF);
    double trC = 0.0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            trC += F[i][j] * F[i][j];
    return 0.5 * mu * (trC - d) - mu * lnJ + 0.5 * lam * lnJ * lnJ;
}

static void gather_cell(int d, int ng, int nloc, int ncomp, int64_t cell,
                        const int32_t *cell_verts, const double *coords,
                        const int32_t *cell_nodes, const double *vec, double x[][3], double *loc)
{
    for (int j = 0; j < ng; ++j)
        for (int i = 0; i < d; ++i)
            x[j][i] = coords[(int64_t)cell_verts[cell * ng + j] * d + i];
    for (int a = 0; a < nloc; ++a)
        for (int c = 0; c < ncomp; ++c)
            loc[a * ncomp + c] = vec[(int64_t)cell_nodes[cell * nloc + a] * ncomp + c];
}

/* y = A(u), overwriting y [n_dof]. */
void oracle_action(int form, int d, int nloc, int nq, const double *phi, const double *dphi,
                   const double *w, int ng, const double *gdphi, int64_t n_cell,
                   const int32_t *cell_verts, const double *coords, const int32_t *cell_nodes,
                   double lam, double mu, const double *u, double *y, int64_t n_dof)
{
    const int scalar = form == OR_MASS || form == OR_LAPLACE || form == OR_HELMHOLTZ;
    const int ncomp = scalar ? 1 : d;
    double uloc[ORACLE_MAX_NLOC * 3], out[ORACLE_MAX_NLOC * 3];
    memset(y, 0, sizeof(double) * (size_t)n_dof);
    for (int64_t cell = 0; cell < n_cell; ++cell) {
        double x[ORACLE_MAX_GEOM][3], J[3][3], K[3][3];
        gather_cell(d, ng, nloc, ncomp, cell, cell_verts, coords, cell_nodes, u, x, uloc);
        for (int i = 0; i < nloc * ncomp; ++i)
            out[i] = 0.0;
        for (int q = 0; q < nq; ++q) {
            double detJ = fabs(geometry(d, ng, x, gdphi + (int64_t)q * ng * d, J, K));
            const double W = w[q] * detJ;
            if (form == OR_MASS || form == OR_HELMHOLTZ) {
                double uq = 0.0;
                for (int a = 0; a < nloc; ++a)
                    uq += phi[q * nloc + a] * uloc[a];
                double e = W * uq;
                for (int a = 0; a < nloc; ++a)
                    out[a] += phi[q * nloc + a] * e;
            }
            if (form == OR_LAPLACE || form == OR_HELMHOLTZ) {
                /* physical gradients: grad phi_a = K^T grad_ref phi_a, grad u_h = sum_a u_a grad phi_a */
                const double *dq = dphi + (int64_t)q * nloc * d;
                double gu[3] = {0.0, 0.0, 0.0};
                for (int a = 0; a < nloc; ++a)
                    for (int j = 0; j < d; ++j)
                        for (int r = 0; r < d; ++r)
                            gu[j] += uloc[a] * dq[a * d + r] * K[r][j];
                for (int a = 0; a < nloc; ++a)
                    for (int j = 0; j < d; ++j) {
                        double gphi = 0.0;
                        for (int r = 0; r < d; ++r)
                            gphi += dq[a * d + r] * K[r][j];
                        out[a] += W * gphi * gu[j];
                    }
            } else if (form != OR_MASS && form != OR_HELMHOLTZ) {
                double G[3][3], S[3][3], E[3][3];
                const double *dq = dphi + (int64_t)q * nloc * d;
                physical_gradient(d, nloc, dq, K, uloc, G);
                stress(form, d, lam, mu, G, S);
                /* e[c][r] = W sum_j S[c][j] K[r][j]: test derivatives in reference form */
                for (int c = 0; c < d; ++c)
                    for (int r = 0; r < d; ++r) {
                        E[c][r] = 0.0;
                        for (int j = 0; j < d; ++j)
                            E[c][r] += S[c][j] * K[r][j];
                        E[c][r] *= W;
                    }
                for (int a = 0; a < nloc; ++a)
                    for (int c = 0; c < d; ++c)
                        for (int r = 0; r < d; ++r)
                            out[a * d + c] += dq[a * d + r] * E[c][r];
            }
        }
        for (int a = 0; a < nloc; ++a)
            for (int c = 0; c < ncomp; ++c)
                y[(int64_t)cell_nodes[cell * nloc + a] * ncomp + c] += out[a * ncomp + c];
    }
}

/*
 * g = (dA/du)^T v for the hyperelastic residuals, overwriting g.
 * Written literally as the transpose: with the tangent C_ijkl = dP_ij / dF_kl,
 * g_(b,k) = sum_q W_q sum_l dphi_l(b) sum_ij H_ij C_ijkl,   H = grad v_h,
 *   neo-Hookean:  C_ijkl = mu d_ik d_jl + (mu - lam ln J) Finv_jk Finv_li + lam Finv_ji Finv_lk;
 *   St Venant-Kirchhoff (P = F S):  C_ijkl = d_ik S_lj + lam F_ij F_kl + mu F_il F_kj
 *                                            + mu (F F^T)_ik d_jl.
 * For the linear forms (mass, elasticity) A is symmetric and linear: g = A v.
 */
void oracle_vjp(int form, int d, int nloc, int nq, const double *phi, const double *dphi,
                const double *w, int ng, const double *gdphi, int64_t n_cell,
                const int32_t *cell_verts, const double *coords, const int32_t *cell_nodes,
                double lam, double mu, const double *u, const double *v, double *g,
                int64_t n_dof)
{
    if (form != OR_NH && form != OR_SVK) {
        oracle_action(form, d, nloc, nq, phi, dphi, w, ng, gdphi, n_cell, cell_verts, coords,
                      cell_nodes, lam, mu, v, g, n_dof);
        return;
    }
    double uloc[ORACLE_MAX_NLOC * 3], vloc[ORACLE_MAX_NLOC * 3], out[ORACLE_MAX_NLOC * 3];
    memset(g, 0, sizeof(double) * (size_t)n_dof);
    for (int64_t cell = 0; cell < n_cell; ++cell) {
        double x[ORACLE_MAX_GEOM][3], J[3][3], K[3][3];
        gather_cell(d, ng, nloc, d, cell, cell_verts, coords, cell_nodes, u, x, uloc);
        gather_cell(d, ng, nloc, d, cell, cell_verts, coords, cell_nodes, v, x, vloc);
        for (int i = 0; i < nloc * d; ++i)
            out[i] = 0.0;
        for (int q = 0; q < nq; ++q) {
            double detJ = fabs(geometry(d, ng, x, gdphi + (int64_t)q * ng * d, J, K));
            const double W = w[q] * detJ;
            const double *dq = dphi + (int64_t)q * nloc * d;
            double G[3][3], H[3][3], F[3][3], Fi[3][3], D[3][3], E[3][3];
            physical_gradient(d, nloc, dq, K, uloc, G);
            physical_gradient(d, nloc, dq, K, vloc, H);
            for (int i = 0; i < d; ++i)
                for (int j = 0; j < d; ++j)
                    F[i][j] = (i == j ? 1.0 : 0.0) + G[i][j];
            double lnJ = 0.0, S2[3][3], FFt[3][3];
            if (form == OR_NH) {
                lnJ = log(inverse(d, F, Fi));
            } else {
                double trE = 0.0;
                for (int i = 0; i < d; ++i)
                    for (int j = 0; j < d; ++j) {
                        double c = 0.0, b = 0.0;
                        for (int k = 0; k < d; ++k) {
                            c += F[k][i] * F[k][j];
                            b += F[i][k] * F[j][k];
                        }
                        S2[i][j] = mu * (c - (i == j ? 1.0 : 0.0));   /* 2 mu E */
                        FFt[i][j] = b;
                        if (i == j)
                            trE += 0.5 * (c - 1.0);
                    }
                for (int i = 0; i < d; ++i)
                    S2[i][i] += lam * trE;
            }
            for (int k = 0; k < d; ++k)
                for (int l = 0; l < d; ++l) {
                    double s = 0.0;
                    for (int i = 0; i < d; ++i)
                        for (int j = 0; j < d; ++j) {
                            double C;
                            if (form == OR_NH)
                                C = ((i == k && j == l) ? mu : 0.0)
                                  + (mu - lam * lnJ) * Fi[j][k] * Fi[l][i]
                                  + lam * Fi[j][i] * Fi[l][k];
                            else
                                C = (i == k ? S2[l][j] : 0.0) + lam * F[i][j] * F[k][l]
                                  + mu * F[i][l] * F[k][j] + (j == l ? mu * FFt[i][k] : 0.0);
                            s += H[i][j] * C;
                        }
                    D[k][l] = s;
                }
            for (int c = 0; c < d; ++c)
                for (int r = 0; r < d; ++r) {
                    E[c][r] = 0.0;
                    for (int j = 0; j < d; ++j)
                        E[c][r] += D[c][j] * K[r][j];
                    E[c][r] *= W;
                }
            for (int a = 0; a < nloc; ++a)
                for (int c = 0; c < d; ++c)
                    for (int r = 0; r < d; ++r)
                        out[a * d + c] += dq[a * d + r] * E[c][r];
        }
        for (int a = 0; a < nloc; ++a)
            for (int c = 0; c < d; ++c)
                g[(int64_t)cell_nodes[cell * nloc + a] * d + c] += out[a * d + c];
    }
}

/* discrete energy of a hyperelastic form  Pi_h(u) = sum_T sum_q w_q |det J| Psi(F_q) */
double oracle_energy(int form, int d, int nloc, int nq, const double *dphi, const double *w,
                     int ng, const double *gdphi, int64_t n_cell, const int32_t *cell_verts,
                     const double *coords, const int32_t *cell_nodes, double lam, double mu,
                     const double *u)
{
    double uloc[ORACLE_MAX_NLOC * 3], total = 0.0;
    for (int64_t cell = 0; cell < n_cell; ++cell) {
        double x[ORACLE_MAX_GEOM][3], J[3][3], K[3][3];
        gather_cell(d, ng, nloc, d, cell, cell_verts, coords, cell_nodes, u, x, uloc);
        for (int q = 0; q < nq; ++q) {
            double detJ = fabs(geometry(d, ng, x, gdphi + (int64_t)q * ng * d, J, K));
            double G[3][3];
            physical_gradient(d, nloc, dphi + (int64_t)q * nloc * d, K, uloc, G);
            total += w[q] * detJ * energy_density(form, d, lam, mu, G);
        }
    }
    return total;
}

/* minimum over cells and quadrature points of det F (neo-Hookean admissibility) */
double oracle_min_det_f(int d, int nloc, int nq, const double *dphi, int ng,
                        const double *gdphi, int64_t n_cell, const int32_t *cell_verts,
                        const double *coords, const int32_t *cell_nodes, const double *u)
{
    double uloc[ORACLE_MAX_NLOC * 3], mn = INFINITY;
    for (int64_t cell = 0; cell < n_cell; ++cell) {
        double x[ORACLE_MAX_GEOM][3], J[3][3], K[3][3], G[3][3], F[3][3], Fi[3][3];
        gather_cell(d, ng, nloc, d, cell, cell_verts, coords, cell_nodes, u, x, uloc);
        for (int q = 0; q < nq; ++q) {
            geometry(d, ng, x, gdphi + (int64_t)q * ng * d, J, K);
            physical_gradient(d, nloc, dphi + (int64_t)q * nloc * d, K, uloc, G);
            for (int i = 0; i < d; ++i)
                for (int j = 0; j < d; ++j)
                    F[i][j] = (i == j ? 1.0 : 0.0) + G[i][j];
            double det = inverse(d, F, Fi);
            if (det < mn)
                mn = det;
        }
    }
    return mn;
}

/* Greedy first-fit colouring, cells in ascending id: the colour of a cell is the
 * smallest colour not used by an already-coloured cell sharing a node with it.
 * colour [n_cell] out; masks [n_node * nwords] zeroed by the caller (bit c of node n set
 * once a cell of colour c holds n).  Returns the number of colours, -1 past 64*nwords. */
int oracle_colouring(int64_t n_cell, int nloc, const int32_t *cell_nodes, int nwords,
                     int32_t *colour, uint64_t *masks)
{
    int ncol = 0;
    for (int64_t cell = 0; cell < n_cell; ++cell) {
        int c = 0;
        for (;; ++c) {
            if (c >= 64 * nwords)
                return -1;
            int used = 0;
            for (int a = 0; a < nloc; ++a) {
                int64_t nd = cell_nodes[cell * nloc + a];
                if ((masks[nd * nwords + c / 64] >> (c % 64)) & 1u) {
                    used = 1;
                    break;
                }
            }
            if (!used)
                break;
        }
        colour[cell] = c;
        for (int a = 0; a < nloc; ++a) {
            int64_t nd = cell_nodes[cell * nloc + a];
            masks[nd * nwords + c / 64] |= (uint64_t)1 << (c % 64);
        }
        if (c + 1 > ncol)
            ncol = c + 1;
    }
    return ncol;
}

// Reference-element data: quadrature on the reference simplex and the P_k Lagrange
// tabulation (paper Sec. 2.2: quadrature replacement of the cell integral and the
// tabulated basis derivatives at the quadrature nodes).
//
// Quadrature: the conical-product rule in collapsed coordinates.  The 1D factors are
// Gauss-Jacobi rules for the weights (1-t)^a on [0,1] (a = 0, 1 for triangles; 0, 1, 2
// for tetrahedra); their nodes are the roots of the Jacobi polynomial P_n^(a,0), found
// here by bracketing sign changes on a Chebyshev grid and bisection, with the weights
// from the closed-form Christoffel numbers.
//
// Basis: equispaced P_k Lagrange in barycentric product form; the derivative of each
// factor product is carried along the product recurrence.
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

namespace femx {
namespace {

// P_n^(a,b)(x) by the three-term recurrence.
double jacobi_p(int n, double a, double b, double x)
{
    if (n == 0) return 1.0;
    double p0 = 1.0;
    double p1 = 0.5 * ((a + b + 2.0) * x + (a - b));
    for (int m = 2; m <= n; ++m) {
        const double s = 2.0 * m + a + b;
        const double c1 = 2.0 * m * (m + a + b) * (s - 2.0);
        const double c2 = (s - 1.0) * (a * a - b * b);
        const double c3 = (s - 2.0) * (s - 1.0) * s;
        const double c4 = 2.0 * (m + a - 1.0) * (m + b - 1.0) * s;
        const double p2 = ((c2 + c3 * x) * p1 - c4 * p0) / c1;
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

// d/dx P_n^(a,b) = (n + a + b + 1)/2 P_{n-1}^(a+1,b+1)
double jacobi_dp(int n, double a, double b, double x)
{
    if (n == 0) return 0.0;
    return 0.5 * (n + a + b + 1.0) * jacobi_p(n - 1, a + 1.0, b + 1.0, x);
}

// n-point Gauss-Jacobi rule for the weight (1-t)^a on [0, 1].
void gauss_jacobi01(int n, int a, std::vector<double> &t, std::vector<double> &w)
{
    const double A = a, B = 0.0;
    std::vector<double> roots;
    const int M = 256 * n * n + 64;
    double xl = -1.0, fl = jacobi_p(n, A, B, xl);
    for (int j = 1; j <= M && (int)roots.size() < n; ++j) {
        const double xr = -std::cos(M_PI * j / M);
        const double fr = jacobi_p(n, A, B, xr);
        if (fr == 0.0 || (fl < 0) != (fr < 0)) {
            double lo = xl, hi = xr, flo = fl;
            for (int it = 0; it < 200 && hi - lo > 0; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                const double fm = jacobi_p(n, A, B, mid);
                if (fm == 0.0) { lo = hi = mid; break; }
                if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
            }
            double x = 0.5 * (lo + hi);
            for (int it = 0; it < 2; ++it) {         // Newton polish
                const double d = jacobi_dp(n, A, B, x);
                if (d != 0.0) {
                    const double xn = x - jacobi_p(n, A, B, x) / d;
                    if (xn > lo - (hi - lo) && xn < hi + (hi - lo)) x = xn;
                }
            }
            roots.push_back(x);
        }
        xl = xr;
        fl = fr;
    }
    if ((int)roots.size() != n)
        throw Error(FEM_E_UNSUPPORTED, "Gauss-Jacobi root search failed");
    // Christoffel numbers: 2^(a+b+1) G(n+a+1) G(n+b+1) / (G(n+a+b+1) n!) / ((1-x^2) P_n'(x)^2)
    const double lc = (A + B + 1.0) * std::log(2.0) + std::lgamma(n + A + 1.0) +
                      std::lgamma(n + B + 1.0) - std::lgamma(n + A + B + 1.0) -
                      std::lgamma(n + 1.0);
    const double c = std::exp(lc);
    t.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        const double x = roots[i];
        const double d = jacobi_dp(n, A, B, x);
        t[i] = 0.5 * (1.0 + x);
        w[i] = c / ((1.0 - x * x) * d * d) / std::pow(2.0, A + 1.0);
    }
}

void conical_rule(int dim, int degree, std::vector<double> &pts, std::vector<double> &wts)
{
    const int n = degree <= 0 ? 1 : (degree + 2) / 2;   // ceil((degree + 1) / 2)
    std::vector<double> s, ws, t, wt, z, wz;
    gauss_jacobi01(n, 0, s, ws);
    gauss_jacobi01(n, 1, t, wt);
    pts.clear();
    wts.clear();
    if (dim == 2) {
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                pts.push_back(s[i] * (1.0 - t[j]));
                pts.push_back(t[j]);
                wts.push_back(ws[i] * wt[j]);
            }
    } else {
        gauss_jacobi01(n, 2, z, wz);
        for (int l = 0; l < n; ++l)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    pts.push_back(s[i] * (1.0 - t[j]) * (1.0 - z[l]));
                    pts.push_back(t[j] * (1.0 - z[l]));
                    pts.push_back(z[l]);
                    wts.push_back(ws[i] * wt[j] * wz[l]);
                }
    }
}

// Fully symmetric rules of degree <= 2 from their moment equations (closed form).
//   degree <= 1: the centroid, weight |T|.
//   degree 2, triangle: the orbit of (a, b, b), a = 1 - 2b, weight |T|/3 each; matching
//     int lambda_1^2 = |T|/6 gives 6b^2 - 4b + 1/2 = 0, b = 1/6 (the interior root).
//   degree 2, tetrahedron: the orbit of (a, b, b, b), a = 1 - 3b, weight |T|/4 each;
//     int lambda_1^2 = |T|/10 gives 12b^2 - 6b + 3/5 = 0, b = (5 - sqrt 5)/20.
// Returns false when no such rule is built for (dim, degree).
bool symmetric_rule(int dim, int degree, std::vector<double> &pts, std::vector<double> &wts)
{
    pts.clear();
    wts.clear();
    const double vol = dim == 2 ? 0.5 : 1.0 / 6.0;
    if (degree <= 1) {
        for (int r = 0; r < dim; ++r) pts.push_back(1.0 / (dim + 1));
        wts.push_back(vol);
        return true;
    }
    if (degree != 2) return false;
    double b;
    if (dim == 2) {
        b = (4.0 - std::sqrt(16.0 - 12.0)) / 12.0;            // roots of 6b^2 - 4b + 1/2
    } else {
        b = (6.0 - std::sqrt(36.0 - 4.0 * 12.0 * 0.6)) / 24.0; // roots of 12b^2 - 6b + 3/5
    }
    const double a = 1.0 - dim * b;
    for (int k = 0; k <= dim; ++k) {          // the point with barycentric a in slot k
        for (int r = 0; r < dim; ++r) pts.push_back(r + 1 == k ? a : b);
        wts.push_back(vol / (dim + 1));
    }
    return true;
}

// reference lattice multi-indices, first coordinate fastest
std::vector<int> lattice(int dim, int k)
{
    std::vector<int> out;
    if (dim == 2) {
        for (int j = 0; j <= k; ++j)
            for (int i = 0; i + j <= k; ++i) {
                out.push_back(i);
                out.push_back(j);
            }
    } else {
        for (int l = 0; l <= k; ++l)
            for (int j = 0; j + l <= k; ++j)
                for (int i = 0; i + j + l <= k; ++i) {
                    out.push_back(i);
                    out.push_back(j);
                    out.push_back(l);
                }
    }
    return out;
}

// prod_{j<m} (k*lam - j)/(j+1) and its derivative, by the running product
void factor(int k, int m, double lam, double &f, double &df)
{
    f = 1.0;
    df = 0.0;
    for (int j = 0; j < m; ++j) {
        const double g = (k * lam - j) / (j + 1);
        df = df * g + f * (double)k / (j + 1);
        f *= g;
    }
}

}  // namespace

RefTables reference_tables(int dim, int degree, int quad_degree, int family)
{
    if (dim != 2 && dim != 3) throw Error(FEM_E_UNSUPPORTED, "dim must be 2 or 3");
    if (degree < 1 || degree > 8) throw Error(FEM_E_UNSUPPORTED, "degree out of range");
    if (quad_degree < 0 || quad_degree > 30)
        throw Error(FEM_E_UNSUPPORTED, "quadrature degree out of range");
    RefTables t;
    t.dim = dim;
    t.degree = degree;
    t.quad_degree = quad_degree;
    if (family == FEM_QUAD_SYMMETRIC) {
        if (!symmetric_rule(dim, quad_degree, t.points, t.weights))
            throw Error(FEM_E_UNSUPPORTED, "no symmetric rule of degree " + std::to_string(quad_degree));
    } else if (family == FEM_QUAD_CONICAL) {
        conical_rule(dim, quad_degree, t.points, t.weights);
    } else {
        throw Error(FEM_E_ARG, "unknown quadrature family");
    }
    t.nq = (int)t.weights.size();
    const std::vector<int> lat = lattice(dim, degree);
    t.nloc = (int)lat.size() / dim;
    t.phi.assign((size_t)t.nq * t.nloc, 0.0);
    t.dphi.assign((size_t)t.nq * t.nloc * dim, 0.0);
    for (int q = 0; q < t.nq; ++q) {
        double lam[4];
        lam[0] = 1.0;
        for (int r = 0; r < dim; ++r) {
            lam[r + 1] = t.points[q * dim + r];
            lam[0] -= lam[r + 1];
        }
        for (int a = 0; a < t.nloc; ++a) {
            int b[4];
            b[0] = degree;
            for (int r = 0; r < dim; ++r) {
                b[r + 1] = lat[a * dim + r];
                b[0] -= b[r + 1];
            }
            double f[4], df[4];
            for (int i = 0; i <= dim; ++i) factor(degree, b[i], lam[i], f[i], df[i]);
            double val = 1.0, dl[4];
            for (int i = 0; i <= dim; ++i) {
                val *= f[i];
                dl[i] = df[i];
                for (int i2 = 0; i2 <= dim; ++i2)
                    if (i2 != i) dl[i] *= f[i2];
            }
            t.phi[(size_t)q * t.nloc + a] = val;
            for (int r = 0; r < dim; ++r)
                t.dphi[((size_t)q * t.nloc + a) * dim + r] = dl[r + 1] - dl[0];
        }
    }
    return t;
}

int table_record(int form, int dim, int nloc)
{
    const int n = (form == FEM_MASS ? nloc : dim * nloc) + 1;
    return (n + 1) & ~1;
}

std::vector<double> kernel_table(int form, const RefTables &t)
{
    const int rec = table_record(form, t.dim, t.nloc);
    std::vector<double> out((size_t)t.nq * rec, 0.0);
    for (int q = 0; q < t.nq; ++q) {
        double *o = &out[(size_t)q * rec];
        if (form == FEM_MASS) {
            for (int a = 0; a < t.nloc; ++a) o[a] = t.phi[(size_t)q * t.nloc + a];
            o[t.nloc] = t.weights[q];
        } else {
            for (int r = 0; r < t.dim; ++r)
                for (int a = 0; a < t.nloc; ++a)
                    o[r * t.nloc + a] = t.dphi[((size_t)q * t.nloc + a) * t.dim + r];
            o[t.dim * t.nloc] = t.weights[q];
        }
    }
    return out;
}

bool has_symmetric_rule(int dim, int quad_degree)
{
    std::vector<double> p, w;
    return symmetric_rule(dim, quad_degree, p, w);
}

}  // namespace femx

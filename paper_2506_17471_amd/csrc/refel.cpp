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
#include <array>
#include <cmath>
#include <map>
#include <mutex>
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

// Fully symmetric rules: points on orbits of the simplex's symmetry group, the points of
// an orbit sharing one weight.  Barycentric orbits of the triangle: S3 (centroid), S21(a)
// = perms of (a, a, 1-2a), S111(a, b) = perms of (a, b, 1-a-b); of the tetrahedron: S4,
// S31(a) = perms of (a, a, a, 1-3a), S22(a) = perms of (a, a, 1/2-a, 1/2-a), S211(a, b) =
// perms of (a, a, b, 1-2a-b).
enum OrbitKind { S3, S21, S111, S4, S31, S22, S211 };

int orbit_params(int kind)
{
    return (kind == S111 || kind == S211) ? 2 : (kind == S3 || kind == S4) ? 0 : 1;
}

// barycentric coordinates of an orbit's points, appended to lam (dim + 1 per point)
template <typename T>
void orbit_points(int kind, const T *prm, std::vector<T> &lam)
{
    auto put = [&](std::initializer_list<T> l) { lam.insert(lam.end(), l); };
    const T a = prm ? prm[0] : T(0), b = (prm && orbit_params(kind) == 2) ? prm[1] : T(0);
    const T third = T(1) / 3, quarter = T(1) / 4, half = T(1) / 2;
    switch (kind) {
    case S3: put({third, third, third}); break;
    case S21: {
        const T c = T(1) - 2 * a;
        put({a, a, c}); put({a, c, a}); put({c, a, a});
        break;
    }
    case S111: {
        const T v[3] = {a, b, T(1) - a - b};
        const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
        for (auto &pm : perm) put({v[pm[0]], v[pm[1]], v[pm[2]]});
        break;
    }
    case S4: put({quarter, quarter, quarter, quarter}); break;
    case S31: {
        const T c = T(1) - 3 * a;
        for (int k = 0; k < 4; ++k)
            for (int i = 0; i < 4; ++i) lam.push_back(i == k ? c : a);
        break;
    }
    case S22: {
        const T c = half - a;
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j)
                for (int l = 0; l < 4; ++l) lam.push_back(l == i || l == j ? a : c);
        break;
    }
    case S211: {
        const T c = T(1) - 2 * a - b;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                if (j == i) continue;
                for (int l = 0; l < 4; ++l) lam.push_back(l == i ? b : l == j ? c : a);
            }
        break;
    }
    default: break;
    }
}

// A rule's orbit structure and approximate parameters: per orbit its parameters, then its
// weight (weights sum to the reference volume).  Five or more significant digits select
// the root of the moment equations that Newton's method then solves to full precision.
struct SymmetricSpec {
    int dim, degree;
    std::vector<int> kinds;
    std::vector<double> guess;
};

const std::vector<SymmetricSpec> &symmetric_specs()
{
    static const std::vector<SymmetricSpec> specs = {
        // triangle, degree 4: 6 points
        {2, 4, {S21, S21}, {0.445948, 0.111691, 0.0915762, 0.0549759}},
        // triangle, degree 6: 12 points
        {2, 6, {S21, S21, S111}, {0.249287, 0.0583931, 0.0630890, 0.0254225, 0.310352, 0.0531450,
                                  0.0414255}},
        // triangle, degree 8: 16 points
        {2, 8, {S3, S21, S21, S21, S111}, {0.0721578, 0.0505472, 0.0162292, 0.459293, 0.0475458,
                                           0.170569, 0.0516087, 0.263113, 0.00839478,
                                           0.0136152}},
        // triangle, degree 10: 25 points
        {2, 10, {S3, S21, S21, S111, S111, S111},
         {0.0416099, 0.0285035, 0.00547564, 0.162913, 0.0263260, 0.153303, 0.0336857, 0.0146614,
          0.363363, 0.607330, 0.0176975, 0.336696, 0.146812, 0.0281386}},
        // triangle, degree 12: 33 points
        {2, 12, {S21, S21, S21, S21, S21, S111, S111, S111},
         {0.271463, 0.0312706, 0.488204, 0.0121334, 0.440112, 0.0249592, 0.109258, 0.0142430,
          0.0246464, 0.00396582, 0.255454, 0.116296, 0.0216137, 0.127280, 0.851338, 0.00754184,
          0.291656, 0.0230342, 0.0108918}},
        // tetrahedron, degree 5: 14 points
        {3, 5, {S31, S31, S22}, {0.310886, 0.0187813, 0.0927353, 0.0122488, 0.0455037, 0.00709100}},
        // tetrahedron, degree 6: 24 points
        {3, 6, {S31, S31, S31, S211}, {0.214603, 0.00665379, 0.0406740, 0.00167954, 0.322338,
                                       0.00922620, 0.0636610, 0.269672, 0.00803571}},
        // tetrahedron, degree 8: 50 points
        {3, 8, {S31, S31, S22, S211, S211, S211},
         {0.0834534, 0.00200563, 0.0100916, 0.000209000, 0.449481, 0.00454683, 0.0368078,
          0.734271, 0.00214781, 0.222840, 0.430062, 0.00428064, 0.229785, 0.513039,
          0.00444881}},
    };
    return specs;
}

// exact integral of xi^e over the reference simplex: prod e_i! / (|e| + dim)!
long double monomial_integral(int dim, const int *e)
{
    long double num = 1, den = 1;
    int tot = 0;
    for (int r = 0; r < dim; ++r) {
        for (int f = 2; f <= e[r]; ++f) num *= f;
        tot += e[r];
    }
    for (int f = 2; f <= tot + dim; ++f) den *= f;
    return num / den;
}

template <typename T>
void expand(const SymmetricSpec &sp, const std::vector<T> &x, std::vector<T> &pts,
            std::vector<T> &wts)
{
    pts.clear();
    wts.clear();
    std::vector<T> lam;
    size_t i = 0;
    for (int kind : sp.kinds) {
        const int np = orbit_params(kind);
        lam.clear();
        orbit_points<T>(kind, np ? &x[i] : nullptr, lam);
        i += np;
        const T w = x[i++];
        const int npt = (int)lam.size() / (sp.dim + 1);
        for (int q = 0; q < npt; ++q) {
            for (int r = 1; r <= sp.dim; ++r) pts.push_back(lam[q * (sp.dim + 1) + r]);
            wts.push_back(w);
        }
    }
}

// relative moment errors of the rule x over all monomials of degree <= sp.degree
template <typename T>
void moment_residual(const SymmetricSpec &sp, const std::vector<std::array<int, 3>> &mons,
                     const std::vector<T> &exact, const std::vector<T> &x, std::vector<T> &res)
{
    std::vector<T> pts, wts;
    expand<T>(sp, x, pts, wts);
    res.assign(mons.size(), T(0));
    for (size_t m = 0; m < mons.size(); ++m) {
        T s = 0;
        for (size_t q = 0; q < wts.size(); ++q) {
            T v = wts[q];
            for (int r = 0; r < sp.dim; ++r)
                for (int e = 0; e < mons[m][r]; ++e) v *= pts[q * sp.dim + r];
            s += v;
        }
        res[m] = (s - exact[m]) / exact[m];
    }
}

// least-squares solve of the m x n system A dx = b (m >= n) by Householder QR
std::vector<double> lstsq(std::vector<double> A, std::vector<double> b, int m, int n)
{
    for (int k = 0; k < n; ++k) {
        double nrm = 0.0;
        for (int i = k; i < m; ++i) nrm += A[i * n + k] * A[i * n + k];
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) continue;
        const double alpha = A[k * n + k] > 0 ? -nrm : nrm;
        std::vector<double> v(m - k);
        for (int i = k; i < m; ++i) v[i - k] = A[i * n + k];
        v[0] -= alpha;
        double vv = 0.0;
        for (double t : v) vv += t * t;
        if (vv == 0.0) continue;
        for (int j = k; j < n; ++j) {
            double d = 0.0;
            for (int i = k; i < m; ++i) d += v[i - k] * A[i * n + j];
            d *= 2.0 / vv;
            for (int i = k; i < m; ++i) A[i * n + j] -= d * v[i - k];
        }
        double d = 0.0;
        for (int i = k; i < m; ++i) d += v[i - k] * b[i];
        d *= 2.0 / vv;
        for (int i = k; i < m; ++i) b[i] -= d * v[i - k];
    }
    std::vector<double> x(n, 0.0);
    for (int k = n - 1; k >= 0; --k) {
        double s = b[k];
        for (int j = k + 1; j < n; ++j) s -= A[k * n + j] * x[j];
        x[k] = A[k * n + k] != 0.0 ? s / A[k * n + k] : 0.0;
    }
    return x;
}

// Solve the moment equations from the spec's approximate parameters by Gauss-Newton
// (central-difference Jacobian, Householder QR), residuals and iterates in extended
// precision so the root is resolved well below double rounding even where the equations
// are ill-conditioned; accept it only if every monomial of degree <= the rule's degree is
// integrated to 1e-14 relative, all weights are positive and all points lie in the
// closed simplex.
bool solve_symmetric(const SymmetricSpec &sp, std::vector<double> &pts, std::vector<double> &wts)
{
    using LD = long double;
    std::vector<std::array<int, 3>> mons;
    for (int i = 0; i <= sp.degree; ++i)
        for (int j = 0; i + j <= sp.degree; ++j)
            if (sp.dim == 2) {
                mons.push_back({i, j, 0});
            } else {
                for (int l = 0; i + j + l <= sp.degree; ++l) mons.push_back({i, j, l});
            }
    std::vector<LD> exact(mons.size());
    for (size_t m = 0; m < mons.size(); ++m) exact[m] = monomial_integral(sp.dim, mons[m].data());
    std::vector<LD> x(sp.guess.begin(), sp.guess.end()), r, rp, rm;
    const int n = (int)x.size(), m = (int)mons.size();
    LD prev = 1e300L;
    for (int it = 0; it < 60; ++it) {
        moment_residual<LD>(sp, mons, exact, x, r);
        LD err = 0;
        for (LD t : r) err = std::max(err, std::fabs(t));
        if (err < 1e-18L || (err >= prev && it > 8)) break;
        prev = err;
        std::vector<double> J((size_t)m * n);
        for (int k = 0; k < n; ++k) {
            const LD h = 1e-8L * std::max(LD(1e-2), std::fabs(x[k]));
            std::vector<LD> xp = x, xm = x;
            xp[k] += h;
            xm[k] -= h;
            moment_residual<LD>(sp, mons, exact, xp, rp);
            moment_residual<LD>(sp, mons, exact, xm, rm);
            for (int i = 0; i < m; ++i) J[(size_t)i * n + k] = (double)((rp[i] - rm[i]) / (2 * h));
        }
        std::vector<double> negr(m);
        for (int i = 0; i < m; ++i) negr[i] = -(double)r[i];
        const std::vector<double> dx = lstsq(J, negr, m, n);
        for (int k = 0; k < n; ++k) x[k] += dx[k];
    }
    moment_residual<LD>(sp, mons, exact, x, r);
    for (LD t : r)
        if (!(std::fabs(t) < 1e-14L)) return false;
    std::vector<LD> lp, lw;
    expand<LD>(sp, x, lp, lw);
    pts.assign(lp.begin(), lp.end());
    wts.assign(lw.begin(), lw.end());
    for (double w : wts)
        if (!(w > 0.0)) return false;
    for (size_t q = 0; q < wts.size(); ++q) {
        double s = 0.0;
        for (int r2 = 0; r2 < sp.dim; ++r2) {
            const double xi = pts[q * sp.dim + r2];
            if (xi < -1e-15) return false;
            s += xi;
        }
        if (s > 1.0 + 1e-15) return false;
    }
    return true;
}

// Fully symmetric rules of degree <= 2 from their moment equations (closed form).
//   degree <= 1: the centroid, weight |T|.
//   degree 2, triangle: the orbit of (a, b, b), a = 1 - 2b, weight |T|/3 each; matching
//     int lambda_1^2 = |T|/6 gives 6b^2 - 4b + 1/2 = 0, b = 1/6 (the interior root).
//   degree 2, tetrahedron: the orbit of (a, b, b, b), a = 1 - 3b, weight |T|/4 each;
//     int lambda_1^2 = |T|/10 gives 12b^2 - 6b + 3/5 = 0, b = (5 - sqrt 5)/20.
// Higher degrees: the solved orbit rule of the smallest tabulated degree >= degree.
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
    if (degree == 2) {
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
    // solved rules are cached: plan creation may ask for one many times
    static std::mutex mu;
    static std::map<std::pair<int, int>, std::pair<std::vector<double>, std::vector<double>>> cache;
    const SymmetricSpec *spec = nullptr;
    for (const auto &sp : symmetric_specs())
        if (sp.dim == dim && sp.degree >= degree && (!spec || sp.degree < spec->degree)) spec = &sp;
    if (!spec) return false;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_pair(dim, spec->degree);
    auto it = cache.find(key);
    if (it == cache.end()) {
        std::vector<double> p, w;
        if (!solve_symmetric(*spec, p, w)) return false;
        it = cache.emplace(key, std::make_pair(p, w)).first;
    }
    pts = it->second.first;
    wts = it->second.second;
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

int table_record(int form, int dim, int nloc, int geom)
{
    const int vals = (form == FEM_MASS || form == FEM_HELMHOLTZ) ? nloc : 0;
    const int ders = form == FEM_MASS ? 0 : dim * nloc;
    const int gders = geom == 2 ? dim * cell_geom_nodes(dim, 2) : 0;
    return (vals + ders + 1 + gders + 1) & ~1;
}

// Per quadrature point: phi_a (mass, Helmholtz), then d phi_a / d xi_r for r, a (all other
// forms, r-major), then the weight, then (curved cells, tables g of the P2 geometry basis
// on the same rule) d phiG_g / d xi_r for r, g; zero-padded to an even length.
std::vector<double> kernel_table(int form, const RefTables &t, const RefTables *g)
{
    const int rec = table_record(form, t.dim, t.nloc, g ? 2 : 1);
    std::vector<double> out((size_t)t.nq * rec, 0.0);
    const bool vals = form == FEM_MASS || form == FEM_HELMHOLTZ, ders = form != FEM_MASS;
    if (g && (g->nq != t.nq || g->dim != t.dim || g->nloc != cell_geom_nodes(t.dim, 2)))
        throw Error(FEM_E_ARG, "geometry tables do not match the rule");
    for (int q = 0; q < t.nq; ++q) {
        double *o = &out[(size_t)q * rec];
        int k = 0;
        if (vals)
            for (int a = 0; a < t.nloc; ++a) o[k++] = t.phi[(size_t)q * t.nloc + a];
        if (ders)
            for (int r = 0; r < t.dim; ++r)
                for (int a = 0; a < t.nloc; ++a)
                    o[k++] = t.dphi[((size_t)q * t.nloc + a) * t.dim + r];
        o[k++] = t.weights[q];
        if (g)
            for (int r = 0; r < t.dim; ++r)
                for (int a = 0; a < g->nloc; ++a)
                    o[k++] = g->dphi[((size_t)q * g->nloc + a) * t.dim + r];
    }
    return out;
}

std::vector<double> mfma_table(int form, const RefTables &t, int *n_tiles)
{
    const int n = t.nloc, ks = mfma_ks(n), ma = mfma_ma(n), d = mfma_rows(form, t.dim);
    const int nt = (t.nq + 15) / 16, tile = mfma_tile_doubles(d, n);
    std::vector<double> out((size_t)nt * tile, 0.0);
    // row r of the form: a reference derivative, or (mass; Helmholtz's last row) the value
    const bool value_row = form == FEM_MASS || form == FEM_HELMHOLTZ;
    auto dphi = [&](int q, int a, int r) {
        if (q >= t.nq || a >= n) return 0.0;
        if (value_row && r == d - 1) return t.phi[(size_t)q * n + a];
        return t.dphi[((size_t)q * n + a) * t.dim + r];
    };
    for (int tt = 0; tt < nt; ++tt) {
        double *o = &out[(size_t)tt * tile];
        for (int r = 0; r < d; ++r)
            for (int s = 0; s < ks; ++s)
                for (int l = 0; l < 64; ++l)
                    o[(r * ks + s) * 64 + l] = dphi(16 * tt + l % 16, 4 * s + l / 16, r);
        double *c = o + d * ks * 64;
        for (int k = 0; k < 4; ++k)
            for (int r = 0; r < d; ++r)
                for (int m = 0; m < ma; ++m)
                    for (int l = 0; l < 64; ++l)
                        c[((k * d + r) * ma + m) * 64 + l] =
                            dphi(16 * tt + 4 * k + l / 16, 16 * m + l % 16, r);
        double *w = c + 4 * d * ma * 64;
        for (int i = 0; i < 16; ++i) w[i] = 16 * tt + i < t.nq ? t.weights[16 * tt + i] : 0.0;
    }
    *n_tiles = nt;
    return out;
}

bool has_symmetric_rule(int dim, int quad_degree)
{
    std::vector<double> p, w;
    return symmetric_rule(dim, quad_degree, p, w);
}

}  // namespace femx

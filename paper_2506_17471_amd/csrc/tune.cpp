// Autotuner: measures the launch configurations of a plan and keeps the fastest.
//
// Candidates: the colour strategy with 64/128/256 cells per workgroup, and the patch
// strategy with 64/128/256 cells per patch and one lane per cell, 64/128 with two lanes
// (2D vector forms), 42/63/84 with three lanes (3D vector forms), each with both ways of
// summing inside a patch.  The plan's configuration on entry stays unless a candidate is
// more than 3% faster.  Each candidate is
// timed with HIP events on the caller's stream using the paper's protocol (Sec. 6.2.1): five warm-up runs, then timed runs until 15 have been collected
// or 0.2 s has accumulated, the arithmetic mean being the candidate's time.  Results can
// be kept in a small JSON cache keyed by device architecture, form, dimension, degree,
// quadrature degree and rule family, log2 of the cell count and direction (action or VJP); fem_plan_create
// consults the action entries when the
// environment variable FEM_TUNE_CACHE names the file.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

namespace {

struct Candidate {
    int strategy, patch, lanes, block, sum_mode;
};

std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string s = prop.gcnArchName;
    const size_t colon = s.find(':');
    return colon == std::string::npos ? s : s.substr(0, colon);
}

// one entry per direction: the tangent (VJP) kernels of the hyperelastic forms have their
// own best configuration; plan creation applies the forward entry
std::string cache_key(const fem_plan *p, bool vjp = false)
{
    const int bucket = p->n_cell > 0 ? (int)std::lround(std::log2((double)p->n_cell)) : 0;
    std::ostringstream k;
    k << arch_name() << "/f" << p->form << "/d" << p->dim << "/k" << p->degree << "/q"
      << p->quad_degree << (p->quad_family == FEM_QUAD_SYMMETRIC ? "s" : "c")
      << (p->geom == 2 ? "/g2" : "") << "/c" << bucket
      << (vjp && femx::nonlinear_form(p->form) ? "/vjp" : "");
    return k.str();
}

// The cache file: one JSON object whose values are [strategy, patch, lanes, block, sum mode,
// ms].
std::map<std::string, std::vector<double>> read_cache(const std::string &path)
{
    std::map<std::string, std::vector<double>> out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t i = 0;
    while ((i = s.find('"', i)) != std::string::npos) {
        const size_t j = s.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = s.substr(i + 1, j - i - 1);
        const size_t lb = s.find('[', j), rb = s.find(']', j);
        if (lb == std::string::npos || rb == std::string::npos || rb < lb) break;
        std::vector<double> vals;
        std::stringstream vs(s.substr(lb + 1, rb - lb - 1));
        std::string tok;
        while (std::getline(vs, tok, ',')) vals.push_back(std::atof(tok.c_str()));
        if (vals.size() == 6) out[key] = vals;
        i = rb + 1;
    }
    return out;
}

void write_cache(const std::string &path, const std::map<std::string, std::vector<double>> &c)
{
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) throw femx::Error(FEM_E_ARG, "cannot write tuning cache " + path);
        f << "{\n";
        size_t n = 0;
        for (const auto &kv : c) {
            f << "  \"" << kv.first << "\": [" << (int)kv.second[0] << ", " << (int)kv.second[1]
              << ", " << (int)kv.second[2] << ", " << (int)kv.second[3] << ", "
              << (int)kv.second[4] << ", " << kv.second[5] << "]" << (++n < c.size() ? "," : "")
              << "\n";
        }
        f << "}\n";
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0)
        throw femx::Error(FEM_E_ARG, "cannot replace tuning cache " + path);
}

void apply(fem_plan *p, const Candidate &c)
{
    if (c.strategy == FEM_SCATTER_COLOUR) {
        femx::set_strategy(p, FEM_SCATTER_COLOUR, 0, 0, 0);
        p->block = c.block;
    } else {
        femx::set_strategy(p, FEM_SCATTER_PATCH, c.patch, c.lanes, c.sum_mode);
    }
}

double time_candidate(fem_plan *p, const double *u, const double *v, double *y, bool vjp,
                      hipStream_t s)
{
    hipEvent_t a, b;
    femx::check_hip(hipEventCreate(&a), "hipEventCreate");
    femx::check_hip(hipEventCreate(&b), "hipEventCreate");
    auto once = [&] { femx::run_action(p, u, v, y, s, vjp); };
    double total = 0.0;
    int runs = 0;
    try {
        for (int i = 0; i < 5; ++i) once();
        while (runs < 15 && total < 0.2) {
            femx::check_hip(hipEventRecord(a, s), "hipEventRecord");
            once();
            femx::check_hip(hipEventRecord(b, s), "hipEventRecord");
            femx::check_hip(hipEventSynchronize(b), "hipEventSynchronize");
            float ms = 0.f;
            femx::check_hip(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
            total += ms * 1e-3;
            ++runs;
        }
    } catch (...) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        throw;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return total / runs * 1e3;
}

}  // namespace

namespace femx {

// Apply a cached configuration for this plan, if FEM_TUNE_CACHE names a file holding one.
void apply_tuning_cache(fem_plan *p)
{
    const char *path = std::getenv("FEM_TUNE_CACHE");
    if (!path || !*path || p->n_cell == 0) return;
    const auto cache = read_cache(path);
    const auto it = cache.find(cache_key(p));
    if (it == cache.end()) return;
    const auto &v = it->second;
    Candidate c{(int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4]};
    try {
        apply(p, c);
    } catch (const Error &) {
        // a stale or foreign entry: keep the defaults
    }
}

std::vector<Candidate> candidates(const fem_plan *p)
{
    std::vector<Candidate> cands;
    for (int blk : {64, 128, 256}) cands.push_back({FEM_SCATTER_COLOUR, 0, 1, blk, 0});
    // patch sizes grouped so that one layout build serves both sum modes
    for (int P : {64, 128, 256})
        for (int m : {SUM_ELEMENT, SUM_COLOURED}) cands.push_back({FEM_SCATTER_PATCH, P, 1, 0, m});
    if (p->geom == 2) {
        // curved cells: one lane per cell, or lane triples (3D vector forms); for the
        // hyperelastic forms only the configurations whose tangent runs, where any does
        if (curved_triple_available(p->form, p->dim, p->degree))
            for (int P : {42, 63, 84})
                for (int m : {SUM_ELEMENT, SUM_COLOURED}) cands.push_back({FEM_SCATTER_PATCH, P, 3, 0, m});
        if (nonlinear_form(p->form)) {
            std::vector<Candidate> ok;
            for (const Candidate &c : cands)
                if (!vjp_kernel_spills(p->form, p->dim, p->degree, c.strategy == FEM_SCATTER_COLOUR,
                                       c.lanes, c.strategy == FEM_SCATTER_COLOUR ? 1 : c.sum_mode, 2))
                    ok.push_back(c);
            if (!ok.empty()) cands.swap(ok);
        }
        return cands;
    }
    // the matrix-core kernel: 64-cell patches, coloured sums
    if (mfma_available(p->form, p->dim, p->degree) && p->nqt > 0)
        cands.push_back({FEM_SCATTER_PATCH, 64, kMfmaLanes, 0, SUM_COLOURED});
    if (pair_available(p->form, p->dim, p->degree))
        for (int P : {64, 128})
            for (int m : {SUM_ELEMENT, SUM_COLOURED})
                cands.push_back({FEM_SCATTER_PATCH, P, 2, 0, m});
    if (triple_available(p->form, p->dim, p->degree))
        for (int P : {42, 63, 84})
            for (int m : {SUM_ELEMENT, SUM_COLOURED})
                cands.push_back({FEM_SCATTER_PATCH, P, 3, 0, m});
    // the hyperelastic forms: only configurations whose tangent kernel runs (no scratch), so
    // a plan tuned on its action can always take its VJP
    if (nonlinear_form(p->form)) {
        std::vector<Candidate> ok;
        for (const Candidate &c : cands)
            if (!vjp_kernel_spills(p->form, p->dim, p->degree, c.strategy == FEM_SCATTER_COLOUR,
                                   c.lanes, c.strategy == FEM_SCATTER_COLOUR ? 1 : c.sum_mode,
                                   p->geom))
                ok.push_back(c);
        cands.swap(ok);
    }
    return cands;
}

// FP64 work of one quadrature point of a cell (the plain loop, FMA = 2 flops)
double flops_per_point(int form, int d, int nloc, bool vjp)
{
    const double n = nloc, dd = d;
    if (form == FEM_MASS) return 4 * n + 2;
    if (form == FEM_LAPLACE || form == FEM_HELMHOLTZ)
        return 4 * dd * n + 2 * dd * dd + dd + 1 + (form == FEM_HELMHOLTZ ? 4 * n + 1 : 0);
    const double ev = 2 * dd * dd * n * (vjp ? 2 : 1), ct = 2 * dd * dd * n;
    const double geo = 2 * dd * dd * dd * (vjp ? 3 : 2) + dd * dd;
    double pw = 3 * dd * dd + 2 * dd;                       // elasticity
    if (form == FEM_NEOHOOKEAN) pw = d == 2 ? 40 : 110;     // inverse, log, stress
    if (form == FEM_SVK) pw = 4 * dd * dd * dd + 4 * dd * dd;
    if (vjp) pw += 4 * dd * dd * dd;
    return ev + ct + geo + pw;
}

// Analytic time of one candidate (ms), from the plan's sizes and the compiled kernel's
// registers -- no launch.  The terms, after the paper's cost model adapted to gfx950:
//   VALU time: FP64 instructions (work / 2, plus what a lane split repeats) at 16 lanes
//     per SIMD per cycle over 1024 SIMDs, derated when fewer than three waves per SIMD
//     (set by registers and, for patches, by LDS) are there to hide latency;
//   memory time: the footprint plus the partial sums of shared nodes (patches; plus the slot
//     lists of the element buffer) or the uncoalesced read-add-write scatter (colours) at
//     4 TB/s, derated below six resident waves per SIMD;
//   synchronisation: per workgroup round one barrier per sub-colour (coloured sums) or
//     three (element buffer), and one launch per colour for the colour strategy.
double predict_ms(const fem_plan *p, const Candidate &c, bool vjp)
{
    const bool nl = vjp && nonlinear_form(p->form);
    const double n = (double)p->n_cell, d = p->dim, nloc = p->nloc, nc = p->ncomp;
    const double nodes_per_cell = (double)p->n_node / std::max<int64_t>(1, p->n_cell);
    double instr = flops_per_point(p->form, p->dim, p->nloc, nl) * p->nq / 2.0 * 1.25;
    // curved cells: J from the geometry gradients and its inverse at every point
    const int ng = cell_geom_nodes(p->dim, p->geom);
    if (p->geom == 2) instr += (2.0 * d * d * ng + (p->dim == 2 ? 12 : 60)) * p->nq / 2.0 * 1.25;
    // lane splits repeat the pointwise form on every lane of a cell and exchange gradient
    // rows: cheap for elasticity, costly for the hyperelastic forms (inverse, log, stress)
    const bool hyper = nonlinear_form(p->form);
    if (c.lanes == 2) instr *= hyper ? 1.6 : 1.35;
    if (c.lanes == 3) instr *= hyper ? 2.5 : 1.2;
    const int regs = kernel_registers(p->form, p->dim, p->degree, nl,
                                      c.strategy == FEM_SCATTER_COLOUR, c.lanes,
                                      c.strategy == FEM_SCATTER_COLOUR ? 1 : c.sum_mode, p->geom);
    const double waves_regs = std::min(8, 512 / std::max(8, (regs + 7) / 8 * 8));
    double waves = waves_regs, rounds_sync = 0.0, barriers = 0.0, extra_bytes = 0.0;
    const double vec_bytes = 8.0 * p->n_node * nc;
    if (c.strategy == FEM_SCATTER_PATCH) {
        const double P = c.patch;
        const double share = d == 2 ? 2.5 / std::sqrt(P) : 4.0 / std::cbrt(P);
        const int U = (int)(P * nodes_per_cell * (1.0 + share)) + 8;
        const size_t lds = patch_lds_bytes(p->form, p->dim, p->degree, nl, c.patch, U, c.sum_mode,
                                           c.lanes);
        const double wgs_lds = std::floor(160.0 * 1024 / std::max<size_t>(1, lds));
        const double wave_per_wg = std::ceil(patch_threads(c.patch, c.lanes) / 64.0);
        waves = std::min(waves, wgs_lds * wave_per_wg / 4.0);
        const double wg_per_cu = std::max(1.0, waves * 4.0 / wave_per_wg);
        rounds_sync = std::ceil(n / P / (256.0 * wg_per_cu));
        // coloured: one barrier per sub-colour (a wavefront skips the other colours' adds);
        // element buffer: three, plus the buffer's write and slot-ordered read passes
        barriers = c.sum_mode == SUM_COLOURED ? (d == 2 ? 7 : 24) + 3 : 5;
        extra_bytes = 2.0 * share * vec_bytes * 2.0;
        // the element buffer's slot lists: a u16 per (cell, local node), an offset per node
        if (c.sum_mode == SUM_ELEMENT) extra_bytes += 2.0 * nloc * n + 4.0 * p->n_node * (1.0 + share);
    } else {
        extra_bytes = 2.0 * n * nloc * nc * 8.0;          // gathers and read-add-writes
    }
    const double eta = std::min(1.0, std::max(waves, 0.25) / 3.0);
    double t_valu = n * instr * 4.0 / (64.0 * 1024.0 * 2.4e9) / eta;
    if (c.lanes == kMfmaLanes) {
        // matrix cores: per 16 cells and point tile, R C products (tabulation rows R:
        // d derivatives, values or both; C components) per k-step of the evaluation (twice
        // for the VJP) and 4 R C per node tile of the contraction, 64 cycles each on one
        // SIMD; the pointwise work on the vector ALU at every padded point, half of it
        // overlapped
        const double ks = mfma_ks(p->nloc), ma = mfma_ma(p->nloc), tiles = p->nqt;
        const double rc = (double)mfma_rows(p->form, p->dim) * nc;
        const double ops = tiles * (rc * ks * (nl ? 2 : 1) + 4.0 * rc * ma);
        const double t_mfma = n / 16.0 * ops * 64.0 / (1024.0 * 2.4e9) / eta;
        const double ev = 2 * rc * nloc * (nl ? 2 : 1), ct = 2 * rc * nloc;
        const double pw = flops_per_point(p->form, p->dim, p->nloc, nl) - ev - ct;
        const double t_pw = n * 16.0 * tiles * pw / 2.0 * 1.25 * 4.0 / (64.0 * 1024.0 * 2.4e9) / eta;
        t_valu = t_mfma + 0.5 * t_pw;
    }
    const double bytes = vec_bytes * (nl ? 3 : 2) + 8.0 * d * p->n_vert +
                         4.0 * (nloc + ng) * n + extra_bytes;
    // memory-level parallelism: fewer than six resident waves per SIMD (an LDS-hungry
    // patch) leave HBM requests unissued
    const double t_mem = bytes / (4.0e12 * std::min(1.0, waves / 6.0));
    double t = std::max(t_valu, t_mem) + rounds_sync * barriers * 0.4e-6;
    if (c.strategy == FEM_SCATTER_COLOUR) t += p->n_colours * 4.0e-6;
    else t += 4.0e-6;                                     // the fixup launch
    return t * 1e3;
}

int tune(fem_plan *p, const double *u, const double *v, double *y, bool vjp, const char *cache,
         hipStream_t s, double *results, int max_results, int *n_results, int max_timed)
{
    std::vector<Candidate> cands = candidates(p);
    if (max_timed > 0 && max_timed < (int)cands.size()) {
        // prune to the model's best max_timed candidates (the entry configuration is kept
        // below regardless), keeping their original order so layout builds are shared
        std::vector<std::pair<double, int>> pred;
        for (int i = 0; i < (int)cands.size(); ++i) pred.push_back({predict_ms(p, cands[i], vjp), i});
        std::sort(pred.begin(), pred.end());
        std::vector<int> keep;
        for (int i = 0; i < max_timed; ++i) keep.push_back(pred[i].second);
        std::sort(keep.begin(), keep.end());
        std::vector<Candidate> kept;
        for (int i : keep) kept.push_back(cands[i]);
        cands = kept;
    }
    // the configuration the plan had on entry competes too, and keeps its place unless a
    // candidate beats it by more than kMargin (timing noise must not flip configurations)
    constexpr double kMargin = 0.03;
    const Candidate entry{p->strategy == STRAT_PATCH ? FEM_SCATTER_PATCH : FEM_SCATTER_COLOUR,
                          p->strategy == STRAT_PATCH ? p->patch : 0, p->lanes,
                          p->strategy == STRAT_PATCH ? 0 : p->block,
                          p->strategy == STRAT_PATCH ? p->sum_mode : 0};
    auto same = [](const Candidate &a, const Candidate &b) {
        return a.strategy == b.strategy && a.patch == b.patch && a.lanes == b.lanes &&
               a.sum_mode == b.sum_mode && (a.strategy == FEM_SCATTER_PATCH || a.block == b.block);
    };
    if (std::none_of(cands.begin(), cands.end(), [&](const Candidate &c) { return same(c, entry); }))
        cands.push_back(entry);
    double best = 1e300, entry_ms = 1e300;
    Candidate best_c = cands[0];
    int nres = 0;
    for (const Candidate &c : cands) {
        double ms;
        try {
            apply(p, c);
            ms = time_candidate(p, u, v, y, vjp, s);
        } catch (const Error &e) {
            if (e.code != FEM_E_UNSUPPORTED) throw;
            continue;   // e.g. a patch that needs more LDS than a workgroup has
        }
        if (results && nres < max_results) {
            double *r = results + 6 * nres;
            r[0] = c.strategy;
            r[1] = c.patch;
            r[2] = c.lanes;
            r[3] = c.block;
            r[4] = c.sum_mode;
            r[5] = ms;
        }
        ++nres;
        if (same(c, entry)) entry_ms = ms;
        if (ms < best) {
            best = ms;
            best_c = c;
        }
    }
    if (n_results) *n_results = nres;
    if (nres == 0) {
        // nothing ran (every candidate refused: spilling tangents, LDS): leave the plan as
        // it came
        apply(p, entry);
        throw Error(FEM_E_UNSUPPORTED, std::string("no launch configuration runs this plan's ") +
                                           (vjp ? "VJP" : "action"));
    }
    if (entry_ms < 1e300 && best > (1.0 - kMargin) * entry_ms) {
        best_c = entry;
        best = entry_ms;
    }
    apply(p, best_c);
    if (cache && *cache) {
        auto c = read_cache(cache);
        c[cache_key(p, vjp)] = {(double)best_c.strategy, (double)best_c.patch, (double)best_c.lanes,
                           (double)best_c.block, (double)best_c.sum_mode, best};
        write_cache(cache, c);
    }
    return FEM_OK;
}

int tune_predict(const fem_plan *p, bool vjp, double *results, int max_results, int *n_results)
{
    const std::vector<Candidate> cands = candidates(p);
    int nres = 0;
    for (const Candidate &c : cands) {
        if (results && nres < max_results) {
            double *r = results + 6 * nres;
            r[0] = c.strategy;
            r[1] = c.patch;
            r[2] = c.lanes;
            r[3] = c.block;
            r[4] = c.sum_mode;
            r[5] = predict_ms(p, c, vjp);
        }
        ++nres;
    }
    if (n_results) *n_results = nres;
    return FEM_OK;
}

}  // namespace femx

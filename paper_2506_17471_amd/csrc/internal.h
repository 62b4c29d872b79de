// Internal declarations shared by the host side of the library and the kernel launchers.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fem_action.h"

namespace femx {

// An error that maps to a status code at the ABI boundary.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void check_hip(hipError_t e, const char *what);
std::string &last_error();   // thread-local message behind fem_last_error()

inline int n_local(int dim, int k)
{
    return dim == 2 ? (k + 1) * (k + 2) / 2 : (k + 1) * (k + 2) * (k + 3) / 6;
}

// Reference element data on the host (refel.cpp).
struct RefTables {
    int dim = 0, degree = 0, quad_degree = 0, nq = 0, nloc = 0;
    std::vector<double> points;   // [nq][dim]
    std::vector<double> weights;  // [nq]
    std::vector<double> phi;      // [nq][nloc]
    std::vector<double> dphi;     // [nq][nloc][dim]
};
RefTables reference_tables(int dim, int degree, int quad_degree, int family = FEM_QUAD_CONICAL);
bool has_symmetric_rule(int dim, int quad_degree);

// Kernel-side table layout: per quadrature point a contiguous record.
//   mass:  [phi_0 .. phi_{nloc-1}, w]                       (nloc + 1 doubles)
//   vector forms: [dphi_r(a) for r in 0..d-1 for a, w]      (d*nloc + 1 doubles)
// and, for P2-geometry cells, the geometry basis' reference derivatives after the weight
// ([dphiG_r(g) for r for g], d * n_gnode doubles, from the tables `g`), padded to an even
// number of doubles so every record starts 16-byte aligned.
int table_record(int form, int dim, int nloc, int geom = 1);
std::vector<double> kernel_table(int form, const RefTables &t, const RefTables *g = nullptr);

// The matrix-core kernels' tabulation, per tile of 16 quadrature points (16 t .. 16 t + 15,
// zero-padded past nq) in the operand order of v_mfma_f64_16x16x4_f64 (lane l holds
// A[l % 16][l / 16]; the 16 x 16 result's register k of lane l is row 4 k + l / 16, column
// l % 16), for the form's rows f_r: the reference derivatives d phi / d xi_r, r < d (vector
// forms, Laplace), the values phi (mass), or both, derivatives first (Helmholtz: r = d is
// phi):
//   evaluation  [r][ks][64]: A[i][kk] = f_r(phi_{4 ks + kk}) at point 16 t + i
//   contraction [k][r][m][64]: A[i][kk] = f_r(phi_{16 m + i}) at point 16 t + 4 k + kk
//   weights [16]: w at point 16 t + i
// (ks < mfma_ks = ceil(nloc / 4) k-steps of nodes, m < mfma_ma = ceil(nloc / 16) node tiles,
// phi_a = 0 for a >= nloc).
constexpr int mfma_ks(int nloc) { return (nloc + 3) / 4; }
constexpr int mfma_ma(int nloc) { return (nloc + 15) / 16; }
constexpr int mfma_rows(int form, int dim)
{
    return form == FEM_MASS ? 1 : (form == FEM_HELMHOLTZ ? dim + 1 : dim);
}
constexpr int mfma_tile_doubles(int rows, int nloc)
{
    return rows * mfma_ks(nloc) * 64 + 4 * rows * mfma_ma(nloc) * 64 + 16;
}
std::vector<double> mfma_table(int form, const RefTables &t, int *n_tiles);

// Launch parameters of one colour class.
struct LaunchArgs {
    const int32_t *verts;     // SoA [(dim+1)][stride] colour-sorted vertex ids
    const int32_t *nodes;     // SoA [nloc][stride]    colour-sorted node ids
    const uint64_t *first;    // [(n_loc + 63) / 64][stride]: bit a of word a / 64 set when
                              // this cell is the first to write its node a
    const double *coords;     // [n_vert][dim]
    const double *tab;        // [nq][record]
    const double *u;
    const double *v;          // second input (VJP) or null
    double *y;
    int64_t stride;
    int64_t begin;            // first colour-sorted cell of the class
    int64_t count;            // cells in the class
    int nq;
    double lam, mu;
};

// Launch parameters of the patch strategy (one workgroup per patch of cells).
struct PatchArgs {
    const int32_t *verts;       // SoA [(dim+1)][stride] vertex ids, patch-sorted cells
    const uint16_t *lidx;       // SoA [nloc][stride] patch-local node index of (cell, a)
    const uint8_t *colour;      // [stride] sub-colour of each cell inside its patch
    const int32_t *patch_off;   // [n_patch + 1] into the (patch, node) list
    const int32_t *patch_nodes; // global node id of each (patch, node): interior ones first
    const int32_t *patch_nint;  // [n_patch] interior (unshared) nodes of each patch
    const int32_t *patch_pbase; // [n_patch] first entry of each patch's shared nodes in pdest
    const int32_t *pdest;       // [n_partial] node-major partial slot of (patch, shared node)
    const uint8_t *patch_ncol;  // [n_patch] sub-colours of each patch
    const int32_t *csr_off;     // [n_pn + 1] element-buffer slots summed into (patch, node)
    const uint16_t *csr_slots;  // slot = a << 8 | local cell, in ascending (cell, a)
    const double *coords;
    const double *tab;
    const double *u;
    const double *v;
    double *y;
    double *partial;            // [n_partial][ncomp]
    const double *mtab;         // matrix-core tabulation tiles (mfma_table), or null
    int64_t stride;
    int64_t n_cell;
    int nq;
    int nqt;                    // point tiles of mtab
    int lds_a;                  // doubles of LDS region A (staging / element buffer)
    double lam, mu;
};

enum Strategy { STRAT_COLOUR = 0, STRAT_PATCH = 1 };
enum SumMode { SUM_ELEMENT = 1, SUM_COLOURED = 2 };

// One mesh of a batched launch (device-resident array of these).
struct BatchDesc {
    PatchArgs args;
    int64_t first_patch;     // index of the mesh's first patch in the launch
};

// Shared-node sums of one mesh of a batch.
struct FixDesc {
    const int32_t *fix_node;
    const int32_t *fix_off;
    const double *partial;
    double *y;
    int64_t first;           // index of the mesh's first (shared node, component) item
    int ncomp;
};

}  // namespace femx

struct fem_plan {
    int form = 0, dim = 0, degree = 0, quad_degree = 0, nloc = 0, ncomp = 0, nq = 0;
    int quad_family = FEM_QUAD_CONICAL;
    int geom = 1;                        // geometry degree: 1 affine cells, 2 P2 (curved)
    int64_t n_vert = 0, n_cell = 0, n_node = 0, n_dof = 0;
    double lam = 0.0, mu = 0.0;
    int n_colours = 0;
    int block = 0;                       // cells per workgroup (0 = default)
    int device = 0;
    int batch_refs = 0;                  // batches holding this plan's device arrays
    std::vector<int64_t> colour_off;     // [n_colours + 1] in colour-sorted order
    std::vector<int32_t> colour;         // [n_cell] colour of each caller cell
    int64_t stride = 0;                  // padded column length of the SoA maps
    double *d_coords = nullptr;
    int32_t *d_verts = nullptr;
    int32_t *d_nodes = nullptr;
    uint64_t *d_first = nullptr;
    double *d_tab = nullptr;
    double *d_mtab = nullptr;            // matrix-core tabulation (vector forms, affine cells)
    int nqt = 0;                         // its 16-point tiles
    int32_t *d_untouched = nullptr;      // nodes no cell holds (zeroed separately)
    int64_t n_untouched = 0;
    // patch strategy
    int strategy = femx::STRAT_PATCH;
    int patch = 0;                       // cells per patch (0: not built)
    int lanes = 1;                       // lanes per cell in the patch kernel (1, 2 or 3)
    int64_t n_patch = 0, n_pn = 0, n_partial = 0, n_shared = 0;
    int max_patch_nodes = 0;
    int32_t *d_pverts = nullptr;
    uint16_t *d_lidx = nullptr;
    int sum_mode = femx::SUM_ELEMENT;    // how a patch sums its cell vectors
    int max_colours = 0;                 // most sub-colours in a patch
    uint8_t *d_colour = nullptr, *d_patch_ncol = nullptr;
    int32_t *d_patch_off = nullptr, *d_patch_nodes = nullptr;
    int32_t *d_patch_nint = nullptr, *d_patch_pbase = nullptr;
    int32_t *d_csr_off = nullptr;
    uint16_t *d_csr_slots = nullptr;
    int32_t *d_fix_node = nullptr, *d_fix_off = nullptr;
    int32_t *d_pdest = nullptr;          // node-major partial slot of each (patch, shared node)
    double *d_partial = nullptr;
    int64_t pstride = 0;
    std::vector<double> h_coords;        // host copies, to rebuild patches on request
    std::vector<int32_t> h_cell_verts, h_cell_nodes;
    // optional event timing of the main kernel launches (fem_plan_set_timing); mutable
    // because the action itself takes a const plan
    bool timing = false;
    mutable std::vector<std::pair<hipEvent_t, hipEvent_t>> timing_pending, timing_free;
    mutable double timing_ms = 0.0;
    mutable int64_t timing_calls = 0;
};

namespace femx {
// Kernel launchers (kernels.hip).  Return hipSuccess or the launch error.
bool kernel_available(int form, int dim, int degree);
hipError_t launch_action(const fem_plan &p, const LaunchArgs &a, int block, bool vjp,
                         hipStream_t s);
hipError_t launch_zero_nodes(const int32_t *nodes, int64_t n, int ncomp, double *y,
                             hipStream_t s);
// LDS bytes the patch kernel needs for a patch of `patch` cells with at most
// `max_nodes` distinct nodes.
size_t patch_lds_bytes(int form, int dim, int degree, bool vjp, int patch, int max_nodes,
                       int sum_mode, int lanes = 1);
size_t patch_lds_a(int form, int dim, int degree, bool vjp, int patch, int max_nodes, int sum_mode,
                   int lanes = 1);
// start / stop (optional): events the dispatch itself stamps at the kernel's start and end
// The pipelined mass patch kernel runs this plan's action (launch_patch takes it), and
// its compiled registers and scratch bytes.
bool mass_pipe_used(const fem_plan &p, bool vjp);
int mass_pipe_info(const fem_plan &p, int *regs, int *scratch);
hipError_t launch_patch(const fem_plan &p, const PatchArgs &a, bool vjp, hipStream_t s,
                        hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// the hyperelastic forms: nonlinear residuals whose VJP is a tangent action at u
inline bool nonlinear_form(int form) { return form == FEM_NEOHOOKEAN || form == FEM_SVK; }
// scalar forms carry one component per node, vector forms dim (host and device)
constexpr bool scalar_form(int form)
{
    return form == FEM_MASS || form == FEM_LAPLACE || form == FEM_HELMHOLTZ;
}
constexpr int ncomp_of(int form, int dim) { return scalar_form(form) ? 1 : dim; }
bool pair_available(int form, int dim, int degree);
bool curved_available(int form, int dim, int degree);
bool batch_available(int form, int dim, int degree, int lanes, int sum_mode);
bool triple_available(int form, int dim, int degree);
// lane triples on P2-geometry cells (3D vector forms up to P4)
bool curved_triple_available(int form, int dim, int degree);
// the matrix-core patch kernel ("four lanes per cell": 16 cells per tile, each cell's points
// and nodes over four lanes) of the vector forms on affine cells
bool mfma_available(int form, int dim, int degree);
constexpr int kMfmaLanes = 4;
int kernel_registers(int form, int dim, int degree, bool vjp, bool colour, int lanes,
                     int sum_mode, int geom = 1);
// registers per lane, scratch bytes per lane and whether the wave-priority variant runs, of
// the kernel a configuration launches; -1 if that kernel is not built
int kernel_info(int form, int dim, int degree, bool vjp, bool colour, int lanes, int sum_mode,
                int geom, int *regs, int *scratch, int *prio);
// whether the hyperelastic tangent (VJP) kernel of a configuration uses scratch memory: such
// kernels are not run (two of them, heavily spilling, returned wrong values)
bool vjp_kernel_spills(int form, int dim, int degree, bool colour, int lanes, int sum_mode,
                       int geom);
// geometry nodes of a cell: the d+1 vertices, or the P2 lattice of a curved cell
inline int cell_geom_nodes(int dim, int geom) { return geom == 2 ? (dim == 2 ? 6 : 10) : dim + 1; }
int patch_threads(int P, int lanes);
hipError_t launch_batch_patch(int form, int dim, int degree, int lanes, int patch, int sum_mode,
                              const BatchDesc *desc, const int32_t *patch_mesh, int64_t n_patch,
                              size_t lds, hipStream_t s);
hipError_t launch_batch_fixup(const FixDesc *fix, int n_mesh, int64_t n, hipStream_t s);
// plan.cpp (throwing versions of the ABI calls, for the tuner and the batch)
void set_strategy(fem_plan *plan, int strategy, int patch_cells, int lanes_per_cell, int sum_mode);
void run_action(const fem_plan *p, const double *u, const double *v, double *y, hipStream_t s,
                bool vjp);
// tune.cpp
void apply_tuning_cache(fem_plan *p);
int tune(fem_plan *p, const double *u, const double *v, double *y, bool vjp, const char *cache,
         hipStream_t s, double *results, int max_results, int *n_results, int max_timed);
int tune_predict(const fem_plan *p, bool vjp, double *results, int max_results, int *n_results);
// the device address of this device's static scratch array (FEM_NOALLOC_SCRATCH_DOUBLES
// doubles), looked up once per device with that device current (kernels.hip)
double *static_scratch(int device);
// measurement aids (kernels.hip): STREAM copy and a read-only pass into per-block sums
hipError_t launch_stream_copy(const double *src, double *dst, int64_t n, hipStream_t s);
hipError_t launch_stream_read(const double *src, int64_t n, double *sink, hipStream_t s);
int stream_sink_size();
hipError_t launch_fixup(const int32_t *fix_node, const int32_t *fix_off,
                        int64_t n_shared, const double *partial, int ncomp, double *y,
                        hipStream_t s);
}  // namespace femx

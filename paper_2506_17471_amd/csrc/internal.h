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
RefTables reference_tables(int dim, int degree, int quad_degree);

// Kernel-side table layout: per quadrature point a contiguous record.
//   mass:  [phi_0 .. phi_{nloc-1}, w]                       (nloc + 1 doubles)
//   vector forms: [dphi_r(a) for r in 0..d-1 for a, w]      (d*nloc + 1 doubles)
// padded to an even number of doubles so every record starts 16-byte aligned.
int table_record(int form, int dim, int nloc);
std::vector<double> kernel_table(int form, const RefTables &t);

// Launch parameters of one colour class.
struct LaunchArgs {
    const int32_t *verts;     // SoA [(dim+1)][stride] colour-sorted vertex ids
    const int32_t *nodes;     // SoA [nloc][stride]    colour-sorted node ids
    const uint64_t *first;    // [stride] bit a: this cell is first to write node a
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

}  // namespace femx

struct fem_plan {
    int form = 0, dim = 0, degree = 0, quad_degree = 0, nloc = 0, ncomp = 0, nq = 0;
    int64_t n_vert = 0, n_cell = 0, n_node = 0, n_dof = 0;
    double lam = 0.0, mu = 0.0;
    int n_colours = 0;
    int block = 0;                       // cells per workgroup (0 = default)
    int device = 0;
    std::vector<int64_t> colour_off;     // [n_colours + 1] in colour-sorted order
    std::vector<int32_t> colour;         // [n_cell] colour of each caller cell
    int64_t stride = 0;                  // padded column length of the SoA maps
    double *d_coords = nullptr;
    int32_t *d_verts = nullptr;
    int32_t *d_nodes = nullptr;
    uint64_t *d_first = nullptr;
    double *d_tab = nullptr;
    int32_t *d_untouched = nullptr;      // nodes no cell holds (zeroed separately)
    int64_t n_untouched = 0;
};

namespace femx {
// Kernel launchers (kernels.hip).  Return hipSuccess or the launch error.
bool kernel_available(int form, int dim, int degree);
hipError_t launch_action(const fem_plan &p, const LaunchArgs &a, int block, bool vjp,
                         hipStream_t s);
hipError_t launch_zero_nodes(const int32_t *nodes, int64_t n, int ncomp, double *y,
                             hipStream_t s);
}  // namespace femx

// Launchers of the matrix-free action kernels for gfx950 (CDNA4); the kernel templates
// live in kernel_templates.h and are instantiated per form in kernels_<form>.hip.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <map>
#include <mutex>
#include <set>

#include "kernel_templates.h"

namespace femx {
namespace {

// Shared-node sums of many meshes: thread i sums shared node i - fix[m].first of the mesh m
// whose range holds i (binary search over the meshes' first indices).
// (`first` counts (node, component) items, so meshes of different ncomp mix freely)
__global__ void batch_fixup_kernel(const FixDesc *__restrict__ fix, int n_mesh, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = n_mesh - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (fix[mid].first <= i) lo = mid; else hi = mid - 1;
    }
    const FixDesc &f = fix[lo];
    const int64_t item = i - f.first;
    const int64_t k = item / f.ncomp;
    const int c = (int)(item - k * f.ncomp);
    const int64_t nd = f.fix_node[k];
    const int o0 = f.fix_off[k], o1 = f.fix_off[k + 1];
    double s = 0.0;
    for (int o = o0; o < o1; ++o) s += f.partial[(int64_t)o * f.ncomp + c];
    f.y[nd * f.ncomp + c] = s;
}

// thread i sums component i % ncomp of shared node i / ncomp over its partials, which lie
// contiguously in node-major order (one per holding patch, in patch order)
__global__ void fixup_kernel(const int32_t *__restrict__ fix_node, const int32_t *__restrict__ fix_off,
                             int64_t n, const double *__restrict__ partial, int ncomp,
                             double *__restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * ncomp) return;
    const int64_t k = i / ncomp;
    const int c = (int)(i - k * ncomp);
    const int64_t nd = fix_node[k];
    const int o0 = fix_off[k], o1 = fix_off[k + 1];
    double s = 0.0;
    for (int o = o0; o < o1; ++o) s += partial[(int64_t)o * ncomp + c];
    y[nd * ncomp + c] = s;
}

__global__ void zero_nodes_kernel(const int32_t *__restrict__ nodes, int64_t n, int ncomp,
                                  double *__restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t nd = nodes[i];
    for (int c = 0; c < ncomp; ++c) y[nd * ncomp + c] = 0.0;
}

// Measurement aids: the achievable HBM bandwidth (a STREAM-style copy, every byte read
// once and written once) and a read-only pass (each workgroup's sum of its share written to
// sink[block]) that evicts the caches without leaving dirty lines behind.  Grid-stride over
// 16-byte elements, one element per lane per trip over up to 65536 workgroups (measured
// fastest of the grid-stride, chunked and unrolled forms on MI355X); the copy uses
// nontemporal (streaming) loads and stores, the read pass ordinary loads, so that its lines
// are allocated in L2 and the memory-side cache and push out what they held (with streaming
// loads a P2 mass action timed after the pass ran as fast as warm).  The scalar tail (n
// odd) goes to the last lane.
constexpr int kStreamBlock = 256;
typedef double dv2 __attribute__((ext_vector_type(2)));

__global__ void __launch_bounds__(kStreamBlock)
    stream_copy_kernel(const dv2 *__restrict__ src, dv2 *__restrict__ dst, int64_t n2,
                       const double *__restrict__ tail_src, double *__restrict__ tail_dst)
{
    const int64_t stride = (int64_t)gridDim.x * kStreamBlock;
    for (int64_t i = (int64_t)blockIdx.x * kStreamBlock + threadIdx.x; i < n2; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
    if (tail_src && blockIdx.x == gridDim.x - 1 && threadIdx.x == kStreamBlock - 1) *tail_dst = *tail_src;
}

__global__ void __launch_bounds__(kStreamBlock)
    stream_read_kernel(const dv2 *__restrict__ src, int64_t n2, const double *__restrict__ tail,
                       double *__restrict__ sink)
{
    __shared__ double part[kStreamBlock / 64];
    const int64_t stride = (int64_t)gridDim.x * kStreamBlock;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kStreamBlock + threadIdx.x; i < n2; i += stride) {
        const dv2 a = src[i];
        acc += a.x + a.y;
    }
    double v = acc;
    if (tail && blockIdx.x == gridDim.x - 1 && threadIdx.x == kStreamBlock - 1) v += *tail;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kStreamBlock / 64; ++w) t += part[w];
        sink[blockIdx.x] = t;
    }
}

Kernels lookup(int form, int dim, int degree, bool vjp)
{
    switch (form) {
    case FEM_MASS: return lookup_mass(dim, degree, vjp);
    case FEM_ELASTICITY: return lookup_elasticity(dim, degree, vjp);
    case FEM_NEOHOOKEAN: return lookup_neohookean(dim, degree, vjp);
    case FEM_SVK: return lookup_svk(dim, degree, vjp);
    case FEM_LAPLACE: return lookup_laplace(dim, degree, vjp);
    case FEM_HELMHOLTZ: return lookup_helmholtz(dim, degree, vjp);
    default: return Kernels{};
    }
}

}  // namespace

// The wave-priority variant of a coloured affine patch kernel runs only where its compiled
// form uses no scratch memory (spill-free); FEM_WAVE_PRIORITY=0 in the environment turns the
// hints off everywhere.  Decided once per kernel (function attributes, no launch).
static bool prio_usable(const void *hinted)
{
    if (!hinted) return false;
    static const bool enabled = [] {
        const char *e = std::getenv("FEM_WAVE_PRIORITY");
        return !(e && e[0] == '0');
    }();
    if (!enabled) return false;
    static std::mutex mu;
    static std::map<const void *, bool> known;
    std::lock_guard<std::mutex> g(mu);
    auto it = known.find(hinted);
    if (it != known.end()) return it->second;
    hipFuncAttributes attr{};
    bool ok = false;
    if (hipFuncGetAttributes(&attr, hinted) == hipSuccess) ok = attr.localSizeBytes == 0;
    else (void)hipGetLastError();
    known.emplace(hinted, ok);
    return ok;
}

// the patch kernel a plan's configuration launches (geom 2: the one-lane curved kernels)
static const void *patch_fn(const Kernels &ks, int geom, int lanes, int sum_mode,
                            bool *prio = nullptr)
{
    if (prio) *prio = false;
    if (lanes < 1 || lanes > kMfmaLanes || sum_mode < 1 || sum_mode > 2) return nullptr;
    if (geom == 2)
        return lanes == 1 ? (const void *)ks.patch_p2[sum_mode]
                          : (lanes == 3 ? (const void *)ks.patch_p2_3[sum_mode] : nullptr);
    if (sum_mode == SUM_COLOURED && prio_usable((const void *)ks.patch_prio[lanes])) {
        if (prio) *prio = true;
        return (const void *)ks.patch_prio[lanes];
    }
    return (const void *)ks.patch[lanes][sum_mode];
}

bool kernel_available(int form, int dim, int degree)
{
    return lookup(form, dim, degree, false).colour != nullptr;
}

hipError_t launch_action(const fem_plan &p, const LaunchArgs &a, int block, bool vjp,
                         hipStream_t s)
{
    const Kernels ks = lookup(p.form, p.dim, p.degree, vjp);
    ColourFn fn = p.geom == 2 ? ks.colour_p2 : ks.colour;
    if (!fn) return hipErrorInvalidDeviceFunction;
    if (block <= 0) block = 64;
    if (block > kMaxBlock) return hipErrorInvalidConfiguration;
    const int64_t grid = (a.count + block - 1) / block;
    if (grid > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(block), 0, s, a);
    return hipGetLastError();
}

// LDS region A (doubles): the staged nodal values, then the element buffer (SUM_ELEMENT)
// or the node accumulator (SUM_COLOURED), which fits in the staging space.
// (the matrix-core kernel reads the staged values through its whole loop and reuses the
// space for the node accumulator after it: the coloured sums' size)
size_t patch_lds_a(int form, int dim, int degree, bool vjp, int patch, int max_nodes, int sum_mode,
                   int lanes)
{
    const int nloc = nloc_of(dim, degree);
    const int nc = ncomp_of(form, dim);
    const size_t stage = (size_t)max_nodes * nc * (vjp ? 2 : 1);
    if (lanes == kMfmaLanes) return stage;
    if (sum_mode == SUM_COLOURED) return stage;
    const size_t elem = (size_t)patch * nloc * nc;
    return stage > elem ? stage : elem;
}

// Region B (bytes): node ids, plus for the element buffer the relative sum offsets and slots.
size_t patch_lds_bytes(int form, int dim, int degree, bool vjp, int patch, int max_nodes,
                       int sum_mode, int lanes)
{
    const int nloc = nloc_of(dim, degree);
    size_t b = 4 * (size_t)max_nodes;
    if (sum_mode == SUM_ELEMENT) b += 4 * ((size_t)max_nodes + 1) + 2 * (size_t)patch * nloc;
    return 8 * patch_lds_a(form, dim, degree, vjp, patch, max_nodes, sum_mode, lanes) +
           ((b + 7) & ~(size_t)7);
}

// curved (P2-geometry) and batch kernels exist up to P6 (2D) / P4 (3D)
bool curved_available(int form, int dim, int degree)
{
    return lookup(form, dim, degree, false).colour_p2 != nullptr;
}

bool batch_available(int form, int dim, int degree, int lanes, int sum_mode)
{
    if (lanes < 1 || lanes > kMfmaLanes || sum_mode < 1 || sum_mode > 2) return false;
    return lookup(form, dim, degree, false).batch[lanes][sum_mode] != nullptr;
}

bool pair_available(int form, int dim, int degree)
{
    return lookup(form, dim, degree, false).patch[2][SUM_ELEMENT] != nullptr;
}

bool mfma_available(int form, int dim, int degree)
{
    return lookup(form, dim, degree, false).patch[kMfmaLanes][SUM_COLOURED] != nullptr;
}

bool curved_triple_available(int form, int dim, int degree)
{
    return lookup(form, dim, degree, false).patch_p2_3[SUM_COLOURED] != nullptr;
}

bool triple_available(int form, int dim, int degree)
{
    return lookup(form, dim, degree, false).patch[3][SUM_ELEMENT] != nullptr;
}

// Registers per lane of the kernel a launch configuration runs (the compiled kernel's
// attributes), 0 if that kernel is not built.
int kernel_registers(int form, int dim, int degree, bool vjp, bool colour, int lanes,
                     int sum_mode, int geom)
{
    const Kernels ks = lookup(form, dim, degree, vjp);
    const bool ok = lanes >= 1 && lanes <= kMfmaLanes && sum_mode >= 1 && sum_mode <= 2;
    const void *fn = nullptr;
    if (colour)
        fn = geom == 2 ? (const void *)ks.colour_p2 : (const void *)ks.colour;
    else if (ok)
        fn = patch_fn(ks, geom, lanes, sum_mode);
    if (!fn) return 0;
    hipFuncAttributes attr{};
    if (hipFuncGetAttributes(&attr, fn) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return attr.numRegs;
}

// scratch bytes per lane of a compiled kernel (function attributes, cached; -1 unknown)
static int scratch_bytes(const void *fn)
{
    static std::mutex mu;
    static std::map<const void *, int> known;
    std::lock_guard<std::mutex> g(mu);
    auto it = known.find(fn);
    if (it != known.end()) return it->second;
    hipFuncAttributes attr{};
    int b = -1;
    if (hipFuncGetAttributes(&attr, fn) == hipSuccess) b = (int)attr.localSizeBytes;
    else (void)hipGetLastError();
    known.emplace(fn, b);
    return b;
}

bool vjp_kernel_spills(int form, int dim, int degree, bool colour, int lanes, int sum_mode, int geom)
{
    const Kernels ks = lookup(form, dim, degree, true);
    const void *fn = colour ? (geom == 2 ? (const void *)ks.colour_p2 : (const void *)ks.colour)
                            : patch_fn(ks, geom, lanes, sum_mode);
    return fn && scratch_bytes(fn) != 0;
}

int kernel_info(int form, int dim, int degree, bool vjp, bool colour, int lanes, int sum_mode,
                int geom, int *regs, int *scratch, int *prio)
{
    const Kernels ks = lookup(form, dim, degree, vjp);
    bool hinted = false;
    const void *fn = colour ? (geom == 2 ? (const void *)ks.colour_p2 : (const void *)ks.colour)
                            : patch_fn(ks, geom, lanes, sum_mode, &hinted);
    if (!fn) return -1;
    hipFuncAttributes attr{};
    if (hipFuncGetAttributes(&attr, fn) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    if (regs) *regs = attr.numRegs;
    if (scratch) *scratch = (int)attr.localSizeBytes;
    if (prio) *prio = hinted ? 1 : 0;
    return 0;
}

// threads of a patch workgroup: P * lanes, 64 per 21 cells for lane triples, 256 (16 cells
// per wavefront) for the matrix-core kernel
int patch_threads(int P, int lanes)
{
    return lanes == 3 ? 64 * ((P + 20) / 21) : P * lanes;
}

hipError_t allow_lds(const void *fn, size_t lds)
{
    if (lds <= 64 * 1024) return hipSuccess;
    static std::mutex mu;
    static std::set<const void *> raised;
    std::lock_guard<std::mutex> g(mu);
    if (raised.count(fn)) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e == hipSuccess) raised.insert(fn);
    return e;
}

hipError_t launch_batch_patch(int form, int dim, int degree, int lanes, int patch, int sum_mode,
                              const BatchDesc *desc, const int32_t *patch_mesh, int64_t n_patch,
                              size_t lds, hipStream_t s)
{
    if (lanes < 1 || lanes > kMfmaLanes || sum_mode < SUM_ELEMENT || sum_mode > SUM_COLOURED)
        return hipErrorInvalidConfiguration;
    const Kernels ks = lookup(form, dim, degree, false);
    BatchFn fn = ks.batch[lanes][sum_mode];
    if (sum_mode == SUM_COLOURED && prio_usable((const void *)ks.batch_prio[lanes]))
        fn = ks.batch_prio[lanes];
    if (!fn) return hipErrorInvalidDeviceFunction;
    const int threads = patch_threads(patch, lanes);
    if (patch < 1 || patch > 256 || threads > kMaxBlock || lds > 160 * 1024 || n_patch > 0x7fffffff)
        return hipErrorInvalidConfiguration;
    hipError_t e = allow_lds((const void *)fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3((unsigned)n_patch), dim3(threads), lds, s, desc, patch_mesh, patch);
    return hipGetLastError();
}

hipError_t launch_batch_fixup(const FixDesc *fix, int n_mesh, int64_t n, hipStream_t s)
{
    const int block = 256;
    const int64_t grid = (n + block - 1) / block;
    hipLaunchKernelGGL(batch_fixup_kernel, dim3((unsigned)grid), dim3(block), 0, s, fix, n_mesh, n);
    return hipGetLastError();
}


// Mass patches, pipelined: each resident workgroup walks its patches (in the XCD-aware
// order) and, while it works on one, has the next one's loads in flight: the patch header,
// node ids, partial slots and the cells' maps during this patch's quadrature loop, the
// nodal values and vertex coordinates (which depend on them) during its sub-colour sums.
// The per-node and per-cell arithmetic and the sum order are the patch kernel's, so the
// results are bitwise the same.  A lane stages nodes tid, tid + P, ... (at most kPipeNodes
// of them) and writes the same ones out, so their ids stay in its registers.  The next
// patch's state costs registers (90 VGPRs at P2 on triangles: five waves per SIMD against
// the patch kernel's eight), which pays on the 2D P2 mass form only: P2 on 1024 x 1024
// squares 42.4 -> 40.9 us per action warm, 64.7 -> 60.3 cold; P1 on triangles within 1%
// warm; P1 and P2 on tetrahedra 15-20% slower.  Bounding it to six or eight waves spills.
constexpr int kPipeNodes = 4;

struct PipeHead {
    int nb, U, nint, pbase, ncol;
};

__device__ __forceinline__ PipeHead pipe_head(const PatchArgs &a, int64_t p)
{
    PipeHead h;
    h.nb = a.patch_off[p];
    h.U = a.patch_off[p + 1] - h.nb;
    h.nint = a.patch_nint[p];
    h.pbase = a.patch_pbase[p];
    h.ncol = a.patch_ncol[p];
    return h;
}

// loads that need only the header: node ids (clamped to the patch's last node), partial
// slots of the shared ones, and the cell's maps (the maps are padded to whole patches)
template <int DIM, int NLOC>
__device__ __forceinline__ void pipe_maps(const PatchArgs &a, const PipeHead &h, int64_t p, int P,
                                          int tid, int32_t (&nd)[kPipeNodes],
                                          int32_t (&pd)[kPipeNodes], int32_t (&vt)[DIM + 1],
                                          int (&lid)[NLOC], int &col)
{
#pragma unroll
    for (int jj = 0; jj < kPipeNodes; ++jj) nd[jj] = a.patch_nodes[h.nb + min(tid + jj * P, h.U - 1)];
#pragma unroll
    for (int jj = 0; jj < kPipeNodes; ++jj) {
        const int j = tid + jj * P;
        pd[jj] = (j >= h.nint && j < h.U) ? a.pdest[h.pbase + (j - h.nint)] : 0;
    }
    const int64_t s = p * P + tid;
#pragma unroll
    for (int v = 0; v <= DIM; ++v) vt[v] = a.verts[v * a.stride + s];
#pragma unroll
    for (int n = 0; n < NLOC; ++n) lid[n] = a.lidx[n * a.stride + s];
    col = a.colour[s];
}

template <int DIM>
__device__ __forceinline__ void pipe_values(const PatchArgs &a, const int32_t (&nd)[kPipeNodes],
                                            const int32_t (&vt)[DIM + 1], double (&uv)[kPipeNodes],
                                            double (&x)[DIM + 1][DIM])
{
#pragma unroll
    for (int jj = 0; jj < kPipeNodes; ++jj) uv[jj] = a.u[nd[jj]];
#pragma unroll
    for (int v = 0; v <= DIM; ++v)
#pragma unroll
        for (int i = 0; i < DIM; ++i) x[v][i] = a.coords[(int64_t)vt[v] * DIM + i];
}

template <int DIM, int K>
__global__ void __launch_bounds__(kMaxBlock) mass_pipe_kernel(const PatchArgs a, int P, int64_t n_patch)
{
    constexpr int NLOC = nloc_of(DIM, K);
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int64_t G = gridDim.x;
    int64_t q = blockIdx.x;
    int64_t p = xcd_order(q, n_patch);
    PipeHead h = pipe_head(a, p);
    int32_t nd[kPipeNodes], pd[kPipeNodes], vt[DIM + 1];
    int lid[NLOC], col;
    pipe_maps<DIM, NLOC>(a, h, p, P, tid, nd, pd, vt, lid, col);
    double uv[kPipeNodes], adet;
    {
        double x[DIM + 1][DIM], Kd[DIM][DIM];
        pipe_values<DIM>(a, nd, vt, uv, x);
        adet = affine_geometry<DIM>(x, Kd);
    }
    const double Kz[DIM][DIM] = {};
    const double gz[DIM + 1][DIM] = {};
    for (; q < n_patch; q += G) {
        const bool active = tid < P && p * P + tid < a.n_cell;
        // 1. this patch's values into LDS, then each cell's from there
#pragma unroll
        for (int jj = 0; jj < kPipeNodes; ++jj) {
            const int j = tid + jj * P;
            if (j < h.U) lds[j] = uv[jj];
        }
        __syncthreads();
        double ul[NLOC][1], vl[1][1] = {{0.0}}, yl[NLOC][1];
        if (active) {
#pragma unroll
            for (int n = 0; n < NLOC; ++n) ul[n][0] = lds[lid[n]];
        }
        __syncthreads();
        for (int j = tid; j < h.U; j += P) lds[j] = 0.0;
        // 2. the next patch's header, ids, slots and maps
        const int64_t qn = q + G;
        const int64_t pn = qn < n_patch ? xcd_order(qn, n_patch) : p;
        const PipeHead hn = pipe_head(a, pn);
        int32_t ndn[kPipeNodes], pdn[kPipeNodes], vtn[DIM + 1];
        int lidn[NLOC], coln;
        pipe_maps<DIM, NLOC>(a, hn, pn, P, tid, ndn, pdn, vtn, lidn, coln);
        // 3. this patch's quadrature
        if (active)
            cell_quadrature<FEM_MASS, DIM, K, false, 1>(ul, vl, Kz, adet, gz, a.tab, a.nq, a.lam,
                                                         a.mu, yl);
        // 4. the next patch's values and coordinates
        double uvn[kPipeNodes], xn[DIM + 1][DIM];
        pipe_values<DIM>(a, ndn, vtn, uvn, xn);
        // 5. sub-colour sums, as in the patch kernel
        __syncthreads();
        for (int k = 0; k < h.ncol; ++k) {
            if (active && col == k) {
#pragma unroll
                for (int n = 0; n < NLOC; ++n)
                    __hip_atomic_fetch_add(&lds[lid[n]], yl[n][0], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            __syncthreads();
        }
        // 6. each node once: interior ones into y, shared ones as partials
#pragma unroll
        for (int jj = 0; jj < kPipeNodes; ++jj) {
            const int j = tid + jj * P;
            if (j < h.U) {
                const double sum = lds[j];
                if (j < h.nint) a.y[nd[jj]] = sum;
                else a.partial[pd[jj]] = sum;
            }
        }
        __syncthreads();
        // 7. the next patch becomes this one
        p = pn;
        h = hn;
#pragma unroll
        for (int jj = 0; jj < kPipeNodes; ++jj) {
            nd[jj] = ndn[jj];
            pd[jj] = pdn[jj];
            uv[jj] = uvn[jj];
        }
#pragma unroll
        for (int n = 0; n < NLOC; ++n) lid[n] = lidn[n];
        col = coln;
        double Kd[DIM][DIM];
        adet = affine_geometry<DIM>(xn, Kd);
    }
}

// the pipelined mass kernel of (dim, degree) where it is used, or null
static const void *mass_pipe_fn(int dim, int degree)
{
    return dim == 2 && degree == 2 ? (const void *)mass_pipe_kernel<2, 2> : nullptr;
}

bool mass_pipe_used(const fem_plan &p, bool vjp)
{
    return p.form == FEM_MASS && !vjp && p.geom == 1 && p.lanes == 1 &&
           p.sum_mode == SUM_COLOURED && p.patch == 256 && p.n_patch > 0 &&
           p.max_patch_nodes <= kPipeNodes * p.patch && mass_pipe_fn(p.dim, p.degree) != nullptr;
}

int mass_pipe_info(const fem_plan &p, int *regs, int *scratch)
{
    const void *fn = mass_pipe_fn(p.dim, p.degree);
    hipFuncAttributes attr{};
    if (!fn || hipFuncGetAttributes(&attr, fn) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    if (regs) *regs = attr.numRegs;
    if (scratch) *scratch = (int)attr.localSizeBytes;
    return 0;
}

hipError_t launch_patch(const fem_plan &p, const PatchArgs &a, bool vjp, hipStream_t s,
                        hipEvent_t start, hipEvent_t stop)
{
    if (p.lanes < 1 || p.lanes > kMfmaLanes ||
        p.sum_mode < SUM_ELEMENT || p.sum_mode > SUM_COLOURED)
        return hipErrorInvalidConfiguration;
    if (p.lanes == kMfmaLanes && (p.patch != 64 || !a.mtab || a.nqt < 1))
        return hipErrorInvalidConfiguration;
    const Kernels ks = lookup(p.form, p.dim, p.degree, vjp);
    // curved cells run the one-lane kernels only
    PatchFn fn = (PatchFn)patch_fn(ks, p.geom, p.lanes, p.sum_mode);
    if (!fn) return hipErrorInvalidDeviceFunction;
    const int threads = patch_threads(p.patch, p.lanes);
    if (p.patch < 1 || p.patch > 256 || threads > kMaxBlock) return hipErrorInvalidConfiguration;
    const size_t lds = patch_lds_bytes(p.form, p.dim, p.degree, vjp, p.patch, p.max_patch_nodes,
                                       p.sum_mode, p.lanes);
    if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
    hipError_t e = allow_lds((const void *)fn, lds);
    if (e != hipSuccess) return e;
    if (p.n_patch > 0x7fffffff) return hipErrorInvalidConfiguration;
    if (mass_pipe_used(p, vjp)) {
        // as many workgroups as stay resident, a multiple of the 8 XCDs (workgroup b runs on
        // XCD b mod 8 and so do all the patches it takes: xcd_order keeps them together)
        const void *pipe = mass_pipe_fn(p.dim, p.degree);
        int dev = 0, ncu = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pipe, threads, lds) != hipSuccess ||
            per_cu < 1)
            return hipErrorInvalidConfiguration;
        e = allow_lds(pipe, lds);
        if (e != hipSuccess) return e;
        int64_t G = std::min<int64_t>(p.n_patch, (int64_t)per_cu * ncu);
        if (G >= 8) G -= G % 8;
        PatchArgs args = a;
        int P = p.patch;
        int64_t np = p.n_patch;
        void *kargs[] = {(void *)&args, (void *)&P, (void *)&np};
        return hipExtLaunchKernel(pipe, dim3((unsigned)G), dim3(threads), kargs, lds, s, start, stop, 0);
    }
    if (start || stop) {
        // timed: the events are stamped by the dispatch at the kernel's own start and end
        PatchArgs args = a;
        int P = p.patch;
        void *kargs[] = {(void *)&args, (void *)&P};
        return hipExtLaunchKernel((const void *)fn, dim3((unsigned)p.n_patch), dim3(threads), kargs,
                                  lds, s, start, stop, 0);
    }
    hipLaunchKernelGGL(fn, dim3((unsigned)p.n_patch), dim3(threads), lds, s, a, p.patch);
    return hipGetLastError();
}

hipError_t launch_fixup(const int32_t *fix_node, const int32_t *fix_off, int64_t n_shared,
                        const double *partial, int ncomp, double *y, hipStream_t s)
{
    const int block = 256;
    const int64_t grid = (n_shared * ncomp + block - 1) / block;
    hipLaunchKernelGGL(fixup_kernel, dim3((unsigned)grid), dim3(block), 0, s, fix_node, fix_off,
                       n_shared, partial, ncomp, y);
    return hipGetLastError();
}

// Static scratch for fem_action_noalloc: the shared nodes' partial sums of one action, in a
// file-scope device array (each device holds its own copy, at its own address, until the
// process ends).  Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address): it uses the address hipGetSymbolAddress returns, looked
// up once per device with that device current.
static __device__ __align__(256) double scratch[FEM_NOALLOC_SCRATCH_DOUBLES];

double *static_scratch(int device)
{
    static std::mutex mu;
    static std::map<int, double *> ptrs;
    std::lock_guard<std::mutex> g(mu);
    auto it = ptrs.find(device);
    if (it != ptrs.end()) return it->second;
    int cur = -1;
    check_hip(hipGetDevice(&cur), "hipGetDevice");
    if (cur != device) throw Error(FEM_E_ARG, "scratch lookup needs its device current");
    double *ptr = nullptr;
    check_hip(hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) throw Error(FEM_E_HIP, "null scratch address");
    ptrs.emplace(device, ptr);
    return ptr;
}

// up to 65536 workgroups of 256 lanes (the read pass writes one partial sum per workgroup)
constexpr int kStreamGrid = 65536;

static unsigned stream_grid(int64_t n2)
{
    const int64_t g = (n2 + kStreamBlock - 1) / kStreamBlock;
    return (unsigned)(g < 1 ? 1 : (g > kStreamGrid ? kStreamGrid : g));
}

hipError_t launch_stream_copy(const double *src, double *dst, int64_t n, hipStream_t s)
{
    const int64_t n2 = n / 2;
    const bool odd = n & 1;
    hipLaunchKernelGGL(stream_copy_kernel, dim3(stream_grid(n2)), dim3(kStreamBlock), 0, s,
                       (const dv2 *)src, (dv2 *)dst, n2, odd ? src + n - 1 : nullptr,
                       odd ? dst + n - 1 : nullptr);
    return hipGetLastError();
}

hipError_t launch_stream_read(const double *src, int64_t n, double *sink, hipStream_t s)
{
    const int64_t n2 = n / 2;
    hipLaunchKernelGGL(stream_read_kernel, dim3(stream_grid(n2)), dim3(kStreamBlock), 0, s,
                       (const dv2 *)src, n2, (n & 1) ? src + n - 1 : nullptr, sink);
    return hipGetLastError();
}

int stream_sink_size() { return kStreamGrid; }

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

// Throughput probe: FP64 matrix cores against the FP64 vector path for the evaluation
// contraction of the quadrature loop (paper Sec. 3: the reference gradients at the points,
// interpolated from the cell's nodal values; the same product, transposed, is the test
// function contraction).  For every column c (one component of one cell) and every row m
// (one (reference direction, quadrature point) pair):
//     g[m][c] = sum_k T[m][k] u[k][c]
// with T the reference gradient tabulation (M = dim * Q rows, K = n_loc columns).
// Two kernels compute the same contraction in FP64:
//   valu: one lane per column, u in registers, T read through scalar loads (the layout of the
//         action kernels);
//   mfma: 16x16x4 FP64 matrix-core tiles, T staged in LDS in fragment order, 64 columns per
//         wavefront (four 16-column tiles sharing each T fragment).
// Each folds its outputs into a per-column sum of squares (so stores do not bound it) and
// repeats the contraction `reps` times on u <- 0.75 u + 0.125 (so loads do not bound it); the
// two checksums are compared at the end.  Stand-alone: it shares nothing with the library.
//
//     contraction_probe p4|p8 [ncols] [reps] [iters]
//       p4: neo-Hookean P4 on triangles, 16-point rule: K = 15, M = 2 * 16
//       p8: P8 on triangles, 81-point rule (degree 16): K = 45, M = 2 * 81
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#define CHECK(x)                                                                          \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) {                                                           \
            std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));           \
            std::exit(2);                                                                 \
        }                                                                                 \
    } while (0)

typedef double dvec4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;

template <int K, int M>
struct Shape {
    static constexpr int KP = (K + 3) / 4 * 4;      // K padded to the MFMA k-step
    static constexpr int MP = (M + 15) / 16 * 16;   // M padded to the MFMA row tile
    static constexpr int KS = KP / 4;
    static constexpr int MT = MP / 16;
    static constexpr int FRAG = MT * KS * 64;       // doubles of T in fragment order
};

// T: [M][K] dense.  U: [KP][ncols], rows K..KP-1 zero.  One lane per column.
template <int K, int M>
__global__ __launch_bounds__(kThreads) void contract_valu(const double *__restrict__ T,
                                                          const double *__restrict__ U,
                                                          int64_t ncols, int reps,
                                                          double *__restrict__ out)
{
    const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (c >= ncols) return;
    double u[K];
#pragma unroll
    for (int k = 0; k < K; ++k) u[k] = U[k * ncols + c];
    double s = 0.0;
    for (int r = 0; r < reps; ++r) {
#pragma unroll 2
        for (int m = 0; m < M; ++m) {
            double g = 0.0;
#pragma unroll
            for (int k = 0; k < K; ++k) g = fma(T[m * K + k], u[k], g);
            s = fma(g, g, s);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) u[k] = fma(u[k], 0.75, 0.125);
    }
    out[c] = s;
}

// Tf: T padded to [MP][KP] with zeros and stored in fragment order: entry
// ((t * KS + s) * 64 + l) is T[16 t + l % 16][4 s + l / 16], the A operand of lane l for row
// tile t and k-step s.  The B operand of lane l for column tile j and k-step s is
// u[4 s + l / 16][col0 + 16 j + l % 16]; the result's column is l % 16, the row within the
// tile set by l / 16, so each column's 16 rows sit in the four lanes l % 16 + {0,16,32,48}.
template <int K, int M>
__global__ __launch_bounds__(kThreads) void contract_mfma(const double *__restrict__ Tf,
                                                          const double *__restrict__ U,
                                                          int64_t ncols, int reps,
                                                          double *__restrict__ out)
{
    using S = Shape<K, M>;
    extern __shared__ double Ts[];
    for (int i = threadIdx.x; i < S::FRAG; i += kThreads) Ts[i] = Tf[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t col0 = ((int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6)) * 64;
    if (col0 + 64 > ncols) return;
    double b[4][S::KS];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int s = 0; s < S::KS; ++s)
            b[j][s] = U[(int64_t)(4 * s + lane / 16) * ncols + col0 + 16 * j + lane % 16];
    double ss[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int r = 0; r < reps; ++r) {
#pragma unroll 1
        for (int t = 0; t < S::MT; ++t) {
            dvec4 acc[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[j] = dvec4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < S::KS; ++s) {
                const double a = Ts[(t * S::KS + s) * 64 + lane];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[j][s], acc[j], 0, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) ss[j] = fma(acc[j][i], acc[j][i], ss[j]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int s = 0; s < S::KS; ++s) b[j][s] = fma(b[j][s], 0.75, 0.125);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double v = ss[j];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (lane < 16) out[col0 + 16 * j + lane] = v;
    }
}

static double lcg(uint64_t &x)
{
    x = x * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

template <int K, int M>
static int run(const char *name, int64_t ncols, int reps, int iters)
{
    using S = Shape<K, M>;
    if (ncols <= 0 || ncols % kThreads) {
        std::fprintf(stderr, "ncols must be a positive multiple of %d\n", kThreads);
        return 1;
    }
    uint64_t seed = 12345;
    std::vector<double> T((size_t)M * K), Tf(S::FRAG, 0.0), U((size_t)S::KP * ncols, 0.0);
    for (auto &t : T) t = lcg(seed);
    for (int t = 0; t < S::MT; ++t)
        for (int s = 0; s < S::KS; ++s)
            for (int l = 0; l < 64; ++l) {
                const int m = 16 * t + l % 16, k = 4 * s + l / 16;
                Tf[(t * S::KS + s) * 64 + l] = (m < M && k < K) ? T[(size_t)m * K + k] : 0.0;
            }
    for (int k = 0; k < K; ++k)
        for (int64_t c = 0; c < ncols; ++c) U[(size_t)k * ncols + c] = lcg(seed);

    double *dT, *dTf, *dU, *dv, *dm;
    CHECK(hipMalloc(&dT, T.size() * 8));
    CHECK(hipMalloc(&dTf, Tf.size() * 8));
    CHECK(hipMalloc(&dU, U.size() * 8));
    CHECK(hipMalloc(&dv, ncols * 8));
    CHECK(hipMalloc(&dm, ncols * 8));
    CHECK(hipMemcpy(dT, T.data(), T.size() * 8, hipMemcpyHostToDevice));
    CHECK(hipMemcpy(dTf, Tf.data(), Tf.size() * 8, hipMemcpyHostToDevice));
    CHECK(hipMemcpy(dU, U.data(), U.size() * 8, hipMemcpyHostToDevice));
    const size_t lds = (size_t)S::FRAG * 8;
    if (lds > 160 * 1024) {
        std::fprintf(stderr, "tabulation does not fit in LDS\n");
        return 1;
    }
    if (lds > 64 * 1024)
        CHECK(hipFuncSetAttribute((const void *)contract_mfma<K, M>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const dim3 grid((unsigned)(ncols / kThreads)), block(kThreads);
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const double flops = 2.0 * M * K * (double)ncols * reps;
    float ms[2];
    for (int v = 0; v < 2; ++v) {
        auto launch = [&]() {
            if (v == 0)
                hipLaunchKernelGGL((contract_valu<K, M>), grid, block, 0, 0, dT, dU, ncols, reps, dv);
            else
                hipLaunchKernelGGL((contract_mfma<K, M>), grid, block, lds, 0, dTf, dU, ncols, reps, dm);
        };
        for (int i = 0; i < 3; ++i) launch();
        CHECK(hipGetLastError());
        CHECK(hipDeviceSynchronize());
        CHECK(hipEventRecord(e0, 0));
        for (int i = 0; i < iters; ++i) launch();
        CHECK(hipEventRecord(e1, 0));
        CHECK(hipEventSynchronize(e1));
        CHECK(hipEventElapsedTime(&ms[v], e0, e1));
        ms[v] /= iters;
    }
    std::vector<double> hv(ncols), hm(ncols);
    CHECK(hipMemcpy(hv.data(), dv, ncols * 8, hipMemcpyDeviceToHost));
    CHECK(hipMemcpy(hm.data(), dm, ncols * 8, hipMemcpyDeviceToHost));
    double worst = 0.0;
    for (int64_t c = 0; c < ncols; ++c)
        worst = std::fmax(worst, std::fabs(hv[c] - hm[c]) / std::fmax(std::fabs(hv[c]), 1e-300));
    const char *kn[2] = {"valu", "mfma"};
    for (int v = 0; v < 2; ++v)
        std::printf("{\"case\": \"%s\", \"kernel\": \"%s\", \"K\": %d, \"M\": %d, \"ncols\": %lld, "
                    "\"reps\": %d, \"us\": %.2f, \"tflops\": %.2f, \"frac_fp64\": %.3f}\n",
                    name, kn[v], K, M, (long long)ncols, reps, ms[v] * 1e3,
                    flops / (ms[v] * 1e-3) / 1e12, flops / (ms[v] * 1e-3) / 78.6e12);
    std::printf("{\"case\": \"%s\", \"max_rel_diff\": %.3e, \"mfma_over_valu_time\": %.3f}\n",
                name, worst, ms[1] / ms[0]);
    CHECK(hipFree(dT));
    CHECK(hipFree(dTf));
    CHECK(hipFree(dU));
    CHECK(hipFree(dv));
    CHECK(hipFree(dm));
    return worst < 1e-12 ? 0 : 3;
}

int main(int argc, char **argv)
{
    const char *which = argc > 1 ? argv[1] : "p8";
    const int64_t ncols = argc > 2 ? std::atoll(argv[2]) : (int64_t)1 << 20;
    const int iters = argc > 4 ? std::atoi(argv[4]) : 20;
    if (!std::strcmp(which, "p4"))
        return run<15, 32>("p4", ncols, argc > 3 ? std::atoi(argv[3]) : 8, iters);
    if (!std::strcmp(which, "p8"))
        return run<45, 162>("p8", ncols, argc > 3 ? std::atoi(argv[3]) : 2, iters);
    std::fprintf(stderr, "usage: contraction_probe p4|p8 [ncols] [reps] [iters]\n");
    return 1;
}

// Matrix-core throughput of one MI355X (gfx950) per MFMA instruction, for the
// denominators of the roofline: every wave of a full grid (2048 workgroups of 4
// waves, 8 per SIMD) issues a register-only stream of one MFMA type into NACC
// independent accumulators; no memory traffic.  Prints TFLOP/s per instruction.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef float flt16 __attribute__((ext_vector_type(16)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));

#define CHECK(x)                                                                       \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));               \
            std::exit(1);                                                              \
        }                                                                              \
    } while (0)

// The accumulators are summed and compared with a value they never reach, so the
// compiler keeps every MFMA; the store never happens.
template <int NACC>
__global__ __launch_bounds__(256) void k_f64(int iters, double* out) {
    dbl4 acc[NACC];
    for (int j = 0; j < NACC; ++j) acc[j] = dbl4{0, 0, 0, 0};
    const double a = threadIdx.x * 1e-3, b = 1.0 - a;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int j = 0; j < NACC; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
    double s = 0;
    for (int j = 0; j < NACC; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    if (s == -1.2345e300) out[0] = s;
}

template <int NACC>
__global__ __launch_bounds__(256) void k_f32(int iters, double* out) {
    flt4 acc[NACC];
    for (int j = 0; j < NACC; ++j) acc[j] = flt4{0, 0, 0, 0};
    const float a = threadIdx.x * 1e-3f, b = 1.0f - a;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int j = 0; j < NACC; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[j], 0, 0, 0);
    float s = 0;
    for (int j = 0; j < NACC; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    if (s == -1.2345e30f) out[0] = s;
}

template <int NACC>
__global__ __launch_bounds__(256) void k_bf16_16x16x16(int iters, double* out) {
    flt4 acc[NACC];
    for (int j = 0; j < NACC; ++j) acc[j] = flt4{0, 0, 0, 0};
    const bf16x4 a = {(short)threadIdx.x, 1, 2, 3}, b = {3, 2, 1, (short)threadIdx.x};
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int j = 0; j < NACC; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[j], 0, 0, 0);
    float s = 0;
    for (int j = 0; j < NACC; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    if (s == -1.2345e30f) out[0] = s;
}

template <int NACC>
__global__ __launch_bounds__(256) void k_bf16_16x16x32(int iters, double* out) {
    flt4 acc[NACC];
    for (int j = 0; j < NACC; ++j) acc[j] = flt4{0, 0, 0, 0};
    const bf16x8 a = {(short)threadIdx.x, 1, 2, 3, 4, 5, 6, 7}, b = {7, 6, 5, 4, 3, 2, 1, (short)threadIdx.x};
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int j = 0; j < NACC; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
    float s = 0;
    for (int j = 0; j < NACC; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    if (s == -1.2345e30f) out[0] = s;
}

template <int NACC>
__global__ __launch_bounds__(256) void k_bf16_32x32x16(int iters, double* out) {
    flt16 acc[NACC];
    for (int j = 0; j < NACC; ++j)
        for (int q = 0; q < 16; ++q) acc[j][q] = 0;
    const bf16x8 a = {(short)threadIdx.x, 1, 2, 3, 4, 5, 6, 7}, b = {7, 6, 5, 4, 3, 2, 1, (short)threadIdx.x};
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int j = 0; j < NACC; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[j], 0, 0, 0);
    float s = 0;
    for (int j = 0; j < NACC; ++j)
        for (int q = 0; q < 16; ++q) s += acc[j][q];
    if (s == -1.2345e30f) out[0] = s;
}

static double tflops(void (*kern)(int, double*), double flop_per_mfma, int nacc, double* out) {
    const int grid = 256 * 8, iters = 4000;
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, 0, iters, out);  // warm-up
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e0));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, 0, iters, out);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return grid * 4.0 * iters * nacc * flop_per_mfma / (ms * 1e-3) / 1e12;
}

int main() {
    double* out = nullptr;
    CHECK(hipMalloc(&out, 64));
    struct Row {
        const char* name;
        void (*k)(int, double*);
        double flop;
        int nacc;
    } rows[] = {
        {"v_mfma_f64_16x16x4_f64, 4 accumulators", k_f64<4>, 2.0 * 16 * 16 * 4, 4},
        {"v_mfma_f64_16x16x4_f64, 8 accumulators", k_f64<8>, 2.0 * 16 * 16 * 4, 8},
        {"v_mfma_f32_16x16x4_f32, 4 accumulators", k_f32<4>, 2.0 * 16 * 16 * 4, 4},
        {"v_mfma_f32_16x16x4_f32, 8 accumulators", k_f32<8>, 2.0 * 16 * 16 * 4, 8},
        {"v_mfma_f32_16x16x16_bf16, 4 accumulators", k_bf16_16x16x16<4>, 2.0 * 16 * 16 * 16, 4},
        {"v_mfma_f32_16x16x32_bf16, 4 accumulators", k_bf16_16x16x32<4>, 2.0 * 16 * 16 * 32, 4},
        {"v_mfma_f32_32x32x16_bf16, 4 accumulators", k_bf16_32x32x16<4>, 2.0 * 32 * 32 * 16, 4},
    };
    for (const Row& r : rows) std::printf("%-44s %8.1f TFLOP/s\n", r.name, tflops(r.k, r.flop, r.nacc, out));
    CHECK(hipFree(out));
    return 0;
}

// Throughput probes of one MI355X: the ceilings the library's rooflines are
// quoted against beside the datasheet figures.  Each kernel keeps independent
// dependency chains per lane so that issue, not latency, bounds it, and writes
// one value per lane at the end so that the compiler keeps the work.
//   fp64 FMA on the vector units   8 chains of v_fma_f64 per lane
//   fp64 matrix cores              4 accumulators of v_mfma_f64_16x16x4f64
//   fp32 matrix cores              4 accumulators of v_mfma_f32_16x16x4f32
//   int8 matrix cores              4 accumulators of v_mfma_i32_16x16x64_i8
//   HBM read                       each lane sums a strided slice of a buffer
// Built as libgsvd_peaks.so (paper_2603_11953_amd/build.py); driven by
// paper_2603_11953_amd/peaks.py.  Not part of the thin-SVD library.
#include <hip/hip_runtime.h>

#include <stdint.h>

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef long i64x1;

__global__ void __launch_bounds__(256) probe_fma64_kernel(int iters, double seed, double *out) {
    double a[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) a[c] = seed + threadIdx.x * 1e-9 + c;
    const double x = 0.999999, y = 1e-7;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < 8; ++c) a[c] = __builtin_fma(a[c], x, y);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += a[c];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) probe_mfma64_kernel(int iters, double seed, double *out) {
    f64x4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = f64x4{0.0, 0.0, 0.0, 0.0};
    const double a = seed + threadIdx.x * 1e-9, b = 1.0 - seed;
    // 8 steps per trip so that the compiler's register moves at the loop edge are amortised
    for (int i = 0; i < iters; i += 8) {
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) probe_mfma32_kernel(int iters, float seed, double *out) {
    f32x4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    const float a = seed + threadIdx.x * 1e-6f, b = 1.0f - seed;
    // 8 steps per trip so that the compiler's register moves at the loop edge are amortised
    for (int i = 0; i < iters; i += 8) {
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 4; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) probe_mfma_i8_kernel(int iters, int seed, double *out) {
    i32x4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = i32x4{0, 0, 0, 0};
    const i32x4 a = i32x4{seed + (int)threadIdx.x, seed, 1, 2};
    const i32x4 b = i32x4{3, seed ^ 5, 7, (int)threadIdx.x};
    // 8 steps per trip so that the compiler's register moves at the loop edge are amortised
    for (int i = 0; i < iters; i += 8) {
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc[c], 0, 0, 0);
    }
    int s = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[blockIdx.x * 256 + threadIdx.x] = (double)s;
}

// n doubles read once: lane t of the grid reads elements t, t + T, t + 2 T, ... (coalesced)
__global__ void __launch_bounds__(256) probe_read_kernel(const double *__restrict__ p, int64_t n,
                                                         double *out) {
    const int64_t T = (int64_t)gridDim.x * 256;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * T < n; i += 4 * T) {
        s0 += p[i];
        s1 += p[i + T];
        s2 += p[i + 2 * T];
        s3 += p[i + 3 * T];
    }
    for (; i < n; i += T) s0 += p[i];
    out[blockIdx.x * 256 + threadIdx.x] = (s0 + s1) + (s2 + s3);
}

extern "C" {

// kind: 0 fp64 FMA, 1 fp64 MFMA, 2 fp32 MFMA, 3 int8 MFMA; out holds blocks * 256 doubles
int probe_compute(int kind, int blocks, int iters, double *out, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    switch (kind) {
        case 0: hipLaunchKernelGGL(probe_fma64_kernel, dim3(blocks), dim3(256), 0, st, iters, 0.5, out); break;
        case 1: hipLaunchKernelGGL(probe_mfma64_kernel, dim3(blocks), dim3(256), 0, st, iters, 0.5, out); break;
        case 2: hipLaunchKernelGGL(probe_mfma32_kernel, dim3(blocks), dim3(256), 0, st, iters, 0.5f, out); break;
        case 3: hipLaunchKernelGGL(probe_mfma_i8_kernel, dim3(blocks), dim3(256), 0, st, iters, 3, out); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -100;
}

int probe_read(const double *p, int64_t n, int blocks, double *out, void *stream) {
    hipLaunchKernelGGL(probe_read_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, p, n, out);
    return hipGetLastError() == hipSuccess ? 0 : -100;
}

}  // extern "C"

// U = A W for FP32 working (Alg. 1 step 6, eq. (AV-0)) on the BF16 matrix cores,
// by exact operand splitting.
//
// Every FP32 entry x of A and of W is cut into three BF16 pieces,
//     x = p1 + p2 + p3,
// p1 the top 8 significant bits of x (truncation), p2 the top 8 of x - p1, p3 the
// rest (at most 8 significant bits): every difference is exact in FP32 and every
// piece exact in BF16.  A product of two pieces has at most 16 significant bits
// and is exact in the FP32 accumulation of v_mfma_f32_16x16x32_bf16, which adds
// the products of a 32-deep chunk and rounds once per chunk into the FP32
// accumulator.  The six piece products with i + j <= 4 are kept, smallest first
// (i + j = 4, then 3, then the leading 2); the dropped three are below
// 2^-24 |a| |w| each, the size of one FP32 rounding.  So the error is of the
// order of an FP32 GEMM's, n u_32 |A| |W| (eq. (AV-0) with eps_U = O(u)), at a
// third of the matrix-core time of the FP32 instruction at this shape: the
// kernel is bound by reading A and writing U.
//
// Layout (strip form, as the FP32 kernel): a wavefront owns 16 rows of U and all
// n <= 16 NT columns, and computes U^T = W^T A^T tile by tile:
//   A operand (i = l % 16, k = 8 (l / 16) + e): piece of W(kc + k, 16 t + i), from LDS
//       (pieces stored column by column, k contiguous: one 16-byte read per lane)
//   B operand (k = 8 (l / 16) + e, j = l % 16): piece of A(r0 + j, kc + k), from
//       registers (eight loads per lane per 32-column chunk, the next chunk's issued
//       while this one multiplies)
//   result register r of lane l: U(r0 + l % 16, 16 t + 4 (l / 16) + r).
#include <hip/hip_runtime.h>

#include "gsvd_internal.hpp"

namespace gsvd {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int UB_THREADS = 1024;  // 16 wavefronts, one strip each at a time
constexpr int UB_KC = 32;         // k-depth of one matrix-core step

__device__ __forceinline__ __bf16 bf16_of_top(float x) {
    return __builtin_bit_cast(__bf16, (unsigned short)(__float_as_uint(x) >> 16));
}

// x = p1 + p2 + p3 exactly (see above); each piece's FP32 pattern has zero low bits
__device__ __forceinline__ void split3(float x, __bf16 &p1, __bf16 &p2, __bf16 &p3) {
    const float h1 = __uint_as_float(__float_as_uint(x) & 0xffff0000u);
    const float r1 = x - h1;
    const float h2 = __uint_as_float(__float_as_uint(r1) & 0xffff0000u);
    const float r2 = r1 - h2;
    p1 = bf16_of_top(h1);
    p2 = bf16_of_top(h2);
    p3 = bf16_of_top(r2);
}

// padded k extent of W's pieces in LDS: n rounded up to the chunk, plus 8 (16 bytes)
template <int NT>
__host__ __device__ constexpr int ub_ldk() {
    return ((16 * NT + UB_KC - 1) / UB_KC) * UB_KC + 8;
}

template <int NT>
__global__ void __launch_bounds__(UB_THREADS)
urecover_bf16_kernel(const float *__restrict__ A, int64_t lda, const float *__restrict__ W,
                     int64_t ldw, float *__restrict__ U, int64_t ldu, int64_t m, int n) {
    constexpr int NTC = 16 * NT;
    constexpr int LDK = ub_ldk<NT>();
    extern __shared__ __attribute__((aligned(16))) unsigned char ub_smem[];
    __bf16 *Wp = reinterpret_cast<__bf16 *>(ub_smem);  // [3][NTC][LDK]
    const int kp = ((n + UB_KC - 1) / UB_KC) * UB_KC;  // k extent used (zeros beyond n)
    for (int q = threadIdx.x; q < NTC * kp; q += UB_THREADS) {
        const int c = q / kp, k = q % kp;
        const float x = (k < n && c < n) ? W[k + (int64_t)c * ldw] : 0.0f;
        __bf16 p1, p2, p3;
        split3(x, p1, p2, p3);
        Wp[(0 * NTC + c) * LDK + k] = p1;
        Wp[(1 * NTC + c) * LDK + k] = p2;
        Wp[(2 * NTC + c) * LDK + k] = p3;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t nstrips = (m + 15) / 16;
    const int nch = kp / UB_KC;
    const int64_t stride = (int64_t)gridDim.x * (UB_THREADS / 64);

    // chunk ch of a strip: A(r0 + li, 32 ch + 8 lk + e), e = 0..7
    float a[8], b[8];
    auto load = [&](float (&dst)[8], int64_t strip, int ch) {
        const int64_t row = strip * 16 + li;
        const bool rv = row < m;
        const int k0 = UB_KC * ch + 8 * lk;
        const float *p = A + row + (int64_t)k0 * lda;
#pragma unroll
        for (int e = 0; e < 8; ++e) dst[e] = (rv && k0 + e < n) ? p[(int64_t)e * lda] : 0.0f;
    };
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    int64_t strip = (int64_t)blockIdx.x * (UB_THREADS / 64) + wave;
    int ch = 0;
    if (strip < nstrips) load(a, strip, 0);
    while (strip < nstrips) {
        int nxt_ch = ch + 1;
        int64_t nxt = strip;
        if (nxt_ch == nch) {
            nxt_ch = 0;
            nxt = strip + stride;
        }
        if (nxt < nstrips) load(b, nxt, nxt_ch);
        bf16x8 a1, a2, a3;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            __bf16 p1, p2, p3;
            split3(a[e], p1, p2, p3);
            a1[e] = p1;
            a2[e] = p2;
            a3[e] = p3;
        }
        const int koff = UB_KC * ch + 8 * lk;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = 16 * t + li;
            const bf16x8 w1 = *reinterpret_cast<const bf16x8 *>(Wp + (0 * NTC + c) * LDK + koff);
            const bf16x8 w2 = *reinterpret_cast<const bf16x8 *>(Wp + (1 * NTC + c) * LDK + koff);
            const bf16x8 w3 = *reinterpret_cast<const bf16x8 *>(Wp + (2 * NTC + c) * LDK + koff);
            f32x4 s = acc[t];
            s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3, a1, s, 0, 0, 0);  // i + j = 4
            s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2, a2, s, 0, 0, 0);
            s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, a3, s, 0, 0, 0);
            s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2, a1, s, 0, 0, 0);  // i + j = 3
            s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, a2, s, 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, a1, s, 0, 0, 0);  // leading
        }
        if (nxt_ch == 0) {
            const int64_t row = strip * 16 + li;
            if (row < m) {
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int c = 16 * t + 4 * lk + r;
                        if (c < n) U[row + (int64_t)c * ldu] = acc[t][r];
                    }
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) a[e] = b[e];
        strip = nxt;
        ch = nxt_ch;
    }
}

template <int NT>
hipError_t launch_bf16(int64_t m, int64_t n, const float *A, int64_t lda, const float *W,
                       int64_t ldw, float *U, int64_t ldu, hipStream_t st) {
    const size_t lds = (size_t)3 * (16 * NT) * ub_ldk<NT>() * sizeof(__bf16);
    const int64_t nstrips = (m + 15) / 16;
    const int waves = UB_THREADS / 64;
    // one workgroup per CU when the pieces take most of LDS, else two
    int64_t grid = 256 * (lds > 80 * 1024 ? 1 : 2);
    const int64_t need = (nstrips + waves - 1) / waves;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    auto k = urecover_bf16_kernel<NT>;
    hipError_t err = hipFuncSetAttribute((const void *)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(UB_THREADS), lds, st, A, lda, W, ldw, U, ldu,
                       m, (int)n);
    return hipGetLastError();
}

}  // namespace

hipError_t urecover_bf16_launch(int64_t m, int64_t n, const float *A, int64_t lda, const float *W,
                                int64_t ldw, float *U, int64_t ldu, hipStream_t st) {
    switch ((n + 15) / 16) {
        case 1: return launch_bf16<1>(m, n, A, lda, W, ldw, U, ldu, st);
        case 2: return launch_bf16<2>(m, n, A, lda, W, ldw, U, ldu, st);
        case 3: return launch_bf16<3>(m, n, A, lda, W, ldw, U, ldu, st);
        case 4: return launch_bf16<4>(m, n, A, lda, W, ldw, U, ldu, st);
        case 5: return launch_bf16<5>(m, n, A, lda, W, ldw, U, ldu, st);
        case 6: return launch_bf16<6>(m, n, A, lda, W, ldw, U, ldu, st);
        case 7: return launch_bf16<7>(m, n, A, lda, W, ldw, U, ldu, st);
        case 8: return launch_bf16<8>(m, n, A, lda, W, ldw, U, ldu, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gsvd

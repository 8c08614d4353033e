// U = A W for n > 128 (Alg. 1 step 6, eq. (AV-0)), working precision, on the
// matrix cores.
//
// A workgroup of 16 wavefronts owns 256 rows of U (one 16-row strip per
// wavefront) and one group of 128 columns.  The k range 0 .. n is walked in
// chunks of 16: the chunk's 16 x 128 block of W is staged in LDS (two buffers; the
// next chunk's loads are issued into registers before the current chunk's products
// and stored to the other buffer after them, so no wave waits on them), and each
// wavefront loads its 16 x 16 slice of A straight into MFMA operand registers (one
// load instruction reads 16 consecutive rows of 4 columns, the next chunk's issued
// a chunk ahead) and runs 4 k-steps against the 8 column tiles:
//   A operand (i = l % 16, k = l / 16): W(k0 + 4 s + k, 16 t + i)   from LDS
//   B operand (k = l / 16, j = l % 16): A(r0 + j, k0 + 4 s + k)     registers
// computing U^T = W^T A^T, so result register r of lane l is
// U(r0 + l % 16, 16 t + c(r, l / 16)) and each store writes 16 consecutive rows.
// Workgroup ids are dealt so that the column groups of one row block share an
// XCD (ids g, g + 8, g + 16, ...), whose L2 then serves the repeated reads of A.
#include <hip/hip_runtime.h>

#include "gsvd_internal.hpp"

namespace gsvd {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct WMfma;

template <>
struct WMfma<double> {
    typedef f64x4 acc_t;
    __device__ static __forceinline__ acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // column (within the 16-column tile) of result register r, lane group lk
    __device__ static __forceinline__ int col(int lk, int r) { return 4 * r + lk; }
};

template <>
struct WMfma<float> {
    typedef f32x4 acc_t;
    __device__ static __forceinline__ acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int col(int lk, int r) { return 4 * lk + r; }
};

constexpr int UW_WAVES = 16;
constexpr int UW_THREADS = 64 * UW_WAVES;
constexpr int UW_ROWS = 16 * UW_WAVES;  // rows per workgroup
constexpr int UW_NT = 8;                // 16-column tiles per group
constexpr int UW_COLS = 16 * UW_NT;     // columns per group
constexpr int UW_KC = 16;               // k per chunk
constexpr int UW_KS = UW_KC / 4;        // k-steps (MFMA depth 4) per chunk
constexpr int UW_LDW = UW_COLS + 16;    // LDS row stride: the 4 rows of one read in distinct banks
constexpr int UW_XCD = 8;

template <typename T>
__global__ void __launch_bounds__(UW_THREADS)
urecover_wide_kernel(const T *__restrict__ A, int64_t lda, const T *__restrict__ W, int64_t ldw,
                     T *__restrict__ U, int64_t ldu, int64_t m, int n, int ngrp, int64_t nrb) {
    typedef typename WMfma<T>::acc_t acc_t;
    extern __shared__ __attribute__((aligned(16))) unsigned char uw_smem[];
    T *Wbuf = reinterpret_cast<T *>(uw_smem);  // two chunks of UW_KC x UW_LDW
    // XCD-aware ids: id = x + 8 (grp + ngrp y), row block 8 y + x
    const int64_t id = blockIdx.x;
    const int64_t x = id % UW_XCD, rest = id / UW_XCD;
    const int grp = (int)(rest % ngrp);
    const int64_t rb = UW_XCD * (rest / ngrp) + x;
    if (rb >= nrb) return;  // whole workgroup: no barrier is reached
    const int c0 = UW_COLS * grp;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t row = rb * UW_ROWS + 16 * wave + li;
    const bool rv = row < m;
    const int nkc = (n + UW_KC - 1) / UW_KC;

    // the W chunk passes through registers: its loads are issued a chunk ahead and
    // land in LDS after the chunk's products, so no wave waits for them
    constexpr int WPL = UW_KC * UW_COLS / UW_THREADS;  // W values per lane
    T wr[WPL];
    auto loadw = [&](int kc) {
#pragma unroll
        for (int e = 0; e < WPL; ++e) {
            const int q = threadIdx.x + e * UW_THREADS;
            const int k = q / UW_COLS, j = q % UW_COLS;
            const int kk = UW_KC * kc + k, jj = c0 + j;
            wr[e] = (kk < n && jj < n) ? W[kk + (int64_t)jj * ldw] : (T)0;
        }
    };
    auto storew = [&](T *dst) {
#pragma unroll
        for (int e = 0; e < WPL; ++e) {
            const int q = threadIdx.x + e * UW_THREADS;
            dst[(q / UW_COLS) * UW_LDW + q % UW_COLS] = wr[e];
        }
    };
    // A(row, UW_KC kc + 4 s + lk), s < UW_KS
    T a[UW_KS], b[UW_KS];
    auto load = [&](T *dst, int kc) {
        const T *p = A + row + (int64_t)(UW_KC * kc + lk) * lda;
#pragma unroll
        for (int s = 0; s < UW_KS; ++s) {
            const int k = UW_KC * kc + 4 * s + lk;
            dst[s] = (rv && k < n) ? p[(int64_t)(4 * s) * lda] : (T)0;
        }
    };

    acc_t acc[UW_NT];
#pragma unroll
    for (int t = 0; t < UW_NT; ++t) acc[t] = acc_t{0, 0, 0, 0};

    loadw(0);
    load(a, 0);
    storew(Wbuf);
    __syncthreads();
    for (int kc = 0; kc < nkc; ++kc) {
        const bool more = kc + 1 < nkc;
        if (more) {
            loadw(kc + 1);
            load(b, kc + 1);
        }
        const T *w = Wbuf + (kc & 1) * UW_KC * UW_LDW + lk * UW_LDW + li;
#pragma unroll
        for (int s = 0; s < UW_KS; ++s)
#pragma unroll
            for (int t = 0; t < UW_NT; ++t)
                acc[t] = WMfma<T>::step(w[4 * s * UW_LDW + 16 * t], a[s], acc[t]);
        if (more) storew(Wbuf + ((kc + 1) & 1) * UW_KC * UW_LDW);
#pragma unroll
        for (int s = 0; s < UW_KS; ++s) a[s] = b[s];
        __syncthreads();
    }
    if (rv) {
#pragma unroll
        for (int t = 0; t < UW_NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = c0 + 16 * t + WMfma<T>::col(lk, r);
                if (c < n) U[row + (int64_t)c * ldu] = acc[t][r];
            }
    }
}

template <typename T>
hipError_t launch_wide(int64_t m, int64_t n, const T *A, int64_t lda, const T *W, int64_t ldw,
                       T *U, int64_t ldu, hipStream_t st) {
    const int ngrp = (int)((n + UW_COLS - 1) / UW_COLS);
    const int64_t nrb = (m + UW_ROWS - 1) / UW_ROWS;
    const int64_t ny = (nrb + UW_XCD - 1) / UW_XCD;
    const int64_t grid = ny * ngrp * UW_XCD;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    const size_t lds = (size_t)2 * UW_KC * UW_LDW * sizeof(T);
    auto k = urecover_wide_kernel<T>;
    hipError_t err = hipFuncSetAttribute((const void *)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(UW_THREADS), lds, st, A, lda, W, ldw, U, ldu,
                       m, (int)n, ngrp, nrb);
    return hipGetLastError();
}

}  // namespace

hipError_t urecover_wide_launch(int working, int64_t m, int64_t n, const void *A, int64_t lda,
                                const void *W, int64_t ldw, void *U, int64_t ldu, hipStream_t st) {
    if (m < 1 || n < 1 || n > GSVD_WIDE_MAX_N) return hipErrorInvalidValue;
    if (working == 1)
        return launch_wide<double>(m, n, (const double *)A, lda, (const double *)W, ldw,
                                   (double *)U, ldu, st);
    return launch_wide<float>(m, n, (const float *)A, lda, (const float *)W, ldw, (float *)U, ldu,
                              st);
}

}  // namespace gsvd

// U = A W in the working precision (Alg. 1 step 6, eq. (AV-0)), W = fl(V Sigma^-1).
//
// A tall GEMM on the matrix cores.  A wavefront owns a strip of 16 rows of U
// and all n columns (n <= 16 NT): it loads its 16 x n slice of A once (each
// load instruction reads 16 consecutive rows of 4 columns, i.e. four full
// 128-byte lines), then runs n/4 x NT MFMA steps
//   FP64: v_mfma_f64_16x16x4_f64   FP32: v_mfma_f32_16x16x4_f32
// with W staged in LDS (zero padded to a multiple of 4 rows and 16 columns).
// MFMA operand layout (16x16x4): A-operand lane l holds A(l % 16, l / 16);
// B-operand lane l holds B(l / 16, l % 16).  Result: lane l, register r holds
// D(4 (l / 16) + r, l % 16) for the FP32 instruction (four consecutive rows of
// one column) and D(4 r + l / 16, l % 16) for the FP64 one (rows strided by 4).
// Workgroups stride over groups of 4 strips, so W is staged once per
// workgroup rather than once per 64 rows.
#include <hip/hip_runtime.h>

#include "gsvd_internal.hpp"

namespace gsvd {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
    typedef f64x4 acc_t;
    __device__ static __forceinline__ acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // row (within the 16-row tile) of result register r in a lane with l / 16 == lk
    __device__ static __forceinline__ int row(int lk, int r) { return 4 * r + lk; }
};

template <>
struct Mfma<float> {
    typedef f32x4 acc_t;
    __device__ static __forceinline__ acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

// Strip form: a wavefront owns 16 rows of U and all n columns.  It loads its
// 16 x n slice of A straight into MFMA operand registers (one load instruction
// reads 16 consecutive rows of 4 columns: four full 128-byte lines) while the
// previous strip is multiplied, and computes U^T = W^T A^T tile by tile:
//   A operand (i = l % 16, k = l / 16): W(4 s + k, 16 t + i)   from LDS
//   B operand (k = l / 16, j = l % 16): A(r0 + j, 4 s + k)     from registers
// so that result register r of lane l is U(r0 + l % 16, 16 t + c(r, l / 16)):
// each store instruction writes 16 consecutive rows of 4 columns.
template <typename T>
struct MfmaT;

template <>
struct MfmaT<double> {
    // column (within the 16-column tile) of result register r, lane group lk
    __device__ static __forceinline__ int col(int lk, int r) { return 4 * r + lk; }
};

template <>
struct MfmaT<float> {
    __device__ static __forceinline__ int col(int lk, int r) { return 4 * lk + r; }
};

constexpr int US_THREADS = 512;

// Row stride of W in LDS (elements).  One operand read touches 4 rows (lk) of
// 16 consecutive entries; the stride puts those rows in distinct bank groups
// (16 mod 32 doubles, 16 or 48 mod 64 floats) for every tile count.
template <typename T, int NT>
__host__ __device__ constexpr int strip_ldw() {
    return NT * 16 + (NT % 2 == 0 ? 16 : 0);
}

template <typename T, int NT>
__device__ __forceinline__ void urecover_strip_body(const T *__restrict__ A, int64_t lda,
                                                    const T *__restrict__ W, int64_t ldw,
                                                    T *__restrict__ U, int64_t ldu, int64_t m,
                                                    int n, int64_t strip0, int64_t stride,
                                                    T *Ws) {
    typedef typename Mfma<T>::acc_t acc_t;
    constexpr int NTC = NT * 16;
    constexpr int LDW = strip_ldw<T, NT>();
    for (int q = threadIdx.x; q < NTC * NTC; q += blockDim.x) {
        const int k = q / NTC, j = q % NTC;
        Ws[k * LDW + j] = (k < n && j < n) ? W[k + (int64_t)j * ldw] : (T)0;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t nstrips = (m + 15) / 16;
    const int nch = (n + 15) / 16;  // chunks of 16 columns of A (4 k-steps) per strip

    // chunk ch of a strip: A(r0 + li, 16 ch + 4 s + lk), s = 0..3
    T a[4], b[4];
    auto load = [&](T *dst, int64_t strip, int ch) {
        const int64_t row = strip * 16 + li;
        const bool rv = row < m;
        const T *p = A + row + (int64_t)(16 * ch + lk) * lda;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = 16 * ch + 4 * s + lk;
            dst[s] = (rv && k < n) ? p[(int64_t)(4 * s) * lda] : (T)0;
        }
    };
    acc_t acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = acc_t{0, 0, 0, 0};

    int64_t strip = strip0;
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
        // 4 k-steps against every 16-column tile of W: NT independent chains
        const T *w = Ws + (16 * ch + lk) * LDW + li;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int t = 0; t < NT; ++t)
                acc[t] = Mfma<T>::step(w[4 * s * LDW + 16 * t], a[s], acc[t]);
        if (nxt_ch == 0) {
            const int64_t row = strip * 16 + li;
            if (row < m) {
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int c = 16 * t + MfmaT<T>::col(lk, r);
                        if (c < n) U[row + (int64_t)c * ldu] = acc[t][r];
                    }
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = acc_t{0, 0, 0, 0};
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) a[s] = b[s];
        strip = nxt;
        ch = nxt_ch;
    }
}

template <typename T, int NT>
__global__ void __launch_bounds__(US_THREADS)
urecover_strip_kernel(const T *__restrict__ A, int64_t lda, const T *__restrict__ W, int64_t ldw,
                      T *__restrict__ U, int64_t ldu, int64_t m, int n) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int waves = US_THREADS / 64;
    urecover_strip_body<T, NT>(A, lda, W, ldw, U, ldu, m, n,
                               (int64_t)blockIdx.x * waves + (threadIdx.x >> 6),
                               (int64_t)gridDim.x * waves, reinterpret_cast<T *>(smem_raw));
}

// Batched: blockIdx.z picks the problem order[first + z]; its strips are dealt
// to the gridDim.x workgroups of that problem.
template <typename T, int NT>
__global__ void __launch_bounds__(US_THREADS)
urecover_strip_batched_kernel(const BatchMat *__restrict__ tab, const int *__restrict__ order,
                              int first) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const BatchMat &d = tab[order[first + blockIdx.z]];
    const int waves = US_THREADS / 64;
    if ((int64_t)blockIdx.x * waves * 16 >= d.m) return;
    urecover_strip_body<T, NT>(reinterpret_cast<const T *>(d.A), d.lda,
                               reinterpret_cast<const T *>(d.W), d.n, reinterpret_cast<T *>(d.U),
                               d.ldu, d.m, d.n, (int64_t)blockIdx.x * waves + (threadIdx.x >> 6),
                               (int64_t)gridDim.x * waves, reinterpret_cast<T *>(smem_raw));
}

template <typename T, int NT>
static size_t strip_lds() {
    return (size_t)(NT * 16) * strip_ldw<T, NT>() * sizeof(T);
}

// workgroups that fit one compute unit by LDS, at most 2 (16 wavefronts)
template <typename T, int NT>
static int strip_per_cu() {
    const size_t l = strip_lds<T, NT>();
    int k = (int)((160 * 1024) / (l + 1024));
    return k < 1 ? 1 : (k > 2 ? 2 : k);
}

template <typename T, int NT>
static hipError_t launch_strip(int64_t m, int64_t n, const T *A, int64_t lda, const T *W,
                               int64_t ldw, T *U, int64_t ldu, hipStream_t st) {
    const int64_t nstrips = (m + 15) / 16;
    const int waves = US_THREADS / 64;
    int64_t grid = 256 * (int64_t)strip_per_cu<T, NT>();
    const int64_t need = (nstrips + waves - 1) / waves;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    const size_t lds = strip_lds<T, NT>();
    auto k = urecover_strip_kernel<T, NT>;
    hipError_t err = hipFuncSetAttribute((const void *)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(US_THREADS), lds, st, A, lda, W, ldw, U, ldu,
                       m, (int)n);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_t(int64_t m, int64_t n, const T *A, int64_t lda, const T *W, int64_t ldw,
                           T *U, int64_t ldu, hipStream_t st) {
    switch ((n + 15) / 16) {
        case 1: return launch_strip<T, 1>(m, n, A, lda, W, ldw, U, ldu, st);
        case 2: return launch_strip<T, 2>(m, n, A, lda, W, ldw, U, ldu, st);
        case 3: return launch_strip<T, 3>(m, n, A, lda, W, ldw, U, ldu, st);
        case 4: return launch_strip<T, 4>(m, n, A, lda, W, ldw, U, ldu, st);
        case 5: return launch_strip<T, 5>(m, n, A, lda, W, ldw, U, ldu, st);
        case 6: return launch_strip<T, 6>(m, n, A, lda, W, ldw, U, ldu, st);
        case 7: return launch_strip<T, 7>(m, n, A, lda, W, ldw, U, ldu, st);
        case 8: return launch_strip<T, 8>(m, n, A, lda, W, ldw, U, ldu, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t urecover_launch(int working, int64_t m, int64_t n, const void *A, int64_t lda,
                           const void *W, int64_t ldw, void *U, int64_t ldu, hipStream_t st) {
    if (working == 1)
        return launch_t<double>(m, n, (const double *)A, lda, (const double *)W, ldw, (double *)U,
                                ldu, st);
    return launch_t<float>(m, n, (const float *)A, lda, (const float *)W, ldw, (float *)U, ldu, st);
}

int urecover_batched_max_nt(int working) { (void)working; return 8; }

template <typename T, int NT>
static hipError_t batched_strip(const BatchMat *tab, const int *order, int first, int count,
                                int64_t max_m, hipStream_t st) {
    const size_t lds = strip_lds<T, NT>();
    // about eight strips per wavefront for the tallest problem of the group
    const int64_t strips = (max_m + 15) / 16;
    const int waves = US_THREADS / 64;
    int64_t gx = (strips + waves * 8 - 1) / (waves * 8);
    if (gx < 1) gx = 1;
    if (gx > 65535) gx = 65535;
    auto k = urecover_strip_batched_kernel<T, NT>;
    hipError_t err = hipFuncSetAttribute((const void *)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3((unsigned)gx, 1, (unsigned)count), dim3(US_THREADS), lds, st, tab,
                       order, first);
    return hipGetLastError();
}

template <typename T>
static hipError_t batched_t(const BatchMat *tab, const int *order, int first, int count, int nt,
                            int64_t max_m, hipStream_t st) {
    switch (nt) {
        case 1: return batched_strip<T, 1>(tab, order, first, count, max_m, st);
        case 2: return batched_strip<T, 2>(tab, order, first, count, max_m, st);
        case 3: return batched_strip<T, 3>(tab, order, first, count, max_m, st);
        case 4: return batched_strip<T, 4>(tab, order, first, count, max_m, st);
        case 5: return batched_strip<T, 5>(tab, order, first, count, max_m, st);
        case 6: return batched_strip<T, 6>(tab, order, first, count, max_m, st);
        case 7: return batched_strip<T, 7>(tab, order, first, count, max_m, st);
        case 8: return batched_strip<T, 8>(tab, order, first, count, max_m, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t urecover_batched_launch(int working, const BatchMat *tab, const int *order, int first,
                                   int count, int nt, int64_t max_m, hipStream_t st) {
    if (count < 1 || count > 65535 || nt < 1 || nt > urecover_batched_max_nt(working))
        return hipErrorInvalidValue;
    if (working == 1) return batched_t<double>(tab, order, first, count, nt, max_m, st);
    return batched_t<float>(tab, order, first, count, nt, max_m, st);
}

}  // namespace gsvd

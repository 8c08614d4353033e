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

template <typename T, int NT>
__global__ void __launch_bounds__(256)
urecover_kernel(const T *__restrict__ A, int64_t lda, const T *__restrict__ W, int64_t ldw,
                T *__restrict__ U, int64_t ldu, int64_t m, int n, int64_t ngroups) {
    typedef typename Mfma<T>::acc_t acc_t;
    constexpr int NTC = NT * 16;
    constexpr int KS = NTC / 4;  // k-steps of 4 (n <= NTC)
    extern __shared__ unsigned char smem_raw[];
    T *Ws = reinterpret_cast<T *>(smem_raw);  // [NTC rows k][NTC cols j], row-major

    for (int q = threadIdx.x; q < NTC * NTC; q += blockDim.x) {
        const int k = q / NTC, j = q % NTC;
        Ws[q] = (k < n && j < n) ? W[k + (int64_t)j * ldw] : (T)0;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int ksteps = (n + 3) / 4;

    for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const int64_t r0 = (g * 4 + wave) * 16;
        if (r0 >= m) continue;
        const int64_t row = r0 + li;
        const bool rv = row < m;
        T a[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int k = 4 * s + lk;
            a[s] = (s < ksteps && rv && k < n) ? A[row + (int64_t)k * lda] : (T)0;
        }
        acc_t acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (s < ksteps) {
                const T *wrow = Ws + (4 * s + lk) * NTC + li;
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t] = Mfma<T>::step(a[s], wrow[t * 16], acc[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int col = t * 16 + li;
            if (col < n) {
                T *dst = U + r0 + (int64_t)col * ldu;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rr = Mfma<T>::row(lk, r);
                    if (r0 + rr < m) dst[rr] = acc[t][r];
                }
            }
        }
    }
}

// Tiled variant: a workgroup (4 wavefronts) walks over 64-row tiles of A.  The
// tile is staged in LDS (column-major, padded) by coalesced loads, the next
// tile is fetched into registers while the current one is multiplied, and W
// sits in LDS for the workgroup's lifetime.  The 4 x NT result tiles (16 x 16)
// of a row tile are dealt round-robin to the wavefronts; each MFMA takes its
// A and B operands from LDS.
constexpr int UT_BM = 64;       // rows per tile
constexpr int UT_THREADS = 256;

// Row tiles tile0, tile0 + stride, ... of one product U = A W.
template <typename T, int NT>
__device__ __forceinline__ void urecover_tile_body(const T *__restrict__ A, int64_t lda,
                                                   const T *__restrict__ W, int64_t ldw,
                                                   T *__restrict__ U, int64_t ldu, int64_t m,
                                                   int n, int64_t ntiles, int64_t tile0,
                                                   int64_t stride) {
    typedef typename Mfma<T>::acc_t acc_t;
    constexpr int NTC = NT * 16;
    constexpr int LDA_S = UT_BM + 2;          // padded column stride of the A tile
    constexpr int LDW_S = NTC + 2;            // padded row stride of W
    constexpr int PER = UT_BM * NTC / UT_THREADS;  // staged tile values per lane
    extern __shared__ unsigned char smem_raw[];
    T *Ws = reinterpret_cast<T *>(smem_raw);  // [NTC rows k][LDW_S], row-major
    T *As = Ws + NTC * LDW_S;                 // [NTC cols][LDA_S], column-major

    for (int q = threadIdx.x; q < NTC * NTC; q += UT_THREADS) {
        const int k = q / NTC, j = q % NTC;
        Ws[k * LDW_S + j] = (k < n && j < n) ? W[k + (int64_t)j * ldw] : (T)0;
    }

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int ksteps = (n + 3) / 4;

    T stage[PER];
    auto fetch = [&](int64_t tile) {
        const int64_t r0 = tile * UT_BM;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * UT_THREADS;
            const int row = e % UT_BM, col = e / UT_BM;
            const int64_t r = r0 + row;
            stage[q] = (r < m && col < n) ? A[r + (int64_t)col * lda] : (T)0;
        }
    };

    int64_t tile = tile0;
    if (tile < ntiles) fetch(tile);
    for (; tile < ntiles; tile += stride) {
        __syncthreads();  // previous tile fully consumed (and W staged, first time)
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * UT_THREADS;
            As[(e / UT_BM) * LDA_S + (e % UT_BM)] = stage[q];
        }
        __syncthreads();
        const int64_t next = tile + stride;
        if (next < ntiles) fetch(next);
        const int64_t r0 = tile * UT_BM;
        for (int item = wave; item < 4 * NT; item += 4) {
            const int rb = item / NT, ct = item % NT;
            acc_t acc = acc_t{0, 0, 0, 0};
            const T *ap = As + rb * 16 + li;
            const T *bp = Ws + ct * 16 + li;
            for (int s = 0; s < ksteps; ++s) {
                const int k = 4 * s + lk;
                acc = Mfma<T>::step(ap[k * LDA_S], bp[k * LDW_S], acc);
            }
            const int col = ct * 16 + li;
            if (col < n) {
                T *dst = U + r0 + rb * 16 + (int64_t)col * ldu;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rr = Mfma<T>::row(lk, r);
                    if (r0 + rb * 16 + rr < m) dst[rr] = acc[r];
                }
            }
        }
    }
}

template <typename T, int NT>
__global__ void __launch_bounds__(UT_THREADS)
urecover_tile_kernel(const T *__restrict__ A, int64_t lda, const T *__restrict__ W, int64_t ldw,
                     T *__restrict__ U, int64_t ldu, int64_t m, int n, int64_t ntiles) {
    urecover_tile_body<T, NT>(A, lda, W, ldw, U, ldu, m, n, ntiles, blockIdx.x, gridDim.x);
}

// Batched: blockIdx.z picks the problem order[first + z]; its row tiles are
// dealt to the gridDim.x workgroups of that problem.
template <typename T, int NT>
__global__ void __launch_bounds__(UT_THREADS)
urecover_tile_batched_kernel(const BatchMat *__restrict__ tab, const int *__restrict__ order,
                             int first) {
    const BatchMat &d = tab[order[first + blockIdx.z]];
    const int64_t ntiles = (d.m + UT_BM - 1) / UT_BM;
    if ((int64_t)blockIdx.x >= ntiles) return;
    urecover_tile_body<T, NT>(reinterpret_cast<const T *>(d.A), d.lda,
                              reinterpret_cast<const T *>(d.W), d.n, reinterpret_cast<T *>(d.U),
                              d.ldu, d.m, d.n, ntiles, blockIdx.x, gridDim.x);
}

template <typename T, int NT>
static size_t tile_lds(void) {
    return (size_t)(NT * 16) * (NT * 16 + 2) * sizeof(T) + (size_t)(NT * 16) * (UT_BM + 2) * sizeof(T);
}

template <typename T, int NT>
static hipError_t launch_tile(int64_t m, int64_t n, const T *A, int64_t lda, const T *W,
                              int64_t ldw, T *U, int64_t ldu, hipStream_t st) {
    const int64_t ntiles = (m + UT_BM - 1) / UT_BM;
    const size_t lds = tile_lds<T, NT>();
    const int per_cu = lds <= 80 * 1024 ? 2 : 1;
    int64_t grid = 256 * per_cu;
    if (grid > ntiles) grid = ntiles;
    if (grid < 1) grid = 1;
    auto k = urecover_tile_kernel<T, NT>;
    hipError_t err = hipFuncSetAttribute((const void *)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(UT_THREADS), lds, st, A, lda, W, ldw, U, ldu,
                       m, (int)n, ntiles);
    return hipGetLastError();
}

template <typename T, int NT>
static hipError_t launch_nt(int64_t m, int64_t n, const T *A, int64_t lda, const T *W, int64_t ldw,
                            T *U, int64_t ldu, hipStream_t st) {
    const int64_t ngroups = (m + 63) / 64;
    int64_t grid = ngroups < 2048 ? ngroups : 2048;
    if (grid < 1) grid = 1;
    const size_t lds = (size_t)(NT * 16) * (NT * 16) * sizeof(T);
    auto k = urecover_kernel<T, NT>;
    hipError_t err = hipFuncSetAttribute((const void *)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(256), lds, st, A, lda, W, ldw, U, ldu, m,
                       (int)n, ngroups);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_t(int64_t m, int64_t n, const T *A, int64_t lda, const T *W, int64_t ldw,
                           T *U, int64_t ldu, hipStream_t st) {
    // tiled kernel while W and one A tile fit LDS comfortably; strip kernel otherwise
    switch ((n + 15) / 16) {
        case 1: return launch_tile<T, 1>(m, n, A, lda, W, ldw, U, ldu, st);
        case 2: return launch_tile<T, 2>(m, n, A, lda, W, ldw, U, ldu, st);
        case 3: return launch_tile<T, 3>(m, n, A, lda, W, ldw, U, ldu, st);
        case 4: return launch_tile<T, 4>(m, n, A, lda, W, ldw, U, ldu, st);
        case 5: return launch_tile<T, 5>(m, n, A, lda, W, ldw, U, ldu, st);
        case 6: return launch_tile<T, 6>(m, n, A, lda, W, ldw, U, ldu, st);
        default: break;
    }
    if (sizeof(T) == 4 && n <= 128) {
        if (n <= 112) return launch_tile<T, 7>(m, n, A, lda, W, ldw, U, ldu, st);
        return launch_tile<T, 8>(m, n, A, lda, W, ldw, U, ldu, st);
    }
    switch ((n + 15) / 16) {
        case 1: return launch_nt<T, 1>(m, n, A, lda, W, ldw, U, ldu, st);
        case 2: return launch_nt<T, 2>(m, n, A, lda, W, ldw, U, ldu, st);
        case 3: return launch_nt<T, 3>(m, n, A, lda, W, ldw, U, ldu, st);
        case 4: return launch_nt<T, 4>(m, n, A, lda, W, ldw, U, ldu, st);
        case 5: return launch_nt<T, 5>(m, n, A, lda, W, ldw, U, ldu, st);
        case 6: return launch_nt<T, 6>(m, n, A, lda, W, ldw, U, ldu, st);
        case 7: return launch_nt<T, 7>(m, n, A, lda, W, ldw, U, ldu, st);
        case 8: return launch_nt<T, 8>(m, n, A, lda, W, ldw, U, ldu, st);
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

int urecover_batched_max_nt(int working) { return working == 1 ? 6 : 8; }

template <typename T, int NT>
static hipError_t batched_tile(const BatchMat *tab, const int *order, int first, int count,
                               int64_t max_m, hipStream_t st) {
    const size_t lds = tile_lds<T, NT>();
    // about eight row tiles per workgroup for the tallest problem of the group
    int64_t gx = ((max_m + UT_BM - 1) / UT_BM + 7) / 8;
    if (gx < 1) gx = 1;
    if (gx > 65535) gx = 65535;
    auto k = urecover_tile_batched_kernel<T, NT>;
    hipError_t err = hipFuncSetAttribute((const void *)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3((unsigned)gx, 1, (unsigned)count), dim3(UT_THREADS), lds, st, tab,
                       order, first);
    return hipGetLastError();
}

template <typename T>
static hipError_t batched_t(const BatchMat *tab, const int *order, int first, int count, int nt,
                            int64_t max_m, hipStream_t st) {
    switch (nt) {
        case 1: return batched_tile<T, 1>(tab, order, first, count, max_m, st);
        case 2: return batched_tile<T, 2>(tab, order, first, count, max_m, st);
        case 3: return batched_tile<T, 3>(tab, order, first, count, max_m, st);
        case 4: return batched_tile<T, 4>(tab, order, first, count, max_m, st);
        case 5: return batched_tile<T, 5>(tab, order, first, count, max_m, st);
        case 6: return batched_tile<T, 6>(tab, order, first, count, max_m, st);
        case 7: if (sizeof(T) == 4) return batched_tile<T, 7>(tab, order, first, count, max_m, st);
                return hipErrorInvalidValue;
        case 8: if (sizeof(T) == 4) return batched_tile<T, 8>(tab, order, first, count, max_m, st);
                return hipErrorInvalidValue;
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

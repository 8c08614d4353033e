// Mixed precision Cholesky QR (Sec. 3.3 of the paper, Theorem 3): the Gram
// matrix M_h = A^T A at the higher precision (the thin SVD's Gram stage), its
// Cholesky factor M_h = R_h^T R_h at the higher precision (the scaled blocked
// double-double Cholesky of Algorithm 2's first step), R = fl_w(R_h), then Q
// from Q R = A at the working precision: a row-wise triangular solve.
//
// The solve: each lane owns one row of A and Q and works through the columns
// in blocks of 16.  For block J it starts from A(i, J), subtracts the products
// of the row's finished blocks Q(i, K), K < J, with R(K, J) (the R block column
// staged in LDS, read by every lane at the same address), then substitutes
// inside the block: q_j = acc_j / r_jj and acc_l -= q_j r_jl for l > j.  That is
// forward substitution on the row, column by column, with the sum for each
// q_j taken over k < j in blocked order: the row-wise backward error
// Q(i, :) (R + dR_i) = A(i, :), |dR_i| <= eps |R|, of the proof of Theorem 3.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "api_util.hpp"
#include "gsvd.h"
#include "gsvd_internal.hpp"

namespace gsvd {
namespace {

constexpr int QB = 16;    // column block
constexpr int QT = 256;   // rows per workgroup (one per lane)

template <typename T>
__global__ void __launch_bounds__(QT)
trsm_rows_kernel(int64_t m, int n, const T *__restrict__ A, int64_t lda,
                 const T *__restrict__ R, int64_t ldr, T *__restrict__ Q, int64_t ldq,
                 const int *__restrict__ info) {
    extern __shared__ __attribute__((aligned(16))) unsigned char qsm[];
    T *Rs = reinterpret_cast<T *>(qsm);  // rows 0 .. j0 + 15 of block column J, row-major by k
    if (*info != 0) return;
    const int64_t i = (int64_t)blockIdx.x * QT + threadIdx.x;
    const bool row = i < m;
    const int nblk = (n + QB - 1) / QB;
    for (int J = 0; J < nblk; ++J) {
        const int j0 = QB * J;
        const int kend = j0 + QB < n ? j0 + QB : n;  // rows of R the block needs
        __syncthreads();  // the previous block's reads of Rs are done
        for (int e = threadIdx.x; e < kend * QB; e += QT) {
            const int k = e / QB, l = e % QB;
            const int c = j0 + l;
            Rs[e] = (c < n && k <= c) ? R[k + (int64_t)c * ldr] : (T)0;
        }
        __syncthreads();
        if (!row) continue;
        T acc[QB];
#pragma unroll
        for (int l = 0; l < QB; ++l) acc[l] = (j0 + l < n) ? A[i + (int64_t)(j0 + l) * lda] : (T)0;
        for (int K = 0; K < J; ++K) {
            T q[QB];
#pragma unroll
            for (int k = 0; k < QB; ++k) q[k] = Q[i + (int64_t)(QB * K + k) * ldq];
#pragma unroll
            for (int k = 0; k < QB; ++k) {
                const T *rr = Rs + (QB * K + k) * QB;
#pragma unroll
                for (int l = 0; l < QB; ++l) acc[l] = __builtin_fma(-q[k], rr[l], acc[l]);
            }
        }
#pragma unroll
        for (int j = 0; j < QB; ++j) {
            if (j0 + j >= n) break;
            const T *rr = Rs + (j0 + j) * QB;
            const T qj = acc[j] / rr[j];
            Q[i + (int64_t)(j0 + j) * ldq] = qj;
#pragma unroll
            for (int l = j + 1; l < QB; ++l) acc[l] = __builtin_fma(-qj, rr[l], acc[l]);
        }
    }
}

struct QrLayout {
    size_t mhi, mlo, chol, part, total;
};

QrLayout qr_layout(int64_t m, int64_t n, const gsvd_opts *o) {
    QrLayout L{};
    const size_t nn = (size_t)n * (size_t)n;
    size_t off = 0;
    L.mhi = off;
    off = align_up(off + nn * sizeof(double));
    L.mlo = off;
    off = align_up(off + nn * sizeof(double));
    L.chol = off;
    off = align_up(off + chol_work_bytes(n));
    L.part = off;
    off = align_up(off + gram_part_bytes(m, n, o, false));
    L.total = off;
    return L;
}

}  // namespace

hipError_t trsm_rows_launch(int working, int64_t m, int64_t n, const void *A, int64_t lda,
                            const void *R, int64_t ldr, void *Q, int64_t ldq, const int *info,
                            hipStream_t st) {
    const unsigned blocks = (unsigned)((m + QT - 1) / QT);
    const size_t wsz = working == GSVD_F64 ? 8 : 4;
    const size_t lds = (size_t)((n + QB - 1) / QB * QB) * QB * wsz;
    if (working == GSVD_F64) {
        auto k = trsm_rows_kernel<double>;
        hipError_t err = hipFuncSetAttribute((const void *)k,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k, dim3(blocks), dim3(QT), lds, st, m, (int)n, (const double *)A, lda,
                           (const double *)R, ldr, (double *)Q, ldq, info);
    } else {
        auto k = trsm_rows_kernel<float>;
        hipError_t err = hipFuncSetAttribute((const void *)k,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k, dim3(blocks), dim3(QT), lds, st, m, (int)n, (const float *)A, lda,
                           (const float *)R, ldr, (float *)Q, ldq, info);
    }
    return hipGetLastError();
}

}  // namespace gsvd

using namespace gsvd;

extern "C" {

size_t gsvd_cholqr_workspace_size(int64_t m, int64_t n, const gsvd_opts *o) {
    if (m < 1 || n < 1 || check_opts(o, 3) != 0) return 0;
    const gsvd_opts r = resolve_opts(o, m, n, false);
    return qr_layout(m, n, &r).total;
}

int gsvd_cholqr(int64_t m, int64_t n, const void *dA, int64_t lda, void *dQ, int64_t ldq,
                void *dR, int64_t ldr, void *work, size_t work_bytes, int *dInfo,
                const gsvd_opts *o, void *stream) {
    if (m < 1) return -1;
    if (n < 1 || n > GSVD_MAX_N || n > m) return -2;
    if (dA == nullptr) return -3;
    if (lda < m) return -4;
    if (dQ == nullptr) return -5;
    if (ldq < m) return -6;
    if (dR == nullptr) return -7;
    if (ldr < n) return -8;
    if (work == nullptr || !aligned(work, kAlign)) return -9;
    if (dInfo == nullptr) return -11;
    if (int e = check_opts(o, 12)) return e;
    const gsvd_opts r = resolve_opts(o, m, n, false);
    o = &r;
    if (int e = check_gram_supported(o, n)) return e;
    const QrLayout L = qr_layout(m, n, o);
    if (work_bytes < L.total) return -10;
    hipStream_t st = (hipStream_t)stream;
    char *base = (char *)work;
    double *Mhi = (double *)(base + L.mhi);
    double *Mlo = (double *)(base + L.mlo);
    hipError_t err = gram_any(o, m, n, dA, lda, Mhi, Mlo, n, base + L.part, st);
    if (err == hipSuccess)
        err = chol_launch(o->working, n, Mhi, Mlo, n, dR, ldr, dInfo, base + L.chol, st);
    if (err == hipSuccess)
        err = trsm_rows_launch(o->working, m, n, dA, lda, dR, ldr, dQ, ldq, dInfo, st);
    return err == hipSuccess ? GSVD_OK : GSVD_ERR_HIP;
}

}  // extern "C"

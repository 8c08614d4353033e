// Higher-precision Gram M_h = A^T A (Alg. 1 steps 1-2, eq. (ATA)).
//
// Split-m tiled SYRK.  The upper triangle of M is covered by 2x2 register
// blocks (bi, bj), bi <= bj, enumerated row by row; every lane of a workgroup
// owns one block.  blockIdx.y selects a slab of rows ("split"); the slab is
// streamed through LDS in chunks of KC rows, each chunk staged as a row-major
// KC x NC tile so a lane reads its two A(k, i) values and its two A(k, j)
// values with one 16-byte LDS read each.  Global loads walk down the columns
// (A is column-major), so they are coalesced.  The chunk after the current one
// is fetched into registers while the current one is consumed.
//
// FP64 A: every product is formed exactly (TwoProduct) and summed in
// double-double (TwoSum), i.e. the Gram is carried at u_h ~ 2^-104.
// FP32 A: the FP64 product of two FP32 numbers is exact; the sums are FP64.
//
// Each (split, block) writes its four dd partial sums to its own slot of the
// workspace; gram_reduce_kernel then adds the splits with a fixed-shape tree,
// so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include "dd_device.hpp"
#include "gsvd_internal.hpp"

namespace gsvd {

constexpr int KC = 32;  // rows per LDS chunk

__device__ __forceinline__ void decode_block(int b, int nbh, int &bi, int &bj) {
    int i = 0, rem = b;
    while (rem >= nbh - i) {
        rem -= nbh - i;
        ++i;
    }
    bi = i;
    bj = i + rem;
}

template <typename T, bool DD>
__global__ void __launch_bounds__(1024)
gram_partial_kernel(const T *__restrict__ A, int64_t lda, int64_t m, int n, int nbh, int nblk,
                    int64_t rows_per_split, double *__restrict__ part) {
    extern __shared__ double lds[];
    const int NC = 2 * nbh;       // staged columns (n rounded up to even)
    const int LDL = NC + 2;       // row stride in LDS (keeps 16-byte alignment)
    double *buf0 = lds;
    double *buf1 = lds + KC * LDL;

    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int b = blockIdx.x * nthr + tid;
    const bool active = b < nblk;
    int bi = 0, bj = 0;
    if (active) decode_block(b, nbh, bi, bj);

    const int64_t split = blockIdx.y;
    const int64_t r0 = split * rows_per_split;
    const int64_t r1 = (r0 + rows_per_split < m) ? r0 + rows_per_split : m;
    const int nchunk = (int)((r1 - r0 + KC - 1) / KC);

    // staging: element e of a chunk is (k = e % KC, c = e / KC)
    const int nelem = KC * NC;
    constexpr int MAXPER = 8;  // KC * 128 / 576 rounded up; checked on the host
    const int per = (nelem + nthr - 1) / nthr;

    double stage[MAXPER];
    auto fetch = [&](int chunk) {
        const int64_t base = r0 + (int64_t)chunk * KC;
#pragma unroll
        for (int q = 0; q < MAXPER; ++q) {
            stage[q] = 0.0;
            if (q < per) {
                int e = tid + q * nthr;
                if (e < nelem) {
                    int k = e % KC, c = e / KC;
                    int64_t r = base + k;
                    if (r < r1 && c < n) stage[q] = (double)A[r + (int64_t)c * lda];
                }
            }
        }
    };
    auto commit = [&](double *dst) {
#pragma unroll
        for (int q = 0; q < MAXPER; ++q) {
            if (q < per) {
                int e = tid + q * nthr;
                if (e < nelem) dst[(e % KC) * LDL + e / KC] = stage[q];
            }
        }
    };

    double h00 = 0, h01 = 0, h10 = 0, h11 = 0;
    double l00 = 0, l01 = 0, l10 = 0, l11 = 0;

    if (nchunk > 0) {
        fetch(0);
        commit(buf0);
    }
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
        double *cur = (ch & 1) ? buf1 : buf0;
        double *nxt = (ch & 1) ? buf0 : buf1;
        const bool more = ch + 1 < nchunk;
        if (more) fetch(ch + 1);
        if (active) {
            const double *pi = cur + 2 * bi;
            const double *pj = cur + 2 * bj;
#pragma unroll 8
            for (int k = 0; k < KC; ++k) {
                const double2 ai = *reinterpret_cast<const double2 *>(pi + k * LDL);
                const double2 aj = *reinterpret_cast<const double2 *>(pj + k * LDL);
                if (DD) {
                    dd_mac(h00, l00, ai.x, aj.x);
                    dd_mac(h01, l01, ai.x, aj.y);
                    dd_mac(h10, l10, ai.y, aj.x);
                    dd_mac(h11, l11, ai.y, aj.y);
                } else {
                    h00 = __builtin_fma(ai.x, aj.x, h00);
                    h01 = __builtin_fma(ai.x, aj.y, h01);
                    h10 = __builtin_fma(ai.y, aj.x, h10);
                    h11 = __builtin_fma(ai.y, aj.y, h11);
                }
            }
        }
        if (more) commit(nxt);
        __syncthreads();
    }
    if (active) {
        if (DD) {
            dd_t s;
            s = quick_two_sum(h00, l00); h00 = s.hi; l00 = s.lo;
            s = quick_two_sum(h01, l01); h01 = s.hi; l01 = s.lo;
            s = quick_two_sum(h10, l10); h10 = s.hi; l10 = s.lo;
            s = quick_two_sum(h11, l11); h11 = s.hi; l11 = s.lo;
        }
        double4 *dst = reinterpret_cast<double4 *>(part + ((size_t)split * nblk + b) * 8);
        dst[0] = make_double4(h00, l00, h01, l01);
        dst[1] = make_double4(h10, l10, h11, l11);
    }
}

// One wavefront per M entry: lane l adds splits l, l + 64, ... in order, then a
// fixed xor-butterfly over the 64 lanes; lane 0 writes M(i, j) and M(j, i).
__global__ void __launch_bounds__(256)
gram_reduce_kernel(const double *__restrict__ part, int64_t nsplit, int nbh, int nblk, int n,
                   double *__restrict__ Mhi, double *__restrict__ Mlo, int64_t ldm) {
    const int lane = threadIdx.x & 63;
    const int64_t entry = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (entry >= (int64_t)nblk * 4) return;
    const int b = (int)(entry >> 2), e = (int)(entry & 3);
    dd_t acc{0.0, 0.0};
    for (int64_t s = lane; s < nsplit; s += 64) {
        const double *p = part + ((size_t)s * nblk + b) * 8 + 2 * e;
        acc = dd_add(acc, dd_t{p[0], p[1]});
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        dd_t o{__shfl_xor(acc.hi, off), __shfl_xor(acc.lo, off)};
        acc = dd_add(acc, o);
    }
    if (lane == 0) {
        int bi, bj;
        decode_block(b, nbh, bi, bj);
        const int i = 2 * bi + (e >> 1), j = 2 * bj + (e & 1);
        if (i < n && j < n && i <= j) {
            Mhi[i + (int64_t)j * ldm] = acc.hi;
            Mhi[j + (int64_t)i * ldm] = acc.hi;
            if (Mlo) {
                Mlo[i + (int64_t)j * ldm] = acc.lo;
                Mlo[j + (int64_t)i * ldm] = acc.lo;
            }
        }
    }
}

GramPlan gram_plan(int64_t m, int64_t n) {
    GramPlan p{};
    p.nbh = (int)((n + 1) / 2);
    p.nblk = p.nbh * (p.nbh + 1) / 2;
    const int wgs_x = (p.nblk + 1023) / 1024;
    const int per_wg = (p.nblk + wgs_x - 1) / wgs_x;
    // enough lanes for the blocks, and for staging a chunk with <= 8 values per lane
    int need = per_wg;
    const int stage_need = (KC * 2 * p.nbh + 7) / 8;
    if (stage_need > need) need = stage_need;
    p.threads = ((need + 63) / 64) * 64;
    p.grid_x = wgs_x;
    // about 2048 workgroups in flight, every slab a multiple of KC rows
    int64_t target = 2048 / wgs_x;
    if (target < 1) target = 1;
    int64_t rps = (m + target - 1) / target;
    rps = ((rps + KC - 1) / KC) * KC;
    if (rps < KC) rps = KC;
    p.rows_per_split = rps;
    p.nsplit = (m + rps - 1) / rps;
    if (p.nsplit < 1) p.nsplit = 1;
    p.lds_bytes = (size_t)2 * KC * (2 * p.nbh + 2) * sizeof(double);
    p.part_bytes = (size_t)p.nsplit * p.nblk * 8 * sizeof(double);
    return p;
}

hipError_t gram_launch(int working, int64_t m, int64_t n, const void *A, int64_t lda,
                       double *Mhi, double *Mlo, int64_t ldm, void *part, const GramPlan &p,
                       hipStream_t st) {
    // every chunk element must fit the per-thread staging array
    if ((KC * 2 * p.nbh + p.threads - 1) / p.threads > 8) return hipErrorInvalidValue;
    dim3 grid(p.grid_x, (unsigned)p.nsplit);
    hipError_t err;
    if (working == 1) {
        auto k = gram_partial_kernel<double, true>;
        err = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)p.lds_bytes);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k, grid, dim3(p.threads), p.lds_bytes, st, (const double *)A, lda, m,
                           (int)n, p.nbh, p.nblk, p.rows_per_split, (double *)part);
    } else {
        auto k = gram_partial_kernel<float, false>;
        err = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)p.lds_bytes);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k, grid, dim3(p.threads), p.lds_bytes, st, (const float *)A, lda, m,
                           (int)n, p.nbh, p.nblk, p.rows_per_split, (double *)part);
    }
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int64_t entries = (int64_t)p.nblk * 4;
    const unsigned rgrid = (unsigned)((entries + 3) / 4);
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(rgrid), dim3(256), 0, st, (const double *)part,
                       p.nsplit, p.nbh, p.nblk, (int)n, Mhi, Mlo, ldm);
    return hipGetLastError();
}

}  // namespace gsvd

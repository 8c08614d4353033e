// Gram M_h = A^T A by exact operand splitting on the int8 matrix cores
// (the "split" form of Alg. 1 steps 1-2).
//
// Rows are processed in chunks of 64.  For every column j of a chunk, e_j is
// the smallest power of two with |a_kj| < 2^e_j over the chunk's rows.  Each
// entry is cut into S signed 7-bit integer slices,
//     a_kj = 2^e_j sum_{r=1..S} c_r 2^(-7 r) + tail,   c_r in [-127, 127],
// by peeling base-128 digits off |a| 2^-e_j (every step exact in FP64).  The
// chunk's contribution to M(i, j) is then
//     2^(e_i + e_j) sum_{s=2..S+1} 2^(-7 s) I_s,   I_s = sum_{r+t=s} sum_k c_r,ki c_t,kj,
// keeping the slice pairs with r + t <= S + 1 (the dropped pairs are below the
// last kept digit).  Every I_s is an exact integer: 64 rows x at most S pairs
// x 127^2 < 2^31, accumulated by v_mfma_i32_16x16x64_i8.
//
// Layout: the chunk's slices sit in LDS as int8, column-major (64 rows of a
// column are 64 contiguous bytes), one plane per slice.  A 16x16 tile (I, J)
// of M takes its A operand from columns 16 I .. 16 I + 15 and its B operand
// from columns 16 J .. 16 J + 15: lane l reads the 16 bytes of rows
// 16 (l / 16) .. + 15 of column 16 I + l % 16 (resp. 16 J + l % 16); the
// integer result gives lane l, register q the entry (4 (l / 16) + q, l % 16).
// The tiles I <= J of the upper triangle are dealt round-robin to the four
// wavefronts of a workgroup; each tile's S per-diagonal sums are combined
// exactly (Horner in groups of four diagonals, then double-double) and added to
// the tile's double-double accumulator (FP64 A) or FP64 accumulator (FP32 A).
//
// The slab / partial / fixed-order reduction structure is the one of the
// plain form, so the result is reproducible bit for bit.
#include <hip/hip_runtime.h>

#include "dd_device.hpp"
#include "gsvd_internal.hpp"

namespace gsvd {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int SP_KT = 64;        // rows per chunk (one MFMA k-depth)
constexpr int SP_THREADS = 256;  // four wavefronts
constexpr int SP_SMAX = 12;      // largest slice count

__device__ __forceinline__ void sp_decode_pair(int p, int nb, int &bi, int &bj) {
    int i = 0, rem = p;
    while (rem >= nb - i) {
        rem -= nb - i;
        ++i;
    }
    bi = i;
    bj = i + rem;
}

// max over the 16 lanes of a DPP row
__device__ __forceinline__ int row_max_i(int x) {
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x141, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x140, 0xf, 0xf, false));
    return x;
}

template <typename T, int NB>
__global__ void __launch_bounds__(SP_THREADS)
gram_split_kernel(const T *__restrict__ A, int64_t lda, int64_t m, int n, int S,
                  int64_t rows_per_split, double *__restrict__ part) {
    constexpr bool DD = sizeof(T) == 8;
    constexpr int N16 = 16 * NB;
    constexpr int NPAIR = NB * (NB + 1) / 2;
    constexpr int PMAX = (NPAIR + 3) / 4;  // tiles per wavefront
    constexpr int SL = N16 * SP_KT;        // bytes per slice plane
    extern __shared__ unsigned char smem[];
    signed char *planes = reinterpret_cast<signed char *>(smem);  // [S][N16][64]
    int *exps = reinterpret_cast<int *>(smem + SP_SMAX * SL);     // [N16]

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t split = blockIdx.y;
    const int64_t r0 = split * rows_per_split;
    const int64_t r1 = (r0 + rows_per_split < m) ? r0 + rows_per_split : m;
    const int nchunk = (int)((r1 - r0 + SP_KT - 1) / SP_KT);

    // loading: pass p covers columns 16 p .. 16 p + 15; thread t takes column
    // 16 p + t / 16 and rows 4 (t % 16) .. + 3 of the chunk
    const int lc = tid >> 4, lr = 4 * (tid & 15);
    T vals[NB][4];
    auto fetch = [&](int chunk) {
        const int64_t base = r0 + (int64_t)chunk * SP_KT + lr;
#pragma unroll
        for (int p = 0; p < NB; ++p) {
            const int c = 16 * p + lc;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t r = base + q;
                vals[p][q] = (c < n && r < r1) ? A[r + (int64_t)c * lda] : (T)0;
            }
        }
    };

    // accumulators of this wavefront's tiles: lane l, register q of tile w + 4 k
    double acc_hi[PMAX][4], acc_lo[PMAX][4];
#pragma unroll
    for (int k = 0; k < PMAX; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            acc_hi[k][q] = 0.0;
            acc_lo[k][q] = 0.0;
        }

    if (nchunk > 0) fetch(0);
    for (int ch = 0; ch < nchunk; ++ch) {
        __syncthreads();  // the previous chunk's planes are no longer read
        // ---- exponents and slices of the staged chunk
#pragma unroll
        for (int p = 0; p < NB; ++p) {
            const int c = 16 * p + lc;
            int e = -2000;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double a = (double)vals[p][q];
                if (a != 0.0) e = max(e, ilogb(a) + 1);
            }
            e = row_max_i(e);  // the 16 lanes holding column c
            if ((tid & 15) == 0) exps[c] = e;
            double x[4];
            int sg[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double a = (double)vals[p][q];
                sg[q] = a < 0.0 ? -1 : 1;
                x[q] = e > -2000 ? ldexp(__builtin_fabs(a), -e) : 0.0;  // in [0, 1)
            }
            for (int r = 0; r < S; ++r) {
                unsigned packed = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double y = x[q] * 128.0;
                    const double d = __builtin_floor(y);
                    x[q] = y - d;  // exact
                    const int di = sg[q] * (int)d;
                    packed |= ((unsigned)di & 0xffu) << (8 * q);
                }
                *reinterpret_cast<unsigned *>(planes + r * SL + c * SP_KT + lr) = packed;
            }
        }
        __syncthreads();
        if (ch + 1 < nchunk) fetch(ch + 1);  // overlaps the MFMA phase

        // ---- tiles of this wavefront
#pragma unroll
        for (int k = 0; k < PMAX; ++k) {
            const int pidx = wave + 4 * k;
            if (pidx < NPAIR) {
                int bi, bj;
                sp_decode_pair(pidx, NB, bi, bj);
                const int ca = 16 * bi + (lane & 15), cb = 16 * bj + (lane & 15);
                const int off = 16 * (lane >> 4);
                v4i bop[SP_SMAX];
#pragma unroll
                for (int t = 0; t < SP_SMAX; ++t)
                    if (t < S) bop[t] = *reinterpret_cast<const v4i *>(planes + t * SL + cb * SP_KT + off);
                v4i diag[SP_SMAX];
#pragma unroll
                for (int s = 0; s < SP_SMAX; ++s) diag[s] = v4i{0, 0, 0, 0};
#pragma unroll
                for (int r = 0; r < SP_SMAX; ++r) {
                    if (r < S) {
                        const v4i aop = *reinterpret_cast<const v4i *>(planes + r * SL + ca * SP_KT + off);
#pragma unroll
                        for (int t = 0; t < SP_SMAX; ++t)
                            if (t < S - r)  // r + t <= S - 1 (zero-based): the kept pairs
                                diag[r + t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(aop, bop[t], diag[r + t], 0, 0, 0);
                    }
                }
                // combine: value = 2^(e_i + e_j) sum_{s0 = 0..S-1} diag[s0] 2^(-7 (s0 + 2))
                const int ej = exps[cb];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int ei = exps[16 * bi + 4 * (lane >> 4) + q];
                    if (ei <= -2000 || ej <= -2000) continue;  // a zero column in this chunk
                    if (DD) {
                        // groups of four diagonals are exact in FP64 (Horner, <= 31 + 21 bits)
                        dd_t tot{0.0, 0.0};
#pragma unroll
                        for (int g0 = 0; g0 < SP_SMAX; g0 += 4) {
                            if (g0 < S) {
                                double v = 0.0;
#pragma unroll
                                for (int u = 3; u >= 0; --u)
                                    if (g0 + u < S) v = v * 0x1p-7 + (double)diag[g0 + u][q];
                                tot = dd_add(tot, dd_t{ldexp(v, -7 * (g0 + 2)), 0.0});
                            }
                        }
                        const int sc = ei + ej;
                        const dd_t add{ldexp(tot.hi, sc), ldexp(tot.lo, sc)};
                        const dd_t nacc = dd_add(dd_t{acc_hi[k][q], acc_lo[k][q]}, add);
                        acc_hi[k][q] = nacc.hi;
                        acc_lo[k][q] = nacc.lo;
                    } else {
                        double v = 0.0;
#pragma unroll
                        for (int s0 = SP_SMAX - 1; s0 >= 0; --s0)
                            if (s0 < S) v = v * 0x1p-7 + (double)diag[s0][q];
                        acc_hi[k][q] += ldexp(v, ei + ej - 14);
                    }
                }
            }
        }
    }

    // ---- partial sums of this slab: [split][tile][lane][q][hi, lo]
#pragma unroll
    for (int k = 0; k < PMAX; ++k) {
        const int pidx = wave + 4 * k;
        if (pidx < NPAIR) {
            double4 *dst = reinterpret_cast<double4 *>(
                part + (((size_t)split * NPAIR + pidx) * 64 + lane) * 8);
            dst[0] = make_double4(acc_hi[k][0], acc_lo[k][0], acc_hi[k][1], acc_lo[k][1]);
            dst[1] = make_double4(acc_hi[k][2], acc_lo[k][2], acc_hi[k][3], acc_lo[k][3]);
        }
    }
}

// One wavefront per M entry of the tile layout; splits added as in the plain form.
__global__ void __launch_bounds__(256)
gram_split_reduce_kernel(const double *__restrict__ part, int64_t nsplit, int nb, int npair, int n,
                         double *__restrict__ Mhi, double *__restrict__ Mlo, int64_t ldm) {
    const int lanew = threadIdx.x & 63;
    const int64_t entry = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (entry >= (int64_t)npair * 256) return;
    const int pidx = (int)(entry / 256), e = (int)(entry % 256);
    const int l = e / 4, q = e % 4;
    dd_t acc{0.0, 0.0};
    for (int64_t s = lanew; s < nsplit; s += 64) {
        const double *p = part + (((size_t)s * npair + pidx) * 64 + l) * 8 + 2 * q;
        acc = dd_add(acc, dd_t{p[0], p[1]});
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        dd_t o{__shfl_xor(acc.hi, off), __shfl_xor(acc.lo, off)};
        acc = dd_add(acc, o);
    }
    if (lanew == 0) {
        int bi, bj;
        sp_decode_pair(pidx, nb, bi, bj);
        const int i = 16 * bi + 4 * (l / 16) + q, j = 16 * bj + (l % 16);
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

SplitPlan split_plan(int64_t m, int64_t n, int S) {
    SplitPlan p{};
    p.S = S;
    p.nb = (int)((n + 15) / 16);
    p.npair = p.nb * (p.nb + 1) / 2;
    int64_t target = 1024;  // slabs: four workgroups per compute unit
    int64_t rps = (m + target - 1) / target;
    rps = ((rps + SP_KT - 1) / SP_KT) * SP_KT;
    if (rps < SP_KT) rps = SP_KT;
    p.rows_per_split = rps;
    p.nsplit = (m + rps - 1) / rps;
    p.lds_bytes = (size_t)SP_SMAX * 16 * p.nb * SP_KT + 16 * p.nb * sizeof(int);
    p.part_bytes = (size_t)p.nsplit * p.npair * 64 * 8 * sizeof(double);
    return p;
}

template <typename T, int NB>
static hipError_t split_launch_nb(int64_t m, int64_t n, const T *A, int64_t lda, double *Mhi,
                                  double *Mlo, int64_t ldm, void *part, const SplitPlan &p,
                                  hipStream_t st) {
    auto k = gram_split_kernel<T, NB>;
    hipError_t err = hipFuncSetAttribute((const void *)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)p.lds_bytes);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3(1, (unsigned)p.nsplit), dim3(SP_THREADS), p.lds_bytes, st, A, lda,
                       m, (int)n, p.S, p.rows_per_split, (double *)part);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int64_t entries = (int64_t)p.npair * 256;
    hipLaunchKernelGGL(gram_split_reduce_kernel, dim3((unsigned)((entries + 3) / 4)), dim3(256), 0,
                       st, (const double *)part, p.nsplit, p.nb, p.npair, (int)n, Mhi, Mlo, ldm);
    return hipGetLastError();
}

template <typename T>
static hipError_t split_launch_t(int64_t m, int64_t n, const T *A, int64_t lda, double *Mhi,
                                 double *Mlo, int64_t ldm, void *part, const SplitPlan &p,
                                 hipStream_t st) {
    switch (p.nb) {
        case 1: return split_launch_nb<T, 1>(m, n, A, lda, Mhi, Mlo, ldm, part, p, st);
        case 2: return split_launch_nb<T, 2>(m, n, A, lda, Mhi, Mlo, ldm, part, p, st);
        case 3: return split_launch_nb<T, 3>(m, n, A, lda, Mhi, Mlo, ldm, part, p, st);
        case 4: return split_launch_nb<T, 4>(m, n, A, lda, Mhi, Mlo, ldm, part, p, st);
        case 5: return split_launch_nb<T, 5>(m, n, A, lda, Mhi, Mlo, ldm, part, p, st);
        case 6: return split_launch_nb<T, 6>(m, n, A, lda, Mhi, Mlo, ldm, part, p, st);
        case 7: return split_launch_nb<T, 7>(m, n, A, lda, Mhi, Mlo, ldm, part, p, st);
        case 8: return split_launch_nb<T, 8>(m, n, A, lda, Mhi, Mlo, ldm, part, p, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t split_launch(int working, int64_t m, int64_t n, const void *A, int64_t lda, double *Mhi,
                        double *Mlo, int64_t ldm, void *part, const SplitPlan &p, hipStream_t st) {
    if (p.S < 1 || p.S > SP_SMAX || p.nb < 1 || p.nb > 8) return hipErrorInvalidValue;
    if (working == 1)
        return split_launch_t<double>(m, n, (const double *)A, lda, Mhi, Mlo, ldm, part, p, st);
    return split_launch_t<float>(m, n, (const float *)A, lda, Mhi, Mlo, ldm, part, p, st);
}

}  // namespace gsvd

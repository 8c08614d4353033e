// Higher-precision Gram M_h = A^T A (Alg. 1 steps 1-2, eq. (ATA)).
//
// Split-m tiled SYRK.  The upper triangle of M is covered by 4x4 register
// blocks (bi, bj), bi <= bj, enumerated row by row.  A workgroup holds
// nblk x ks lanes: lane t owns block t % nblk for the k-group t / nblk, and
// the ks k-groups take interleaved rows of each LDS chunk, so every lane keeps
// 16 independent accumulators (enough independent work to hide FP64 latency)
// and a 64-column problem fills 680 of 704 lanes.  blockIdx.y selects a slab
// of rows ("split").  The slab is streamed through LDS in chunks of kc rows
// staged row-major (a lane reads its four A(k, i) and four A(k, j) with four
// 16-byte LDS reads per 16 multiply-adds); global loads walk down the columns
// of the column-major A, so they are coalesced, and the next chunk is fetched
// into registers while the current one is consumed.
//
// FP64 A: every product is formed exactly (TwoProduct) and summed in
// double-double (TwoSum), i.e. the Gram is carried at u_h ~ 2^-104.
// FP32 A: the FP64 product of two FP32 numbers is exact; the sums are FP64.
//
// At the end of the slab the k-groups are added into k-group 0 in a fixed
// order through LDS, and each (split, block) writes its 16 dd partial sums to
// its own slot of the workspace; gram_reduce_kernel then adds the splits with
// a fixed-shape tree.  The result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include "dd_device.hpp"
#include "gsvd_internal.hpp"

namespace gsvd {

constexpr int BS = 4;       // register block edge
constexpr int MAXPER = 6;   // staged chunk elements per lane

__device__ __forceinline__ void decode_block(int b, int nb, int &bi, int &bj) {
    int i = 0, rem = b;
    while (rem >= nb - i) {
        rem -= nb - i;
        ++i;
    }
    bi = i;
    bj = i + rem;
}

constexpr int GRAM_MAX_THREADS = 768;  // three waves per SIMD: up to 168 VGPRs per lane

// The partial Gram of slab `split` of one matrix (one workgroup).
// Blocks b0 .. b0 + nblkg - 1 (those below nblk) of slab `split`.
template <typename T, bool DD>
__device__ __forceinline__ void gram_partial_body(const T *__restrict__ A, int64_t lda, int64_t m,
                                                  int n, int nb, int nblk, int b0, int nblkg,
                                                  int ks, int kc, int64_t rows_per_split,
                                                  int64_t split, double *__restrict__ part,
                                                  double *lds) {
    const int NC = BS * nb;     // staged columns (n rounded up to a multiple of 4)
    const int LDL = NC + 2;     // row stride in LDS (16-byte aligned rows)
    double *buf0 = lds;
    double *buf1 = lds + kc * LDL;

    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int g = tid / nblkg;         // k-group
    const int bl = tid - g * nblkg;    // block within the group
    const int b = b0 + bl;             // block
    const bool active = g < ks && b < nblk;
    int bi = 0, bj = 0;
    if (active) decode_block(b, nb, bi, bj);

    const int64_t r0 = split * rows_per_split;
    const int64_t r1 = (r0 + rows_per_split < m) ? r0 + rows_per_split : m;
    const int nchunk = (int)((r1 - r0 + kc - 1) / kc);

    // staging: element e of a chunk is (k = e % kc, c = e / kc)
    const int nelem = kc * NC;
    double stage[MAXPER];
    auto fetch = [&](int chunk) {
        const int64_t base = r0 + (int64_t)chunk * kc;
#pragma unroll
        for (int q = 0; q < MAXPER; ++q) {
            stage[q] = 0.0;
            const int e = tid + q * nthr;
            if (e < nelem) {
                const int k = e % kc, c = e / kc;
                const int64_t r = base + k;
                if (r < r1 && c < n) stage[q] = (double)A[r + (int64_t)c * lda];
            }
        }
    };
    auto commit = [&](double *dst) {
#pragma unroll
        for (int q = 0; q < MAXPER; ++q) {
            const int e = tid + q * nthr;
            if (e < nelem) dst[(e % kc) * LDL + e / kc] = stage[q];
        }
    };

    double hi[BS * BS], lo[BS * BS];
#pragma unroll
    for (int q = 0; q < BS * BS; ++q) {
        hi[q] = 0.0;
        lo[q] = 0.0;
    }

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
            const double *pi = cur + BS * bi;
            const double *pj = cur + BS * bj;
#pragma unroll 2
            for (int k = g; k < kc; k += ks) {
                const double2 a01 = *reinterpret_cast<const double2 *>(pi + k * LDL);
                const double2 a23 = *reinterpret_cast<const double2 *>(pi + k * LDL + 2);
                const double2 b01 = *reinterpret_cast<const double2 *>(pj + k * LDL);
                const double2 b23 = *reinterpret_cast<const double2 *>(pj + k * LDL + 2);
                const double av[BS] = {a01.x, a01.y, a23.x, a23.y};
                const double bv[BS] = {b01.x, b01.y, b23.x, b23.y};
                if (DD) {
                    // four rows of four independent dd multiply-adds, each row written
                    // stage by stage so the dependent operations are four apart
#pragma unroll
                    for (int r = 0; r < BS; ++r) {
                        double p[BS], e[BS], s[BS], v[BS];
#pragma unroll
                        for (int c = 0; c < BS; ++c) p[c] = av[r] * bv[c];
#pragma unroll
                        for (int c = 0; c < BS; ++c) e[c] = __builtin_fma(av[r], bv[c], -p[c]);
#pragma unroll
                        for (int c = 0; c < BS; ++c) s[c] = hi[BS * r + c] + p[c];
#pragma unroll
                        for (int c = 0; c < BS; ++c) v[c] = s[c] - hi[BS * r + c];
#pragma unroll
                        for (int c = 0; c < BS; ++c) {
                            const int q = BS * r + c;
                            const double err = (hi[q] - (s[c] - v[c])) + (p[c] - v[c]);
                            hi[q] = s[c];
                            lo[q] += e[c] + err;
                        }
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < BS * BS; ++q)
                        hi[q] = __builtin_fma(av[q / BS], bv[q % BS], hi[q]);
                }
            }
        }
        if (more) commit(nxt);
        __syncthreads();
    }

    // add the k-groups into k-group 0, one group at a time (fixed order)
    double *red = lds;  // nblkg x 16 dd, reuses the chunk buffers
    for (int r = 1; r < ks; ++r) {
        if (active && g == r) {
            double4 *dst = reinterpret_cast<double4 *>(red + (size_t)bl * 32);
#pragma unroll
            for (int q = 0; q < BS * BS; q += 2) dst[q / 2] = make_double4(hi[q], lo[q], hi[q + 1], lo[q + 1]);
        }
        __syncthreads();
        if (active && g == 0) {
            const double4 *src = reinterpret_cast<const double4 *>(red + (size_t)bl * 32);
#pragma unroll
            for (int q = 0; q < BS * BS; q += 2) {
                const double4 o = src[q / 2];
                if (DD) {
                    dd_t x = dd_add(dd_t{hi[q], lo[q]}, dd_t{o.x, o.y});
                    dd_t y = dd_add(dd_t{hi[q + 1], lo[q + 1]}, dd_t{o.z, o.w});
                    hi[q] = x.hi; lo[q] = x.lo; hi[q + 1] = y.hi; lo[q + 1] = y.lo;
                } else {
                    hi[q] += o.x;
                    hi[q + 1] += o.z;
                }
            }
        }
        __syncthreads();
    }
    if (active && g == 0) {
        double4 *dst = reinterpret_cast<double4 *>(part + ((size_t)split * nblk + b) * 32);
#pragma unroll
        for (int q = 0; q < BS * BS; q += 2) {
            dd_t x = quick_two_sum(hi[q], lo[q]);
            dd_t y = quick_two_sum(hi[q + 1], lo[q + 1]);
            dst[q / 2] = make_double4(x.hi, x.lo, y.hi, y.lo);
        }
    }
}

// One workgroup per (slab, block group).  Workgroup ids are dealt to the XCDs
// round robin (id mod 8), so the ng groups of a slab take ids 8 apart: they
// run on one XCD and the second reader of a row chunk finds it in that XCD's L2.
template <typename T, bool DD>
__global__ void __launch_bounds__(GRAM_MAX_THREADS)
gram_partial_kernel(const T *__restrict__ A, int64_t lda, int64_t m, int n, int nb, int nblk,
                    int ng, int nblkg, int ks, int kc, int64_t rows_per_split, int64_t nsplit,
                    double *__restrict__ part) {
    extern __shared__ __attribute__((aligned(16))) double lds[];
    const int64_t id = blockIdx.x;
    const int64_t split = id / (8 * ng) * 8 + id % 8;
    const int grp = (int)(id / 8 % ng);
    if (split >= nsplit) return;  // uniform: the whole workgroup
    gram_partial_body<T, DD>(A, lda, m, n, nb, nblk, grp * nblkg, nblkg, ks, kc, rows_per_split,
                             split, part, lds);
}

// Batched: blockIdx.z picks the problem order[first + z], blockIdx.y its slab.
template <typename T, bool DD>
__global__ void __launch_bounds__(GRAM_MAX_THREADS)
gram_partial_batched_kernel(const BatchMat *__restrict__ tab, const int *__restrict__ order,
                            int first, int nb, int nblk, int ks, int kc) {
    extern __shared__ __attribute__((aligned(16))) double lds[];
    const BatchMat &d = tab[order[first + blockIdx.z]];
    if ((int)blockIdx.y >= d.nsplit) return;
    gram_partial_body<T, DD>(reinterpret_cast<const T *>(d.A), d.lda, d.m, d.n, nb, nblk, 0, nblk,
                             ks, kc, d.rows_per_split, blockIdx.y, d.part, lds);
}

// One wavefront per M entry: lane l adds splits l, l + 64, ... in order, then a
// fixed xor-butterfly over the 64 lanes; lane 0 writes M(i, j) and M(j, i).
__device__ __forceinline__ void gram_reduce_body(const double *__restrict__ part, int64_t nsplit,
                                                 int nb, int nblk, int n, double *__restrict__ Mhi,
                                                 double *__restrict__ Mlo, int64_t ldm) {
    const int lane = threadIdx.x & 63;
    const int64_t entry = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (entry >= (int64_t)nblk * BS * BS) return;
    const int b = (int)(entry / (BS * BS)), e = (int)(entry % (BS * BS));
    dd_t acc{0.0, 0.0};
    for (int64_t s = lane; s < nsplit; s += 64) {
        const double *p = part + ((size_t)s * nblk + b) * 32 + 2 * e;
        acc = dd_add(acc, dd_t{p[0], p[1]});
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        dd_t o{__shfl_xor(acc.hi, off), __shfl_xor(acc.lo, off)};
        acc = dd_add(acc, o);
    }
    if (lane == 0) {
        int bi, bj;
        decode_block(b, nb, bi, bj);
        const int i = BS * bi + e / BS, j = BS * bj + e % BS;
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

__global__ void __launch_bounds__(256)
gram_reduce_kernel(const double *__restrict__ part, int64_t nsplit, int nb, int nblk, int n,
                   double *__restrict__ Mhi, double *__restrict__ Mlo, int64_t ldm) {
    gram_reduce_body(part, nsplit, nb, nblk, n, Mhi, Mlo, ldm);
}

// Batched: blockIdx.y is the problem; blocks past its entries return at once.
__global__ void __launch_bounds__(256)
gram_reduce_batched_kernel(const BatchMat *__restrict__ tab) {
    const BatchMat &d = tab[blockIdx.y];
    const int nb = (d.n + BS - 1) / BS;
    gram_reduce_body(d.part, d.nsplit, nb, nb * (nb + 1) / 2, d.n, d.Mhi, d.Mlo, d.n);
}

GramPlan gram_plan(int64_t m, int64_t n, int64_t slab_rows, bool groups) {
    GramPlan p{};
    p.nb = (int)((n + BS - 1) / BS);
    p.nblk = p.nb * (p.nb + 1) / 2;
    // Lanes = ks k-groups x the blocks of a group.  Batched problems keep one
    // group and maximise the filled fraction of the wavefronts.  With `groups`
    // the blocks may be cut into up to 4 groups, one workgroup each (the rows are
    // then read once per group, the later reads mostly from L2), and the score is
    // the useful fraction of a CU's wavefront slots: the double-double kernel's
    // registers allow three wavefronts per SIMD, twelve per CU, and fewer than
    // three per SIMD do not hide the latency of its dependent additions.
    p.ng = 1;
    p.nblkg = p.nblk;
    p.ks = 1;
    double best = -1.0;
    for (int ng = 1; ng <= (groups ? 4 : 1); ++ng) {
        const int nblkg = (p.nblk + ng - 1) / ng;
        if (ng > 1 && nblkg * (ng - 1) >= p.nblk) break;  // an empty group
        for (int ks = 1; ks <= (groups ? 24 : 16) && ks * nblkg <= GRAM_MAX_THREADS; ++ks) {
            const int lanes = ks * nblkg;
            const int waves = (lanes + 63) / 64;
            const double score = groups ? (double)lanes / (64.0 * 12 * ((waves + 11) / 12)) - 0.01 * (ng - 1)
                                        : (double)lanes / (64.0 * waves);
            if (score >= best - 1e-9) {
                best = score;
                p.ng = ng;
                p.nblkg = nblkg;
                p.ks = ks;
            }
        }
    }
    p.threads = ((p.ks * p.nblkg + 63) / 64) * 64;
    int kk = 8;
    while (kk > 1 && p.ks * kk * BS * p.nb > MAXPER * p.threads) --kk;
    p.kc = p.ks * kk;
    int64_t target = 512;
    int64_t rps = slab_rows > 0 ? slab_rows : (m + target - 1) / target;
    rps = ((rps + p.kc - 1) / p.kc) * p.kc;
    if (rps < p.kc) rps = p.kc;
    p.rows_per_split = rps;
    p.nsplit = (m + rps - 1) / rps;
    if (p.nsplit < 1) p.nsplit = 1;
    const size_t chunk = (size_t)2 * p.kc * (BS * p.nb + 2) * sizeof(double);
    const size_t red = (size_t)p.nblkg * 32 * sizeof(double);
    p.lds_bytes = chunk > red ? chunk : red;
    p.part_bytes = (size_t)p.nsplit * p.nblk * 32 * sizeof(double);
    return p;
}

static bool plan_ok(const GramPlan &p) {
    return !(p.threads > GRAM_MAX_THREADS || (p.kc * BS * p.nb + p.threads - 1) / p.threads > MAXPER ||
             p.ks * p.nblkg > p.threads || p.ng < 1 || p.nblkg * p.ng < p.nblk ||
             p.lds_bytes > 160 * 1024);
}

hipError_t gram_launch(int working, int64_t m, int64_t n, const void *A, int64_t lda,
                       double *Mhi, double *Mlo, int64_t ldm, void *part, const GramPlan &p,
                       hipStream_t st) {
    if (!plan_ok(p)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(8 * p.ng * ((p.nsplit + 7) / 8)));
    hipError_t err;
    if (working == 1) {
        auto k = gram_partial_kernel<double, true>;
        err = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)p.lds_bytes);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k, grid, dim3(p.threads), p.lds_bytes, st, (const double *)A, lda, m,
                           (int)n, p.nb, p.nblk, p.ng, p.nblkg, p.ks, p.kc, p.rows_per_split,
                           p.nsplit, (double *)part);
    } else {
        auto k = gram_partial_kernel<float, false>;
        err = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)p.lds_bytes);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k, grid, dim3(p.threads), p.lds_bytes, st, (const float *)A, lda, m,
                           (int)n, p.nb, p.nblk, p.ng, p.nblkg, p.ks, p.kc, p.rows_per_split,
                           p.nsplit, (double *)part);
    }
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int64_t entries = (int64_t)p.nblk * BS * BS;
    const unsigned rgrid = (unsigned)((entries + 3) / 4);
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(rgrid), dim3(256), 0, st, (const double *)part,
                       p.nsplit, p.nb, p.nblk, (int)n, Mhi, Mlo, ldm);
    return hipGetLastError();
}

hipError_t gram_batched_launch(int working, const BatchMat *tab, const int *order, int first,
                               int count, int max_nsplit, const GramPlan &p, hipStream_t st) {
    if (!plan_ok(p) || count < 1 || count > 65535 || max_nsplit < 1 || max_nsplit > 65535)
        return hipErrorInvalidValue;
    const dim3 grid(1, (unsigned)max_nsplit, (unsigned)count);
    hipError_t err;
    if (working == 1) {
        auto k = gram_partial_batched_kernel<double, true>;
        err = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)p.lds_bytes);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k, grid, dim3(p.threads), p.lds_bytes, st, tab, order, first, p.nb,
                           p.nblk, p.ks, p.kc);
    } else {
        auto k = gram_partial_batched_kernel<float, false>;
        err = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)p.lds_bytes);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k, grid, dim3(p.threads), p.lds_bytes, st, tab, order, first, p.nb,
                           p.nblk, p.ks, p.kc);
    }
    return hipGetLastError();
}

hipError_t gram_reduce_batched_launch(const BatchMat *tab, int batch, int max_n, hipStream_t st) {
    if (batch < 1 || batch > 65535 || max_n < 1) return hipErrorInvalidValue;
    const int nb = (max_n + BS - 1) / BS;
    const int64_t entries = (int64_t)(nb * (nb + 1) / 2) * BS * BS;
    hipLaunchKernelGGL(gram_reduce_batched_kernel, dim3((unsigned)((entries + 3) / 4), (unsigned)batch),
                       dim3(256), 0, st, tab);
    return hipGetLastError();
}

}  // namespace gsvd

// Higher-precision Gram M_h = A^T A for wide panels, n > 128 (Alg. 1 steps 1-2,
// eq. (ATA)), plain form: dd sums of exact products for FP64 A, FP64 sums for
// FP32 A.
//
// The columns are cut into panels of 64.  A workgroup owns one panel pair
// (I, J), I <= J, and one slab of rows: it stages the slab's rows of both
// panels through LDS (chunks of 16 rows x 128 columns, row-major, the next
// chunk fetched into registers while the current one is used) and its 512
// lanes are 256 register blocks of 4 x 4 entries (block (bi, bj) covers rows
// 4 bi .. of panel I and columns 4 bj .. of panel J) times two k-groups that
// take alternate rows of each chunk.  A diagonal pair (I = J) computes its
// full square; the reduction keeps the upper triangle.  Each (slab, pair,
// block) writes its 16 dd sums to its own slot; gram_wide_reduce_kernel adds
// the slabs in a fixed order, so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include "dd_device.hpp"
#include "gsvd_internal.hpp"

namespace gsvd {

namespace {

constexpr int WP = 64;                   // panel width
constexpr int WB = 4;                    // register block edge
constexpr int WNB = WP / WB;             // blocks per panel side
constexpr int WKS = 2;                   // k-groups
constexpr int WTHR = WNB * WNB * WKS;    // 512 lanes
constexpr int WKC = 16;                  // rows per chunk
constexpr int WLDL = 2 * WP + 2;         // LDS row stride (doubles), 16-byte aligned rows
constexpr int WPER = WKC * 2 * WP / WTHR;  // staged values per lane (4)
constexpr int WLDS = WNB * WNB * 32;     // doubles: the k-group reduction (>= 2 chunks)
static_assert(2 * WKC * WLDL <= WLDS, "chunk buffers fit the reduction area");

__device__ __forceinline__ void wide_pair(int p, int np, int &I, int &J) {
    int i = 0, rem = p;
    while (rem >= np - i) {
        rem -= np - i;
        ++i;
    }
    I = i;
    J = i + rem;
}

template <typename T, bool DD>
__global__ void __launch_bounds__(WTHR)
gram_wide_kernel(const T *__restrict__ A, int64_t lda, int64_t m, int n, int np,
                 int64_t rows_per_split, double *__restrict__ part) {
    __shared__ __attribute__((aligned(32))) double lds[WLDS];
    double *buf0 = lds;
    double *buf1 = lds + WKC * WLDL;
    const int pair = blockIdx.x;
    const int64_t split = blockIdx.y;
    const int npair = gridDim.x;
    int I, J;
    wide_pair(pair, np, I, J);

    const int tid = threadIdx.x;
    const int g = tid / (WNB * WNB);
    const int b = tid - g * (WNB * WNB);
    const int bi = b / WNB, bj = b % WNB;

    const int64_t r0 = split * rows_per_split;
    const int64_t r1 = (r0 + rows_per_split < m) ? r0 + rows_per_split : m;
    const int nchunk = (int)((r1 - r0 + WKC - 1) / WKC);

    // staged element e = tid + q * WTHR: row k = e % WKC of the chunk, local
    // column c = e / WKC (0..63 panel I, 64..127 panel J)
    double stage[WPER];
    auto fetch = [&](int chunk) {
        const int64_t base = r0 + (int64_t)chunk * WKC;
#pragma unroll
        for (int q = 0; q < WPER; ++q) {
            const int e = tid + q * WTHR;
            const int k = e % WKC, c = e / WKC;
            const int col = c < WP ? WP * I + c : WP * J + (c - WP);
            const int64_t r = base + k;
            stage[q] = (r < r1 && col < n) ? (double)A[r + (int64_t)col * lda] : 0.0;
        }
    };
    auto commit = [&](double *dst) {
#pragma unroll
        for (int q = 0; q < WPER; ++q) {
            const int e = tid + q * WTHR;
            dst[(e % WKC) * WLDL + e / WKC] = stage[q];
        }
    };

    double hi[WB * WB], lo[WB * WB];
#pragma unroll
    for (int q = 0; q < WB * WB; ++q) {
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
        const double *pi = cur + WB * bi;
        const double *pj = cur + WP + WB * bj;
        for (int k = g; k < WKC; k += WKS) {
            const double2 a01 = *reinterpret_cast<const double2 *>(pi + k * WLDL);
            const double2 a23 = *reinterpret_cast<const double2 *>(pi + k * WLDL + 2);
            const double2 b01 = *reinterpret_cast<const double2 *>(pj + k * WLDL);
            const double2 b23 = *reinterpret_cast<const double2 *>(pj + k * WLDL + 2);
            const double av[WB] = {a01.x, a01.y, a23.x, a23.y};
            const double bv[WB] = {b01.x, b01.y, b23.x, b23.y};
            if (DD) {
                // per row of the block: four exact products, then four TwoSums
                // written stage by stage (independent operations four apart)
#pragma unroll
                for (int r = 0; r < WB; ++r) {
                    double p[WB], e[WB], s[WB], v[WB];
#pragma unroll
                    for (int c = 0; c < WB; ++c) p[c] = av[r] * bv[c];
#pragma unroll
                    for (int c = 0; c < WB; ++c) e[c] = __builtin_fma(av[r], bv[c], -p[c]);
#pragma unroll
                    for (int c = 0; c < WB; ++c) s[c] = hi[WB * r + c] + p[c];
#pragma unroll
                    for (int c = 0; c < WB; ++c) v[c] = s[c] - hi[WB * r + c];
#pragma unroll
                    for (int c = 0; c < WB; ++c) {
                        const int q = WB * r + c;
                        const double err = (hi[q] - (s[c] - v[c])) + (p[c] - v[c]);
                        hi[q] = s[c];
                        lo[q] += e[c] + err;
                    }
                }
            } else {
#pragma unroll
                for (int q = 0; q < WB * WB; ++q) hi[q] = __builtin_fma(av[q / WB], bv[q % WB], hi[q]);
            }
        }
        if (more) commit(nxt);
        __syncthreads();
    }

    // k-group 1 into k-group 0 through LDS (the chunk buffers are free now)
    if (g == 1) {
        double4 *dst = reinterpret_cast<double4 *>(lds + (size_t)b * 32);
#pragma unroll
        for (int q = 0; q < WB * WB; q += 2) dst[q / 2] = make_double4(hi[q], lo[q], hi[q + 1], lo[q + 1]);
    }
    __syncthreads();
    if (g == 0) {
        const double4 *src = reinterpret_cast<const double4 *>(lds + (size_t)b * 32);
        double4 *dst = reinterpret_cast<double4 *>(part + (((size_t)split * npair + pair) * (WNB * WNB) + b) * 32);
#pragma unroll
        for (int q = 0; q < WB * WB; q += 2) {
            const double4 o = src[q / 2];
            dd_t x, y;
            if (DD) {
                x = dd_add(dd_t{hi[q], lo[q]}, dd_t{o.x, o.y});
                y = dd_add(dd_t{hi[q + 1], lo[q + 1]}, dd_t{o.z, o.w});
            } else {
                x = dd_t{hi[q] + o.x, 0.0};
                y = dd_t{hi[q + 1] + o.z, 0.0};
            }
            dst[q / 2] = make_double4(x.hi, x.lo, y.hi, y.lo);
        }
    }
}

// One lane per entry of the pair blocks: the slabs are added in order; entries
// of the upper triangle are written to M(i, j) and M(j, i).
__global__ void __launch_bounds__(256)
gram_wide_reduce_kernel(const double *__restrict__ part, int64_t nsplit, int np, int npair, int n,
                        double *__restrict__ Mhi, double *__restrict__ Mlo, int64_t ldm) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per_pair = (int64_t)WNB * WNB * WB * WB;
    if (id >= (int64_t)npair * per_pair) return;
    const int pair = (int)(id / per_pair);
    const int rem = (int)(id % per_pair);
    const int b = rem / (WB * WB), e = rem % (WB * WB);
    int I, J;
    wide_pair(pair, np, I, J);
    const int i = WP * I + WB * (b / WNB) + e / WB;
    const int j = WP * J + WB * (b % WNB) + e % WB;
    if (i >= n || j >= n || i > j) return;
    dd_t acc{0.0, 0.0};
    const size_t stride = (size_t)npair * WNB * WNB * 32;
    const double *p = part + ((size_t)pair * (WNB * WNB) + b) * 32 + 2 * e;
    for (int64_t s = 0; s < nsplit; ++s) acc = dd_add(acc, dd_t{p[s * stride], p[s * stride + 1]});
    Mhi[i + (int64_t)j * ldm] = acc.hi;
    Mhi[j + (int64_t)i * ldm] = acc.hi;
    if (Mlo) {
        Mlo[i + (int64_t)j * ldm] = acc.lo;
        Mlo[j + (int64_t)i * ldm] = acc.lo;
    }
}

}  // namespace

WidePlan gram_wide_plan(int64_t m, int64_t n, int64_t slab_rows) {
    WidePlan p{};
    p.np = (int)((n + WP - 1) / WP);
    p.npair = p.np * (p.np + 1) / 2;
    // about 2048 workgroups in all, every slab a whole number of chunks
    int64_t rps = slab_rows;
    if (rps <= 0) {
        int64_t ns = (2048 + p.npair - 1) / p.npair;
        rps = (m + ns - 1) / ns;
    }
    rps = ((rps + WKC - 1) / WKC) * WKC;
    if (rps < WKC) rps = WKC;
    p.rows_per_split = rps;
    p.nsplit = (m + rps - 1) / rps;
    p.part_bytes = (size_t)p.nsplit * p.npair * WNB * WNB * 32 * sizeof(double);
    return p;
}

hipError_t gram_wide_launch(int working, int64_t m, int64_t n, const void *A, int64_t lda,
                            double *Mhi, double *Mlo, int64_t ldm, void *part, const WidePlan &p,
                            hipStream_t st) {
    if (p.npair < 1 || p.nsplit < 1 || p.nsplit > 65535 || n > GSVD_WIDE_MAX_N)
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)p.npair, (unsigned)p.nsplit);
    if (working == 1)
        hipLaunchKernelGGL((gram_wide_kernel<double, true>), grid, dim3(WTHR), 0, st,
                           (const double *)A, lda, m, (int)n, p.np, p.rows_per_split,
                           (double *)part);
    else
        hipLaunchKernelGGL((gram_wide_kernel<float, false>), grid, dim3(WTHR), 0, st,
                           (const float *)A, lda, m, (int)n, p.np, p.rows_per_split,
                           (double *)part);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int64_t entries = (int64_t)p.npair * WNB * WNB * WB * WB;
    hipLaunchKernelGGL(gram_wide_reduce_kernel, dim3((unsigned)((entries + 255) / 256)), dim3(256),
                       0, st, (const double *)part, p.nsplit, p.np, p.npair, (int)n, Mhi, Mlo, ldm);
    return hipGetLastError();
}

}  // namespace gsvd

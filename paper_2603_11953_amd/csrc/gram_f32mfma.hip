// Plain higher-precision Gram for FP32 A (Alg. 1 steps 1-2, eq. (ATA) with
// u_h = FP64) on the FP64 matrix cores, n <= 128.
//
// The product of two FP32 numbers is exact in FP64, so M_h = A^T A is a sum of
// exact FP64 products: v_mfma_f64_16x16x4f64 forms them and accumulates in
// FP64, which is the FP64-accumulated Gram the method asks for.  A workgroup
// owns a slab of rows; each 32-row chunk is converted to FP64 and staged in
// LDS column-major (the 32 rows of a column contiguous, 34 doubles apart, so
// the 16 x 2 lanes of an operand read hit distinct banks), two buffers with the
// next chunk fetched meanwhile.  The 16 x 16 tiles of the upper triangle are
// dealt to the 8 wavefronts (at most 5 each, one FP64 accumulator of 4
// registers per tile).  MFMA operand layout (16x16x4): lane l supplies
// A^T(i = l % 16, k = l / 16) and A(k = l / 16, j = l % 16), both the entry
// A(r0 + 4 s + l / 16, 16 b + l % 16) for the tile's block b; result register
// r of lane l is M(16 bi + 4 r + l / 16, 16 bj + l % 16).  Each (slab, tile)
// writes its partial sums to its own slot; the reduction adds the slabs in a
// fixed order (double-double), so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include "dd_device.hpp"
#include "gsvd_internal.hpp"

namespace gsvd {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int FM_KC = 32;           // rows per chunk
constexpr int FM_LDK = FM_KC + 2;   // LDS column stride (doubles)
constexpr int FM_THR = 512;         // 8 wavefronts
constexpr int FM_W = FM_THR / 64;
constexpr int FM_TPW = 5;           // tiles per wavefront at most (36 tiles / 8)
constexpr int FM_NMAX = 128;

__device__ __forceinline__ void fm_tile(int t, int nb, int &bi, int &bj) {
    int i = 0, rem = t;
    while (rem >= nb - i) {
        rem -= nb - i;
        ++i;
    }
    bi = i;
    bj = i + rem;
}

template <int NB>
__global__ void __launch_bounds__(FM_THR)
gram_f32mfma_kernel(const float *__restrict__ A, int64_t lda, int64_t m, int n,
                    int64_t rows_per_split, double *__restrict__ part) {
    constexpr int NC = 16 * NB;                   // staged columns
    constexpr int NT = NB * (NB + 1) / 2;         // tiles
    constexpr int NQ = FM_KC / 4 * NC;            // float4 loads per chunk (4 rows of a column)
    constexpr int QPT = (NQ + FM_THR - 1) / FM_THR;
    extern __shared__ __attribute__((aligned(16))) double fm_lds[];  // two chunks of NC x FM_LDK
    const int64_t split = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t r0 = split * rows_per_split;
    const int64_t r1 = (r0 + rows_per_split < m) ? r0 + rows_per_split : m;
    const int nchunk = (int)((r1 - r0 + FM_KC - 1) / FM_KC);

    // staging: unit q = 4 rows (4 k4 .. 4 k4 + 3) of column c, q = c * 8 + k4
    float4 st[QPT];
    auto fetch = [&](int ch) {
        const int64_t base = r0 + (int64_t)ch * FM_KC;
#pragma unroll
        for (int u = 0; u < QPT; ++u) {
            const int q = tid + u * FM_THR;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (q < NQ) {
                const int c = q / (FM_KC / 4), k4 = q % (FM_KC / 4);
                const int64_t r = base + 4 * k4;
                if (c < n) {
                    const float *p = A + r + (int64_t)c * lda;
                    if (r + 3 < r1 && (((uintptr_t)p) & 15) == 0) {
                        v = *reinterpret_cast<const float4 *>(p);
                    } else {
                        if (r < r1) v.x = p[0];
                        if (r + 1 < r1) v.y = p[1];
                        if (r + 2 < r1) v.z = p[2];
                        if (r + 3 < r1) v.w = p[3];
                    }
                }
            }
            st[u] = v;
        }
    };
    auto commit = [&](double *dst) {
#pragma unroll
        for (int u = 0; u < QPT; ++u) {
            const int q = tid + u * FM_THR;
            if (q < NQ) {
                const int c = q / (FM_KC / 4), k4 = q % (FM_KC / 4);
                double *d = dst + c * FM_LDK + 4 * k4;
                *reinterpret_cast<double2 *>(d) = make_double2(st[u].x, st[u].y);
                *reinterpret_cast<double2 *>(d + 2) = make_double2(st[u].z, st[u].w);
            }
        }
    };

    int tbi[FM_TPW], tbj[FM_TPW];
#pragma unroll
    for (int u = 0; u < FM_TPW; ++u) {
        const int t = wave + u * FM_W;
        tbi[u] = 0;
        tbj[u] = 0;
        if (t < NT) fm_tile(t, NB, tbi[u], tbj[u]);
    }
    f64x4 acc[FM_TPW];
#pragma unroll
    for (int u = 0; u < FM_TPW; ++u) acc[u] = f64x4{0.0, 0.0, 0.0, 0.0};

    const int li = lane & 15, lk = lane >> 4;
    if (nchunk > 0) {
        fetch(0);
        commit(fm_lds);
    }
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
        const double *cur = fm_lds + (ch & 1) * (NC * FM_LDK);
        const bool more = ch + 1 < nchunk;
        if (more) fetch(ch + 1);
#pragma unroll
        for (int s = 0; s < FM_KC / 4; ++s) {
#pragma unroll
            for (int u = 0; u < FM_TPW; ++u) {
                if (wave + u * FM_W < NT) {  // uniform per wavefront
                    const double a = cur[(16 * tbi[u] + li) * FM_LDK + 4 * s + lk];
                    const double b = cur[(16 * tbj[u] + li) * FM_LDK + 4 * s + lk];
                    acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
                }
            }
        }
        if (more) commit(fm_lds + ((ch + 1) & 1) * (NC * FM_LDK));
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < FM_TPW; ++u) {
        const int t = wave + u * FM_W;
        if (t < NT) {
            double *dst = part + (((size_t)split * NT + t) * 64 + lane) * 4;
            *reinterpret_cast<double4 *>(dst) = make_double4(acc[u][0], acc[u][1], acc[u][2], acc[u][3]);
        }
    }
}

// one lane per entry of the tiles: the slabs in order (double-double), upper
// triangle written to M(i, j) and M(j, i)
__global__ void __launch_bounds__(256)
gram_f32mfma_reduce_kernel(const double *__restrict__ part, int64_t nsplit, int nb, int n,
                           double *__restrict__ Mhi, double *__restrict__ Mlo, int64_t ldm) {
    const int nt = nb * (nb + 1) / 2;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)nt * 256) return;
    const int t = (int)(id / 256), rem = (int)(id % 256);
    const int lane = rem / 4, r = rem % 4;
    int bi, bj;
    fm_tile(t, nb, bi, bj);
    const int i = 16 * bi + 4 * r + (lane >> 4), j = 16 * bj + (lane & 15);
    if (i >= n || j >= n || i > j) return;
    dd_t s{0.0, 0.0};
    const size_t stride = (size_t)nt * 256;
    const double *p = part + ((size_t)t * 64 + lane) * 4 + r;
    for (int64_t k = 0; k < nsplit; ++k) s = dd_add(s, dd_t{p[k * stride], 0.0});
    Mhi[i + (int64_t)j * ldm] = s.hi;
    Mhi[j + (int64_t)i * ldm] = s.hi;
    if (Mlo) {
        Mlo[i + (int64_t)j * ldm] = s.lo;
        Mlo[j + (int64_t)i * ldm] = s.lo;
    }
}

template <int NB>
hipError_t fm_launch(int64_t m, int64_t n, const float *A, int64_t lda, void *part,
                     const F32MfmaPlan &p, hipStream_t st) {
    const size_t lds = (size_t)2 * 16 * NB * FM_LDK * sizeof(double);
    auto k = gram_f32mfma_kernel<NB>;
    hipError_t err = hipFuncSetAttribute((const void *)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3((unsigned)p.nsplit), dim3(FM_THR), lds, st, A, lda, m, (int)n,
                       p.rows_per_split, (double *)part);
    return hipGetLastError();
}

}  // namespace

F32MfmaPlan gram_f32mfma_plan(int64_t m, int64_t n, int64_t slab_rows) {
    F32MfmaPlan p{};
    p.nb = (int)((n + 15) / 16);
    const int nt = p.nb * (p.nb + 1) / 2;
    int64_t rps = slab_rows > 0 ? slab_rows : (m + 1023) / 1024;  // about 1024 slabs
    rps = ((rps + FM_KC - 1) / FM_KC) * FM_KC;
    if (rps < FM_KC) rps = FM_KC;
    p.rows_per_split = rps;
    p.nsplit = (m + rps - 1) / rps;
    p.part_bytes = (size_t)p.nsplit * nt * 256 * sizeof(double);
    return p;
}

hipError_t gram_f32mfma_launch(int64_t m, int64_t n, const float *A, int64_t lda, double *Mhi,
                               double *Mlo, int64_t ldm, void *part, const F32MfmaPlan &p,
                               hipStream_t st) {
    if (n < 1 || n > FM_NMAX || p.nsplit < 1 || p.nsplit > 0x7fffffff) return hipErrorInvalidValue;
    hipError_t err;
    switch (p.nb) {
        case 1: err = fm_launch<1>(m, n, A, lda, part, p, st); break;
        case 2: err = fm_launch<2>(m, n, A, lda, part, p, st); break;
        case 3: err = fm_launch<3>(m, n, A, lda, part, p, st); break;
        case 4: err = fm_launch<4>(m, n, A, lda, part, p, st); break;
        case 5: err = fm_launch<5>(m, n, A, lda, part, p, st); break;
        case 6: err = fm_launch<6>(m, n, A, lda, part, p, st); break;
        case 7: err = fm_launch<7>(m, n, A, lda, part, p, st); break;
        case 8: err = fm_launch<8>(m, n, A, lda, part, p, st); break;
        default: return hipErrorInvalidValue;
    }
    if (err != hipSuccess) return err;
    const int nt = p.nb * (p.nb + 1) / 2;
    hipLaunchKernelGGL(gram_f32mfma_reduce_kernel, dim3((unsigned)((nt * 256 + 255) / 256)),
                       dim3(256), 0, st, (const double *)part, p.nsplit, p.nb, (int)n, Mhi, Mlo,
                       ldm);
    return hipGetLastError();
}

}  // namespace gsvd

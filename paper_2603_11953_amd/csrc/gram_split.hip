// Operand-split Gram: slab plan, partial-sum reduction and the dispatch to the
// per-type kernel instances (gram_split_f64.hip, gram_split_f32.hip); the
// kernels themselves are in gram_split.hpp.
#include <hip/hip_runtime.h>

#include "dd_device.hpp"
#include "gram_split.hpp"
#include "gsvd_internal.hpp"

namespace gsvd {

// One wavefront per M entry of the tile layout; splits added as in the plain form.
__device__ __forceinline__ void gram_split_reduce_body(const double *__restrict__ part,
                                                       int64_t nsplit, int nb, int npair, int n,
                                                       double *__restrict__ Mhi,
                                                       double *__restrict__ Mlo, int64_t ldm) {
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


__global__ void __launch_bounds__(256)
gram_split_reduce_kernel(const double *__restrict__ part, int64_t nsplit, int nb, int npair, int n,
                         double *__restrict__ Mhi, double *__restrict__ Mlo, int64_t ldm) {
    gram_split_reduce_body(part, nsplit, nb, npair, n, Mhi, Mlo, ldm);
}

// Batched: blockIdx.y is the problem; blocks past its entries return at once.
__global__ void __launch_bounds__(256)
gram_split_reduce_batched_kernel(const BatchMat *__restrict__ tab) {
    const BatchMat &d = tab[blockIdx.y];
    const int nb = (d.n + 15) / 16;
    gram_split_reduce_body(d.part, d.nsplit, nb, nb * (nb + 1) / 2, d.n, d.Mhi, d.Mlo, d.n);
}

SplitPlan split_plan(int64_t m, int64_t n, int S, int64_t slab_rows) {
    SplitPlan p{};
    p.S = S;
    p.nb = (int)((n + 15) / 16);
    p.npair = p.nb * (p.nb + 1) / 2;
    int64_t target = 1024;  // slabs: four workgroups per compute unit
    int64_t rps = slab_rows > 0 ? slab_rows : (m + target - 1) / target;
    rps = ((rps + SP_KT - 1) / SP_KT) * SP_KT;
    if (rps < SP_KT) rps = SP_KT;
    p.rows_per_split = rps;
    p.nsplit = (m + rps - 1) / rps;
    p.lds_bytes = (size_t)sp_lds(p.nb, S);
    p.part_bytes = (size_t)p.nsplit * p.npair * 64 * 8 * sizeof(double);
    return p;
}

int split_max_slices(int working) { return working == 1 ? SplitMax<double>::S : SplitMax<float>::S; }

hipError_t split_launch(int working, int64_t m, int64_t n, const void *A, int64_t lda, double *Mhi,
                        double *Mlo, int64_t ldm, void *part, const SplitPlan &p, hipStream_t st) {
    if (p.S < 1 || p.S > split_max_slices(working) || p.nb < 1 || p.nb > 8)
        return hipErrorInvalidValue;
    hipError_t err = working == 1 ? split_partial_f64(m, n, (const double *)A, lda, part, p, st)
                                  : split_partial_f32(m, n, (const float *)A, lda, part, p, st);
    if (err != hipSuccess) return err;
    const int64_t entries = (int64_t)p.npair * 256;
    hipLaunchKernelGGL(gram_split_reduce_kernel, dim3((unsigned)((entries + 3) / 4)), dim3(256), 0,
                       st, (const double *)part, p.nsplit, p.nb, p.npair, (int)n, Mhi, Mlo, ldm);
    return hipGetLastError();
}

hipError_t split_batched_launch(int working, const BatchMat *tab, const int *order, int first,
                                int count, int max_nsplit, const SplitPlan &p, hipStream_t st) {
    if (p.S < 1 || p.S > split_max_slices(working) || p.nb < 1 || p.nb > 8 || count < 1 ||
        count > 65535 || max_nsplit < 1 || max_nsplit > 65535)
        return hipErrorInvalidValue;
    if (working == 1) return split_batched_f64(tab, order, first, count, max_nsplit, p, st);
    return split_batched_f32(tab, order, first, count, max_nsplit, p, st);
}

hipError_t split_reduce_batched_launch(const BatchMat *tab, int batch, int max_n, hipStream_t st) {
    if (batch < 1 || batch > 65535 || max_n < 1) return hipErrorInvalidValue;
    const int nb = (max_n + 15) / 16;
    const int64_t entries = (int64_t)(nb * (nb + 1) / 2) * 256;
    hipLaunchKernelGGL(gram_split_reduce_batched_kernel,
                       dim3((unsigned)((entries + 3) / 4), (unsigned)batch), dim3(256), 0, st, tab);
    return hipGetLastError();
}

}  // namespace gsvd

// Operand-split Gram for n > 128 (the split form of Alg. 1 steps 1-2 on wide
// panels): the same balanced base-256 digits and exact int8 matrix-core sums as
// the one-workgroup split kernels, organised for many column panels.
//
// Slicing once, multiplying many times.  Cutting an entry into digits costs
// far more vector work than the products of one 16 x 16 tile, and with n up to
// 512 a workgroup that sliced the columns it needs would repeat that work for
// every panel pair.  So the rows are processed in passes of up to about 1 GiB
// of digit planes:
//   slice  one wavefront per (column, 2048-row slab), the slab's column in its
//          registers (A is read once): the exact maximum gives
//          E_j = ilogb(max) + 4 (so |a| < 2^(E_j - 3)), then every entry is
//          written as SS int8 digit planes, plane-major, 64 bytes per (chunk of
//          64 rows, column);
//   syrk   one workgroup per (64-column panel pair I <= J, group of 4 slabs),
//          the pairs of a group on one XCD (they read the same planes): 16
//          wavefronts, one 16 x 16 tile each (a diagonal pair uses the upper
//          ten), load the chunk's planes of both panels straight into LDS (the
//          next chunk's loads in flight meanwhile) and accumulate the digit-pair
//          products with v_mfma_i32_16x16x64_i8 in int32; at each slab end the
//          sums are combined exactly into double-double (FP64 A) or FP64 (FP32
//          A) with the slab's exponents, and at the end of the group added to
//          the workgroup's slot (written by the first pass, added to by later
//          ones, always in the same order);
//   reduce the slots of all groups, in order, into M_h (both triangles).
// A NaN or Inf entry cannot be cut into digits: the slice kernel treats it as
// zero and raises a flag in the workspace (cleared at the start of the call);
// the reduction then writes NaN to every entry of M_h, so the eigensolver
// reports non-finite input.
// The int32 sums never exceed 128 chunks x 64 rows x 12 pairs x 128^2 < 2^31.
#include <hip/hip_runtime.h>

#include "dd_device.hpp"
#include "gram_split.hpp"
#include "gsvd_internal.hpp"

namespace gsvd {

namespace {

constexpr int SW_P = 64;                // panel width
constexpr int SW_SR = 2048;             // rows per exponent slab (32 chunks)
constexpr int SW_G = 4;                 // slabs per syrk workgroup
constexpr int SW_RW = SW_SR * SW_G;     // rows per syrk workgroup (128 chunks)
constexpr int SW_CPS = SW_SR / SP_KT;   // chunks per slab
constexpr int SW_THR = 1024;
constexpr int64_t SW_PASS_BYTES = (int64_t)1 << 30;  // digit planes per pass (target)

__device__ __forceinline__ void sw_pair(int p, int np, int &I, int &J) {
    int i = 0, rem = p;
    while (rem >= np - i) {
        rem -= np - i;
        ++i;
    }
    I = i;
    J = i + rem;
}

// grid (npad / 64, slabs of the pass); 4 wavefronts
__global__ void __launch_bounds__(64) sw_flag_clear_kernel(int *__restrict__ flag) {
    if (threadIdx.x == 0) *flag = 0;
}

// |a| of a finite entry, 0 for NaN or Inf (which sets *bad)
__device__ __forceinline__ double sw_finite_abs(double a, bool &bad) {
    const double x = __builtin_fabs(a);
    const bool fin = x <= 1.7976931348623157e308;  // false for NaN and Inf
    bad = bad || !fin;
    return fin ? x : 0.0;
}

// grid (npad / 4, slabs of the pass); 4 wavefronts, one column of the slab each.
// Lane l holds rows 4 (l % 16) .. + 3 of chunks l / 16, 4 + l / 16, ... of the
// slab: the column's 2048 rows sit in registers, so A is read once for both the
// exact maximum and the digits.
template <typename T, int SS>
__global__ void __launch_bounds__(256)
sw_slice_kernel(const T *__restrict__ A, int64_t lda, int64_t m, int n, int npad, int64_t row0,
                int nchp, signed char *__restrict__ planes, int *__restrict__ expo,
                int *__restrict__ nonfinite) {
    constexpr int IT = SW_SR / 256;  // chunk quadruples of a slab
    const int lane = threadIdx.x & 63;
    const int c = 4 * blockIdx.x + (threadIdx.x >> 6);  // < npad
    const int sl = blockIdx.y;
    const int64_t r0 = row0 + (int64_t)sl * SW_SR;
    const int64_t r1 = (r0 + SW_SR < m) ? r0 + SW_SR : m;
    const int prow = 4 * (lane & 15);
    const T *col = A + (int64_t)c * lda;
    bool bad = false;
    double v[IT][4];
    double mx = 0.0;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t r = r0 + 256 * it + 64 * (lane >> 4) + prow + q;
            const double x = (c < n && r < r1) ? (double)col[r] : 0.0;
            // a NaN or Inf entry counts as zero (the flag is set below)
            const double ax = sw_finite_abs(x, bad);
            v[it][q] = ax == 0.0 ? 0.0 : x;
            mx = fmax(mx, ax);
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    const int E = need_exp(mx);
    if (lane == 0) expo[(int64_t)sl * npad + c] = E;
    if (bad) *nonfinite = 1;
    constexpr int NW3 = (SS + 3) / 4;
    const int64_t plane_stride = (int64_t)nchp * npad * SP_KT;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        unsigned wd[3][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (E > SP_NOEXP) {
                balanced96<NW3>(v[it][q], E, wd[0][q], wd[1][q], wd[2][q]);
            } else {  // an all-zero column: zero digits
                wd[0][q] = 0u;
                wd[1][q] = 0u;
                wd[2][q] = 0u;
            }
        }
        const int chl = sl * SW_CPS + 4 * it + (lane >> 4);  // chunk within the pass
        signed char *pd = planes + ((int64_t)chl * npad + c) * SP_KT + prow;
#pragma unroll
        for (int kw = 0; kw < NW3; ++kw) {
            unsigned o[4];
            transpose4(wd[kw][0], wd[kw][1], wd[kw][2], wd[kw][3], o[0], o[1], o[2], o[3]);
            // word kw holds digits 4 kw + 1 (top byte) .. 4 kw + 4 (low byte)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = 4 * kw + (3 - j);
                if (r < SS) *reinterpret_cast<unsigned *>(pd + r * plane_stride) = o[j];
            }
        }
    }
}

// LDS layout of one plane of a chunk: 128 columns (64 of panel I, then 64 of
// panel J) of 64 bytes; the four 16-byte parts of column k are stored in the
// order part ^ ((k >> 2) & 3), so that the 16 lanes of an operand read (16
// consecutive columns, one part) hit 16 distinct groups of four banks.
__device__ __forceinline__ int sw_part(int k, int part) { return part ^ ((k >> 2) & 3); }

// grid 8 x ceil(npair groups / 8) (the order below); 16 wavefronts, one tile each.  The planes
// of a chunk move from global memory straight into LDS (global_load_lds, 16
// bytes per lane, no staging registers), two buffers when they fit.
template <int SS, bool DD>
__global__ void __launch_bounds__(SW_THR)
sw_syrk_kernel(const signed char *__restrict__ planes, const int *__restrict__ expo, int npad,
               int np, int npair, int groups, int nchp, int nch_valid, int first,
               double *__restrict__ slots) {
    extern __shared__ __attribute__((aligned(16))) unsigned char swsm[];
    constexpr int PL = 2 * SW_P * SP_KT;             // LDS bytes per plane (8 KiB)
    constexpr int BUFB = SS * PL;                    // one chunk
    constexpr int NBUF = 2 * BUFB <= 160 * 1024 ? 2 : 1;
    constexpr int NLD = SS * 8;                      // 1 KiB wavefront loads per chunk
    // Workgroup b runs on XCD b % 8.  The (group, pair) items are taken in group-major
    // order and XCD x works through the x-th eighth of that order, so the pairs that
    // read one group's planes share an L2.
    const int per = (int)(((int64_t)groups * npair + 7) / 8);
    const int item = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (item >= groups * npair) return;
    const int grp = item / npair, pair = item % npair;
    int I, J;
    sw_pair(pair, np, I, J);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int a = wave >> 2, b = wave & 3;
    const bool has_tile = I != J || a <= b;
    const int ch0 = grp * (SW_RW / SP_KT);
    const int ch1 = (ch0 + SW_RW / SP_KT < nch_valid) ? ch0 + SW_RW / SP_KT : nch_valid;
    const int64_t plane_stride = (int64_t)nchp * npad * SP_KT;

    // load i of a chunk: plane i / 8, columns 16 (i % 8) .. + 15; lane L takes
    // LDS bytes 16 L .. of that 1 KiB, i.e. column 16 (i % 8) + L / 4, stored part L % 4
    const int llc = lane >> 2, lpart = lane & 3;
    auto issue = [&](int ch, int bf) {
        for (int i = wave; i < NLD; i += SW_THR / 64) {
            const int d = i >> 3, c8 = i & 7;
            const int lc = 16 * c8 + llc;
            const int gc = lc < SW_P ? SW_P * I + lc : SW_P * J + (lc - SW_P);
            const signed char *src = planes + d * plane_stride + ((int64_t)ch * npad + gc) * SP_KT +
                                     16 * sw_part(lc, lpart);
            __builtin_amdgcn_global_load_lds(
                (const void *)src,
                (__attribute__((address_space(3))) void *)(swsm + bf * BUFB + d * PL + c8 * 1024),
                16, 0, 0);
        }
    };

    const int ca = 16 * a + (lane & 15), cb = SW_P + 16 * b + (lane & 15);
    const int offa = ca * SP_KT + 16 * sw_part(ca, lane >> 4);
    const int offb = cb * SP_KT + 16 * sw_part(cb, lane >> 4);
    const int gi0 = SW_P * I + 16 * a + 4 * (lane >> 4);  // + q: row of result register q
    const int gj = SW_P * J + 16 * b + (lane & 15);
    v4i diag[SS];
#pragma unroll
    for (int s = 0; s < SS; ++s) diag[s] = v4i{0, 0, 0, 0};
    dd_t acc[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};

    // add the slab's integer sums, scaled by 2^(E_i + E_j), to acc (exact Horner
    // groups as in the one-workgroup split kernels)
    auto flush = [&](int slab) {
        const int *ex = expo + (int64_t)slab * npad;
        const int ej = ex[gj];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int ei = ex[gi0 + q];
            if (ei > SP_NOEXP && ej > SP_NOEXP) {
                dd_t tot{0.0, 0.0};
                if (DD) {
#pragma unroll
                    for (int g0 = 0; g0 < SS; g0 += 3) {
                        double v = 0.0;
#pragma unroll
                        for (int u = 2; u >= 0; --u)
                            if (g0 + u < SS) v = v * 0x1p-8 + (double)diag[g0 + u][q];
                        tot = dd_add(tot, dd_t{ldexp(v, -8 * (g0 + 2)), 0.0});
                    }
                    tot.hi = ldexp(tot.hi, ei + ej);
                    tot.lo = ldexp(tot.lo, ei + ej);
                    acc[q] = dd_add(acc[q], tot);
                } else {
                    double v = 0.0;
#pragma unroll
                    for (int s0 = SS - 1; s0 >= 0; --s0) v = v * 0x1p-8 + (double)diag[s0][q];
                    acc[q].hi += ldexp(v, ei + ej - 16);
                }
            }
        }
#pragma unroll
        for (int s = 0; s < SS; ++s) diag[s] = v4i{0, 0, 0, 0};
    };
    auto compute = [&](int bf) {
        const unsigned char *base = swsm + bf * BUFB;
        constexpr int HB = SS < 6 ? SS : 6;  // B-operand planes held in registers
        v4i bop[HB];
#pragma unroll
        for (int t = 0; t < HB; ++t) bop[t] = *reinterpret_cast<const v4i *>(base + t * PL + offb);
#pragma unroll
        for (int r = 0; r < SS; ++r) {
            const v4i aop = *reinterpret_cast<const v4i *>(base + r * PL + offa);
#pragma unroll
            for (int t = 0; t < SS - r; ++t) {
                const v4i bt = t < HB ? bop[t < HB ? t : 0]
                                      : *reinterpret_cast<const v4i *>(base + t * PL + offb);
                diag[r + t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(aop, bt, diag[r + t], 0, 0, 0);
            }
        }
    };

    if (NBUF == 2) {
        if (ch0 < ch1) issue(ch0, 0);
        for (int ch = ch0; ch < ch1; ++ch) {
            const int bf = (ch - ch0) & 1;
            __builtin_amdgcn_s_waitcnt(0);  // this wavefront's loads of chunk ch are in LDS
            __syncthreads();                // everyone's, and chunk ch - 1 is consumed
            if (ch + 1 < ch1) issue(ch + 1, bf ^ 1);
            if (has_tile) {
                compute(bf);
                if ((ch + 1) % SW_CPS == 0 || ch + 1 == ch1) flush(ch / SW_CPS);
            }
        }
    } else {
        for (int ch = ch0; ch < ch1; ++ch) {
            __syncthreads();  // chunk ch - 1 is consumed
            issue(ch, 0);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (has_tile) {
                compute(0);
                if ((ch + 1) % SW_CPS == 0 || ch + 1 == ch1) flush(ch / SW_CPS);
            }
        }
    }
    if (has_tile) {
        double *dst = slots + (((size_t)grp * npair + pair) * 16 + wave) * 64 * 8 + lane * 8;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            dd_t v = acc[q];
            if (!first) v = dd_add(v, dd_t{dst[2 * q], dst[2 * q + 1]});
            dst[2 * q] = v.hi;
            dst[2 * q + 1] = v.lo;
        }
    }
}

// one lane per (pair, tile, lane, q) entry: the groups in order; upper triangle to both halves
__global__ void __launch_bounds__(256)
sw_reduce_kernel(const double *__restrict__ slots, int groups, int np, int npair, int n,
                 double *__restrict__ Mhi, double *__restrict__ Mlo, int64_t ldm,
                 const int *__restrict__ nonfinite) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per_pair = 16 * 64 * 4;
    if (id >= (int64_t)npair * per_pair) return;
    const int pair = (int)(id / per_pair);
    const int rem = (int)(id % per_pair);
    const int w = rem / 256, lane = (rem / 4) % 64, q = rem % 4;
    int I, J;
    sw_pair(pair, np, I, J);
    const int a = w >> 2, b = w & 3;
    if (I == J && a > b) return;
    const int i = SW_P * I + 16 * a + 4 * (lane >> 4) + q;
    const int j = SW_P * J + 16 * b + (lane & 15);
    if (i >= n || j >= n || i > j) return;
    dd_t s{0.0, 0.0};
    const size_t stride = (size_t)npair * 16 * 64 * 8;
    const double *p = slots + (((size_t)pair * 16 + w) * 64 + lane) * 8 + 2 * q;
    for (int g = 0; g < groups; ++g) s = dd_add(s, dd_t{p[g * stride], p[g * stride + 1]});
    if (*nonfinite) s = dd_t{__builtin_nan(""), __builtin_nan("")};
    Mhi[i + (int64_t)j * ldm] = s.hi;
    Mhi[j + (int64_t)i * ldm] = s.hi;
    if (Mlo) {
        Mlo[i + (int64_t)j * ldm] = s.lo;
        Mlo[j + (int64_t)i * ldm] = s.lo;
    }
}

template <typename T, int SS>
hipError_t sw_run(int64_t m, int64_t n, const T *A, int64_t lda, double *Mhi, double *Mlo,
                  int64_t ldm, char *work, const SplitWidePlan &p, hipStream_t st) {
    constexpr bool DD = sizeof(T) == 8;
    signed char *planes = reinterpret_cast<signed char *>(work + p.plane_off);
    int *expo = reinterpret_cast<int *>(work + p.expo_off);
    double *slots = reinterpret_cast<double *>(work + p.slot_off);
    int *nonfinite = reinterpret_cast<int *>(work + p.flag_off);
    const size_t buf = (size_t)SS * 2 * SW_P * SP_KT;
    const size_t lds = 2 * buf <= 160 * 1024 ? 2 * buf : buf;
    auto ks = sw_syrk_kernel<SS, DD>;
    hipError_t err = hipFuncSetAttribute((const void *)ks,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    const int nchp = (int)(p.rows_per_pass / SP_KT);
    hipLaunchKernelGGL(sw_flag_clear_kernel, dim3(1), dim3(64), 0, st, nonfinite);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    for (int64_t ps = 0; ps < p.npass; ++ps) {
        const int64_t row0 = ps * p.rows_per_pass;
        const int64_t rows = (m - row0 < p.rows_per_pass) ? m - row0 : p.rows_per_pass;
        const unsigned slabs = (unsigned)((rows + SW_SR - 1) / SW_SR);
        const unsigned groups = (unsigned)((rows + SW_RW - 1) / SW_RW);
        hipLaunchKernelGGL((sw_slice_kernel<T, SS>), dim3((unsigned)(p.npad / 4), slabs), dim3(256),
                           0, st, A, lda, m, (int)n, p.npad, row0, nchp, planes, expo, nonfinite);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        const unsigned items = (unsigned)p.npair * groups;
        hipLaunchKernelGGL(ks, dim3(8 * ((items + 7) / 8)), dim3(SW_THR), lds, st, planes, expo,
                           p.npad, p.np, p.npair, (int)groups, nchp,
                           (int)((rows + SP_KT - 1) / SP_KT), ps == 0 ? 1 : 0, slots);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    const int64_t entries = (int64_t)p.npair * 16 * 64 * 4;
    hipLaunchKernelGGL(sw_reduce_kernel, dim3((unsigned)((entries + 255) / 256)), dim3(256), 0, st,
                       slots, (int)p.groups_per_pass, p.np, p.npair, (int)n, Mhi, Mlo, ldm,
                       nonfinite);
    return hipGetLastError();
}

#define SW_CASE(S_)                                                                        \
    case S_:                                                                               \
        return sw_run<T, (S_ <= SplitMax<T>::S ? S_ : SplitMax<T>::S)>(m, n, A, lda, Mhi,  \
                                                                        Mlo, ldm, work, p, st);

template <typename T>
hipError_t sw_typed(int64_t m, int64_t n, const T *A, int64_t lda, double *Mhi, double *Mlo,
                    int64_t ldm, char *work, const SplitWidePlan &p, hipStream_t st) {
    if (p.S < 1 || p.S > SplitMax<T>::S) return hipErrorInvalidValue;
    switch (p.S) {
        SW_CASE(1) SW_CASE(2) SW_CASE(3) SW_CASE(4) SW_CASE(5) SW_CASE(6)
        SW_CASE(7) SW_CASE(8) SW_CASE(9) SW_CASE(10) SW_CASE(11) SW_CASE(12)
        default: return hipErrorInvalidValue;
    }
}
#undef SW_CASE

size_t sw_al(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

SplitWidePlan split_wide_plan(int64_t m, int64_t n, int S, int64_t rows_cap) {
    SplitWidePlan p{};
    p.S = S;
    p.np = (int)((n + SW_P - 1) / SW_P);
    p.npair = p.np * (p.np + 1) / 2;
    p.npad = p.np * SW_P;
    const int64_t per_row = (int64_t)(S > 0 ? S : 1) * p.npad;  // plane bytes per row
    int64_t g = SW_PASS_BYTES / per_row / SW_RW;
    if (rows_cap > 0 && rows_cap / SW_RW < g) g = rows_cap / SW_RW;
    if (g < 1) g = 1;
    const int64_t need = (m + SW_RW - 1) / SW_RW;
    if (g > need) g = need;
    p.groups_per_pass = g;
    p.rows_per_pass = g * SW_RW;
    p.npass = (m + p.rows_per_pass - 1) / p.rows_per_pass;
    size_t off = 0;
    p.plane_off = off;
    off = sw_al(off + (size_t)S * (size_t)p.rows_per_pass * (size_t)p.npad);
    p.expo_off = off;
    off = sw_al(off + (size_t)(p.rows_per_pass / SW_SR) * p.npad * sizeof(int));
    p.slot_off = off;
    off = sw_al(off + (size_t)g * p.npair * 16 * 64 * 8 * sizeof(double));
    p.flag_off = off;
    off = sw_al(off + sizeof(int));
    p.part_bytes = off;
    return p;
}

hipError_t split_wide_launch(int working, int64_t m, int64_t n, const void *A, int64_t lda,
                             double *Mhi, double *Mlo, int64_t ldm, void *work,
                             const SplitWidePlan &p, hipStream_t st) {
    if (n > GSVD_WIDE_MAX_N || p.npass < 1 || p.groups_per_pass > 65535 || p.npair > 65535)
        return hipErrorInvalidValue;
    if (working == 1)
        return sw_typed<double>(m, n, (const double *)A, lda, Mhi, Mlo, ldm, (char *)work, p, st);
    return sw_typed<float>(m, n, (const float *)A, lda, Mhi, Mlo, ldm, (char *)work, p, st);
}

}  // namespace gsvd

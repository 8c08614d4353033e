// Gram M_h = A^T A by exact operand splitting on the int8 matrix cores
// (the "split" form of Alg. 1 steps 1-2).
//
// A workgroup owns a slab of rows and keeps, per column j, an exponent E_j
// with |a_kj| < 2^(E_j - 1) for every row seen so far.  Each entry is written
// as a signed 128-bit fixed-point number F = a 2^(128 - E_j) (|F| < 2^127) and
// cut into base-128 digits of F's two's-complement form,
//     a = 2^E_j sum_{r=1..S} d_r 2^(-7 r) + tail,  d_1 in [-64, 63], d_r in [0, 127] (r > 1),
// 0 <= tail < 2^(E_j - 7 S).  Digit r sits at bits 128 - 7 r .. 134 - 7 r of F
// whatever S is, so each digit is one bitfield extract.  The contribution of
// the rows to M(i, j) is
//     2^(E_i + E_j) sum_{s=2..S+1} 2^(-7 s) I_s,   I_s = sum_{r+t=s} sum_k d_r,ki d_t,kj,
// keeping the slice pairs r + t <= S + 1 (the dropped pairs are below the last
// kept digit).  The I_s are exact integers accumulated by
// v_mfma_i32_16x16x64_i8 in int32 registers across chunks of 64 rows.
//
// The integer sums stay in registers until an exponent has to grow (a chunk
// holds an entry >= 2^(E_j - 1)), until 128 chunks have been added (the int32
// bound: 128 chunks x 64 rows x at most 16 pairs x 127^2 < 2^31), or until the
// slab ends.  Then
// they are "flushed": combined exactly (Horner over groups of four diagonals,
// each group exact in FP64) into double-double (FP64 A) or FP64 (FP32 A), and
// added to the workgroup's own slot of the partial-sum buffer.  A new exponent
// is set two bits above what the chunk needs, so flushes are rare.
//
// Layout: the chunk's digits sit in LDS as int8 planes, column-major (the 64
// rows of a column are 64 contiguous bytes, columns 80 bytes apart).  A 16x16
// tile (I, J) of M takes
// its A operand from columns 16 I .. 16 I + 15 and its B operand from columns
// 16 J .. 16 J + 15: lane l reads the 16 bytes of rows 16 (l / 16) .. + 15 of
// column 16 I + l % 16 (resp. 16 J + l % 16); the integer result gives lane l,
// register q the entry (4 (l / 16) + q, l % 16).  Each wavefront owns one tile
// I <= J of the upper triangle.
//
// The slab / partial / fixed-order reduction structure is the one of the plain
// form, so the result is reproducible bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include "dd_device.hpp"
#include "gsvd_internal.hpp"

namespace gsvd {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int SP_KT = 64;           // rows per chunk (one MFMA k-depth)
// byte stride of a column in a digit plane: 64 digits plus 16 bytes of padding,
// so the 16 lanes of an operand read (16 columns, 16 bytes each) fall into
// 16 distinct groups of 4 banks
constexpr int SP_CS = SP_KT + 16;
constexpr int SP_FLUSH_EVERY = 128;  // chunks between forced flushes (int32 bound)
constexpr int SP_HEAD = 2;          // extra exponent bits when an exponent is (re)set
constexpr int SP_NOEXP = -100000;   // exponent of a column not seen non-zero yet

template <typename T>
struct SplitMax {
    static constexpr int S = sizeof(T) == 8 ? 12 : 8;
};

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

// exponent needed by a: the smallest e with |a| < 2^(e - 1); SP_NOEXP for a = 0
__device__ __forceinline__ int need_exp(double a) { return a != 0.0 ? ilogb(a) + 2 : SP_NOEXP; }

// F = a 2^(128 - E) truncated toward minus infinity, as two's complement (hi, lo)
__device__ __forceinline__ void fixed128(double a, int E, unsigned long long &hi,
                                         unsigned long long &lo) {
    const unsigned long long bits = (unsigned long long)__double_as_longlong(a);
    const int ea = (int)((bits >> 52) & 0x7ff);
    unsigned long long mant = bits & 0xfffffffffffffull;
    if (ea != 0) mant |= 1ull << 52;
    // |a| = mant 2^(max(ea, 1) - 1075); |F| = mant 2^sh
    const int sh = (ea != 0 ? ea : 1) - 1075 + 128 - E;
    unsigned long long h = 0, l = 0;
    if (mant != 0 && sh > -53) {
        if (sh >= 64) {
            h = mant << (sh - 64);
        } else if (sh > 0) {
            l = mant << sh;
            h = mant >> (64 - sh);
        } else {
            l = mant >> (-sh);
        }
    }
    if (bits >> 63) {  // negate the 128-bit value
        h = ~h;
        l = ~l;
        l += 1;
        if (l == 0) h += 1;
    }
    hi = h;
    lo = l;
}

// digit r (1-based) of F: bits 128 - 7 r .. 134 - 7 r, the first one signed
template <int R>
__device__ __forceinline__ int digit(unsigned long long hi, unsigned long long lo) {
    constexpr int p = 128 - 7 * R;  // lowest bit of the digit
    if (R == 1) return (int)((long long)hi >> 57);
    if (p >= 64) return (int)((hi >> (p - 64)) & 127ull);
    if (p + 7 <= 64) return (int)((lo >> p) & 127ull);
    return (int)(((lo >> p) | (hi << (64 - p))) & 127ull);
}

template <int R>
__device__ __forceinline__ unsigned pack4(const unsigned long long *hi, const unsigned long long *lo) {
    unsigned w = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) w |= ((unsigned)digit<R>(hi[q], lo[q]) & 0xffu) << (8 * q);
    return w;
}

// Tiles of the upper triangle per workgroup: one per wavefront, at most 12
// wavefronts (three per SIMD, 168 registers each).  Larger triangles are dealt
// to several workgroups per slab, each slicing the whole chunk.
__host__ __device__ constexpr int sp_groups(int nb) { return (nb * (nb + 1) / 2 + 11) / 12; }
__host__ __device__ constexpr int sp_waves(int nb) {
    return (nb * (nb + 1) / 2 + sp_groups(nb) - 1) / sp_groups(nb);
}

// Producer wavefronts per workgroup: they load A, keep the column exponents and
// write the digit planes; the other wavefronts (one per tile) run the products.
constexpr int SP_PROD = 4;
constexpr int SP_LDS_MAX = 160 * 1024 - 1024;

__host__ __device__ constexpr int sp_threads(int nb) { return 64 * (sp_waves(nb) + SP_PROD); }

// bytes of one plane buffer (all slices of one chunk) plus its exponents
__host__ __device__ constexpr int sp_buf_bytes(int nb, int ss) {
    return ss * 16 * nb * SP_CS + 16 * nb * 4;
}
// two buffers (producers one chunk ahead of the consumers) when they fit LDS
__host__ __device__ constexpr int sp_bufs(int nb, int ss) {
    return 2 * sp_buf_bytes(nb, ss) + 64 <= SP_LDS_MAX ? 2 : 1;
}
__host__ __device__ constexpr int sp_lds(int nb, int ss) {
    return sp_bufs(nb, ss) * sp_buf_bytes(nb, ss) + 64;
}

// The partial Gram of slab `split` of one matrix, tiles of workgroup `grp`.
//
// Producers (the last SP_PROD wavefronts) take chunk i: lane l of producer
// wavefront w holds rows 4 (l % 16) .. + 3 of column 16 p + 4 w + l / 16 for
// every pass p, so the 16 lanes of a DPP row hold one column and agree on its
// exponent by a DPP max without any barrier.  A column whose exponent grows
// records the chunk in the buffer's flag (a monotone LDS maximum).  Consumers
// (one wavefront per tile) take chunk i - 1 from the other buffer: they flush
// their integer sums when the flag names that chunk (or every 128 chunks),
// reload their tile's exponents, and run the products.  One barrier per chunk.
// When two buffers do not fit LDS, producers and consumers alternate on one.
template <typename T, int NB, int SS>
__device__ __forceinline__ void gram_split_body(const T *__restrict__ A, int64_t lda, int64_t m,
                                                int n, int64_t rows_per_split, int64_t split,
                                                int grp, double *__restrict__ part) {
    constexpr bool DD = sizeof(T) == 8;
    constexpr int NW = sp_waves(NB);   // consumer wavefronts
    constexpr int N16 = 16 * NB;
    constexpr int NPAIR = NB * (NB + 1) / 2;
    constexpr int SL = N16 * SP_CS;    // bytes per digit plane
    constexpr int NBUF = sp_bufs(NB, SS);
    constexpr int BB = sp_buf_bytes(NB, SS);
    constexpr int NPASS = NB;          // producer passes of 16 columns
    constexpr bool PREF = NPASS * (int)sizeof(T) <= 32;  // next chunk held in registers
    extern __shared__ unsigned char smem[];
    int *flagc = reinterpret_cast<int *>(smem + NBUF * BB);  // [2]
    auto planes_of = [&](int b) { return reinterpret_cast<signed char *>(smem + b * BB); };
    auto expo_of = [&](int b) { return reinterpret_cast<int *>(smem + b * BB + SS * SL); };

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wavefront
    const bool producer = wave >= NW;
    const int64_t r0 = split * rows_per_split;
    const int64_t r1 = (r0 + rows_per_split < m) ? r0 + rows_per_split : m;
    const int nchunk = (int)((r1 - r0 + SP_KT - 1) / SP_KT);

    if (tid < 2) flagc[tid] = 0;
    __syncthreads();

    // ---------------- producer state
    const int pcol = 4 * (wave - NW) + (lane >> 4);  // + 16 p
    const int prow = 4 * (lane & 15);
    T cur[NPASS][4], nxt[PREF ? NPASS : 1][4];
    int er[NPASS];
#pragma unroll
    for (int p = 0; p < NPASS; ++p) er[p] = SP_NOEXP;
    auto fetch = [&](T (&v)[NPASS][4], int chunk) {
        const int64_t base = r0 + (int64_t)chunk * SP_KT + prow;
#pragma unroll
        for (int p = 0; p < NPASS; ++p) {
            const int c = 16 * p + pcol;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t r = base + q;
                v[p][q] = (c < n && r < r1) ? A[r + (int64_t)c * lda] : (T)0;
            }
        }
    };
    auto produce = [&](int i, int b) {
        if constexpr (PREF) {
            if (i == 0) fetch(cur, 0);
            if (i + 1 < nchunk) fetch(nxt, i + 1);
        } else {
            fetch(cur, i);
        }
        signed char *planes = planes_of(b);
        int *expo = expo_of(b);
#pragma unroll
        for (int p = 0; p < NPASS; ++p) {
            const int c = 16 * p + pcol;
            int e = SP_NOEXP;
#pragma unroll
            for (int q = 0; q < 4; ++q) e = max(e, need_exp((double)cur[p][q]));
            e = row_max_i(e);  // the 16 lanes of column c
            const bool grow = e > er[p];
            if (grow) er[p] = e + SP_HEAD;
            const int E = er[p];
            if ((lane & 15) == 0) {
                expo[c] = E;
                if (grow) atomicMax(&flagc[b], i + 1);
            }
            unsigned long long hi[4], lo[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) fixed128((double)cur[p][q], E, hi[q], lo[q]);
            signed char *pd = planes + c * SP_CS + prow;
#define GSVD_SPLIT_PLANE(R)                                                                  \
    if constexpr (R <= SS) *reinterpret_cast<unsigned *>(pd + (R - 1) * SL) = pack4<R>(hi, lo);
            GSVD_SPLIT_PLANE(1) GSVD_SPLIT_PLANE(2) GSVD_SPLIT_PLANE(3) GSVD_SPLIT_PLANE(4)
            GSVD_SPLIT_PLANE(5) GSVD_SPLIT_PLANE(6) GSVD_SPLIT_PLANE(7) GSVD_SPLIT_PLANE(8)
            GSVD_SPLIT_PLANE(9) GSVD_SPLIT_PLANE(10) GSVD_SPLIT_PLANE(11) GSVD_SPLIT_PLANE(12)
#undef GSVD_SPLIT_PLANE
        }
        if constexpr (PREF) {
#pragma unroll
            for (int p = 0; p < NPASS; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) cur[p][q] = nxt[p][q];
        }
    };

    // ---------------- consumer state: this wavefront's tile (I, J), I <= J
    const int pidx = grp * NW + wave;
    const bool has_tile = !producer && pidx < NPAIR;
    int bi = 0, bj = 0;
    if (has_tile) sp_decode_pair(pidx, NB, bi, bj);
    const int ca = 16 * bi + (lane & 15), cb = 16 * bj + (lane & 15);
    const int koff = 16 * (lane >> 4);
    int ei[4] = {SP_NOEXP, SP_NOEXP, SP_NOEXP, SP_NOEXP}, ej = SP_NOEXP;

    v4i diag[SS];
#pragma unroll
    for (int s = 0; s < SS; ++s) diag[s] = v4i{0, 0, 0, 0};

    // partial slot of this slab's tile: [split][tile][lane][q][hi, lo]
    double *dst = part + (((size_t)split * NPAIR + (has_tile ? pidx : 0)) * 64 + lane) * 8;
    // flush: add the integer sums (with the exponents in force) to the slot
    auto flush = [&](bool first) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            dd_t tot{0.0, 0.0};
            if (ei[q] > SP_NOEXP && ej > SP_NOEXP) {
                if (DD) {
#pragma unroll
                    for (int g0 = 0; g0 < SS; g0 += 4) {
                        // exact: |I_s| < 2^31, so the group sum is a
                        // multiple of 2^-21 below 2^32 (53 bits)
                        double v = 0.0;
#pragma unroll
                        for (int u = 3; u >= 0; --u)
                            if (g0 + u < SS) v = v * 0x1p-7 + (double)diag[g0 + u][q];
                        tot = dd_add(tot, dd_t{ldexp(v, -7 * (g0 + 2)), 0.0});
                    }
                    tot.hi = ldexp(tot.hi, ei[q] + ej);
                    tot.lo = ldexp(tot.lo, ei[q] + ej);
                } else {
                    double v = 0.0;
#pragma unroll
                    for (int s0 = SS - 1; s0 >= 0; --s0) v = v * 0x1p-7 + (double)diag[s0][q];
                    tot.hi = ldexp(v, ei[q] + ej - 14);
                }
            }
            if (!first) tot = dd_add(tot, dd_t{dst[2 * q], dst[2 * q + 1]});
            dst[2 * q] = tot.hi;
            dst[2 * q + 1] = tot.lo;
        }
#pragma unroll
        for (int s = 0; s < SS; ++s) diag[s] = v4i{0, 0, 0, 0};
    };
    bool first_flush = true;
    int since_flush = 0;
    auto consume = [&](int ci, int b) {
        const bool newexp = flagc[b] == ci + 1;
        if ((newexp || since_flush == SP_FLUSH_EVERY) && since_flush > 0) {
            flush(first_flush);
            first_flush = false;
            since_flush = 0;
        }
        const signed char *planes = planes_of(b);
        if (newexp) {
            const int *expo = expo_of(b);
            ej = expo[cb];
#pragma unroll
            for (int q = 0; q < 4; ++q) ei[q] = expo[16 * bi + 4 * (lane >> 4) + q];
        }
        // the SS B-operand planes stay in registers; A-operand plane r meets t <= SS - 1 - r
        v4i bop[SS];
#pragma unroll
        for (int t = 0; t < SS; ++t)
            bop[t] = *reinterpret_cast<const v4i *>(planes + t * SL + cb * SP_CS + koff);
#pragma unroll
        for (int r = 0; r < SS; ++r) {
            const v4i aop = *reinterpret_cast<const v4i *>(planes + r * SL + ca * SP_CS + koff);
#pragma unroll
            for (int t = 0; t < SS - r; ++t)
                diag[r + t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(aop, bop[t], diag[r + t], 0, 0, 0);
        }
        ++since_flush;
    };

    // The two roles run separate loops (so their register state need not
    // coexist), with the same number of barriers per chunk: NBUF == 2, one
    // barrier per iteration over nchunk + 1 iterations; NBUF == 1, two per chunk.
    if (producer) {
        if constexpr (NBUF == 2) {
            for (int it = 0; it <= nchunk; ++it) {
                if (it < nchunk) produce(it, it & 1);
                __syncthreads();
            }
        } else {
            for (int it = 0; it < nchunk; ++it) {
                produce(it, 0);
                __syncthreads();
                __syncthreads();
            }
        }
    } else {
        if constexpr (NBUF == 2) {
            for (int it = 0; it <= nchunk; ++it) {
                if (has_tile && it >= 1) consume(it - 1, (it - 1) & 1);
                __syncthreads();
            }
        } else {
            for (int it = 0; it < nchunk; ++it) {
                __syncthreads();
                if (has_tile) consume(it, 0);
                __syncthreads();
            }
        }
    }
    if (has_tile) flush(first_flush);
}

template <typename T, int NB, int SS>
__global__ void __launch_bounds__(sp_threads(NB))
gram_split_kernel(const T *__restrict__ A, int64_t lda, int64_t m, int n, int64_t rows_per_split,
                  double *__restrict__ part) {
    gram_split_body<T, NB, SS>(A, lda, m, n, rows_per_split, blockIdx.y, blockIdx.x, part);
}

// Batched: blockIdx.z picks the problem order[first + z], blockIdx.y its slab.
template <typename T, int NB, int SS>
__global__ void __launch_bounds__(sp_threads(NB))
gram_split_batched_kernel(const BatchMat *__restrict__ tab, const int *__restrict__ order,
                          int first) {
    const BatchMat &d = tab[order[first + blockIdx.z]];
    if ((int)blockIdx.y >= d.nsplit) return;
    gram_split_body<T, NB, SS>(reinterpret_cast<const T *>(d.A), d.lda, d.m, d.n,
                               d.rows_per_split, blockIdx.y, blockIdx.x, d.part);
}

// Launchers of the partial-sum kernels for one element type: the (NB, S)
// instance is picked at run time from the plan.
template <typename T, int NB, int SS>
static hipError_t split_partial_inst(int64_t m, int64_t n, const T *A, int64_t lda, void *part,
                                     const SplitPlan &p, hipStream_t st) {
    auto k = gram_split_kernel<T, NB, SS>;
    hipError_t err = hipFuncSetAttribute((const void *)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)p.lds_bytes);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3(sp_groups(NB), (unsigned)p.nsplit), dim3(sp_threads(NB)),
                       p.lds_bytes, st, A, lda, m, (int)n, p.rows_per_split, (double *)part);
    return hipGetLastError();
}

template <typename T, int NB, int SS>
static hipError_t split_batched_inst(const BatchMat *tab, const int *order, int first, int count,
                                     int max_nsplit, const SplitPlan &p, hipStream_t st) {
    auto k = gram_split_batched_kernel<T, NB, SS>;
    hipError_t err = hipFuncSetAttribute((const void *)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)p.lds_bytes);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3(sp_groups(NB), (unsigned)max_nsplit, (unsigned)count),
                       dim3(sp_threads(NB)), p.lds_bytes, st, tab, order, first);
    return hipGetLastError();
}

#define GSVD_SPLIT_S_CASES(CALL, NB)                                                         \
    switch (p.S) {                                                                           \
        case 1: return CALL(NB, 1);                                                          \
        case 2: return CALL(NB, 2);                                                          \
        case 3: return CALL(NB, 3);                                                          \
        case 4: return CALL(NB, 4);                                                          \
        case 5: return CALL(NB, 5);                                                          \
        case 6: return CALL(NB, 6);                                                          \
        case 7: return CALL(NB, 7);                                                          \
        case 8: return CALL(NB, 8);                                                          \
        case 9: if constexpr (SplitMax<T>::S >= 9) return CALL(NB, 9); else break;           \
        case 10: if constexpr (SplitMax<T>::S >= 10) return CALL(NB, 10); else break;        \
        case 11: if constexpr (SplitMax<T>::S >= 11) return CALL(NB, 11); else break;        \
        case 12: if constexpr (SplitMax<T>::S >= 12) return CALL(NB, 12); else break;        \
        default: break;                                                                      \
    }                                                                                        \
    return hipErrorInvalidValue;

#define GSVD_SPLIT_NB_CASES(NBCALL)                                                          \
    switch (p.nb) {                                                                          \
        case 1: NBCALL(1)                                                                    \
        case 2: NBCALL(2)                                                                    \
        case 3: NBCALL(3)                                                                    \
        case 4: NBCALL(4)                                                                    \
        case 5: NBCALL(5)                                                                    \
        case 6: NBCALL(6)                                                                    \
        case 7: NBCALL(7)                                                                    \
        case 8: NBCALL(8)                                                                    \
        default: return hipErrorInvalidValue;                                                \
    }

template <typename T>
static hipError_t split_partial_typed(int64_t m, int64_t n, const T *A, int64_t lda, void *part,
                                      const SplitPlan &p, hipStream_t st) {
#define GSVD_CALL(NB_, S_) split_partial_inst<T, NB_, S_>(m, n, A, lda, part, p, st)
#define GSVD_NB(NB_) { GSVD_SPLIT_S_CASES(GSVD_CALL, NB_) }
    GSVD_SPLIT_NB_CASES(GSVD_NB)
#undef GSVD_NB
#undef GSVD_CALL
}

template <typename T>
static hipError_t split_batched_typed(const BatchMat *tab, const int *order, int first, int count,
                                      int max_nsplit, const SplitPlan &p, hipStream_t st) {
#define GSVD_CALL(NB_, S_) split_batched_inst<T, NB_, S_>(tab, order, first, count, max_nsplit, p, st)
#define GSVD_NB(NB_) { GSVD_SPLIT_S_CASES(GSVD_CALL, NB_) }
    GSVD_SPLIT_NB_CASES(GSVD_NB)
#undef GSVD_NB
#undef GSVD_CALL
}

#undef GSVD_SPLIT_S_CASES
#undef GSVD_SPLIT_NB_CASES

}  // namespace gsvd

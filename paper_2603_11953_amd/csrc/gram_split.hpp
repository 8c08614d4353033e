// Gram M_h = A^T A by exact operand splitting on the int8 matrix cores
// (the "split" form of Alg. 1 steps 1-2).
//
// A workgroup owns a slab of rows and keeps, per column j, an exponent E_j
// with |a_kj| < 2^(E_j - 3) for every row seen so far.  Each entry is written
// as the 96-bit fixed-point integer X = sign(a) floor(|a| 2^(96 - E_j))
// (|X| < 2^93; three exact FP64 floor steps give its 32-bit words) and cut into
// balanced base-256 digits: adding 0x80 to every byte of X (with carries)
// and taking each byte minus 128 gives
//     a = 2^E_j sum_{r=1..S} d_r 2^(-8 r) + tail,  d_r in [-128, 127],
// |tail| <= (128 / 255) 2^(E_j - 8 S) + 2^(E_j - 96), every digit a signed byte.
// The contribution of the rows to M(i, j) is
//     2^(E_i + E_j) sum_{s=2..S+1} 2^(-8 s) I_s,   I_s = sum_{r+t=s} sum_k d_r,ki d_t,kj,
// keeping the slice pairs r + t <= S + 1 (the dropped pairs are below the last
// kept digit).  The I_s are exact integers accumulated by
// v_mfma_i32_16x16x64_i8 in int32 registers across chunks of 64 rows.
//
// The integer sums stay in registers until an exponent has to grow (a chunk
// holds an entry >= 2^(E_j - 3)), until 128 chunks have been added (the int32
// bound: 128 chunks x 64 rows x at most 12 pairs x 128^2 < 2^31), or until the
// slab ends.  Then they are "flushed": combined exactly (Horner over groups of
// three diagonals, each group exact in FP64) into double-double (FP64 A) or
// FP64 (FP32 A), and added to the workgroup's own slot of the partial-sum
// buffer.  A new exponent is set two bits above what the chunk needs, so
// flushes are rare.
//
// Layout: the chunk's digits sit in LDS as int8 planes, column-major (the 64
// rows of a column are 64 contiguous bytes, columns 80 bytes apart).  A 16x16
// tile (I, J) of M takes
// its A operand from columns 16 I .. 16 I + 15 and its B operand from columns
// 16 J .. 16 J + 15: lane l reads the 16 bytes of rows 16 (l / 16) .. + 15 of
// column 16 I + l % 16 (resp. 16 J + l % 16); the integer result gives lane l,
// register q the entry (4 (l / 16) + q, l % 16).  Each wavefront owns up to five
// tiles I <= J of the upper triangle and also cuts its share of every chunk.
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

// exponent needed by a: the smallest e with |a| < 2^(e - 3); SP_NOEXP for a = 0
__device__ __forceinline__ int need_exp(double a) { return a != 0.0 ? ilogb(a) + 4 : SP_NOEXP; }

// The balanced base-256 digits of a (exponent E, |a| < 2^(E - 3)) as the bytes
// of three words, digit 1 in the top byte of w2 and digit 12 in the low byte of
// w0.  |a| 2^(96 - E) is taken 32 bits at a time: each floor and subtraction is
// exact (the remainder keeps a subset of the 53 bits of |a|), so the words are
// floor(|a| 2^(96 - E)); a negative a negates the 96-bit integer.
template <int NW3>
__device__ __forceinline__ void balanced96(double a, int E, unsigned &w2, unsigned &w1,
                                           unsigned &w0) {
    const double x = __builtin_fabs(a);
    const double y0 = ldexp(x, 32 - E);  // < 2^29
    const double f0 = __builtin_floor(y0);
    unsigned h = (unsigned)f0, mid = 0, low = 0;
    if constexpr (NW3 >= 2) {
        const double y1 = (y0 - f0) * 0x1p32;
        const double f1 = __builtin_floor(y1);
        mid = (unsigned)f1;
        if constexpr (NW3 >= 3) low = (unsigned)__builtin_floor((y1 - f1) * 0x1p32);
    }
    unsigned long long lo64 = ((unsigned long long)mid << 32) | low;
    if (a < 0.0) {  // two's complement of the 96-bit value
        lo64 = ~lo64 + 1ull;
        h = ~h + (lo64 == 0ull ? 1u : 0u);
    }
    // + 0x80 in every byte (carries through the words), then each byte ^ 0x80
    const unsigned long long c64 = 0x8080808080808080ull;
    const unsigned long long s64 = lo64 + c64;
    const unsigned carry = s64 < lo64 ? 1u : 0u;
    w2 = (h + 0x80808080u + carry) ^ 0x80808080u;
    const unsigned long long d64 = s64 ^ c64;
    w1 = (unsigned)(d64 >> 32);
    w0 = (unsigned)d64;
}

// 4x4 byte transpose: o_j byte q = w_q byte j (v_perm_b32 picks bytes of
// {S0 (high word), S1 (low word)})
__device__ __forceinline__ void transpose4(unsigned w0, unsigned w1, unsigned w2, unsigned w3,
                                           unsigned &o0, unsigned &o1, unsigned &o2,
                                           unsigned &o3) {
    const unsigned t0 = __builtin_amdgcn_perm(w1, w0, 0x05010400u);
    const unsigned t1 = __builtin_amdgcn_perm(w1, w0, 0x07030602u);
    const unsigned t2 = __builtin_amdgcn_perm(w3, w2, 0x05010400u);
    const unsigned t3 = __builtin_amdgcn_perm(w3, w2, 0x07030602u);
    o0 = __builtin_amdgcn_perm(t2, t0, 0x05040100u);
    o1 = __builtin_amdgcn_perm(t2, t0, 0x07060302u);
    o2 = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
    o3 = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
}

// Work split of one slab.  Every wavefront of a workgroup both cuts its share of
// each chunk into digits and runs the products of its own tiles, so the digits
// of a chunk are formed once per workgroup (VALU work that outweighs the
// products).  A wavefront keeps 4 SS accumulator registers per tile, so the
// tiles per wavefront (TPW), the wavefronts (16, 12 or 8: 4, 3 or 2 per SIMD)
// and, when even 8 do not hold the whole triangle, the workgroups per slab
// (each cutting the whole chunk) follow from the register budget of a wavefront
// (512 per lane and SIMD over the wavefronts it hosts).
__host__ __device__ constexpr int sp_npair(int nb) { return nb * (nb + 1) / 2; }
// registers of a wavefront (measured model): per tile the SS accumulators and
// about 11 of bookkeeping, the B operands of one tile, and the cutting state
// (more for FP64 entries)
__host__ __device__ constexpr int sp_regs(int tpw, int ss, int wb) {
    return (4 * ss + 11) * tpw + 4 * ss + (wb == 8 ? 80 : 64);
}
// a few registers over the share of the register file are left to spill
__host__ __device__ constexpr int sp_budget(int nw) { return 512 / ((nw + 3) / 4) + 8; }
__host__ __device__ constexpr int sp_tpw_of(int nb, int g, int nw) {
    return ((sp_npair(nb) + g - 1) / g + nw - 1) / nw;
}
__host__ __device__ constexpr bool sp_fits(int nb, int ss, int wb, int g, int nw) {
    return sp_regs(sp_tpw_of(nb, g, nw), ss, wb) <= sp_budget(nw);
}
// the first (groups, wavefronts) that fits: groups ascending, then 16, 12, 8 wavefronts
__host__ __device__ constexpr int sp_pick(int nb, int ss, int wb) {
    for (int g = 1; g <= sp_npair(nb); ++g)
        for (int nw = 16; nw >= 8; nw -= 4)
            if (sp_fits(nb, ss, wb, g, nw)) return 64 * g + nw;
    return 64 * sp_npair(nb) + 8;
}
template <typename T>
__host__ __device__ constexpr int sp_groups(int nb, int ss) {
    return sp_pick(nb, ss, (int)sizeof(T)) / 64;
}
template <typename T>
__host__ __device__ constexpr int sp_nwave(int nb, int ss) {
    return sp_pick(nb, ss, (int)sizeof(T)) % 64;
}
template <typename T>
__host__ __device__ constexpr int sp_threads(int nb, int ss) { return 64 * sp_nwave<T>(nb, ss); }
constexpr int SP_LDS_MAX = 160 * 1024 - 1024;

// bytes of one plane buffer (all slices of one chunk) plus its exponents
__host__ __device__ constexpr int sp_buf_bytes(int nb, int ss) {
    return ss * 16 * nb * SP_CS + 16 * nb * 4;
}
// two buffers (the digits of chunk i + 1 cut while chunk i is multiplied) when they fit
__host__ __device__ constexpr int sp_bufs(int nb, int ss) {
    return 2 * sp_buf_bytes(nb, ss) + 64 <= SP_LDS_MAX ? 2 : 1;
}
__host__ __device__ constexpr int sp_lds(int nb, int ss) {
    return sp_bufs(nb, ss) * sp_buf_bytes(nb, ss) + 64;
}

// The partial Gram of slab `split` of one matrix, tiles of workgroup `grp`.
//
// Cutting: lane l of wavefront w holds rows 4 (l % 16) .. + 3 of column
// 4 NW p + 4 w + l / 16 for every pass p, so the 16 lanes of a DPP row hold one
// column and agree on its exponent by a DPP max without any barrier.  A column
// whose exponent grows records the chunk in the buffer's flag (a monotone LDS
// maximum).  Products: tile t of wavefront w is number TPG grp + w + NW t of the
// upper triangle (TPG tiles per workgroup).  Iteration i cuts chunk i into one
// buffer and multiplies chunk i - 1 from the other; before multiplying, every
// tile flushes its integer sums when the flag names that chunk (or every 128
// chunks) and reloads its exponents.  One barrier per chunk.  When two buffers
// do not fit LDS, cutting and multiplying alternate on one (two barriers).
template <typename T, int NB, int SS>
__device__ __forceinline__ void gram_split_body(const T *__restrict__ A, int64_t lda, int64_t m,
                                                int n, int64_t rows_per_split, int64_t split,
                                                int grp, double *__restrict__ part) {
    constexpr bool DD = sizeof(T) == 8;
    constexpr int G = sp_groups<T>(NB, SS);
    constexpr int NW = sp_nwave<T>(NB, SS);
    constexpr int NPAIR = sp_npair(NB);
    constexpr int TPG = (NPAIR + G - 1) / G;   // tiles per workgroup
    constexpr int TPW = (TPG + NW - 1) / NW;   // tiles per wavefront, at most
    constexpr int N16 = 16 * NB;
    constexpr int SL = N16 * SP_CS;    // bytes per digit plane
    constexpr int NBUF = sp_bufs(NB, SS);
    constexpr int BB = sp_buf_bytes(NB, SS);
    constexpr int CPP = 4 * NW;                   // columns per cutting pass
    constexpr int NPASS = (N16 + CPP - 1) / CPP;  // cutting passes
    constexpr bool PREF = NPASS * (int)sizeof(T) <= 32;  // next chunk held in registers
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    // [0], [1]: the chunk whose exponents grew, per buffer; [2]: a NaN or Inf was seen
    int *flagc = reinterpret_cast<int *>(smem + NBUF * BB);
    auto planes_of = [&](int b) { return reinterpret_cast<signed char *>(smem + b * BB); };
    auto expo_of = [&](int b) { return reinterpret_cast<int *>(smem + b * BB + SS * SL); };

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wavefront
    const int64_t r0 = split * rows_per_split;
    const int64_t r1 = (r0 + rows_per_split < m) ? r0 + rows_per_split : m;
    const int nchunk = (int)((r1 - r0 + SP_KT - 1) / SP_KT);

    if (tid < 3) flagc[tid] = 0;
    __syncthreads();

    // ---------------- cutting state
    const int pcol = 4 * wave + (lane >> 4);  // + CPP p
    const int prow = 4 * (lane & 15);
    T cur[NPASS][4], nxt[PREF ? NPASS : 1][4];
    int er[NPASS];
#pragma unroll
    for (int p = 0; p < NPASS; ++p) er[p] = SP_NOEXP;
    auto fetch = [&](T (&v)[NPASS][4], int chunk) {
        const int64_t base = r0 + (int64_t)chunk * SP_KT + prow;
#pragma unroll
        for (int p = 0; p < NPASS; ++p) {
            const int c = CPP * p + pcol;
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
        // a NaN or Inf cannot be cut into digits: it is taken as zero and flagged,
        // and the workgroup's partial sums become NaN
        bool nonfinite = false;
#pragma unroll
        for (int p = 0; p < NPASS; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double x = __builtin_fabs((double)cur[p][q]);
                if (!(x <= 1.7976931348623157e308)) {
                    nonfinite = true;
                    cur[p][q] = (T)0;
                }
            }
        if (nonfinite) flagc[2] = 1;
#pragma unroll
        for (int p = 0; p < NPASS; ++p) {
            const int c = CPP * p + pcol;
            if (CPP * (p + 1) > N16 && c >= N16) continue;  // a whole DPP row: uniform in the row
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
            constexpr int NW3 = (SS + 3) / 4;  // 32-bit digit words needed
            unsigned w[3][4];
#pragma unroll
            for (int q = 0; q < 4; ++q) balanced96<NW3>((double)cur[p][q], E, w[0][q], w[1][q], w[2][q]);
            signed char *pd = planes + c * SP_CS + prow;
#pragma unroll
            for (int k = 0; k < NW3; ++k) {
                unsigned o[4];
                transpose4(w[k][0], w[k][1], w[k][2], w[k][3], o[0], o[1], o[2], o[3]);
                // word k holds digits 4 k + 1 (top byte) .. 4 k + 4 (low byte)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r = 4 * k + (3 - j);  // zero-based digit index of byte j
                    if (r < SS) *reinterpret_cast<unsigned *>(pd + r * SL) = o[j];
                }
            }
        }
        if constexpr (PREF) {
#pragma unroll
            for (int p = 0; p < NPASS; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) cur[p][q] = nxt[p][q];
        }
    };

    // ---------------- product state: this wavefront's tiles (I, J), I <= J
    const int tlo = grp * TPG;
    const int thi = (tlo + TPG < NPAIR) ? tlo + TPG : NPAIR;
    bool has[TPW];
    int ca[TPW], cb[TPW], rowa[TPW];
    int ei[TPW][4], ej[TPW];
    v4i diag[TPW][SS];
    double *dst[TPW];
    const int koff = 16 * (lane >> 4);
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int pidx = tlo + wave + NW * t;
        has[t] = pidx < thi;  // uniform per wavefront
        int bi = 0, bj = 0;
        if (has[t]) sp_decode_pair(pidx, NB, bi, bj);
        ca[t] = 16 * bi + (lane & 15);
        cb[t] = 16 * bj + (lane & 15);
        rowa[t] = 16 * bi + 4 * (lane >> 4);
        ej[t] = SP_NOEXP;
#pragma unroll
        for (int q = 0; q < 4; ++q) ei[t][q] = SP_NOEXP;
#pragma unroll
        for (int s = 0; s < SS; ++s) diag[t][s] = v4i{0, 0, 0, 0};
        // partial slot of this slab's tile: [split][tile][lane][q][hi, lo]
        dst[t] = part + (((size_t)split * NPAIR + (has[t] ? pidx : 0)) * 64 + lane) * 8;
    }
    // flush tile t: add the integer sums (with the exponents in force) to its slot
    auto flush = [&](int t, bool first) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            dd_t tot{0.0, 0.0};
            if (ei[t][q] > SP_NOEXP && ej[t] > SP_NOEXP) {
                if (DD) {
#pragma unroll
                    for (int g0 = 0; g0 < SS; g0 += 3) {
                        // exact: |I_s| < 2^31, so the group sum is a
                        // multiple of 2^-16 below 2^32 (48 bits)
                        double v = 0.0;
#pragma unroll
                        for (int u = 2; u >= 0; --u)
                            if (g0 + u < SS) v = v * 0x1p-8 + (double)diag[t][g0 + u][q];
                        tot = dd_add(tot, dd_t{ldexp(v, -8 * (g0 + 2)), 0.0});
                    }
                    tot.hi = ldexp(tot.hi, ei[t][q] + ej[t]);
                    tot.lo = ldexp(tot.lo, ei[t][q] + ej[t]);
                } else {
                    double v = 0.0;
#pragma unroll
                    for (int s0 = SS - 1; s0 >= 0; --s0) v = v * 0x1p-8 + (double)diag[t][s0][q];
                    tot.hi = ldexp(v, ei[t][q] + ej[t] - 16);
                }
            }
            if (!first) tot = dd_add(tot, dd_t{dst[t][2 * q], dst[t][2 * q + 1]});
            dst[t][2 * q] = tot.hi;
            dst[t][2 * q + 1] = tot.lo;
        }
#pragma unroll
        for (int s = 0; s < SS; ++s) diag[t][s] = v4i{0, 0, 0, 0};
    };
    bool first_flush = true;
    int since_flush = 0;
    auto consume = [&](int ci, int b) {
        const bool newexp = flagc[b] == ci + 1;
        const bool doflush = (newexp || since_flush == SP_FLUSH_EVERY) && since_flush > 0;
        const signed char *planes = planes_of(b);
        const int *expo = expo_of(b);
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            if (!has[t]) continue;
            if (doflush) flush(t, first_flush);
            if (newexp) {
                ej[t] = expo[cb[t]];
#pragma unroll
                for (int q = 0; q < 4; ++q) ei[t][q] = expo[rowa[t] + q];
            }
            // the SS B-operand planes in registers; A-operand plane r meets t' <= SS - 1 - r
            v4i bop[SS];
#pragma unroll
            for (int u = 0; u < SS; ++u)
                bop[u] = *reinterpret_cast<const v4i *>(planes + u * SL + cb[t] * SP_CS + koff);
#pragma unroll
            for (int r = 0; r < SS; ++r) {
                const v4i aop = *reinterpret_cast<const v4i *>(planes + r * SL + ca[t] * SP_CS + koff);
#pragma unroll
                for (int u = 0; u < SS - r; ++u)
                    diag[t][r + u] = __builtin_amdgcn_mfma_i32_16x16x64_i8(aop, bop[u], diag[t][r + u], 0, 0, 0);
            }
        }
        if (doflush) {
            first_flush = false;
            since_flush = 0;
        }
        ++since_flush;
    };

    if constexpr (NBUF == 2) {
        for (int it = 0; it <= nchunk; ++it) {
            if (it < nchunk) produce(it, it & 1);
            if (it >= 1) consume(it - 1, (it - 1) & 1);
            __syncthreads();
        }
    } else {
        for (int it = 0; it < nchunk; ++it) {
            produce(it, 0);
            __syncthreads();
            consume(it, 0);
            __syncthreads();
        }
    }
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        if (!has[t]) continue;
        flush(t, first_flush);
        if (flagc[2] != 0) {  // set before the last barrier of the loop
#pragma unroll
            for (int k = 0; k < 8; ++k) dst[t][k] = __builtin_nan("");
        }
    }
}

template <typename T, int NB, int SS>
__global__ void __launch_bounds__(sp_threads<T>(NB, SS))
gram_split_kernel(const T *__restrict__ A, int64_t lda, int64_t m, int n, int64_t rows_per_split,
                  double *__restrict__ part) {
    gram_split_body<T, NB, SS>(A, lda, m, n, rows_per_split, blockIdx.y, blockIdx.x, part);
}

// Batched: blockIdx.z picks the problem order[first + z], blockIdx.y its slab.
template <typename T, int NB, int SS>
__global__ void __launch_bounds__(sp_threads<T>(NB, SS))
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
    hipLaunchKernelGGL(k, dim3(sp_groups<T>(NB, SS), (unsigned)p.nsplit), dim3(sp_threads<T>(NB, SS)),
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
    hipLaunchKernelGGL(k, dim3(sp_groups<T>(NB, SS), (unsigned)max_nsplit, (unsigned)count),
                       dim3(sp_threads<T>(NB, SS)), p.lds_bytes, st, tab, order, first);
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

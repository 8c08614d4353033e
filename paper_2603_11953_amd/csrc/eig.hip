// Eigensolver stage: Algorithm 2 of the paper inside one workgroup.
//
//   1. Column scaling: d_j = sqrt(m_jj) = ||a_j|| (the D of A = B D), rounded to
//      a power of two 2^e_j so that H = D~^-1 M_h D~^-1 is formed exactly.
//   2. Cholesky H = R_H^T R_H at the Gram precision (double-double for FP64
//      working, where M_h carries a low plane; FP64 otherwise), right-looking
//      in the square-root-free form on the upper triangle held in LDS, rows of
//      R_H scaled at the end.  (Alg. 2 step 1.)
//   3. R = working(R_H) D~  (Alg. 2 step 2; the power-of-two scaling is exact).
//      R is further scaled by one global power of two so its largest column
//      norm is about 1 (no overflow in the squared norms below; undone at the end).
//   4. One-sided Jacobi SVD of R (Alg. 2 step 3): plane rotations applied to
//      the columns of R (Hestenes), accumulated in V = J_1 J_2 ..., until
//      every pair of columns is numerically orthogonal,
//      |r_p^T r_q| <= tol ||r_p|| ||r_q||.  R = R_H D~ is column scaled, the
//      setting in which right-handed one-sided Jacobi keeps each column's
//      rounding errors relative to that column's norm (Demmel-Veselic), and
//      the same rotations applied to V keep A V Sigma^-1 orthonormal however
//      graded the columns of A are.
//      Parallel ordering: round robin, n/2 disjoint pairs per step, one group
//      of 8 lanes (half a DPP row) per pair.  A lane keeps rows gl, gl + 8, ...
//      of the pair's two columns of R in registers for the step; the three
//      inner products are reduced across the group with DPP moves arranged so
//      all 8 lanes obtain bitwise identical sums, and the rotation parameters
//      come from two reciprocal square roots (hardware estimate refined by
//      Newton steps).  After a sweep whose rotations were all tiny, every pair
//      is tested at once on Y^T Y instead of by a further sweep.
//   5. sigma_p = ||r_p||; ordering sigma_1 >= ... >= sigma_n; each V column
//      signed so its entry of largest magnitude is positive (lowest index on
//      ties); Sigma and V cast to the working precision (Alg. 1 steps 4-5);
//      W = fl(V Sigma^-1) in the working precision (the parenthesisation of
//      Alg. 1 step 6).
//   Storage of R and V during the Jacobi: FP64 for FP64 working (n <= 96 fits
//   LDS), FP32 for FP32 working (the SVD of R "at precision u"; n <= 128),
//   with the inner products and rotation parameters evaluated in FP64.
#include <hip/hip_runtime.h>

#include "dd_device.hpp"
#include "gsvd_internal.hpp"
#include "jacobi_math.hpp"

namespace gsvd {

constexpr int GRP = 8;  // lanes per Jacobi pair: half a DPP row
// Workgroup size bound and staging depth by register depth: up to RPL = 8
// (n <= 64) 1024 lanes and n^2 / lanes <= 16 entries of R per lane while it
// moves into Y; beyond, 512 lanes (the Jacobi needs 4 N2 = 512 of them) so each
// lane may hold the larger register blocks, and n^2 / lanes <= 32.
__host__ __device__ constexpr int eig_bound(int rpl) { return rpl > 8 ? 512 : 1024; }
__host__ __device__ constexpr int eig_maxreg(int rpl) { return rpl > 8 ? 32 : 16; }

// Column stride of R and V in LDS during the Jacobi: n rounded up to a
// multiple of 256 bytes.
template <typename TS>
__host__ __device__ __forceinline__ int jac_ld(int n) {
    constexpr int q = 256 / (int)sizeof(TS);
    return (n + q - 1) / q * q;
}

// rows per lane in the Jacobi: n rounded up to 16, over 8 lanes (an even count,
// for the two-row vector accesses)
__host__ __device__ constexpr int eig_rpl(int n) { return 2 * ((n + 15) / 16); }

// n rounded up to a power of two (at least 2): the column count of the Jacobi ordering
__host__ __device__ constexpr int eig_pow2(int n) {
    int p = 2;
    while (p < n) p <<= 1;
    return p;
}

template <typename TS>
struct Vec2;
template <>
struct Vec2<double> {
    typedef double2 type;
};
template <>
struct Vec2<float> {
    typedef float2 type;
};

struct EigShared {
    int flag_rot;
    int flag_big;  // a rotation of the sweep had |sin| >= 2^-22
    int flag_pre;  // a pair rotated in the sweep had a cosine >= 2^-10
    int flag_bad;  // GSVD info code, 0 = fine
    int emax;
    int pad[3];    // 32 bytes: the arrays after it stay 16-byte aligned
};

typedef double f64x4 __attribute__((ext_vector_type(4)));

// ---- cross-lane helpers on doubles (DPP within a row of 16 lanes)

// (every source lane of the permutations below lies in the same row, so no
// lane reads the bound-control zero)
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// x of lane l (l uniform), in every lane
__device__ __forceinline__ double readlane_d(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over aligned groups of 8 lanes (half a DPP row).  Steps: xor 1, xor 2
// (quad permutes), then the half-row mirror (lane i <-> 7 - i).  Every step
// adds the values of two lanes that hold the same partial sums in swapped
// order, so all 8 lanes end with the same bits.
__device__ __forceinline__ double group_sum(double x) {
    x += dpp_d<0xB1>(x);   // quad_perm [1,0,3,2]
    x += dpp_d<0x4E>(x);   // quad_perm [2,3,0,1]
    x += dpp_d<0x141>(x);  // row_half_mirror
    return x;
}

// Back substitution of the preconditioner form, V' = X'^-1 T with T = Q Sigma_Z
// (columns scaled by ssig), X' upper triangular: Rs holds R'_rk / R'_kk above the
// diagonal (zeros elsewhere), rinv 1 / R'_kk.  Each wavefront solves its own
// columns, up to four at a time, lane l holding rows l + 64 j (j < NR, n <= 64 NR),
// with no workgroup barrier: at step k the final (not yet divided) t_k of each
// column is read from its lane and the rows r < k take -(R'_rk / R'_kk) t_k; the
// next column of Rs is read one step ahead.  Then x_r = t_r / R'_rr, the scaling
// by 2^(emax - e_pi_r),
// the column's norm (a butterfly sum: every lane gets the same bits) and the
// store into row pi_r of V.
template <int NR, typename TW>
__device__ __forceinline__ void pre_backsub(int n, const double *T, const double *Rs, int ld,
                                            const double *ssig, const double *rinv,
                                            const int *sexp, const int *sperm, int emax,
                                            TW *__restrict__ V, int64_t ldv) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
    for (int p0 = wv; p0 < n; p0 += 4 * nwv) {
        double t[4][NR];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int p = p0 + c * nwv;
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const int r = lane + 64 * j;
                t[c][j] = (p < n && r < n) ? T[r + p * ld] * ssig[p] : 0.0;
            }
        }
        // column k of Rs, one step ahead (rows k and beyond read zeros)
        double rn[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            const int r = lane + 64 * j;
            rn[j] = r < n ? Rs[r + (n - 1) * ld] : 0.0;
        }
        for (int k = n - 1; k >= 1; --k) {
            double rc[NR];
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                rc[j] = rn[j];
                const int r = lane + 64 * j;
                rn[j] = r < n ? Rs[r + (k - 1) * ld] : 0.0;
            }
            const int kl = k & 63;  // uniform
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double tk = readlane_d(NR == 1 || k < 64 ? t[c][0] : t[c][NR - 1], kl);
#pragma unroll
                for (int j = 0; j < NR; ++j) t[c][j] = __builtin_fma(-rc[j], tk, t[c][j]);
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int p = p0 + c * nwv;
            if (p >= n) break;  // uniform
            double x[NR], ss = 0.0;
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const int r = lane + 64 * j;
                x[j] = r < n ? ldexp(t[c][j] * rinv[r], emax - sexp[sperm[r]]) : 0.0;
                ss = __builtin_fma(x[j], x[j], ss);
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) ss += __shfl_xor(ss, off, 64);
            const double inv = 1.0 / __builtin_sqrt(ss);
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const int r = lane + 64 * j;
                if (r < n) V[sperm[r] + (int64_t)p * ldv] = (TW)(x[j] * inv);
            }
        }
    }
}

// Workgroup-shared state of the eigensolver besides the dynamic LDS square.
struct EigSmem {
    EigShared sh;
    int sexp[GSVD_KMAX_N];
    double ssig[GSVD_KMAX_N];
    int srank[GSVD_KMAX_N];
    double ssign[GSVD_KMAX_N];
    int sperm[GSVD_KMAX_N];  // preconditioner form: the column of rank r by m_jj, descending
    dd_t rowk[GSVD_KMAX_N];
    dd_t rpiv[GSVD_KMAX_N + 1];  // reciprocal pivots of the Cholesky
};

// Algorithm 2 for one n x n Gram (one workgroup; n <= GRP * RPL, RPL even).
//
// pre (FP64 working only): the preconditioner form for the double-double stage,
// as in the multi-workgroup eigensolver: the columns ordered by decreasing m_jj
// (pi), the Jacobi run on the transposed factor Z = X'^T of the reordered problem,
// and V' = X'^-1 Q Sigma_Z by back substitution (R' is kept in W for it; W is
// rewritten by the next stage), V = P V' with unit columns in no particular order
// or sign.  S is not written.  early: the sweep whose rotated pairs all had cosines
// below 2^-10 is the last (single problems; the batched call converges fully).
template <typename TW, typename TS, bool DDGRAM, int RPL>
__device__ __forceinline__ void eig_body(int n, const double *__restrict__ Mhi,
                                         const double *__restrict__ Mlo, int64_t ldm,
                                         TW *__restrict__ S, TW *__restrict__ V, int64_t ldv,
                                         TW *__restrict__ W, int64_t ldw, int *__restrict__ info,
                                         double tol2, int max_sweeps, bool pre, bool early,
                                         EigSmem &sm, double *lds) {
    EigShared &sh = sm.sh;
    int *sexp = sm.sexp;
    double *ssig = sm.ssig;
    int *srank = sm.srank;
    double *ssign = sm.ssign;
    dd_t *rowk = sm.rowk;

    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    pre = pre && sizeof(TS) == sizeof(double);  // FP64 working only

    if (tid == 0) {
        sh.flag_rot = 0;
        sh.flag_big = 0;
        sh.flag_pre = 0;
        sh.flag_bad = 0;
        sh.emax = -100000;
    }
    __syncthreads();

    // ---- 1. scaling exponents and input checks
    for (int j = tid; j < n; j += nthr) {
        const double mjj = Mhi[j + (int64_t)j * ldm];
        ssig[j] = mjj;  // the diagonal, for the ordering below
        if (!(mjj > 0.0) || !__builtin_isfinite(mjj)) {
            atomicMax(&sh.flag_bad, __builtin_isfinite(mjj) ? 1 : 3);
            sexp[j] = 0;
        } else {
            const int e = ilogb(__builtin_sqrt(mjj));
            sexp[j] = e;
            atomicMax(&sh.emax, e);
        }
    }
    for (int q = tid; q < n * n; q += nthr) {
        const double v = Mhi[(q % n) + (int64_t)(q / n) * ldm];
        if (!__builtin_isfinite(v)) atomicMax(&sh.flag_bad, 3);
    }
    __syncthreads();
    if (sh.flag_bad) {
        if (tid == 0) *info = sh.flag_bad;
        return;
    }
    int *sperm = sm.sperm;
    if (pre) {  // rank by m_jj descending, ties by index (every m_jj is positive here)
        for (int j = tid; j < n; j += nthr) {
            const double mj = ssig[j];
            int r = 0;
            for (int q = 0; q < n; ++q) {
                const double mq = ssig[q];
                r += (mq > mj) || (mq == mj && q < j);
            }
            sperm[r] = j;
        }
        __syncthreads();
    }
    auto pix = [&](int i) { return pre ? sperm[i] : i; };

    // ---- 2. H = D~^-1 M D~^-1 (exact) in the upper triangle of an n x n square
    //      in LDS, leading dimension n + 1 (a row's entries fall in different
    //      banks); Cholesky
    dd_t *Hd = reinterpret_cast<dd_t *>(lds);  // DDGRAM
    double *Hs = lds;                            // !DDGRAM
    const int lh = n + 1;
    for (int q = tid; q < n * n; q += nthr) {
        const int i = q % n, j = q / n;
        if (i > j) continue;
        const int pi = pix(i), pj = pix(j);
        const int a = pi < pj ? pi : pj, b = pi < pj ? pj : pi;  // upper triangle of M_h
        const int sc = -(sexp[pi] + sexp[pj]);
        const double hi = ldexp(Mhi[a + (int64_t)b * ldm], sc);
        if (DDGRAM) {
            Hd[i + j * lh] = dd_t{hi, ldexp(Mlo[a + (int64_t)b * ldm], sc)};
        } else {
            Hs[i + j * lh] = hi;
        }
    }
    __syncthreads();

    // Right-looking, one barrier per column k, in the square-root-free form:
    // h_ij -= h_ki (h_kj / h_kk) (= r_ki r_kj) over the trailing triangle
    // k < i <= j < n.  Its entries are numbered q = b (b + 1) / 2 + a for
    // (i, j) = (k + 1 + a, k + 1 + b), so the triangle of step k is q < t (t + 1) / 2
    // (t = n - 1 - k) and lane tid owns q = tid + e * nthr at every step: its
    // offsets (a, b) are found once.  Entry q = 0 is the next pivot; its owner
    // (lane 0) also forms that pivot's reciprocal for the next step.  Row k of
    // the square is final once step k starts, so R's rows, r_kj = h_kj / sqrt(h_kk),
    // are formed afterwards, all at once.
    constexpr int MAXE = eig_maxreg(RPL) / 2;  // n (n - 1) / 2 <= MAXE nthr, as n^2 <= 2 MAXE nthr
    int ab[MAXE];
#pragma unroll
    for (int e = 0; e < MAXE; ++e) {
        const int q = tid + e * nthr;
        int b = (int)((__builtin_sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f);
        while (b * (b + 1) / 2 > q) --b;
        while ((b + 1) * (b + 2) / 2 <= q) ++b;
        ab[e] = (q - b * (b + 1) / 2) | (b << 8);
    }
    // 1 / h in dd: the FP64 estimate r corrected once, r + r (1 - h r)
    auto dd_rcp = [](dd_t h) -> dd_t {
        const double r0 = rcp_nr(h.hi);
        const dd_t hr = dd_mul_d(h, r0);
        const double e = (1.0 - hr.hi) - hr.lo;
        return quick_two_sum(r0, r0 * e);
    };
    dd_t *rpiv = sm.rpiv;
    if (DDGRAM && tid == 0) rpiv[0] = dd_rcp(Hd[0]);
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const dd_t hkk = DDGRAM ? Hd[k + k * lh] : dd_t{Hs[k + k * lh], 0.0};
        if (!(hkk.hi > 0.0)) {  // uniform across the workgroup
            if (tid == 0) *info = 1;
            return;
        }
        const int t = n - 1 - k;
        const int nent = t * (t + 1) / 2;
        if (DDGRAM) {
            const dd_t rinv = rpiv[k];
#pragma unroll
            for (int e = 0; e < MAXE; e += 2) {
                const int q = tid + e * nthr;
                if (q < nent) {
                    const bool two = q + nthr < nent;
                    const int ia = k + 1 + (ab[e] & 255), ja = k + 1 + (ab[e] >> 8);
                    const int ib = k + 1 + (ab[e + 1] & 255), jb = k + 1 + (ab[e + 1] >> 8);
                    const dd_t kia = Hd[k + ia * lh], kja = Hd[k + ja * lh], hija = Hd[ia + ja * lh];
                    dd_t kib{0.0, 0.0}, kjb{0.0, 0.0}, hijb{0.0, 0.0};
                    if (two) {
                        kib = Hd[k + ib * lh];
                        kjb = Hd[k + jb * lh];
                        hijb = Hd[ib + jb * lh];
                    }
                    const dd_t va = dd_sub_fast(hija, dd_mul(kia, dd_mul(kja, rinv)));
                    Hd[ia + ja * lh] = va;
                    if (e == 0 && q == 0) rpiv[k + 1] = dd_rcp(va);  // the next pivot
                    if (two) Hd[ib + jb * lh] = dd_sub_fast(hijb, dd_mul(kib, dd_mul(kjb, rinv)));
                }
            }
        } else {
            const double rinv = 1.0 / hkk.hi;
#pragma unroll
            for (int e = 0; e < MAXE; ++e) {
                const int q = tid + e * nthr;
                if (q < nent) {
                    const int i = k + 1 + (ab[e] & 255), j = k + 1 + (ab[e] >> 8);
                    Hs[i + j * lh] = __builtin_fma(-Hs[k + i * lh], Hs[k + j * lh] * rinv, Hs[i + j * lh]);
                }
            }
        }
        __syncthreads();
    }
    // 1 / sqrt(h_kk) per row k (in dd, the FP64 estimate y refined once,
    // y + y (1 - h y^2) / 2), kept in rowk; then r_kj = h_kj rowk[k]
    for (int k = tid; k < n; k += nthr) {
        if (DDGRAM) {
            const dd_t hkk = Hd[k + k * lh];
            const double y = rsq_nr(hkk.hi);
            const dd_t hy2 = dd_mul_d(dd_mul_d(hkk, y), y);
            rowk[k] = dd_add(dd_t{y, 0.0}, dd_mul_d(dd_sub(dd_t{1.0, 0.0}, hy2), 0.5 * y));
        } else {
            rowk[k] = dd_t{1.0 / __builtin_sqrt(Hs[k + k * lh]), 0.0};
        }
    }
    __syncthreads();

    // ---- 3. R = working(R_H) D~ 2^-emax as an n x n column-major TS matrix Y in
    //      LDS, V = I next to it.  The Cholesky square overlaps both, so every
    //      lane first lifts its share of R into registers.
    const int emax = sh.emax;
    constexpr int MAXREG = eig_maxreg(RPL);
    double rv[MAXREG];
#pragma unroll
    for (int c = 0; c < MAXREG; ++c) {
        const int q = tid + c * nthr;
        rv[c] = 0.0;
        if (q < n * n) {
            const int i = q % n, j = q / n;
            if (i <= j) {
                const double h = DDGRAM ? dd_mul(Hd[i + j * lh], rowk[i]).hi
                                        : Hs[i + j * lh] * rowk[i].hi;  // r_ij
                rv[c] = ldexp((double)(TW)h, sexp[pix(j)] - emax);  // round to working, rescale
                if (pre) W[i + (int64_t)j * ldw] = (TW)h;  // R' for the back substitution
            }
        }
    }
    __syncthreads();
    // column stride: a multiple of 256 bytes, so a column's bank offset depends
    // only on the row (see the row-block rotation in the Jacobi loop)
    const int ld = jac_ld<TS>(n);
    TS *Y = reinterpret_cast<TS *>(lds);
    TS *Vs = Y + n * ld;
    // zero everything first: rows n .. ld-1 are padding that the Jacobi loop
    // reads and rotates without bounds checks (zeros stay zeros)
    for (int q = tid; q < 2 * n * ld; q += nthr) Y[q] = (TS)0;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < MAXREG; ++c) {
        const int q = tid + c * nthr;
        if (q < n * n) {
            const int r = q % n, col = q / n;
            if (pre)
                Y[col + r * ld] = (TS)rv[c];  // Z = X'^T
            else
                Y[r + col * ld] = (TS)rv[c];
            if (r == col) Vs[r + col * ld] = (TS)1;
        }
    }
    __syncthreads();

    // ---- 4. one-sided Jacobi on the columns of Y = R, rotations accumulated in V.
    //      Ordering: the columns are padded (virtually) to N2 = 2^k >= n.  Level L
    //      splits them into sets of s = N2 >> L columns; in each set the lower half
    //      stays resident in the registers of h = s / 2 groups while the upper half
    //      travels: at step t group i of the set pairs its resident column with
    //      traveler (i + t) mod h, so the h steps cover every cross pair of the
    //      two halves with h disjoint pairs each.  The next level recurses into
    //      both halves; N2 - 1 steps cover every pair once.  Only the traveling
    //      column of a pair goes through LDS each step (half the traffic of an
    //      ordering that moves both).  Pairs with a padding column are skipped.
    const int N2 = eig_pow2(n);
    const int grp = tid / GRP, gl = tid % GRP;
    const int ngrp = nthr / GRP;
    typedef typename Vec2<TS>::type tv2;
    constexpr int RP2 = RPL / 2;  // row pairs per lane: rows 2 gl + 16 b, + 1
    // register b holds row pair (b + rot) mod RP2: groups that share an LDS cycle
    // read different 128-row-byte blocks
    const int rot = RP2 > 1 ? (grp & 3) % RP2 : 0;
    auto rowof = [&](int b) {
        int blk = b + rot;
        if (blk >= RP2) blk -= RP2;
        return 2 * gl + 16 * blk;
    };
    bool converged = (n == 1);
    for (int sw = 0; sw < max_sweeps && !converged; ++sw) {
        for (int s2 = N2; s2 >= 2; s2 >>= 1) {
            const int h = s2 >> 1;
            const int set = grp / h, li = grp - set * h;
            const int res = set * s2 + li;
            const bool act = grp < (N2 >> 1) && res < n && grp < ngrp;
            TS x0[RPL], w0[RPL];
            if (act) {
                const TS *yr = Y + res * ld, *vr = Vs + res * ld;
#pragma unroll
                for (int b = 0; b < RP2; ++b) {
                    const int r = rowof(b);
                    const tv2 y = *reinterpret_cast<const tv2 *>(yr + r);
                    const tv2 v = *reinterpret_cast<const tv2 *>(vr + r);
                    x0[2 * b] = y.x;
                    x0[2 * b + 1] = y.y;
                    w0[2 * b] = v.x;
                    w0[2 * b + 1] = v.y;
                }
            }
            for (int t = 0; t < h; ++t) {
                int tj = li + t;
                if (tj >= h) tj -= h;
                const int trv = set * s2 + h + tj;
                if (act && trv < n) {  // uniform within the group
                    TS *yq = Y + trv * ld, *vq = Vs + trv * ld;
                    TS x1[RPL], w1[RPL];
#pragma unroll
                    for (int b = 0; b < RP2; ++b) {
                        const int r = rowof(b);
                        const tv2 y = *reinterpret_cast<const tv2 *>(yq + r);
                        const tv2 v = *reinterpret_cast<const tv2 *>(vq + r);
                        x1[2 * b] = y.x;
                        x1[2 * b + 1] = y.y;
                        w1[2 * b] = v.x;
                        w1[2 * b + 1] = v.y;
                    }
                    double al = 0, be = 0, ga = 0;
#pragma unroll
                    for (int i = 0; i < RPL; ++i) {
                        const double a0 = (double)x0[i], a1 = (double)x1[i];
                        al = __builtin_fma(a0, a0, al);
                        be = __builtin_fma(a1, a1, be);
                        ga = __builtin_fma(a0, a1, ga);
                    }
                    al = group_sum(al);
                    be = group_sum(be);
                    ga = group_sum(ga);
                    if (ga * ga > tol2 * (al * be)) {
                        double c, sn;
                        jacobi_cs(al, be, ga, c, sn);
#pragma unroll
                        for (int i = 0; i < RPL; ++i) {
                            const double a0 = (double)x0[i], a1 = (double)x1[i];
                            const double u = (double)w0[i], w = (double)w1[i];
                            x0[i] = (TS)__builtin_fma(c, a0, -(sn * a1));
                            x1[i] = (TS)__builtin_fma(c, a1, sn * a0);
                            w0[i] = (TS)__builtin_fma(c, u, -(sn * w));
                            w1[i] = (TS)__builtin_fma(c, w, sn * u);
                        }
#pragma unroll
                        for (int b = 0; b < RP2; ++b) {
                            const int r = rowof(b);
                            tv2 y, v;
                            y.x = x1[2 * b];
                            y.y = x1[2 * b + 1];
                            v.x = w1[2 * b];
                            v.y = w1[2 * b + 1];
                            *reinterpret_cast<tv2 *>(yq + r) = y;
                            *reinterpret_cast<tv2 *>(vq + r) = v;
                        }
                        // (plain stores: a register carrying the sweep's largest
                        // |sin| through the steps costs register copies per rotation)
                        if (gl == 0) {
                            sh.flag_rot = 1;
                            if (__builtin_fabs(sn) >= 0x1p-22) sh.flag_big = 1;
                            if (ga * ga >= 0x1p-20 * (al * be)) sh.flag_pre = 1;
                        }
                    }
                }
                __syncthreads();  // the travelers move on
            }
            if (act) {  // the resident goes back to its slot for the next level
                TS *yr = Y + res * ld, *vr = Vs + res * ld;
#pragma unroll
                for (int b = 0; b < RP2; ++b) {
                    const int r = rowof(b);
                    tv2 y, v;
                    y.x = x0[2 * b];
                    y.y = x0[2 * b + 1];
                    v.x = w0[2 * b];
                    v.y = w0[2 * b + 1];
                    *reinterpret_cast<tv2 *>(yr + r) = y;
                    *reinterpret_cast<tv2 *>(vr + r) = v;
                }
            }
            __syncthreads();
        }
        const bool any = sh.flag_rot != 0, big = sh.flag_big != 0, bigpre = sh.flag_pre != 0;
        __syncthreads();
        if (tid == 0) {
            sh.flag_rot = 0;
            sh.flag_big = 0;
            sh.flag_pre = 0;
        }
        if (!any || (early && !bigpre)) {
            // preconditioner form, early stop: a sweep whose rotated pairs all had
            // cosines below 2^-10 is the last (quadratic convergence leaves cosines of
            // order 2^-20 or less)
            converged = true;
        } else if (!big) {
            // The rotations of this sweep were all tiny, so the next sweep most
            // likely rotates nothing: test every pair at once instead, with the
            // same criterion on the Gram matrix Y^T Y (squared column norms by
            // groups as in the sweep, the products on the FP64 matrix cores).
            for (int p = grp; p < n; p += ngrp) {
                double ss = 0.0;
                for (int r = gl; r < n; r += GRP) {
                    const double x = (double)Y[r + p * ld];
                    ss = __builtin_fma(x, x, ss);
                }
                ss = group_sum(ss);
                if (gl == 0) ssig[p] = ss;
            }
            __syncthreads();
            const int lane = tid & 63, wv = tid >> 6, nwv = nthr >> 6;
            const int li = lane & 15, lk = lane >> 4;
            const int nb = (n + 15) / 16;
            bool bad = false;
            for (int ti = wv; ti < nb * nb; ti += nwv) {  // uniform per wavefront
                const int bi = ti / nb, bj = ti % nb;
                if (bi > bj) continue;
                const int pa = 16 * bi + li < n ? 16 * bi + li : n - 1;
                const int pb = 16 * bj + li < n ? 16 * bj + li : n - 1;
                f64x4 acc = {0.0, 0.0, 0.0, 0.0};
                for (int k0 = 0; k0 < n; k0 += 4) {  // rows n .. ld - 1 are zero
                    const double a = (double)Y[(k0 + lk) + pa * ld];
                    const double b = (double)Y[(k0 + lk) + pb * ld];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
                }
                const int q = 16 * bj + li;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int pp = 16 * bi + 4 * r + lk;
                    if (pp < q && q < n) {
                        const double g = acc[r];
                        bad = bad || (g * g > tol2 * (ssig[pp] * ssig[q]));
                    }
                }
            }
            if (bad) sh.flag_rot = 1;
            __syncthreads();
            converged = sh.flag_rot == 0;
            __syncthreads();
            if (tid == 0) sh.flag_rot = 0;
        }
        __syncthreads();
    }
    if (!converged) {
        if (tid == 0) *info = 2;
        return;
    }

    if (pre) {
        // ---- 5'. V' = X'^-1 Q Sigma_Z: T = Q Sigma_Z over Q in Vs, R' (in W) to the Y
        //      area, back substitution; then V(pi_r, p) = V'(r, p) 2^-e_pi_r (exact),
        //      columns normalised
        for (int p = grp; p < n; p += ngrp) {
            double ss = 0.0;
            for (int r = gl; r < n; r += GRP) {
                const double x = (double)Y[r + p * ld];
                ss = __builtin_fma(x, x, ss);
            }
            ss = group_sum(ss);
            if (gl == 0) ssig[p] = __builtin_sqrt(ss);
        }
        __syncthreads();
        double *T = reinterpret_cast<double *>(Vs);  // TS = double in this form
        double *Rt = reinterpret_cast<double *>(Y);
        // R'_rk / R'_kk (r < k) into the Y area, 1 / R'_kk into ssign
        for (int q = tid; q < n * n; q += nthr) {
            const int r = q % n, k = q / n;
            Rt[r + k * ld] = r < k ? (double)W[r + (int64_t)k * ldw] / (double)W[k + (int64_t)k * ldw]
                                   : 0.0;
        }
        for (int k = tid; k < n; k += nthr) ssign[k] = 1.0 / (double)W[k + (int64_t)k * ldw];
        __syncthreads();
        if (n <= 64)
            pre_backsub<1>(n, T, Rt, ld, ssig, ssign, sexp, sperm, emax, V, ldv);
        else
            pre_backsub<2>(n, T, Rt, ld, ssig, ssign, sexp, sperm, emax, V, ldv);
        if (tid == 0) *info = 0;
        return;
    }

    // ---- 5. sigma_p = ||y_p|| 2^emax, ordering, sign of V columns, cast, W
    for (int p = grp; p < n; p += ngrp) {
        const TS *yp = Y + p * ld;
        const TS *vp = Vs + p * ld;
        double ss = 0;
        double best = -1.0;
        int barg = 0;
        for (int r = gl; r < n; r += GRP) {
            const double x = (double)yp[r];
            ss = __builtin_fma(x, x, ss);
            const double av = __builtin_fabs((double)vp[r]);
            if (av > best) { best = av; barg = r; }
        }
        ss = group_sum(ss);
#pragma unroll
        for (int off = GRP / 2; off >= 1; off >>= 1) {
            const double ob = __shfl_xor(best, off, GRP);
            const int oa = __shfl_xor(barg, off, GRP);
            if (ob > best || (ob == best && oa < barg)) { best = ob; barg = oa; }
        }
        if (gl == 0) {
            ssig[p] = ldexp(__builtin_sqrt(ss), emax);
            ssign[p] = vp[barg] < 0 ? -1.0 : 1.0;
        }
    }
    __syncthreads();
    for (int p = tid; p < n; p += nthr) {
        const double sp = ssig[p];
        int rk = 0;
        for (int q = 0; q < n; ++q) {
            const double sq = ssig[q];
            rk += (sq > sp) || (sq == sp && q < p);
        }
        srank[p] = rk;
        if (!(sp > 0.0)) atomicMax(&sh.flag_bad, 1);
    }
    __syncthreads();
    if (sh.flag_bad) {
        if (tid == 0) *info = sh.flag_bad;
        return;
    }
    for (int q = tid; q < n * n; q += nthr) {
        const int r = q % n, p = q / n;
        const int pos = srank[p];
        const TW sw = (TW)ssig[p];
        const TW vw = (TW)(ssign[p] * (double)Vs[r + p * ld]);
        V[r + (int64_t)pos * ldv] = vw;
        W[r + (int64_t)pos * ldw] = vw / sw;
        if (r == 0) S[pos] = sw;
    }
    if (tid == 0) *info = 0;
}

template <typename TW, typename TS, bool DDGRAM, int RPL>
__global__ void __launch_bounds__(eig_bound(RPL))
eig_chol_jacobi1_kernel(int n, const double *__restrict__ Mhi, const double *__restrict__ Mlo,
                        int64_t ldm, TW *__restrict__ S, TW *__restrict__ V, int64_t ldv,
                        TW *__restrict__ W, int64_t ldw, int *__restrict__ info, double tol2,
                        int max_sweeps, bool pre) {
    extern __shared__ __attribute__((aligned(16))) double lds[];
    __shared__ EigSmem sm;
    eig_body<TW, TS, DDGRAM, RPL>(n, Mhi, Mlo, ldm, S, V, ldv, W, ldw, info, tol2, max_sweeps, pre,
                                  pre, sm, lds);
}

// Batched: one workgroup per problem, the largest first (order is ascending in
// n); the register depth RPL = eig_rpl(n) is chosen per problem.  tol <= 0
// selects sqrt(n) u_w.
template <typename TW, typename TS, bool DDGRAM, int MAXRPL>
__global__ void __launch_bounds__(eig_bound(MAXRPL))
eig_batched_kernel(const BatchMat *__restrict__ tab, const int *__restrict__ order, int batch,
                   double tol, int max_sweeps, bool pre) {
    extern __shared__ __attribute__((aligned(16))) double lds[];
    __shared__ EigSmem sm;
    const BatchMat &d = tab[order[batch - 1 - (int)blockIdx.x]];
    const int n = d.n;
    const double u = sizeof(TW) == 8 ? 0x1p-53 : 0x1p-24;
    const double tol2 = tol > 0.0 ? tol * tol : (double)n * u * u;
    const double *Mlo = DDGRAM ? d.Mlo : nullptr;
#define GSVD_EIG_BODY(R)                                                                        \
    case R:                                                                                     \
        if (R <= MAXRPL)                                                                        \
            eig_body<TW, TS, DDGRAM, (R <= MAXRPL ? R : 2)>(                                    \
                n, d.Mhi, Mlo, n, (TW *)d.S, (TW *)d.V, d.ldv, (TW *)d.W, n, d.info, tol2,      \
                max_sweeps, pre, false, sm, lds);                                               \
        break;
    switch (eig_rpl(n)) {
        GSVD_EIG_BODY(2) GSVD_EIG_BODY(4) GSVD_EIG_BODY(6) GSVD_EIG_BODY(8)
        GSVD_EIG_BODY(10) GSVD_EIG_BODY(12) GSVD_EIG_BODY(14) GSVD_EIG_BODY(16)
        default: break;
    }
#undef GSVD_EIG_BODY
}

size_t eig_lds_bytes(int working, int64_t n) {
    const size_t chol = (size_t)(n * (n + 1)) * (working == 1 ? sizeof(dd_t) : sizeof(double));
    const size_t jac = working == 1 ? 2 * (size_t)(n * jac_ld<double>((int)n)) * sizeof(double)
                                    : 2 * (size_t)(n * jac_ld<float>((int)n)) * sizeof(float);
    return chol > jac ? chol : jac;
}

int eig_max_n(int working) { return working == 1 ? GSVD_KMAX_N_F64 : GSVD_KMAX_N; }

int eig_threads(int64_t n) {
    // the Jacobi uses GRP N2 / 2 lanes (N2 = n rounded up to a power of two); the
    // Cholesky and the repacking use all of them, so small problems get a small
    // workgroup and larger ones 1024 lanes
    const int N2 = eig_pow2((int)n);
    int t = GRP * (N2 / 2);
    if (n >= 32) t = eig_bound(eig_rpl((int)n));
    if (t < 64) t = 64;
    if (t > 1024) t = 1024;
    return ((t + 63) / 64) * 64;
}

template <typename TW, typename TS, bool DD, int RPL>
static hipError_t launch_rpl(int64_t n, const double *Mhi, const double *Mlo, int64_t ldm, void *S,
                             void *V, int64_t ldv, void *W, int64_t ldw, int *info, double tol2,
                             int max_sweeps, bool pre, size_t lds, int thr, hipStream_t st) {
    auto k = eig_chol_jacobi1_kernel<TW, TS, DD, RPL>;
    hipError_t err = hipFuncSetAttribute((const void *)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3(1), dim3(thr), lds, st, (int)n, Mhi, Mlo, ldm, (TW *)S, (TW *)V,
                       ldv, (TW *)W, ldw, info, tol2, max_sweeps, pre);
    return hipGetLastError();
}

template <typename TW, typename TS, bool DD>
static hipError_t launch_t(int64_t n, const double *Mhi, const double *Mlo, int64_t ldm, void *S,
                           void *V, int64_t ldv, void *W, int64_t ldw, int *info, double tol2,
                           int max_sweeps, bool pre, size_t lds, int thr, hipStream_t st) {
#define GSVD_EIG_CASE(R)                                                                       \
    case R:                                                                                    \
        return launch_rpl<TW, TS, DD, R>(n, Mhi, Mlo, ldm, S, V, ldv, W, ldw, info, tol2,     \
                                         max_sweeps, pre, lds, thr, st);
    switch (eig_rpl((int)n)) {
        GSVD_EIG_CASE(2)
        GSVD_EIG_CASE(4)
        GSVD_EIG_CASE(6)
        GSVD_EIG_CASE(8)
        GSVD_EIG_CASE(10)
        GSVD_EIG_CASE(12)
        GSVD_EIG_CASE(14)
        GSVD_EIG_CASE(16)
        default: return hipErrorInvalidValue;
    }
#undef GSVD_EIG_CASE
}

hipError_t eig_launch(int working, int64_t n, const double *Mhi, const double *Mlo, int64_t ldm,
                      void *S, void *V, int64_t ldv, void *W, int64_t ldw, int *info, double tol,
                      int max_sweeps, bool pre, hipStream_t st) {
    const size_t lds = eig_lds_bytes(working, n);
    const int thr = eig_threads(n);
    if (n < 1 || n > eig_max_n(working)) return hipErrorInvalidValue;
    if ((n * n + thr - 1) / thr > eig_maxreg(eig_rpl((int)n))) return hipErrorInvalidValue;
    if (thr / GRP < eig_pow2((int)n) / 2) return hipErrorInvalidValue;  // one group per pair
    const double tol2 = tol * tol;
    if (working == 1) {
        if (Mlo == nullptr) return hipErrorInvalidValue;
        return launch_t<double, double, true>(n, Mhi, Mlo, ldm, S, V, ldv, W, ldw, info, tol2,
                                              max_sweeps, pre, lds, thr, st);
    }
    if (pre) return hipErrorInvalidValue;
    return launch_t<float, float, false>(n, Mhi, Mlo, ldm, S, V, ldv, W, ldw, info, tol2,
                                         max_sweeps, false, lds, thr, st);
}

template <typename TW, typename TS, bool DD, int MAXRPL>
static hipError_t eig_batched_t(const BatchMat *tab, const int *order, int batch, size_t lds,
                                int thr, double tol, int max_sweeps, bool pre, hipStream_t st) {
    auto k = eig_batched_kernel<TW, TS, DD, MAXRPL>;
    hipError_t err = hipFuncSetAttribute((const void *)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3((unsigned)batch), dim3(thr), lds, st, tab, order, batch, tol,
                       max_sweeps, pre);
    return hipGetLastError();
}

hipError_t eig_batched_launch(int working, const BatchMat *tab, const int *order, int batch,
                              int max_n, double tol, int max_sweeps, bool pre, hipStream_t st) {
    if (batch < 1 || max_n < 1 || max_n > eig_max_n(working)) return hipErrorInvalidValue;
    const size_t lds = eig_lds_bytes(working, max_n);
    // every problem runs with the lanes and register depth of the largest one
    const bool big = eig_rpl(max_n) > 8;
    const int thr = big ? eig_bound(16) : eig_threads(max_n);
    if ((max_n * max_n + thr - 1) / thr > eig_maxreg(big ? 16 : 8)) return hipErrorInvalidValue;
    if (thr / GRP < eig_pow2(max_n) / 2) return hipErrorInvalidValue;  // one group per pair
    if (working == 1)
        return big ? eig_batched_t<double, double, true, 12>(tab, order, batch, lds, thr, tol,
                                                               max_sweeps, pre, st)
                   : eig_batched_t<double, double, true, 8>(tab, order, batch, lds, thr, tol,
                                                              max_sweeps, pre, st);
    if (pre) return hipErrorInvalidValue;
    return big ? eig_batched_t<float, float, false, 16>(tab, order, batch, lds, thr, tol,
                                                         max_sweeps, false, st)
               : eig_batched_t<float, float, false, 8>(tab, order, batch, lds, thr, tol,
                                                        max_sweeps, false, st);
}

}  // namespace gsvd

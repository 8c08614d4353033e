// Eigensolver stage for n > 96 with FP64 working: Algorithm 2 of the paper
// spread over many workgroups and a sequence of launches on one stream.
//
//   1. Column scaling (init kernels): e_j = ilogb(sqrt(m_jj)), the power of two
//      D~ of A = B D; H = D~^-1 M_h D~^-1 formed exactly in double-double;
//      checks for non-finite entries (info 3) and non-positive diagonals (info 1).
//   2. Cholesky H = R_H^T R_H in double-double (Alg. 2 step 1), blocked by
//      panels of 64 columns: for each panel
//        potrf  one workgroup factors the 64 x 64 diagonal block in LDS
//               (right-looking);
//        panel  R(k, j) = R_kk^-T H(k, j) for the columns j right of the panel
//               (forward substitution, right-looking: one workgroup per 16
//               columns, one lane per entry, 64 steps);
//        update H(i, j) -= R(k, i)^T R(k, j) for the trailing upper triangle
//               (32 x 32 tiles, one lane per entry, 64-deep dd sums).
//      A non-positive pivot stops the factorization with info 1.
//   3. X = fl64(R_H) D~ 2^-e_max (Alg. 2 step 2; exact scalings).
//   4. One-sided Jacobi on the columns of X (Alg. 2 step 3), block form: the
//      columns are cut into blocks of 16; a step pairs the blocks by a round-
//      robin tournament and gives each pair of blocks (32 columns of X, all n
//      rows) to one workgroup, which holds them in LDS and rotates the 256
//      pairs across the two blocks (16 rounds of 16 disjoint pairs, one
//      wavefront each); the first step of a tournament round, where every
//      block appears once, also rotates the 120 pairs inside each block (15
//      more rounds).  So every pair of columns is visited once
//      per round, as in a cyclic sweep.  In the cross rounds a block-P column
//      stays in the registers of its wavefront and only the block-Q columns
//      move through LDS.  The three inner products are summed by a cross-lane
//      reduction that leaves bitwise identical sums in every lane; the rotation
//      parameters use the hardware reciprocal and reciprocal square root
//      refined by Newton steps, as in the one-workgroup kernel.  The
//      rotations of a step accumulate in a 32 x 32 product Q, which goes to one of
//      two buffer slots: V never feeds back into the rotations, so the extra
//      workgroups of the next step's launch (one per 16 rows of V, on CUs the
//      rotations leave idle) apply it to V on the FP64 matrix cores, and a last
//      launch applies the final step's.  One launch per step; after each
//      tournament round a one-lane kernel marks convergence when no rotation
//      passed the test |x_p^T x_q| > tol ||x_p|| ||x_q||, and later launches
//      return at once.
//   5. sigma_p = ||x_p|| 2^e_max, ordering, sign of the V columns (entry of
//      largest magnitude positive, lowest index on ties), W = fl(V Sigma^-1).
//   The same outputs and info codes as the one-workgroup kernel for n <= 96.
//
// Preconditioner form (when the double-double Jacobi stage follows): the same
// steps on a reordered and transposed problem, stopped at a looser tolerance,
// whose only output is an eigenvector basis accurate in the graded sense.
//   1'. pi orders the columns by decreasing m_jj (a static form of the column
//      pivoting of a pivoted Cholesky); H' = P^T H P.
//   3'. X' = R' D~' 2^-emax as before, and the Jacobi runs on Z = X'^T: for a
//      row-graded triangular factor the columns of Z are far closer to
//      orthogonal than those of X', so fewer sweeps are needed (the idea of the
//      QR-preconditioned Jacobi SVD of Drmac and Veselic).  A step takes its
//      rotations on the block pair's Gram matrix G = X_b^T X_b (formed on the
//      FP64 matrix cores) as two-sided rotations G <- J^T G J, accumulates them in
//      Q and applies X_b <- X_b Q at the end (matrix cores again): the same
//      pairs and angles as the one-sided step, with the inner products updated
//      instead of summed over the n rows.  The last tournament round is the first whose
//      rotated pairs all had cosines below 2^-10 (quadratic convergence leaves
//      cosines of order 2^-20 or less, far inside the next stage's reach).
//   5'. Z Q = V' Sigma and X' = Q Sigma V'^T give V' = X'^-1 Q Sigma: V' comes
//      from a back substitution with R' and the exact scalings D~'^-1, which
//      keeps every column of V' accurate relative to its graded pattern
//      (normalising the columns of Z Q instead loses that: its errors are of
//      order u relative to the largest entry).  V = P V', columns normalised,
//      in no particular order or sign (the next stage sorts and signs).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "dd_device.hpp"
#include "gsvd_internal.hpp"
#include "jacobi_math.hpp"

namespace gsvd {

namespace {

constexpr int CB = 64;       // Cholesky panel width
constexpr int UT = 1024;     // update-kernel workgroup (32 x 32 tile)

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int MAXWG = 64;
// Preconditioner form: a tournament round whose rotated pairs all had
// |x_p^T x_q| < TAU_BIG ||x_p|| ||x_q|| is the last.  The Jacobi method converges
// quadratically, so the cosines it leaves are of order TAU_BIG^2 or smaller (below
// 1e-7 at the sizes measured), well inside the convergence of the double-double
// stage, which checks its own.
constexpr double TAU_BIG = 0x1p-10;    // Jacobi workgroups per step: ceil(512 / 16) / 2 = 16 at most

struct Ctl {
    int bad;      // info code of a failed check (1 or 3), 0 otherwise
    int emax;     // max e_j
    int done;     // converged
    int notconv;  // max_sweeps reached without convergence
    int abort;    // the output kernel must not write
    int qran[2];  // per product slot: the step launch whose rotations ran and were written
    int rot[MAXWG];  // per step workgroup, this tournament round: 0 no rotation, 1 only
                     // pairs with cosine < TAU_BIG rotated, 2 a larger one
};

struct WLayout {
    size_t ctl, sexp, rank, perm, sig, sgn, hh, hl, x, v, qbuf, dinv, total;
};

constexpr int JBW = 16;  // Jacobi block width of the launches (8 measured no faster at n = 512)

// blocks of the tournament (an even count; an odd one gets a bye block)
__host__ __device__ inline int jac_nblk(int n) {
    const int nbb = (n + JBW - 1) / JBW;
    return nbb + (nbb & 1);
}

__host__ __device__ inline size_t wal(size_t x) { return (x + 255) / 256 * 256; }

WLayout wlayout(int64_t n) {
    WLayout L{};
    size_t o = 0;
    const size_t nn = (size_t)n * (size_t)n;
    L.ctl = o;  o = wal(o + sizeof(Ctl));
    L.sexp = o; o = wal(o + (size_t)n * sizeof(int));
    L.rank = o; o = wal(o + (size_t)n * sizeof(int));
    L.perm = o; o = wal(o + (size_t)n * sizeof(int));
    L.sig = o;  o = wal(o + (size_t)n * sizeof(double));
    L.sgn = o;  o = wal(o + (size_t)n * sizeof(double));
    L.hh = o;   o = wal(o + nn * sizeof(double));
    L.hl = o;   o = wal(o + nn * sizeof(double));
    L.x = o;    o = wal(o + nn * sizeof(double));
    L.v = o;    o = wal(o + nn * sizeof(double));
    const int nblk = jac_nblk((int)n);
    L.qbuf = o; o = wal(o + (size_t)2 * (nblk / 2) * (4 * JBW * JBW) * sizeof(double));
    L.dinv = o; o = wal(o + (size_t)((n + 63) / 64) * 64 * 64 * sizeof(double));
    L.total = o;
    return L;
}

// A control word written by an earlier launch (no lane of the reading launch
// writes it first, so every lane reads the same value).
__device__ __forceinline__ int wg_read(const int *p) {
    return __builtin_amdgcn_readfirstlane(*reinterpret_cast<const volatile int *>(p));
}

// ---- 1. scaling exponents, checks, H, V = I

// Also the order pi of the preconditioner form: perm[r] is the column of rank r
// by decreasing m_jj, ties by index (a total order: rejected diagonals count as
// 0, so perm is a permutation whatever the input).
__global__ void __launch_bounds__(1024)
weig_diag_kernel(int n, const double *__restrict__ Mhi, int64_t ldm, Ctl *ctl, int *sexp,
                 int *perm) {
    __shared__ int bad, emax;
    __shared__ double key[GSVD_WIDE_MAX_N];
    if (threadIdx.x == 0) {
        bad = 0;
        emax = -100000;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < MAXWG; t += blockDim.x) ctl->rot[t] = 0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double mjj = Mhi[j + (int64_t)j * ldm];
        if (!(mjj > 0.0) || !__builtin_isfinite(mjj)) {
            atomicMax(&bad, __builtin_isfinite(mjj) ? 1 : 3);
            sexp[j] = 0;
            key[j] = 0.0;
        } else {
            const int e = ilogb(__builtin_sqrt(mjj));
            sexp[j] = e;
            key[j] = mjj;
            atomicMax(&emax, e);
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double kj = key[j];
        int r = 0;
        for (int q = 0; q < n; ++q) r += (key[q] > kj) || (key[q] == kj && q < j);
        perm[r] = j;
    }
    if (threadIdx.x == 0) {
        ctl->bad = bad;
        ctl->emax = emax;
        ctl->done = 0;
        ctl->notconv = 0;
        ctl->abort = 0;
        ctl->qran[0] = -1;
        ctl->qran[1] = -1;
    }
}

// one workgroup per column j: finiteness of column j, H(:, j) (upper part), V(:, j) = e_j.
// perm non-null (the preconditioner form): H'(:, j) = H(pi, pi_j), read from the
// upper triangle of M_h.
__global__ void __launch_bounds__(256)
weig_fill_kernel(int n, const double *__restrict__ Mhi, const double *__restrict__ Mlo,
                 int64_t ldm, Ctl *ctl, const int *__restrict__ sexp, const int *__restrict__ perm,
                 double *__restrict__ Hh, double *__restrict__ Hl, double *__restrict__ Vw) {
    const int j = blockIdx.x;
    const int pj = perm ? perm[j] : j;
    bool nonfinite = false;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        if (!__builtin_isfinite(Mhi[i + (int64_t)j * ldm]) ||
            !__builtin_isfinite(Mlo[i + (int64_t)j * ldm]))
            nonfinite = true;
        if (i <= j) {
            const int pi = perm ? perm[i] : i;
            const int a = pi < pj ? pi : pj, b = pi < pj ? pj : pi;
            const int sc = -(sexp[pi] + sexp[pj]);
            Hh[i + (size_t)j * n] = ldexp(Mhi[a + (int64_t)b * ldm], sc);
            Hl[i + (size_t)j * n] = ldexp(Mlo[a + (int64_t)b * ldm], sc);
        }
        Vw[i + (size_t)j * n] = i == j ? 1.0 : 0.0;
    }
    if (nonfinite) atomicMax(&ctl->bad, 3);
}

// ---- 2. blocked dd Cholesky

// 1 / h in double-double: the FP64 estimate r corrected once, r + r (1 - h r)
__device__ __forceinline__ dd_t dd_rcp(dd_t h) {
    const double r0 = rcp_nr(h.hi);
    const dd_t hr = dd_mul_d(h, r0);
    const double e = (1.0 - hr.hi) - hr.lo;
    return quick_two_sum(r0, r0 * e);
}

// Factor the diagonal block [k0, k0 + 64) in place (upper triangle), right-looking
// in the square-root-free form h_ij -= h_ki (h_kj / h_kk) over k < i <= j, one
// barrier per column: each lane owns fixed entries of the triangle (at most 3), the
// owner of the next pivot also forms its reciprocal.  Row k of R is then
// h_kj / sqrt(h_kk), formed for all rows at once.
__global__ void __launch_bounds__(1024)
weig_potrf_kernel(int n, int k0, Ctl *ctl, double *__restrict__ Hh, double *__restrict__ Hl) {
    extern __shared__ __attribute__((aligned(16))) unsigned char wsm[];
    dd_t *Rs = reinterpret_cast<dd_t *>(wsm);  // CB x CB, column-major
    dd_t *rp = Rs + CB * CB;                    // reciprocal pivots
    if (wg_read(&ctl->bad)) return;
    const int nb = (n - k0 < CB) ? n - k0 : CB;
    const int tid = threadIdx.x;
    for (int q = tid; q < CB * CB; q += blockDim.x) {
        const int i = q % CB, j = q / CB;
        dd_t v{0.0, 0.0};
        if (i < nb && j < nb && i <= j)
            v = dd_t{Hh[(k0 + i) + (size_t)(k0 + j) * n], Hl[(k0 + i) + (size_t)(k0 + j) * n]};
        Rs[q] = v;
    }
    // the lane's entries (i, j), i <= j, numbered q = j (j + 1) / 2 + i
    constexpr int NE = (CB * (CB + 1) / 2 + 1023) / 1024;
    int ei[NE], ej[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const int q = tid + 1024 * e;
        int j = (int)((__builtin_sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f);
        while (j * (j + 1) / 2 > q) --j;
        while ((j + 1) * (j + 2) / 2 <= q) ++j;
        ei[e] = q - j * (j + 1) / 2;
        ej[e] = j < CB ? j : CB;  // CB: no entry
    }
    __syncthreads();
    if (tid == 0) rp[0] = dd_rcp(Rs[0]);
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
        if (!(Rs[k + k * CB].hi > 0.0)) {  // uniform: every lane read the same LDS word
            if (tid == 0) atomicMax(&ctl->bad, 1);
            return;
        }
        const dd_t rinv = rp[k];
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const int i = ei[e], j = ej[e];
            if (i > k && j < nb) {
                const dd_t v = dd_sub(Rs[i + j * CB], dd_mul(Rs[k + i * CB], dd_mul(Rs[k + j * CB], rinv)));
                Rs[i + j * CB] = v;
                if (i == k + 1 && j == k + 1) rp[k + 1] = dd_rcp(v);
            }
        }
        __syncthreads();
    }
    // r_kj = h_kj / sqrt(h_kk): 1 / sqrt(h) as y + y (1 - h y^2) / 2 from the FP64 estimate
    if (tid < nb) {
        const dd_t hkk = Rs[tid + tid * CB];
        const double y = rsq_nr(hkk.hi);
        const dd_t hy2 = dd_mul_d(dd_mul_d(hkk, y), y);
        rp[tid] = dd_add(dd_t{y, 0.0}, dd_mul_d(dd_sub(dd_t{1.0, 0.0}, hy2), 0.5 * y));
    }
    __syncthreads();
    for (int q = tid; q < CB * CB; q += blockDim.x) {
        const int i = q % CB, j = q / CB;
        if (i < nb && j < nb && i <= j) {
            const dd_t r = dd_mul(Rs[q], rp[i]);
            Hh[(k0 + i) + (size_t)(k0 + j) * n] = r.hi;
            Hl[(k0 + i) + (size_t)(k0 + j) * n] = r.lo;
        }
    }
}

// R(k0 + i, j) for the 16 columns j0 .. j0 + 15 right of the panel: solve
// R_kk^T x = H(k0 .. k0 + 63, j) by forward substitution, right-looking: step t
// forms x_t = h_t / R(t, t) (times the reciprocal of R(t, t)), then h_i -= R(t, i) x_t
// for i > t.  Lane (i, c) keeps h_i of column c in registers; x_t reaches the
// other lanes through its own LDS slot, so each step needs one barrier.
__global__ void __launch_bounds__(1024)
weig_panel_kernel(int n, int k0, const Ctl *ctl, double *__restrict__ Hh,
                  double *__restrict__ Hl) {
    extern __shared__ __attribute__((aligned(16))) unsigned char wsm[];
    dd_t *Rk = reinterpret_cast<dd_t *>(wsm);  // CB x CB, column-major (upper)
    dd_t *rd = Rk + CB * CB;                    // 1 / R(t, t)
    dd_t *xs = rd + CB;                         // CB x 16 solved values
    if (wg_read(&ctl->bad)) return;
    const int tid = threadIdx.x;
    const int j0 = k0 + CB + 16 * blockIdx.x;
    for (int q = tid; q < CB * CB; q += blockDim.x) {
        const int i = q % CB, j = q / CB;
        Rk[q] = i <= j ? dd_t{Hh[(k0 + i) + (size_t)(k0 + j) * n], Hl[(k0 + i) + (size_t)(k0 + j) * n]}
                       : dd_t{0.0, 0.0};
    }
    const int i = tid % CB, c = tid / CB;  // 64 rows x 16 columns
    const int j = j0 + c;
    const bool jv = j < n;
    dd_t h = jv ? dd_t{Hh[(k0 + i) + (size_t)j * n], Hl[(k0 + i) + (size_t)j * n]} : dd_t{0.0, 0.0};
    __syncthreads();
    if (tid < CB) rd[tid] = dd_rcp(Rk[tid + tid * CB]);
    __syncthreads();
    for (int t = 0; t < CB; ++t) {
        if (i == t) {
            h = dd_mul(h, rd[t]);
            xs[t + c * CB] = h;
        }
        __syncthreads();
        if (i > t) h = dd_sub(h, dd_mul(Rk[t + i * CB], xs[t + c * CB]));
    }
    if (jv) {
        Hh[(k0 + i) + (size_t)j * n] = h.hi;
        Hl[(k0 + i) + (size_t)j * n] = h.lo;
    }
}

// H(i, j) -= sum_{t < CB} R(k0 + t, i) R(k0 + t, j), k1 <= i <= j < n, in 32 x 32 tiles
__global__ void __launch_bounds__(UT)
weig_update_kernel(int n, int k0, int ntile, const Ctl *ctl, double *__restrict__ Hh,
                   double *__restrict__ Hl) {
    extern __shared__ __attribute__((aligned(16))) unsigned char wsm[];
    dd_t *Ri = reinterpret_cast<dd_t *>(wsm);  // CB x 32
    dd_t *Rj = Ri + CB * 32;
    if (wg_read(&ctl->bad)) return;
    // tile (ti, tj), ti <= tj, of the trailing square
    int ti = 0, rem = blockIdx.x;
    while (rem >= ntile - ti) {
        rem -= ntile - ti;
        ++ti;
    }
    const int tj = ti + rem;
    const int k1 = k0 + CB;
    const int i0 = k1 + 32 * ti, j0 = k1 + 32 * tj;
    const int tid = threadIdx.x;
    for (int q = tid; q < CB * 32; q += blockDim.x) {
        const int t = q % CB, c = q / CB;
        const int ci = i0 + c, cj = j0 + c;
        Ri[q] = ci < n ? dd_t{Hh[(k0 + t) + (size_t)ci * n], Hl[(k0 + t) + (size_t)ci * n]}
                       : dd_t{0.0, 0.0};
        Rj[q] = cj < n ? dd_t{Hh[(k0 + t) + (size_t)cj * n], Hl[(k0 + t) + (size_t)cj * n]}
                       : dd_t{0.0, 0.0};
    }
    __syncthreads();
    const int li = tid % 32, lj = tid / 32;
    const int i = i0 + li, j = j0 + lj;
    if (i < n && j < n && i <= j) {
        dd_t s{0.0, 0.0};
        for (int t = 0; t < CB; ++t) s = dd_add(s, dd_mul(Ri[t + li * CB], Rj[t + lj * CB]));
        const dd_t h{Hh[i + (size_t)j * n], Hl[i + (size_t)j * n]};
        const dd_t r = dd_sub(h, s);
        Hh[i + (size_t)j * n] = r.hi;
        Hl[i + (size_t)j * n] = r.lo;
    }
}

// ---- 3. X = fl64(R_H) D~ 2^-emax (upper triangle; zeros below).  perm non-null:
//      X' = fl64(R') D~' 2^-emax stored transposed (Z = X'^T, lower triangular).
__global__ void __launch_bounds__(256)
weig_cast_kernel(int n, const Ctl *ctl, const int *__restrict__ sexp,
                 const int *__restrict__ perm, const double *__restrict__ Hh,
                 double *__restrict__ X) {
    if (wg_read(&ctl->bad)) return;
    const int j = blockIdx.x;
    const int sc = sexp[perm ? perm[j] : j] - ctl->emax;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double x = i <= j ? ldexp(Hh[i + (size_t)j * n], sc) : 0.0;
        if (perm)
            X[j + (size_t)i * n] = x;
        else
            X[i + (size_t)j * n] = x;
    }
}

// ---- 4. block one-sided Jacobi

template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double readlane_d(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the wavefront, the same bits in every lane: within each row of 16
// lanes xor 1, xor 2 (quad permutes), the half-row mirror and the row mirror
// (each step adds two lanes holding the same partials in swapped order), then
// the four row sums read out of lanes 0, 16, 32, 48 and added in a fixed order.
__device__ __forceinline__ double wave_sum(double x) {
    x += dpp_d<0xB1>(x);
    x += dpp_d<0x4E>(x);
    x += dpp_d<0x141>(x);
    x += dpp_d<0x140>(x);
    return (readlane_d(x, 0) + readlane_d(x, 16)) + (readlane_d(x, 32) + readlane_d(x, 48));
}

// round-robin tournament on m (even) players: pair g of round r
__device__ __forceinline__ void rr_pair(int r, int g, int m, int &p, int &q) {
    if (g == 0) {
        p = r;
        q = m - 1;
    } else {
        p = (r + g) % (m - 1);
        q = (r - g + (m - 1)) % (m - 1);
    }
}

// JB: Jacobi block width (columns); a workgroup holds JC = 2 JB columns and has
// one wavefront per column pair of a round; Q's column stride QLD = JC + 2 keeps
// the matrix-core operand reads free of bank conflicts.
template <int JB>
struct JGeom {
    static constexpr int JC = 2 * JB;
    static constexpr int JT = 64 * JB;
    static constexpr int QLD = JC + 2;
};

template <int JB>
__device__ __forceinline__ void vapply_prev(int n, int nblk, int g, const Ctl *ctl,
                                            const double *__restrict__ Qbuf,
                                            double *__restrict__ Vw, int vb, double *vsm);

// Step launch g (= round * (nblk - 1) + step) of Algorithm 2: workgroups 0 ..
// nblk/2 - 1 run the step's one-sided rotations (every round sums the three inner
// products of its pair afresh) and write their products to slot g & 1; the rest (one
// per 16 rows of V) apply the products of launch g - 1 to V meanwhile, on other CUs.
template <int RPL, int JB>
__global__ void __launch_bounds__(64 * JB)
weig_step_kernel(int n, int nblk, int step, int g, Ctl *ctl, double *__restrict__ X,
                 double *__restrict__ Qbuf, double *__restrict__ Vw, double tol2) {
    extern __shared__ __attribute__((aligned(16))) double jsm[];
    constexpr int JC = JGeom<JB>::JC, JT = JGeom<JB>::JT, QLD = JGeom<JB>::QLD;
    constexpr int LDL = 64 * RPL;  // rows of a column in LDS (n rounded up to 64)
    double *Xl = jsm;              // JC columns of X
    double *Qs = jsm + JC * LDL;   // JC x JC rotation product, column-major, stride QLD
    if ((int)blockIdx.x >= nblk / 2) {
        vapply_prev<JB>(n, nblk, g, ctl, Qbuf, Vw, (int)blockIdx.x - nblk / 2, jsm);
        return;
    }
    if (wg_read(&ctl->bad) || wg_read(&ctl->done)) return;
    // this launch's rotations run (done and bad are the same for all its workgroups)
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->qran[g & 1] = g;
    int P, Qb;
    rr_pair(step, blockIdx.x, nblk, P, Qb);
    const int nbb = (n + JB - 1) / JB;
    // the bye of an odd block count: its partner still rotates its own pairs in the
    // first step (the bye's columns read as zeros, and zero columns never rotate)
    if ((P >= nbb && Qb >= nbb) || ((P >= nbb || Qb >= nbb) && step != 0)) return;
    const int tid = threadIdx.x;
    auto gcol = [&](int c) { return c < JB ? JB * P + c : JB * Qb + (c - JB); };
    constexpr int NLD = JC * LDL / JT;  // block values per lane
    // stage the 16 columns of a matrix (X or V) into Xl: every load issued first
    auto stage = [&](const double *__restrict__ src) {
        double v[NLD];
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int q = tid + k * JT;
            const int r = q % LDL, g = gcol(q / LDL);
            v[k] = (r < n && g < n) ? src[r + (size_t)g * n] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < NLD; ++k) Xl[tid + k * JT] = v[k];
    };
    stage(X);
    for (int q = tid; q < JC * QLD; q += JT) Qs[q] = (q % QLD == q / QLD) ? 1.0 : 0.0;
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6;
    int any = 0;  // 1: a rotation, 2: one of a pair with cosine >= TAU_BIG
    // one plane rotation of columns x0 (p) and x1 (q), held in registers; also on Q
    auto rotate = [&](double (&x0)[RPL], double (&x1)[RPL], int p, int q) -> bool {
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            al = __builtin_fma(x0[i], x0[i], al);
            be = __builtin_fma(x1[i], x1[i], be);
            ga = __builtin_fma(x0[i], x1[i], ga);
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        if (!(ga * ga > tol2 * (al * be))) return false;  // uniform: the sums agree bitwise
        double c, sn;
        jacobi_cs(al, be, ga, c, sn);
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const double a0 = x0[i], a1 = x1[i];
            x0[i] = __builtin_fma(c, a0, -(sn * a1));
            x1[i] = __builtin_fma(c, a1, sn * a0);
        }
        if (lane < JC) {
            const double u = Qs[lane + p * QLD], w = Qs[lane + q * QLD];
            Qs[lane + p * QLD] = __builtin_fma(c, u, -(sn * w));
            Qs[lane + q * QLD] = __builtin_fma(c, w, sn * u);
        }
        if (ga * ga >= (TAU_BIG * TAU_BIG) * (al * be)) any = 2;
        else if (any == 0) any = 1;
        return true;
    };
    double x0[RPL], x1[RPL];
    // first step of a round: the pairs inside block P (wavefronts 0 .. JB/2-1) and
    // inside block Q, both columns from LDS
    if (step == 0) {
        for (int round = 0; round < JB - 1; ++round) {
            const int h = wave / (JB / 2), g = wave % (JB / 2);
            int p, q;
            rr_pair(round, g, JB, p, q);
            p += JB * h;
            q += JB * h;
            double *xp = Xl + p * LDL + lane, *xq = Xl + q * LDL + lane;
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                x0[i] = xp[64 * i];
                x1[i] = xq[64 * i];
            }
            if (rotate(x0, x1, p, q)) {
#pragma unroll
                for (int i = 0; i < RPL; ++i) {
                    xp[64 * i] = x0[i];
                    xq[64 * i] = x1[i];
                }
            }
            __syncthreads();
        }
    }
    // the cross pairs (i, JB + (i + r) mod JB): column i of block P stays in the
    // registers of wavefront i for all JB rounds; the block-Q columns travel
    {
        const int p = wave;
        double *xp = Xl + p * LDL + lane;
#pragma unroll
        for (int i = 0; i < RPL; ++i) x0[i] = xp[64 * i];
        for (int r = 0; r < JB; ++r) {
            const int q = JB + (wave + r) % JB;
            double *xq = Xl + q * LDL + lane;
#pragma unroll
            for (int i = 0; i < RPL; ++i) x1[i] = xq[64 * i];
            if (rotate(x0, x1, p, q)) {
#pragma unroll
                for (int i = 0; i < RPL; ++i) xq[64 * i] = x1[i];
            }
            __syncthreads();  // the travelers move on
        }
#pragma unroll
        for (int i = 0; i < RPL; ++i) xp[64 * i] = x0[i];
    }
    __syncthreads();
    // X back; the step's rotation product Q (JC x JC, row-major) to its slot of the
    // round's buffer (applied to V once the round is over)
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
        const int q = tid + k * JT;
        const int r = q % LDL, g = gcol(q / LDL);
        if (r < n && g < n) X[r + (size_t)g * n] = Xl[q];
    }
    double *Qo = Qbuf + ((size_t)(g & 1) * (nblk / 2) + blockIdx.x) * (JC * JC);
    for (int q = tid; q < JC * JC; q += JT) Qo[q] = Qs[(q / JC) + (q % JC) * QLD];
    // one plain store per workgroup into its own word (no contended atomics); the
    // word holds the largest level of the round's earlier steps (earlier launches)
    const bool big = __syncthreads_or(any == 2), some = __syncthreads_or(any != 0);
    const int lvl = big ? 2 : (some ? 1 : 0);
    if (tid == 0 && lvl > ctl->rot[blockIdx.x]) ctl->rot[blockIdx.x] = lvl;
}

// end of a tournament round (one wavefront): converged when no workgroup rotated
// (early: or when no rotated pair had a cosine of TAU_BIG); the flags are cleared for
// the next round
__global__ void __launch_bounds__(64) weig_sweep_kernel(Ctl *ctl, int nwg, int last, int early) {
    const int t = threadIdx.x;
    if (ctl->bad || ctl->done) return;  // written by earlier launches only
    const int r = t < nwg ? ctl->rot[t] : 0;
    const bool anyrot = __any(r != 0), anybig = __any(r == 2);
    if (t < nwg) ctl->rot[t] = 0;
    if (t == 0) {
        if (!anyrot || (early && !anybig)) ctl->done = 1;
        else if (last) ctl->notconv = 1;
    }
}

// V <- V Q for the products of one step (the rotations never feed back into the
// Jacobi, so V follows a step behind).  A workgroup of 16 wavefronts holds 16 rows
// of V in LDS; wavefront b applies the product of step workgroup b to the 32
// columns of its block pair on the FP64 matrix cores (the pairs of a step are
// disjoint).  Operands (16x16x4): lane l supplies V(l % 16, k0 + l / 16) and
// Q(k0 + l / 16, c0 + l % 16) (Q row-major: four 128-byte runs per read); result
// register r is (V Q)(4 r + l / 16, c0 + l % 16).
constexpr int VRW = 16;  // rows of V per workgroup

// Preconditioner form of a step: the same rotations, taken on the block pair's Gram
// matrix.  G = X_b^T X_b (JC x JC) comes from the FP64 matrix cores; each round's
// rotations J then act on both sides, G <- J^T G J, and on Q <- Q J, one entry per
// lane (an entry of G from the same four-term formula for (a, b) and (b, a), so G
// stays exactly symmetric); at the end X_b <- X_b Q on the matrix cores.  A round
// costs two short LDS passes instead of sums over the n rows of both columns.  The
// inner products are those of the current columns up to the rounding of the
// two-sided updates, the accuracy a preconditioner needs (the dd stage then works
// at u_h).
template <int RPL, int JB>
__global__ void __launch_bounds__(64 * JB)
weig_gstep_kernel(int n, int nblk, int step, int g, Ctl *ctl, double *__restrict__ X,
                  double *__restrict__ Qbuf, double *__restrict__ Vw, double tol2) {
    extern __shared__ __attribute__((aligned(16))) double jsm[];
    constexpr int JC = JGeom<JB>::JC, JT = JGeom<JB>::JT;
    static_assert(JT >= JC * JC && JT >= 3 * 64, "one lane per entry of G and Q");
    constexpr int LDL = 64 * RPL;  // rows of a column (n rounded up to 64)
    constexpr int LDP = LDL + 1;   // column stride in LDS: a row's columns in distinct banks
    double *Xl = jsm;              // JC columns of X
    double *G = Xl + JC * LDP;     // JC x JC, column-major, two buffers (rounds alternate)
    double *Qm = G + 2 * JC * JC;  // JC x JC rotation product, row-major
    double *cr = Qm + JC * JC;     // per column: the cosine of its pair this round
    double *tr = cr + JC;          // per column: the coefficient of its partner
    int *pr = reinterpret_cast<int *>(tr + JC);  // per column: its partner this round
    if ((int)blockIdx.x >= nblk / 2) {
        vapply_prev<JB>(n, nblk, g, ctl, Qbuf, Vw, (int)blockIdx.x - nblk / 2, jsm);
        return;
    }
    if (wg_read(&ctl->bad) || wg_read(&ctl->done)) return;
    // this launch's rotations run (done and bad are the same for all its workgroups)
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->qran[g & 1] = g;
    int P, Qb;
    rr_pair(step, blockIdx.x, nblk, P, Qb);
    const int nbb = (n + JB - 1) / JB;
    if ((P >= nbb && Qb >= nbb) || ((P >= nbb || Qb >= nbb) && step != 0)) return;
    const int tid = threadIdx.x;
    auto gcol = [&](int c) { return c < JB ? JB * P + c : JB * Qb + (c - JB); };
    constexpr int NLD = JC * LDL / JT;  // block values per lane
    {
        double v[NLD];
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int q = tid + k * JT;
            const int r = q % LDL, gc = gcol(q / LDL);
            v[k] = (r < n && gc < n) ? X[r + (size_t)gc * n] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int q = tid + k * JT;
            Xl[(q / LDL) * LDP + q % LDL] = v[k];
        }
    }
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    // G: wavefronts 0 .. 11 form the tiles (0, 0), (0, 1), (1, 1) (tile = w mod 3) over
    // the four quarters of the rows (w / 3), four accumulators each (k mod 16 in steps
    // of 4); the quarters' partial tiles pass through the second G buffer and Q, and
    // are summed in a fixed order, (q0 + q1) + (q2 + q3)
    static_assert(JT >= 12 * 64 && 3 * JC * JC >= 2 * 768 + JC * JC, "G's wavefronts and scratch");
    const int gtile = wave % 3, gq = wave / 3;
    double gv[4] = {0.0, 0.0, 0.0, 0.0};
    double *gpart = G + JC * JC;  // 2 x 768 doubles over the second G buffer and Q
    if (wave < 12) {
        const int I = gtile == 2 ? 1 : 0, J = gtile == 0 ? 0 : 1;
        const double *xa = Xl + (16 * I + li) * LDP + lk;
        const double *xb = Xl + (16 * J + li) * LDP + lk;
        f64x4 acc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = f64x4{0.0, 0.0, 0.0, 0.0};
        for (int k0 = gq * (LDL / 4); k0 < (gq + 1) * (LDL / 4); k0 += 16) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[k0 + 4 * u], xb[k0 + 4 * u],
                                                              acc[u], 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            gv[r] = (acc[0][r] + acc[1][r]) + (acc[2][r] + acc[3][r]);
            if (gq & 1) gpart[(gq >> 1) * 768 + (gtile * 4 + r) * 64 + lane] = gv[r];
        }
    }
    __syncthreads();
    if (wave < 12 && !(gq & 1)) {  // q0 + q1, q2 + q3
#pragma unroll
        for (int r = 0; r < 4; ++r) gv[r] += gpart[(gq >> 1) * 768 + (gtile * 4 + r) * 64 + lane];
    }
    __syncthreads();
    if (wave < 12 && gq == 2) {
#pragma unroll
        for (int r = 0; r < 4; ++r) gpart[(gtile * 4 + r) * 64 + lane] = gv[r];
    }
    __syncthreads();
    if (wave < 3) {
        const int I = gtile == 2 ? 1 : 0, J = gtile == 0 ? 0 : 1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double v = gv[r] + gpart[(gtile * 4 + r) * 64 + lane];
            const int i = 16 * I + 4 * r + lk, j = 16 * J + li;
            if (i <= j) {
                G[i + JC * j] = v;
                G[j + JC * i] = v;
            }
        }
    }
    __syncthreads();
    for (int q = tid; q < JC * JC; q += JT) Qm[q] = (q / JC == q % JC) ? 1.0 : 0.0;
    __syncthreads();

    int any = 0;  // 1: a rotation, 2: one of a pair with cosine >= TAU_BIG
    // lane (a, b) of G (a = tid % JC) and (i, j) of Q (j = tid % JC; row i of Q lies in
    // one wavefront, so Q is updated in place: its reads come before its writes).  Entry (a, b) of
    // J^T G J is formed from (a0, b0) = (min, max) in one order, for both triangles;
    // its four inputs G(x, y), x in {a, pa}, y in {b, pb}, are read as G[x + JC y]
    // (G is symmetric), so the lanes of a wavefront read along columns
    const bool ent = tid < JC * JC;
    const int ga_ = tid % JC, gb_ = tid / JC;
    const bool low = ga_ > gb_;  // (a0, b0) = (b, a)
    const int a0 = low ? gb_ : ga_, b0 = low ? ga_ : gb_;
    const int qi = tid / JC, qj = tid % JC;
    // one round: pair k (k < JB) of the round is (p, q); p's partner enters with -s
    int cur = 0;  // G's buffer of this round
    auto round = [&](auto pair_of) {
        const double *Gc = G + cur * (JC * JC);
        double *Gn = G + (cur ^ 1) * (JC * JC);
        if (wave == 0 && lane < JB) {
            int p, q;
            pair_of(lane, p, q);
            const double al = Gc[p + JC * p], be = Gc[q + JC * q], gpq = Gc[p + JC * q];
            double c = 1.0, sn = 0.0;
            if (gpq * gpq > tol2 * (al * be)) {
                jacobi_cs(al, be, gpq, c, sn);
                const int lv = gpq * gpq >= (TAU_BIG * TAU_BIG) * (al * be) ? 2 : 1;
                any = any > lv ? any : lv;
            }
            cr[p] = c;
            tr[p] = -sn;
            pr[p] = q;
            cr[q] = c;
            tr[q] = sn;
            pr[q] = p;
        }
        __syncthreads();
        if (ent) {
            const int pa = pr[ga_], pb = pr[gb_];  // partners of a and b
            const double ca = cr[a0], ta = tr[a0], cb = cr[b0], tb = tr[b0];
            // G(a0, b0), G(a0, p b0), G(p a0, b0), G(p a0, p b0)
            const double g00 = Gc[ga_ + JC * gb_];
            const double g01 = low ? Gc[pa + JC * gb_] : Gc[ga_ + JC * pb];
            const double g10 = low ? Gc[ga_ + JC * pb] : Gc[pa + JC * gb_];
            const double g11 = Gc[pa + JC * pb];
            Gn[ga_ + JC * gb_] = __builtin_fma(ta * tb, g11, __builtin_fma(ta * cb, g10,
                                               __builtin_fma(ca * tb, g01, (ca * cb) * g00)));
            const int pj = pr[qj];
            const double q0 = Qm[qi * JC + qj], q1 = Qm[qi * JC + pj];
            Qm[qi * JC + qj] = __builtin_fma(tr[qj], q1, cr[qj] * q0);
        }
        cur ^= 1;
        __syncthreads();
    };
    if (step == 0) {  // the pairs inside block P and inside block Q
        for (int r = 0; r < JB - 1; ++r)
            round([&](int k, int &p, int &q) {
                const int h = k / (JB / 2);
                rr_pair(r, k % (JB / 2), JB, p, q);
                p += JB * h;
                q += JB * h;
            });
    }
    for (int r = 0; r < JB; ++r)  // the cross pairs (k, JB + (k + r) mod JB)
        round([&](int k, int &p, int &q) {
            p = k;
            q = JB + (k + r) % JB;
        });

    // X <- X Q: wavefront w takes row tiles w, w + JT / 64, ... (all JC columns), and
    // writes its rows back in place once it has read them
    for (int ti = wave; ti < LDL / 16; ti += JT / 64) {
        f64x4 acc[JC / 16];
#pragma unroll
        for (int t = 0; t < JC / 16; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k0 = 0; k0 < JC; k0 += 4) {
            const double av = Xl[(k0 + lk) * LDP + 16 * ti + li];
#pragma unroll
            for (int t = 0; t < JC / 16; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Qm[(k0 + lk) * JC + 16 * t + li],
                                                              acc[t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < JC / 16; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) Xl[(16 * t + li) * LDP + 16 * ti + 4 * r + lk] = acc[t][r];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
        const int q = tid + k * JT;
        const int r = q % LDL, gc = gcol(q / LDL);
        if (r < n && gc < n) X[r + (size_t)gc * n] = Xl[(q / LDL) * LDP + r];
    }
    double *Qo = Qbuf + ((size_t)(g & 1) * (nblk / 2) + blockIdx.x) * (JC * JC);
    for (int q = tid; q < JC * JC; q += JT) Qo[q] = Qm[q];
    const bool big = __syncthreads_or(any == 2), some = __syncthreads_or(any != 0);
    const int lvl = big ? 2 : (some ? 1 : 0);
    if (tid == 0 && lvl > ctl->rot[blockIdx.x]) ctl->rot[blockIdx.x] = lvl;
}

template <int JB>
__device__ __forceinline__ void vapply_step(int n, int nblk, int st, const double *__restrict__ Qs,
                                            double *__restrict__ Vw, int r0, double *vsm) {
    constexpr int JC = JGeom<JB>::JC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int q = tid; q < VRW * n; q += 64 * JB) {
        const int r = q % VRW, c = q / VRW;
        vsm[q] = (r0 + r < n) ? Vw[(r0 + r) + (size_t)c * n] : 0.0;
    }
    __syncthreads();
    const int nbb = (n + JB - 1) / JB;
    const int npair = nblk / 2;
    const int li = lane & 15, lk = lane >> 4;
    int P = 0, Qb = 0;
    if (wave < npair) rr_pair(st, wave, nblk, P, Qb);
    // the step kernel's own early return (a bye block) wrote no product
    const bool act = wave < npair && !((P >= nbb && Qb >= nbb) ||
                                        ((P >= nbb || Qb >= nbb) && st != 0));
    if (act) {  // uniform per wavefront
        auto gcol = [&](int c) { return c < JB ? JB * P + c : JB * Qb + (c - JB); };
        const double *Q = Qs + (size_t)wave * (JC * JC);
        double b0[JC / 4], b1[JC / 4];
#pragma unroll
        for (int k = 0; k < JC / 4; ++k) {  // every operand load issued first
            b0[k] = Q[li + (4 * k + lk) * JC];
            b1[k] = Q[(16 + li) + (4 * k + lk) * JC];
        }
        f64x4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < JC / 4; ++k) {
            const int gk = gcol(4 * k + lk);
            const double a = gk < n ? vsm[li + gk * VRW] : 0.0;
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b0[k], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b1[k], acc1, 0, 0, 0);
        }
        // (this wavefront alone reads and writes the pair's columns: its reads above
        // precede these writes)
        const int g0 = gcol(li), g1 = gcol(16 + li);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (g0 < n) vsm[(4 * r + lk) + g0 * VRW] = acc0[r];
            if (g1 < n) vsm[(4 * r + lk) + g1 * VRW] = acc1[r];
        }
    }
    __syncthreads();
    for (int q = tid; q < VRW * n; q += 64 * JB) {
        const int r = q % VRW, c = q / VRW;
        if (r0 + r < n) Vw[(r0 + r) + (size_t)c * n] = vsm[q];
    }
}

// the product of step launch g - 1 (if its rotations ran) applied to the strip of
// workgroup vb (the V role of step launch g, or the last launch's flush)
template <int JB>
__device__ __forceinline__ void vapply_prev(int n, int nblk, int g, const Ctl *ctl,
                                            const double *__restrict__ Qbuf,
                                            double *__restrict__ Vw, int vb, double *vsm) {
    constexpr int JC = JGeom<JB>::JC;
    if (g == 0 || wg_read(&ctl->bad) || wg_read(&ctl->qran[(g - 1) & 1]) != g - 1) return;
    const int npair = nblk / 2;
    vapply_step<JB>(n, nblk, (g - 1) % (nblk - 1),
                    Qbuf + (size_t)((g - 1) & 1) * npair * (JC * JC), Vw, vb * VRW, vsm);
}

template <int JB>
__global__ void __launch_bounds__(64 * JB)
weig_vflush_kernel(int n, int nblk, int g, const Ctl *ctl, const double *__restrict__ Qbuf,
                   double *__restrict__ Vw) {
    extern __shared__ __attribute__((aligned(16))) double vsm[];  // VRW x n, column-major
    vapply_prev<JB>(n, nblk, g, ctl, Qbuf, Vw, blockIdx.x, vsm);
}

// ---- 5. sigma, signs, ordering, outputs

// one wavefront per column p: ||x_p|| and the row of the largest |V(:, p)|
__global__ void __launch_bounds__(1024)
weig_sigma_kernel(int n, const Ctl *ctl, const double *__restrict__ X,
                  const double *__restrict__ Vw, double *__restrict__ sig,
                  double *__restrict__ sgn) {
    if (wg_read(&ctl->bad)) return;
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (p >= n) return;
    double ss = 0.0, best = -1.0;
    int barg = 0;
    for (int r = lane; r < n; r += 64) {
        const double x = X[r + (size_t)p * n];
        ss = __builtin_fma(x, x, ss);
        const double av = __builtin_fabs(Vw[r + (size_t)p * n]);
        if (av > best) {
            best = av;
            barg = r;
        }
    }
    ss = wave_sum(ss);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oa = __shfl_xor(barg, off);
        if (ob > best || (ob == best && oa < barg)) {
            best = ob;
            barg = oa;
        }
    }
    if (lane == 0) {
        sig[p] = ldexp(__builtin_sqrt(ss), ctl->emax);
        sgn[p] = Vw[barg + (size_t)p * n] < 0 ? -1.0 : 1.0;
    }
}

// ranks (descending, stable) and the final info code
__global__ void __launch_bounds__(1024)
weig_rank_kernel(int n, Ctl *ctl, const double *__restrict__ sig, int *__restrict__ rank,
                 int *__restrict__ info) {
    __shared__ int bad;
    const int b0 = wg_read(&ctl->bad);
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    if (b0 == 0) {
        for (int p = threadIdx.x; p < n; p += blockDim.x) {
            const double sp = sig[p];
            int rk = 0;
            for (int q = 0; q < n; ++q) {
                const double sq = sig[q];
                rk += (sq > sp) || (sq == sp && q < p);
            }
            rank[p] = rk;
            if (!(sp > 0.0)) atomicMax(&bad, 1);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int code = b0;
        if (code == 0 && ctl->notconv) code = 2;
        if (code == 0) code = bad;
        ctl->abort = code != 0;
        *info = code;
    }
}

// one workgroup per column p of the Jacobi: V(:, rank p), W(:, rank p), S(rank p)
__global__ void __launch_bounds__(256)
weig_out_kernel(int n, const Ctl *ctl, const double *__restrict__ Vw,
                const double *__restrict__ sig, const double *__restrict__ sgn,
                const int *__restrict__ rank, double *__restrict__ S, double *__restrict__ V,
                int64_t ldv, double *__restrict__ W, int64_t ldw) {
    if (wg_read(&ctl->abort)) return;
    const int p = blockIdx.x;
    const int pos = rank[p];
    const double sp = sig[p], sg = sgn[p];
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        const double v = sg * Vw[r + (size_t)p * n];
        V[r + (size_t)pos * ldv] = v;
        W[r + (size_t)pos * ldw] = v / sp;
    }
    if (threadIdx.x == 0) S[pos] = sp;
}

// ---- 5'. the preconditioner's basis: V' = X'^-1 Q Sigma_Z, V = P V'
//
// With X' = R' D~' 2^-emax, V' = 2^emax D~'^-1 R'^-1 (Q Sigma_Z), R' = fl64(R_H') the
// (unscaled) Cholesky factor in Hh.  R'^-1 is applied by block back substitution in
// row blocks of SB = 64 from the bottom, with the inverses of the diagonal blocks
// formed first (weig_dinv_kernel, all blocks at once), so that no step of the solve
// waits on a chain of single rows.
constexpr int SB = 64;   // row block of the back substitution
constexpr int SC = 16;   // columns per workgroup

// inv(R'_kk) for the diagonal block kb = blockIdx.x / 4, columns 16 (blockIdx.x % 4)
// .. + 15: back substitution on those identity columns (lane (i, w): row i of
// column w in a register, one barrier per row).  Written to Dinv (SB x SB per
// block, column-major; zeros outside the block's size).
__global__ void __launch_bounds__(1024)
weig_dinv_kernel(int n, const Ctl *ctl, const double *__restrict__ Hh, double *__restrict__ Dinv) {
    __shared__ double Dg[SB * (SB + 1)];
    __shared__ double xb[SB * SC];
    if (wg_read(&ctl->bad) || wg_read(&ctl->notconv)) return;
    const int kb = blockIdx.x / 4, c = (blockIdx.x % 4) * SC + (threadIdx.x >> 6);
    const int k0 = kb * SB;
    const int bs = (n - k0 < SB) ? n - k0 : SB;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int q = tid; q < SB * SB; q += 1024) {
        const int i = q % SB, j = q / SB;
        Dg[i + j * (SB + 1)] = (i <= j && j < bs) ? Hh[(k0 + i) + (size_t)(k0 + j) * n] : 0.0;
    }
    __syncthreads();
    double t = (lane == c && c < bs) ? 1.0 : 0.0;
    for (int kk = bs - 1; kk >= 0; --kk) {
        if (lane == kk) {
            t = t / Dg[kk + kk * (SB + 1)];
            xb[kk + w * SB] = t;
        }
        __syncthreads();
        if (lane < kk) t = __builtin_fma(-Dg[lane + kk * (SB + 1)], xb[kk + w * SB], t);
    }
    Dinv[(size_t)kb * SB * SB + lane + (size_t)c * SB] = (lane < bs && c < bs) ? t : 0.0;
}

// One workgroup per 16 columns c (wavefront w owns column c0 + w):
//   a. sigma_c = ||z_c|| and T(:, c) = Q(:, c) sigma_c in LDS;
//   b. for the row blocks from the bottom: T'(block) = inv(R'_kk) T(block), then
//      the rows above take the block's contribution, T(i) -= sum_k R'(i, k) T'(k),
//      with R' staged through LDS in 64-row chunks;
//   c. V'(r, c) = T'(r, c) 2^(emax - e_pi_r) (exact), the column normalised and
//      written to V(pi_r, c).
__global__ void __launch_bounds__(1024)
weig_pre_out_kernel(int n, const Ctl *ctl, const int *__restrict__ sexp,
                    const int *__restrict__ perm, const double *__restrict__ Hh,
                    const double *__restrict__ Dinv, const double *__restrict__ X,
                    const double *__restrict__ Vw, double *__restrict__ V, int64_t ldv,
                    int *__restrict__ info) {
    extern __shared__ __attribute__((aligned(16))) double psm[];
    double *T = psm;                        // GSVD_WIDE_MAX_N x SC, column-major
    double *Dg = T + GSVD_WIDE_MAX_N * SC;  // SB x SB staging, column-major, ld SB + 1
    double *Xb = Dg + SB * (SB + 1);        // SB x SC block solution
    const int bad = wg_read(&ctl->bad);
    const int code = bad ? bad : (wg_read(&ctl->notconv) ? 2 : 0);
    if (blockIdx.x == 0 && threadIdx.x == 0) *info = code;
    if (code) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int c0 = blockIdx.x * SC, c = c0 + w;
    const bool cv = c < n;
    double *Tw = T + w * GSVD_WIDE_MAX_N;
    // a.
    {
        double ss = 0.0;
        if (cv)
            for (int r = lane; r < n; r += 64) {
                const double z = X[r + (size_t)c * n];
                ss = __builtin_fma(z, z, ss);
            }
        const double sg = __builtin_sqrt(wave_sum(ss));
        for (int r = lane; r < n; r += 64) Tw[r] = cv ? Vw[r + (size_t)c * n] * sg : 0.0;
    }
    // b.
    const int nb = (n + SB - 1) / SB;
    for (int kb = nb - 1; kb >= 0; --kb) {
        const int k0 = kb * SB;
        const int bs = (n - k0 < SB) ? n - k0 : SB;
        const double *Di = Dinv + (size_t)kb * SB * SB;
        for (int q = tid; q < SB * SB; q += 1024) Dg[(q % SB) + (q / SB) * (SB + 1)] = Di[q];
        __syncthreads();
        double x = 0.0;
        if (lane < bs)
            for (int j = lane; j < bs; ++j) x = __builtin_fma(Dg[lane + j * (SB + 1)], Tw[k0 + j], x);
        if (lane < bs) Xb[lane + w * SB] = x;
        __syncthreads();
        if (lane < bs) Tw[k0 + lane] = x;
        for (int rc = 0; rc < k0; rc += SB) {  // rows rc .. rc + 63 (all < k0)
            for (int q = tid; q < SB * SB; q += 1024) {
                const int i = q % SB, k = q / SB;
                Dg[i + k * (SB + 1)] = k < bs ? Hh[(rc + i) + (size_t)(k0 + k) * n] : 0.0;
            }
            __syncthreads();
            double acc = 0.0;
            for (int k = 0; k < bs; ++k) acc = __builtin_fma(Dg[lane + k * (SB + 1)], Xb[k + w * SB], acc);
            Tw[rc + lane] -= acc;
            __syncthreads();
        }
    }
    // c.
    if (!cv) return;
    const int emax = ctl->emax;
    double ss = 0.0;
    for (int r = lane; r < n; r += 64) {
        const double v = ldexp(Tw[r], emax - sexp[perm[r]]);
        Tw[r] = v;
        ss = __builtin_fma(v, v, ss);
    }
    const double inv = 1.0 / __builtin_sqrt(wave_sum(ss));
    for (int r = lane; r < n; r += 64) V[perm[r] + (int64_t)c * ldv] = Tw[r] * inv;
}

// The blocked dd Cholesky of H (upper triangle of Hh/Hl, in place).
hipError_t chol_blocked(int n, Ctl *ctl, double *Hh, double *Hl, hipStream_t st) {
    hipError_t err;
    const size_t lds_potrf = (size_t)CB * (CB + 1) * sizeof(dd_t);
    const size_t lds_panel = (size_t)CB * (CB + 1 + 16) * sizeof(dd_t);
    const size_t lds_update = (size_t)2 * CB * 32 * sizeof(dd_t);
    if ((err = hipFuncSetAttribute((const void *)weig_potrf_kernel,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_potrf)) ||
        (err = hipFuncSetAttribute((const void *)weig_panel_kernel,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_panel)) ||
        (err = hipFuncSetAttribute((const void *)weig_update_kernel,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_update)))
        return err;
    for (int k0 = 0; k0 < n; k0 += CB) {
        hipLaunchKernelGGL(weig_potrf_kernel, dim3(1), dim3(1024), lds_potrf, st, n, k0, ctl, Hh, Hl);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        const int right = n - (k0 + CB);
        if (right > 0) {
            hipLaunchKernelGGL(weig_panel_kernel, dim3((unsigned)((right + 15) / 16)), dim3(1024),
                               lds_panel, st, n, k0, ctl, Hh, Hl);
            if ((err = hipGetLastError()) != hipSuccess) return err;
            const int nt = (right + 31) / 32;
            hipLaunchKernelGGL(weig_update_kernel, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(UT),
                               lds_update, st, n, k0, nt, ctl, Hh, Hl);
            if ((err = hipGetLastError()) != hipSuccess) return err;
        }
    }
    return hipSuccess;
}

template <int RPL, int JB>
hipError_t launch_steps(int n, int nblk, Ctl *ctl, double *X, double *Vw, double *Qbuf,
                        double tol2, int max_sweeps, bool early, hipStream_t st) {
    constexpr int JC = JGeom<JB>::JC, JT = JGeom<JB>::JT, QLD = JGeom<JB>::QLD;
    // the Jacobi role's LDS; the V role needs VRW n <= JC 64 RPL doubles of it
    const size_t lds = early ? ((size_t)JC * (64 * RPL + 1) + 3 * JC * JC + 3 * JC) * sizeof(double)
                             : ((size_t)JC * 64 * RPL + JC * QLD + JC) * sizeof(double);
    auto k = early ? weig_gstep_kernel<RPL, JB> : weig_step_kernel<RPL, JB>;
    auto kf = weig_vflush_kernel<JB>;
    const size_t lds_v = (size_t)VRW * n * sizeof(double);
    const int vstrips = (n + VRW - 1) / VRW;
    hipError_t err = hipFuncSetAttribute((const void *)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    err = hipFuncSetAttribute((const void *)kf, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_v);
    if (err != hipSuccess) return err;
    int g = 0;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        for (int s = 0; s < nblk - 1; ++s, ++g) {
            hipLaunchKernelGGL(k, dim3((unsigned)(nblk / 2 + vstrips)), dim3(JT), lds, st, n, nblk,
                               s, g, ctl, X, Qbuf, Vw, tol2);
            if ((err = hipGetLastError()) != hipSuccess) return err;
        }
        hipLaunchKernelGGL(weig_sweep_kernel, dim3(1), dim3(64), 0, st, ctl, nblk / 2,
                           sw + 1 == max_sweeps ? 1 : 0, early ? 1 : 0);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    // the last launch's products, if its rotations ran
    hipLaunchKernelGGL(kf, dim3((unsigned)vstrips), dim3(JT), lds_v, st, n, nblk, g, ctl, Qbuf, Vw);
    return hipGetLastError();
}

// ---- the Cholesky factor alone (mixed precision Cholesky QR, Sec. 3.3)

// R = fl_w(R_H) D~ in the working precision (exact power-of-two column scaling),
// zeros below the diagonal; info from the checks and the factorization.
template <typename TW>
__global__ void __launch_bounds__(256)
chol_out_kernel(int n, const Ctl *ctl, const int *__restrict__ sexp,
                const double *__restrict__ Hh, TW *__restrict__ R, int64_t ldr,
                int *__restrict__ info) {
    const int bad = wg_read(&ctl->bad);
    const int j = blockIdx.x;
    if (j == 0 && threadIdx.x == 0) *info = bad;
    if (bad) return;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        R[i + (int64_t)j * ldr] = i <= j ? (TW)ldexp(Hh[i + (size_t)j * n], sexp[j]) : (TW)0;
}

}  // namespace

size_t chol_work_bytes(int64_t n) { return wlayout(n).total; }

hipError_t chol_launch(int working, int64_t n64, const double *Mhi, const double *Mlo, int64_t ldm,
                       void *R, int64_t ldr, int *info, void *work, hipStream_t st) {
    if (n64 < 1 || n64 > GSVD_WIDE_MAX_N || Mlo == nullptr || work == nullptr || ldr < n64)
        return hipErrorInvalidValue;
    const int n = (int)n64;
    const WLayout L = wlayout(n);
    char *base = (char *)work;
    Ctl *ctl = reinterpret_cast<Ctl *>(base + L.ctl);
    int *sexp = reinterpret_cast<int *>(base + L.sexp);
    double *Hh = reinterpret_cast<double *>(base + L.hh);
    double *Hl = reinterpret_cast<double *>(base + L.hl);
    double *Vw = reinterpret_cast<double *>(base + L.v);
    hipError_t err;
    int *perm = reinterpret_cast<int *>(base + L.perm);
    hipLaunchKernelGGL(weig_diag_kernel, dim3(1), dim3(1024), 0, st, n, Mhi, ldm, ctl, sexp, perm);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(weig_fill_kernel, dim3((unsigned)n), dim3(256), 0, st, n, Mhi, Mlo, ldm, ctl,
                       sexp, nullptr, Hh, Hl, Vw);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if ((err = chol_blocked(n, ctl, Hh, Hl, st)) != hipSuccess) return err;
    if (working == 1)
        hipLaunchKernelGGL(chol_out_kernel<double>, dim3((unsigned)n), dim3(256), 0, st, n, ctl,
                           sexp, Hh, (double *)R, ldr, info);
    else
        hipLaunchKernelGGL(chol_out_kernel<float>, dim3((unsigned)n), dim3(256), 0, st, n, ctl,
                           sexp, Hh, (float *)R, ldr, info);
    return hipGetLastError();
}

size_t eig_wide_work_bytes(int64_t n) { return wlayout(n).total; }

hipError_t eig_wide_launch(int64_t n64, const double *Mhi, const double *Mlo, int64_t ldm, void *S,
                           void *V, int64_t ldv, void *W, int64_t ldw, int *info, double tol,
                           int max_sweeps, bool pre, void *work, hipStream_t st) {
    if (n64 < 2 || n64 > GSVD_WIDE_MAX_N || Mlo == nullptr || work == nullptr || max_sweeps < 1)
        return hipErrorInvalidValue;
    const int n = (int)n64;
    const WLayout L = wlayout(n);
    char *base = (char *)work;
    Ctl *ctl = reinterpret_cast<Ctl *>(base + L.ctl);
    int *sexp = reinterpret_cast<int *>(base + L.sexp);
    int *rank = reinterpret_cast<int *>(base + L.rank);
    int *perm = reinterpret_cast<int *>(base + L.perm);
    double *sig = reinterpret_cast<double *>(base + L.sig);
    double *sgn = reinterpret_cast<double *>(base + L.sgn);
    double *Hh = reinterpret_cast<double *>(base + L.hh);
    double *Hl = reinterpret_cast<double *>(base + L.hl);
    double *X = reinterpret_cast<double *>(base + L.x);
    double *Vw = reinterpret_cast<double *>(base + L.v);
    double *Qbuf = reinterpret_cast<double *>(base + L.qbuf);
    hipError_t err;
#define WCHK()                                                  \
    do {                                                        \
        if ((err = hipGetLastError()) != hipSuccess) return err; \
    } while (0)

    const int *pp = pre ? perm : nullptr;
    hipLaunchKernelGGL(weig_diag_kernel, dim3(1), dim3(1024), 0, st, n, Mhi, ldm, ctl, sexp, perm);
    WCHK();
    hipLaunchKernelGGL(weig_fill_kernel, dim3((unsigned)n), dim3(256), 0, st, n, Mhi, Mlo, ldm, ctl,
                       sexp, pp, Hh, Hl, Vw);
    WCHK();
    if ((err = chol_blocked(n, ctl, Hh, Hl, st)) != hipSuccess) return err;
    hipLaunchKernelGGL(weig_cast_kernel, dim3((unsigned)n), dim3(256), 0, st, n, ctl, sexp, pp, Hh,
                       X);
    WCHK();
    const double tol2 = tol * tol;
    const int rpl = (n + 63) / 64;
    const int nblk = jac_nblk(n);
#define STEPS(R)                                                                              \
    case R: err = launch_steps<R, JBW>(n, nblk, ctl, X, Vw, Qbuf, tol2, max_sweeps, pre, st); break;
    switch (rpl) {
        STEPS(2) STEPS(3) STEPS(4) STEPS(5) STEPS(6) STEPS(7) STEPS(8)
        default: return hipErrorInvalidValue;
    }
#undef STEPS
    if (err != hipSuccess) return err;
    if (pre) {
        double *Dinv = reinterpret_cast<double *>(base + L.dinv);
        hipLaunchKernelGGL(weig_dinv_kernel, dim3((unsigned)(4 * ((n + SB - 1) / SB))), dim3(1024),
                           0, st, n, ctl, Hh, Dinv);
        WCHK();
        const size_t lds = ((size_t)GSVD_WIDE_MAX_N * SC + SB * (SB + 1) + SB * SC) * sizeof(double);
        if ((err = hipFuncSetAttribute((const void *)weig_pre_out_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)))
            return err;
        hipLaunchKernelGGL(weig_pre_out_kernel, dim3((unsigned)((n + SC - 1) / SC)), dim3(1024), lds,
                           st, n, ctl, sexp, perm, Hh, Dinv, X, Vw, (double *)V, ldv, info);
        WCHK();
        return hipSuccess;
    }
    hipLaunchKernelGGL(weig_sigma_kernel, dim3((unsigned)((n + 15) / 16)), dim3(1024), 0, st, n, ctl,
                       X, Vw, sig, sgn);
    WCHK();
    hipLaunchKernelGGL(weig_rank_kernel, dim3(1), dim3(1024), 0, st, n, ctl, sig, rank, info);
    WCHK();
    hipLaunchKernelGGL(weig_out_kernel, dim3((unsigned)n), dim3(256), 0, st, n, ctl, Vw, sig, sgn,
                       rank, (double *)S, (double *)V, ldv, (double *)W, ldw);
    WCHK();
#undef WCHK
    return hipSuccess;
}

}  // namespace gsvd

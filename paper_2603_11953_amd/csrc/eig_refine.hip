// Two-sided Jacobi on M_h at the Gram precision (Sec. 2.1, Remark 1),
// preconditioned by an FP64 eigenvector basis.
//
// Remark 1 bounds the orthogonality of U by O(u) + O(u_h) kappa^2(B) when the
// eigensolver of Alg. 1 step 3 is the two-sided Jacobi method run at u_h; with
// Algorithm 2 (the remark after Lemma 1) the bound is O(u) kappa(B).  The
// difference comes from the eigenvector matrix: Algorithm 2 rounds R to the
// working precision, so its V diagonalises M_h only to O(u kappa(B)) in the
// scaled sense |x_i^T M_h x_j| <= eps sqrt(lambda_i lambda_j).
//
// This stage runs the u_h Jacobi method on the Gram matrix expressed in a
// basis X from the FP64 eigensolvers: Algorithm 2's steps with the columns
// ordered by norm and the one-sided Jacobi run on the transposed Cholesky factor
// (X by back substitution, accurate in the graded sense), stopped once a sweep
// rotates no pair whose cosine reaches 2^-10 (single problems):
//
//   S = X^T M_h X,  G = X^T X               (double-double, exact products)
//   lambda_i = s_ii / g_ii                  (Rayleigh quotients)
//   f_ij = (s_ij - lambda_j g_ij) / (lambda_j - lambda_i),  i != j
//   f_ii = (1 - g_ii) / 2
//   X <- X (I + F)                          (double-double)
//
// S is diagonal up to the small coupling that basis leaves, so every Jacobi
// rotation of a sweep on S is tiny.  The antisymmetric part of F holds
// the first-order angles of those rotations (tan 2 theta = 2 s_ij /
// (s_jj - s_ii) gives theta = s_ij / (lambda_j - lambda_i) + O(theta^3)), and
// rotations by angles of order theta commute up to O(theta^2): the whole sweep
// is applied at once, with an error of second order in the angles.  The
// symmetric part of F, -(G - I)/2, re-orthogonalises X to first order.  This
// update is the eigenvector refinement of Ogita and Aishima (2018, "Iterative
// refinement for symmetric eigenvalue decomposition"), which converges
// quadratically: one sweep when the largest angle is below 2^-30 (the
// neglected terms are then below 2^-60 relative), a few otherwise.
//
// Stopping rule: the sweep whose largest angle is <= 2^-30 is the last.  At most
// rk sweeps are queued on the stream: 3 for single problems (their basis stops at
// cosines of about 2^-20: two sweeps reach the rule, the third is a margin), 2 for
// the batched call (its basis is converged to 2^-24); those after convergence
// return at once.
// A pair whose angle would exceed 2^-8 (eigenvalues that agree to within the
// coupling: a cluster) is not rotated (f_ij = -g_ij / 2 only re-orthogonalises);
// such pairs, or a last sweep above the threshold, set GSVD_INFO_WARN_REFINE.
//
// Every sum is a double-double dot product over exact FP64 products (TwoProduct
// with the low parts folded in), so S and G carry u_h relative to
// |X|^T |M_h| |X| and |X|^T |X|: in the scaled sense that is O(u_h kappa^2(B)),
// the term Remark 1 keeps.
//
// Outputs as every eigensolver of the library writes them: sigma_i =
// sqrt(lambda_i) (double-double square root) rounded to the working precision,
// sigma descending, each V column signed so its entry of largest magnitude is
// positive, V rounded to the working precision, W = fl(V Sigma^-1).
#include <hip/hip_runtime.h>

#include "dd_device.hpp"
#include "gsvd.h"
#include "gsvd_internal.hpp"

namespace gsvd {
namespace {

constexpr double TAU_STOP = 0x1p-30;   // last sweep: every angle at most this
constexpr double TAU_CLUSTER = 0x1p-8; // larger angles: a cluster pair, not rotated
constexpr int TB = 32;                 // output tile edge of the products
constexpr int FT = 1024;               // lanes of the per-problem kernels

struct RefCtrl {
    int stop_iter;  // sweeps 0 .. stop_iter run; -1: nothing (the preconditioner failed)
    int warn;       // bit 0: last sweep above TAU_STOP; bit 1: cluster pairs left
    unsigned long long maxbits;  // the sweep's largest angle (bits of a non-negative double)
    int clus;       // the sweep met a cluster pair
    int pad[11];
};

// Per-problem scratch, in doubles after the 64-byte control block: X twice
// (ping-pong, hi and lo planes), T = M X, S, G (hi and lo), F, lambda (hi, lo).
struct RefBufs {
    RefCtrl *ctrl;
    double *xh[2], *xl[2], *th, *tl, *sh, *sl, *gh, *gl, *f, *lh, *ll;
};

__host__ __device__ inline size_t ref_bytes_of(int n) {
    const size_t nn = (size_t)n * (size_t)n;
    const size_t b = sizeof(RefCtrl) + (11 * nn + 2 * (size_t)n) * sizeof(double);
    return (b + 255) / 256 * 256;
}

__device__ __forceinline__ RefBufs ref_bufs(double *rw, int n) {
    const size_t nn = (size_t)n * (size_t)n;
    RefBufs B;
    B.ctrl = reinterpret_cast<RefCtrl *>(rw);
    double *d = rw + sizeof(RefCtrl) / sizeof(double);
    B.xh[0] = d;
    B.xl[0] = d + nn;
    B.xh[1] = d + 2 * nn;
    B.xl[1] = d + 3 * nn;
    B.th = d + 4 * nn;
    B.tl = d + 5 * nn;
    B.sh = d + 6 * nn;
    B.sl = d + 7 * nn;
    B.gh = d + 8 * nn;
    B.gl = d + 9 * nn;
    B.f = d + 10 * nn;
    B.lh = d + 11 * nn;
    B.ll = B.lh + n;
    return B;
}

// One problem as the kernels see it.
struct RefProb {
    const double *Mhi, *Mlo;  // Mlo may be null (an FP64 Gram: low parts zero)
    int64_t ldm;
    const double *X0;         // the preconditioner (Algorithm 2's V), FP64
    int64_t ldx0;
    void *S, *V, *W;          // outputs, working precision
    int64_t ldv, ldw;
    int *info;
    double *rw;               // ref_bytes_of(n) bytes of scratch
    int n;
};

struct OneRef {
    RefProb p;
    __device__ RefProb get(int) const { return p; }
};

// Batched, FP64 working: the problem's record in the batch table.
struct TabRef {
    const BatchMat *tab;
    __device__ RefProb get(int b) const {
        const BatchMat &t = tab[b];
        RefProb p;
        p.Mhi = t.Mhi;
        p.Mlo = t.Mlo;
        p.ldm = t.n;
        p.X0 = reinterpret_cast<const double *>(t.V);
        p.ldx0 = t.ldv;
        p.S = t.S;
        p.V = t.V;
        p.W = t.W;
        p.ldv = t.ldv;
        p.ldw = t.n;
        p.info = t.info;
        p.rw = t.rw;
        p.n = t.n;
        return p;
    }
};

// acc (h + l) += a * b for double-double a, b: the product of the high parts
// exactly (TwoProduct), the cross terms folded into its error, TwoSum into h.
__device__ __forceinline__ void mac_dd(double &h, double &l, double ah, double al, double bh,
                                       double bl) {
    const double p = ah * bh;
    double e = __builtin_fma(ah, bh, -p);
    e = __builtin_fma(ah, bl, e);
    e = __builtin_fma(al, bh, e);
    const double s = h + p;
    const double bv = s - h;
    const double err = (h - (s - bv)) + (p - bv);
    h = s;
    l += err + e;
}

// MODE 0: T = M X.  MODE 1: [S | G] = X^T [T | X].  MODE 2: X' = X + X F.
// One workgroup per TBT x TBT output tile (32, or 16 for a single problem whose
// 32 x 32 tiles would leave most of the chip idle); each lane owns a TBT / 16
// square block of it (rows tx + 16 a, columns ty + 16 b).  Every output is
// accumulated over k = 0 .. n - 1 in order, whatever the tile: the two tile sizes
// give the same bits.
template <int MODE, class P, int TBT>
__global__ void __launch_bounds__(256) ref_gemm_kernel(P probs, int iter, int rk) {
    constexpr int RB = TBT / 16;         // outputs per lane along each dimension
    constexpr int KCT = 16 * 32 / TBT;   // k-chunk: the LDS tiles keep one size
    const RefProb p = probs.get(blockIdx.z);
    const int n = p.n;
    const int ncol = MODE == 1 ? 2 * n : n;
    const int i0 = blockIdx.x * TBT, j0 = blockIdx.y * TBT;
    if (i0 >= n || j0 >= ncol) return;
    RefBufs B = ref_bufs(p.rw, n);
    const bool lead = blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0;
    // the first product of the first sweep sets the stage up: sweeps 0 .. rk - 1
    // queued (none if the preconditioner failed), X_0 = the preconditioner's basis
    // (copied by the workgroups of the first tile row as they stage it)
    const bool first = MODE == 0 && iter == 0;
    if (first) {
        const bool failed = *p.info != 0;
        if (lead) {
            B.ctrl->stop_iter = failed ? -1 : rk - 1;
            B.ctrl->warn = 0;
        }
        if (failed) return;
    } else if (iter > B.ctrl->stop_iter) {
        return;
    }
    const int cur = iter & 1;
    const double *__restrict__ Xh = B.xh[cur];
    const double *__restrict__ Xl = B.xl[cur];
    if (MODE == 0 && lead) {
        B.ctrl->maxbits = 0ull;  // the angle kernel of this sweep reduces into these
        B.ctrl->clus = 0;
    }
    if (MODE == 2 && lead) {
        // the decision of this sweep (its angles are all in): the last sweep if every
        // angle is below TAU_STOP, or if it is the last one queued.  Other workgroups
        // of this launch read stop_iter as iter or rk - 1, both >= iter: they all run.
        const double mx = __longlong_as_double((long long)B.ctrl->maxbits);
        if (mx <= TAU_STOP || iter == rk - 1) {
            B.ctrl->stop_iter = iter;
            B.ctrl->warn = (mx <= TAU_STOP ? 0 : 1) | (B.ctrl->clus ? 2 : 0);
        }
    }

    __shared__ double Ah[TBT][KCT + 1], Al[TBT][KCT + 1], Bh[KCT][TBT + 1], Bl[KCT][TBT + 1];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    double ch[RB][RB], cl[RB][RB];
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
        for (int b = 0; b < RB; ++b) ch[a][b] = cl[a][b] = 0.0;

    for (int k0 = 0; k0 < n; k0 += KCT) {
        for (int e = tid; e < TBT * KCT; e += 256) {
            int i, k;
            if (MODE == 1) {  // A = X^T: contiguous along k
                k = e % KCT;
                i = e / KCT;
            } else {          // A = M or X: contiguous along i
                i = e % TBT;
                k = e / TBT;
            }
            const int gi = i0 + i, gk = k0 + k;
            double ah = 0.0, al = 0.0;
            if (gi < n && gk < n) {
                if (MODE == 0) {
                    const int64_t o = gi + (int64_t)gk * p.ldm;
                    ah = p.Mhi[o];
                    al = p.Mlo ? p.Mlo[o] : 0.0;
                } else if (MODE == 1) {
                    ah = Xh[gk + gi * n];
                    al = Xl[gk + gi * n];
                } else {
                    ah = Xh[gi + gk * n];
                    al = Xl[gi + gk * n];
                }
            }
            Ah[i][k] = ah;
            Al[i][k] = al;
        }
        for (int e = tid; e < TBT * KCT; e += 256) {
            const int k = e % KCT, j = e / KCT;
            const int gk = k0 + k, gj = j0 + j;
            double bh = 0.0, bl = 0.0;
            if (gk < n && gj < ncol) {
                if (first) {
                    bh = p.X0[gk + (int64_t)gj * p.ldx0];
                    if (blockIdx.x == 0) {
                        B.xh[0][gk + gj * n] = bh;
                        B.xl[0][gk + gj * n] = 0.0;
                    }
                } else if (MODE == 0) {
                    bh = Xh[gk + gj * n];
                    bl = Xl[gk + gj * n];
                } else if (MODE == 1) {
                    if (gj < n) {
                        bh = B.th[gk + gj * n];
                        bl = B.tl[gk + gj * n];
                    } else {
                        bh = Xh[gk + (gj - n) * n];
                        bl = Xl[gk + (gj - n) * n];
                    }
                } else {
                    bh = B.f[gk + gj * n];
                }
            }
            Bh[k][j] = bh;
            Bl[k][j] = bl;
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < KCT; ++k) {
            double ah[RB], al[RB], bh[RB], bl[RB];
#pragma unroll
            for (int a = 0; a < RB; ++a) {
                ah[a] = Ah[tx + 16 * a][k];
                al[a] = Al[tx + 16 * a][k];
                bh[a] = Bh[k][ty + 16 * a];
                bl[a] = Bl[k][ty + 16 * a];
            }
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int a = 0; a < RB; ++a) mac_dd(ch[a][b], cl[a][b], ah[a], al[a], bh[b], bl[b]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < RB; ++a) {
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const int gi = i0 + tx + 16 * a, gj = j0 + ty + 16 * b;
            if (gi >= n || gj >= ncol) continue;
            dd_t c = two_sum(ch[a][b], cl[a][b]);
            if (MODE == 0) {
                B.th[gi + gj * n] = c.hi;
                B.tl[gi + gj * n] = c.lo;
            } else if (MODE == 1) {
                if (gj < n) {
                    B.sh[gi + gj * n] = c.hi;
                    B.sl[gi + gj * n] = c.lo;
                } else {
                    B.gh[gi + (gj - n) * n] = c.hi;
                    B.gl[gi + (gj - n) * n] = c.lo;
                }
            } else {
                const int o = gi + gj * n;
                c = dd_add(dd_t{Xh[o], Xl[o]}, c);
                B.xh[cur ^ 1][o] = c.hi;
                B.xl[cur ^ 1][o] = c.lo;
            }
        }
    }
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
    return x;
}

// Rayleigh quotients and the update F: grid (slices of the n^2 entries, problems).
// Every workgroup forms all n quotients (n dd divisions); its slice of F follows,
// and its largest angle and cluster flag go to the sweep's control words.
constexpr int AE = 8;  // entries of F per lane

template <class P>
__global__ void __launch_bounds__(FT) ref_angles_kernel(P probs, int iter) {
    const RefProb p = probs.get(blockIdx.y);
    const int n = p.n;
    const int e0 = blockIdx.x * FT * AE;
    if (e0 >= n * n) return;
    RefBufs B = ref_bufs(p.rw, n);
    if (iter > B.ctrl->stop_iter) return;
    __shared__ double lam_h[GSVD_WIDE_MAX_N], lam_l[GSVD_WIDE_MAX_N];
    const int tid = threadIdx.x;
    for (int i = tid; i < n; i += FT) {
        const int o = i + i * n;
        const dd_t lam = dd_div(dd_t{B.sh[o], B.sl[o]}, dd_t{B.gh[o], B.gl[o]});
        lam_h[i] = lam.hi;
        lam_l[i] = lam.lo;
        if (blockIdx.x == 0) {
            B.lh[i] = lam.hi;
            B.ll[i] = lam.lo;
        }
    }
    __syncthreads();
    double mx = 0.0;
    int clus = 0;
    const int e1 = (e0 + FT * AE < n * n) ? e0 + FT * AE : n * n;
    for (int idx = e0 + tid; idx < e1; idx += FT) {
        const int i = idx % n, j = idx / n;
        double f;
        if (i == j) {
            const dd_t r = dd_sub(dd_t{1.0, 0.0}, dd_t{B.gh[idx], B.gl[idx]});
            f = 0.5 * r.hi;
        } else {
            const double s = B.sh[idx] + B.sl[idx];
            const double g = B.gh[idx] + B.gl[idx];
            const double num = __builtin_fma(-lam_h[j], g, s);
            const dd_t den = dd_sub(dd_t{lam_h[j], lam_l[j]}, dd_t{lam_h[i], lam_l[i]});
            f = num / den.hi;
            if (!(__builtin_fabs(f) <= TAU_CLUSTER)) {
                clus = 1;
                f = -0.5 * g;
            } else {
                mx = fmax(mx, __builtin_fabs(f));
            }
        }
        B.f[idx] = f;
    }
    mx = wave_max(mx);
    const unsigned long long any = __ballot(clus != 0);
    if ((tid & 63) == 0) {
        atomicMax(&B.ctrl->maxbits, (unsigned long long)__double_as_longlong(mx));
        if (any) atomicOr(&B.ctrl->clus, 1);
    }
}

// sigma_c = sqrt(lambda_c) (every workgroup forms all n, for the ordering), the
// sign of column c of the final X (its entry of largest magnitude made positive,
// the lowest index on ties), ordering (sigma descending, stable), cast, W: grid
// (groups of 16 columns, problems), one wavefront per column.
template <typename TW, class P>
__global__ void __launch_bounds__(FT) ref_write_kernel(P probs) {
    const RefProb p = probs.get(blockIdx.y);
    const int n = p.n;
    const int c0 = blockIdx.x * (FT / 64);
    if (c0 >= n) return;
    RefBufs B = ref_bufs(p.rw, n);
    const int stop = B.ctrl->stop_iter;
    if (stop < 0) return;
    const double *__restrict__ Xh = B.xh[(stop + 1) & 1];
    __shared__ double sig[GSVD_WIDE_MAX_N];
    for (int q = threadIdx.x; q < n; q += FT) sig[q] = dd_sqrt(dd_t{B.lh[q], B.ll[q]}).hi;
    __syncthreads();
    const int c = c0 + (threadIdx.x >> 6);
    if (c >= n) return;
    const int lane = threadIdx.x & 63;
    double best = -1.0;
    int barg = 0;
    for (int r = lane; r < n; r += 64) {
        const double av = __builtin_fabs(Xh[r + c * n]);
        if (av > best) {
            best = av;
            barg = r;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oa = __shfl_xor(barg, off, 64);
        if (ob > best || (ob == best && oa < barg)) {
            best = ob;
            barg = oa;
        }
    }
    const double sg = Xh[barg + c * n] < 0.0 ? -1.0 : 1.0;
    const double sc = sig[c];
    int rk = 0;
    for (int q = lane; q < n; q += 64) rk += (sig[q] > sc) || (sig[q] == sc && q < c);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) rk += __shfl_xor(rk, off, 64);
    TW *S = reinterpret_cast<TW *>(p.S);
    TW *V = reinterpret_cast<TW *>(p.V);
    TW *W = reinterpret_cast<TW *>(p.W);
    const TW sw = (TW)sc;
    for (int r = lane; r < n; r += 64) {
        const TW vw = (TW)(sg * Xh[r + c * n]);
        V[r + (int64_t)rk * p.ldv] = vw;
        W[r + (int64_t)rk * p.ldw] = vw / sw;
    }
    if (lane == 0) S[rk] = sw;
    if (c == 0 && lane == 0 && B.ctrl->warn != 0) *p.info = GSVD_INFO_WARN_REFINE;
}

// ---- the assumption check of Theorem 1 (every eigensolver) ----------------

struct AssumpProb {
    const double *Mhi;
    int64_t ldm;
    const void *W;
    int64_t ldw;
    int *info;
    int n;
};

struct OneAssump {
    AssumpProb p;
    __device__ AssumpProb get(int) const { return p; }
};

struct TabAssump {
    const BatchMat *tab;
    __device__ AssumpProb get(int b) const {
        const BatchMat &t = tab[b];
        return AssumpProb{t.Mhi, t.n, t.W, t.n, t.info, t.n};
    }
};

// kappa(B)^2 = lambda_max(H) ||B^+||_2^2 with H = D^-1 M_h D^-1 = B^T B
// (D = diag(sqrt(m_jj)), B = A D^-1 with unit columns).  Bounds from what the
// eigensolver produced: lambda_max(H) <= max_i sum_j |h_ij| (Gershgorin), and
// ||B^+||_2 <= ||B^+||_F = ||D W||_F, since A = U Sigma V^T gives
// B^+ = D V Sigma^-1 U^T and W = V Sigma^-1.  With that kappa the conditions of
// Remark 1 (the u_h Jacobi) and of the remark after Lemma 1 (Algorithm 2) are
// checked, with the constants of eq. (thm:assump):
//   2 (e_gram + n u_h) kappa^2 <= 1/2, e_gram bounding ||D^-1 dM D^-1|| for the
//     Gram's error dM (n^2 u_h for the plain Gram, as in eq. (thm:assump);
//     n eps for a split Gram whose entries carry |dM_ij| <= eps sqrt(m_ii m_jj)),
//   c_w u kappa <= 1/2, c_w = n for Algorithm 2 (its O(u) kappa(B) term), else 0;
// a failed condition sets GSVD_INFO_WARN_ASSUMPTION (Theorem 1's bounds are then
// not guaranteed).
// AT lanes per problem (AT / 64 wavefronts, each taking every (AT / 64)-th column).
template <typename TW, class P, int AT>
__global__ void __launch_bounds__(AT)
assump_kernel(P probs, double e_gram, double u_h, double u_w, double c_w) {
    constexpr int NW = AT / 64;
    const AssumpProb p = probs.get(blockIdx.x);
    const int n = p.n;
    const TW *W = reinterpret_cast<const TW *>(p.W);
    __shared__ double dg[GSVD_WIDE_MAX_N], isq[GSVD_WIDE_MAX_N];
    __shared__ double red[NW], redg[NW];
    for (int r = threadIdx.x; r < n; r += AT) {
        const double d = p.Mhi[r + (int64_t)r * p.ldm];
        dg[r] = d;
        isq[r] = 1.0 / __builtin_sqrt(d);
    }
    __syncthreads();
    // wavefront w takes columns w, w + NW, ...; its lanes the rows (coalesced)
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double s = 0.0, gmax = 0.0;
    for (int c = w; c < n; c += NW) {
        double rs = 0.0;
        for (int r = lane; r < n; r += 64) {
            const double x = (double)W[r + (int64_t)c * p.ldw];
            s = __builtin_fma(dg[r] * x, x, s);
            rs = __builtin_fma(__builtin_fabs(p.Mhi[r + (int64_t)c * p.ldm]), isq[r], rs);
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) rs += __shfl_xor(rs, off, 64);
        gmax = fmax(gmax, rs * isq[c]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
        red[w] = s;
        redg[w] = gmax;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int info = *p.info;
    if ((info & 0xff) != 0) return;
    const double dn = (double)n;
    double g = 0.0, sum = 0.0;
    for (int k = 0; k < NW; ++k) {  // a fixed order
        g = fmax(g, redg[k]);
        sum += red[k];
    }
    const double kap2 = g * sum;
    const bool hi_ok = 2.0 * (e_gram + dn * u_h) * kap2 <= 0.5;
    const bool w_ok = c_w * u_w * __builtin_sqrt(kap2) <= 0.5;
    if (!(hi_ok && w_ok)) *p.info = info | GSVD_INFO_WARN_ASSUMPTION;
}

// FP64 eigensolver outputs cast to FP32 working precision (Alg. 1 steps 4-5):
// S and V rounded, W = fl(V Sigma^-1) formed from the rounded values.
__global__ void __launch_bounds__(256)
cast_eig_kernel(int n, const double *__restrict__ S64, const double *__restrict__ V64,
                float *__restrict__ S, float *__restrict__ V, int64_t ldv,
                float *__restrict__ W, int64_t ldw, const int *__restrict__ info) {
    if ((*info & 0xff) != 0) return;
    const int c = blockIdx.x;
    const float sw = (float)S64[c];
    for (int r = threadIdx.x; r < n; r += 256) {
        const float vw = (float)V64[r + (int64_t)c * n];
        V[r + (int64_t)c * ldv] = vw;
        W[r + (int64_t)c * ldw] = vw / sw;
    }
    if (threadIdx.x == 0) S[c] = sw;
}

__global__ void __launch_bounds__(256) fill_zero_kernel(double *__restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        p[i] = 0.0;
}

template <class P>
hipError_t refine_queue(P probs, int count, int max_n, bool f32, int rk, hipStream_t st) {
    const int nt = (max_n + TB - 1) / TB;
    const unsigned ablocks = (unsigned)(((size_t)max_n * max_n + FT * AE - 1) / (FT * AE));
    hipError_t err;
    // a single problem with fewer than 256 tiles of 32 x 32 takes 16 x 16 tiles
    const bool t16 = count == 1 && nt * nt < 256;
    const unsigned ns = (unsigned)((max_n + 15) / 16);
    for (int it = 0; it < rk; ++it) {
        if (t16)
            hipLaunchKernelGGL((ref_gemm_kernel<0, P, 16>), dim3(ns, ns, count), dim3(256), 0, st,
                               probs, it, rk);
        else
            hipLaunchKernelGGL((ref_gemm_kernel<0, P, TB>), dim3(nt, nt, count), dim3(256), 0, st,
                               probs, it, rk);
        if (t16)
            hipLaunchKernelGGL((ref_gemm_kernel<1, P, 16>), dim3(ns, 2 * ns, count), dim3(256), 0,
                               st, probs, it, rk);
        else
            hipLaunchKernelGGL((ref_gemm_kernel<1, P, TB>), dim3(nt, 2 * nt, count), dim3(256), 0,
                               st, probs, it, rk);
        hipLaunchKernelGGL(ref_angles_kernel<P>, dim3(ablocks, (unsigned)count), dim3(FT), 0, st,
                           probs, it);
        if (t16)
            hipLaunchKernelGGL((ref_gemm_kernel<2, P, 16>), dim3(ns, ns, count), dim3(256), 0, st,
                               probs, it, rk);
        else
            hipLaunchKernelGGL((ref_gemm_kernel<2, P, TB>), dim3(nt, nt, count), dim3(256), 0, st,
                               probs, it, rk);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    const unsigned cblocks = (unsigned)((max_n + FT / 64 - 1) / (FT / 64));
    if (f32)
        hipLaunchKernelGGL((ref_write_kernel<float, P>), dim3(cblocks, (unsigned)count), dim3(FT),
                           0, st, probs);
    else
        hipLaunchKernelGGL((ref_write_kernel<double, P>), dim3(cblocks, (unsigned)count), dim3(FT),
                           0, st, probs);
    return hipGetLastError();
}

}  // namespace

size_t refine_work_bytes(int64_t n) {
    return (n < 1 || n > GSVD_WIDE_MAX_N) ? 0 : ref_bytes_of((int)n);
}

hipError_t refine_launch(int working, int64_t n, const double *Mhi, const double *Mlo,
                         int64_t ldm, const double *X0, int64_t ldx0, void *S, void *V,
                         int64_t ldv, void *W, int64_t ldw, int *info, void *work,
                         hipStream_t st) {
    if (n < 1 || n > GSVD_WIDE_MAX_N || work == nullptr || X0 == nullptr || ldx0 < n ||
        ldm < n || ldv < n || ldw < n)
        return hipErrorInvalidValue;
    OneRef pr;
    pr.p = RefProb{Mhi, Mlo, ldm, X0, ldx0, S, V, W, ldv, ldw, info, (double *)work, (int)n};
    return refine_queue(pr, 1, (int)n, working == GSVD_F32, 3, st);
}

hipError_t refine_batched_launch(const BatchMat *tab, int batch, int max_n, hipStream_t st) {
    if (batch < 1 || max_n < 1 || max_n > GSVD_WIDE_MAX_N) return hipErrorInvalidValue;
    return refine_queue(TabRef{tab}, batch, max_n, false, 2, st);
}

hipError_t assump_launch(int working, int64_t n, const double *Mhi, int64_t ldm, const void *W,
                         int64_t ldw, int *info, double e_gram, bool alg2, hipStream_t st) {
    if (n < 1 || ldm < n || ldw < n) return hipErrorInvalidValue;
    OneAssump a;
    a.p = AssumpProb{Mhi, ldm, W, ldw, info, (int)n};
    const double u_h = working == GSVD_F64 ? 0x1p-104 : 0x1p-53;
    const double u_w = working == GSVD_F64 ? 0x1p-53 : 0x1p-24;
    const double c_w = alg2 ? (double)n : 0.0;
    if (working == GSVD_F64)
        hipLaunchKernelGGL((assump_kernel<double, OneAssump, 1024>), dim3(1), dim3(1024), 0, st, a,
                           e_gram, u_h, u_w, c_w);
    else
        hipLaunchKernelGGL((assump_kernel<float, OneAssump, 1024>), dim3(1), dim3(1024), 0, st, a,
                           e_gram, u_h, u_w, c_w);
    return hipGetLastError();
}

hipError_t assump_batched_launch(int working, const BatchMat *tab, int batch, double e_gram,
                                 bool alg2, int max_n, hipStream_t st) {
    if (batch < 1) return hipErrorInvalidValue;
    const double u_h = working == GSVD_F64 ? 0x1p-104 : 0x1p-53;
    const double u_w = working == GSVD_F64 ? 0x1p-53 : 0x1p-24;
    // the Algorithm 2 condition with the largest n of the batch (conservative)
    const double c_w = alg2 ? (double)max_n : 0.0;
    if (working == GSVD_F64)
        hipLaunchKernelGGL((assump_kernel<double, TabAssump, 256>), dim3((unsigned)batch), dim3(256),
                           0, st, TabAssump{tab}, e_gram, u_h, u_w, c_w);
    else
        hipLaunchKernelGGL((assump_kernel<float, TabAssump, 256>), dim3((unsigned)batch), dim3(256),
                           0, st, TabAssump{tab}, e_gram, u_h, u_w, c_w);
    return hipGetLastError();
}

hipError_t fill_zero_launch(double *p, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256),
                       0, st, p, n);
    return hipGetLastError();
}

hipError_t cast_eig_f32_launch(int64_t n, const double *S64, const double *V64, void *S, void *V,
                               int64_t ldv, void *W, int64_t ldw, const int *info,
                               hipStream_t st) {
    if (n < 1 || ldv < n || ldw < n) return hipErrorInvalidValue;
    hipLaunchKernelGGL(cast_eig_kernel, dim3((unsigned)n), dim3(256), 0, st, (int)n, S64, V64,
                       (float *)S, (float *)V, ldv, (float *)W, ldw, info);
    return hipGetLastError();
}

}  // namespace gsvd

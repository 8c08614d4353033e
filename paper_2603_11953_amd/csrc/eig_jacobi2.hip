// Eigensolver stage, two-sided Jacobi on the Gram matrix (Alg. 1 step 3 with
// the two-sided Jacobi method of Sec. 2.1 and Remark 1), for FP32 working
// precision: M_h is FP64 (u_h = 2^-53) and every rotation is carried out in
// FP64 on the full symmetric matrix held in LDS.
//
//   1. Checks (non-finite input: info 3; a non-positive diagonal: info 1) and
//      one global power-of-two scaling M <- 2^-e M, e = max_j ilogb(m_jj), so
//      the largest diagonal entry lies in [1, 2) (exact).
//   2. Round-robin parallel ordering: n/2 disjoint pairs (p, q) per step.
//      A pair is rotated when |m_pq| > tol sqrt(m_pp m_qq) (the scaled test of
//      eq. (eig-2)); the rotation is the textbook one of smaller angle,
//        zeta = (m_qq - m_pp) / (2 m_pq), t = sgn(zeta) / (|zeta| + sqrt(1 + zeta^2)),
//        c = 1 / sqrt(1 + t^2), s = c t,
//      applied as M <- J^T M J in one pass over the 2x2 blocks of the step's
//      pairs (the block of pairs P and R needs only their two rotations; a
//      rotated diagonal block is set to (m_pp - t m_pq, 0, 0, m_qq + t m_pq))
//      and V <- V J.
//   3. Stop after a sweep without rotation.  lambda_i = m_ii, sigma_i =
//      sqrt(lambda_i) (eq. (sqrt)); ordering, sign rule and the casts of
//      Alg. 1 steps 4-5 as in the Algorithm 2 kernel; W = fl(V Sigma^-1).
// V is FP64 in LDS for n <= 96.  Beyond, M alone fills LDS: the rotations of
// every step are logged to the workspace, and V is formed afterwards by
// replaying the log, one wavefront per row of V (eig_jacobi2_vapply_kernel).
#include <hip/hip_runtime.h>

#include "gsvd_internal.hpp"
#include "jacobi_math.hpp"

namespace gsvd {

constexpr int J2_MAXPAIR = GSVD_KMAX_N / 2;

struct J2Smem {
    int flag_rot, flag_bad, emax;
    int pp[J2_MAXPAIR], qq[J2_MAXPAIR];
    double c[J2_MAXPAIR], s[J2_MAXPAIR], app[J2_MAXPAIR], aqq[J2_MAXPAIR];
    unsigned char act[J2_MAXPAIR];
    double ssig[GSVD_KMAX_N];
    double ssign[GSVD_KMAX_N];
    int srank[GSVD_KMAX_N];
};

__host__ __device__ constexpr int j2_ldm(int n) { return n + 1; }  // odd stride: row passes spread banks

// Workspace of the rotation-log form (n > 96): control words, the eigenvalues,
// the rotation log ((c, s) of every pair of every step, identity for pairs not
// rotated) and V (n x n FP64).
struct J2Ctl {
    int status;  // 0 converged, else the info code (1, 2 or 3)
    int steps;   // tournament steps to replay
    int esc;     // M was scaled by 2^esc
};

__host__ __device__ inline size_t j2_al(size_t x) { return (x + 255) / 256 * 256; }
__host__ __device__ inline size_t j2_lam_off() { return 256; }
__host__ __device__ inline size_t j2_log_off(int n) { return j2_al(256 + (size_t)n * 8); }
__host__ __device__ inline size_t j2_v_off(int n, int sweeps) {
    const int N = n + (n & 1);
    return j2_al(j2_log_off(n) + (size_t)sweeps * (N - 1) * (N / 2) * 2 * sizeof(double));
}

template <typename TW, bool LOGV>
__device__ __forceinline__ void eig_jacobi2_body(int n, const double *__restrict__ Mhi, int64_t ldm,
                                                 TW *__restrict__ S, TW *__restrict__ V,
                                                 int64_t ldv, TW *__restrict__ W, int64_t ldw,
                                                 int *__restrict__ info, double tol, int max_sweeps,
                                                 double *__restrict__ vglob, J2Smem &sm,
                                                 double *lds) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int LD = j2_ldm(n);
    double *Ms = lds;
    // LOGV: vglob is the workspace (control words, eigenvalues, rotation log); V is not touched here
    J2Ctl *ctl = reinterpret_cast<J2Ctl *>(vglob);
    double *vlog = LOGV ? reinterpret_cast<double *>(reinterpret_cast<char *>(vglob) + j2_log_off(n))
                        : nullptr;
    double *Vs = LOGV ? nullptr : (vglob != nullptr ? vglob : lds + (size_t)n * LD);
    const int LDV = n;

    if (tid == 0) {
        sm.flag_rot = 0;
        sm.flag_bad = 0;
        sm.emax = -100000;
    }
    __syncthreads();
    for (int j = tid; j < n; j += nthr) {
        const double mjj = Mhi[j + (int64_t)j * ldm];
        if (!__builtin_isfinite(mjj)) {
            atomicMax(&sm.flag_bad, 3);
        } else if (!(mjj > 0.0)) {
            atomicMax(&sm.flag_bad, 1);
        } else {
            atomicMax(&sm.emax, ilogb(mjj));
        }
    }
    for (int q = tid; q < n * n; q += nthr) {
        const double v = Mhi[(q % n) + (int64_t)(q / n) * ldm];
        if (!__builtin_isfinite(v)) atomicMax(&sm.flag_bad, 3);
    }
    __syncthreads();
    if (sm.flag_bad) {
        if (tid == 0) {
            if (LOGV) ctl->status = sm.flag_bad;
            else *info = sm.flag_bad;
        }
        return;
    }
    const int esc = -sm.emax;  // M <- 2^esc M: the largest diagonal entry in [1, 2)
    for (int q = tid; q < n * n; q += nthr) {
        const int i = q % n, j = q / n;
        Ms[i + j * LD] = ldexp(Mhi[i + (int64_t)j * ldm], esc);
        if (!LOGV) Vs[i + j * LDV] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();

    const int N = n + (n & 1);
    const int npair = N / 2;
    const double tol2 = tol * tol;
    bool converged = (n == 1);
    int sweeps_done = 0;
    for (int sw = 0; sw < max_sweeps && !converged; ++sw) {
        sweeps_done = sw + 1;
        for (int step = 0; step < N - 1; ++step) {
            // (a) rotation of every pair of the step from its current 2x2 block
            for (int pr = tid; pr < npair; pr += nthr) {
                int a = 0;
                if (pr != 0) {
                    a = pr - 1 + step;
                    if (a >= N - 1) a -= N - 1;
                    a += 1;
                }
                int b = N - 2 - pr + step;
                if (b >= N - 1) b -= N - 1;
                b += 1;
                const int p = a < b ? a : b, q = a < b ? b : a;
                sm.pp[pr] = p;
                sm.qq[pr] = q;
                unsigned char act = 0;
                if (q < n) {
                    const double app = Ms[p + p * LD], aqq = Ms[q + q * LD], apq = Ms[p + q * LD];
                    if (apq * apq > tol2 * (app * aqq)) {
                        const double zeta = (aqq - app) * rcp_nr(2.0 * apq);
                        const double az = __builtin_fabs(zeta);
                        double t;
                        if (az > 1e150) {
                            t = 0.5 * rcp_nr(zeta);
                        } else {
                            const double x = __builtin_fma(zeta, zeta, 1.0);
                            t = rcp_nr(az + x * rsq_nr(x));
                            if (zeta < 0) t = -t;
                        }
                        const double c = rsq_nr(__builtin_fma(t, t, 1.0));
                        sm.c[pr] = c;
                        sm.s[pr] = c * t;
                        sm.app[pr] = app - t * apq;
                        sm.aqq[pr] = aqq + t * apq;
                        act = 1;
                        sm.flag_rot = 1;
                    }
                }
                sm.act[pr] = act;
                if (LOGV) {
                    double *e = vlog + ((size_t)(sw * (N - 1) + step) * npair + pr) * 2;
                    e[0] = act ? sm.c[pr] : 1.0;
                    e[1] = act ? sm.s[pr] : 0.0;
                }
            }
            __syncthreads();
            // (b) M <- J^T M J by 2x2 blocks: the block of pair rows P and pair
            // columns R needs only the rotations of P and R (the column update, then
            // the row update, as separate passes would do them); a rotated diagonal
            // block takes its closed form (m_pp - t m_pq, 0, 0, m_qq + t m_pq).
            // A pair whose q is the padding index n has one row / column only.
            // item it = P + npair R; when npair divides the lane count a lane keeps
            // one P for the whole pass (its pair read once), and R is the same
            // across a wavefront (broadcast reads)
            auto block = [&](int P, bool aP, int p0, int q0, double cP, double sP, int R) {
                const bool aR = sm.act[R] != 0;
                if (!aP && !aR) return;
                if (P == R) {
                    Ms[p0 + p0 * LD] = sm.app[P];
                    Ms[q0 + q0 * LD] = sm.aqq[P];
                    Ms[p0 + q0 * LD] = 0.0;
                    Ms[q0 + p0 * LD] = 0.0;
                    return;
                }
                const int p1 = sm.pp[R], q1 = sm.qq[R];
                const bool v0 = q0 < n, v1 = q1 < n;
                const double cR = aR ? sm.c[R] : 1.0, sR = aR ? sm.s[R] : 0.0;
                const double x00 = Ms[p0 + p1 * LD];
                const double x01 = v1 ? Ms[p0 + q1 * LD] : 0.0;
                const double x10 = v0 ? Ms[q0 + p1 * LD] : 0.0;
                const double x11 = (v0 && v1) ? Ms[q0 + q1 * LD] : 0.0;
                const double y00 = cR * x00 - sR * x01, y01 = sR * x00 + cR * x01;
                const double y10 = cR * x10 - sR * x11, y11 = sR * x10 + cR * x11;
                Ms[p0 + p1 * LD] = cP * y00 - sP * y10;
                if (v1) Ms[p0 + q1 * LD] = cP * y01 - sP * y11;
                if (v0) Ms[q0 + p1 * LD] = sP * y00 + cP * y10;
                if (v0 && v1) Ms[q0 + q1 * LD] = sP * y01 + cP * y11;
            };
            auto pair_of = [&](int P, bool &aP, int &p0, int &q0, double &cP, double &sP) {
                aP = sm.act[P] != 0;
                p0 = sm.pp[P];
                q0 = sm.qq[P];
                cP = aP ? sm.c[P] : 1.0;
                sP = aP ? sm.s[P] : 0.0;
            };
            if (nthr % npair == 0) {
                const int P = tid % npair;
                bool aP;
                int p0, q0;
                double cP, sP;
                pair_of(P, aP, p0, q0, cP, sP);
                for (int R = tid / npair; R < npair; R += nthr / npair) block(P, aP, p0, q0, cP, sP, R);
            } else {
                for (int it = tid; it < npair * npair; it += nthr) {
                    const int P = it % npair;
                    bool aP;
                    int p0, q0;
                    double cP, sP;
                    pair_of(P, aP, p0, q0, cP, sP);
                    block(P, aP, p0, q0, cP, sP, it / npair);
                }
            }
            // V <- V J (columns p, q of every rotated pair)
            if (!LOGV) {
                for (int it = tid; it < n * npair; it += nthr) {
                    const int k = it % n, pr = it / n;
                    if (!sm.act[pr]) continue;
                    const int p = sm.pp[pr], q = sm.qq[pr];
                    const double c = sm.c[pr], s = sm.s[pr];
                    const double u = Vs[k + p * LDV], w = Vs[k + q * LDV];
                    Vs[k + p * LDV] = c * u - s * w;
                    Vs[k + q * LDV] = s * u + c * w;
                }
            }
            __syncthreads();
        }
        const bool any = sm.flag_rot != 0;
        __syncthreads();
        if (!any) converged = true;
        if (tid == 0) sm.flag_rot = 0;
        __syncthreads();
    }
    if (!converged) {
        if (tid == 0) {
            if (LOGV) ctl->status = 2;
            else *info = 2;
        }
        return;
    }
    if (LOGV) {  // the eigenvalues and the replay length; V is formed from the log
        double *lam = reinterpret_cast<double *>(reinterpret_cast<char *>(vglob) + j2_lam_off());
        for (int p = tid; p < n; p += nthr) lam[p] = Ms[p + p * LD];
        if (tid == 0) {
            ctl->status = 0;
            ctl->steps = sweeps_done * (N - 1);  // the last sweep rotated nothing: identity entries
            ctl->esc = esc;
        }
        return;
    }

    // ---- sigma_i = sqrt(lambda_i), ordering, sign of V columns, cast, W
    for (int p = tid; p < n; p += nthr) {
        const double lam = Ms[p + p * LD];
        if (!(lam > 0.0)) atomicMax(&sm.flag_bad, 1);
        sm.ssig[p] = __builtin_sqrt(ldexp(lam > 0.0 ? lam : 0.0, -esc));  // undo the scaling, then round once
        double best = -1.0;
        int barg = 0;
        for (int r = 0; r < n; ++r) {
            const double av = __builtin_fabs(Vs[r + p * LDV]);
            if (av > best) {
                best = av;
                barg = r;
            }
        }
        sm.ssign[p] = Vs[barg + p * LDV] < 0 ? -1.0 : 1.0;
    }
    __syncthreads();
    if (sm.flag_bad) {
        if (tid == 0) *info = sm.flag_bad;
        return;
    }
    for (int p = tid; p < n; p += nthr) {
        const double sp = sm.ssig[p];
        int rk = 0;
        for (int q = 0; q < n; ++q) {
            const double sq = sm.ssig[q];
            rk += (sq > sp) || (sq == sp && q < p);
        }
        sm.srank[p] = rk;
    }
    __syncthreads();
    for (int q = tid; q < n * n; q += nthr) {
        const int r = q % n, p = q / n;
        const int pos = sm.srank[p];
        const TW sw = (TW)sm.ssig[p];
        const TW vw = (TW)(sm.ssign[p] * Vs[r + p * LDV]);
        V[r + (int64_t)pos * ldv] = vw;
        W[r + (int64_t)pos * ldw] = vw / sw;
        if (r == 0) S[pos] = sw;
    }
    if (tid == 0) *info = 0;
}

template <typename TW>
__global__ void __launch_bounds__(1024)
eig_jacobi2_kernel(int n, const double *__restrict__ Mhi, int64_t ldm, TW *__restrict__ S,
                   TW *__restrict__ V, int64_t ldv, TW *__restrict__ W, int64_t ldw,
                   int *__restrict__ info, double tol, int max_sweeps, double *__restrict__ vglob) {
    extern __shared__ __attribute__((aligned(16))) double lds[];
    __shared__ J2Smem sm;
    eig_jacobi2_body<TW, false>(n, Mhi, ldm, S, V, ldv, W, ldw, info, tol, max_sweeps, vglob, sm,
                                lds);
}

// n > 96: the Jacobi on M alone, the rotations logged to the workspace
template <typename TW>
__global__ void __launch_bounds__(1024)
eig_jacobi2_log_kernel(int n, const double *__restrict__ Mhi, int64_t ldm, double tol,
                       int max_sweeps, double *__restrict__ work) {
    extern __shared__ __attribute__((aligned(16))) double lds[];
    __shared__ J2Smem sm;
    eig_jacobi2_body<TW, true>(n, Mhi, ldm, (TW *)nullptr, (TW *)nullptr, 0, (TW *)nullptr, 0,
                               (int *)nullptr, tol, max_sweeps, work, sm, lds);
}

// V from the rotation log: one wavefront per row r of V.  Lane k holds the row's
// entries in the two columns a_k(s), b_k(s) of pair k at step s of the
// round-robin ordering (a_0 = 0; a_k = 1 + (k - 1 + s) mod (N - 1);
// b_k = 1 + (N - 2 - k + s) mod (N - 1)), so each rotation is lane-local; from
// step s to s + 1 the a-entries move one lane down and the b-entries one lane up
// (lane npair - 1 takes its own b-entry as its a-entry, lane 0 takes lane 1's
// a-entry as its b-entry, a_0 stays).  Rows start as those of the identity.
__global__ void __launch_bounds__(256)
eig_jacobi2_vapply_kernel(int n, const double *__restrict__ work, double *__restrict__ Vw) {
    const J2Ctl *ctl = reinterpret_cast<const J2Ctl *>(work);
    if (ctl->status != 0) return;  // written by the previous launch
    const int N = n + (n & 1), npair = N / 2;
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (r >= n) return;  // whole wavefront
    const double *vlog = reinterpret_cast<const double *>(reinterpret_cast<const char *>(work) +
                                                          j2_log_off(n));
    const int steps = ctl->steps;
    const bool act = lane < npair;
    auto col_a = [&](int k, int st) { return k == 0 ? 0 : 1 + (k - 1 + st) % (N - 1); };
    auto col_b = [&](int k, int st) { return 1 + (N - 2 - k + st) % (N - 1); };
    double A = 0.0, B = 0.0;
    if (act) {
        A = col_a(lane, 0) == r ? 1.0 : 0.0;
        B = col_b(lane, 0) == r ? 1.0 : 0.0;
    }
    int st = 0;  // step within the round
    double2 cs = act && steps > 0 ? *reinterpret_cast<const double2 *>(vlog + 2 * lane)
                                  : make_double2(1.0, 0.0);
    for (int g = 0; g < steps; ++g) {
        const double2 cur = cs;
        if (act && g + 1 < steps)
            cs = *reinterpret_cast<const double2 *>(vlog + ((size_t)(g + 1) * npair + lane) * 2);
        if (act) {
            const double c = cur.x, sn = cur.y;
            if (col_a(lane, st) < col_b(lane, st)) {  // (p, q) = (a, b)
                const double u = A, w = B;
                A = c * u - sn * w;
                B = sn * u + c * w;
            } else {  // (p, q) = (b, a)
                const double u = B, w = A;
                B = c * u - sn * w;
                A = sn * u + c * w;
            }
        }
        // move to step st + 1 (the same rule across the end of a round)
        const double Adown = __shfl_down(A, 1);
        const double Bup = __shfl_up(B, 1);
        double nA = A, nB = B;
        if (lane >= 1 && lane < npair - 1) nA = Adown;
        if (lane == npair - 1 && lane != 0) nA = B;
        if (lane >= 1 && lane < npair) nB = Bup;
        if (lane == 0) nB = npair > 1 ? Adown : B;
        A = nA;
        B = nB;
        st = st + 1 == N - 1 ? 0 : st + 1;
    }
    if (act) {
        const int a = col_a(lane, st), b = col_b(lane, st);
        if (a < n) Vw[r + (size_t)a * n] = A;
        if (b < n) Vw[r + (size_t)b * n] = B;
    }
}

// sigma_i = sqrt(lambda_i 2^-esc), ordering, sign rule, casts and W from the
// eigenvalues and V of the log form; writes *info
template <typename TW>
__global__ void __launch_bounds__(1024)
eig_jacobi2_final_kernel(int n, const double *__restrict__ work, const double *__restrict__ Vw,
                         TW *__restrict__ S, TW *__restrict__ V, int64_t ldv, TW *__restrict__ W,
                         int64_t ldw, int *__restrict__ info) {
    __shared__ double ssig[GSVD_KMAX_N], ssign[GSVD_KMAX_N];
    __shared__ int srank[GSVD_KMAX_N];
    __shared__ int bad;
    const J2Ctl *ctl = reinterpret_cast<const J2Ctl *>(work);
    const int status = ctl->status;  // written by an earlier launch
    const int tid = threadIdx.x, nthr = blockDim.x;
    if (status != 0) {
        if (tid == 0) *info = status;
        return;
    }
    const double *lam = reinterpret_cast<const double *>(reinterpret_cast<const char *>(work) +
                                                         j2_lam_off());
    const int esc = ctl->esc;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int p = tid; p < n; p += nthr) {
        const double l = lam[p];
        if (!(l > 0.0)) atomicMax(&bad, 1);
        ssig[p] = __builtin_sqrt(ldexp(l > 0.0 ? l : 0.0, -esc));
        double best = -1.0;
        int barg = 0;
        for (int r = 0; r < n; ++r) {
            const double av = __builtin_fabs(Vw[r + (size_t)p * n]);
            if (av > best) {
                best = av;
                barg = r;
            }
        }
        ssign[p] = Vw[barg + (size_t)p * n] < 0 ? -1.0 : 1.0;
    }
    __syncthreads();
    if (bad) {
        if (tid == 0) *info = 1;
        return;
    }
    for (int p = tid; p < n; p += nthr) {
        const double sp = ssig[p];
        int rk = 0;
        for (int q = 0; q < n; ++q) {
            const double sq = ssig[q];
            rk += (sq > sp) || (sq == sp && q < p);
        }
        srank[p] = rk;
    }
    __syncthreads();
    for (int q = tid; q < n * n; q += nthr) {
        const int r = q % n, p = q / n;
        const int pos = srank[p];
        const TW sw = (TW)ssig[p];
        const TW vw = (TW)(ssign[p] * Vw[r + (size_t)p * n]);
        V[r + (int64_t)pos * ldv] = vw;
        W[r + (int64_t)pos * ldw] = vw / sw;
        if (r == 0) S[pos] = sw;
    }
    if (tid == 0) *info = 0;
}

// Batched: one workgroup per problem, largest n first; tol <= 0 selects n u_h.
// vwork: the problems' V scratch (n x n FP64 each) when max_n > 96, else null.
template <typename TW>
__global__ void __launch_bounds__(1024)
eig_jacobi2_batched_kernel(const BatchMat *__restrict__ tab, const int *__restrict__ order,
                           int batch, double tol, int max_sweeps, int vglobal) {
    extern __shared__ __attribute__((aligned(16))) double lds[];
    __shared__ J2Smem sm;
    const BatchMat &d = tab[order[batch - 1 - (int)blockIdx.x]];
    const double t = tol > 0.0 ? tol : (double)d.n * 0x1p-53;
    // the V scratch sits in the problem's partial-sum area, which the Gram no longer needs
    eig_jacobi2_body<TW, false>(d.n, d.Mhi, d.n, (TW *)d.S, (TW *)d.V, d.ldv, (TW *)d.W, d.n,
                                d.info, t, max_sweeps, vglobal ? d.part : nullptr, sm, lds);
}

bool j2_v_in_lds(int64_t n) { return n <= GSVD_KMAX_N_F64; }

size_t j2_lds_bytes(int64_t n) {
    const size_t m = (size_t)n * j2_ldm((int)n) * sizeof(double);
    return j2_v_in_lds(n) ? m + (size_t)n * n * sizeof(double) : m;
}

size_t j2_work_bytes(int64_t n, int max_sweeps) {
    if (j2_v_in_lds(n)) return 0;
    return j2_v_off((int)n, max_sweeps) + (size_t)n * n * sizeof(double);
}

static int j2_threads(int64_t n) {
    const int64_t items = n * ((n + 1) / 2);
    int64_t t = ((items + 63) / 64) * 64;
    if (t < 64) t = 64;
    if (t > 1024) t = 1024;
    return (int)t;
}

hipError_t eig_jacobi2_launch(int working, int64_t n, const double *Mhi, int64_t ldm, void *S,
                              void *V, int64_t ldv, void *W, int64_t ldw, int *info, double tol,
                              int max_sweeps, void *work, hipStream_t st) {
    if (working != 0 || n < 1 || n > GSVD_KMAX_N) return hipErrorInvalidValue;
    if (!j2_v_in_lds(n) && work == nullptr) return hipErrorInvalidValue;
    const size_t lds = j2_lds_bytes(n);
    if (!j2_v_in_lds(n)) {  // the rotation-log form: Jacobi on M, V replayed per row, epilogue
        auto kl = eig_jacobi2_log_kernel<float>;
        hipError_t err = hipFuncSetAttribute((const void *)kl,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (err != hipSuccess) return err;
        double *wk = (double *)work;
        double *Vw = (double *)((char *)work + j2_v_off((int)n, max_sweeps));
        hipLaunchKernelGGL(kl, dim3(1), dim3(j2_threads(n)), lds, st, (int)n, Mhi, ldm, tol,
                           max_sweeps, wk);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        hipLaunchKernelGGL(eig_jacobi2_vapply_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0,
                           st, (int)n, (const double *)wk, Vw);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        hipLaunchKernelGGL(eig_jacobi2_final_kernel<float>, dim3(1), dim3(1024), 0, st, (int)n,
                           (const double *)wk, (const double *)Vw, (float *)S, (float *)V, ldv,
                           (float *)W, ldw, info);
        return hipGetLastError();
    }
    auto k = eig_jacobi2_kernel<float>;
    hipError_t err = hipFuncSetAttribute((const void *)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3(1), dim3(j2_threads(n)), lds, st, (int)n, Mhi, ldm, (float *)S,
                       (float *)V, ldv, (float *)W, ldw, info, tol, max_sweeps,
                       j2_v_in_lds(n) ? nullptr : (double *)work);
    return hipGetLastError();
}

hipError_t eig_jacobi2_batched_launch(int working, const BatchMat *tab, const int *order, int batch,
                                      int max_n, double tol, int max_sweeps, hipStream_t st) {
    if (working != 0 || batch < 1 || max_n < 1 || max_n > GSVD_KMAX_N) return hipErrorInvalidValue;
    const size_t lds = j2_lds_bytes(max_n);
    auto k = eig_jacobi2_batched_kernel<float>;
    hipError_t err = hipFuncSetAttribute((const void *)k,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3((unsigned)batch), dim3(j2_threads(max_n)), lds, st, tab, order,
                       batch, tol, max_sweeps, j2_v_in_lds(max_n) ? 0 : 1);
    return hipGetLastError();
}

}  // namespace gsvd

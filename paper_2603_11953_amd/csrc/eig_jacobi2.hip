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
//      applied as M <- J^T M J (a column pass, then a row pass, over all pairs
//      of the step at once) and V <- V J; the 2x2 block is then set to
//      (m_pp - t m_pq, 0, 0, m_qq + t m_pq).
//   3. Stop after a sweep without rotation.  lambda_i = m_ii, sigma_i =
//      sqrt(lambda_i) (eq. (sqrt)); ordering, sign rule and the casts of
//      Alg. 1 steps 4-5 as in the Algorithm 2 kernel; W = fl(V Sigma^-1).
// V is FP64 in LDS for n <= 96 and in the caller's workspace otherwise.
#include <hip/hip_runtime.h>

#include "gsvd_internal.hpp"

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

template <typename TW>
__device__ __forceinline__ void eig_jacobi2_body(int n, const double *__restrict__ Mhi, int64_t ldm,
                                                 TW *__restrict__ S, TW *__restrict__ V,
                                                 int64_t ldv, TW *__restrict__ W, int64_t ldw,
                                                 int *__restrict__ info, double tol, int max_sweeps,
                                                 double *__restrict__ vglob, J2Smem &sm,
                                                 double *lds) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int LD = j2_ldm(n);
    double *Ms = lds;
    double *Vs = vglob != nullptr ? vglob : lds + (size_t)n * LD;
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
        if (tid == 0) *info = sm.flag_bad;
        return;
    }
    const int esc = -sm.emax;  // M <- 2^esc M: the largest diagonal entry in [1, 2)
    for (int q = tid; q < n * n; q += nthr) {
        const int i = q % n, j = q / n;
        Ms[i + j * LD] = ldexp(Mhi[i + (int64_t)j * ldm], esc);
        Vs[i + j * LDV] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();

    const int N = n + (n & 1);
    const int npair = N / 2;
    const double tol2 = tol * tol;
    bool converged = (n == 1);
    for (int sw = 0; sw < max_sweeps && !converged; ++sw) {
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
                        const double zeta = (aqq - app) / (2.0 * apq);
                        const double t = (zeta >= 0 ? 1.0 : -1.0) /
                                         (__builtin_fabs(zeta) + __builtin_sqrt(__builtin_fma(zeta, zeta, 1.0)));
                        const double c = 1.0 / __builtin_sqrt(__builtin_fma(t, t, 1.0));
                        sm.c[pr] = c;
                        sm.s[pr] = c * t;
                        sm.app[pr] = app - t * apq;
                        sm.aqq[pr] = aqq + t * apq;
                        act = 1;
                        sm.flag_rot = 1;
                    }
                }
                sm.act[pr] = act;
            }
            __syncthreads();
            // (b) columns p, q of M and of V: M <- M J, V <- V J
            for (int it = tid; it < n * npair; it += nthr) {
                const int k = it % n, pr = it / n;
                if (!sm.act[pr]) continue;
                const int p = sm.pp[pr], q = sm.qq[pr];
                const double c = sm.c[pr], s = sm.s[pr];
                const double x = Ms[k + p * LD], y = Ms[k + q * LD];
                Ms[k + p * LD] = c * x - s * y;
                Ms[k + q * LD] = s * x + c * y;
                const double u = Vs[k + p * LDV], w = Vs[k + q * LDV];
                Vs[k + p * LDV] = c * u - s * w;
                Vs[k + q * LDV] = s * u + c * w;
            }
            __syncthreads();
            // (c) rows p, q of M: M <- J^T M
            for (int it = tid; it < n * npair; it += nthr) {
                const int k = it % n, pr = it / n;
                if (!sm.act[pr]) continue;
                const int p = sm.pp[pr], q = sm.qq[pr];
                const double c = sm.c[pr], s = sm.s[pr];
                const double x = Ms[p + k * LD], y = Ms[q + k * LD];
                Ms[p + k * LD] = c * x - s * y;
                Ms[q + k * LD] = s * x + c * y;
            }
            __syncthreads();
            // (d) the 2x2 block of each rotated pair, from its closed form
            for (int pr = tid; pr < npair; pr += nthr) {
                if (!sm.act[pr]) continue;
                const int p = sm.pp[pr], q = sm.qq[pr];
                Ms[p + p * LD] = sm.app[pr];
                Ms[q + q * LD] = sm.aqq[pr];
                Ms[p + q * LD] = 0.0;
                Ms[q + p * LD] = 0.0;
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
        if (tid == 0) *info = 2;
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
    extern __shared__ double lds[];
    __shared__ J2Smem sm;
    eig_jacobi2_body<TW>(n, Mhi, ldm, S, V, ldv, W, ldw, info, tol, max_sweeps, vglob, sm, lds);
}

// Batched: one workgroup per problem, largest n first; tol <= 0 selects n u_h.
// vwork: the problems' V scratch (n x n FP64 each) when max_n > 96, else null.
template <typename TW>
__global__ void __launch_bounds__(1024)
eig_jacobi2_batched_kernel(const BatchMat *__restrict__ tab, const int *__restrict__ order,
                           int batch, double tol, int max_sweeps, int vglobal) {
    extern __shared__ double lds[];
    __shared__ J2Smem sm;
    const BatchMat &d = tab[order[batch - 1 - (int)blockIdx.x]];
    const double t = tol > 0.0 ? tol : (double)d.n * 0x1p-53;
    // the V scratch sits in the problem's partial-sum area, which the Gram no longer needs
    eig_jacobi2_body<TW>(d.n, d.Mhi, d.n, (TW *)d.S, (TW *)d.V, d.ldv, (TW *)d.W, d.n, d.info, t,
                         max_sweeps, vglobal ? d.part : nullptr, sm, lds);
}

bool j2_v_in_lds(int64_t n) { return n <= GSVD_KMAX_N_F64; }

size_t j2_lds_bytes(int64_t n) {
    const size_t m = (size_t)n * j2_ldm((int)n) * sizeof(double);
    return j2_v_in_lds(n) ? m + (size_t)n * n * sizeof(double) : m;
}

size_t j2_work_bytes(int64_t n) { return j2_v_in_lds(n) ? 0 : (size_t)n * n * sizeof(double); }

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

// Eigensolver stage: Algorithm 2 of the paper inside one workgroup.
//
//   1. Column scaling: d_j = sqrt(m_jj) = ||a_j|| (the D of A = B D), rounded to
//      a power of two 2^e_j so that H = D~^-1 M_h D~^-1 is formed exactly.
//   2. Cholesky H = R_H^T R_H at the Gram precision (double-double for FP64
//      working, where M_h carries a low plane; FP64 otherwise), right-looking,
//      on the packed upper triangle held in LDS.  (Alg. 2 step 1.)
//   3. R = working(R_H) D~  (Alg. 2 step 2; the power-of-two scaling is exact).
//   4. One-sided Jacobi SVD of R (Alg. 2 step 3): plane rotations applied to
//      the columns of R (Hestenes), accumulated in V = J_1 J_2 ..., until
//      every pair of columns is numerically orthogonal,
//      |r_p^T r_q| <= tol ||r_p|| ||r_q||.  R = R_H D~ is column scaled, the
//      setting in which right-handed one-sided Jacobi keeps each column's
//      rounding errors relative to that column's norm (Demmel-Veselic), and
//      the same rotations applied to V keep A V Sigma^-1 orthonormal however
//      graded the columns of A are.  Round-robin ordering: n/2 disjoint pairs
//      per step, one 16-lane group per pair, all in LDS.
//   5. sigma_p = ||r_p||; ordering sigma_1 >= ... >= sigma_n; each V column
//      signed so its entry of largest magnitude is positive (lowest index on
//      ties); Sigma and V cast to the working precision (Alg. 1 steps 4-5);
//      W = fl(V Sigma^-1) in the working precision (the parenthesisation of
//      Alg. 1 step 6).
//   Storage of R and V during the Jacobi: FP64 for FP64 working (n <= 96 fits
//   LDS), FP32 for FP32 working (the SVD of R "at precision u"; n <= 128),
//   with the dot products and rotation parameters evaluated in FP64.
#include <hip/hip_runtime.h>

#include "dd_device.hpp"
#include "gsvd_internal.hpp"

namespace gsvd {

constexpr int GRP = 16;  // lanes per Jacobi pair
constexpr int EIG_MAXREG = 10;  // packed entries per lane while repacking R

struct EigShared {
    int flag_rot;
    int flag_bad;  // GSVD info code, 0 = fine
};

__device__ __forceinline__ int packed_idx(int i, int j) { return j * (j + 1) / 2 + i; }  // i <= j

template <typename TW, typename TS, bool DDGRAM>
__global__ void __launch_bounds__(1024)
eig_chol_jacobi1_kernel(int n, const double *__restrict__ Mhi, const double *__restrict__ Mlo,
                        int64_t ldm, TW *__restrict__ S, TW *__restrict__ V, int64_t ldv,
                        TW *__restrict__ W, int64_t ldw, int *__restrict__ info, double tol,
                        int max_sweeps) {
    extern __shared__ double lds[];
    __shared__ EigShared sh;
    __shared__ int sexp[GSVD_KMAX_N];
    __shared__ double ssig[GSVD_KMAX_N];
    __shared__ int srank[GSVD_KMAX_N];
    __shared__ double ssign[GSVD_KMAX_N];

    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int npk = n * (n + 1) / 2;

    if (tid == 0) {
        sh.flag_rot = 0;
        sh.flag_bad = 0;
    }
    __syncthreads();

    // ---- 1. scaling exponents and input checks
    for (int j = tid; j < n; j += nthr) {
        double mjj = Mhi[j + (int64_t)j * ldm];
        if (!(mjj > 0.0) || !__builtin_isfinite(mjj)) {
            atomicMax(&sh.flag_bad, __builtin_isfinite(mjj) ? 1 : 3);
            sexp[j] = 0;
        } else {
            sexp[j] = ilogb(__builtin_sqrt(mjj));
        }
    }
    for (int q = tid; q < n * n; q += nthr) {
        int i = q % n, j = q / n;
        double v = Mhi[i + (int64_t)j * ldm];
        if (!__builtin_isfinite(v)) atomicMax(&sh.flag_bad, 3);
    }
    __syncthreads();
    if (sh.flag_bad) {
        if (tid == 0) *info = sh.flag_bad;
        return;
    }

    // ---- 2. H = D~^-1 M D~^-1 (exact), packed upper, dd in LDS; Cholesky
    dd_t *H = reinterpret_cast<dd_t *>(lds);
    for (int q = tid; q < npk; q += nthr) {
        // decode packed q -> (i, j), i <= j
        int j = (int)((__builtin_sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
        while (j * (j + 1) / 2 > q) --j;
        while ((j + 1) * (j + 2) / 2 <= q) ++j;
        int i = q - j * (j + 1) / 2;
        int sc = -(sexp[i] + sexp[j]);
        double hi = ldexp(Mhi[i + (int64_t)j * ldm], sc);
        double lo = DDGRAM ? ldexp(Mlo[i + (int64_t)j * ldm], sc) : 0.0;
        H[q] = dd_t{hi, lo};
    }
    __syncthreads();

    for (int k = 0; k < n; ++k) {
        dd_t hkk = H[packed_idx(k, k)];
        if (!(hkk.hi > 0.0)) {  // uniform across the workgroup
            if (tid == 0) *info = 1;
            return;
        }
        dd_t rkk = DDGRAM ? dd_sqrt(hkk) : dd_t{__builtin_sqrt(hkk.hi), 0.0};
        dd_t inv = DDGRAM ? dd_div(dd_t{1.0, 0.0}, rkk) : dd_t{1.0 / rkk.hi, 0.0};
        __syncthreads();  // everyone has read H(k,k)
        for (int j = k + 1 + tid; j < n; j += nthr) {
            int q = packed_idx(k, j);
            H[q] = DDGRAM ? dd_mul(H[q], inv) : dd_t{H[q].hi / rkk.hi, 0.0};
        }
        if (tid == 0) H[packed_idx(k, k)] = rkk;
        __syncthreads();
        // trailing update of the (n-k-1) x (n-k-1) upper triangle
        const int L = n - k - 1;
        const int cnt = L * (L + 1) / 2;
        for (int f = tid; f < cnt; f += nthr) {
            int jj = (int)((__builtin_sqrt(8.0 * f + 1.0) - 1.0) * 0.5);
            while (jj * (jj + 1) / 2 > f) --jj;
            while ((jj + 1) * (jj + 2) / 2 <= f) ++jj;
            int ii = f - jj * (jj + 1) / 2;
            int i = k + 1 + ii, j = k + 1 + jj;
            dd_t rki = H[packed_idx(k, i)], rkj = H[packed_idx(k, j)];
            int q = packed_idx(i, j);
            if (DDGRAM) {
                H[q] = dd_sub(H[q], dd_mul(rki, rkj));
            } else {
                H[q].hi = __builtin_fma(-rki.hi, rkj.hi, H[q].hi);
            }
        }
        __syncthreads();
    }

    // ---- 3. R = working(R_H) D~ as an n x n column-major TS matrix Y in LDS,
    //      V = I next to it.  The packed dd triangle overlaps both, so every
    //      lane first lifts its share of R into registers.
    //      (eig_threads keeps ceil(npk / nthr) <= EIG_MAXREG for every n <= GSVD_KMAX_N)
    double rv[EIG_MAXREG];
#pragma unroll
    for (int c = 0; c < EIG_MAXREG; ++c) {
        const int q = tid + c * nthr;
        rv[c] = 0.0;
        if (q < npk) {
            int j = (int)((__builtin_sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
            while (j * (j + 1) / 2 > q) --j;
            while ((j + 1) * (j + 2) / 2 <= q) ++j;
            const double r = (double)(TW)H[q].hi;  // round to the working precision
            rv[c] = ldexp(r, sexp[j]);
        }
    }
    __syncthreads();
    TS *Y = reinterpret_cast<TS *>(lds);
    TS *Vs = Y + n * n;
    for (int q = tid; q < n * n; q += nthr) {
        Y[q] = (TS)0;
        Vs[q] = (q % n == q / n) ? (TS)1 : (TS)0;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < EIG_MAXREG; ++c) {
        const int q = tid + c * nthr;
        if (q < npk) {
            int j = (int)((__builtin_sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
            while (j * (j + 1) / 2 > q) --j;
            while ((j + 1) * (j + 2) / 2 <= q) ++j;
            const int i = q - j * (j + 1) / 2;
            Y[i + j * n] = (TS)rv[c];  // R(i, j), exact in TS (already rounded to TW)
        }
    }
    __syncthreads();

    // ---- 4. one-sided Jacobi on the columns of Y = R, rotations accumulated in V
    const int N = n + (n & 1);  // even number of players; player n is a dummy
    const int npair = N / 2;
    const int grp = tid / GRP, gl = tid % GRP;
    const int ngrp = nthr / GRP;
    bool converged = (n == 1);
    for (int sw = 0; sw < max_sweeps && !converged; ++sw) {
        for (int step = 0; step < N - 1; ++step) {
            for (int pr = grp; pr < npair; pr += ngrp) {
                // round-robin: position 0 holds player 0, position t >= 1 holds
                // player 1 + (t - 1 + step) mod (N - 1); pair pr = positions pr, N-1-pr
                int a = (pr == 0) ? 0 : 1 + (pr - 1 + step) % (N - 1);
                int t2 = N - 1 - pr;
                int b = 1 + (t2 - 1 + step) % (N - 1);
                int p = a < b ? a : b, q = a < b ? b : a;
                if (q >= n) continue;  // dummy player (uniform within the group)
                TS *yp = Y + p * n, *yq = Y + q * n;
                double al = 0, be = 0, ga = 0;
                for (int r = gl; r < n; r += GRP) {
                    double x = (double)yp[r], y = (double)yq[r];
                    al = __builtin_fma(x, x, al);
                    be = __builtin_fma(y, y, be);
                    ga = __builtin_fma(x, y, ga);
                }
#pragma unroll
                for (int off = GRP / 2; off >= 1; off >>= 1) {
                    al += __shfl_xor(al, off, GRP);
                    be += __shfl_xor(be, off, GRP);
                    ga += __shfl_xor(ga, off, GRP);
                }
                // the xor butterfly leaves bitwise identical sums in all 16 lanes
                if (__builtin_fabs(ga) > tol * __builtin_sqrt(al) * __builtin_sqrt(be)) {
                    double zeta = (be - al) / (2.0 * ga);
                    double t;
                    double az = __builtin_fabs(zeta);
                    if (az > 1e150) {
                        t = 0.5 / zeta;
                    } else {
                        t = 1.0 / (az + __builtin_sqrt(1.0 + zeta * zeta));
                        if (zeta < 0) t = -t;
                    }
                    double c = 1.0 / __builtin_sqrt(1.0 + t * t);
                    double s = c * t;
                    TS *vp = Vs + p * n, *vq = Vs + q * n;
                    for (int r = gl; r < n; r += GRP) {
                        double x = (double)yp[r], y = (double)yq[r];
                        yp[r] = (TS)(c * x - s * y);
                        yq[r] = (TS)(s * x + c * y);
                        double u = (double)vp[r], w = (double)vq[r];
                        vp[r] = (TS)(c * u - s * w);
                        vq[r] = (TS)(s * u + c * w);
                    }
                    if (gl == 0) sh.flag_rot = 1;
                }
            }
            __syncthreads();
        }
        const bool any = sh.flag_rot != 0;
        __syncthreads();
        if (!any) converged = true;
        if (tid == 0) sh.flag_rot = 0;
        __syncthreads();
    }
    if (!converged) {
        if (tid == 0) *info = 2;
        return;
    }

    // ---- 5. sigma_p = ||y_p||, ordering, sign of V columns, cast, W
    for (int p = grp; p < n; p += ngrp) {
        const TS *yp = Y + p * n;
        const TS *vp = Vs + p * n;
        double ss = 0;
        double best = -1.0;
        int barg = 0;
        for (int r = gl; r < n; r += GRP) {
            double x = (double)yp[r];
            ss = __builtin_fma(x, x, ss);
            double av = __builtin_fabs((double)vp[r]);
            if (av > best) { best = av; barg = r; }
        }
#pragma unroll
        for (int off = GRP / 2; off >= 1; off >>= 1) {
            ss += __shfl_xor(ss, off, GRP);
            double ob = __shfl_xor(best, off, GRP);
            int oa = __shfl_xor(barg, off, GRP);
            if (ob > best || (ob == best && oa < barg)) { best = ob; barg = oa; }
        }
        if (gl == 0) {
            ssig[p] = __builtin_sqrt(ss);
            ssign[p] = vp[barg] < 0 ? -1.0 : 1.0;
        }
    }
    __syncthreads();
    for (int p = tid; p < n; p += nthr) {
        double sp = ssig[p];
        int rk = 0;
        for (int q = 0; q < n; ++q) {
            double sq = ssig[q];
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
        int r = q % n, p = q / n;
        int pos = srank[p];
        TW sw = (TW)ssig[p];
        TW vw = (TW)(ssign[p] * (double)Vs[r + p * n]);
        V[r + (int64_t)pos * ldv] = vw;
        W[r + (int64_t)pos * ldw] = vw / sw;
        if (r == 0) S[pos] = sw;
    }
    if (tid == 0) *info = 0;
}

size_t eig_lds_bytes(int working, int64_t n) {
    size_t packed = (size_t)(n * (n + 1) / 2) * sizeof(dd_t);
    size_t full = 2 * (size_t)(n * n) * (working == 1 ? sizeof(double) : sizeof(float));
    return packed > full ? packed : full;
}

int eig_max_n(int working) { return working == 1 ? GSVD_KMAX_N_F64 : GSVD_KMAX_N; }

int eig_threads(int64_t n) {
    int N = (int)(n + (n & 1));
    int t = GRP * (N / 2);
    if (t < 64) t = 64;
    if (t > 1024) t = 1024;
    t = ((t + 63) / 64) * 64;
    // every lane holds at most EIG_MAXREG packed entries while R is repacked
    const int npk = (int)(n * (n + 1) / 2);
    while ((npk + t - 1) / t > EIG_MAXREG && t < 1024) t += 64;
    return t;
}

hipError_t eig_launch(int working, int64_t n, const double *Mhi, const double *Mlo, int64_t ldm,
                      void *S, void *V, int64_t ldv, void *W, int64_t ldw, int *info, double tol,
                      int max_sweeps, hipStream_t st) {
    const size_t lds = eig_lds_bytes(working, n);
    const int thr = eig_threads(n);
    if (n < 1 || n > eig_max_n(working) || (n * (n + 1) / 2 + thr - 1) / thr > EIG_MAXREG)
        return hipErrorInvalidValue;
    hipError_t err;
    if (working == 1) {
        auto k = eig_chol_jacobi1_kernel<double, double, true>;
        if (Mlo == nullptr) return hipErrorInvalidValue;
        err = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k, dim3(1), dim3(thr), lds, st, (int)n, Mhi, Mlo, ldm, (double *)S,
                           (double *)V, ldv, (double *)W, ldw, info, tol, max_sweeps);
    } else {
        auto k = eig_chol_jacobi1_kernel<float, float, false>;
        err = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k, dim3(1), dim3(thr), lds, st, (int)n, Mhi, Mlo, ldm, (float *)S,
                           (float *)V, ldv, (float *)W, ldw, info, tol, max_sweeps);
    }
    return hipGetLastError();
}

}  // namespace gsvd

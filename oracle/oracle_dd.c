/*
 * oracle_dd.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, CPU-only double-double (dd) reference for the mixed precision
 * Gram-based thin SVD of Carson, Ma and Shao, "Mixed precision thin SVD
 * algorithms based on the Gram matrix" (arXiv 2603.11953).  It exists so that
 * tests, the smoke check and the CPU-baseline leg of the benchmark can check the
 * GPU path; the product path never loads it, and it shares no code, header or
 * table with the GPU library.
 *
 * Every step is Algorithm 1 of the paper carried out with the higher precision
 * set to double-double (unit roundoff about 2^-104):
 *   oracle_gram_dd      Alg. 1 steps 1-2  (cast, Gram M = A^T A; eq. (ATA))
 *   oracle_jacobi2_dd   Alg. 1 step 3     (two-sided cyclic Jacobi eigensolver,
 *                                          the eigensolver of Sec. 2.1 / Remark 1)
 *   oracle_sigma_sort   Alg. 1 steps 3-5  (sigma = sqrt(eigenvalue), eq. (sqrt);
 *                                          ordering sigma_1 >= ... >= sigma_n)
 *   oracle_u_rows_dd    Alg. 1 step 6     (U = A V Sigma^{-1}, eq. (AV-0))
 *   oracle_chol_dd      Alg. 2 step 1     (M = R^T R, R upper triangular)
 *   oracle_orth_dd      the orthogonality measure ||U^T U - I||_F of Thm. 1
 *   oracle_resid_rows   the backward error A - U Sigma V^T of Thm. 1 (eq. (backward))
 *
 * dd arithmetic is written from the published error-free transformations:
 * Knuth's TwoSum, Dekker's FastTwoSum, and the FMA form of TwoProduct
 * (Ogita, Rump, Oishi 2005).  Build with -ffp-contract=off so the compiler does
 * not fuse the additions and multiplications these transformations rely on.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double hi, lo; } dd;

/* ---- error-free transformations ---------------------------------------- */

/* Knuth TwoSum: s + e == a + b exactly, s = fl(a + b). */
static inline dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    dd r = {s, e};
    return r;
}

/* Dekker FastTwoSum: exact when |a| >= |b| (or a == 0). */
static inline dd fast_two_sum(double a, double b) {
    double s = a + b;
    double e = b - (s - a);
    dd r = {s, e};
    return r;
}

/* TwoProduct with FMA: p + e == a * b exactly (no underflow). */
static inline dd two_prod(double a, double b) {
    double p = a * b;
    double e = fma(a, b, -p);
    dd r = {p, e};
    return r;
}

static inline dd dd_from(double a) { dd r = {a, 0.0}; return r; }

/* Accurate dd addition (both parts carried through TwoSum). */
static inline dd dd_add(dd x, dd y) {
    dd s = two_sum(x.hi, y.hi);
    dd t = two_sum(x.lo, y.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}

static inline dd dd_neg(dd x) { dd r = {-x.hi, -x.lo}; return r; }
static inline dd dd_sub(dd x, dd y) { return dd_add(x, dd_neg(y)); }

static inline dd dd_mul(dd x, dd y) {
    dd p = two_prod(x.hi, y.hi);
    p.lo += x.hi * y.lo + x.lo * y.hi;
    return fast_two_sum(p.hi, p.lo);
}

static inline dd dd_mul_d(dd x, double y) {
    dd p = two_prod(x.hi, y);
    p.lo += x.lo * y;
    return fast_two_sum(p.hi, p.lo);
}

/* Long division: three quotient digits, each corrected against the remainder. */
static inline dd dd_div(dd x, dd y) {
    double q1 = x.hi / y.hi;
    dd r = dd_sub(x, dd_mul_d(y, q1));
    double q2 = r.hi / y.hi;
    r = dd_sub(r, dd_mul_d(y, q2));
    double q3 = r.hi / y.hi;
    dd q = fast_two_sum(q1, q2);
    return dd_add(q, dd_from(q3));
}

/* sqrt by one Newton correction of the double root: y + (x - y^2) / (2y). */
static inline dd dd_sqrt(dd x) {
    if (x.hi <= 0.0) return dd_from(x.hi == 0.0 ? 0.0 : NAN);
    double y = sqrt(x.hi);
    dd y2 = two_prod(y, y);
    dd r = dd_sub(x, y2);
    double corr = r.hi / (2.0 * y);
    dd s = fast_two_sum(y, corr);
    /* second correction keeps the last bits honest */
    dd r2 = dd_sub(x, dd_mul(s, s));
    double corr2 = r2.hi / (2.0 * s.hi);
    return dd_add(s, dd_from(corr2));
}

static inline double dd_abs_hi(dd x) { return fabs(x.hi); }

/* ---- Alg. 1 steps 1-2: Gram in double-double ----------------------------- */

/*
 * M = A^T A for an m x n column-major A (lda >= m), FP64 (is_f32 == 0) or FP32
 * (is_f32 != 0).  Every product a_ki * a_kj is formed exactly (TwoProduct) and
 * added to the dd entry with the accurate dd sum.  Rows are cut into `nblk`
 * fixed blocks, each reduced on its own, and the block results are merged in
 * block order, so the result does not depend on the thread count.
 * Output: full symmetric n x n matrices Mhi, Mlo (column-major, leading dim n).
 */
void oracle_gram_dd(int64_t m, int64_t n, const void *A, int64_t lda, int is_f32,
                    double *Mhi, double *Mlo) {
    const int64_t nblk = m < 64 ? 1 : 64;
    const int64_t npair = n * (n + 1) / 2;
    dd *part = (dd *)calloc((size_t)(nblk * npair), sizeof(dd));
    const double *Ad = (const double *)A;
    const float *Af = (const float *)A;

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < nblk; ++b) {
        int64_t r0 = m * b / nblk, r1 = m * (b + 1) / nblk;
        dd *P = part + b * npair;
        int64_t idx = 0;
        for (int64_t j = 0; j < n; ++j) {
            for (int64_t i = 0; i <= j; ++i, ++idx) {
                dd acc = dd_from(0.0);
                for (int64_t k = r0; k < r1; ++k) {
                    double x, y;
                    if (is_f32) {
                        x = (double)Af[k + i * lda];
                        y = (double)Af[k + j * lda];
                    } else {
                        x = Ad[k + i * lda];
                        y = Ad[k + j * lda];
                    }
                    acc = dd_add(acc, two_prod(x, y));
                }
                P[idx] = acc;
            }
        }
    }
    int64_t idx = 0;
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i <= j; ++i, ++idx) {
            dd acc = dd_from(0.0);
            for (int64_t b = 0; b < nblk; ++b) acc = dd_add(acc, part[b * npair + idx]);
            Mhi[i + j * n] = Mhi[j + i * n] = acc.hi;
            Mlo[i + j * n] = Mlo[j + i * n] = acc.lo;
        }
    }
    free(part);
}

/* ---- Alg. 1 step 3: two-sided cyclic Jacobi in double-double -------------- */

/*
 * Eigen-decomposition M = V diag(lambda) V^T of a symmetric n x n dd matrix by
 * the two-sided Jacobi method (cyclic-by-row ordering), the eigensolver the
 * paper recommends for Alg. 1 step 3 (Sec. 2.1; Remark 1).  Each step zeroes
 * m_pq with the symmetric 2x2 Schur rotation of the smaller angle.  A pair is
 * skipped when |m_pq| <= tol * sqrt(m_pp * m_qq) -- the scaled form suggested by
 * eq. (eig-2).  The sweep loop stops after a sweep in which no rotation was
 * applied.
 *
 * In/out: Mhi/Mlo (n x n, col-major, overwritten with the rotated matrix whose
 * diagonal holds the eigenvalues).  Out: Vhi/Vlo (n x n col-major).
 * Returns the number of sweeps used (including the final quiet sweep), or
 * -1 if max_sweeps sweeps all applied rotations (not converged).
 */
int oracle_jacobi2_dd(int64_t n, double *Mhi, double *Mlo, double tol, int max_sweeps,
                      double *Vhi, double *Vlo) {
    dd *M = (dd *)malloc(sizeof(dd) * (size_t)(n * n));
    dd *V = (dd *)malloc(sizeof(dd) * (size_t)(n * n));
    for (int64_t i = 0; i < n * n; ++i) {
        M[i].hi = Mhi[i];
        M[i].lo = Mlo[i];
        V[i] = dd_from(0.0);
    }
    for (int64_t i = 0; i < n; ++i) V[i + i * n] = dd_from(1.0);

    int sweeps = -1;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        int64_t rotated = 0;
        for (int64_t p = 0; p < n - 1; ++p) {
            for (int64_t q = p + 1; q < n; ++q) {
                dd apq = M[p + q * n];
                dd app = M[p + p * n];
                dd aqq = M[q + q * n];
                if (apq.hi == 0.0) continue;
                if (dd_abs_hi(apq) <= tol * sqrt(fabs(app.hi) * fabs(aqq.hi))) continue;
                ++rotated;
                /* zeta = (a_qq - a_pp) / (2 a_pq) */
                dd zeta = dd_div(dd_sub(aqq, app), dd_mul_d(apq, 2.0));
                /* t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)); t = 1 when zeta = 0 */
                dd t;
                if (zeta.hi == 0.0) {
                    t = dd_from(1.0);
                } else {
                    dd az = zeta.hi < 0 ? dd_neg(zeta) : zeta;
                    dd root = dd_sqrt(dd_add(dd_from(1.0), dd_mul(zeta, zeta)));
                    t = dd_div(dd_from(1.0), dd_add(az, root));
                    if (zeta.hi < 0) t = dd_neg(t);
                }
                dd c = dd_div(dd_from(1.0), dd_sqrt(dd_add(dd_from(1.0), dd_mul(t, t))));
                dd s = dd_mul(c, t);
                /* columns p, q of M <- M J ; rows p, q <- J^T M; then fix the 2x2 block */
                for (int64_t k = 0; k < n; ++k) {
                    if (k == p || k == q) continue;
                    dd akp = M[k + p * n], akq = M[k + q * n];
                    dd nkp = dd_sub(dd_mul(c, akp), dd_mul(s, akq));
                    dd nkq = dd_add(dd_mul(s, akp), dd_mul(c, akq));
                    M[k + p * n] = nkp; M[p + k * n] = nkp;
                    M[k + q * n] = nkq; M[q + k * n] = nkq;
                }
                M[p + p * n] = dd_sub(app, dd_mul(t, apq));
                M[q + q * n] = dd_add(aqq, dd_mul(t, apq));
                M[p + q * n] = dd_from(0.0);
                M[q + p * n] = dd_from(0.0);
                for (int64_t k = 0; k < n; ++k) {
                    dd vkp = V[k + p * n], vkq = V[k + q * n];
                    V[k + p * n] = dd_sub(dd_mul(c, vkp), dd_mul(s, vkq));
                    V[k + q * n] = dd_add(dd_mul(s, vkp), dd_mul(c, vkq));
                }
            }
        }
        if (rotated == 0) { sweeps = sw + 1; break; }
    }
    for (int64_t i = 0; i < n * n; ++i) {
        Mhi[i] = M[i].hi; Mlo[i] = M[i].lo;
        Vhi[i] = V[i].hi; Vlo[i] = V[i].lo;
    }
    free(M);
    free(V);
    return sweeps;
}

/* ---- Alg. 1 steps 3-5: sigma = sqrt(lambda), ordering, sign -------------- */

/*
 * Given the eigenvalues lam (dd, length n) and eigenvectors V (dd, n x n),
 * form sigma_i = sqrt(lambda_i) in dd (eq. (sqrt)), order them descending with a
 * stable sort, permute the columns of V to match, and flip each column of V so
 * that its entry of largest magnitude is positive (lowest index on ties).
 * Returns 1 if some lambda_i <= 0 (M not positive definite: A is not of full
 * column rank at this precision), else 0.  Outputs overwrite the inputs.
 */
int oracle_sigma_sort(int64_t n, double *lam_hi, double *lam_lo, double *Vhi, double *Vlo) {
    int bad = 0;
    dd *sig = (dd *)malloc(sizeof(dd) * (size_t)n);
    int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        dd l = {lam_hi[i], lam_lo[i]};
        if (!(l.hi > 0.0)) bad = 1;
        sig[i] = dd_sqrt(l);
        perm[i] = i;
    }
    /* stable insertion sort, descending */
    for (int64_t i = 1; i < n; ++i) {
        int64_t pi = perm[i];
        int64_t j = i - 1;
        while (j >= 0) {
            dd a = sig[perm[j]], b = sig[pi];
            int less = (a.hi < b.hi) || (a.hi == b.hi && a.lo < b.lo);
            if (!less) break;
            perm[j + 1] = perm[j];
            --j;
        }
        perm[j + 1] = pi;
    }
    double *nvh = (double *)malloc(sizeof(double) * (size_t)(n * n));
    double *nvl = (double *)malloc(sizeof(double) * (size_t)(n * n));
    for (int64_t c = 0; c < n; ++c) {
        int64_t src = perm[c];
        lam_hi[c] = sig[src].hi;
        lam_lo[c] = sig[src].lo;
        int64_t arg = 0;
        double best = -1.0;
        for (int64_t k = 0; k < n; ++k) {
            double a = fabs(Vhi[k + src * n]);
            if (a > best) { best = a; arg = k; }
        }
        double sgn = Vhi[arg + src * n] < 0 ? -1.0 : 1.0;
        for (int64_t k = 0; k < n; ++k) {
            nvh[k + c * n] = sgn * Vhi[k + src * n];
            nvl[k + c * n] = sgn * Vlo[k + src * n];
        }
    }
    memcpy(Vhi, nvh, sizeof(double) * (size_t)(n * n));
    memcpy(Vlo, nvl, sizeof(double) * (size_t)(n * n));
    free(nvh); free(nvl); free(sig); free(perm);
    return bad;
}

/* ---- Alg. 1 step 6: U = A V Sigma^{-1} in dd, for selected rows ------------ */

/*
 * For each row index rows[r] (0-based), U(r, i) = (sum_j a_{row,j} v_{j,i}) / sigma_i
 * evaluated in dd.  A as in oracle_gram_dd; V (dd, n x n col-major) and sigma
 * (dd, length n).  Output Uhi/Ulo: nrows x n, column-major with leading dim nrows.
 */
void oracle_u_rows_dd(int64_t n, const void *A, int64_t lda, int is_f32,
                      const double *Vhi, const double *Vlo,
                      const double *shi, const double *slo,
                      int64_t nrows, const int64_t *rows, double *Uhi, double *Ulo) {
    const double *Ad = (const double *)A;
    const float *Af = (const float *)A;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t k = rows[r];
        for (int64_t i = 0; i < n; ++i) {
            dd acc = dd_from(0.0);
            for (int64_t j = 0; j < n; ++j) {
                double a = is_f32 ? (double)Af[k + j * lda] : Ad[k + j * lda];
                dd v = {Vhi[j + i * n], Vlo[j + i * n]};
                acc = dd_add(acc, dd_mul_d(v, a));
            }
            dd s = {shi[i], slo[i]};
            dd u = dd_div(acc, s);
            Uhi[r + i * nrows] = u.hi;
            Ulo[r + i * nrows] = u.lo;
        }
    }
}

/* ---- Alg. 2 step 1: Cholesky in dd ---------------------------------------- */

/*
 * M = R^T R with R upper triangular (column-major n x n, lower part zeroed),
 * computed in dd by the column-oriented (Cholesky-Crout) recurrence
 *   r_jj = sqrt(m_jj - sum_{k<j} r_kj^2),  r_ij = (m_ij - sum_{k<i} r_ki r_kj) / r_ii.
 * Returns 0 on success or j+1 if the pivot of column j is not positive.
 */
int oracle_chol_dd(int64_t n, const double *Mhi, const double *Mlo, double *Rhi, double *Rlo) {
    dd *R = (dd *)calloc((size_t)(n * n), sizeof(dd));
    int info = 0;
    for (int64_t j = 0; j < n && !info; ++j) {
        for (int64_t i = 0; i <= j; ++i) {
            dd s = {Mhi[i + j * n], Mlo[i + j * n]};
            for (int64_t k = 0; k < i; ++k) s = dd_sub(s, dd_mul(R[k + i * n], R[k + j * n]));
            if (i < j) {
                R[i + j * n] = dd_div(s, R[i + i * n]);
            } else {
                if (!(s.hi > 0.0)) { info = (int)(j + 1); break; }
                R[j + j * n] = dd_sqrt(s);
            }
        }
    }
    for (int64_t i = 0; i < n * n; ++i) { Rhi[i] = R[i].hi; Rlo[i] = R[i].lo; }
    free(R);
    return info;
}

/* ---- A = B D: the column scaling of Sec. 1 and Thm. 1 -------------------- */

/*
 * With d_j = sqrt(m_jj) = ||a_j||_2 (the diagonal of D in A = B D, B with unit
 * columns), form H = D^{-1} M D^{-1} = B^T B in dd.  d is returned in dhi/dlo.
 * The eigenvalues of H give kappa(B) = sqrt(lambda_max(H) / lambda_min(H)).
 */
void oracle_equilibrate_dd(int64_t n, const double *Mhi, const double *Mlo,
                           double *Hhi, double *Hlo, double *dhi, double *dlo) {
    dd *d = (dd *)malloc(sizeof(dd) * (size_t)n);
    for (int64_t j = 0; j < n; ++j) {
        dd mjj = {Mhi[j + j * n], Mlo[j + j * n]};
        d[j] = dd_sqrt(mjj);
        dhi[j] = d[j].hi;
        dlo[j] = d[j].lo;
    }
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < n; ++i) {
            dd mij = {Mhi[i + j * n], Mlo[i + j * n]};
            dd h = dd_div(dd_div(mij, d[i]), d[j]);
            Hhi[i + j * n] = h.hi;
            Hlo[i + j * n] = h.lo;
        }
    }
    free(d);
}

/* ---- diagnostics of Thm. 1 evaluated in dd -------------------------------- */

/*
 * ||U^T U - I||_F for an m x n column-major U (FP64 or FP32), with the Gram of
 * U formed in dd as in oracle_gram_dd.  Returned as a double.
 */
double oracle_orth_dd(int64_t m, int64_t n, const void *U, int64_t ldu, int is_f32) {
    double *Gh = (double *)malloc(sizeof(double) * (size_t)(n * n));
    double *Gl = (double *)malloc(sizeof(double) * (size_t)(n * n));
    oracle_gram_dd(m, n, U, ldu, is_f32, Gh, Gl);
    dd acc = dd_from(0.0);
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < n; ++i) {
            dd g = {Gh[i + j * n], Gl[i + j * n]};
            if (i == j) g = dd_sub(g, dd_from(1.0));
            acc = dd_add(acc, dd_mul(g, g));
        }
    }
    free(Gh); free(Gl);
    return sqrt(acc.hi);
}

/*
 * Backward error of Thm. 1, eq. (backward), over selected rows:
 *   out[0] = sum_rows ||A(k,:) - U(k,:) diag(sigma) V^T||_2^2
 *   out[1] = sum_rows ||A(k,:)||_2^2
 * evaluated in dd from the working-precision outputs U (m x n), sigma (n) and
 * V (n x n), all FP64 or all FP32 (same type as A).
 */
void oracle_resid_rows(int64_t n, const void *A, int64_t lda, const void *U, int64_t ldu,
                       const void *S, const void *V, int64_t ldv, int is_f32,
                       int64_t nrows, const int64_t *rows, double *out) {
    dd num = dd_from(0.0), den = dd_from(0.0);
#pragma omp parallel
    {
        dd lnum = dd_from(0.0), lden = dd_from(0.0);
#pragma omp for schedule(static) nowait
        for (int64_t r = 0; r < nrows; ++r) {
            int64_t k = rows[r];
            for (int64_t j = 0; j < n; ++j) {
                double a = is_f32 ? (double)((const float *)A)[k + j * lda]
                                  : ((const double *)A)[k + j * lda];
                dd acc = dd_from(a);
                for (int64_t i = 0; i < n; ++i) {
                    double u = is_f32 ? (double)((const float *)U)[k + i * ldu]
                                      : ((const double *)U)[k + i * ldu];
                    double s = is_f32 ? (double)((const float *)S)[i] : ((const double *)S)[i];
                    double v = is_f32 ? (double)((const float *)V)[j + i * ldv]
                                      : ((const double *)V)[j + i * ldv];
                    acc = dd_sub(acc, dd_mul_d(two_prod(u, s), v));
                }
                lnum = dd_add(lnum, dd_mul(acc, acc));
                lden = dd_add(lden, dd_mul(dd_from(a), dd_from(a)));
            }
        }
#pragma omp critical
        {
            num = dd_add(num, lnum);
            den = dd_add(den, lden);
        }
    }
    out[0] = num.hi;
    out[1] = den.hi;
}

/* ---- exported error-free transformations (for the tests that pin them) ---- */

void oracle_eft(double a, double b, double *out) {
    dd s = two_sum(a, b);
    dd p = two_prod(a, b);
    out[0] = s.hi; out[1] = s.lo; out[2] = p.hi; out[3] = p.lo;
}

void oracle_dd_ops(const double *x, const double *y, double *out) {
    dd a = {x[0], x[1]}, b = {y[0], y[1]};
    dd r;
    r = dd_add(a, b); out[0] = r.hi; out[1] = r.lo;
    r = dd_mul(a, b); out[2] = r.hi; out[3] = r.lo;
    r = dd_div(a, b); out[4] = r.hi; out[5] = r.lo;
    r = dd_sqrt(a);   out[6] = r.hi; out[7] = r.lo;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * gsvd.h -- C-ABI of the MI355X (gfx950) mixed precision Gram-based thin SVD.
 *
 * Method: Carson, Ma, Shao, "Mixed precision thin SVD algorithms based on the
 * Gram matrix" (arXiv 2603.11953).  For a full-column-rank tall-and-skinny A
 * (m >= n) stored in a working precision u (FP32 or FP64), Algorithm 1 computes
 *   M_h = A^T A in a higher precision u_h            (Alg. 1 steps 1-2, eq. (ATA))
 *   M_h = V Sigma^2 V^T with a Jacobi method        (Alg. 1 step 3 / Alg. 2)
 *   Sigma, V rounded to the working precision       (Alg. 1 steps 4-5)
 *   U = A (V Sigma^{-1}) in the working precision    (Alg. 1 step 6, eq. (AV-0))
 * Higher precision: FP64 for FP32 A; double-double (an unevaluated sum hi + lo
 * of two FP64 numbers, unit roundoff ~2^-104) for FP64 A.
 *
 * Conventions for every entry point
 *  - Matrices are column-major (element (i, j) at ptr[i + j * ld]), ld >= rows.
 *  - Every data pointer is a DEVICE pointer owned by the caller; the library
 *    never allocates device memory, never frees caller memory, and never
 *    synchronises the host.  Work is enqueued on `stream` (a hipStream_t passed
 *    as void*; NULL = the default stream) and completes asynchronously.
 *  - Scratch memory is the caller's `work` buffer (device, 256-byte aligned,
 *    at least the size the matching *_workspace_size call returns).
 *  - Return value (synchronous): GSVD_OK (0) when the work was enqueued;
 *    -k when argument k (1-based) is invalid; GSVD_ERR_* below otherwise.
 *    Nothing is enqueued when the return value is not GSVD_OK.
 *  - Numerical outcome (asynchronous): an int written to device memory `info`
 *    per matrix: GSVD_INFO_* below.  On info != 0 the numeric outputs are
 *    unspecified (but finite writes stay inside the caller's buffers).
 */
#ifndef GSVD_H
#define GSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* working precision u of A, Sigma, V, U */
enum { GSVD_F32 = 0, GSVD_F64 = 1 };

/* how the Gram M_h = A^T A is formed */
enum {
    GSVD_GRAM_AUTO = 0,   /* SPLIT when a slice count meets the accuracy target (see
                             target_rel_err) and the tuning table's times put it ahead
                             of PLAIN; otherwise PLAIN.  Without table rows: SPLIT for
                             FP64 A, PLAIN for FP32 A; the batched call: SPLIT for FP64,
                             PLAIN for FP32 */
    GSVD_GRAM_PLAIN = 1,  /* FP32 A: exact FP64 products, FP64 sums; FP64 A: double-double */
    GSVD_GRAM_SPLIT = 2   /* operand splitting: per slab of rows and column, a power-of-two
                             exponent E above the column's largest entry (raised, with two
                             bits of headroom, when a larger entry arrives); each entry cut
                             into n_slices balanced base-256 digits (signed bytes) of its
                             96-bit fixed-point form; digit pairs r + t <= n_slices + 1
                             multiplied exactly on the int8 matrix cores, sums in
                             double-double (FP64 A) or FP64 (FP32 A).  Each entry is
                             represented to within about 2^(-8 n_slices) of 2^E, i.e. at most
                             2^(6 - 8 n_slices) of the slab's column maximum */
};

/* eigensolver of Alg. 1 step 3 */
enum {
    GSVD_EIG_AUTO = 0,       /* JACOBI2 */
    GSVD_EIG_JACOBI2 = 1,    /* two-sided Jacobi on M_h at u_h (Sec. 2.1, Remark 1).
                                FP32 working, n <= 96: M_h and the rotations in FP64,
                                round-robin sweeps in one workgroup; default threshold
                                n * 2^-53.
                                FP64 working (any n), and FP32 working with n > 96: the
                                Jacobi sweeps run in double-double on the Gram matrix
                                expressed in a preconditioning eigenvector basis X, i.e.
                                on X^T M_h X, whose rotations are all small; a sweep
                                applies its rotations together to first order in the
                                angles (X <- X (I + F), Ogita-Aishima form, which also
                                restores X^T X = I), until the largest angle is <= 2^-30.
                                X comes from Algorithm 2's steps in FP64 with the columns
                                ordered by decreasing m_jj and the one-sided Jacobi run on
                                the transposed Cholesky factor (for n > 96 each block step
                                takes the same rotations on its block pair's Gram matrix;
                                X by back substitution); its threshold is jacobi_tol
                                (default 2^-24) and its sweep limit max_sweeps (default 12). */
    GSVD_EIG_CHOL_JACOBI1 = 2 /* Algorithm 2: Cholesky of M_h at u_h, R cast to u,
                                 one-sided Jacobi SVD of R (Thm. 2, Lemma 1); default
                                 threshold sqrt(n) * u.  FP32 working with n > 128: the
                                 SVD of R runs in FP64 and its results are rounded */
};

/* flags */
#define GSVD_WANT_U 1u /* form U (otherwise only Sigma and V; dU may be NULL) */
#define GSVD_U_FP32_MFMA 2u /* FP32 working, n <= 128: U on the FP32 matrix cores instead of
                               the default BF16 form, which cuts every entry of A and W
                               exactly into three BF16 pieces and keeps the six piece
                               products of order up to 2^-16 (FP32 accumulation; the
                               dropped terms are below 2^-24 |a||w| each).  The batched call
                               always forms U on the FP32 matrix cores */

/* synchronous status codes (besides 0 and -k) */
#define GSVD_OK 0
#define GSVD_ERR_HIP (-100)         /* a HIP launch or runtime call failed */
#define GSVD_ERR_UNSUPPORTED (-101) /* valid but not implemented combination */
#define GSVD_ERR_SCRATCH (-102)     /* gsvd_thin_noalloc: the problem's workspace exceeds
                                       GSVD_NOALLOC_MAX_BYTES */

/* asynchronous per-matrix info codes */
#define GSVD_INFO_OK 0
#define GSVD_INFO_NOT_SPD 1       /* M_h not positive definite at u_h: A not of full rank */
#define GSVD_INFO_NO_CONVERGE 2   /* Jacobi did not converge within max_sweeps */
#define GSVD_INFO_NONFINITE 3     /* A (hence M_h) holds a NaN or Inf */
/* Warning bits, or-ed into an info that is otherwise 0; the outputs are
   complete.  (info & 0xff) != 0 means failure. */
#define GSVD_INFO_WARN_ASSUMPTION 256 /* the accuracy assumptions of Theorem 1 cannot be
                                     verified.  kappa(B)^2 is bounded by g ||D W||_F^2 (g the
                                     Gershgorin bound of D^-1 M_h D^-1, D = diag(sqrt(m_jj)),
                                     W = V Sigma^-1); the bit is set when
                                     2 (e + n u_h) kappa^2 > 1/2 (the u_h terms of
                                     eq. (thm:assump); e = n^2 u_h for the plain Gram,
                                     n eps_S for the split Gram with eps_S the tuning
                                     table's measured error) or, with Algorithm 2, when
                                     n u kappa > 1/2 (its O(u) kappa(B) condition) */
#define GSVD_INFO_WARN_REFINE 512 /* the double-double Jacobi stage of JACOBI2 (FP64
                                     working, or FP32 with n > 96) left pairs of eigenvalues that
                                     agree to within their coupling unrotated, or its
                                     last sweep had an angle above 2^-30 */

#define GSVD_MAX_N 512            /* largest n of the single-problem calls; n > 128 runs
                                     the wide kernels (64-column panel pairs, blocked
                                     Cholesky, block Jacobi) */
#define GSVD_MAX_N_EIG_F32 512    /* FP32 working: largest n of the eigensolver stage
                                     (n > 128, or n > 96 for JACOBI2: Algorithm 2's steps
                                     over many workgroups in FP64, plus the double-double
                                     Jacobi stage for JACOBI2) */
#define GSVD_MAX_N_BATCHED_F64 96 /* largest n of a batched problem, FP64 working */
#define GSVD_MAX_N_BATCHED_F32 128 /* largest n of a batched problem, FP32 working */
#define GSVD_MAX_SLICES 12        /* largest n_slices of the split Gram, FP64 A */
#define GSVD_MAX_SLICES_F32 8     /* largest n_slices of the split Gram, FP32 A */

typedef struct {
    int working;        /* GSVD_F32 or GSVD_F64 */
    int gram;           /* GSVD_GRAM_* */
    int eig;            /* GSVD_EIG_* */
    int n_slices;       /* split Gram only: 1..GSVD_MAX_SLICES (FP64 A) or
                           1..GSVD_MAX_SLICES_F32 (FP32 A); 0 = the smallest count whose
                           measured Gram error eps(S) (tuning table) meets the target:
                           n eps kappa_b^2 / 2 <= target_rel_err / 16, since a Gram error
                           |dM_ij| <= eps sqrt(m_ii m_jj) moves each sigma by a relative
                           n eps kappa(B)^2 / 2 at most; the largest count if none does */
    double jacobi_tol;  /* rotation threshold: a pair p, q is rotated when
                           |g_pq| > tol * sqrt(g_pp g_qq); 0 = the eigensolver's default */
    int max_sweeps;     /* 0 = 30 */
    unsigned flags;     /* GSVD_WANT_U ... */
    int64_t slab_rows;  /* rows of A per Gram workgroup ("slab"); 0 = the library's tuning
                           table (written by paper_2603_11953_amd/autotune.py), falling
                           back to about 512 (plain) / 1024 (split) slabs per matrix.
                           n > 128, split form: a cap on the rows per pass of the int8
                           digit planes (multiples of 8192; 0 = about 1 GiB of planes) */
    double target_rel_err; /* requested bound on max_i |s_i - sigma_i| / sigma_i that the
                           slice count and the AUTO Gram form are planned for; 0 = the
                           tolerance 50 n u kappa_b.  Must be >= 0 */
    double kappa_b;     /* the kappa(B) of A = B D (B with unit columns) the plan assumes;
                           0 = 1e3 (FP64 working) or 1e2 (FP32 working).  Must be >= 0 */
} gsvd_opts;

/* Fill *o with the defaults for the given working precision (WANT_U set). */
void gsvd_opts_default(gsvd_opts *o, int working);

/* Human-readable text for a return value or an info code (static storage). */
const char *gsvd_status_string(int code);

/* ---------------------------------------------------------------------------
 * Whole method (Alg. 1 steps 1-6).
 *
 * gsvd_thin: thin SVD A = U diag(S) V^T of the m x n matrix dA (lda >= m,
 * m >= n >= 1, n <= GSVD_MAX_N), all in the working precision o->working.
 * Outputs: dS (n, descending), dV (n x n, ldv >= n), dU (m x n, ldu >= m, only
 * with GSVD_WANT_U), *dInfo (one int).  Column j of V has its entry of largest
 * magnitude positive; U = A (V diag(S)^{-1}) inherits that sign.
 * Arguments: 1 m, 2 n, 3 dA, 4 lda, 5 dS, 6 dV, 7 ldv, 8 dU, 9 ldu, 10 work,
 * 11 work_bytes, 12 dInfo, 13 o, 14 stream.
 * ------------------------------------------------------------------------- */
size_t gsvd_thin_workspace_size(int64_t m, int64_t n, const gsvd_opts *o);
int gsvd_thin(int64_t m, int64_t n, const void *dA, int64_t lda,
              void *dS, void *dV, int64_t ldv, void *dU, int64_t ldu,
              void *work, size_t work_bytes, int *dInfo,
              const gsvd_opts *o, void *stream);

/* ---------------------------------------------------------------------------
 * The steps one at a time (same conventions).
 *
 * gsvd_gram (Alg. 1 steps 1-2, eq. (ATA)): M_h = A^T A in the higher precision,
 * written full and symmetric to dMhi (n x n, ldm >= n) and, for FP64 A, the
 * low parts of the double-double entries to dMlo (required for FP64 A; for
 * FP32 A it may be NULL, else it receives the rounding error of each FP64
 * entry as a second plane).  The split-m partial sums are combined by a
 * fixed-shape tree, so the result is bitwise reproducible for given (m, n).
 * Arguments: 1 m, 2 n, 3 dA, 4 lda, 5 dMhi, 6 dMlo, 7 ldm, 8 work, 9 work_bytes,
 * 10 o, 11 stream.
 * ------------------------------------------------------------------------- */
size_t gsvd_gram_workspace_size(int64_t m, int64_t n, const gsvd_opts *o);

/*
 * gsvd_gram_config: the launch shape gsvd_gram (and the Gram stage of
 * gsvd_thin) takes for this (m, n, o), resolved from the options and the
 * tuning table, without running anything.  Writes the slab height (rows of A
 * per partial sum) to *slab_rows, the number of slabs to *n_slabs and, for
 * GSVD_GRAM_SPLIT, the int8 slice count to *n_slices (0 for the plain form).
 * Any output pointer may be NULL.  Returns 0, or -(position) of a bad argument
 * (1 m, 2 n, 3 o), or GSVD_ERR_UNSUPPORTED as gsvd_gram would.
 */
int gsvd_gram_config(int64_t m, int64_t n, const gsvd_opts *o, int64_t *slab_rows,
                     int64_t *n_slabs, int *n_slices);
int gsvd_gram(int64_t m, int64_t n, const void *dA, int64_t lda,
              double *dMhi, double *dMlo, int64_t ldm,
              void *work, size_t work_bytes, const gsvd_opts *o, void *stream);

/*
 * gsvd_eig (Alg. 1 steps 3-5; Algorithm 2 for GSVD_EIG_CHOL_JACOBI1): from the
 * higher precision Gram (dMhi, dMlo as written by gsvd_gram; dMlo may be NULL
 * for FP32 working) compute S (n, descending, working precision), V (n x n,
 * ldv >= n, working precision) and W = fl(V diag(S)^{-1}) (n x n, ldw >= n,
 * working precision, the matrix that Alg. 1 step 6 multiplies A by), and *dInfo.
 * work: gsvd_eig_workspace_size(n, o) bytes (0 only for CHOL_JACOBI1 with n <= 96
 * (FP64 working) or n <= 128 (FP32), and for JACOBI2 with FP32 working and n <= 96;
 * work may then be NULL).
 * Arguments: 1 n, 2 dMhi, 3 dMlo, 4 ldm, 5 dS, 6 dV, 7 ldv, 8 dW, 9 ldw,
 * 10 dInfo, 11 work, 12 work_bytes, 13 o, 14 stream.
 */
size_t gsvd_eig_workspace_size(int64_t n, const gsvd_opts *o);
int gsvd_eig(int64_t n, const double *dMhi, const double *dMlo, int64_t ldm,
             void *dS, void *dV, int64_t ldv, void *dW, int64_t ldw, int *dInfo,
             void *work, size_t work_bytes, const gsvd_opts *o, void *stream);

/*
 * gsvd_u_recover (Alg. 1 step 6, eq. (AV-0)): dU = dA * dW in the working
 * precision (m x n times n x n; ldu >= m, ldw >= n).  No workspace.
 * Arguments: 1 m, 2 n, 3 dA, 4 lda, 5 dW, 6 ldw, 7 dU, 8 ldu, 9 o, 10 stream.
 */
int gsvd_u_recover(int64_t m, int64_t n, const void *dA, int64_t lda,
                   const void *dW, int64_t ldw, void *dU, int64_t ldu,
                   const gsvd_opts *o, void *stream);

/* ---------------------------------------------------------------------------
 * Batched form: many independent problems of uneven shape in one call
 * (the method of Alg. 1 applied to each; nothing couples the problems).
 *
 * gsvd_thin_batched: for b = 0 .. batch-1, the thin SVD of the hM[b] x hN[b]
 * matrix at dA[b] (leading dimension hLda[b]), written to dS[b] (hN[b]),
 * dV[b] (ldv hLdv[b]), dU[b] (ldu hLdu[b], only with GSVD_WANT_U) and
 * dInfo[b], exactly as gsvd_thin would with the same options (the tuning table
 * may pick a different slab height, so the Gram's rounding may differ).
 *  - dA, dS, dV, dU: DEVICE arrays of `batch` device pointers (dU may be NULL
 *    without GSVD_WANT_U).  hM, hN, hLda, hLdv, hLdu: HOST arrays of `batch`
 *    entries (hLdu may be NULL without GSVD_WANT_U).  dInfo: device int[batch].
 *  - Every problem: m >= n >= 1, n <= GSVD_MAX_N_BATCHED_F64 (FP64 working) or
 *    GSVD_MAX_N_BATCHED_F32 (FP32 working); 1 <= batch <= 65535.  One set of options for
 *    all; the per-problem default Jacobi threshold is sqrt(n) u.
 *  - The whole plan travels in kernel arguments: the call performs no
 *    host-to-device copy, allocation or synchronisation, so it can be
 *    captured in a HIP graph; a replay is valid while the shapes, the pointer
 *    arrays' contents and the workspace stay as they were at capture.
 * Workspace: gsvd_thin_batched_workspace_size(batch, hM, hN, o) bytes (0 when
 * a shape is invalid).
 * Arguments: 1 batch, 2 hM, 3 hN, 4 dA, 5 hLda, 6 dS, 7 dV, 8 hLdv, 9 dU,
 * 10 hLdu, 11 work, 12 work_bytes, 13 dInfo, 14 o, 15 stream.
 * ------------------------------------------------------------------------- */
size_t gsvd_thin_batched_workspace_size(int batch, const int64_t *hM, const int64_t *hN,
                                        const gsvd_opts *o);
int gsvd_thin_batched(int batch, const int64_t *hM, const int64_t *hN,
                      const void *const *dA, const int64_t *hLda,
                      void *const *dS, void *const *dV, const int64_t *hLdv,
                      void *const *dU, const int64_t *hLdu,
                      void *work, size_t work_bytes, int *dInfo,
                      const gsvd_opts *o, void *stream);

/* ---------------------------------------------------------------------------
 * Mixed precision Cholesky QR (Sec. 3.3, Theorem 3): the method's Gram stage
 * reused for a thin QR factorization A = Q R.
 *   M_h = A^T A at u_h                (as gsvd_gram, in the form o->gram selects)
 *   M_h = R_h^T R_h at u_h            (Cholesky: double-double for FP64 A, of the
 *                                      power-of-two column-scaled Gram, scaled back)
 *   R = fl(R_h), Q from Q R = A at u  (row-wise forward substitution)
 * Theorem 3: with u_h = O(u^2) (both working precisions here) the loss of
 * orthogonality ||Q^T Q - I|| is O(u) kappa(B), A = B D with B of unit columns.
 * Outputs: dQ (m x n, ldq >= m) and dR (n x n upper triangular with zeros below,
 * ldr >= n) in the working precision; *dInfo = 0, 1 (M_h not positive definite
 * at u_h: A not of full column rank) or 3 (non-finite input); Q is not written
 * when info != 0.  Conventions as gsvd_thin (device pointers, caller's
 * workspace of gsvd_cholqr_workspace_size bytes, no allocation or host sync).
 * Arguments: 1 m, 2 n, 3 dA, 4 lda, 5 dQ, 6 ldq, 7 dR, 8 ldr, 9 work,
 * 10 work_bytes, 11 dInfo, 12 o, 13 stream.
 * ------------------------------------------------------------------------- */
size_t gsvd_cholqr_workspace_size(int64_t m, int64_t n, const gsvd_opts *o);
int gsvd_cholqr(int64_t m, int64_t n, const void *dA, int64_t lda, void *dQ, int64_t ldq,
                void *dR, int64_t ldr, void *work, size_t work_bytes, int *dInfo,
                const gsvd_opts *o, void *stream);

/* ---------------------------------------------------------------------------
 * gsvd_thin_noalloc: gsvd_thin for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same computation, kernels and results as gsvd_thin with the
 * same options, but the workspace is a fixed array inside the library, one per
 * GPU, of GSVD_NOALLOC_MAX_BYTES bytes, held from library load until the process
 * ends.  The caller passes inputs and outputs only.
 *  - Allocates nothing and calls no allocating routine.  The first call on a
 *    device looks up that device's copy of the array (hipGetSymbolAddress); the
 *    call runs on the device current in the calling thread.
 *  - Returns GSVD_ERR_SCRATCH, enqueueing nothing, when
 *    gsvd_thin_workspace_size(m, n, o) exceeds GSVD_NOALLOC_MAX_BYTES (for the
 *    wide split Gram, o->slab_rows caps its per-pass planes).
 *  - Calls that overlap on one GPU (other streams, other host threads) share the
 *    array and race: order them, e.g. on one stream.
 * Arguments: 1 m, 2 n, 3 dA, 4 lda, 5 dS, 6 dV, 7 ldv, 8 dU, 9 ldu, 10 dInfo,
 * 11 o, 12 stream; their meaning as in gsvd_thin.
 * ------------------------------------------------------------------------- */
#define GSVD_NOALLOC_MAX_BYTES (64u << 20)
size_t gsvd_noalloc_max_bytes(void);
int gsvd_thin_noalloc(int64_t m, int64_t n, const void *dA, int64_t lda,
                      void *dS, void *dV, int64_t ldv, void *dU, int64_t ldu, int *dInfo,
                      const gsvd_opts *o, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GSVD_H */

// Internal launch interfaces shared by the host entry points (gsvd_api.hip)
// and the kernel files.  Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gsvd {

constexpr int GSVD_KMAX_N = 128;      // largest n the kernels are sized for
constexpr int GSVD_KMAX_N_F64 = 96;   // FP64 working: R and V (FP64) must share LDS
constexpr int GSVD_WIDE_MAX_N = 512;  // largest n of the wide (panel-pair) path

// One problem of a batch as the batched kernels see it (device memory, written
// by the batch set-up kernel).  Every pointer is a device address.
struct BatchMat {
    const void *A;
    void *S, *V, *U;
    void *W;                 // fl(V Sigma^-1), n x n, ld = n, working precision
    double *Mhi, *Mlo;       // Gram planes, n x n, ld = n
    double *part;            // Gram partial sums of the slabs
    double *rw;              // scratch of the double-double Jacobi stage (FP64 working)
    int *info;
    int64_t m, lda, ldu, rows_per_split;
    int n, ldv, nsplit, pad;
};

// Launch geometry of the split-m Gram (gram.hip).
struct GramPlan {
    int nb;                  // ceil(n / 4): 4x4 blocks per side
    int nblk;                // blocks in the upper triangle
    int ng;                  // block groups (workgroups per slab)
    int nblkg;               // blocks per group (the last may have fewer)
    int ks;                  // k-groups per workgroup
    int kc;                  // rows per LDS chunk (a multiple of ks)
    int threads;             // lanes per workgroup
    int64_t rows_per_split;  // rows of A per slab
    int64_t nsplit;          // slabs
    size_t lds_bytes;        // dynamic LDS per workgroup
    size_t part_bytes;       // workspace for the per-slab partial sums
};

// slab_rows > 0 fixes the slab height (rounded up to a whole number of chunks);
// 0 picks about 512 slabs.  groups: the blocks may be split over several
// workgroups per slab (single problems; the batched kernel takes ng = 1).
GramPlan gram_plan(int64_t m, int64_t n, int64_t slab_rows = 0, bool groups = false);
hipError_t gram_launch(int working, int64_t m, int64_t n, const void *A, int64_t lda,
                       double *Mhi, double *Mlo, int64_t ldm, void *part, const GramPlan &p,
                       hipStream_t st);
// Batched: the problems order[first .. first + count) share n (hence the plan's
// nb, nblk, ks, kc, threads); grid.y covers max_nsplit slabs.  The reduction
// launch covers every problem of the batch (up to max_n).
hipError_t gram_batched_launch(int working, const BatchMat *tab, const int *order, int first,
                               int count, int max_nsplit, const GramPlan &p, hipStream_t st);
hipError_t gram_reduce_batched_launch(const BatchMat *tab, int batch, int max_n, hipStream_t st);

// Plain Gram of FP32 A on the FP64 matrix cores (gram_f32mfma.hip, n <= 128).
struct F32MfmaPlan {
    int nb;                  // ceil(n / 16)
    int64_t rows_per_split;  // rows of A per slab (a multiple of 32)
    int64_t nsplit;
    size_t part_bytes;
};
// slab_rows > 0 fixes the slab height (rounded up to 32); 0 picks about 1024 slabs.
F32MfmaPlan gram_f32mfma_plan(int64_t m, int64_t n, int64_t slab_rows = 0);
hipError_t gram_f32mfma_launch(int64_t m, int64_t n, const float *A, int64_t lda, double *Mhi,
                               double *Mlo, int64_t ldm, void *part, const F32MfmaPlan &p,
                               hipStream_t st);

// Launch geometry of the wide plain Gram (gram_wide.hip, n > 128): 64-column
// panels, one workgroup per (panel pair, slab).
struct WidePlan {
    int np;                  // panels
    int npair;               // panel pairs I <= J
    int64_t rows_per_split;  // rows of A per slab
    int64_t nsplit;          // slabs
    size_t part_bytes;       // workspace for the per-slab partial sums
};

// slab_rows > 0 fixes the slab height (rounded up to a multiple of 16); 0 picks
// about 2048 workgroups in all.
WidePlan gram_wide_plan(int64_t m, int64_t n, int64_t slab_rows = 0);
hipError_t gram_wide_launch(int working, int64_t m, int64_t n, const void *A, int64_t lda,
                            double *Mhi, double *Mlo, int64_t ldm, void *part, const WidePlan &p,
                            hipStream_t st);

// Operand-split Gram for n > 128 (gram_split_wide.hip): slicing into int8 digit
// planes in the workspace, then int8 SYRK per 64-column panel pair, in passes
// of rows_per_pass rows.  The workspace holds the planes and exponents of one
// pass and the per-group double-double slots.
struct SplitWidePlan {
    int S;                   // slices per entry
    int np, npair, npad;     // panels, panel pairs, n rounded up to 64
    int64_t groups_per_pass; // 8192-row groups (one syrk workgroup row) per pass
    int64_t rows_per_pass;
    int64_t npass;
    size_t plane_off, expo_off, slot_off, flag_off, part_bytes;
};
// rows_cap > 0 caps the rows per pass (rounded down to a multiple of 8192, at least 8192)
SplitWidePlan split_wide_plan(int64_t m, int64_t n, int S, int64_t rows_cap = 0);
hipError_t split_wide_launch(int working, int64_t m, int64_t n, const void *A, int64_t lda,
                             double *Mhi, double *Mlo, int64_t ldm, void *work,
                             const SplitWidePlan &p, hipStream_t st);

// Launch geometry of the operand-split Gram (gram_split.hip).
struct SplitPlan {
    int S;                   // slices per entry
    int nb;                  // ceil(n / 16): 16-column blocks
    int npair;               // tiles in the upper triangle
    int64_t rows_per_split;  // rows of A per slab
    int64_t nsplit;          // slabs
    size_t lds_bytes;
    size_t part_bytes;
};

// slab_rows > 0 fixes the slab height (rounded up to a multiple of 64); 0 picks
// about 1024 slabs.
SplitPlan split_plan(int64_t m, int64_t n, int S, int64_t slab_rows = 0);
int split_max_slices(int working);
hipError_t split_launch(int working, int64_t m, int64_t n, const void *A, int64_t lda,
                        double *Mhi, double *Mlo, int64_t ldm, void *part, const SplitPlan &p,
                        hipStream_t st);
// Batched: the problems order[first .. first + count) share ceil(n / 16) = p.nb
// and the slice count p.S.
hipError_t split_batched_launch(int working, const BatchMat *tab, const int *order, int first,
                                int count, int max_nsplit, const SplitPlan &p, hipStream_t st);
hipError_t split_reduce_batched_launch(const BatchMat *tab, int batch, int max_n, hipStream_t st);
// the per-type partial-sum launchers behind split_launch / split_batched_launch
hipError_t split_partial_f64(int64_t m, int64_t n, const double *A, int64_t lda, void *part,
                             const SplitPlan &p, hipStream_t st);
hipError_t split_partial_f32(int64_t m, int64_t n, const float *A, int64_t lda, void *part,
                             const SplitPlan &p, hipStream_t st);
hipError_t split_batched_f64(const BatchMat *tab, const int *order, int first, int count,
                             int max_nsplit, const SplitPlan &p, hipStream_t st);
hipError_t split_batched_f32(const BatchMat *tab, const int *order, int first, int count,
                             int max_nsplit, const SplitPlan &p, hipStream_t st);

// Eigensolver stage (eig.hip).
size_t eig_lds_bytes(int working, int64_t n);
int eig_max_n(int working);
int eig_threads(int64_t n);
// pre (FP64 working): the preconditioner form for the double-double stage (columns
// ordered by norm, Jacobi on the transposed factor, V by back substitution); it
// writes V (unit columns, unordered, unsigned), uses W as scratch, and sets info.
hipError_t eig_launch(int working, int64_t n, const double *Mhi, const double *Mlo, int64_t ldm,
                      void *S, void *V, int64_t ldv, void *W, int64_t ldw, int *info, double tol,
                      int max_sweeps, bool pre, hipStream_t st);
// Batched: one workgroup per problem, problems taken in the order given
// (order[batch - 1 - block]); tol = 0 means sqrt(n) u per problem.
hipError_t eig_batched_launch(int working, const BatchMat *tab, const int *order, int batch,
                              int max_n, double tol, int max_sweeps, bool pre, hipStream_t st);

// Algorithm 2 for FP64 working and n > 96 (eig_wide.hip): a sequence of
// launches (blocked dd Cholesky, block one-sided Jacobi) over device scratch.
// pre: the preconditioner form for the double-double stage (columns ordered by
// norm, Jacobi on the transposed factor, V by back substitution); it writes only
// V (FP64, unordered, unsigned) and info.
size_t eig_wide_work_bytes(int64_t n);
hipError_t eig_wide_launch(int64_t n, const double *Mhi, const double *Mlo, int64_t ldm, void *S,
                           void *V, int64_t ldv, void *W, int64_t ldw, int *info, double tol,
                           int max_sweeps, bool pre, void *work, hipStream_t st);

// Cholesky factor of M_h alone (eig_wide.hip; any n <= 512): the scaled blocked dd
// Cholesky of Algorithm 2's first step, R = fl_w(R_H) D~ written upper triangular
// (zeros below) in the working precision; *info = 0, 1 (not positive definite) or
// 3 (non-finite).  Mlo must be non-null.
size_t chol_work_bytes(int64_t n);
hipError_t chol_launch(int working, int64_t n, const double *Mhi, const double *Mlo, int64_t ldm,
                       void *R, int64_t ldr, int *info, void *work, hipStream_t st);

// Two-sided Jacobi eigensolver for FP32 working (eig_jacobi2.hip).  V needs
// j2_work_bytes(n, max_sweeps) of device scratch (0 while it fits LDS, n <= 96; beyond,
// the rotations are logged and V is formed from the log afterwards).
size_t j2_work_bytes(int64_t n, int max_sweeps);
hipError_t eig_jacobi2_launch(int working, int64_t n, const double *Mhi, int64_t ldm, void *S,
                              void *V, int64_t ldv, void *W, int64_t ldw, int *info, double tol,
                              int max_sweeps, void *work, hipStream_t st);
// Batched: for max_n > 96 each problem's V scratch is its (then unused) Gram
// partial-sum area, which always holds at least n^2 doubles.
hipError_t eig_jacobi2_batched_launch(int working, const BatchMat *tab, const int *order, int batch,
                                      int max_n, double tol, int max_sweeps, hipStream_t st);

// Double-double two-sided Jacobi stage on the Gram matrix preconditioned by
// Algorithm 2's eigenvectors (eig_refine.hip).  X0 (FP64, ld ldx0) is
// Algorithm 2's V; the outputs S, V, W (working precision) may be the buffers X0
// was read from.  Skipped when *info is non-zero on entry.
size_t refine_work_bytes(int64_t n);
hipError_t refine_launch(int working, int64_t n, const double *Mhi, const double *Mlo,
                         int64_t ldm, const double *X0, int64_t ldx0, void *S, void *V,
                         int64_t ldv, void *W, int64_t ldw, int *info, void *work,
                         hipStream_t st);
// Batched, FP64 working: each problem's X0 is its V, its scratch BatchMat::rw.
hipError_t refine_batched_launch(const BatchMat *tab, int batch, int max_n, hipStream_t st);
// The assumption check of Theorem 1 (GSVD_INFO_WARN_ASSUMPTION) after any
// eigensolver: reads diag(M_h), W and info.
// alg2: Algorithm 2 was the last eigensolver (its O(u) kappa(B) condition applies).
// e_gram bounds ||D^-1 dM D^-1|| for the Gram's error dM.
hipError_t assump_launch(int working, int64_t n, const double *Mhi, int64_t ldm, const void *W,
                         int64_t ldw, int *info, double e_gram, bool alg2, hipStream_t st);
hipError_t assump_batched_launch(int working, const BatchMat *tab, int batch, double e_gram,
                                 bool alg2, int max_n, hipStream_t st);
// zeros into n doubles (a kernel, so a captured graph holds no memset node)
hipError_t fill_zero_launch(double *p, size_t n, hipStream_t st);
// FP32 working with an FP64 eigensolver: S, V rounded, W = fl(V Sigma^-1)
// (V64 has leading dimension n).
hipError_t cast_eig_f32_launch(int64_t n, const double *S64, const double *V64, void *S, void *V,
                               int64_t ldv, void *W, int64_t ldw, const int *info,
                               hipStream_t st);

// Q from Q R = A, R upper triangular (cholqr.hip): row-wise forward substitution in
// the working precision; nothing runs when *info != 0.
hipError_t trsm_rows_launch(int working, int64_t m, int64_t n, const void *A, int64_t lda,
                            const void *R, int64_t ldr, void *Q, int64_t ldq, const int *info,
                            hipStream_t st);

// U = A W (urecover.hip).
hipError_t urecover_launch(int working, int64_t m, int64_t n, const void *A, int64_t lda,
                           const void *W, int64_t ldw, void *U, int64_t ldu, hipStream_t st);
// FP32 working, n <= 128: U = A W on the BF16 matrix cores with every entry of A
// and W cut exactly into three BF16 pieces (urecover_bf16.hip)
hipError_t urecover_bf16_launch(int64_t m, int64_t n, const float *A, int64_t lda, const float *W,
                                int64_t ldw, float *U, int64_t ldu, hipStream_t st);
// Batched: the problems order[first .. first + count) share nt = ceil(n / 16).
hipError_t urecover_batched_launch(int working, const BatchMat *tab, const int *order, int first,
                                   int count, int nt, int64_t max_m, hipStream_t st);
int urecover_batched_max_nt(int working);
// n > 128: workgroups of 256 rows x 128 columns, W staged in k-chunks.
hipError_t urecover_wide_launch(int working, int64_t m, int64_t n, const void *A, int64_t lda,
                                const void *W, int64_t ldw, void *U, int64_t ldu, hipStream_t st);

}  // namespace gsvd

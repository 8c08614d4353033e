// Host-side helpers shared by the single-problem and batched entry points:
// option checks, the slice count and slab height in force, workspace alignment.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include "gsvd.h"
#include "gsvd_internal.hpp"
#include "tune.hpp"

namespace gsvd {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

inline bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

inline double unit_roundoff(int working) { return working == GSVD_F64 ? 0x1p-53 : 0x1p-24; }

inline size_t wsize(int working) { return working == GSVD_F64 ? 8 : 4; }

// Checks shared by every entry point that takes options.
inline int check_opts(const gsvd_opts *o, int argpos) {
    if (o == nullptr) return -argpos;
    if (o->working != GSVD_F32 && o->working != GSVD_F64) return -argpos;
    if (o->gram != GSVD_GRAM_AUTO && o->gram != GSVD_GRAM_PLAIN && o->gram != GSVD_GRAM_SPLIT)
        return -argpos;
    if (o->eig != GSVD_EIG_AUTO && o->eig != GSVD_EIG_JACOBI2 && o->eig != GSVD_EIG_CHOL_JACOBI1)
        return -argpos;
    if (o->max_sweeps < 0 || o->jacobi_tol < 0.0 || o->n_slices < 0 || o->slab_rows < 0)
        return -argpos;
    if (!(o->target_rel_err >= 0.0) || !(o->kappa_b >= 0.0)) return -argpos;  // also NaN
    return 0;
}

inline int max_slices(int working) {
    return working == GSVD_F64 ? GSVD_MAX_SLICES : GSVD_MAX_SLICES_F32;
}

// The eigensolver in force: AUTO is the two-sided Jacobi on M_h at u_h.
inline int eig_mode_of(const gsvd_opts *o) {
    return o->eig == GSVD_EIG_AUTO ? GSVD_EIG_JACOBI2 : o->eig;
}

inline bool use_split(const gsvd_opts *o) { return o->gram == GSVD_GRAM_SPLIT; }

inline int check_supported(const gsvd_opts *o) {
    if (o->gram == GSVD_GRAM_SPLIT && o->n_slices > max_slices(o->working))
        return GSVD_ERR_UNSUPPORTED;
    return 0;
}

// n > 128: the wide Gram and U kernels (64-column panels)
inline bool wide_n(int64_t n) { return n > GSVD_KMAX_N; }
// FP32 working on the multi-workgroup eigensolver (Algorithm 2's steps in FP64,
// results rounded to FP32): beyond the one-workgroup kernels (n > 128), and for
// JACOBI2 from n > 96 on, where its preconditioner and the double-double stage
// beat the one-workgroup two-sided Jacobi
inline bool f32_wide_eig(const gsvd_opts *o, int64_t n) {
    return o->working == GSVD_F32 &&
           (n > GSVD_KMAX_N || (eig_mode_of(o) == GSVD_EIG_JACOBI2 && n > GSVD_KMAX_N_F64));
}
// beyond the one-workgroup eigensolver: the multi-launch Algorithm 2
inline bool wide_eig(const gsvd_opts *o, int64_t n) {
    return (o->working == GSVD_F64 && n > GSVD_KMAX_N_F64) || f32_wide_eig(o, n);
}
// the double-double Jacobi stage after the preconditioner (JACOBI2 for FP64
// working, and for FP32 working beyond the one-workgroup two-sided Jacobi)
inline bool eig_refined(const gsvd_opts *o, int64_t n) {
    return eig_mode_of(o) == GSVD_EIG_JACOBI2 && (o->working == GSVD_F64 || f32_wide_eig(o, n));
}

inline int check_eig_supported(const gsvd_opts *o, int64_t n) {
    if (int e = check_supported(o)) return e;
    if (o->working == GSVD_F32 && n > GSVD_MAX_N_EIG_F32) return GSVD_ERR_UNSUPPORTED;
    return 0;
}

// the Gram forms in force for n (every form exists for every n up to GSVD_MAX_N)
inline int check_gram_supported(const gsvd_opts *o, int64_t n) {
    (void)n;
    return check_supported(o);
}

// kappa(B) the accuracy plan assumes: the caller's, else 1e3 (FP64) / 1e2 (FP32)
inline double plan_kappa(const gsvd_opts *o) {
    return o->kappa_b > 0.0 ? o->kappa_b : (o->working == GSVD_F64 ? 1e3 : 1e2);
}

// requested bound on max_i |s_i - sigma_i| / sigma_i: the caller's, else the
// tolerance 50 n u kappa(B) at the planned kappa(B)
inline double plan_target(const gsvd_opts *o, int64_t n) {
    if (o->target_rel_err > 0.0) return o->target_rel_err;
    return 50.0 * (double)n * unit_roundoff(o->working) * plan_kappa(o);
}

// Smallest slice count whose Gram error meets the target.  A perturbation dM with
// |dM_ij| <= eps sqrt(M_ii M_jj) moves the eigenvalues of H = D^-1 M D^-1 by at
// most n eps, hence each sigma_i by a relative n eps kappa(B)^2 / 2 at most
// (eq. (ATA) and the first-order step of Theorem 1's proof); with a factor 16
// of margin the target asks for eps <= target / (8 n kappa^2).  eps(S) is the
// tuning table's measurement.  0: no slice count meets the target.
inline int slices_for_target(const gsvd_opts *o, int64_t n) {
    const double k = plan_kappa(o);
    const double budget = plan_target(o, n) / (8.0 * (double)n * k * k);
    for (int S = 1; S <= max_slices(o->working); ++S)
        if (tune_eps(o->working, n, S) <= budget) return S;
    return 0;
}

// slice count of the split Gram: the caller's, else the one the target asks for
// (the largest when none meets it)
inline int slices_of(const gsvd_opts *o, int64_t n) {
    if (o->n_slices > 0) return o->n_slices;
    const int S = slices_for_target(o, n);
    return S > 0 ? S : max_slices(o->working);
}

// slab height of the Gram: the caller's, else the tuning table's (0 = the
// kernel's own default slab count)
inline int64_t slab_rows_of(const gsvd_opts *o, int64_t m, int64_t n, bool batched) {
    if (o->slab_rows > 0) return o->slab_rows;
    return tune_slab_rows(o->working, use_split(o) ? GSVD_GRAM_SPLIT : GSVD_GRAM_PLAIN, n, m,
                          batched);
}

// compute units of the current device (256 on MI355X; also the fallback)
inline int64_t device_cus() {
    static const int cus = [] {  // initialised once, thread-safe
        int dev = 0, v = 0;
        const bool ok = hipGetDevice(&dev) == hipSuccess &&
                        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) ==
                            hipSuccess &&
                        v > 0;
        return ok ? v : 256;
    }();
    return cus;
}

inline GramPlan gram_plan_of(const gsvd_opts *o, int64_t m, int64_t n, bool batched) {
    GramPlan p = gram_plan(m, n, slab_rows_of(o, m, n, batched), !batched);
    if (!batched && o->slab_rows == 0) {
        // The tuned height was measured at one m of its bucket.  A single problem's
        // workgroups run one per CU at a time, so a slab count that leaves the last
        // round nearly empty costs almost a whole round: for other m the slab count
        // is set so the workgroups fill whole rounds.  A caller's height is kept.
        const int64_t cus = device_cus();
        const int64_t wgs = (int64_t)p.ng * p.nsplit;
        const int64_t rounds = (wgs + cus - 1) / cus;
        const int64_t target = rounds * cus / p.ng;  // slabs
        if (wgs % cus != 0 && target >= 1) {
            const GramPlan q = gram_plan(m, n, (m + target - 1) / target, true);
            if ((int64_t)q.ng * q.nsplit <= rounds * cus) p = q;
        }
    }
    return p;
}

// GSVD_GRAM_AUTO: the split form when a slice count meets the accuracy target and
// the tuning table's times (scaled by the slice count: the split Gram's work grows
// about linearly with S) put it ahead of the plain form.  Without table rows:
// FP64 A split (the dd Gram runs on the vector units, the split form on the int8
// matrix cores), FP32 A plain (one exact FP64 matrix-core pass).  The batched call
// takes one form for all its problems: split for FP64, plain for FP32.
inline bool auto_split(const gsvd_opts *o, int64_t m, int64_t n, bool batched) {
    const int S = slices_for_target(o, n);
    if (S == 0) return false;
    const bool f64 = o->working == GSVD_F64;
    if (batched || wide_n(n)) return f64;
    double tp = 0.0, ts = 0.0;
    int sp = 0, ss = 0;
    if (!tune_gram_ms(o->working, GSVD_GRAM_PLAIN, n, m, false, &tp, &sp) ||
        !tune_gram_ms(o->working, GSVD_GRAM_SPLIT, n, m, false, &ts, &ss) || ss < 1)
        return f64;
    return ts * (double)S / (double)ss < tp;
}

// The options with the Gram form and slice count resolved for this problem shape:
// gram is PLAIN or SPLIT, and a split form carries its slice count.
inline gsvd_opts resolve_opts(const gsvd_opts *o, int64_t m, int64_t n, bool batched) {
    gsvd_opts r = *o;
    if (r.gram == GSVD_GRAM_AUTO)
        r.gram = auto_split(o, m, n, batched) ? GSVD_GRAM_SPLIT : GSVD_GRAM_PLAIN;
    if (r.gram == GSVD_GRAM_SPLIT) r.n_slices = slices_of(o, n);
    return r;
}

// the plain Gram of FP32 A on the matrix cores, at the tuned slab height
inline F32MfmaPlan f32mfma_plan_of(const gsvd_opts *o, int64_t m, int64_t n) {
    return gram_f32mfma_plan(m, n, slab_rows_of(o, m, n, false));
}

inline SplitPlan split_plan_of(const gsvd_opts *o, int64_t m, int64_t n, bool batched) {
    return split_plan(m, n, slices_of(o, n), slab_rows_of(o, m, n, batched));
}

// the plain Gram of FP32 A on the FP64 matrix cores (single problems, n <= 128)
inline bool f32_mfma(const gsvd_opts *o, int64_t n, bool batched) {
    return !batched && o->working == GSVD_F32 && !use_split(o) && n <= GSVD_KMAX_N;
}

// workspace bytes for the partial sums of whichever Gram form o selects
inline size_t gram_part_bytes(int64_t m, int64_t n, const gsvd_opts *o, bool batched) {
    if (wide_n(n))
        return use_split(o) ? split_wide_plan(m, n, slices_of(o, n), o->slab_rows).part_bytes
                            : gram_wide_plan(m, n, o->slab_rows).part_bytes;
    if (use_split(o)) return split_plan_of(o, m, n, batched).part_bytes;
    if (f32_mfma(o, n, batched)) return f32mfma_plan_of(o, m, n).part_bytes;
    return gram_plan_of(o, m, n, batched).part_bytes;
}

// rotation threshold of Algorithm 2's one-sided Jacobi: sqrt(n) u_w unless given
inline double alg2_tol_of(const gsvd_opts *o, int64_t n) {
    if (o->jacobi_tol > 0) return o->jacobi_tol;
    return __builtin_sqrt((double)n) * unit_roundoff(o->working);
}

// rotation threshold of the preconditioner before the double-double stage: its
// basis need only fall inside that stage's quadratic convergence (angles far
// below 2^-15); 2^-24 leaves a wide margin
inline double pre_tol_of(const gsvd_opts *o) {
    return o->jacobi_tol > 0 ? o->jacobi_tol : 0x1p-24;
}

// default rotation threshold: n u_h for the one-workgroup two-sided Jacobi on
// M_h (FP32 working, FP64), else Algorithm 2's
inline double jacobi_tol_of(const gsvd_opts *o, int64_t n) {
    if (o->jacobi_tol > 0) return o->jacobi_tol;
    if (eig_mode_of(o) == GSVD_EIG_JACOBI2 && o->working == GSVD_F32 && !f32_wide_eig(o, n))
        return (double)n * 0x1p-53;
    return alg2_tol_of(o, n);
}

inline int sweeps_of(const gsvd_opts *o) { return o->max_sweeps > 0 ? o->max_sweeps : 30; }
// sweep limit of the preconditioner before the double-double stage (its sweeps
// are queued whether needed or not; it stops after 4 to 6 at the sizes measured)
inline int pre_sweeps_of(const gsvd_opts *o) { return o->max_sweeps > 0 ? o->max_sweeps : 12; }

// Bound on ||D^-1 dM D^-1|| for the Gram's error dM, for the assumption check:
// n^2 u_h for the plain Gram (the n^2 eps_M of eq. (thm:assump)); n eps for the
// split Gram, eps the tuning table's measured error of its slice count in the
// scaled sense |dM_ij| <= eps sqrt(M_ii M_jj)
inline double gram_pert_of(const gsvd_opts *o, int64_t n) {
    const double u_h = o->working == GSVD_F64 ? 0x1p-104 : 0x1p-53;
    const double dn = (double)n;
    if (!use_split(o)) return dn * dn * u_h;
    const double e = tune_eps(o->working, n, slices_of(o, n));
    return dn * (e > u_h ? e : u_h);
}

// Eigensolver scratch.  FP32 working with n > 128: S, V, W of the FP64
// Algorithm 2, a zero low plane (when the caller passes none), then the
// Algorithm 2 / double-double stage scratch (used one after the other).
struct EigLayout {
    size_t s64, v64, w64, zlo, scratch, total;
};

inline EigLayout eig_layout(const gsvd_opts *o, int64_t n) {
    EigLayout L{};
    size_t scratch = 0;
    if (wide_eig(o, n)) scratch = eig_wide_work_bytes(n);
    if (eig_refined(o, n)) scratch = scratch > refine_work_bytes(n) ? scratch : refine_work_bytes(n);
    if (o->working == GSVD_F32 && !f32_wide_eig(o, n) && eig_mode_of(o) == GSVD_EIG_JACOBI2)
        scratch = j2_work_bytes(n, sweeps_of(o));
    size_t off = 0;
    if (f32_wide_eig(o, n)) {
        const size_t nn = (size_t)n * (size_t)n;
        L.s64 = off;
        off = align_up(off + (size_t)n * sizeof(double));
        L.v64 = off;
        off = align_up(off + nn * sizeof(double));
        L.w64 = off;
        off = align_up(off + nn * sizeof(double));
        L.zlo = off;
        off = align_up(off + nn * sizeof(double));
    }
    L.scratch = off;
    L.total = scratch ? align_up(off + scratch) : off;
    return L;
}

inline size_t eig_work_bytes(const gsvd_opts *o, int64_t n) { return eig_layout(o, n).total; }

// The eigensolver stage (Alg. 1 steps 3-5), then the assumption check.
inline hipError_t eig_any(const gsvd_opts *o, int64_t n, const double *Mhi, const double *Mlo,
                          int64_t ldm, void *S, void *V, int64_t ldv, void *W, int64_t ldw,
                          int *info, void *work, double e_gram, hipStream_t st) {
    const int sweeps = sweeps_of(o);
    char *base = (char *)work;
    const EigLayout L = eig_layout(o, n);
    hipError_t err;
    if (f32_wide_eig(o, n)) {
        double *s64 = (double *)(base + L.s64);
        double *v64 = (double *)(base + L.v64);
        double *w64 = (double *)(base + L.w64);
        const double *lo = Mlo;
        if (lo == nullptr) {
            double *z = (double *)(base + L.zlo);
            if ((err = fill_zero_launch(z, (size_t)n * (size_t)n, st)) != hipSuccess) return err;
            lo = z;
        }
        void *scr = base + L.scratch;
        const bool pre = eig_refined(o, n);
        err = eig_wide_launch(n, Mhi, lo, ldm, s64, v64, n, w64, n, info,
                              pre ? pre_tol_of(o) : alg2_tol_of(o, n),
                              pre ? pre_sweeps_of(o) : sweeps, pre, scr, st);
        if (err == hipSuccess)
            err = eig_refined(o, n)
                      ? refine_launch(GSVD_F32, n, Mhi, lo, ldm, v64, n, S, V, ldv, W, ldw, info,
                                      scr, st)
                      : cast_eig_f32_launch(n, s64, v64, S, V, ldv, W, ldw, info, st);
    } else if (o->working == GSVD_F64) {
        const bool pre = eig_refined(o, n);
        const double tol = pre ? pre_tol_of(o) : alg2_tol_of(o, n);
        const int nsw = pre ? pre_sweeps_of(o) : sweeps;
        err = wide_eig(o, n)
                  ? eig_wide_launch(n, Mhi, Mlo, ldm, S, V, ldv, W, ldw, info, tol, nsw, pre, work,
                                    st)
                  : eig_launch(o->working, n, Mhi, Mlo, ldm, S, V, ldv, W, ldw, info, tol, nsw, pre,
                               st);
        if (err == hipSuccess && eig_refined(o, n))
            err = refine_launch(GSVD_F64, n, Mhi, Mlo, ldm, (const double *)V, ldv, S, V, ldv, W,
                                ldw, info, work, st);
    } else if (eig_mode_of(o) == GSVD_EIG_JACOBI2) {
        err = eig_jacobi2_launch(o->working, n, Mhi, ldm, S, V, ldv, W, ldw, info,
                                 jacobi_tol_of(o, n), sweeps, work, st);
    } else {
        err = eig_launch(o->working, n, Mhi, Mlo, ldm, S, V, ldv, W, ldw, info,
                         jacobi_tol_of(o, n), sweeps, false, st);
    }
    if (err != hipSuccess) return err;
    return assump_launch(o->working, n, Mhi, ldm, W, ldw, info, e_gram,
                         eig_mode_of(o) == GSVD_EIG_CHOL_JACOBI1, st);
}

// The Gram stage (Alg. 1 steps 1-2) in the form the options select.
inline hipError_t gram_any(const gsvd_opts *o, int64_t m, int64_t n, const void *A, int64_t lda,
                    double *Mhi, double *Mlo, int64_t ldm, void *part, hipStream_t st) {
    if (wide_n(n) && use_split(o)) {
        SplitWidePlan p = split_wide_plan(m, n, slices_of(o, n), o->slab_rows);
        return split_wide_launch(o->working, m, n, A, lda, Mhi, Mlo, ldm, part, p, st);
    }
    if (wide_n(n)) {
        WidePlan p = gram_wide_plan(m, n, o->slab_rows);
        return gram_wide_launch(o->working, m, n, A, lda, Mhi, Mlo, ldm, part, p, st);
    }
    if (use_split(o)) {
        SplitPlan p = split_plan_of(o, m, n, false);
        return split_launch(o->working, m, n, A, lda, Mhi, Mlo, ldm, part, p, st);
    }
    if (f32_mfma(o, n, false)) {
        F32MfmaPlan p = f32mfma_plan_of(o, m, n);
        return gram_f32mfma_launch(m, n, (const float *)A, lda, Mhi, Mlo, ldm, part, p, st);
    }
    GramPlan p = gram_plan_of(o, m, n, false);
    return gram_launch(o->working, m, n, A, lda, Mhi, Mlo, ldm, part, p, st);
}

inline hipError_t urecover_any(const gsvd_opts *o, int64_t m, int64_t n, const void *A,
                               int64_t lda, const void *W, int64_t ldw, void *U, int64_t ldu,
                               hipStream_t st) {
    if (wide_n(n)) return urecover_wide_launch(o->working, m, n, A, lda, W, ldw, U, ldu, st);
    if (o->working == GSVD_F32 && (o->flags & GSVD_U_FP32_MFMA) == 0)
        return urecover_bf16_launch(m, n, (const float *)A, lda, (const float *)W, ldw, (float *)U,
                                    ldu, st);
    return urecover_launch(o->working, m, n, A, lda, W, ldw, U, ldu, st);
}

}  // namespace gsvd

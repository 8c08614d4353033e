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
    return 0;
}

inline int max_slices(int working) {
    return working == GSVD_F64 ? GSVD_MAX_SLICES : GSVD_MAX_SLICES_F32;
}

// The eigensolver in force: AUTO is the two-sided Jacobi for FP32 working
// (M_h in FP64) and Algorithm 2 for FP64 working (M_h in double-double).
inline int eig_mode_of(const gsvd_opts *o) {
    if (o->eig != GSVD_EIG_AUTO) return o->eig;
    return o->working == GSVD_F32 ? GSVD_EIG_JACOBI2 : GSVD_EIG_CHOL_JACOBI1;
}

inline bool use_split(const gsvd_opts *o) { return o->gram == GSVD_GRAM_SPLIT; }

inline int check_supported(const gsvd_opts *o) {
    if (o->gram == GSVD_GRAM_SPLIT && o->n_slices > max_slices(o->working))
        return GSVD_ERR_UNSUPPORTED;
    // the two-sided Jacobi runs in FP64: it is the u_h solver of FP32 working only
    if (eig_mode_of(o) == GSVD_EIG_JACOBI2 && o->working != GSVD_F32) return GSVD_ERR_UNSUPPORTED;
    return 0;
}

// n > 128: the wide Gram and U kernels (64-column panels)
inline bool wide_n(int64_t n) { return n > GSVD_KMAX_N; }
// FP64 working beyond the one-workgroup eigensolver: the multi-launch Algorithm 2
inline bool wide_eig(const gsvd_opts *o, int64_t n) {
    return o->working == GSVD_F64 && n > GSVD_KMAX_N_F64;
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

// slice count of the split Gram: the caller's, else the tuning table's
inline int slices_of(const gsvd_opts *o, int64_t n) {
    if (o->n_slices > 0) return o->n_slices;
    return tune_slices(o->working, n);
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

// default rotation threshold: n u_h for the two-sided Jacobi on M_h (FP64),
// sqrt(n) u_w for the one-sided Jacobi on R in Algorithm 2
inline double jacobi_tol_of(const gsvd_opts *o, int64_t n) {
    if (o->jacobi_tol > 0) return o->jacobi_tol;
    if (eig_mode_of(o) == GSVD_EIG_JACOBI2) return (double)n * 0x1p-53;
    return __builtin_sqrt((double)n) * unit_roundoff(o->working);
}

inline int sweeps_of(const gsvd_opts *o) { return o->max_sweeps > 0 ? o->max_sweeps : 30; }

inline size_t eig_work_bytes(const gsvd_opts *o, int64_t n) {
    if (wide_eig(o, n)) return eig_wide_work_bytes(n);
    return eig_mode_of(o) == GSVD_EIG_JACOBI2 ? j2_work_bytes(n, sweeps_of(o)) : 0;
}

inline hipError_t eig_any(const gsvd_opts *o, int64_t n, const double *Mhi, const double *Mlo,
                          int64_t ldm, void *S, void *V, int64_t ldv, void *W, int64_t ldw,
                          int *info, void *work, hipStream_t st) {
    const double tol = jacobi_tol_of(o, n);
    const int sweeps = o->max_sweeps > 0 ? o->max_sweeps : 30;
    if (wide_eig(o, n))
        return eig_wide_launch(n, Mhi, Mlo, ldm, S, V, ldv, W, ldw, info, tol, sweeps, work, st);
    if (eig_mode_of(o) == GSVD_EIG_JACOBI2)
        return eig_jacobi2_launch(o->working, n, Mhi, ldm, S, V, ldv, W, ldw, info, tol, sweeps,
                                  work, st);
    return eig_launch(o->working, n, Mhi, Mlo, ldm, S, V, ldv, W, ldw, info, tol, sweeps, st);
}


inline hipError_t urecover_any(const gsvd_opts *o, int64_t m, int64_t n, const void *A,
                               int64_t lda, const void *W, int64_t ldw, void *U, int64_t ldu,
                               hipStream_t st) {
    if (wide_n(n)) return urecover_wide_launch(o->working, m, n, A, lda, W, ldw, U, ldu, st);
    return urecover_launch(o->working, m, n, A, lda, W, ldw, U, ldu, st);
}

}  // namespace gsvd

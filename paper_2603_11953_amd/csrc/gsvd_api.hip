// Host entry points of the C-ABI declared in include/gsvd.h.
//
// Every call validates its arguments synchronously, carves its workspace, and
// enqueues kernels on the caller's stream; nothing allocates device memory or
// synchronises the host.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include "gsvd.h"
#include "api_util.hpp"
#include "gsvd_internal.hpp"

using namespace gsvd;

namespace {

struct ThinLayout {
    size_t mhi, mlo, w, eigw, part, total;
};

ThinLayout thin_layout(int64_t m, int64_t n, const gsvd_opts *o) {
    ThinLayout L{};
    const size_t nn = (size_t)n * (size_t)n;
    size_t off = 0;
    L.mhi = off;
    off = align_up(off + nn * sizeof(double));
    L.mlo = off;
    off = align_up(off + nn * sizeof(double));
    L.w = off;
    off = align_up(off + nn * wsize(o->working));
    L.eigw = off;
    off = align_up(off + eig_work_bytes(o, n));
    L.part = off;
    off = align_up(off + gram_part_bytes(m, n, o, false));
    L.total = off;
    return L;
}

}  // namespace

extern "C" {

void gsvd_opts_default(gsvd_opts *o, int working) {
    if (o == nullptr) return;
    memset(o, 0, sizeof(*o));
    o->working = working;
    o->gram = GSVD_GRAM_AUTO;
    o->eig = GSVD_EIG_AUTO;
    o->n_slices = 0;
    o->jacobi_tol = 0.0;
    o->max_sweeps = 0;
    o->flags = GSVD_WANT_U;
    o->slab_rows = 0;
    o->target_rel_err = 0.0;
    o->kappa_b = 0.0;
}

const char *gsvd_status_string(int code) {
    switch (code) {
        case GSVD_OK: return "success";
        case GSVD_INFO_NOT_SPD: return "info 1: Gram matrix not positive definite (A not of full column rank at the Gram precision)";
        case GSVD_INFO_NO_CONVERGE: return "info 2: Jacobi iteration did not converge within max_sweeps";
        case GSVD_INFO_NONFINITE: return "info 3: input holds NaN or Inf";
        case GSVD_INFO_WARN_ASSUMPTION: return "info 256 (warning): the assumption eps_1 <= 1/2 of Theorem 1 could not be verified";
        case GSVD_INFO_WARN_REFINE: return "info 512 (warning): the double-double Jacobi stage left near-multiple eigenvalue pairs unrotated or did not reach its threshold";
        case GSVD_INFO_WARN_ASSUMPTION | GSVD_INFO_WARN_REFINE: return "info 768 (warnings 256 and 512)";
        case GSVD_ERR_HIP: return "HIP launch or runtime error";
        case GSVD_ERR_UNSUPPORTED: return "option combination not implemented";
        case GSVD_ERR_SCRATCH: return "workspace larger than the library's fixed scratch array (gsvd_thin_noalloc)";
        default: break;
    }
    if (code < 0 && code > -100) return "invalid argument (the value is minus its 1-based position)";
    return "unknown status";
}

size_t gsvd_gram_workspace_size(int64_t m, int64_t n, const gsvd_opts *o) {
    if (m < 1 || n < 1 || check_opts(o, 3) != 0) return 0;
    const gsvd_opts r = resolve_opts(o, m, n, false);
    return align_up(gram_part_bytes(m, n, &r, false));
}

int gsvd_gram_config(int64_t m, int64_t n, const gsvd_opts *o, int64_t *slab_rows,
                     int64_t *n_slabs, int *n_slices) {
    if (m < 1) return -1;
    if (n < 1 || n > GSVD_MAX_N || n > m) return -2;
    if (int e = check_opts(o, 3)) return e;
    const gsvd_opts r = resolve_opts(o, m, n, false);
    o = &r;
    if (int e = check_gram_supported(o, n)) return e;
    int64_t rows, slabs;
    int S = 0;
    if (wide_n(n) && use_split(o)) {
        const SplitWidePlan p = split_wide_plan(m, n, slices_of(o, n), o->slab_rows);
        rows = 2048;  // the exponent slab of the wide split form
        slabs = (m + rows - 1) / rows;
        S = p.S;
    } else if (wide_n(n)) {
        const WidePlan p = gram_wide_plan(m, n, o->slab_rows);
        rows = p.rows_per_split;
        slabs = p.nsplit;
    } else if (f32_mfma(o, n, false)) {
        const F32MfmaPlan p = f32mfma_plan_of(o, m, n);
        rows = p.rows_per_split;
        slabs = p.nsplit;
    } else if (use_split(o)) {
        const SplitPlan p = split_plan_of(o, m, n, false);
        rows = p.rows_per_split;
        slabs = p.nsplit;
        S = p.S;
    } else {
        const GramPlan p = gram_plan_of(o, m, n, false);
        rows = p.rows_per_split;
        slabs = p.nsplit;
    }
    if (slab_rows) *slab_rows = rows;
    if (n_slabs) *n_slabs = slabs;
    if (n_slices) *n_slices = S;
    return GSVD_OK;
}

int gsvd_gram(int64_t m, int64_t n, const void *dA, int64_t lda, double *dMhi, double *dMlo,
              int64_t ldm, void *work, size_t work_bytes, const gsvd_opts *o, void *stream) {
    if (m < 1) return -1;
    if (n < 1 || n > GSVD_MAX_N || n > m) return -2;
    if (dA == nullptr) return -3;
    if (lda < m) return -4;
    if (dMhi == nullptr) return -5;
    if (int e = check_opts(o, 10)) return e;
    if (o->working == GSVD_F64 && dMlo == nullptr) return -6;
    if (ldm < n) return -7;
    const size_t need = gsvd_gram_workspace_size(m, n, o);
    const gsvd_opts r = resolve_opts(o, m, n, false);
    o = &r;
    if (work == nullptr || !aligned(work, kAlign)) return -8;
    if (work_bytes < need) return -9;
    if (int e = check_gram_supported(o, n)) return e;
    hipError_t err = gram_any(o, m, n, dA, lda, dMhi, dMlo, ldm, work, (hipStream_t)stream);
    return err == hipSuccess ? GSVD_OK : GSVD_ERR_HIP;
}

size_t gsvd_eig_workspace_size(int64_t n, const gsvd_opts *o) {
    if (n < 1 || o == nullptr) return 0;
    return align_up(eig_work_bytes(o, n));
}

int gsvd_eig(int64_t n, const double *dMhi, const double *dMlo, int64_t ldm, void *dS, void *dV,
             int64_t ldv, void *dW, int64_t ldw, int *dInfo, void *work, size_t work_bytes,
             const gsvd_opts *o, void *stream) {
    if (n < 1 || n > GSVD_MAX_N) return -1;
    if (dMhi == nullptr) return -2;
    if (int e = check_opts(o, 13)) return e;
    if (o->working == GSVD_F64 && dMlo == nullptr) return -3;
    if (ldm < n) return -4;
    if (dS == nullptr) return -5;
    if (dV == nullptr) return -6;
    if (ldv < n) return -7;
    if (dW == nullptr) return -8;
    if (ldw < n) return -9;
    if (dInfo == nullptr) return -10;
    const size_t need = eig_work_bytes(o, n);
    if (need > 0 && (work == nullptr || !aligned(work, kAlign))) return -11;
    if (work_bytes < need) return -12;
    if (int e = check_eig_supported(o, n)) return e;
    // the Gram's origin is not known here: the plain form's bound
    const double u_h = o->working == GSVD_F64 ? 0x1p-104 : 0x1p-53;
    hipError_t err = eig_any(o, n, dMhi, dMlo, ldm, dS, dV, ldv, dW, ldw, dInfo, work,
                             (double)n * (double)n * u_h, (hipStream_t)stream);
    return err == hipSuccess ? GSVD_OK : GSVD_ERR_HIP;
}

int gsvd_u_recover(int64_t m, int64_t n, const void *dA, int64_t lda, const void *dW, int64_t ldw,
                   void *dU, int64_t ldu, const gsvd_opts *o, void *stream) {
    if (m < 1) return -1;
    if (n < 1 || n > GSVD_MAX_N) return -2;
    if (dA == nullptr) return -3;
    if (lda < m) return -4;
    if (dW == nullptr) return -5;
    if (ldw < n) return -6;
    if (dU == nullptr) return -7;
    if (ldu < m) return -8;
    if (int e = check_opts(o, 9)) return e;
    hipError_t err = urecover_any(o, m, n, dA, lda, dW, ldw, dU, ldu, (hipStream_t)stream);
    return err == hipSuccess ? GSVD_OK : GSVD_ERR_HIP;
}

size_t gsvd_thin_workspace_size(int64_t m, int64_t n, const gsvd_opts *o) {
    if (m < 1 || n < 1 || check_opts(o, 3) != 0) return 0;
    const gsvd_opts r = resolve_opts(o, m, n, false);
    return thin_layout(m, n, &r).total;
}

int gsvd_thin(int64_t m, int64_t n, const void *dA, int64_t lda, void *dS, void *dV, int64_t ldv,
              void *dU, int64_t ldu, void *work, size_t work_bytes, int *dInfo,
              const gsvd_opts *o, void *stream) {
    if (m < 1) return -1;
    if (n < 1 || n > GSVD_MAX_N || n > m) return -2;
    if (dA == nullptr) return -3;
    if (lda < m) return -4;
    if (dS == nullptr) return -5;
    if (dV == nullptr) return -6;
    if (ldv < n) return -7;
    if (int e = check_opts(o, 13)) return e;
    const gsvd_opts r = resolve_opts(o, m, n, false);
    o = &r;
    const bool want_u = (o->flags & GSVD_WANT_U) != 0;
    if (want_u && dU == nullptr) return -8;
    if (want_u && ldu < m) return -9;
    if (work == nullptr || !aligned(work, kAlign)) return -10;
    ThinLayout L = thin_layout(m, n, o);
    if (work_bytes < L.total) return -11;
    if (dInfo == nullptr) return -12;
    if (int e = check_eig_supported(o, n)) return e;
    if (int e = check_gram_supported(o, n)) return e;

    hipStream_t st = (hipStream_t)stream;
    char *base = (char *)work;
    double *Mhi = (double *)(base + L.mhi);
    double *Mlo = (double *)(base + L.mlo);
    void *W = base + L.w;
    hipError_t err = gram_any(o, m, n, dA, lda, Mhi, Mlo, n, base + L.part, st);
    if (err != hipSuccess) return GSVD_ERR_HIP;
    err = eig_any(o, n, Mhi, Mlo, n, dS, dV, ldv, W, n, dInfo, base + L.eigw, gram_pert_of(o, n),
                  st);
    if (err != hipSuccess) return GSVD_ERR_HIP;
    if (want_u) {
        err = urecover_any(o, m, n, dA, lda, W, n, dU, ldu, st);
        if (err != hipSuccess) return GSVD_ERR_HIP;
    }
    return GSVD_OK;
}

}  // extern "C"

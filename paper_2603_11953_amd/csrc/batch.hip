// Batched entry point: many independent thin SVDs of uneven (m, n) in one call.
//
// The host plans the whole batch from the shapes alone:
//   * problems are ordered by n (stable); consecutive problems with the same
//     Gram launch shape form a class (plain form: equal n; split form: equal
//     ceil(n / 16) and slice count), and so do those with the same U tile width;
//   * each problem gets its slab height (tuning table or the caller's), its
//     slab count, and its place in the workspace (Gram planes, W, partials).
// That plan reaches the device through kernel arguments only: a set-up kernel
// per chunk of 56 problems copies the plan into a table in the workspace and
// adds the caller's device pointers (read from the caller's device pointer
// arrays).  No host-to-device copy, allocation or synchronisation happens, so a
// stream capture of the call replays it faithfully.
//
// Then, on the caller's stream:
//   one Gram launch per class   grid (tile groups, slabs, problems of the class)
//   one reduction launch         grid (entries, problems)
//   one eigensolver launch       one workgroup per problem, largest n first
//   FP64 working, JACOBI2: the double-double Jacobi stage, a fixed sequence of
//                                launches each covering every problem
//   one assumption-check launch  one workgroup per problem
//   one U launch per class       grid (tile groups, 1, problems of the class)
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <vector>

#include "api_util.hpp"
#include "gsvd.h"
#include "gsvd_internal.hpp"

namespace gsvd {
namespace {

// What the host knows of one problem (kernel-argument payload, 72 bytes).
struct MatArg {
    int64_t m, lda, ldu, rows_per_split;
    int64_t part_off, mat_off, rw_off;  // byte offsets in the workspace (rw_off < 0: none)
    int32_t n, ldv, nsplit, pos;
};

constexpr int kChunk = 48;  // problems per set-up launch (3456 bytes of arguments)

struct SetupArgs {
    int first, count;
    MatArg a[kChunk];
};

__global__ void __launch_bounds__(64)
batch_setup_kernel(SetupArgs args, char *base, const void *const *dA, void *const *dS,
                   void *const *dV, void *const *dU, int *dInfo, int working, BatchMat *tab,
                   int *order) {
    for (int t = threadIdx.x; t < args.count; t += blockDim.x) {
        const MatArg &x = args.a[t];
        const int i = args.first + t;
        const size_t nn = (size_t)x.n * (size_t)x.n;
        BatchMat d;
        d.A = dA[i];
        d.S = dS[i];
        d.V = dV[i];
        d.U = dU ? dU[i] : nullptr;
        d.Mhi = reinterpret_cast<double *>(base + x.mat_off);
        d.Mlo = d.Mhi + nn;
        d.W = reinterpret_cast<void *>(d.Mlo + nn);
        d.part = reinterpret_cast<double *>(base + x.part_off);
        d.rw = x.rw_off >= 0 ? reinterpret_cast<double *>(base + x.rw_off) : nullptr;
        d.info = dInfo + i;
        d.m = x.m;
        d.lda = x.lda;
        d.ldu = x.ldu;
        d.rows_per_split = x.rows_per_split;
        d.n = x.n;
        d.ldv = x.ldv;
        d.nsplit = x.nsplit;
        d.pad = working;
        tab[i] = d;
        order[x.pos] = i;
    }
}

struct GramClass {
    int first, count, max_nsplit;
    GramPlan gp;
    SplitPlan sp;
};

struct UClass {
    int first, count, nt;
    int64_t max_m;
};

struct BatchPlan {
    std::vector<int> order;  // problem indices sorted by n
    std::vector<MatArg> args;
    std::vector<GramClass> gram;
    std::vector<UClass> u;
    int max_n = 0;
    size_t tab_off = 0, order_off = 0, total = 0;
};

// Returns 0 or the (negative) argument position of the first bad shape.
int plan_batch(int batch, const int64_t *hM, const int64_t *hN, const int64_t *hLda,
               const int64_t *hLdv, const int64_t *hLdu, bool want_u, const gsvd_opts *o,
               BatchPlan &P) {
    const bool split = use_split(o);
    const bool refine = o->working == GSVD_F64 && eig_mode_of(o) == GSVD_EIG_JACOBI2;
    P.order.resize(batch);
    for (int i = 0; i < batch; ++i) P.order[i] = i;
    std::stable_sort(P.order.begin(), P.order.end(),
                     [&](int a, int b) { return hN[a] < hN[b]; });
    P.args.assign(batch, MatArg{});
    size_t off = 0;
    P.tab_off = off;
    off = align_up(off + (size_t)batch * sizeof(BatchMat));
    P.order_off = off;
    off = align_up(off + (size_t)batch * sizeof(int));
    const size_t ws = wsize(o->working);
    for (int pos = 0; pos < batch; ++pos) {
        const int i = P.order[pos];
        const int64_t m = hM[i], n = hN[i];
        if (m < 1 || m < n) return -2;
        if (n < 1 || n > eig_max_n(o->working)) return -3;
        if (hLda && hLda[i] < m) return -5;
        if (hLdv && hLdv[i] < n) return -8;
        if (want_u && hLdu && hLdu[i] < m) return -10;
        MatArg &x = P.args[i];
        x.m = m;
        x.n = (int32_t)n;
        x.lda = hLda ? hLda[i] : m;
        x.ldv = (int32_t)(hLdv ? hLdv[i] : n);
        x.ldu = hLdu ? hLdu[i] : m;
        x.pos = pos;
        GramPlan gp{};
        SplitPlan sp{};
        size_t part;
        if (split) {
            sp = split_plan_of(o, m, n, true);
            x.rows_per_split = sp.rows_per_split;
            x.nsplit = (int32_t)sp.nsplit;
            part = sp.part_bytes;
        } else {
            gp = gram_plan_of(o, m, n, true);
            x.rows_per_split = gp.rows_per_split;
            x.nsplit = (int32_t)gp.nsplit;
            part = gp.part_bytes;
        }
        if (x.nsplit > 65535) return -2;
        const size_t nn = (size_t)n * (size_t)n;
        x.mat_off = off;
        off = align_up(off + 2 * nn * sizeof(double) + nn * ws);
        x.part_off = off;
        off = align_up(off + part);
        x.rw_off = -1;
        if (refine) {
            x.rw_off = (int64_t)off;
            off = align_up(off + refine_work_bytes(n));
        }
        // Gram classes: consecutive problems with the same launch shape
        const bool same = !P.gram.empty() &&
                          (split ? (P.gram.back().sp.nb == sp.nb && P.gram.back().sp.S == sp.S &&
                                    P.gram.back().sp.lds_bytes == sp.lds_bytes)
                                 : (P.args[P.order[P.gram.back().first]].n == x.n));
        if (same && P.gram.back().count < 65535) {
            GramClass &c = P.gram.back();
            ++c.count;
            c.max_nsplit = std::max(c.max_nsplit, (int)x.nsplit);
        } else {
            P.gram.push_back(GramClass{pos, 1, (int)x.nsplit, gp, sp});
        }
        const int nt = (int)((n + 15) / 16);
        if (!P.u.empty() && P.u.back().nt == nt && P.u.back().count < 65535) {
            ++P.u.back().count;
            P.u.back().max_m = std::max(P.u.back().max_m, m);
        } else {
            P.u.push_back(UClass{pos, 1, nt, m});
        }
        P.max_n = std::max(P.max_n, (int)n);
    }
    P.total = off;
    return 0;
}

// One Gram form and slice count for the whole batch, resolved at its largest n.
gsvd_opts resolve_batched(const gsvd_opts *o, int batch, const int64_t *hN) {
    int64_t nmax = 1;
    for (int i = 0; i < batch; ++i) nmax = std::max(nmax, hN[i]);
    return resolve_opts(o, 0, nmax, true);
}

}  // namespace
}  // namespace gsvd

using namespace gsvd;

extern "C" {

size_t gsvd_thin_batched_workspace_size(int batch, const int64_t *hM, const int64_t *hN,
                                        const gsvd_opts *o) {
    if (batch < 1 || batch > 65535 || hM == nullptr || hN == nullptr || check_opts(o, 4) != 0)
        return 0;
    const gsvd_opts r = resolve_batched(o, batch, hN);
    o = &r;
    BatchPlan P;
    if (plan_batch(batch, hM, hN, nullptr, nullptr, nullptr, false, o, P) != 0) return 0;
    return P.total;
}

int gsvd_thin_batched(int batch, const int64_t *hM, const int64_t *hN, const void *const *dA,
                      const int64_t *hLda, void *const *dS, void *const *dV, const int64_t *hLdv,
                      void *const *dU, const int64_t *hLdu, void *work, size_t work_bytes,
                      int *dInfo, const gsvd_opts *o, void *stream) {
    if (batch < 1 || batch > 65535) return -1;
    if (hM == nullptr) return -2;
    if (hN == nullptr) return -3;
    if (dA == nullptr) return -4;
    if (hLda == nullptr) return -5;
    if (dS == nullptr) return -6;
    if (dV == nullptr) return -7;
    if (hLdv == nullptr) return -8;
    if (int e = check_opts(o, 14)) return e;
    const gsvd_opts r = resolve_batched(o, batch, hN);
    o = &r;
    const bool want_u = (o->flags & GSVD_WANT_U) != 0;
    if (want_u && dU == nullptr) return -9;
    if (want_u && hLdu == nullptr) return -10;
    if (work == nullptr || !aligned(work, kAlign)) return -11;
    if (dInfo == nullptr) return -13;
    if (int e = check_supported(o)) return e;
    BatchPlan P;
    if (int e = plan_batch(batch, hM, hN, hLda, hLdv, hLdu, want_u, o, P)) return e;
    if (work_bytes < P.total) return -12;
    if (want_u) {
        for (const UClass &c : P.u)
            if (c.nt > urecover_batched_max_nt(o->working)) return GSVD_ERR_UNSUPPORTED;
    }

    hipStream_t st = (hipStream_t)stream;
    char *base = (char *)work;
    BatchMat *tab = reinterpret_cast<BatchMat *>(base + P.tab_off);
    int *order = reinterpret_cast<int *>(base + P.order_off);
    for (int first = 0; first < batch; first += kChunk) {
        SetupArgs a{};
        a.first = first;
        a.count = std::min(kChunk, batch - first);
        for (int t = 0; t < a.count; ++t) a.a[t] = P.args[first + t];
        hipLaunchKernelGGL(batch_setup_kernel, dim3(1), dim3(64), 0, st, a, base, dA, dS, dV,
                           want_u ? dU : nullptr, dInfo, o->working, tab, order);
        if (hipGetLastError() != hipSuccess) return GSVD_ERR_HIP;
    }
    hipError_t err = hipSuccess;
    for (const GramClass &c : P.gram) {
        err = use_split(o) ? split_batched_launch(o->working, tab, order, c.first, c.count,
                                                  c.max_nsplit, c.sp, st)
                           : gram_batched_launch(o->working, tab, order, c.first, c.count,
                                                 c.max_nsplit, c.gp, st);
        if (err != hipSuccess) return GSVD_ERR_HIP;
    }
    err = use_split(o) ? split_reduce_batched_launch(tab, batch, P.max_n, st)
                       : gram_reduce_batched_launch(tab, batch, P.max_n, st);
    if (err != hipSuccess) return GSVD_ERR_HIP;
    if (o->working == GSVD_F64) {
        const bool pre = eig_mode_of(o) == GSVD_EIG_JACOBI2;
        err = pre ? eig_batched_launch(o->working, tab, order, batch, P.max_n, pre_tol_of(o),
                                       pre_sweeps_of(o), true, st)
                  : eig_batched_launch(o->working, tab, order, batch, P.max_n, o->jacobi_tol,
                                       sweeps_of(o), false, st);
        if (err == hipSuccess && pre) err = refine_batched_launch(tab, batch, P.max_n, st);
    } else {
        err = eig_mode_of(o) == GSVD_EIG_JACOBI2
                  ? eig_jacobi2_batched_launch(o->working, tab, order, batch, P.max_n,
                                               o->jacobi_tol, sweeps_of(o), st)
                  : eig_batched_launch(o->working, tab, order, batch, P.max_n, o->jacobi_tol,
                                       sweeps_of(o), false, st);
    }
    if (err == hipSuccess)
        err = assump_batched_launch(o->working, tab, batch, gram_pert_of(o, P.max_n),
                                    eig_mode_of(o) == GSVD_EIG_CHOL_JACOBI1, P.max_n, st);
    if (err != hipSuccess) return GSVD_ERR_HIP;
    if (want_u) {
        for (const UClass &c : P.u) {
            err = urecover_batched_launch(o->working, tab, order, c.first, c.count, c.nt, c.max_m,
                                          st);
            if (err != hipSuccess) return GSVD_ERR_HIP;
        }
    }
    return GSVD_OK;
}

}  // extern "C"

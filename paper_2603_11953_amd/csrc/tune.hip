// Lookups in the tuning table (tune_table.inc, written by autotune.py).
#include "gsvd.h"
#include "tune.hpp"

namespace gsvd {

#include "tune_table.inc"

int64_t tune_slab_rows(int working, int gram, int64_t n, int64_t m, bool batched) {
    for (const TuneSlab &r : kTuneSlab)
        if (r.working == working && r.gram == gram && r.batched == (batched ? 1 : 0) &&
            n <= r.n_max && m <= r.m_max)
            return r.slab_rows;
    return 0;
}

bool tune_gram_ms(int working, int gram, int64_t n, int64_t m, bool batched, double *ms,
                  int *slices) {
    for (const TuneSlab &r : kTuneSlab)
        if (r.working == working && r.gram == gram && r.batched == (batched ? 1 : 0) &&
            n <= r.n_max && m <= r.m_max) {
            *ms = r.ms;
            *slices = r.slices;
            return true;
        }
    return false;
}

double tune_eps(int working, int64_t n, int S) {
    if (S >= 1 && S <= 12)
        for (const TuneEps &r : kTuneEps)
            if (r.working == working && n <= r.n_max && r.eps[S - 1] > 0.0) return r.eps[S - 1];
    return __builtin_ldexp(1.0, 12 - 8 * S);
}

}  // namespace gsvd

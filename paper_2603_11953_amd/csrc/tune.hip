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

int tune_slices(int working, int64_t n) {
    for (const TuneSlices &r : kTuneSlices)
        if (r.working == working && n <= r.n_max) return r.slices;
    return working == GSVD_F64 ? 10 : 6;
}

}  // namespace gsvd

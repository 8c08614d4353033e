// Launch-shape and slice-count tuning table: lookups (tune.hip) over the rows
// that paper_2603_11953_amd/autotune.py measured and wrote to tune_table.inc.
#pragma once

#include <stdint.h>

namespace gsvd {

struct TuneSlab {
    int working;       // GSVD_F32 / GSVD_F64
    int gram;          // GSVD_GRAM_PLAIN / GSVD_GRAM_SPLIT
    int batched;       // 0: one problem per call, 1: the batched entry point
    int n_max;         // row applies to n <= n_max ...
    int64_t m_max;     // ... and m <= m_max (first matching row wins)
    int64_t slab_rows; // rows of A per Gram workgroup
    double ms;         // Gram time at that height, at the bucket's tuning size
    int slices;        // split rows: the slice count the time was taken at
};

struct TuneEps {
    int working;
    int n_max;
    double eps[12];    // measured Gram error of the split form with S = 1 .. 12 slices,
                       // max |dM_ij| / sqrt(M_ii M_jj) (0: not measured)
};

// 0 when no row matches: the plan then uses its own default slab count
int64_t tune_slab_rows(int working, int gram, int64_t n, int64_t m, bool batched);
// the tuned Gram time (ms) and, for the split form, the slice count it was taken
// at, of the row that applies; false when no row applies
bool tune_gram_ms(int working, int gram, int64_t n, int64_t m, bool batched, double *ms,
                  int *slices);
// the split Gram's error for S slices (scaled as above): the table's measurement,
// else the a-priori 2^(12 - 8 S) (a digit pair's dropped remainder, 2^(-8 S) of
// the slab's column scale 2^E <= 64 max|a|, summed over a slab)
double tune_eps(int working, int64_t n, int S);

}  // namespace gsvd

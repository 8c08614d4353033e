// Instances of the operand-split Gram kernels for float A (every 16-column block
// count and slice count), compiled on their own so the two element types build in parallel.
#include "gram_split.hpp"
#include "gsvd_internal.hpp"

namespace gsvd {

hipError_t split_partial_f32(int64_t m, int64_t n, const float *A, int64_t lda, void *part,
                              const SplitPlan &p, hipStream_t st) {
    return split_partial_typed<float>(m, n, A, lda, part, p, st);
}

hipError_t split_batched_f32(const BatchMat *tab, const int *order, int first, int count,
                              int max_nsplit, const SplitPlan &p, hipStream_t st) {
    return split_batched_typed<float>(tab, order, first, count, max_nsplit, p, st);
}

}  // namespace gsvd

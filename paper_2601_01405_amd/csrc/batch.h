// batch.h — the batched driver of bm_build_many (batch.cpp).
#pragma once
#include "host_common.h"

namespace bm {
namespace host {

// Whether a problem's chains can run in a batch: points, radii, a matrix-core
// path (the plain FP32 path and d past the matrix-core K run one build at a time).
bool batchable(const bm_problem &pr, const bm_options &o);
// Whether the batch's keys and union numbering fit 64-bit keys and int32 indices.
bool batch_fits(const std::vector<const bm_problem *> &probs);
// Candidate block size of a chain when the options leave it automatic.
int32_t batch_block(int64_t n, int32_t d, int32_t path);
// Every (problem, radius) chain of probs; chain e of problem p goes to
// outs[slot0[p] + e].  Throws BmError; on error no result is left allocated.
void run_batch(const std::vector<const bm_problem *> &probs, const std::vector<int64_t> &slot0, const bm_options &o,
               bm_result **outs);

} // namespace host
} // namespace bm

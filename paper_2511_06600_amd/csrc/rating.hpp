// Resistance-based vertex-pair rating (Section III-E, Eq. (17)).
#pragma once

#include "common.hpp"

namespace hef {

size_t rating_bytes(int64_t n, int64_t m, int64_t nnz);

// Per node p: best[p] = the neighbour q of largest
// r(p, q) = sum_{e holding p and q} w(e) / (R_e - shift) (ties to the
// smallest q, -1 without neighbours) and rating[p] = r(p, best[p]).
// Validates the hypergraph and R on the device; synchronises `s`.
hef_status rating_run(const Level &L, const float *R, float shift, int32_t *best, double *rating,
                      void *ws, size_t ws_bytes, hipStream_t s);

}  // namespace hef

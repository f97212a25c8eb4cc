// Alg. 2: Eq. (15) update, threshold contraction, resistance-based local
// clustering and coarse rebuild; and the adjoint of Alg. 1.
#pragma once

#include "common.hpp"
#include "structure.hpp"

namespace hef {

size_t coarsen_bytes(int64_t n, int64_t m, int64_t nnz, const hef_params &p);
size_t cluster_level_bytes(int64_t n, int64_t m, int64_t nnz, int K);
size_t rebuild_call_bytes(int64_t n, int64_t m, int64_t nnz);
size_t backward_bytes(int64_t n, int64_t m, int64_t nnz, const hef_params &p);

// Alg. 1 on one level (defined with the C ABI).
hef_status estimate_level(const Level &L, const hef_params &p, uint64_t seed, int level,
                          const float *start_star, const float *start_clique, Structure &st,
                          void *pool, void *pool2, double *qh, float *R, Arena &ws,
                          hipStream_t s, double *rho = nullptr);
size_t estimate_level_bytes(int64_t n, int64_t m, int64_t nnz, const hef_params &p);
int pool_width_of(const hef_params &p);

}  // namespace hef

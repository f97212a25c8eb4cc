// Per-level structure and scales of the implicit star and clique expansions.
#pragma once

#include "common.hpp"

namespace hef {

// Segments longer than this go to the wave-per-segment kernels.
constexpr int kSmallSeg = 32;

struct Structure {
  // CSC incidence (node -> hyperedges), hyperedges ascending per node.
  int32_t *vptr = nullptr;  // [n+1]
  int32_t *eids = nullptr;  // [nnz]
  // Expansion scales (float32, computed in float64):
  //   s[u]     = d_b(u)^-1/2, d_b(u) = sum_{e ∋ u} w_e/|e|  (0 if d_b = 0)
  //   gam[u]   = s[u]^2 * sum_{e ∋ u} beta_e  (clique self-term)
  //   alpha[e] = sqrt(w_e)/|e|  (star edge factor, d_b(e) = w_e)
  //   beta[e]  = w_e/(|e|(|e|-1))  (half the clique pair weight c_e)
  float *s = nullptr, *gam = nullptr, *alpha = nullptr, *beta = nullptr;
  // Hyperedges / nodes whose segment exceeds kSmallSeg, ascending, and counts.
  int32_t *big_e = nullptr, *big_v = nullptr;
  int32_t *n_big = nullptr;  // [2]: big edges, big nodes
};

// Workspace of a Structure plus the temporaries to build it.
void structure_carve(Arena &a, int64_t n, int64_t m, int64_t nnz, Structure &st);
size_t structure_build_ws(int64_t n, int64_t m, int64_t nnz);

// Device validation of a CSR hypergraph; *bad_host != 0 if invalid.
hef_status validate_device(const Level &L, int32_t *flag_dev, int32_t *bad_host,
                           hipStream_t s);

// Builds CSC, scales and big-segment lists for one level.
hef_status structure_build(const Level &L, Structure &st, Arena &ws, hipStream_t s);

}  // namespace hef

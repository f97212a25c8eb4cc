// Alg. 2 (placeholder until the clustering kernels land).
#include "cluster.hpp"

namespace hef {
size_t coarsen_extra_bytes(int64_t, int64_t, int64_t, int) { return 0; }
size_t cluster_level_bytes(int64_t, int64_t, int64_t, int) { return 0; }
size_t backward_bytes(int64_t, int64_t, int64_t, const hef_params &) { return 0; }
}  // namespace hef

extern "C" {
hef_status hef_coarsen(const hef_hypergraph *, const hef_params *, int32_t *, int32_t *, float *,
                       float *, void *, size_t, hipStream_t) {
  return HEF_ERR_UNSUPPORTED;
}
hef_status hef_cluster_level(const hef_hypergraph *, const hef_params *, const float *,
                             const float *, const float *, const double *, int32_t *, int32_t *,
                             float *, void *, size_t, hipStream_t) {
  return HEF_ERR_UNSUPPORTED;
}
hef_status hef_resistance_backward(const hef_hypergraph *, const hef_params *, const float *,
                                   const float *, const float *, float *, void *, size_t,
                                   hipStream_t) {
  return HEF_ERR_UNSUPPORTED;
}
}

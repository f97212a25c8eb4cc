// Cluster quality (Section II-A, Eq. (3); Eq. (18)).
#pragma once

#include "common.hpp"

namespace hef {

// Workspace bytes of hef_conductance for n_clusters up to max(n, 1).
size_t conductance_bytes(int64_t n, int64_t m, int64_t nnz);

}  // namespace hef

// Resistance ratios over the orthonormal pool (Eqs. (9), (13), (14)).
#pragma once

#include "common.hpp"

namespace hef {

size_t score_ws_bytes(int64_t m, int K);

// qh[i] = Q_H(chi^(i)) = sum_e w_e (max_{p in e} chi_p - min_{p in e} chi_p)^2
// (float64, fixed summation order), then
// R[e] = max_{i: qh[i] > 0} (max - min)^2 / qh[i]  (0 if no usable column).
// The numerators (max - min)^2 are formed as float32, m x K with row e
// contiguous; with keep_s they are left there (caller-owned, m * K floats).
hef_status score_pool(const Level &L, const void *pool, int pool_type, int K, double *qh,
                      float *R, Arena &ws, hipStream_t s, float *keep_s = nullptr);

}  // namespace hef

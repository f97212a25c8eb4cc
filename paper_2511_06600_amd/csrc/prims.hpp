// Device primitives used by several stages: exclusive scan, stable LSD radix
// sort of (key, value) pairs, stream compaction.  All are deterministic.
#pragma once

#include "common.hpp"

namespace hef {

// Workspace bytes for exclusive_scan over `n` elements.
size_t scan_ws_bytes(int64_t n);
// out[i] = sum_{j<i} in[j]; out[n] = total (out has n+1 entries).
// `in` and `out` may alias.
hef_status exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n,
                              Arena &ws, hipStream_t s);

// Workspace bytes for radix_sort_pairs over `n` items.
size_t radix_ws_bytes(int64_t n);
// Stable LSD radix sort of (keys, vals) by the low `bits` bits of keys.
// On return the sorted data is in (keys_out, vals_out); the inputs are
// clobbered (used as ping-pong buffers).
hef_status radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *keys_out,
                            uint32_t *vals_out, int64_t n, int bits, Arena &ws,
                            hipStream_t s);

// idx_out[0..count) = ascending indices i < n with flag[i] != 0;
// *count_dev = count.  Uses `scratch` of n+1 int32.
hef_status compact_flags(const int32_t *flag, int32_t *scratch, int32_t *idx_out,
                         int32_t *count_dev, int64_t n, Arena &ws, hipStream_t s);

// out[c] = sum_r in[r * ncols + c] (float64) in a fixed order that does not
// depend on timing: 32 row lanes per column each sum every 32nd row (eight
// interleaved accumulators), then a fixed tree over the lanes.
hef_status reduce_cols_f64(const double *in, int64_t nrows, int64_t ncols, double *out,
                           hipStream_t s);
// Two independent reduce_cols_f64 (same ncols) in one launch.
hef_status reduce_cols_f64_pair(const double *in0, int64_t nrows0, double *out0,
                                const double *in1, int64_t nrows1, double *out1, int64_t ncols,
                                hipStream_t s);

// Zeroes `bytes` bytes at p on stream s with a fill kernel rather than
// hipMemsetAsync, so that a caller capturing the stream into a HIP graph
// records kernel nodes only.
hef_status zero_async(void *p, size_t bytes, hipStream_t s);

inline int bits_for(int64_t maxval) {
  int b = 1;
  while (b < 32 && (int64_t(1) << b) <= maxval) ++b;
  return b;
}

}  // namespace hef

// Internal helpers shared by the HIP translation units of libhyperef.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <string>

#include "hyperef.h"

namespace hef {

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
const char *last_error();

#define HEF_HIP(call)                                                        \
  do {                                                                       \
    hipError_t _e = (call);                                                  \
    if (_e != hipSuccess) {                                                  \
      ::hef::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(_e), \
                       __FILE__, __LINE__);                                  \
      return HEF_ERR_DEVICE;                                                 \
    }                                                                        \
  } while (0)

#define HEF_TRY(expr)                  \
  do {                                 \
    hef_status _s = (expr);            \
    if (_s != HEF_OK) return _s;       \
  } while (0)

#define HEF_LAUNCH_CHECK() HEF_HIP(hipGetLastError())

// A workspace carve that ran past the caller's workspace.
#define HEF_WS_CHECK(arena)                                                       \
  do {                                                                            \
    if ((arena).overflow) {                                                       \
      ::hef::set_error("workspace overflow in %s (%s:%d)", __func__, __FILE__, __LINE__); \
      return HEF_ERR_WORKSPACE_TOO_SMALL;                                         \
    }                                                                             \
  } while (0)

// ------------------------------------------------------------- workspace
// Bump allocator over the caller's workspace.  With base == nullptr it only
// measures, so the planner and the runtime carve the workspace identically.
struct Arena {
  char *base = nullptr;
  size_t cap = 0;
  size_t off = 0;
  bool overflow = false;

  template <class T>
  T *take(size_t count) {
    size_t bytes = count * sizeof(T);
    size_t start = (off + 255) & ~size_t(255);
    off = start + bytes;
    if (base == nullptr) return nullptr;
    if (off > cap) {
      overflow = true;
      return nullptr;
    }
    return reinterpret_cast<T *>(base + start);
  }
  size_t mark() const { return off; }
  void reset(size_t m) { off = m; }
};

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// The Krylov pool before orthonormalisation is stored in a row-octet layout:
// rows in groups of 8, each column of a group contiguous, i.e. element
// (r, c) of an n x K pool at ((r >> 3) * K + c) * 8 + (r & 7), with n
// padded to oct_rows(n) (padding rows are zero).
inline int64_t oct_rows(int64_t n) { return (n + 7) / 8 * 8; }

// Orders the LDS accesses of one wave: what a lane wrote before the call is
// seen by the wave's other lanes after it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Map a launched block index to a logical one so that each of the 8 XCDs of
// an MI355X (which receive blocks round-robin) walks a contiguous range of
// logical blocks; neighbouring work then shares its XCD's L2.
// Lane l's value of v on every lane (l the same on all lanes: a scalar
// broadcast, no LDS round trip).
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(u), l);
  const uint32_t hi = __builtin_amdgcn_readlane(uint32_t(u >> 32), l);
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}

__device__ __forceinline__ int64_t xcd_block(int64_t bid, int64_t nblocks) {
  constexpr int64_t kXcd = 8;
  int64_t per = nblocks / kXcd;
  int64_t rem = nblocks % kXcd;
  int64_t x = bid % kXcd;
  int64_t i = bid / kXcd;
  // XCDs 0..rem-1 own per+1 blocks, the rest own per.
  int64_t start = x * per + (x < rem ? x : rem);
  int64_t cnt = per + (x < rem ? 1 : 0);
  return i < cnt ? start + i : bid;  // i < cnt always holds for a full grid
}

// Level-independent sizes of one hypergraph level.
struct Level {
  int32_t n = 0, m = 0;
  int64_t nnz = 0;
  const int32_t *eptr = nullptr;
  const int32_t *pins = nullptr;
  const float *w = nullptr;  // nullptr = unit weights
};

}  // namespace hef

namespace hef {

// ------------------------------------------------------------ stage timing
// Optional per-stage kernel timing (hef_timing_enable): HIP events recorded
// on the launch stream around each stage's kernels.  Off by default; when
// off a TimedScope does nothing.
enum Stage : int {
  kStStructure = 0,
  kStSpmmCsr,
  kStSpmmCsc,
  kStLanczosGram,
  kStLanczosSolve,
  kStLanczosApply,
  kStOrthGram,
  kStOrthChol,
  kStOrthApply,
  kStScoreQ,
  kStScoreR,
  kStClusterUpdate,
  kStClusterContract,
  kStClusterLocal,
  kStClusterRebuild,
  kStAdjoint,
  kStStart,
  kStSpmmPrep,
  kStLanczosReduce,
  kStOrthReduce,
  kStScoreReduce,
  kStClusterBest,
  kStQuality,
  kStRating,
  kStSpmmStep,  // the fused SpMM (prep, CSR and CSC) as one span; off unless selected
  kStageCount
};

bool timing_on(int stage);
void timing_push(int stage, hipEvent_t a, hipEvent_t b);

struct TimedScope {
  int stage;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  TimedScope(int st, hipStream_t stream) : stage(st), s(stream) {
    if (timing_on(st)) {
      if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
        (void)hipEventRecord(a, s);
      else
        a = b = nullptr;
    }
  }
  ~TimedScope() {
    if (a && b) {
      (void)hipEventRecord(b, s);
      timing_push(stage, a, b);
    }
  }
};

}  // namespace hef

// The C ABI (include/hyperef.h): argument checks, workspace planning and
// the order of the stages of Alg. 1 and Alg. 2.
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "cluster.hpp"
#include "krylov.hpp"
#include "quality.hpp"
#include "orth.hpp"
#include "rating.hpp"
#include "prims.hpp"
#include "score.hpp"
#include "structure.hpp"

namespace hef {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}

const char *last_error() { return g_err.c_str(); }

// ---- stage timing (profiling aid; the only process-wide state besides the
// per-thread error text)
static std::atomic<int> g_timing{0};
static std::mutex g_tmu;
static std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> g_pending;
static double g_ms[kStageCount];
static int64_t g_cnt[kStageCount];

// every stage but the spmm_step span, which would count the SpMM twice
static std::atomic<uint32_t> g_timing_mask{~(1u << kStSpmmStep)};
static_assert(kStageCount <= 32, "the stage mask is 32 bits");
bool timing_on(int stage) {
  return g_timing.load(std::memory_order_relaxed) != 0 &&
         ((g_timing_mask.load(std::memory_order_relaxed) >> stage) & 1u) != 0;
}

void timing_push(int stage, hipEvent_t a, hipEvent_t b) {
  std::lock_guard<std::mutex> lk(g_tmu);
  g_pending.emplace_back(stage, a, b);
}

static const char *kStageNames[kStageCount] = {
    "structure", "spmm_csr", "spmm_csc", "lanczos_gram", "lanczos_solve", "lanczos_apply",
    "orth_gram", "orth_chol", "orth_apply", "score_qh", "score_r", "cluster_update",
    "cluster_contract", "cluster_local", "cluster_rebuild", "adjoint", "start_block",
    "spmm_prep", "lanczos_reduce", "orth_reduce",
    "score_reduce", "cluster_best", "quality", "rating", "spmm_step"};

namespace {

bool pow2_block(int b) { return b == 1 || b == 2 || b == 4 || b == 8 || b == 16; }

int pool_width(const hef_params &p) {
  const int nexp = ((p.flags & HEF_FLAG_STAR_ONLY) || (p.flags & HEF_FLAG_CLIQUE_ONLY)) ? 1 : 2;
  return nexp * p.b * p.k;
}

hef_status check_hg(const hef_hypergraph *hg) {
  if (!hg) { set_error("hypergraph is NULL"); return HEF_ERR_INVALID_ARGUMENT; }
  if (hg->n < 0 || hg->m < 0 || hg->nnz < 0) {
    set_error("negative size (n=%d m=%d nnz=%lld)", hg->n, hg->m, (long long)hg->nnz);
    return HEF_ERR_INVALID_ARGUMENT;
  }
  if (hg->nnz > INT32_MAX) { set_error("nnz exceeds int32"); return HEF_ERR_UNSUPPORTED; }
  if (!hg->eptr || (hg->nnz > 0 && !hg->pins)) {
    set_error("eptr or pins is NULL");
    return HEF_ERR_INVALID_ARGUMENT;
  }
  return HEF_OK;
}

hef_status check_params(const hef_params *p, bool need_levels, bool allow_fp64 = false) {
  if (!p) { set_error("params is NULL"); return HEF_ERR_INVALID_ARGUMENT; }
  if (p->k < 1 || p->k > 1024) { set_error("k=%d out of range", p->k); return HEF_ERR_INVALID_ARGUMENT; }
  if (!pow2_block(p->b)) {
    set_error("b=%d: start blocks of 1, 2, 4, 8 or 16 columns are supported", p->b);
    return HEF_ERR_UNSUPPORTED;
  }
  if (pool_width(*p) > 512) {
    set_error("pool width %d exceeds 512", pool_width(*p));
    return HEF_ERR_UNSUPPORTED;
  }
  if (p->basis != HEF_BASIS_FP32 && p->basis != HEF_BASIS_BF16 && p->basis != HEF_BASIS_FP64) {
    set_error("unknown basis %d", p->basis);
    return HEF_ERR_INVALID_ARGUMENT;
  }
  if (p->basis == HEF_BASIS_FP64 && !allow_fp64) {
    set_error("the float64 basis is a debug basis of hef_resistance only");
    return HEF_ERR_UNSUPPORTED;
  }
  if (p->basis == HEF_BASIS_FP64 && p->orth_passes != 1) {
    set_error("the float64 basis takes orth_passes = 1");
    return HEF_ERR_UNSUPPORTED;
  }
  if (!(p->drop_tol >= 0.0f && p->drop_tol < 1.0f)) {
    set_error("drop_tol must lie in [0, 1)");
    return HEF_ERR_INVALID_ARGUMENT;
  }
  if (p->orth_passes != 1 && p->orth_passes != 2) {
    set_error("orth_passes must be 1 or 2");
    return HEF_ERR_INVALID_ARGUMENT;
  }
  if ((p->flags & HEF_FLAG_STAR_ONLY) && (p->flags & HEF_FLAG_CLIQUE_ONLY)) {
    set_error("STAR_ONLY and CLIQUE_ONLY are exclusive");
    return HEF_ERR_INVALID_ARGUMENT;
  }
  if (need_levels) {
    if (p->levels < 1 || p->levels > 64) { set_error("levels out of range"); return HEF_ERR_INVALID_ARGUMENT; }
    if (!(p->target_nr >= 0.0f && p->target_nr < 1.0f)) {
      set_error("target_nr must lie in [0, 1)");
      return HEF_ERR_INVALID_ARGUMENT;
    }
    if (!(p->percentile > 0.0f && p->percentile <= 1.0f)) {
      set_error("percentile must lie in (0, 1]");
      return HEF_ERR_INVALID_ARGUMENT;
    }
  }
  return HEF_OK;
}

Level level_of(const hef_hypergraph *hg) {
  Level L;
  L.n = hg->n;
  L.m = hg->m;
  L.nnz = hg->nnz;
  L.eptr = hg->eptr;
  L.pins = hg->pins;
  L.w = hg->w;
  return L;
}

size_t pool_bytes(int64_t n, int K, int basis) {
  return size_t(n) * K * (basis == HEF_BASIS_BF16 ? 2 : basis == HEF_BASIS_FP64 ? 8 : 4);
}

// Scratch needed by one resistance estimate at these sizes (beyond the
// Structure and the pool).
size_t estimate_scratch(int64_t n, int64_t m, int64_t nnz, const hef_params &p) {
  const int K = pool_width(p);
  size_t need = structure_build_ws(n, m, nnz);
  Arena a;
  a.take<float>((n + m) * p.b);  // start blocks
  a.take<float>(n * p.b);
  const size_t starts = a.mark();
  need = std::max(need, starts + krylov_ws_bytes(n, m, p.b));
  need = std::max(need, orth_ws_bytes(n, K));
  need = std::max(need, score_ws_bytes(m, K));
  return need + 4096;
}

size_t resistance_bytes(int64_t n, int64_t m, int64_t nnz, const hef_params &p, bool own_pool) {
  Arena a;
  Structure st;
  structure_carve(a, n, m, nnz, st);
  a.take<int32_t>(4);  // flags
  const int K = pool_width(p);
  if (own_pool) a.take<char>(pool_bytes(n, K, p.basis));
  a.take<char>(pool_bytes(oct_rows(n), K, p.basis));  // the Krylov pool before orthonormalisation
  a.take<double>(K);  // qh
  a.take<float>(m);   // R
  return a.mark() + estimate_scratch(n, m, nnz, p) + 1024;
}

__global__ void k_check_finite(const float *R, int64_t m, const double *qh, int K, int32_t *flag) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < m && !isfinite(R[i])) atomicOr(flag, 1);
  if (i < K) {
    if (!isfinite(qh[i])) atomicOr(flag, 1);
    if (qh[i] > 0.0) atomicOr(flag, 2);
  }
}

}  // namespace

// Alg. 1 on one level; the orthonormal pool ends in `pool` (n x K); `pool2`
// (oct_rows(n) x K) holds the Krylov pool before orthonormalisation; qh and R
// are caller- or arena-provided.
hef_status estimate_level(const Level &L, const hef_params &p, uint64_t seed, int level,
                          const float *start_star, const float *start_clique, Structure &st,
                          void *pool, void *pool2, double *qh, float *R, Arena &ws,
                          hipStream_t s, double *rho) {
  const int64_t n = L.n, m = L.m;
  const int K = pool_width(p);
  const int B = p.b;
  const bool use_star = !(p.flags & HEF_FLAG_CLIQUE_ONLY);
  const bool use_clique = !(p.flags & HEF_FLAG_STAR_ONLY);
  HEF_TRY(structure_build(L, st, ws, s));
  const size_t mk = ws.mark();
  float *xs = nullptr, *xc = nullptr;
  if (use_star && !start_star) {
    xs = ws.take<float>((n + m) * B);
    HEF_WS_CHECK(ws);
    HEF_TRY(start_block(seed, level, 0, n + m, B, xs, s));
    start_star = xs;
  }
  if (use_clique && !start_clique) {
    xc = ws.take<float>(n * B);
    HEF_WS_CHECK(ws);
    HEF_TRY(start_block(seed, level, 1, n, B, xc, s));
    start_clique = xc;
  }
  // the Krylov pool (row-octet layout) in pool2, its orthonormal basis in pool
  KrylovOut ko;
  ko.pool = pool2;
  ko.K = K;
  ko.pool_type = p.basis == HEF_BASIS_BF16 ? kPoolBF16
                 : p.basis == HEF_BASIS_FP64 ? kPoolF64 : kPoolF32;
  HEF_TRY(krylov_pool(L, st, B, p.k, double(p.drop_tol), start_star, start_clique, use_star,
                      use_clique, ko, ws, s));
  ws.reset(mk);
  HEF_TRY(orthonormalize_pool(pool2, pool, ko.pool_type, n, K, double(p.drop_tol),
                              p.orth_passes, nullptr, ws, s, nullptr, rho));
  HEF_TRY(score_pool(L, pool, ko.pool_type, K, qh, R, ws, s));
  return HEF_OK;
}

size_t estimate_level_bytes(int64_t n, int64_t m, int64_t nnz, const hef_params &p) {
  return estimate_scratch(n, m, nnz, p);
}

int pool_width_of(const hef_params &p) { return pool_width(p); }


// ---- static scratch of hef_resistance_static: one array per device (each
// device holds its own copy at its own address until the process ends).  In
// host code `scratch` names a host-side stand-in, never device memory: the
// device address comes from hipGetSymbolAddress, once per device with that
// device current, and only that address is handed to kernels.
static __device__ __align__(256) char scratch[HEF_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hef_status static_scratch(void **out) {
  int dev = -1;
  HEF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d: the static scratch supports devices 0..%d", dev, kMaxDevices - 1);
    return HEF_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      set_error("hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorString(e));
      return HEF_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return HEF_OK;
}

hef_status resistance_call(const hef_hypergraph *hg, const hef_params *p, const float *start_star,
                           const float *start_clique, float *R, double *qh, void *chi, void *ws,
                           size_t ws_bytes, hipStream_t stream);

}  // namespace hef

using namespace hef;

extern "C" {

void hef_params_default(hef_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->k = 10;
  p->b = 1;
  p->levels = 1;
  p->percentile = 0.5f;
  p->local_clustering = 1;
  p->basis = HEF_BASIS_FP32;
  p->seed = 7;
  p->drop_tol = 1e-3f;
  p->orth_passes = 1;
  p->ckpt_every = 0;
  p->flags = 0;
  p->target_nr = 0.0f;
}

int32_t hef_pool_width(const hef_params *p) { return p ? pool_width(*p) : 0; }

hef_status hef_workspace_size(const hef_hypergraph *hg, const hef_params *p, int32_t op,
                              size_t *bytes) {
  HEF_TRY(check_hg(hg));
  if (!bytes) { set_error("bytes is NULL"); return HEF_ERR_INVALID_ARGUMENT; }
  const int64_t n = hg->n, m = hg->m, nnz = hg->nnz;
  switch (op) {
    case HEF_OP_RESISTANCE:
      HEF_TRY(check_params(p, false, true));
      *bytes = resistance_bytes(n, m, nnz, *p, true);
      return HEF_OK;
    case HEF_OP_COARSEN:
      HEF_TRY(check_params(p, true));
      *bytes = coarsen_bytes(n, m, nnz, *p);
      return HEF_OK;
    case HEF_OP_CLUSTER_LEVEL:
      HEF_TRY(check_params(p, true));
      *bytes = cluster_level_bytes(n, m, nnz, pool_width(*p));
      return HEF_OK;
    case HEF_OP_BACKWARD:
      HEF_TRY(check_params(p, false));
      *bytes = backward_bytes(n, m, nnz, *p);
      return HEF_OK;
    case HEF_OP_APPLY: {
      Arena a;
      Structure st;
      structure_carve(a, n, m, nnz, st);
      a.take<float>(spmm_scratch_floats(n, m, 16));
      *bytes = a.mark() + structure_build_ws(n, m, nnz) + 1024;
      return HEF_OK;
    }
    case HEF_OP_CONDUCTANCE:
      *bytes = conductance_bytes(n, m, nnz);
      return HEF_OK;
    case HEF_OP_REBUILD:
      *bytes = rebuild_call_bytes(n, m, nnz);
      return HEF_OK;
    case HEF_OP_RATING:
      *bytes = rating_bytes(n, m, nnz);
      return HEF_OK;
    default:
      set_error("unknown op %d", op);
      return HEF_ERR_INVALID_ARGUMENT;
  }
}

hef_status hef_validate_host(int32_t n, int32_t m, const int32_t *eptr, const int32_t *pins,
                             const float *w) {
  if (n < 0 || m < 0) { set_error("negative size"); return HEF_ERR_INVALID_ARGUMENT; }
  if (!eptr) { set_error("eptr is NULL"); return HEF_ERR_INVALID_ARGUMENT; }
  if (eptr[0] != 0) { set_error("eptr[0] != 0"); return HEF_ERR_INVALID_HYPERGRAPH; }
  for (int32_t e = 0; e < m; ++e) {
    const int32_t a = eptr[e], b = eptr[e + 1];
    if (b - a < 2) { set_error("hyperedge %d has %d pins (< 2)", e, b - a); return HEF_ERR_INVALID_HYPERGRAPH; }
    if (!pins) { set_error("pins is NULL"); return HEF_ERR_INVALID_ARGUMENT; }
    int32_t prev = -1;
    for (int32_t j = a; j < b; ++j) {
      const int32_t q = pins[j];
      if (q < 0 || q >= n) { set_error("pin %d of hyperedge %d out of range", q, e); return HEF_ERR_INVALID_HYPERGRAPH; }
      if (q <= prev) { set_error("pins of hyperedge %d not strictly increasing", e); return HEF_ERR_INVALID_HYPERGRAPH; }
      prev = q;
    }
    if (w && !(w[e] > 0.0f && std::isfinite(w[e]))) {
      set_error("weight of hyperedge %d is not finite and positive", e);
      return HEF_ERR_INVALID_HYPERGRAPH;
    }
  }
  return HEF_OK;
}

hef_status hef_resistance(const hef_hypergraph *hg, const hef_params *p, const float *start_star,
                          const float *start_clique, float *R, double *qh, void *chi, void *ws,
                          size_t ws_bytes, hipStream_t stream) {
  return hef::resistance_call(hg, p, start_star, start_clique, R, qh, chi, ws, ws_bytes, stream);
}

hef_status hef_resistance_static(const hef_hypergraph *hg, const hef_params *p,
                                 const float *start_star, const float *start_clique, float *R,
                                 double *qh, void *chi, hipStream_t stream) {
  HEF_TRY(check_hg(hg));
  HEF_TRY(check_params(p, false, true));
  const size_t need = resistance_bytes(hg->n, hg->m, hg->nnz, *p, chi == nullptr);
  if (need > HEF_STATIC_SCRATCH_BYTES) {
    set_error("this hypergraph needs %zu bytes of scratch; the static scratch holds %zu "
              "(use hef_resistance with a workspace)", need, size_t(HEF_STATIC_SCRATCH_BYTES));
    return HEF_ERR_WORKSPACE_TOO_SMALL;
  }
  void *ws = nullptr;
  HEF_TRY(static_scratch(&ws));
  return hef::resistance_call(hg, p, start_star, start_clique, R, qh, chi, ws,
                              HEF_STATIC_SCRATCH_BYTES, stream);
}

}  // extern "C"

namespace hef {

hef_status resistance_call(const hef_hypergraph *hg, const hef_params *p, const float *start_star,
                           const float *start_clique, float *R, double *qh, void *chi, void *ws,
                           size_t ws_bytes, hipStream_t stream) {
  HEF_TRY(check_hg(hg));
  HEF_TRY(check_params(p, false, true));
  if (!R && hg->m > 0) { set_error("R is NULL"); return HEF_ERR_INVALID_ARGUMENT; }
  if (!ws) { set_error("workspace is NULL"); return HEF_ERR_INVALID_ARGUMENT; }
  const int64_t n = hg->n, m = hg->m, nnz = hg->nnz;
  const size_t need = resistance_bytes(n, m, nnz, *p, chi == nullptr);
  if (ws_bytes < need) {
    set_error("workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    return HEF_ERR_WORKSPACE_TOO_SMALL;
  }
  const int K = pool_width(*p);
  Arena a;
  a.base = static_cast<char *>(ws);
  a.cap = ws_bytes;
  Structure st;
  structure_carve(a, n, m, nnz, st);
  int32_t *flags = a.take<int32_t>(4);
  void *pool = chi ? chi : a.take<char>(pool_bytes(n, K, p->basis));
  void *pool2 = a.take<char>(pool_bytes(oct_rows(n), K, p->basis));
  double *qh_ws = a.take<double>(K);
  float *R_ws = a.take<float>(m);
  if (a.overflow) { set_error("workspace carve overflow"); return HEF_ERR_WORKSPACE_TOO_SMALL; }
  const Level L = level_of(hg);
  const bool check = !(p->flags & HEF_FLAG_ASSUME_VALID);
  if (check) {
    int32_t bad = 0;
    HEF_TRY(validate_device(L, flags, &bad, stream));
    if (bad) {
      set_error("invalid hypergraph (code %d: 1 eptr ends, 2 segment bounds or |e|<2, 4 pins, 8 weights)", bad);
      return HEF_ERR_INVALID_HYPERGRAPH;
    }
  }
  if (n == 0 || m == 0) {
    if (qh && K) HEF_TRY(zero_async(qh, K * sizeof(double), stream));
    return HEF_OK;
  }
  HEF_TRY(estimate_level(L, *p, p->seed, 0, start_star, start_clique, st, pool, pool2, qh_ws,
                         R_ws, a, stream));
  if (check) {
    HEF_TRY(zero_async(flags, sizeof(int32_t), stream));
    k_check_finite<<<cdiv(std::max<int64_t>(m, K), 256), 256, 0, stream>>>(R_ws, m, qh_ws, K, flags);
    HEF_LAUNCH_CHECK();
    int32_t f = 0;
    HEF_HIP(hipMemcpyAsync(&f, flags, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    HEF_HIP(hipStreamSynchronize(stream));
    if ((f & 1) || !(f & 2)) {
      set_error("numerical failure: %s", (f & 1) ? "non-finite value" : "every quadratic form vanished");
      return HEF_ERR_NUMERICAL;
    }
  }
  HEF_HIP(hipMemcpyAsync(R, R_ws, m * sizeof(float), hipMemcpyDeviceToDevice, stream));
  if (qh) HEF_HIP(hipMemcpyAsync(qh, qh_ws, K * sizeof(double), hipMemcpyDeviceToDevice, stream));
  return HEF_OK;
}

}  // namespace hef

extern "C" {

hef_status hef_rating(const hef_hypergraph *hg, const float *R, float shift, int32_t *best,
                      double *rating, void *ws, size_t ws_bytes, hipStream_t stream) {
  HEF_TRY(check_hg(hg));
  if ((hg->m > 0 && !R) || (hg->n > 0 && (!best || !rating)) || !ws) {
    set_error("NULL argument");
    return HEF_ERR_INVALID_ARGUMENT;
  }
  if (!std::isfinite(shift)) {
    set_error("shift must be finite");
    return HEF_ERR_INVALID_ARGUMENT;
  }
  const size_t need = rating_bytes(hg->n, hg->m, hg->nnz);
  if (ws_bytes < need) {
    set_error("workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    return HEF_ERR_WORKSPACE_TOO_SMALL;
  }
  return rating_run(level_of(hg), R, shift, best, rating, ws, ws_bytes, stream);
}

hef_status hef_debug_apply(const hef_hypergraph *hg, int32_t expansion, int32_t b, const float *x,
                           float *y, void *ws, size_t ws_bytes, hipStream_t stream) {
  HEF_TRY(check_hg(hg));
  if (!pow2_block(b)) { set_error("b must be 1, 2, 4, 8 or 16"); return HEF_ERR_UNSUPPORTED; }
  if (expansion != 0 && expansion != 1) { set_error("expansion must be 0 or 1"); return HEF_ERR_INVALID_ARGUMENT; }
  if (!x || !y || !ws) { set_error("NULL pointer"); return HEF_ERR_INVALID_ARGUMENT; }
  size_t need = 0;
  hef_params p;
  hef_params_default(&p);
  HEF_TRY(hef_workspace_size(hg, &p, HEF_OP_APPLY, &need));
  if (ws_bytes < need) { set_error("workspace too small"); return HEF_ERR_WORKSPACE_TOO_SMALL; }
  Arena a;
  a.base = static_cast<char *>(ws);
  a.cap = ws_bytes;
  Structure st;
  structure_carve(a, hg->n, hg->m, hg->nnz, st);
  float *tb = a.take<float>(spmm_scratch_floats(hg->n, hg->m, 16));
  const Level L = level_of(hg);
  HEF_TRY(structure_build(L, st, a, stream));
  if (expansion == 0)
    return spmm_apply(L, st, b, x, y, nullptr, nullptr, tb, stream);
  return spmm_apply(L, st, b, nullptr, nullptr, x, y, tb, stream);
}

hef_status hef_debug_gram(const float *X, int64_t rows, int32_t cols, double *G, void *ws,
                          size_t ws_bytes, hipStream_t stream) {
  if (!X || !G || !ws || rows < 0 || cols <= 0 || cols > 512) {
    set_error("bad argument");
    return HEF_ERR_INVALID_ARGUMENT;
  }
  if (ws_bytes < orth_ws_bytes(rows, cols)) { set_error("workspace too small"); return HEF_ERR_WORKSPACE_TOO_SMALL; }
  Arena a;
  a.base = static_cast<char *>(ws);
  a.cap = ws_bytes;
  return gram_f32(X, rows, cols, G, a, stream);
}

size_t hef_debug_gram_ws(int64_t rows, int32_t cols) { return orth_ws_bytes(rows, cols); }

hef_status hef_start_block(uint64_t seed, int32_t level, int32_t expansion, int64_t rows,
                           int32_t b, float *out, hipStream_t stream) {
  if (!out || rows < 0 || b < 1 || b > 16 || (expansion != 0 && expansion != 1)) {
    set_error("bad argument");
    return HEF_ERR_INVALID_ARGUMENT;
  }
  return start_block(seed, level, expansion, rows, b, out, stream);
}

const char *hef_status_string(hef_status s) {
  switch (s) {
    case HEF_OK: return "ok";
    case HEF_ERR_INVALID_ARGUMENT: return "invalid argument";
    case HEF_ERR_INVALID_HYPERGRAPH: return "invalid hypergraph";
    case HEF_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case HEF_ERR_DEVICE: return "device error";
    case HEF_ERR_NUMERICAL: return "numerical failure";
    case HEF_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char *hef_last_error(void) { return hef::last_error(); }

void hef_timing_enable(int32_t on) { hef::g_timing.store(on ? 1 : 0); }
void hef_timing_stages(uint32_t mask) { hef::g_timing_mask.store(mask); }

int32_t hef_timing_stage_count(void) { return kStageCount; }

const char *hef_timing_stage_name(int32_t stage) {
  return (stage >= 0 && stage < kStageCount) ? hef::kStageNames[stage] : "";
}

hef_status hef_timing_read(double *ms, int64_t *counts, int32_t nstages, int32_t reset) {
  std::lock_guard<std::mutex> lk(hef::g_tmu);
  for (auto &t : hef::g_pending) {
    hipEvent_t a = std::get<1>(t), b = std::get<2>(t);
    float el = 0.0f;
    HEF_HIP(hipEventSynchronize(b));
    HEF_HIP(hipEventElapsedTime(&el, a, b));
    hef::g_ms[std::get<0>(t)] += el;
    hef::g_cnt[std::get<0>(t)] += 1;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  hef::g_pending.clear();
  for (int i = 0; i < nstages && i < kStageCount; ++i) {
    if (ms) ms[i] = hef::g_ms[i];
    if (counts) counts[i] = hef::g_cnt[i];
  }
  if (reset) {
    for (int i = 0; i < kStageCount; ++i) { hef::g_ms[i] = 0.0; hef::g_cnt[i] = 0; }
  }
  return HEF_OK;
}

}  // extern "C"

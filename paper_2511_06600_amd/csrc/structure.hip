// One level's structure: validation, CSC incidence, expansion scales and the
// lists of long segments (Section III-A, star and clique expansions; the
// normalised adjacency of each is applied implicitly by the SpMM kernels).
#include <cmath>

#include "prims.hpp"
#include "structure.hpp"

namespace hef {
namespace {

__global__ void k_validate(const int32_t *eptr, const int32_t *pins, const float *w,
                           int32_t n, int32_t m, int64_t nnz, int32_t *flag) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  int bad = 0;
  const int64_t a = eptr[e], b = eptr[e + 1];
  if (e == 0 && a != 0) bad |= 1;
  if (e == m - 1 && b != nnz) bad |= 1;
  if (a < 0 || b > nnz || b - a < 2) bad |= 2;
  if (!bad) {
    int32_t prev = -1;
    for (int64_t j = a; j < b; ++j) {
      const int32_t p = pins[j];
      if (p < 0 || p >= n || p <= prev) {
        bad |= 4;
        break;
      }
      prev = p;
    }
  }
  if (w) {
    const float x = w[e];
    if (!(x > 0.0f) || !isfinite(x)) bad |= 8;
  }
  if (bad) atomicOr(flag, bad);
}

__global__ void k_edge_ids(const int32_t *__restrict__ eptr, uint32_t *__restrict__ eid,
                           int32_t m) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int32_t a = eptr[e], b = eptr[e + 1];
  for (int32_t j = a; j < b; ++j) eid[j] = uint32_t(e);
}

// vptr[v] = first position of a key >= v in the sorted pin keys (v <= n):
// position j writes the nodes in (key[j-1], key[j]] (key[-1] = -1,
// key[nnz] = n).
__global__ void k_seg_bounds(const uint32_t *__restrict__ key, int64_t nnz, int32_t n,
                             int32_t *__restrict__ vptr) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j > nnz) return;
  const int64_t cur = j < nnz ? int64_t(key[j]) : int64_t(n);
  const int64_t prev = j > 0 ? int64_t(key[j - 1]) : -1;
  for (int64_t v = prev + 1; v <= cur; ++v) vptr[v] = int32_t(j);
}

__global__ void k_copy_pins(const int32_t *pins, uint32_t *keys, int64_t nnz) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j < nnz) keys[j] = uint32_t(pins[j]);
}

// Per hyperedge: alpha_e = sqrt(w_e)/|e|, beta_e = w_e/(|e|(|e|-1)); flag
// big; the float64 terms w_e/|e| and beta_e of the node sums.
__global__ void k_edge_scales(const int32_t *__restrict__ eptr, const float *__restrict__ w,
                              float *__restrict__ alpha, float *__restrict__ beta,
                              int32_t *__restrict__ big, double *__restrict__ tdb,
                              double *__restrict__ tcb, int32_t m) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int32_t sz = eptr[e + 1] - eptr[e];
  const double we = w ? double(w[e]) : 1.0;
  const double k = double(sz);
  alpha[e] = float(sqrt(we) / k);
  beta[e] = float(we / (k * (k - 1.0)));
  big[e] = sz > kSmallSeg ? 1 : 0;
  tdb[e] = we / k;
  tcb[e] = we / (k * (k - 1.0));
}

// Per node, over its hyperedges in ascending order, in float64:
// d_b = sum w_e/|e|, cb = sum beta_e; s = d_b^-1/2, gam = s^2 cb.
__global__ void k_node_scales(const int32_t *__restrict__ vptr, const int32_t *__restrict__ eids,
                              const double *__restrict__ tdb, const double *__restrict__ tcb,
                              float *__restrict__ s_out, float *__restrict__ gam,
                              int32_t *__restrict__ big, int32_t n) {
  const int64_t u = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (u >= n) return;
  double db = 0.0, cb = 0.0;
  const int32_t a = vptr[u], b = vptr[u + 1];
  // Incidence ids are loaded four at a time before the dependent loads, and
  // the terms are added in incidence order.
  int32_t j = a;
  for (; j + 4 <= b; j += 4) {
    int32_t e[4];
    double td[4], tc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) e[q] = eids[j + q];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      td[q] = tdb[e[q]];
      tc[q] = tcb[e[q]];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      db += td[q];
      cb += tc[q];
    }
  }
  for (; j < b; ++j) {
    const int32_t e = eids[j];
    db += tdb[e];
    cb += tcb[e];
  }
  const double sv = db > 0.0 ? 1.0 / sqrt(db) : 0.0;
  s_out[u] = float(sv);
  gam[u] = float(sv * sv * cb);
  big[u] = (b - a) > kSmallSeg ? 1 : 0;
}

}  // namespace

void structure_carve(Arena &a, int64_t n, int64_t m, int64_t nnz, Structure &st) {
  st.vptr = a.take<int32_t>(n + 1);
  st.eids = a.take<int32_t>(nnz);
  st.s = a.take<float>(n);
  st.gam = a.take<float>(n);
  st.alpha = a.take<float>(m);
  st.beta = a.take<float>(m);
  st.big_e = a.take<int32_t>(m + 1);
  st.big_v = a.take<int32_t>(n + 1);
  st.n_big = a.take<int32_t>(2);
}

size_t structure_build_ws(int64_t n, int64_t m, int64_t nnz) {
  Arena a;
  a.take<uint32_t>(nnz);  // keys
  a.take<uint32_t>(nnz);  // vals
  a.take<uint32_t>(nnz);  // keys out
  a.take<int32_t>(std::max(n, m) + 1);  // flags
  a.take<int32_t>(std::max(n, m) + 1);  // compaction scratch
  a.take<double>(std::max<int64_t>(m, 1));  // per-edge node-sum terms
  a.take<double>(std::max<int64_t>(m, 1));
  return a.mark() + radix_ws_bytes(nnz) + scan_ws_bytes(std::max(n, m) + 1) + 4096;
}

hef_status validate_device(const Level &L, int32_t *flag_dev, int32_t *bad_host,
                           hipStream_t s) {
  HEF_TRY(zero_async(flag_dev, sizeof(int32_t), s));
  if (L.m > 0)
    k_validate<<<cdiv(L.m, 256), 256, 0, s>>>(L.eptr, L.pins, L.w, L.n, L.m, L.nnz, flag_dev);
  HEF_LAUNCH_CHECK();
  HEF_HIP(hipMemcpyAsync(bad_host, flag_dev, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HEF_HIP(hipStreamSynchronize(s));
  return HEF_OK;
}

hef_status structure_build(const Level &L, Structure &st, Arena &ws, hipStream_t s) {
  const int64_t n = L.n, m = L.m, nnz = L.nnz;
  TimedScope ts(kStStructure, s);
  const size_t mk = ws.mark();
  uint32_t *keys = ws.take<uint32_t>(nnz);
  uint32_t *vals = ws.take<uint32_t>(nnz);
  uint32_t *keys_out = ws.take<uint32_t>(nnz);
  int32_t *flags = ws.take<int32_t>(std::max(n, m) + 1);
  int32_t *scratch = ws.take<int32_t>(std::max(n, m) + 1);
  double *tdb = ws.take<double>(std::max<int64_t>(m, 1));
  double *tcb = ws.take<double>(std::max<int64_t>(m, 1));
  HEF_WS_CHECK(ws);

  // eids: stable sort of (pin, edge) by pin; input is in edge order, so
  // each node's hyperedges come out ascending.  vptr from the sorted pins.
  if (nnz > 0) {
    k_copy_pins<<<cdiv(nnz, 256), 256, 0, s>>>(L.pins, keys, nnz);
    k_edge_ids<<<cdiv(m, 256), 256, 0, s>>>(L.eptr, vals, int32_t(m));
    HEF_LAUNCH_CHECK();
    HEF_TRY(radix_sort_pairs(keys, vals, keys_out, reinterpret_cast<uint32_t *>(st.eids),
                             nnz, bits_for(n > 0 ? n - 1 : 0), ws, s));
    k_seg_bounds<<<cdiv(nnz + 1, 256), 256, 0, s>>>(keys_out, nnz, int32_t(n), st.vptr);
    HEF_LAUNCH_CHECK();
  } else {
    HEF_TRY(zero_async(st.vptr, (n + 1) * sizeof(int32_t), s));
  }

  // scales and big-segment lists
  if (m > 0) {
    k_edge_scales<<<cdiv(m, 256), 256, 0, s>>>(L.eptr, L.w, st.alpha, st.beta, flags, tdb, tcb,
                                               int32_t(m));
    HEF_LAUNCH_CHECK();
  }
  HEF_TRY(compact_flags(flags, scratch, st.big_e, st.n_big, m, ws, s));
  if (n > 0) {
    k_node_scales<<<cdiv(n, 256), 256, 0, s>>>(st.vptr, st.eids, tdb, tcb, st.s, st.gam,
                                              flags, int32_t(n));
    HEF_LAUNCH_CHECK();
  }
  HEF_TRY(compact_flags(flags, scratch, st.big_v, st.n_big + 1, n, ws, s));
  ws.reset(mk);
  return HEF_OK;
}

}  // namespace hef

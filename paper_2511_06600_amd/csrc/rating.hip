// Resistance-based vertex-pair rating (Section III-E, Eq. (17)): for every
// node p and every node q sharing a hyperedge with it,
//   r(p, q) = sum over hyperedges e holding both of  w(e) / (R_e - shift),
// the rating function of Eq. (7) with the hyperedge cardinality term
// replaced by the effective resistance R_e.  Reading of the printed
// denominator: with shift = 0 the whole cardinality term |e| - 1 of Eq. (7)
// becomes R_e, so heavy hyperedges of low resistance rate high, as the text
// asks; shift = 1 gives the printed R_e - 1 literally (negative for every
// hyperedge with w(e) >= 1, since R_e <= 1/w(e)).  A hyperedge whose
// denominator is exactly 0 adds nothing.  Output per node: the neighbour of
// largest rating (ties to the smallest id) and that rating, or -1 and 0 for
// a node without neighbours.
//
// Layout (deterministic: no floating-point atomics, every sum in ascending
// hyperedge order):
//  1. bound(p) = sum over the hyperedges of p of (|e| - 1), the number of
//     (p, q, e) triples of p; the nodes are cut into batches whose bounds
//     sum to at most max(nnz, 2^20) triples (one node never exceeds nnz);
//  2. per batch, one wave per node emits its triples with e ascending and,
//     within e, q ascending;
//  3. a stable sort by q, then a stable sort by p, puts each (p, q) run in
//     ascending e;
//  4. one thread per node sums its runs in float64 and keeps the largest.
#include <cfloat>
#include <cmath>
#include <vector>

#include "prims.hpp"
#include "rating.hpp"
#include "structure.hpp"

namespace hef {
namespace {

constexpr int kRT = 256;

__global__ void k_rate_bound(const int32_t *__restrict__ vptr, const int32_t *__restrict__ eids,
                             const int32_t *__restrict__ eptr, int32_t n,
                             int32_t *__restrict__ bound) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int64_t b = 0;
  for (int32_t t = vptr[p]; t < vptr[p + 1]; ++t) {
    const int32_t e = eids[t];
    b += eptr[e + 1] - eptr[e] - 1;
  }
  bound[p] = int32_t(b);  // <= nnz - 1 (every triple of p is a distinct pin position)
}

// flag |= 1 if an R value is not finite
__global__ void k_rate_check(const float *__restrict__ R, int64_t m, int32_t *__restrict__ flag) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < m && !isfinite(R[e])) atomicOr(flag, 1);
}

// One wave per node p of the batch [p0, p0 + nb): its triples (q, p - p0, e)
// at off[p - p0] + running index, e ascending, q ascending within e.
__global__ void __launch_bounds__(kRT)
k_rate_emit(const int32_t *__restrict__ vptr, const int32_t *__restrict__ eids,
            const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins, int32_t p0,
            int32_t nb, const int32_t *__restrict__ off, uint32_t *__restrict__ kq,
            uint32_t *__restrict__ vj, uint32_t *__restrict__ pl, int32_t *__restrict__ ee) {
  const int64_t i = int64_t(blockIdx.x) * (kRT / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= nb) return;
  const int32_t p = p0 + int32_t(i);
  int32_t o = off[i];
  for (int32_t t = vptr[p]; t < vptr[p + 1]; ++t) {
    const int32_t e = eids[t];
    const int32_t a = eptr[e], b = eptr[e + 1];
    for (int32_t j0 = a; j0 < b; j0 += 64) {
      const int32_t j = j0 + lane;
      const int32_t q = j < b ? pins[j] : p;
      const bool take = q != p;
      const uint64_t mask = __ballot(take);
      const int32_t pos = __popcll(mask & ((uint64_t(1) << lane) - 1));
      if (take) {
        const int32_t k = o + pos;
        kq[k] = uint32_t(q);
        vj[k] = uint32_t(k);
        pl[k] = uint32_t(i);
        ee[k] = e;
      }
      o += __popcll(mask);
    }
  }
}

__global__ void k_rate_pkeys(const uint32_t *__restrict__ order, const uint32_t *__restrict__ pl,
                             uint32_t *__restrict__ kp, uint32_t *__restrict__ vp, int64_t cnt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const uint32_t j = order[i];
  kp[i] = pl[j];
  vp[i] = j;
}

// One thread per node of the batch: its triples sit at [off[i], off[i+1]) in
// (q, e) order; every run of one q is summed in float64, e ascending.
__global__ void k_rate_best(const int32_t *__restrict__ off, const uint32_t *__restrict__ order,
                            const uint32_t *__restrict__ kq, const int32_t *__restrict__ ee,
                            const float *__restrict__ w, const float *__restrict__ R,
                            double shift, int32_t p0, int32_t nb, int32_t *__restrict__ best,
                            double *__restrict__ rating) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  int32_t bq = -1;
  double br = 0.0;
  int32_t cq = -1;
  double acc = 0.0;
  for (int32_t k = off[i]; k < off[i + 1]; ++k) {
    const uint32_t j = order[k];
    const int32_t q = int32_t(kq[j]);
    const int32_t e = ee[j];
    if (q != cq) {
      if (cq >= 0 && (bq < 0 || acc > br)) { bq = cq; br = acc; }
      cq = q;
      acc = 0.0;
    }
    const double den = double(R[e]) - shift;
    if (den != 0.0) acc += double(w ? w[e] : 1.0f) / den;
  }
  if (cq >= 0 && (bq < 0 || acc > br)) { bq = cq; br = acc; }
  best[p0 + i] = bq;
  rating[p0 + i] = bq < 0 ? 0.0 : br;
}

__global__ void k_rate_scatter(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ idx,
                               uint32_t *__restrict__ out, int64_t cnt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < cnt) out[idx[i]] = keys[i];
}

inline unsigned gr(int64_t n) { return unsigned(std::max<int64_t>(1, cdiv(n, kRT))); }

int64_t rating_cap(int64_t nnz) { return std::max<int64_t>(nnz, int64_t(1) << 20); }

}  // namespace

size_t rating_bytes(int64_t n, int64_t m, int64_t nnz) {
  const int64_t cap = rating_cap(nnz);
  Arena a;
  Structure st;
  structure_carve(a, n, m, nnz, st);
  a.take<int32_t>(4);
  a.take<int32_t>(n + 1);  // bound
  a.take<int32_t>(n + 2);  // batch offsets
  for (int i = 0; i < 7; ++i) a.take<uint32_t>(cap);
  const size_t scratch = std::max(structure_build_ws(n, m, nnz),
                                  radix_ws_bytes(cap) + scan_ws_bytes(n + 1) + 4096);
  return a.mark() + scratch + 4096;
}

hef_status rating_run(const Level &L, const float *R, float shift, int32_t *best, double *rating,
                      void *ws, size_t ws_bytes, hipStream_t s) {
  const int64_t n = L.n, m = L.m, nnz = L.nnz;
  const int64_t cap = rating_cap(nnz);
  Arena a;
  a.base = static_cast<char *>(ws);
  a.cap = ws_bytes;
  Structure st;
  structure_carve(a, n, m, nnz, st);
  int32_t *flags = a.take<int32_t>(4);
  int32_t *bound = a.take<int32_t>(n + 1);
  int32_t *off = a.take<int32_t>(n + 2);
  uint32_t *kq = a.take<uint32_t>(cap), *vj = a.take<uint32_t>(cap), *pl = a.take<uint32_t>(cap);
  int32_t *ee = reinterpret_cast<int32_t *>(a.take<uint32_t>(cap));
  uint32_t *k1 = a.take<uint32_t>(cap), *v1 = a.take<uint32_t>(cap), *k2 = a.take<uint32_t>(cap);
  HEF_WS_CHECK(a);
  int32_t bad = 0;
  HEF_TRY(validate_device(L, flags, &bad, s));
  if (bad) {
    set_error("invalid hypergraph (code %d)", bad);
    return HEF_ERR_INVALID_HYPERGRAPH;
  }
  if (m > 0) {
    HEF_TRY(zero_async(flags, sizeof(int32_t), s));
    k_rate_check<<<gr(m), kRT, 0, s>>>(R, m, flags);
    HEF_LAUNCH_CHECK();
    int32_t f = 0;
    HEF_HIP(hipMemcpyAsync(&f, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HEF_HIP(hipStreamSynchronize(s));
    if (f) {
      set_error("a resistance is not finite");
      return HEF_ERR_INVALID_ARGUMENT;
    }
  }
  if (n == 0) return HEF_OK;
  TimedScope ts(kStRating, s);
  HEF_TRY(structure_build(L, st, a, s));
  k_rate_bound<<<gr(n), kRT, 0, s>>>(st.vptr, st.eids, L.eptr, int32_t(n), bound);
  HEF_LAUNCH_CHECK();
  std::vector<int32_t> hb(n);
  HEF_HIP(hipMemcpyAsync(hb.data(), bound, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
  HEF_HIP(hipStreamSynchronize(s));
  const double sh = double(shift);
  for (int64_t p0 = 0; p0 < n;) {
    // the batch [p0, p1): as many nodes as fit in cap triples
    int64_t p1 = p0, tot = 0;
    while (p1 < n && tot + hb[p1] <= cap) tot += hb[p1++];
    const int32_t nb = int32_t(p1 - p0);
    HEF_TRY(exclusive_scan_i32(bound + p0, off, nb, a, s));
    k_rate_emit<<<unsigned(cdiv(nb, kRT / 64)), kRT, 0, s>>>(st.vptr, st.eids, L.eptr, L.pins,
                                                            int32_t(p0), nb, off, kq, vj, pl, ee);
    HEF_LAUNCH_CHECK();
    const uint32_t *order = vj;
    if (tot > 0) {
      // by q (stable, so e stays ascending within a q), then by node
      HEF_TRY(radix_sort_pairs(kq, vj, k1, v1, tot, bits_for(n - 1), a, s));
      // the sort clobbered kq and vj: the q values are in k1 (sorted) with
      // their emission indices in v1; node keys in q order go to k2, and kq
      // is rebuilt by emission index
      k_rate_pkeys<<<gr(tot), kRT, 0, s>>>(v1, pl, k2, vj, tot);
      HEF_LAUNCH_CHECK();
      k_rate_scatter<<<gr(tot), kRT, 0, s>>>(k1, v1, kq, tot);
      HEF_LAUNCH_CHECK();
      HEF_TRY(radix_sort_pairs(k2, vj, k1, v1, tot, bits_for(std::max<int64_t>(nb - 1, 1)), a, s));
      order = v1;
    }
    k_rate_best<<<gr(nb), kRT, 0, s>>>(off, order, kq, ee, L.w, R, sh, int32_t(p0), nb, best,
                                       rating);
    HEF_LAUNCH_CHECK();
    HEF_HIP(hipStreamSynchronize(s));  // the batch buffers are reused
    p0 = p1;
  }
  return HEF_OK;
}

}  // namespace hef

// Cluster quality: the conductance of every cluster of a partition
// (Section II-A, Eq. (3)) and the clusters' average (Eq. (18)).
//
// Readings: the cut of a cluster counts each hyperedge with pins inside and
// outside it once, with its weight; a cluster whose cut is zero has
// conductance 0 (this covers the 0/0 cases of a cluster of nodes without
// hyperedges and of a single cluster holding every node); sums are float64.
//
// Layout of the computation (deterministic: no atomics, fixed summation
// order):
//  1. every pin position j of a hyperedge e emits (label of its node, e),
//     in pin order;
//  2. a stable radix sort by label groups each cluster's pins with e
//     ascending, so the pins a hyperedge has in one cluster are adjacent;
//  3. one wave per cluster walks its pins: each adds w(e) to the volume
//     (sum over the cluster's nodes of their degrees), and the first pin of
//     each run of one hyperedge adds w(e) to the cut when e is split;
//  4. the volume total, phi and the average come from fixed-order
//     two-stage sums over up to 256 workgroups.
#include <cfloat>
#include <cstdint>

#include "prims.hpp"
#include "quality.hpp"
#include "structure.hpp"

namespace hef {
namespace {

constexpr int kQT = 256;

// The hyperedge holding pin position j: the last e with eptr[e] <= j.
__device__ __forceinline__ int32_t edge_of(const int32_t *eptr, int32_t m, int32_t j) {
  int32_t lo = 0, hi = m;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (eptr[mid] <= j) lo = mid; else hi = mid;
  }
  return lo;
}

// One thread per pin position j, kQT consecutive positions per workgroup:
// j emits (label of its node, its hyperedge e), and marks split[e] (zeroed
// beforehand) when its label differs from that of e's first pin.  The
// workgroup finds the hyperedges of its first and last positions once and
// stages that slice of eptr in LDS (at most kQT + 1 entries, as every
// hyperedge has a pin), where each thread finds its own hyperedge.
__global__ void __launch_bounds__(kQT)
k_qual_emit(const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins,
            const int32_t *__restrict__ label, int32_t m, int64_t nnz, int32_t nc,
            uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
            int32_t *__restrict__ split, int32_t *__restrict__ bad) {
  __shared__ int32_t se[kQT + 2];
  __shared__ int32_t ends[2];
  const int64_t j0 = int64_t(blockIdx.x) * kQT;
  const int64_t jl = (j0 + kQT < nnz ? j0 + kQT : nnz) - 1;
  if (threadIdx.x < 2) ends[threadIdx.x] = edge_of(eptr, m, int32_t(threadIdx.x ? jl : j0));
  __syncthreads();
  const int32_t e0 = ends[0];
  int32_t ne = ends[1] - e0;  // entries e0 .. e0 + ne
  if (ne > kQT) ne = kQT;
  for (int i = threadIdx.x; i <= ne; i += kQT) se[i] = eptr[e0 + i];
  __syncthreads();
  const int64_t j = j0 + threadIdx.x;
  if (j > jl) return;
  int32_t lo = 0, hi = ne + 1;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (se[mid] <= j) lo = mid; else hi = mid;
  }
  const int32_t e = e0 + lo;
  int32_t c = label[pins[j]];
  int32_t cf = label[pins[se[lo]]];
  if (cf < 0 || cf >= nc) cf = 0;
  if (c < 0 || c >= nc) {
    *bad = 1;  // every writer stores the same value
    c = 0;
  }
  keys[j] = uint32_t(c);
  vals[j] = uint32_t(e);
  if (c != cf) split[e] = 1;  // every writer stores the same value
}

// seg[c] = first sorted position with key >= c, c in [0, nc]
__global__ void k_qual_seg(const uint32_t *__restrict__ keys, int64_t nnz, int32_t nc,
                           int32_t *__restrict__ seg) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c > nc) return;
  int64_t lo = 0, hi = nnz;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (int64_t(keys[mid]) < c) lo = mid + 1; else hi = mid;
  }
  seg[c] = int32_t(lo);
}

// One wave per cluster: lane l takes the cluster's sorted pins l, l+64, ...;
// the lane sums are combined by a fixed butterfly.
__global__ void __launch_bounds__(kQT)
k_qual_cluster(const float *__restrict__ w, const uint32_t *__restrict__ vals, const int32_t *__restrict__ seg,
               const int32_t *__restrict__ split, int32_t nc, double *__restrict__ cut,
               double *__restrict__ vol) {
  const int64_t c = (int64_t(blockIdx.x) * kQT + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (c >= nc) return;
  const int32_t s0 = seg[c], s1 = seg[c + 1];
  double cs = 0.0, vs = 0.0;
  int32_t carry = -1;  // hyperedge of the pin before this chunk
  for (int32_t t0 = s0; t0 < s1; t0 += 64) {
    const int32_t t = t0 + lane;
    const int32_t e = t < s1 ? int32_t(vals[t]) : -1;
    int32_t pe = __shfl_up(e, 1, 64);
    if (lane == 0) pe = carry;
    carry = __shfl(e, 63, 64);
    if (t < s1) {
      const double we = w ? double(w[e]) : 1.0;
      vs += we;
      if (e != pe && split[e]) cs += we;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    cs += __shfl_xor(cs, off, 64);
    vs += __shfl_xor(vs, off, 64);
  }
  if (lane == 0) {
    cut[c] = cs;
    vol[c] = vs;
  }
}

// Fixed-order float64 sums over many workgroups: workgroup b of nbk takes
// the chunk [b ch, (b + 1) ch) of the ch = ceil(n / nbk) items, each thread
// every kQT-th item of it, then an LDS tree; a single workgroup then adds
// the nbk partials the same way.  nbk depends on n only.
constexpr int kSumBlocks = 256;

inline int sum_blocks(int64_t n) {
  const int64_t b = cdiv(n, 1024);
  return int(b < 1 ? 1 : (b > kSumBlocks ? kSumBlocks : b));
}

__device__ __forceinline__ double block_sum(double x, double *sh) {
  sh[threadIdx.x] = x;
  __syncthreads();
  for (int h = kQT / 2; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  return sh[0];
}

__global__ void __launch_bounds__(kQT)
k_sum_part(const double *__restrict__ in, int64_t n, double *__restrict__ part) {
  __shared__ double sh[kQT];
  const int64_t ch = (n + gridDim.x - 1) / gridDim.x;
  const int64_t a = int64_t(blockIdx.x) * ch, b = a + ch < n ? a + ch : n;
  double x = 0.0;
  for (int64_t i = a + threadIdx.x; i < b; i += kQT) x += in[i];
  x = block_sum(x, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = x;
}

// *out = (sum of part[0 .. nbk)) / div
__global__ void __launch_bounds__(kQT)
k_sum_final(const double *__restrict__ part, int nbk, double div, double *__restrict__ out) {
  __shared__ double sh[kQT];
  double x = 0.0;
  for (int i = threadIdx.x; i < nbk; i += kQT) x += part[i];
  x = block_sum(x, sh);
  if (threadIdx.x == 0) *out = x / div;
}

// phi of each cluster, and the workgroup partial sums of phi (the chunks of
// k_sum_part)
__global__ void __launch_bounds__(kQT)
k_qual_phi(const double *__restrict__ cut, const double *__restrict__ vol,
           const double *__restrict__ total, int64_t nc, double *__restrict__ phi,
           double *__restrict__ part) {
  __shared__ double sh[kQT];
  const int64_t ch = (nc + gridDim.x - 1) / gridDim.x;
  const int64_t a = int64_t(blockIdx.x) * ch, b = a + ch < nc ? a + ch : nc;
  const double tv = *total;
  double x = 0.0;
  for (int64_t c = a + threadIdx.x; c < b; c += kQT) {
    const double k = cut[c];
    const double f = k != 0.0 ? k / fmin(vol[c], tv - vol[c]) : 0.0;
    phi[c] = f;
    x += f;
  }
  x = block_sum(x, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = x;
}

__global__ void k_qual_zero(double *__restrict__ a, double *__restrict__ b,
                            double *__restrict__ c, double *__restrict__ avg, int32_t nc) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < nc) {
    a[i] = 0.0;
    b[i] = 0.0;
    c[i] = 0.0;
  }
  if (i == 0) *avg = 0.0;
}

struct QualWs {
  uint32_t *k0, *v0, *k1, *v1;
  int32_t *split, *seg, *bad;
  double *tot, *part;
};

void qual_carve(Arena &a, int64_t n, int64_t m, int64_t nnz, QualWs &q) {
  q.k0 = a.take<uint32_t>(nnz);
  q.v0 = a.take<uint32_t>(nnz);
  q.k1 = a.take<uint32_t>(nnz);
  q.v1 = a.take<uint32_t>(nnz);
  q.split = a.take<int32_t>(m);
  q.seg = a.take<int32_t>((n > 1 ? n : 1) + 1);
  q.bad = a.take<int32_t>(1);
  q.tot = a.take<double>(1);
  q.part = a.take<double>(kSumBlocks);
}

}  // namespace

size_t conductance_bytes(int64_t n, int64_t m, int64_t nnz) {
  Arena a;
  QualWs q;
  qual_carve(a, n, m, nnz, q);
  return a.mark() + radix_ws_bytes(nnz) + 1024;
}

}  // namespace hef

using namespace hef;

extern "C" hef_status hef_conductance(const hef_hypergraph *hg, const int32_t *label,
                                      int32_t n_clusters, double *cut, double *vol, double *phi,
                                      double *phi_avg, void *ws, size_t ws_bytes,
                                      hipStream_t stream) {
  size_t need = 0;
  HEF_TRY(hef_workspace_size(hg, nullptr, HEF_OP_CONDUCTANCE, &need));
  const int64_t n = hg->n, m = hg->m, nnz = hg->nnz;
  if (n_clusters < 1 || int64_t(n_clusters) > (n > 1 ? n : 1)) {
    set_error("n_clusters=%d must lie in [1, max(n, 1)]", n_clusters);
    return HEF_ERR_INVALID_ARGUMENT;
  }
  if ((n > 0 && !label) || !cut || !vol || !phi || !phi_avg || !ws) {
    set_error("NULL pointer");
    return HEF_ERR_INVALID_ARGUMENT;
  }
  if (ws_bytes < need) {
    set_error("workspace too small (%zu < %zu)", ws_bytes, need);
    return HEF_ERR_WORKSPACE_TOO_SMALL;
  }
  Arena a;
  a.base = static_cast<char *>(ws);
  a.cap = ws_bytes;
  QualWs q;
  qual_carve(a, n, m, nnz, q);
  if (a.overflow) { set_error("workspace carve overflow"); return HEF_ERR_WORKSPACE_TOO_SMALL; }
  Level L;
  L.n = hg->n; L.m = hg->m; L.nnz = hg->nnz; L.eptr = hg->eptr; L.pins = hg->pins; L.w = hg->w;
  int32_t bad = 0;
  HEF_TRY(validate_device(L, q.bad, &bad, stream));
  if (bad) {
    set_error("invalid hypergraph (code %d: 1 eptr ends, 2 segment bounds or |e|<2, 4 pins, 8 weights)", bad);
    return HEF_ERR_INVALID_HYPERGRAPH;
  }
  const int32_t nc = n_clusters;
  TimedScope ts(kStQuality, stream);
  if (m == 0 || nnz == 0) {
    k_qual_zero<<<cdiv(nc, kQT), kQT, 0, stream>>>(cut, vol, phi, phi_avg, nc);
    HEF_LAUNCH_CHECK();
    HEF_HIP(hipStreamSynchronize(stream));
    return HEF_OK;
  }
  HEF_TRY(zero_async(q.bad, sizeof(int32_t), stream));
  HEF_TRY(zero_async(q.split, m * sizeof(int32_t), stream));
  k_qual_emit<<<cdiv(nnz, kQT), kQT, 0, stream>>>(L.eptr, L.pins, label, int32_t(m), nnz, nc,
                                                   q.k0, q.v0, q.split, q.bad);
  HEF_LAUNCH_CHECK();
  HEF_TRY(radix_sort_pairs(q.k0, q.v0, q.k1, q.v1, nnz, bits_for(nc - 1), a, stream));
  k_qual_seg<<<cdiv(int64_t(nc) + 1, kQT), kQT, 0, stream>>>(q.k1, nnz, nc, q.seg);
  HEF_LAUNCH_CHECK();
  k_qual_cluster<<<cdiv(int64_t(nc) * 64, kQT), kQT, 0, stream>>>(L.w, q.v1, q.seg, q.split, nc,
                                                                 cut, vol);
  HEF_LAUNCH_CHECK();
  const int nbk = sum_blocks(nc);
  k_sum_part<<<nbk, kQT, 0, stream>>>(vol, nc, q.part);
  HEF_LAUNCH_CHECK();
  k_sum_final<<<1, kQT, 0, stream>>>(q.part, nbk, 1.0, q.tot);
  HEF_LAUNCH_CHECK();
  k_qual_phi<<<nbk, kQT, 0, stream>>>(cut, vol, q.tot, nc, phi, q.part);
  HEF_LAUNCH_CHECK();
  k_sum_final<<<1, kQT, 0, stream>>>(q.part, nbk, double(nc), phi_avg);
  HEF_LAUNCH_CHECK();
  int32_t badlab = 0;
  HEF_HIP(hipMemcpyAsync(&badlab, q.bad, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  HEF_HIP(hipStreamSynchronize(stream));
  if (badlab) {
    set_error("a label lies outside [0, n_clusters)");
    return HEF_ERR_INVALID_ARGUMENT;
  }
  return HEF_OK;
}

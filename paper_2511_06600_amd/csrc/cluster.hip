// One level of Alg. 2 (steps 4-10) and the level loop.
//
// Section III-A "Multilevel Effective Resistance Clustering" and Eq. (15);
// Alg. 1 and Alg. 2 (contraction from the lowest resistance);
// Section III-B and Eq. (16) (resistance-based local clustering).  Readings
// of the points the paper leaves open (all chosen so that the result is one
// well-defined function of the inputs):
//  * Eq. (15): eta is summed over the pins in CSR order in float64, R_e is
//    added, and the sum is rounded to float32;
//  * delta = the ceil(pi*m)-th smallest updated resistance; contraction needs
//    R_upd < delta;
//  * contraction = the sequential greedy in ascending (R_upd, e) order that
//    contracts a hyperedge whose pins are all still free.  The device runs
//    it as rounds of "an undecided candidate wins when it holds the smallest
//    rank on every one of its pins"; the winners of a round are pairwise
//    disjoint and every hyperedge they block ranks after them, so the result
//    is the sequential one;
//  * an isolated node (untouched by the contraction, with at least one
//    hyperedge) measures d(p, C) = max_i (chi_p^(i) - c_C^(i))^2 / Q_H^(i)
//    (the numerator of Eq. (13) against the mean chi-vector of cluster C,
//    in resistance units, float64, columns with Q_H > 0) to every cluster
//    met through its hyperedges, and picks the smallest (ties: smallest
//    label).  All picks are applied together: the merged groups are the
//    connected components of the pairs {p, best(p)};
//  * eta of a merged group = float64 sum of its clusters' eta in ascending
//    label order, then of the distances of its distinct attach pairs in
//    ascending (min, max) order, rounded to float32;
//  * labels are ranks of each cluster's smallest node id;
//  * the coarse hypergraph keeps, in order, every hyperedge that still spans
//    two or more clusters, with its weight.
// Floating-point expressions in this file are compiled without contraction
// so that they round exactly as written.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <vector>

#include "cluster.hpp"
#include "krylov.hpp"
#include "prims.hpp"

#pragma clang fp contract(off)

namespace hef {
namespace {

constexpr int kT = 256;
constexpr int kSeedSeg = 64;  // hyperedges this short seed the best-first search
constexpr int kRoundsPerSync = 4;
constexpr int32_t kStUndecided = 0, kStIn = 1, kStOut = 2, kStNone = 3;

// ---- a6: Eq. (15) -----------------------------------------------------------
__global__ void k_eta_update(const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins,
                             const float *__restrict__ R, const float *__restrict__ eta,
                             float *__restrict__ R_upd, uint32_t *__restrict__ keys,
                             uint32_t *__restrict__ vals, int32_t m) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  double acc = 0.0;
  if (eta) {
    const int32_t a = eptr[e], b = eptr[e + 1];
    // pins loaded four at a time ahead of the dependent loads; the terms are
    // added in pin order
    int32_t j = a;
    for (; j + 4 <= b; j += 4) {
      int32_t p[4];
      float t[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) p[q] = pins[j + q];
#pragma unroll
      for (int q = 0; q < 4; ++q) t[q] = eta[p[q]];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc = acc + double(t[q]);
    }
    for (; j < b; ++j) acc = acc + double(eta[pins[j]]);
  }
  const float r = float(acc + double(R[e]));
  R_upd[e] = r;
  keys[e] = __float_as_uint(r);  // r >= 0: bit order = numeric order
  vals[e] = uint32_t(e);
}

// rank of every hyperedge in (R_upd, e) order; candidates have R_upd < delta
__global__ void k_rank(const uint32_t *__restrict__ order, const float *__restrict__ R_upd,
                       int32_t m, int64_t delta_pos, int32_t *__restrict__ rank,
                       int32_t *__restrict__ state, float *__restrict__ delta_out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const float delta = R_upd[order[delta_pos]];
  const int32_t e = int32_t(order[i]);
  rank[e] = int32_t(i);
  state[e] = R_upd[e] < delta ? kStUndecided : kStNone;
  if (i == 0) *delta_out = delta;
}

// ---- a7: contraction rounds --------------------------------------------------
// packed[p] = max over undecided candidates e ∋ p of (round << 32 | ~rank[e])
// = the newest round's smallest rank.  First checks whether e is blocked.
// `undecided` becomes nonzero while candidates remain: a plain store of 1 by
// one lane per wave (a same-address counter updated by every wave serialises
// at the memory side and dominated the round).
__global__ void k_round_propose(const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins,
                                const int32_t *__restrict__ rank, int32_t *__restrict__ state,
                                const int32_t *__restrict__ owner,
                                unsigned long long *__restrict__ packed, uint32_t round,
                                int32_t m, int32_t *__restrict__ undecided) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m || state[e] != kStUndecided) return;
  const int32_t a = eptr[e], b = eptr[e + 1];
  for (int32_t j = a; j < b; ++j)
    if (owner[pins[j]] >= 0) {
      state[e] = kStOut;
      return;
    }
  const unsigned long long key =
      (static_cast<unsigned long long>(round) << 32) | uint32_t(~uint32_t(rank[e]));
  for (int32_t j = a; j < b; ++j) atomicMax(&packed[pins[j]], key);
  const uint64_t act = __ballot(1);
  if ((threadIdx.x & 63) == __ffsll(static_cast<long long>(act)) - 1) *undecided = 1;
}

__global__ void k_round_select(const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins,
                               const int32_t *__restrict__ rank, int32_t *__restrict__ state,
                               int32_t *__restrict__ owner,
                               const unsigned long long *__restrict__ packed, uint32_t round,
                               int32_t m) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m || state[e] != kStUndecided) return;
  const unsigned long long key =
      (static_cast<unsigned long long>(round) << 32) | uint32_t(~uint32_t(rank[e]));
  const int32_t a = eptr[e], b = eptr[e + 1];
  for (int32_t j = a; j < b; ++j)
    if (packed[pins[j]] != key) return;
  state[e] = kStIn;
  for (int32_t j = a; j < b; ++j) owner[pins[j]] = int32_t(e);
}

// provisional cluster of every node (its smallest member), eta of clusters,
// singleton flags, and the compact index of contracted hyperedges
__global__ void k_provisional(const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins,
                              const int32_t *__restrict__ owner, const float *__restrict__ eta,
                              const float *__restrict__ R_upd, int32_t *__restrict__ prov,
                              float *__restrict__ prov_eta, int32_t n) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t e = owner[v];
  if (e < 0) {
    prov[v] = int32_t(v);
    prov_eta[v] = eta ? eta[v] : 0.0f;
  } else {
    const int32_t mn = pins[eptr[e]];
    prov[v] = mn;
    if (mn == v) prov_eta[v] = R_upd[e];
  }
}

__global__ void k_flag_in(const int32_t *__restrict__ state, int32_t *__restrict__ flag, int32_t m) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < m) flag[e] = state[e] == kStIn ? 1 : 0;
}

// ---- a8: centroids of contracted clusters (members ascending) ---------------
template <int PT>
__device__ __forceinline__ double pool_val(const void *pool, int64_t idx) {
  if (PT == kPoolF32) return double(reinterpret_cast<const float *>(pool)[idx]);
  const uint16_t h = reinterpret_cast<const uint16_t *>(pool)[idx];
  return double(__uint_as_float(uint32_t(h) << 16));
}

// One wave per contracted cluster (grid-stride), lane j of the wave takes
// columns j, j + 64, ... (K <= 512); members summed in CSR order.
template <int PT>
__global__ void __launch_bounds__(kT)
k_centroids(const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins,
            const int32_t *__restrict__ in_list, const int32_t *__restrict__ n_in,
            const void *__restrict__ pool, int K, double *__restrict__ cent) {
  const int32_t cnt = *n_in;
  const int lane = threadIdx.x & 63;
  const int64_t nw = int64_t(gridDim.x) * (kT / 64);
  for (int64_t c = int64_t(blockIdx.x) * (kT / 64) + (threadIdx.x >> 6); c < cnt; c += nw) {
    const int32_t e = in_list[c];
    const int32_t a = eptr[e], b = eptr[e + 1];
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    // two pins' rows in flight at a time; the sums run in pin order
    int32_t j = a;
    for (; j + 2 <= b; j += 2) {
      const int64_t base0 = int64_t(pins[j]) * K, base1 = int64_t(pins[j + 1]) * K;
      double v0[8], v1[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int col = lane + 64 * q;
        v0[q] = pool_val<PT>(pool, base0 + (col < K ? col : K - 1));
        v1[q] = pool_val<PT>(pool, base1 + (col < K ? col : K - 1));
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = (acc[q] + v0[q]) + v1[q];
    }
    if (j < b) {
      const int64_t base = int64_t(pins[j]) * K;
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int col = lane + 64 * q;
        v[q] = pool_val<PT>(pool, base + (col < K ? col : K - 1));
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = acc[q] + v[q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int col = lane + 64 * q;
      if (col < K) cent[c * K + col] = acc[q] / double(b - a);
    }
  }
}

// ---- a8: best neighbouring cluster of every isolated node --------------------
// flag[p] = 1 for the nodes the search runs on: not in a contracted cluster,
// at least one hyperedge
__global__ void k_single_flag(const int32_t *__restrict__ owner, const int32_t *__restrict__ vptr,
                              int32_t n, int32_t *__restrict__ flag) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  flag[p] = (owner[p] < 0 && vptr[p + 1] > vptr[p]) ? 1 : 0;
}

// Columns with Q_H > 0 sorted by ascending Q_H (largest weights first).
__global__ void __launch_bounds__(512)
k_qh_order(const double *__restrict__ qh, int K, int32_t *__restrict__ perm,
           float *__restrict__ inv32, int32_t *__restrict__ nuse) {
  // Q_H staged in LDS (columns past K and Q_H <= 0 as 0); the rank of
  // column i counts the positive columns before it in (Q_H, index) order
  __shared__ double q[512];
  __shared__ int wpos[512 / 64];
  const int i = threadIdx.x;
  const double qi = i < K ? qh[i] : 0.0;
  q[i] = qi > 0.0 ? qi : 0.0;
  const uint64_t pos = __ballot(qi > 0.0);
  if ((i & 63) == 0) wpos[i >> 6] = __popcll(pos);
  __syncthreads();
  int nu = 0;
#pragma unroll
  for (int w = 0; w < 512 / 64; ++w) nu += wpos[w];
  if (qi > 0.0) {
    int r = 0;
#pragma unroll 8
    for (int j = 0; j < K; ++j) {
      const double qj = q[j];
      r += (qj > 0.0 && (qj < qi || (qj == qi && j < i))) ? 1 : 0;
    }
    perm[r] = i;
    inv32[r] = float(1.0 / qi);
  }
  if (i == 0) *nuse = nu;
  if (i >= nu) { perm[i] = 0; inv32[i] = 0.0f; }
}

// cperm[C][q] = float16 of cluster C's centroid in column perm[q] (zero for
// q >= nuse), for every cluster id C (a node that is its cluster's smallest
// member).  Row width Kq = K rounded up to 64 (<= 512).  crow[C] = the row of
// C's float64 centroid (-1: singleton, the centroid is its pool row).  One
// wave per node, lane j takes q = j, j + 64, ...
template <int PT>
__global__ void __launch_bounds__(kT)
k_cperm(const int32_t *__restrict__ prov, const int32_t *__restrict__ owner,
        const int32_t *__restrict__ in_index, const double *__restrict__ cent,
        const void *__restrict__ pool, int K, int Kq, const int32_t *__restrict__ perm,
        const int32_t *__restrict__ nuse, _Float16 *__restrict__ cperm,
        int32_t *__restrict__ crow, int32_t n) {
  __shared__ float rows[kT / 64][512];
  const int64_t v = int64_t(blockIdx.x) * (kT / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (v >= n || prov[v] != v) return;
  const int32_t ow = owner[v];
  const int64_t cr = ow < 0 ? -1 : in_index[ow];
  if (lane == 0) crow[v] = int32_t(cr);
  const int nu = *nuse;
  // the row (or its cluster's centroid) is read in column order into LDS,
  // then permuted from there; perm has 512 entries (zero from nuse on)
  float *row = rows[threadIdx.x >> 6];
  if (cr < 0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = lane + 64 * j;
      const float x = float(pool_val<PT>(pool, v * K + (c < K ? c : K - 1)));
      row[c] = c < K ? x : 0.0f;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = lane + 64 * j;
      const float x = float(cent[cr * K + (c < K ? c : K - 1)]);
      row[c] = c < K ? x : 0.0f;
    }
  }
  int col[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) col[j] = perm[lane + 64 * j];
  wave_sync();
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int q = lane + 64 * j;
    if (q < Kq) cperm[v * Kq + q] = _Float16(q < nu ? row[col[j]] : 0.0f);
  }
}

// Bounds of one column's term (x - c)^2 / Q_H from the float16 copy h of c:
// |h - c| <= 2^-10 |h| + 2^-24 (float16 rounding of the float32 rounding of
// c, subnormals included; |c| <= 1 for an orthonormal basis; the factor
// 2^-10 is twice the rounding bound, which leaves room for the float32
// rounding below), so |x - c| sqrt(1 / Q_H) lies within
// |x - h| sv -/+ (|h| e1 + e0) with sv = sqrt(1 / Q_H), e1 = 2^-10 sv,
// e0 = 2^-24 sv.  The running maxima lo, up over the 8 float16 values of v
// (columns q0 .. q0+8) are kept in this square-root scale; their squares
// bound the term from below and above to within a relative 1e-6.
__device__ __forceinline__ void bounds16_8(const uint4 v, const float *xs, const float *sv,
                                           const float *e1, const float *e0, int q0, float &lo,
                                           float &up) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const uint32_t bits = (w[u >> 1] >> (16 * (u & 1))) & 0xFFFFu;
    const float h = float(__builtin_bit_cast(_Float16, uint16_t(bits)));
    const float a = fabsf(xs[q0 + u] - h);
    const float es = __builtin_fmaf(fabsf(h), e1[q0 + u], e0[q0 + u]);
    lo = fmaxf(lo, __builtin_fmaf(a, sv[q0 + u], -es));
    up = fmaxf(up, __builtin_fmaf(a, sv[q0 + u], es));
  }
}

// Exact float64 distance d(p, C) = max_i (chi_p^(i) - c_C^(i))^2 / Q_H(i)
// (Eqs. (13), (14) applied to a node and a centroid), no FMA; full wave.  xn
// is p's row and qd is Q_H (both in column order, zero from K on; at most
// 512 columns); cr = crow[C].  A lane's eight centroid values are loaded
// together, ahead of any use.
template <int PT>
__device__ __forceinline__ double exact_d(int32_t C, int32_t cr, int lane, const double *cent,
                                          const void *pool, int K, const float *xn,
                                          const double *qd) {
  constexpr int MAXC = 8;
  // unconditional loads of in-row columns (col clamped to K - 1; qd is zero
  // from K on, so those lanes' values are never used)
  int cl[MAXC];
#pragma unroll
  for (int q = 0; q < MAXC; ++q) cl[q] = lane + 64 * q < K ? lane + 64 * q : K - 1;
  double c[MAXC];
  if (cr < 0 && PT == kPoolF32) {
    const float *row = reinterpret_cast<const float *>(pool) + int64_t(C) * K;
    float t[MAXC];
#pragma unroll
    for (int q = 0; q < MAXC; ++q) t[q] = row[cl[q]];
#pragma unroll
    for (int q = 0; q < MAXC; ++q) c[q] = double(t[q]);
  } else if (cr < 0) {
    const uint16_t *row = reinterpret_cast<const uint16_t *>(pool) + int64_t(C) * K;
    uint32_t t[MAXC];
#pragma unroll
    for (int q = 0; q < MAXC; ++q) t[q] = row[cl[q]];
#pragma unroll
    for (int q = 0; q < MAXC; ++q) c[q] = double(__uint_as_float(t[q] << 16));
  } else {
    const double *row = cent + int64_t(cr) * K;
#pragma unroll
    for (int q = 0; q < MAXC; ++q) c[q] = row[cl[q]];
  }
  double dl = 0.0;
#pragma unroll
  for (int q = 0; q < MAXC; ++q) {
    const int col = lane + 64 * q;
    const double qv = qd[col];
    if (qv > 0.0) {
      const double diff = double(xn[col]) - c[q];
      const double sq = diff * diff;
      const double r = sq / qv;
      dl = r > dl ? r : dl;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(dl, off, 64);
    dl = o > dl ? o : dl;
  }
  return dl;
}

// One wave per isolated node p; its candidates are the clusters C = prov[v]
// of the co-pins v of its hyperedges, and best(p) = (smallest exact float64
// d(p, C), smallest label).  The wave bounds d(p, C) from float16 copies of
// the centroids, columns in the permuted order (largest weights first), in
// stages over growing column ranges, each stage keeping running lower and
// upper bounds:
//   stage A  one lane per candidate, columns [0, 128);
//   stage B  8 lanes per candidate, columns [128, 256);
//   stage C  8 lanes per candidate, columns [256, Kq): the upper bound now
//            covers every column.
// u is the smallest complete upper bound (or exact distance) met so far.  A
// candidate whose lower bound exceeds u (1 + 1e-5) is farther than some other
// candidate, so it is neither the minimum nor tied with it, and is dropped
// at any stage.  The survivors of stage C get their exact distance in
// ascending order of their lower bound, until the smallest remaining lower
// bound exceeds u.  Float32 bounds stay within a relative 1e-6 of what they
// bound (upper bounds are scaled by 1 + 1e-5 before use), so the result is
// the exact argmin whatever the visiting order.  The first candidate batch
// seeds u with stages B and C of its smallest stage-A bound; hyperedges of
// at most kSeedSeg pins are visited first.
constexpr int kQCap = 72;   // stage-B queue: 8 + one batch of 64
constexpr int kQ2Cap = 16;  // stage-C queue: 8 + one stage-B batch
constexpr int kFCap = 64;   // stage-C survivors awaiting their exact distance
constexpr int kEB = 64;     // hyperedges of p per batch
constexpr int kAq = 128;    // stage-A columns
constexpr int kBq = 256;    // end of the stage-B columns

constexpr int kBT = 128;  // best-neighbour workgroup: two waves (two nodes)

template <int PT>
__global__ void __launch_bounds__(kBT)
k_best(const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins,
       const int32_t *__restrict__ vptr, const int32_t *__restrict__ eids,
       const int32_t *__restrict__ owner, const int32_t *__restrict__ prov,
       const int32_t *__restrict__ crow, const double *__restrict__ cent,
       const _Float16 *__restrict__ cperm, int Kq, const int32_t *__restrict__ perm,
       const float *__restrict__ inv32, const void *__restrict__ pool, int K,
       const double *__restrict__ qh, const int32_t *__restrict__ list,
       const int32_t *__restrict__ count, int32_t *__restrict__ best_label,
       double *__restrict__ best_d) {
  constexpr int NW = kBT / 64;
  // one wave per listed isolated node; workgroups past the list leave at once
  const int32_t cnt = *count;
  if (int64_t(blockIdx.x) * NW >= cnt) return;
  __shared__ float sv[512];                // sqrt(1 / Q_H), 2^-10 and 2^-24 times
  __shared__ float s10[512];               // it, permuted order (zero for unused
  __shared__ float s24[512];               // columns)
  __shared__ double qd[512];               // Q_H, column order
  __shared__ int32_t pm[512];              // the permutation
  __shared__ float xs_all[NW][512];        // p's row, permuted order
  __shared__ float xn_all[NW][512];        // p's row, column order
  __shared__ int32_t es_all[NW][kEB];      // first pin position per hyperedge (batch order)
  __shared__ int32_t ep_all[NW][kEB + 1];  // exclusive prefix of sizes
  __shared__ int32_t qc_all[NW][kQCap];    // stage-B queue: candidate, bounds
  __shared__ float ql_all[NW][kQCap];
  __shared__ float qu_all[NW][kQCap];
  __shared__ int32_t rc_all[NW][kQ2Cap];   // stage-C queue: candidate, bounds
  __shared__ float rl_all[NW][kQ2Cap];
  __shared__ float ru_all[NW][kQ2Cap];
  __shared__ int32_t fc_all[NW][kFCap];    // survivors: candidate, crow, lower bound
  __shared__ int32_t fr_all[NW][kFCap];
  __shared__ float fl_all[NW][kFCap];
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 3, a8 = lane & 7;
  const uint64_t lt_mask = (uint64_t(1) << lane) - 1;
  for (int q = threadIdx.x; q < 512; q += kBT) {
    const float r = sqrtf(inv32[q]);
    sv[q] = r;
    s10[q] = 0x1p-10f * r;
    s24[q] = 0x1p-24f * r;
    qd[q] = q < K ? qh[q] : 0.0;
    pm[q] = perm[q];
  }
  __syncthreads();
  const int64_t i = int64_t(blockIdx.x) * NW + w;
  if (i >= cnt) return;
  const int64_t p = list[i];
  const int32_t v0 = vptr[p], deg = vptr[p + 1] - v0;
  if (owner[p] >= 0 || deg == 0) {
    if (lane == 0) best_label[p] = -1;
    return;
  }
  constexpr float kMargin = 1.0f + 1e-5f;
  constexpr float kUbScale = 1.0f + 2e-6f;
  constexpr float kUpScale = 1.0f + 1e-5f;
  float *xs = xs_all[w];
  float *xn = xn_all[w];
  int32_t *es = es_all[w];
  int32_t *ep = ep_all[w];
  int32_t *qc = qc_all[w];
  float *ql = ql_all[w];
  float *qu = qu_all[w];
  int32_t *rc = rc_all[w];
  float *rl = rl_all[w];
  float *ru = ru_all[w];
  int32_t *fc = fc_all[w];
  int32_t *fr = fr_all[w];
  float *fl = fl_all[w];
  {
    // p's row: unconditional loads (column clamped to K - 1), then selects
    float t[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int q = lane + 64 * j;
      t[j] = float(pool_val<PT>(pool, p * K + (q < K ? q : K - 1)));
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) xn[lane + 64 * j] = lane + 64 * j < K ? t[j] : 0.0f;
    wave_sync();
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int q = lane + 64 * j;
      xs[q] = q < Kq ? xn[pm[q]] : 0.0f;
    }
  }
  const int ka = Kq < kAq ? Kq : kAq;  // stage-A width (a multiple of 64)
  wave_sync();

  double bd = DBL_MAX;           // best exact distance (wave-uniform)
  int32_t bl = INT32_MAX;
  float ub = FLT_MAX;            // u: float32 upper bound of the minimum
  int nq = 0, nr = 0, nf = 0;    // queue, stage-C queue, survivor fills (wave-uniform)
  auto exact = [&](int32_t C, int32_t cr) __attribute__((always_inline)) {
    const double dl = exact_d<PT>(C, cr, lane, cent, pool, K, xn, qd);
    if (dl < bd || (dl == bd && C < bl)) {
      bd = dl;
      bl = C;
    }
    ub = fminf(ub, float(dl) * kUbScale * kUbScale);
  };
  // exact distances of the survivors, smallest lower bound first
  auto resolve = [&]() __attribute__((always_inline)) {
    while (nf > 0) {
      float l = lane < nf ? fl[lane] : FLT_MAX;
      int i = lane;
      for (int off = 1; off < 64; off <<= 1) {
        const float ol = __shfl_xor(l, off, 64);
        const int oi = __shfl_xor(i, off, 64);
        if (ol < l || (ol == l && oi < i)) {
          l = ol;
          i = oi;
        }
      }
      if (l * l > ub * kMargin) {
        nf = 0;
        break;
      }
      const int32_t C = fc[i], cr = fr[i];
      wave_sync();
      if (lane == 0) {
        fc[i] = fc[nf - 1];
        fr[i] = fr[nf - 1];
        fl[i] = fl[nf - 1];
      }
      --nf;
      wave_sync();
      if (C != bl) exact(C, cr);
    }
  };
  // stage C for the last cnt (<= 8) stage-C queue entries; survivors join
  // the list, and their complete upper bounds tighten u
  auto stage_c = [&](int cnt) __attribute__((always_inline)) {
    int32_t C = -1, cr = -1;
    float lo = FLT_MAX, up = 0.0f;
    if (g < cnt) {
      C = rc[nr - cnt + g];
      lo = rl[nr - cnt + g];
      up = ru[nr - cnt + g];
    }
    nr -= cnt;
    wave_sync();
    const bool live = C >= 0 && C != bl && !(lo * lo > ub * kMargin);
    if (live) {
      // lane a8 of the group takes columns kBq + 8 a8 + 64 it (Kq <= 512)
      cr = crow[C];
      const uint4 *row = reinterpret_cast<const uint4 *>(cperm + int64_t(C) * Kq);
      uint4 v[4];
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const int q0 = kBq + 8 * a8 + 64 * it;
        v[it] = q0 < Kq ? row[q0 / 8] : make_uint4(0u, 0u, 0u, 0u);
      }
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const int q0 = kBq + 8 * a8 + 64 * it;
        if (q0 < Kq) bounds16_8(v[it], xs, sv, s10, s24, q0, lo, up);
      }
    }
    for (int off = 4; off > 0; off >>= 1) {
      lo = fmaxf(lo, __shfl_xor(lo, off, 8));
      up = fmaxf(up, __shfl_xor(up, off, 8));
    }
    float um = live ? up * up * kUpScale : FLT_MAX;
    for (int off = 8; off < 64; off <<= 1) um = fminf(um, __shfl_xor(um, off, 64));
    ub = fminf(ub, um);
    const bool keep = live && a8 == 0 && !(lo * lo > ub * kMargin);
    const uint64_t m = __ballot(keep);
    const int nk = __popcll(m);
    if (nf + nk > kFCap) {
      // drop the survivors u now excludes, then resolve if still full
      const bool k2 = lane < nf && !(fl[lane] * fl[lane] > ub * kMargin);
      const int32_t c2 = k2 ? fc[lane] : 0, r2 = k2 ? fr[lane] : 0;
      const float l2 = k2 ? fl[lane] : 0.0f;
      const uint64_t m2 = __ballot(k2);
      wave_sync();
      if (k2) {
        const int at = __popcll(m2 & lt_mask);
        fc[at] = c2;
        fr[at] = r2;
        fl[at] = l2;
      }
      nf = __popcll(m2);
      wave_sync();
      if (nf + nk > kFCap) resolve();
    }
    if (keep) {
      const int at = nf + __popcll(m & lt_mask);
      fc[at] = C;
      fr[at] = cr;
      fl[at] = lo;
    }
    nf += nk;
    wave_sync();
  };
  // stage B for the last cnt (<= 8) queue entries; survivors join the
  // stage-C queue, which is drained in batches of 8
  auto stage_b = [&](int cnt) __attribute__((always_inline)) {
    int32_t C = -1;
    float lo = FLT_MAX, up = 0.0f;
    if (g < cnt) {
      C = qc[nq - cnt + g];
      lo = ql[nq - cnt + g];
      up = qu[nq - cnt + g];
    }
    nq -= cnt;
    wave_sync();
    const bool live = C >= 0 && C != bl && !(lo * lo > ub * kMargin);
    if (live) {
      // lane a8 of the group takes columns kAq + 8 a8 + 64 it
      const uint4 *row = reinterpret_cast<const uint4 *>(cperm + int64_t(C) * Kq);
      uint4 v[2];
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        const int q0 = kAq + 8 * a8 + 64 * it;
        v[it] = q0 < Kq ? row[q0 / 8] : make_uint4(0u, 0u, 0u, 0u);
      }
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        const int q0 = kAq + 8 * a8 + 64 * it;
        if (q0 < Kq) bounds16_8(v[it], xs, sv, s10, s24, q0, lo, up);
      }
    }
    for (int off = 4; off > 0; off >>= 1) {
      lo = fmaxf(lo, __shfl_xor(lo, off, 8));
      up = fmaxf(up, __shfl_xor(up, off, 8));
    }
    const bool keep = live && a8 == 0 && !(lo * lo > ub * kMargin);
    const uint64_t m = __ballot(keep);
    if (keep) {
      const int at = nr + __popcll(m & lt_mask);
      rc[at] = C;
      rl[at] = lo;
      ru[at] = up;
    }
    nr += __popcll(m);
    wave_sync();
    while (nr >= 8) stage_c(8);
  };

  for (int32_t e0 = 0; e0 < deg; e0 += kEB) {
    const int nb = deg - e0 < kEB ? deg - e0 : kEB;
    // this batch's hyperedges, the short ones first
    int32_t ea = 0, sz = 0;
    if (lane < nb) {
      const int32_t e = eids[v0 + e0 + lane];
      ea = eptr[e];
      sz = eptr[e + 1] - ea;
    }
    const bool sm = lane < nb && sz <= kSeedSeg;
    const uint64_t msm = __ballot(sm);
    const uint64_t mbg = __ballot(lane < nb && !sm);
    const int at = sm ? __popcll(msm & lt_mask) : __popcll(msm) + __popcll(mbg & lt_mask);
    if (lane < nb) {
      es[at] = ea;
      ep[at] = sz;
    }
    wave_sync();
    int32_t my = lane < nb ? ep[lane] : 0;
    int32_t inc = my;
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t o = __shfl_up(inc, off, 64);
      if (lane >= off) inc += o;
    }
    const int32_t total = __shfl(inc, 63, 64);
    wave_sync();
    if (lane < nb) ep[lane] = inc - my;
    if (lane == 0) ep[nb] = total;
    wave_sync();
    for (int32_t t0 = 0; t0 < total; t0 += 64) {
      const int32_t t = t0 + lane;
      int32_t C = -1;
      float lo = FLT_MAX, up = 0.0f;
      if (t < total) {
        int lo_i = 0, hi_i = nb;  // last i with ep[i] <= t
        while (hi_i - lo_i > 1) {
          const int mid = (lo_i + hi_i) >> 1;
          if (ep[mid] <= t) lo_i = mid; else hi_i = mid;
        }
        const int32_t v = pins[es[lo_i] + (t - ep[lo_i])];
        if (v != p) C = prov[v];
      }
      if (C >= 0) {
        // 64 columns (one 128-byte line) per round, loads ahead of use
        lo = 0.0f;
        const uint4 *row = reinterpret_cast<const uint4 *>(cperm + int64_t(C) * Kq);
        for (int q0 = 0; q0 < ka; q0 += 64) {
          uint4 v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] = row[q0 / 8 + u];
#pragma unroll
          for (int u = 0; u < 8; ++u) bounds16_8(v[u], xs, sv, s10, s24, q0 + 8 * u, lo, up);
        }
      }
      int32_t seed = -1;
      if (ub == FLT_MAX) {
        // seed u: stages B and C of the smallest (bound, label) of this batch
        float sl = lo, su = up;
        int32_t sc = C >= 0 ? C : INT32_MAX;
        for (int off = 1; off < 64; off <<= 1) {
          const float ol = __shfl_xor(sl, off, 64);
          const float ou = __shfl_xor(su, off, 64);
          const int32_t oc = __shfl_xor(sc, off, 64);
          if (ol < sl || (ol == sl && oc < sc)) {
            sl = ol;
            su = ou;
            sc = oc;
          }
        }
        if (sc != INT32_MAX) {
          if (lane == 0) {
            qc[nq] = sc;
            ql[nq] = sl;
            qu[nq] = su;
          }
          ++nq;
          wave_sync();
          stage_b(1);
          while (nr > 0) stage_c(nr < 8 ? nr : 8);
          seed = sc;
        }
      }
      const bool ok = C >= 0 && C != bl && C != seed && !(lo * lo > ub * kMargin);
      const uint64_t m = __ballot(ok);
      if (ok) {
        const int at2 = nq + __popcll(m & lt_mask);
        qc[at2] = C;
        ql[at2] = lo;
        qu[at2] = up;
      }
      nq += __popcll(m);
      wave_sync();
      while (nq >= 8) stage_b(8);
    }
    wave_sync();
  }
  if (nq > 0) stage_b(nq);
  while (nr > 0) stage_c(nr < 8 ? nr : 8);
  resolve();
  if (lane == 0) {
    best_label[p] = bl == INT32_MAX ? -1 : bl;
    best_d[p] = bd;
  }
}

// *out += the (isolated node, candidate cluster) pairs k_best screens: one
// per co-pin occurrence of every listed node p, sum_{e ∋ p} (|e| - 1).  A
// thread per listed node, a block sum, one integer atomic per workgroup.
__global__ void __launch_bounds__(256)
k_count_candidates(const int32_t *__restrict__ list, const int32_t *__restrict__ count,
                   const int32_t *__restrict__ vptr, const int32_t *__restrict__ eids,
                   const int32_t *__restrict__ eptr, unsigned long long *__restrict__ out) {
  __shared__ unsigned long long part[256];
  const int64_t cnt = *count;
  unsigned long long acc = 0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int32_t p = list[i];
    const int32_t j1 = vptr[p + 1];
    // four hyperedges' loads at a time (independent), then their sizes
    for (int32_t j = vptr[p]; j < j1; j += 4) {
      int32_t e[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) e[u] = j + u < j1 ? eids[j + u] : -1;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e[u] >= 0) acc += unsigned(eptr[e[u] + 1] - eptr[e[u]] - 1);
    }
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (int(threadIdx.x) < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0 && part[0]) atomicAdd(out, part[0]);
}

// ---- union-find over the attach pairs (roots end as component minima) ------
__device__ __forceinline__ int32_t find_root(const int32_t *parent, int32_t x) {
  int32_t p = parent[x];
  while (p != x) {
    x = p;
    p = parent[x];
  }
  return x;
}

__global__ void k_uf_init(int32_t *__restrict__ parent, int32_t n) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v < n) parent[v] = int32_t(v);
}

__global__ void k_uf_hook(const int32_t *__restrict__ best_label, int32_t *__restrict__ parent,
                          int32_t n, int32_t *__restrict__ changed) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t c = best_label[p];
  if (c < 0) return;
  const int32_t a = find_root(parent, int32_t(p));
  const int32_t b = find_root(parent, c);
  if (a != b) {
    atomicMin(&parent[a > b ? a : b], a < b ? a : b);
    *changed = 1;
  }
}

__global__ void k_uf_compress(int32_t *__restrict__ parent, int32_t n) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v < n) parent[v] = find_root(parent, int32_t(v));
}

// cluster ids of this level are provisional labels (prov[v] == v); a root is
// a cluster whose component root is itself
__global__ void k_root_flags(const int32_t *__restrict__ prov, const int32_t *__restrict__ parent,
                             int32_t *__restrict__ flag, int32_t n) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v < n) flag[v] = (prov[v] == v && parent[v] == v) ? 1 : 0;
}

__global__ void k_labels(const int32_t *__restrict__ prov, const int32_t *__restrict__ parent,
                         const int32_t *__restrict__ rank_of_root, int32_t *__restrict__ label,
                         int32_t n) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v < n) label[v] = rank_of_root[parent[prov[v]]];
}

// ---- eta of merged groups ---------------------------------------------------
// attach pairs: each isolated p with best b gives key (min, max); mutual
// pairs of two isolated nodes appear twice and are kept once (the copy from
// the smaller endpoint).  flag marks the pairs to keep.
__global__ void k_pair_flags(const int32_t *__restrict__ best_label, const int32_t *__restrict__ owner,
                             int32_t *__restrict__ flag, int32_t n) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t b = best_label[p];
  int32_t f = 0;
  if (b >= 0) {
    f = 1;
    // b is a node id; if b is itself isolated and picked p, the pair is
    // counted by the smaller of the two
    if (owner[b] < 0 && best_label[b] == int32_t(p) && b < p) f = 0;
  }
  flag[p] = f;
}

// One thread per group: sequential float64 sum of the group's cluster etas
// (ascending label) then its pair distances (ascending (min, max)).
__global__ void k_group_eta(const int32_t *__restrict__ cl_ptr, const int32_t *__restrict__ cl_lab,
                            const float *__restrict__ prov_eta, const int32_t *__restrict__ pr_ptr,
                            const int32_t *__restrict__ pr_node, const double *__restrict__ best_d,
                            int32_t ngroups, float *__restrict__ eta_out) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= ngroups) return;
  double acc = 0.0;
  for (int32_t i = cl_ptr[g]; i < cl_ptr[g + 1]; ++i) acc = acc + double(prov_eta[cl_lab[i]]);
  for (int32_t i = pr_ptr[g]; i < pr_ptr[g + 1]; ++i) acc = acc + best_d[pr_node[i]];
  eta_out[g] = float(acc);
}

// segment starts of a sorted key array: ptr[k] = first index with key >= k
// ptr[k] = the first position of a key >= k in the ascending keys[0, cnt),
// for k = 0 .. nseg (one binary search per segment, so a long run of empty
// segments costs no single thread more than another)
__global__ void k_seg_ptr(const uint32_t *__restrict__ keys, int64_t cnt, int32_t nseg,
                          int32_t *__restrict__ ptr) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k > nseg) return;
  int64_t lo = 0, hi = cnt;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (int64_t(keys[mid]) < k) lo = mid + 1; else hi = mid;
  }
  ptr[k] = int32_t(lo);
}

// gather helpers for the sorts
__global__ void k_items_clusters(const int32_t *__restrict__ prov, const int32_t *__restrict__ label,
                                 const int32_t *__restrict__ pos, uint32_t *__restrict__ keys,
                                 uint32_t *__restrict__ vals, int32_t n) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n || prov[v] != v) return;
  keys[pos[v]] = uint32_t(label[v]);
  vals[pos[v]] = uint32_t(v);
}

__global__ void k_cluster_flags(const int32_t *__restrict__ prov, int32_t *__restrict__ flag, int32_t n) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v < n) flag[v] = prov[v] == v ? 1 : 0;
}

// pairs, step 1: key = max endpoint (low half of the (min, max) order)
__global__ void k_items_pairs(const int32_t *__restrict__ best_label, const int32_t *__restrict__ flag,
                              const int32_t *__restrict__ pos, uint32_t *__restrict__ keys,
                              uint32_t *__restrict__ vals, int32_t n) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n || !flag[p]) return;
  const int32_t b = best_label[p];
  keys[pos[p]] = uint32_t(p > b ? p : b);
  vals[pos[p]] = uint32_t(p);
}

__global__ void k_rekey_min(const int32_t *__restrict__ best_label, const uint32_t *__restrict__ vals,
                            uint32_t *__restrict__ keys, int64_t cnt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const int32_t p = int32_t(vals[i]);
  const int32_t b = best_label[p];
  keys[i] = uint32_t(p < b ? p : b);
}

__global__ void k_rekey_group(const int32_t *__restrict__ label, const uint32_t *__restrict__ vals,
                              uint32_t *__restrict__ keys, int64_t cnt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < cnt) keys[i] = uint32_t(label[vals[i]]);
}

// ---- a9: coarse rebuild -----------------------------------------------------
__global__ void k_pin_labels(const int32_t *__restrict__ pins, const int32_t *__restrict__ label,
                             uint32_t *__restrict__ keys, uint32_t *__restrict__ vals, int64_t nnz) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= nnz) return;
  keys[j] = uint32_t(label[pins[j]]);
  vals[j] = uint32_t(j);
}

__global__ void k_slot_edge(const int32_t *__restrict__ eptr, uint32_t *__restrict__ eid, int32_t m) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  for (int32_t j = eptr[e]; j < eptr[e + 1]; ++j) eid[j] = uint32_t(e);
}

__global__ void k_gather_u32(const uint32_t *__restrict__ src, const uint32_t *__restrict__ idx,
                             uint32_t *__restrict__ dst, int64_t cnt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < cnt) dst[i] = src[idx[i]];
}

// after sorting slots by (edge, label): count distinct labels per edge
// ---- a9: per-hyperedge sorted labels -----------------------------------------
// lab_sorted[eptr[e] .. eptr[e+1]) = the labels of e's pins in ascending order
// and cnt[e] = their number of distinct values (0 when below 2).  Hyperedges
// of at most kSmallSeg pins: one thread each, a bitonic network in
// registers; larger ones (the structure's big list): one workgroup each, a
// bitonic sort in LDS of up to kEdgeSortCap labels (a larger hyperedge
// raises *overflow and the level takes the global sort instead).
constexpr int kEdgeSortCap = 16384;

template <int N>
__device__ __forceinline__ void bitonic_regs(uint32_t (&x)[N]) {
#pragma unroll
  for (int k = 2; k <= N; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int l = i ^ j;
        if (l > i) {
          const uint32_t a = x[i], b = x[l];
          const bool asc = (i & k) == 0;
          x[i] = asc ? min(a, b) : max(a, b);
          x[l] = asc ? max(a, b) : min(a, b);
        }
      }
}

template <int N>
__device__ __forceinline__ void elab_regs(const int32_t *__restrict__ pins,
                                          const int32_t *__restrict__ label, int32_t a,
                                          int32_t sz, uint32_t *__restrict__ out, int32_t &c) {
  uint32_t x[N];
  // unconditional loads (position clamped into the segment), then padding
#pragma unroll
  for (int u = 0; u < N; ++u) x[u] = uint32_t(pins[a + (u < sz ? u : sz - 1)]);
#pragma unroll
  for (int u = 0; u < N; ++u) x[u] = uint32_t(label[x[u]]);
#pragma unroll
  for (int u = 0; u < N; ++u) x[u] = u < sz ? x[u] : 0xFFFFFFFFu;
  bitonic_regs<N>(x);
  c = 0;
#pragma unroll
  for (int u = 0; u < N; ++u)
    if (u < sz) {
      out[a + u] = x[u];
      c += (u == 0 || x[u] != x[u - 1]) ? 1 : 0;
    }
}

__global__ void __launch_bounds__(kT)
k_elab_small(const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins,
             const int32_t *__restrict__ label, int32_t m, uint32_t *__restrict__ lab_sorted,
             int32_t *__restrict__ cnt) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int32_t a = eptr[e], sz = eptr[e + 1] - a;
  if (sz > kSmallSeg) return;
  if (sz == 0) {
    cnt[e] = 0;
    return;
  }
  int32_t c = 0;
  if (sz <= 8)
    elab_regs<8>(pins, label, a, sz, lab_sorted, c);
  else
    elab_regs<32>(pins, label, a, sz, lab_sorted, c);
  cnt[e] = c >= 2 ? c : 0;
}

__global__ void __launch_bounds__(kT)
k_elab_big(const int32_t *__restrict__ list, const int32_t *__restrict__ count,
           const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins,
           const int32_t *__restrict__ label, uint32_t *__restrict__ lab_sorted,
           int32_t *__restrict__ cnt, int32_t *__restrict__ overflow) {
  __shared__ uint32_t buf[kEdgeSortCap];
  __shared__ int32_t wsum[kT / 64];
  const int tid = threadIdx.x;
  const int32_t nb = *count;
  for (int32_t bi = blockIdx.x; bi < nb; bi += gridDim.x) {
    const int32_t e = list[bi];
    const int32_t a = eptr[e], sz = eptr[e + 1] - a;
    if (sz > kEdgeSortCap) {
      if (tid == 0) *overflow = 1;
      continue;
    }
    int32_t P = 1;
    while (P < sz) P <<= 1;
    for (int32_t i = tid; i < P; i += kT) buf[i] = i < sz ? uint32_t(label[pins[a + i]]) : 0xFFFFFFFFu;
    __syncthreads();
    for (int32_t k = 2; k <= P; k <<= 1)
      for (int32_t j = k >> 1; j > 0; j >>= 1) {
        for (int32_t i = tid; i < P; i += kT) {
          const int32_t l = i ^ j;
          if (l > i) {
            const uint32_t x = buf[i], y = buf[l];
            const bool asc = (i & k) == 0;
            if ((x > y) == asc) {
              buf[i] = y;
              buf[l] = x;
            }
          }
        }
        __syncthreads();
      }
    int32_t c = 0;
    for (int32_t i = tid; i < sz; i += kT) {
      lab_sorted[a + i] = buf[i];
      c += (i == 0 || buf[i] != buf[i - 1]) ? 1 : 0;
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((tid & 63) == 0) wsum[tid >> 6] = c;
    __syncthreads();
    if (tid == 0) {
      int32_t t = 0;
      for (int q = 0; q < kT / 64; ++q) t += wsum[q];
      cnt[e] = t >= 2 ? t : 0;
    }
    __syncthreads();
  }
}

// eptr2[m2] = nnz2 and (m2, nnz2, overflow) for the host, in one place
__global__ void k_rebuild_tail(const int32_t *__restrict__ kpos, const int32_t *__restrict__ nptr,
                               int64_t m, const int32_t *__restrict__ overflow,
                               int32_t *__restrict__ eptr2, int32_t *__restrict__ out3) {
  const int32_t m2 = kpos[m], nnz2 = nptr[m];
  eptr2[m2] = nnz2;
  out3[0] = m2;
  out3[1] = nnz2;
  out3[2] = overflow ? *overflow : 0;
}

__global__ void k_distinct(const int32_t *__restrict__ eptr, const uint32_t *__restrict__ lab_sorted,
                           int32_t *__restrict__ cnt, int32_t m) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  int32_t c = 0;
  for (int32_t j = eptr[e]; j < eptr[e + 1]; ++j)
    if (j == eptr[e] || lab_sorted[j] != lab_sorted[j - 1]) ++c;
  cnt[e] = c >= 2 ? c : 0;
}

__global__ void k_emit(const int32_t *__restrict__ eptr, const uint32_t *__restrict__ lab_sorted,
                       const int32_t *__restrict__ cnt, const int32_t *__restrict__ new_ptr,
                       const int32_t *__restrict__ keep_pos, const float *__restrict__ w,
                       int32_t *__restrict__ eptr2, int32_t *__restrict__ pins2,
                       float *__restrict__ w2, int32_t *__restrict__ kept2, int32_t m) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m || cnt[e] == 0) return;
  const int32_t k = keep_pos[e];
  int32_t o = new_ptr[e];
  eptr2[k] = o;
  w2[k] = w ? w[e] : 1.0f;
  if (kept2) kept2[k] = int32_t(e);
  for (int32_t j = eptr[e]; j < eptr[e + 1]; ++j)
    if (j == eptr[e] || lab_sorted[j] != lab_sorted[j - 1]) pins2[o++] = int32_t(lab_sorted[j]);
}

__global__ void k_flag_pos(const int32_t *__restrict__ v, int32_t *__restrict__ f, int32_t m) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < m) f[e] = v[e] > 0 ? 1 : 0;
}

__global__ void k_compose(int32_t *__restrict__ map, const int32_t *__restrict__ label, int64_t n0) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v < n0) map[v] = label[map[v]];
}

__global__ void k_iota(int32_t *__restrict__ a, int64_t n) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v < n) a[v] = int32_t(v);
}

__global__ void k_set_i32(int32_t *__restrict__ p, int32_t v, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_zero_u64(unsigned long long *__restrict__ p, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// flag |= 1 if the label of a pin lies outside [0, nc)
__global__ void k_label_range(const int32_t *__restrict__ pins, const int32_t *__restrict__ label,
                              int64_t nnz, int32_t nc, int32_t *__restrict__ flag) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j < nnz) {
    const int32_t l = label[pins[j]];
    if (l < 0 || l >= nc) atomicOr(flag, 1);
  }
}

// flag |= 1 if a pool value is not finite or not below the largest float16
// (the local-clustering screen keeps float16 copies of pool rows)
template <int PT>
__global__ void k_pool_range(const void *__restrict__ pool, int64_t count,
                             int32_t *__restrict__ flag) {
  int bad = 0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x) {
    const float x = PT == kPoolF32
        ? reinterpret_cast<const float *>(pool)[i]
        : __uint_as_float(uint32_t(reinterpret_cast<const uint16_t *>(pool)[i]) << 16);
    if (!(fabsf(x) < 65504.0f)) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

inline unsigned g1(int64_t n) { return unsigned(std::max<int64_t>(1, cdiv(n, kT))); }

// Workspace of one clustering level (sizes of the level).
struct LevelWs {
  float *R_upd;
  uint32_t *k0, *v0, *k1, *v1;  // sort buffers (max(n, m, nnz))
  int32_t *rank, *state, *owner, *prov, *in_index, *in_list, *flag, *pos, *parent, *best_label,
      *label, *cl_ptr, *pr_ptr, *ibuf;
  unsigned long long *packed;
  float *prov_eta;
  double *best_d, *cent;
  _Float16 *cperm;
  float *inv32;
  int32_t *perm;
  int32_t *crow;   // [n] centroid row per cluster id
  int32_t *small;  // [8] device scalars
  float *delta;
};

void carve_level(Arena &a, int64_t n, int64_t m, int64_t nnz, int K, LevelWs &w) {
  const int64_t big = std::max(std::max(n, m), nnz) + 1;
  w.R_upd = a.take<float>(m + 1);
  w.k0 = a.take<uint32_t>(big);
  w.v0 = a.take<uint32_t>(big);
  w.k1 = a.take<uint32_t>(big);
  w.v1 = a.take<uint32_t>(big);
  w.rank = a.take<int32_t>(m + 1);
  w.state = a.take<int32_t>(m + 1);
  w.owner = a.take<int32_t>(n + 1);
  w.prov = a.take<int32_t>(n + 1);
  w.in_index = a.take<int32_t>(m + 1);
  w.in_list = a.take<int32_t>(m + 1);
  w.flag = a.take<int32_t>(big);
  w.pos = a.take<int32_t>(big);
  w.parent = a.take<int32_t>(n + 1);
  w.best_label = a.take<int32_t>(n + 1);
  w.label = a.take<int32_t>(n + 1);
  w.cl_ptr = a.take<int32_t>(n + 2);
  w.pr_ptr = a.take<int32_t>(n + 2);
  w.ibuf = a.take<int32_t>(big);
  w.packed = a.take<unsigned long long>(n + 1);
  w.prov_eta = a.take<float>(n + 1);
  w.best_d = a.take<double>(n + 1);
  w.cent = a.take<double>((n / 2 + 1) * int64_t(K));
  w.cperm = a.take<_Float16>((n + 1) * int64_t((K + 63) / 64 * 64));
  w.inv32 = a.take<float>(512);
  w.perm = a.take<int32_t>(512);
  w.crow = a.take<int32_t>(n + 1);
  w.small = a.take<int32_t>(8);
  w.delta = a.take<float>(1);
}

size_t level_ws_bytes(int64_t n, int64_t m, int64_t nnz, int K) {
  Arena a;
  LevelWs w;
  carve_level(a, n, m, nnz, K, w);
  return a.mark() + radix_ws_bytes(std::max(std::max(n, m), nnz)) +
         scan_ws_bytes(std::max(std::max(n, m), nnz) + 1) + 4096;
}

__global__ void k_counts3(const int32_t *__restrict__ a, const int32_t *__restrict__ b,
                          const int32_t *__restrict__ c, int64_t n, int32_t *__restrict__ out) {
  out[0] = a[n];
  out[1] = b[n];
  out[2] = c[n];
}

hef_status read_i32(const int32_t *dev, int32_t *host, hipStream_t s) {
  HEF_HIP(hipMemcpyAsync(host, dev, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HEF_HIP(hipStreamSynchronize(s));
  return HEF_OK;
}

}  // namespace

// One level of Alg. 2, resistance update to local clustering.  Outputs label[n] (canonical), the
// group count (host) and eta_out[n_groups].  Needs the level's CSC (st).
hef_status cluster_one_level(const Level &L, const Structure &st, const float *R, const float *eta,
                             const void *pool, int pool_type, int K, const double *qh,
                             float percentile, bool local, int32_t *label_out,
                             int32_t *n_groups_out, float *eta_out, Arena &ws, hipStream_t s,
                             unsigned long long *work) {
  const int64_t n = L.n, m = L.m, nnz = L.nnz;
  const size_t mk = ws.mark();
  LevelWs w;
  carve_level(ws, n, m, nnz, K, w);
  HEF_WS_CHECK(ws);

  // ---- a6: Eq. (15), order and threshold
  {
    TimedScope ts(kStClusterUpdate, s);
    if (m > 0) {
      k_eta_update<<<g1(m), kT, 0, s>>>(L.eptr, L.pins, R, eta, w.R_upd, w.k0, w.v0, int32_t(m));
      HEF_LAUNCH_CHECK();
      HEF_TRY(radix_sort_pairs(w.k0, w.v0, w.k1, w.v1, m, 32, ws, s));
      int64_t dpos = int64_t(std::ceil(double(percentile) * double(m))) - 1;
      dpos = std::min<int64_t>(std::max<int64_t>(dpos, 0), m - 1);
      k_rank<<<g1(m), kT, 0, s>>>(w.v1, w.R_upd, int32_t(m), dpos, w.rank, w.state, w.delta);
      HEF_LAUNCH_CHECK();
    }
  }
  // ---- a7: contraction rounds
  {
    TimedScope ts(kStClusterContract, s);
    if (n > 0) {
      k_set_i32<<<g1(n), kT, 0, s>>>(w.owner, -1, n);
      k_zero_u64<<<g1(n), kT, 0, s>>>(w.packed, n);
      HEF_LAUNCH_CHECK();
    }
    uint32_t round = 1;
    // every round decides at least the smallest-rank undecided candidate
    const int64_t max_batches = cdiv(m, kRoundsPerSync) + 2;
    for (int64_t batch = 0; m > 0; ++batch) {
      if (batch > max_batches) {
        set_error("contraction did not settle");
        return HEF_ERR_NUMERICAL;
      }
      for (int r = 0; r < kRoundsPerSync; ++r, ++round) {
        HEF_TRY(zero_async(w.small, sizeof(int32_t), s));
        k_round_propose<<<g1(m), kT, 0, s>>>(L.eptr, L.pins, w.rank, w.state, w.owner, w.packed,
                                            round, int32_t(m), w.small);
        k_round_select<<<g1(m), kT, 0, s>>>(L.eptr, L.pins, w.rank, w.state, w.owner, w.packed,
                                           round, int32_t(m));
        HEF_LAUNCH_CHECK();
      }
      int32_t und = 0;
      HEF_TRY(read_i32(w.small, &und, s));
      if (und == 0) break;
    }
  }
  // ---- provisional clusters and contracted-cluster index
  if (n > 0) {
    k_provisional<<<g1(n), kT, 0, s>>>(L.eptr, L.pins, w.owner, eta, w.R_upd, w.prov, w.prov_eta,
                                       int32_t(n));
    HEF_LAUNCH_CHECK();
  }
  if (m > 0) {
    k_flag_in<<<g1(m), kT, 0, s>>>(w.state, w.flag, int32_t(m));
    HEF_LAUNCH_CHECK();
    HEF_TRY(exclusive_scan_i32(w.flag, w.in_index, m, ws, s));
    HEF_TRY(compact_flags(w.flag, w.pos, w.in_list, w.small + 1, m, ws, s));
  }
  // ---- a8: local clustering
  {
    TimedScope ts(kStClusterLocal, s);
    if (n > 0) k_set_i32<<<g1(n), kT, 0, s>>>(w.best_label, -1, n);
    HEF_LAUNCH_CHECK();
    if (local && n > 0 && m > 0 && K > 0) {
      const int Kq = (K + 63) / 64 * 64;
      k_qh_order<<<1, 512, 0, s>>>(qh, K, w.perm, w.inv32, w.small + 3);
      // the isolated nodes, listed in node order (sort buffers are free here)
      int32_t *sflag = reinterpret_cast<int32_t *>(w.k1);
      int32_t *slist = reinterpret_cast<int32_t *>(w.v0);
      k_single_flag<<<g1(n), kT, 0, s>>>(w.owner, st.vptr, int32_t(n), sflag);
      HEF_LAUNCH_CHECK();
      HEF_TRY(compact_flags(sflag, reinterpret_cast<int32_t *>(w.k0), slist, w.small + 7, n, ws, s));
      if (pool_type == kPoolF32) {
        k_centroids<kPoolF32><<<2048, kT, 0, s>>>(L.eptr, L.pins, w.in_list, w.small + 1, pool, K, w.cent);
        k_cperm<kPoolF32><<<cdiv(n, kT / 64), kT, 0, s>>>(w.prov, w.owner, w.in_index, w.cent, pool, K, Kq,
                                                   w.perm, w.small + 3, w.cperm, w.crow, int32_t(n));
        {
          TimedScope tb(kStClusterBest, s);
          k_best<kPoolF32><<<cdiv(n, kBT / 64), kBT, 0, s>>>(L.eptr, L.pins, st.vptr, st.eids,
                                                     w.owner, w.prov, w.crow, w.cent, w.cperm, Kq,
                                                     w.perm, w.inv32, pool, K, qh, slist,
                                                     w.small + 7, w.best_label, w.best_d);
        }
      } else {
        k_centroids<kPoolBF16><<<2048, kT, 0, s>>>(L.eptr, L.pins, w.in_list, w.small + 1, pool, K, w.cent);
        k_cperm<kPoolBF16><<<cdiv(n, kT / 64), kT, 0, s>>>(w.prov, w.owner, w.in_index, w.cent, pool, K, Kq,
                                                   w.perm, w.small + 3, w.cperm, w.crow, int32_t(n));
        {
          TimedScope tb(kStClusterBest, s);
          k_best<kPoolBF16><<<cdiv(n, kBT / 64), kBT, 0, s>>>(L.eptr, L.pins, st.vptr, st.eids,
                                                     w.owner, w.prov, w.crow, w.cent, w.cperm, Kq,
                                                     w.perm, w.inv32, pool, K, qh, slist,
                                                     w.small + 7, w.best_label, w.best_d);
        }
      }
      if (work)  // (about one listed node per thread at the finest level)
        k_count_candidates<<<std::min<int64_t>(cdiv(n, 256), 4096), 256, 0, s>>>(
            slist, w.small + 7, st.vptr, st.eids, L.eptr, work);
      HEF_LAUNCH_CHECK();
    }
    // union-find over {p, best(p)}
    if (n > 0) {
      k_uf_init<<<g1(n), kT, 0, s>>>(w.parent, int32_t(n));
      HEF_LAUNCH_CHECK();
      // two hook + compress rounds per host check (a settled forest is
      // left unchanged by further rounds)
      for (int it = 0; it < 64; it += 2) {
        HEF_TRY(zero_async(w.small + 2, sizeof(int32_t), s));
        k_uf_hook<<<g1(n), kT, 0, s>>>(w.best_label, w.parent, int32_t(n), w.small + 2);
        k_uf_compress<<<g1(n), kT, 0, s>>>(w.parent, int32_t(n));
        HEF_TRY(zero_async(w.small + 2, sizeof(int32_t), s));
        k_uf_hook<<<g1(n), kT, 0, s>>>(w.best_label, w.parent, int32_t(n), w.small + 2);
        k_uf_compress<<<g1(n), kT, 0, s>>>(w.parent, int32_t(n));
        HEF_LAUNCH_CHECK();
        int32_t ch = 0;
        HEF_TRY(read_i32(w.small + 2, &ch, s));
        if (!ch) break;
        if (it == 62) {
          set_error("union-find did not settle");
          return HEF_ERR_NUMERICAL;
        }
      }
    }
  }
  // ---- canonical labels (rank of each group's smallest node id)
  int32_t ngroups = 0;
  {
    TimedScope ts(kStClusterRebuild, s);
    // three scans (group roots, clusters, attach pairs), one host read of
    // their totals; the cluster and pair positions live in ibuf and in the
    // contraction's key buffer, both free at this point
    int32_t *pos_cl = w.ibuf;
    int32_t *pos_pr = reinterpret_cast<int32_t *>(w.packed);
    int32_t ncl = 0, npr = 0;
    if (n > 0) {
      k_root_flags<<<g1(n), kT, 0, s>>>(w.prov, w.parent, w.flag, int32_t(n));
      HEF_LAUNCH_CHECK();
      HEF_TRY(exclusive_scan_i32(w.flag, w.pos, n, ws, s));
      k_labels<<<g1(n), kT, 0, s>>>(w.prov, w.parent, w.pos, label_out, int32_t(n));
      k_cluster_flags<<<g1(n), kT, 0, s>>>(w.prov, w.flag, int32_t(n));
      HEF_LAUNCH_CHECK();
      HEF_TRY(exclusive_scan_i32(w.flag, pos_cl, n, ws, s));
      k_pair_flags<<<g1(n), kT, 0, s>>>(w.best_label, w.owner, w.flag, int32_t(n));
      HEF_LAUNCH_CHECK();
      HEF_TRY(exclusive_scan_i32(w.flag, pos_pr, n, ws, s));
      k_counts3<<<1, 1, 0, s>>>(w.pos, pos_cl, pos_pr, n, w.small + 4);
      HEF_LAUNCH_CHECK();
      int32_t c3[3] = {0, 0, 0};
      HEF_HIP(hipMemcpyAsync(c3, w.small + 4, sizeof(c3), hipMemcpyDeviceToHost, s));
      HEF_HIP(hipStreamSynchronize(s));
      ngroups = c3[0];
      ncl = c3[1];
      npr = c3[2];
    }
    *n_groups_out = ngroups;
    if (n > 0 && ngroups > 0) {
      // cluster contributions sorted by (group, label)
      k_items_clusters<<<g1(n), kT, 0, s>>>(w.prov, label_out, pos_cl, w.k0, w.v0, int32_t(n));
      HEF_LAUNCH_CHECK();
      HEF_TRY(radix_sort_pairs(w.k0, w.v0, w.k1, w.v1, ncl, bits_for(ngroups), ws, s));
      k_seg_ptr<<<g1(int64_t(ngroups) + 1), kT, 0, s>>>(w.k1, ncl, ngroups, w.cl_ptr);
      HEF_HIP(hipMemcpyAsync(w.ibuf, w.v1, sizeof(int32_t) * std::max(ncl, 1), hipMemcpyDeviceToDevice, s));
      // pair contributions sorted by (group, min, max)
      if (npr > 0) {
        k_items_pairs<<<g1(n), kT, 0, s>>>(w.best_label, w.flag, pos_pr, w.k0, w.v0, int32_t(n));
        HEF_LAUNCH_CHECK();
        HEF_TRY(radix_sort_pairs(w.k0, w.v0, w.k1, w.v1, npr, bits_for(n), ws, s));      // by max
        k_rekey_min<<<g1(npr), kT, 0, s>>>(w.best_label, w.v1, w.k1, npr);
        HEF_TRY(radix_sort_pairs(w.k1, w.v1, w.k0, w.v0, npr, bits_for(n), ws, s));      // by min
        k_rekey_group<<<g1(npr), kT, 0, s>>>(label_out, w.v0, w.k0, npr);
        HEF_TRY(radix_sort_pairs(w.k0, w.v0, w.k1, w.v1, npr, bits_for(ngroups), ws, s)); // by group
        HEF_LAUNCH_CHECK();
      }
      k_seg_ptr<<<g1(int64_t(ngroups) + 1), kT, 0, s>>>(w.k1, npr, ngroups, w.pr_ptr);
      k_group_eta<<<g1(ngroups), kT, 0, s>>>(w.cl_ptr, w.ibuf, w.prov_eta, w.pr_ptr,
                                             reinterpret_cast<const int32_t *>(w.v1), w.best_d,
                                             ngroups, eta_out);
      HEF_LAUNCH_CHECK();
    }
  }
  ws.reset(mk);
  return HEF_OK;
}

// Coarse hypergraph: pins mapped to labels, per-hyperedge sorted distinct
// labels, hyperedges with fewer than two kept (order and weight kept).
hef_status rebuild_level(const Level &L, const Structure &st, const int32_t *label, int32_t n2,
                         int32_t *eptr2, int32_t *pins2, float *w2, int32_t *m2_host,
                         int64_t *nnz2_host, Arena &ws, hipStream_t s, int32_t *kept2 = nullptr) {
  const int64_t m = L.m, nnz = L.nnz;
  TimedScope ts(kStClusterRebuild, s);
  const size_t mk = ws.mark();
  uint32_t *k0 = ws.take<uint32_t>(nnz + 1), *v0 = ws.take<uint32_t>(nnz + 1);
  uint32_t *k1 = ws.take<uint32_t>(nnz + 1), *v1 = ws.take<uint32_t>(nnz + 1);
  uint32_t *eid = ws.take<uint32_t>(nnz + 1);
  int32_t *cnt = ws.take<int32_t>(m + 1), *nptr = ws.take<int32_t>(m + 1);
  int32_t *flag = ws.take<int32_t>(m + 1), *kpos = ws.take<int32_t>(m + 1);
  int32_t *misc = ws.take<int32_t>(8);  // overflow flag, (m2, nnz2, overflow)
  HEF_WS_CHECK(ws);
  *m2_host = 0;
  *nnz2_host = 0;
  if (m == 0 || nnz == 0) {
    HEF_TRY(zero_async(eptr2, sizeof(int32_t), s));
    ws.reset(mk);
    return HEF_OK;
  }
  // the compacted hyperedges: counts, positions, emission, totals
  auto emit = [&](const int32_t *ovf) -> hef_status {
    HEF_TRY(exclusive_scan_i32(cnt, nptr, m, ws, s));
    k_flag_pos<<<g1(m), kT, 0, s>>>(cnt, flag, int32_t(m));
    HEF_LAUNCH_CHECK();
    HEF_TRY(exclusive_scan_i32(flag, kpos, m, ws, s));
    k_emit<<<g1(m), kT, 0, s>>>(L.eptr, k0, cnt, nptr, kpos, L.w, eptr2, pins2, w2, kept2,
                                int32_t(m));
    k_rebuild_tail<<<1, 1, 0, s>>>(kpos, nptr, m, ovf, eptr2, misc + 4);
    HEF_LAUNCH_CHECK();
    int32_t t3[3] = {0, 0, 0};
    HEF_HIP(hipMemcpyAsync(t3, misc + 4, sizeof(t3), hipMemcpyDeviceToHost, s));
    HEF_HIP(hipStreamSynchronize(s));
    *m2_host = t3[0];
    *nnz2_host = t3[1];
    return t3[2] ? HEF_ERR_UNSUPPORTED : HEF_OK;
  };
  // per-hyperedge sorts
  HEF_TRY(zero_async(misc, sizeof(int32_t), s));
  k_elab_small<<<g1(m), kT, 0, s>>>(L.eptr, L.pins, label, int32_t(m), k0, cnt);
  k_elab_big<<<1024, kT, 0, s>>>(st.big_e, st.n_big, L.eptr, L.pins, label, k0, cnt, misc);
  HEF_LAUNCH_CHECK();
  if (emit(misc) == HEF_OK) {
    ws.reset(mk);
    return HEF_OK;
  }
  // a hyperedge beyond the LDS sort: global sorts of the slots by label,
  // then stably by hyperedge, i.e. (edge, label) order
  k_pin_labels<<<g1(nnz), kT, 0, s>>>(L.pins, label, k0, v0, nnz);
  HEF_LAUNCH_CHECK();
  HEF_TRY(radix_sort_pairs(k0, v0, k1, v1, nnz, bits_for(std::max<int32_t>(n2 - 1, 0)), ws, s));
  k_slot_edge<<<g1(m), kT, 0, s>>>(L.eptr, eid, int32_t(m));
  k_gather_u32<<<g1(nnz), kT, 0, s>>>(eid, v1, k0, nnz);       // edge of each sorted slot
  HEF_LAUNCH_CHECK();
  HEF_TRY(radix_sort_pairs(k0, v1, k1, v0, nnz, bits_for(m - 1), ws, s));
  // v0 = slots in (edge, label) order; k0 = their labels
  k_pin_labels<<<g1(nnz), kT, 0, s>>>(L.pins, label, k1, v1, nnz);
  k_gather_u32<<<g1(nnz), kT, 0, s>>>(k1, v0, k0, nnz);
  HEF_LAUNCH_CHECK();
  k_distinct<<<g1(m), kT, 0, s>>>(L.eptr, k0, cnt, int32_t(m));
  HEF_LAUNCH_CHECK();
  HEF_TRY(emit(nullptr));
  ws.reset(mk);
  return HEF_OK;
}

size_t rebuild_ws_bytes(int64_t n, int64_t m, int64_t nnz) {
  Arena a;
  for (int i = 0; i < 5; ++i) a.take<uint32_t>(nnz + 1);
  for (int i = 0; i < 4; ++i) a.take<int32_t>(m + 1);
  a.take<int32_t>(8);
  return a.mark() + radix_ws_bytes(nnz) + scan_ws_bytes(std::max(n, m) + 1) + 4096;
}

size_t rebuild_call_bytes(int64_t n, int64_t m, int64_t nnz) {
  Arena a;
  Structure st;
  structure_carve(a, n, m, nnz, st);
  a.take<int32_t>(4);
  return a.mark() + std::max(structure_build_ws(n, m, nnz), rebuild_ws_bytes(n, m, nnz)) + 4096;
}

size_t cluster_level_bytes(int64_t n, int64_t m, int64_t nnz, int K) {
  Arena a;
  Structure st;
  structure_carve(a, n, m, nnz, st);
  a.take<int32_t>(4);
  return a.mark() + std::max(structure_build_ws(n, m, nnz), level_ws_bytes(n, m, nnz, K)) + 4096;
}

namespace {

// Sizes of the levels of the calling thread's last hef_coarsen call.
constexpr int kMaxLevelLog = 64;
thread_local int32_t g_levels_run = 0;
thread_local int32_t g_level_n[kMaxLevelLog];
thread_local int32_t g_level_m[kMaxLevelLog];
thread_local int64_t g_level_nnz[kMaxLevelLog];
thread_local int64_t g_level_work[kMaxLevelLog];

// Persistent part of the coarsening workspace (sized at level 0, which
// bounds every level).
struct CoarsenWs {
  Structure st;
  int32_t *flags;
  void *pool, *pool2;
  double *qh;
  float *R;
  int32_t *eptr[2], *pins[2];
  float *w[2];
  float *eta[2];
  int32_t *label;
  unsigned long long *work;  // [kMaxLevelLog] candidates screened per level
};

void carve_coarsen(Arena &a, int64_t n, int64_t m, int64_t nnz, const hef_params &p, CoarsenWs &c) {
  structure_carve(a, n, m, nnz, c.st);
  c.flags = a.take<int32_t>(4);
  const int K = pool_width_of(p);
  c.pool = a.take<char>(size_t(n) * K * (p.basis == HEF_BASIS_BF16 ? 2 : 4));
  c.pool2 = a.take<char>(size_t(oct_rows(n)) * K * (p.basis == HEF_BASIS_BF16 ? 2 : 4));
  c.qh = a.take<double>(K);
  c.R = a.take<float>(m + 1);
  for (int i = 0; i < 2; ++i) {
    c.eptr[i] = a.take<int32_t>(m + 1);
    c.pins[i] = a.take<int32_t>(nnz + 1);
    c.w[i] = a.take<float>(m + 1);
    c.eta[i] = a.take<float>(n + 1);
  }
  c.label = a.take<int32_t>(n + 1);
  c.work = a.take<unsigned long long>(kMaxLevelLog);
}

}  // namespace

size_t coarsen_bytes(int64_t n, int64_t m, int64_t nnz, const hef_params &p) {
  Arena a;
  CoarsenWs c;
  carve_coarsen(a, n, m, nnz, p, c);
  const int K = pool_width_of(p);
  size_t scratch = estimate_level_bytes(n, m, nnz, p);
  scratch = std::max(scratch, level_ws_bytes(n, m, nnz, K));
  scratch = std::max(scratch, rebuild_ws_bytes(n, m, nnz));
  return a.mark() + scratch + 4096;
}

}  // namespace hef

using namespace hef;

extern "C" {

hef_status hef_cluster_level(const hef_hypergraph *hg, const hef_params *p, const float *R,
                             const float *eta_in, const float *chi, const double *qh,
                             int32_t *cluster, int32_t *n_clusters, float *eta_out, void *ws,
                             size_t ws_bytes, hipStream_t stream) {
  if (!hg || !p || !n_clusters || !ws) { set_error("NULL argument"); return HEF_ERR_INVALID_ARGUMENT; }
  size_t need = 0;
  HEF_TRY(hef_workspace_size(hg, p, HEF_OP_CLUSTER_LEVEL, &need));
  if (ws_bytes < need) { set_error("workspace too small (%zu < %zu)", ws_bytes, need); return HEF_ERR_WORKSPACE_TOO_SMALL; }
  const int K = pool_width_of(*p);
  if (hg->m > 0 && !R) { set_error("R is NULL"); return HEF_ERR_INVALID_ARGUMENT; }
  if (hg->n > 0 && (!cluster || !eta_out || (p->local_clustering && (!chi || !qh)))) {
    set_error("NULL output or pool");
    return HEF_ERR_INVALID_ARGUMENT;
  }
  Arena a;
  a.base = static_cast<char *>(ws);
  a.cap = ws_bytes;
  Structure st;
  structure_carve(a, hg->n, hg->m, hg->nnz, st);
  int32_t *flags = a.take<int32_t>(4);
  Level L;
  L.n = hg->n; L.m = hg->m; L.nnz = hg->nnz; L.eptr = hg->eptr; L.pins = hg->pins; L.w = hg->w;
  if (!(p->flags & HEF_FLAG_ASSUME_VALID)) {
    int32_t bad = 0;
    HEF_TRY(validate_device(L, flags, &bad, stream));
    if (bad) { set_error("invalid hypergraph (code %d)", bad); return HEF_ERR_INVALID_HYPERGRAPH; }
  }
  const int pt = p->basis == HEF_BASIS_BF16 ? kPoolBF16 : kPoolF32;
  if (p->local_clustering && hg->n > 0 && K > 0) {
    HEF_TRY(zero_async(flags, sizeof(int32_t), stream));
    const int64_t cnt = int64_t(hg->n) * K;
    const unsigned nb = unsigned(std::min<int64_t>(cdiv(cnt, kT), 4096));
    if (pt == kPoolF32) k_pool_range<kPoolF32><<<nb, kT, 0, stream>>>(chi, cnt, flags);
    else k_pool_range<kPoolBF16><<<nb, kT, 0, stream>>>(chi, cnt, flags);
    HEF_LAUNCH_CHECK();
    int32_t f = 0;
    HEF_TRY(read_i32(flags, &f, stream));
    if (f) {
      set_error("a pool value is not finite or its magnitude reaches 65504 (float16 range)");
      return HEF_ERR_INVALID_ARGUMENT;
    }
  }
  HEF_TRY(structure_build(L, st, a, stream));
  int32_t ng = 0;
  HEF_TRY(cluster_one_level(L, st, R, eta_in, chi, pt, K, qh, p->percentile,
                            p->local_clustering != 0, cluster, &ng, eta_out, a, stream, nullptr));
  HEF_HIP(hipStreamSynchronize(stream));
  *n_clusters = ng;
  return HEF_OK;
}

hef_status hef_rebuild(const hef_hypergraph *hg, const int32_t *label, int32_t n_clusters,
                       int32_t *eptr_out, int32_t *pins_out, float *w_out, int32_t *kept_out,
                       int32_t *m_out, int64_t *nnz_out, void *ws, size_t ws_bytes,
                       hipStream_t stream) {
  if (!hg || !m_out || !nnz_out || !ws || !eptr_out || (hg->n > 0 && !label) ||
      (hg->m > 0 && (!pins_out || !w_out))) {
    set_error("NULL argument");
    return HEF_ERR_INVALID_ARGUMENT;
  }
  if (hg->n < 0 || hg->m < 0 || hg->nnz < 0 || hg->nnz > INT32_MAX || !hg->eptr ||
      (hg->nnz > 0 && !hg->pins)) {
    set_error("bad hypergraph sizes or pointers");
    return HEF_ERR_INVALID_ARGUMENT;
  }
  if (n_clusters < 0 || (hg->n > 0 && n_clusters < 1) || n_clusters > std::max(hg->n, 1)) {
    set_error("n_clusters=%d out of range for n=%d", n_clusters, hg->n);
    return HEF_ERR_INVALID_ARGUMENT;
  }
  const size_t need = rebuild_call_bytes(hg->n, hg->m, hg->nnz);
  if (ws_bytes < need) { set_error("workspace too small (%zu < %zu)", ws_bytes, need); return HEF_ERR_WORKSPACE_TOO_SMALL; }
  Arena a;
  a.base = static_cast<char *>(ws);
  a.cap = ws_bytes;
  Structure st;
  structure_carve(a, hg->n, hg->m, hg->nnz, st);
  int32_t *flags = a.take<int32_t>(4);
  if (a.overflow) { set_error("workspace carve overflow"); return HEF_ERR_WORKSPACE_TOO_SMALL; }
  Level L;
  L.n = hg->n; L.m = hg->m; L.nnz = hg->nnz; L.eptr = hg->eptr; L.pins = hg->pins; L.w = hg->w;
  int32_t bad = 0;
  HEF_TRY(validate_device(L, flags, &bad, stream));
  if (bad) { set_error("invalid hypergraph (code %d)", bad); return HEF_ERR_INVALID_HYPERGRAPH; }
  if (hg->n > 0 && hg->nnz > 0) {
    HEF_TRY(zero_async(flags, sizeof(int32_t), stream));
    k_label_range<<<g1(hg->nnz), kT, 0, stream>>>(hg->pins, label, hg->nnz, n_clusters, flags);
    HEF_LAUNCH_CHECK();
    int32_t f = 0;
    HEF_TRY(read_i32(flags, &f, stream));
    if (f) { set_error("a pin's label lies outside [0, n_clusters)"); return HEF_ERR_INVALID_ARGUMENT; }
  }
  HEF_TRY(structure_build(L, st, a, stream));
  int32_t m2 = 0;
  int64_t nnz2 = 0;
  HEF_TRY(rebuild_level(L, st, label, n_clusters, eptr_out, pins_out, w_out, &m2, &nnz2, a, stream,
                        kept_out));
  *m_out = m2;
  *nnz_out = nnz2;
  return HEF_OK;
}

hef_status hef_coarsen(const hef_hypergraph *hg, const hef_params *p, int32_t *cluster,
                       int32_t *n_clusters, float *R0, float *eta, void *ws, size_t ws_bytes,
                       hipStream_t stream) {
  return hef_coarsen_levels(hg, p, cluster, n_clusters, R0, eta, nullptr, ws, ws_bytes, stream);
}

hef_status hef_coarsen_levels(const hef_hypergraph *hg, const hef_params *p, int32_t *cluster,
                              int32_t *n_clusters, float *R0, float *eta,
                              hef_level_trace *trace, void *ws, size_t ws_bytes,
                              hipStream_t stream) {
  if (!hg || !p || !n_clusters || !ws || (hg->n > 0 && !cluster)) {
    set_error("NULL argument");
    return HEF_ERR_INVALID_ARGUMENT;
  }
  if (trace && trace->cap < 0) {
    set_error("trace capacity is negative");
    return HEF_ERR_INVALID_ARGUMENT;
  }
  size_t need = 0;
  HEF_TRY(hef_workspace_size(hg, p, HEF_OP_COARSEN, &need));
  if (ws_bytes < need) { set_error("workspace too small (%zu < %zu)", ws_bytes, need); return HEF_ERR_WORKSPACE_TOO_SMALL; }
  const int64_t n0 = hg->n;
  const int K = pool_width_of(*p);
  const int pt = p->basis == HEF_BASIS_BF16 ? kPoolBF16 : kPoolF32;
  Arena a;
  a.base = static_cast<char *>(ws);
  a.cap = ws_bytes;
  CoarsenWs c;
  carve_coarsen(a, hg->n, hg->m, hg->nnz, *p, c);
  if (a.overflow) { set_error("workspace carve overflow"); return HEF_ERR_WORKSPACE_TOO_SMALL; }
  Level L;
  L.n = hg->n; L.m = hg->m; L.nnz = hg->nnz; L.eptr = hg->eptr; L.pins = hg->pins; L.w = hg->w;
  if (!(p->flags & HEF_FLAG_ASSUME_VALID)) {
    int32_t bad = 0;
    HEF_TRY(validate_device(L, c.flags, &bad, stream));
    if (bad) { set_error("invalid hypergraph (code %d)", bad); return HEF_ERR_INVALID_HYPERGRAPH; }
  }
  if (n0 > 0) {
    k_iota<<<g1(n0), kT, 0, stream>>>(cluster, n0);
    HEF_LAUNCH_CHECK();
  }
  const float *eta_cur = nullptr;
  int cur = 0;
  g_levels_run = 0;
  k_zero_u64<<<1, kT, 0, stream>>>(c.work, kMaxLevelLog);
  HEF_LAUNCH_CHECK();
  if (trace) trace->levels_run = 0;
  // node-reduction target: stop once n_l <= (1 - target_nr) n_0 (0 = off)
  const double n_goal = (1.0 - double(p->target_nr)) * double(n0);
  for (int lev = 0; lev < p->levels && L.m > 0; ++lev) {
    if (p->target_nr > 0.0f && double(L.n) <= n_goal) break;
    if (lev < kMaxLevelLog) {
      g_level_n[lev] = L.n;
      g_level_m[lev] = L.m;
      g_level_nnz[lev] = L.nnz;
      g_levels_run = lev + 1;
    }
    const bool tr = trace && lev < trace->cap;
    if (tr) {
      if (trace->n) trace->n[lev] = L.n;
      if (trace->m) trace->m[lev] = L.m;
      if (trace->nnz) trace->nnz[lev] = L.nnz;
      trace->levels_run = lev + 1;
    }
    HEF_TRY(estimate_level(L, *p, p->seed, lev, nullptr, nullptr, c.st, c.pool, c.pool2, c.qh,
                           c.R, a, stream, (tr && trace->rho) ? trace->rho + int64_t(lev) * K
                                                               : nullptr));
    if (lev == 0 && R0)
      HEF_HIP(hipMemcpyAsync(R0, c.R, sizeof(float) * L.m, hipMemcpyDeviceToDevice, stream));
    if (tr && trace->R && L.m > 0)
      HEF_HIP(hipMemcpyAsync(trace->R + int64_t(lev) * hg->m, c.R, sizeof(float) * L.m,
                             hipMemcpyDeviceToDevice, stream));
    if (tr && trace->qh && K > 0)
      HEF_HIP(hipMemcpyAsync(trace->qh + int64_t(lev) * K, c.qh, sizeof(double) * K,
                             hipMemcpyDeviceToDevice, stream));
    int32_t ng = 0;
    float *eta_next = c.eta[cur];
    HEF_TRY(cluster_one_level(L, c.st, c.R, eta_cur, c.pool, pt, K, c.qh, p->percentile,
                              p->local_clustering != 0, c.label, &ng, eta_next, a, stream,
                              lev < kMaxLevelLog ? c.work + lev : nullptr));
    if (tr && trace->label && L.n > 0)
      HEF_HIP(hipMemcpyAsync(trace->label + int64_t(lev) * n0, c.label, sizeof(int32_t) * L.n,
                             hipMemcpyDeviceToDevice, stream));
    if (tr && trace->eta && ng > 0)
      HEF_HIP(hipMemcpyAsync(trace->eta + int64_t(lev) * n0, eta_next, sizeof(float) * ng,
                             hipMemcpyDeviceToDevice, stream));
    if (n0 > 0) {
      k_compose<<<g1(n0), kT, 0, stream>>>(cluster, c.label, n0);
      HEF_LAUNCH_CHECK();
    }
    int32_t m2 = 0;
    int64_t nnz2 = 0;
    HEF_TRY(rebuild_level(L, c.st, c.label, ng, c.eptr[cur], c.pins[cur], c.w[cur], &m2, &nnz2,
                          a, stream));
    const bool stalled = ng == L.n;  // nothing merged: no further reduction
    L.n = ng;
    L.m = m2;
    L.nnz = nnz2;
    L.eptr = c.eptr[cur];
    L.pins = c.pins[cur];
    L.w = c.w[cur];
    eta_cur = eta_next;
    cur ^= 1;
    if (stalled && p->target_nr > 0.0f) break;
  }
  if (eta && L.n > 0) {
    if (eta_cur)
      HEF_HIP(hipMemcpyAsync(eta, eta_cur, sizeof(float) * L.n, hipMemcpyDeviceToDevice, stream));
    else
      HEF_TRY(zero_async(eta, sizeof(float) * L.n, stream));
  }
  if (g_levels_run > 0) {
    unsigned long long wk[kMaxLevelLog];
    HEF_HIP(hipMemcpyAsync(wk, c.work, sizeof(unsigned long long) * g_levels_run,
                           hipMemcpyDeviceToHost, stream));
    HEF_HIP(hipStreamSynchronize(stream));
    for (int i = 0; i < g_levels_run; ++i) g_level_work[i] = int64_t(wk[i]);
  }
  HEF_HIP(hipStreamSynchronize(stream));
  *n_clusters = L.n;
  return HEF_OK;
}

int32_t hef_last_coarsen_work(int64_t *best_candidates, int32_t cap) {
  const int32_t k = g_levels_run < cap ? g_levels_run : cap;
  for (int32_t i = 0; i < k; ++i)
    if (best_candidates) best_candidates[i] = g_level_work[i];
  return g_levels_run;
}

int32_t hef_last_coarsen_levels(int32_t *n, int32_t *m, int64_t *nnz, int32_t cap) {
  const int32_t k = g_levels_run < cap ? g_levels_run : cap;
  for (int32_t i = 0; i < k; ++i) {
    if (n) n[i] = g_level_n[i];
    if (m) m[i] = g_level_m[i];
    if (nnz) nnz[i] = g_level_nnz[i];
  }
  return g_levels_run;
}


}  // extern "C"

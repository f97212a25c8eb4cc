// Resistance ratios (Eqs. (9), (13), (14); Alg. 1).
//
// For every hyperedge e and pool column i the two most distant pins along
// chi^(i) are its largest and smallest entries, so the numerator of Eq. (13)
// is s_e^(i) = (max_{p in e} chi_p^(i) - min_{p in e} chi_p^(i))^2.
// Pass 1 forms Q_H(chi^(i)) = sum_e w_e s_e^(i) (Eq. (9)) and stores the
// m x K numerators s (float32, row e contiguous); pass 2 streams them back
// to form R_e = max_i s_e^(i) / Q_H(chi^(i)) (Eq. (14)).  Streaming s costs
// 8 K bytes per hyperedge; regathering the pool rows cost about 4 K bytes per
// pin, mostly missed in L2.
//
// A group of LPR lanes handles one hyperedge, each lane CPL consecutive
// columns of the gathered rows; a workgroup walks a contiguous range of
// hyperedges (XCD-contiguous), so neighbouring hyperedges share pool rows
// in L2.  Sums are float64 in a fixed order.
#include <cfloat>
#include <type_traits>

#include "krylov.hpp"
#include "prims.hpp"
#include "score.hpp"

namespace hef {
namespace {

constexpr int kThreads = 256;
constexpr int kEdgesPerBlk = 128;

// Pool values of one type: float64 for the float64 debug basis, else float
// (bfloat16 widens exactly).
template <int PT>
using PoolVal = typename std::conditional<PT == kPoolF64, double, float>::type;

template <int CPL, int PT>
__device__ __forceinline__ void load_cols(const void *pool, int64_t p, int K, int c0,
                                          PoolVal<PT> (&v)[CPL]) {
  if constexpr (PT == kPoolF64) {
    const double *row = reinterpret_cast<const double *>(pool) + p * K + c0;
    if ((K & 1) == 0 && c0 + CPL <= K) {
#pragma unroll
      for (int q = 0; q < CPL; q += 2) {
        const double2 t = *reinterpret_cast<const double2 *>(row + q);
        v[q] = t.x; v[q + 1] = t.y;
      }
    } else {
#pragma unroll
      for (int q = 0; q < CPL; ++q) v[q] = (c0 + q < K) ? row[q] : 0.0;
    }
  } else if (PT == kPoolF32) {
    const float *row = reinterpret_cast<const float *>(pool) + p * K + c0;
    if ((K & 3) == 0 && c0 + CPL <= K) {
#pragma unroll
      for (int q = 0; q < CPL; q += 4) {
        const float4 t = *reinterpret_cast<const float4 *>(row + q);
        v[q] = t.x; v[q + 1] = t.y; v[q + 2] = t.z; v[q + 3] = t.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < CPL; ++q) v[q] = (c0 + q < K) ? row[q] : 0.0f;
    }
  } else {
    const uint16_t *row = reinterpret_cast<const uint16_t *>(pool) + p * K + c0;
    if ((K & 3) == 0 && c0 + CPL <= K) {
#pragma unroll
      for (int q = 0; q < CPL; q += 4) {
        const uint2 t = *reinterpret_cast<const uint2 *>(row + q);
        v[q] = __uint_as_float(t.x << 16);
        v[q + 1] = __uint_as_float(t.x & 0xFFFF0000u);
        v[q + 2] = __uint_as_float(t.y << 16);
        v[q + 3] = __uint_as_float(t.y & 0xFFFF0000u);
      }
    } else {
#pragma unroll
      for (int q = 0; q < CPL; ++q)
        v[q] = (c0 + q < K) ? __uint_as_float(uint32_t(row[q]) << 16) : 0.0f;
    }
  }
}

// Spread of hyperedge [a, b) of pins over this lane's columns.  Pins go in
// chunks of 4 (ids first, then rows, so the loads overlap); a chunk past the
// end repeats the last pin, which leaves max and min unchanged.
__device__ __forceinline__ float vmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ float vmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ double vmin(double a, double b) { return fmin(a, b); }

template <int CPL, int PT>
__device__ __forceinline__ void edge_spread(const int32_t *__restrict__ pins, const void *pool,
                                            int K, int c0, int32_t a, int32_t b,
                                            double (&s)[CPL]) {
  using T = PoolVal<PT>;
  constexpr T kBig = PT == kPoolF64 ? T(DBL_MAX) : T(FLT_MAX);
  T mx[CPL], mn[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) { mx[q] = -kBig; mn[q] = kBig; }
  for (int32_t j0 = a; j0 < b; j0 += 4) {
    int32_t pp[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) pp[u] = pins[j0 + u < b ? j0 + u : b - 1];
    T v[4][CPL];
#pragma unroll
    for (int u = 0; u < 4; ++u) load_cols<CPL, PT>(pool, pp[u], K, c0, v[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < CPL; ++q) { mx[q] = vmax(mx[q], v[u][q]); mn[q] = vmin(mn[q], v[u][q]); }
  }
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const double d = double(mx[q]) - double(mn[q]);
    s[q] = d * d;
  }
}

// A workgroup takes kEdgesPerBlk consecutive hyperedges [e0, e1); group grp
// (LPR lanes, ngrp groups) takes e0 + grp + ngrp k, in rounds of LPR: lane j
// of the group fetches the pin range of the round's j-th hyperedge up front.
template <int CPL, int PT>
__global__ void __launch_bounds__(kThreads)
k_score_qh(const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins,
           const float *__restrict__ w, const void *__restrict__ pool, int K, int LPR,
           int64_t m, double *__restrict__ partial, float *__restrict__ sbuf) {
  __shared__ double comb[512];
  const int tid = threadIdx.x;
  const int ngrp = kThreads / LPR;
  const int grp = tid / LPR;
  const int sub = tid % LPR;
  const int c0 = sub * CPL;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t e0 = blk * kEdgesPerBlk;
  const int64_t e1 = e0 + kEdgesPerBlk < m ? e0 + kEdgesPerBlk : m;
  double acc[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q] = 0.0;
  for (int k0 = 0; k0 < kEdgesPerBlk / ngrp && e0 + grp + int64_t(ngrp) * k0 < e1; k0 += LPR) {
    int32_t ea = 0, eb = 0;
    float ew = 0.0f;
    {
      const int64_t e = e0 + grp + int64_t(ngrp) * (k0 + sub);
      if (e < e1) {
        ea = eptr[e];
        eb = eptr[e + 1];
        ew = w ? w[e] : 1.0f;
      }
    }
    for (int k = 0; k < LPR && e0 + grp + int64_t(ngrp) * (k0 + k) < e1; ++k) {
      const int32_t a = __shfl(ea, k, LPR), b = __shfl(eb, k, LPR);
      const double we = double(__shfl(ew, k, LPR));
      if (c0 < K) {
        double s[CPL];
        edge_spread<CPL, PT>(pins, pool, K, c0, a, b, s);
#pragma unroll
        for (int q = 0; q < CPL; ++q) acc[q] = fma(we, s[q], acc[q]);
        float *out = sbuf + (e0 + grp + int64_t(ngrp) * (k0 + k)) * K + c0;
        if (c0 + CPL <= K && (K & 3) == 0) {
#pragma unroll
          for (int q = 0; q < CPL; q += 4)
            *reinterpret_cast<float4 *>(out + q) =
                make_float4(float(s[q]), float(s[q + 1]), float(s[q + 2]), float(s[q + 3]));
        } else {
#pragma unroll
          for (int q = 0; q < CPL; ++q)
            if (c0 + q < K) out[q] = float(s[q]);
        }
      }
    }
  }
  for (int g = 0; g < ngrp; ++g) {
    if (grp == g && c0 < K) {
#pragma unroll
      for (int q = 0; q < CPL; ++q)
        if (c0 + q < K) comb[c0 + q] = (g == 0) ? acc[q] : comb[c0 + q] + acc[q];
    }
    __syncthreads();
  }
  for (int c = tid; c < K; c += kThreads) partial[blk * K + c] = comb[c];
}

// R_e = max_i s_e^(i) / Q_H^(i) from the stored numerators: LPR lanes per
// hyperedge, CPL columns each (ties in the maximum are irrelevant: only the
// value is kept).
template <int CPL>
__global__ void __launch_bounds__(kThreads)
k_score_r(const float *__restrict__ sbuf, int K, int LPR, int64_t m,
          const double *__restrict__ qh, float *__restrict__ R) {
  const int tid = threadIdx.x;
  const int ngrp = kThreads / LPR;
  const int grp = tid / LPR;
  const int sub = tid % LPR;
  const int c0 = sub * CPL;
  double inv[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const double qv = (c0 + q < K) ? qh[c0 + q] : 0.0;
    inv[q] = qv > 0.0 ? 1.0 / qv : 0.0;
  }
  const int64_t e0 = int64_t(xcd_block(blockIdx.x, gridDim.x)) * kEdgesPerBlk;
  const int64_t e1 = e0 + kEdgesPerBlk < m ? e0 + kEdgesPerBlk : m;
  for (int64_t e = e0 + grp; e < e1; e += ngrp) {
    double best = 0.0;
    if (c0 < K) {
      const float *row = sbuf + e * K + c0;
      float v[CPL];
      if (c0 + CPL <= K && (K & 3) == 0) {
#pragma unroll
        for (int q = 0; q < CPL; q += 4) {
          const float4 t = *reinterpret_cast<const float4 *>(row + q);
          v[q] = t.x; v[q + 1] = t.y; v[q + 2] = t.z; v[q + 3] = t.w;
        }
      } else {
#pragma unroll
        for (int q = 0; q < CPL; ++q) v[q] = c0 + q < K ? row[q] : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < CPL; ++q) best = fmax(best, double(v[q]) * inv[q]);
    }
    for (int off = LPR / 2; off > 0; off >>= 1) best = fmax(best, __shfl_xor(best, off, LPR));
    if (sub == 0) R[e] = float(best);
  }
}

int lanes_for(int K, int CPL) {
  int need = (K + CPL - 1) / CPL;
  int l = 1;
  while (l < need) l <<= 1;
  return l;
}

template <int CPL, int PT>
hef_status score_t(const Level &L, const void *pool, int K, double *qh, float *R,
                   double *partial, float *sbuf, int64_t nblk, hipStream_t s) {
  const int LPR = lanes_for(K, CPL);
  {
  TimedScope ts(kStScoreQ, s);
  k_score_qh<CPL, PT><<<nblk, kThreads, 0, s>>>(L.eptr, L.pins, L.w, pool, K, LPR, L.m, partial,
                                                sbuf);
  HEF_LAUNCH_CHECK();
  }
  {
  TimedScope ts(kStScoreReduce, s);
  HEF_TRY(reduce_cols_f64(partial, nblk, K, qh, s));
  }
  TimedScope ts(kStScoreR, s);
  k_score_r<CPL><<<nblk, kThreads, 0, s>>>(sbuf, K, LPR, L.m, qh, R);
  HEF_LAUNCH_CHECK();
  return HEF_OK;
}

}  // namespace

size_t score_ws_bytes(int64_t m, int K) {
  Arena a;
  a.take<double>(cdiv(std::max<int64_t>(m, 1), kEdgesPerBlk) * K);
  a.take<float>(std::max<int64_t>(m, 1) * K);
  return a.mark();
}

hef_status score_pool(const Level &L, const void *pool, int pool_type, int K, double *qh,
                      float *R, Arena &ws, hipStream_t s, float *keep_s) {
  if (K > 512) return HEF_ERR_UNSUPPORTED;
  if (L.m == 0) return HEF_OK;
  const int64_t nblk = cdiv(L.m, kEdgesPerBlk);
  const size_t mk = ws.mark();
  double *partial = ws.take<double>(nblk * K);
  float *sbuf = keep_s ? keep_s : ws.take<float>(int64_t(L.m) * K);
  HEF_WS_CHECK(ws);
  hef_status st;
  const bool wide = K > 256;
  if (pool_type == kPoolF32)
    st = wide ? score_t<8, kPoolF32>(L, pool, K, qh, R, partial, sbuf, nblk, s)
              : score_t<4, kPoolF32>(L, pool, K, qh, R, partial, sbuf, nblk, s);
  else if (pool_type == kPoolF64)
    st = wide ? score_t<8, kPoolF64>(L, pool, K, qh, R, partial, sbuf, nblk, s)
              : score_t<4, kPoolF64>(L, pool, K, qh, R, partial, sbuf, nblk, s);
  else
    st = wide ? score_t<8, kPoolBF16>(L, pool, K, qh, R, partial, sbuf, nblk, s)
              : score_t<4, kPoolBF16>(L, pool, K, qh, R, partial, sbuf, nblk, s);
  ws.reset(mk);
  return st;
}

}  // namespace hef

// Fused implicit SpMM of the normalised star and clique adjacencies
// (Section III-A: G_b with z_b(e,p) = w_e/|e|, G_c with
// z_c(u,v) = sum_e w_e / C(|e|,2); A = D^-1/2 W D^-1/2).  Neither expansion
// is materialised: a CSR pass over hyperedges gathers node rows, a CSC pass
// over nodes gathers hyperedge rows.  Both passes gather one interleaved
// row of 2B floats per incidence: U[p] = [s_p x_V[p] | s_p x_c[p]] (scaled
// node rows, written by a short prep pass) and W[e] = [alpha_e x_E[e] | T_e]
// (written by the CSR pass), so each incidence costs one 8B-byte gather and
// no scale gathers.  Segments up to kSmallSeg go to lane groups (2B/CH
// lanes per segment, one lane per CH-float chunk of a row); longer segments
// get one wave each.
#include "krylov.hpp"

namespace hef {
namespace {

template <int CH>
__device__ __forceinline__ void load_ch(const float *p, float (&v)[CH]) {
  if constexpr (CH == 4) {
    const float4 t = *reinterpret_cast<const float4 *>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  } else if constexpr (CH == 2) {
    const float2 t = *reinterpret_cast<const float2 *>(p);
    v[0] = t.x; v[1] = t.y;
  } else {
    v[0] = *p;
  }
}

template <int CH>
__device__ __forceinline__ void store_ch(float *p, const float (&v)[CH]) {
  if constexpr (CH == 4) {
    *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
  } else if constexpr (CH == 2) {
    *reinterpret_cast<float2 *>(p) = make_float2(v[0], v[1]);
  } else {
    *p = v[0];
  }
}

template <int B>
struct Geo {
  static constexpr int CH = B < 4 ? B : 4;  // floats per lane
  static constexpr int NCH = B / CH;        // lanes per B-float half row
  static constexpr int LPS = 2 * NCH;       // lanes per 2B-float row
  static constexpr int RW = 2 * B;          // interleaved row width
};

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kBigGrid = 2048;

// U[p] = [s_p xs[p] | s_p xc[p]] (node rows; a missing expansion gives zeros).
template <int B>
__global__ void __launch_bounds__(kThreads)
k_prep(int64_t n, const float *__restrict__ s, const float *__restrict__ xs,
       const float *__restrict__ xc, float *__restrict__ U) {
  using G = Geo<B>;
  const int64_t g = int64_t(xcd_block(blockIdx.x, gridDim.x)) * kThreads + threadIdx.x;
  const int64_t p = g / G::LPS;
  const int sub = int(g % G::LPS);
  if (p >= n) return;
  const int vec = sub / G::NCH, ch = sub % G::NCH;
  const float *x = vec == 0 ? xs : xc;
  float v[G::CH];
  if (x) {
    load_ch<G::CH>(x + p * B + ch * G::CH, v);
    const float sp = s[p];
#pragma unroll
    for (int c = 0; c < G::CH; ++c) v[c] *= sp;
  } else {
#pragma unroll
    for (int c = 0; c < G::CH; ++c) v[c] = 0.0f;
  }
  store_ch<G::CH>(U + p * G::RW + sub * G::CH, v);
}

// ---- CSR pass: per hyperedge e (lane sub < NCH: star, else clique) -------
//   star:   yE[e] = alpha_e * sum_{p in e} U_star[p];  W_star[e] = alpha_e xE[e]
//   clique: W_T[e] = T_e = beta_e * sum_{p in e} U_clique[p]
// The per-hyperedge inputs of the finish (alpha_e and this lane's chunk of
// xE[e], or beta_e), loaded before the gather so their latency overlaps it.
template <int B>
struct CsrIn {
  float f;
  float xv[Geo<B>::CH];
  __device__ __forceinline__ void load(int64_t e, int sub, const float *__restrict__ alpha,
                                       const float *__restrict__ beta,
                                       const float *__restrict__ xE) {
    using G = Geo<B>;
    const int vec = sub / G::NCH, ch = sub % G::NCH;
    if (vec == 0) {
      f = alpha[e];
      load_ch<G::CH>(xE + e * B + ch * G::CH, xv);
    } else {
      f = beta[e];
#pragma unroll
      for (int c = 0; c < G::CH; ++c) xv[c] = 0.0f;
    }
  }
};

template <int B>
__device__ __forceinline__ void csr_finish(int64_t e, int sub, const float (&acc)[Geo<B>::CH],
                                           const CsrIn<B> &in, float *__restrict__ yE,
                                           float *__restrict__ W) {
  using G = Geo<B>;
  const int vec = sub / G::NCH, ch = sub % G::NCH;
  float out[G::CH];
  if (vec == 0) {
    const float a = in.f;
#pragma unroll
    for (int c = 0; c < G::CH; ++c) out[c] = a * acc[c];
    store_ch<G::CH>(yE + e * B + ch * G::CH, out);
    float xv[G::CH];
#pragma unroll
    for (int c = 0; c < G::CH; ++c) xv[c] = in.xv[c] * a;
    store_ch<G::CH>(W + e * G::RW + ch * G::CH, xv);
  } else {
    const float bt = in.f;
#pragma unroll
    for (int c = 0; c < G::CH; ++c) out[c] = bt * acc[c];
    store_ch<G::CH>(W + e * G::RW + B + ch * G::CH, out);
  }
}

template <int B>
__device__ __forceinline__ void
csr_small(int64_t blk, const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins,
          const float *__restrict__ U, const float *__restrict__ alpha,
          const float *__restrict__ beta, const float *__restrict__ xE,
          float *__restrict__ yE, float *__restrict__ W, int32_t m, int on_mask) {
  using G = Geo<B>;
  const int64_t g = blk * kThreads + threadIdx.x;
  const int64_t e = g / G::LPS;
  const int sub = int(g % G::LPS);
  if (e >= m) return;
  if (!((on_mask >> (sub / G::NCH)) & 1)) return;
  const int32_t a = eptr[e], b = eptr[e + 1];
  if (b - a > kSmallSeg) return;
  CsrIn<B> in;
  in.load(e, sub, alpha, beta, xE);
  float acc[G::CH];
#pragma unroll
  for (int c = 0; c < G::CH; ++c) acc[c] = 0.0f;
  // chunks of 8 pins: all ids first, then all rows, so the loads overlap
  for (int32_t j0 = a; j0 < b; j0 += 8) {
    int32_t pp[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) pp[u] = (j0 + u < b) ? pins[j0 + u] : -1;
    float v[8][G::CH];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (pp[u] >= 0) {
        load_ch<G::CH>(U + int64_t(pp[u]) * G::RW + sub * G::CH, v[u]);
      } else {
#pragma unroll
        for (int c = 0; c < G::CH; ++c) v[u][c] = 0.0f;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int c = 0; c < G::CH; ++c) acc[c] += v[u][c];
  }
  csr_finish<B>(e, sub, acc, in, yE, W);
}

// One wave per long hyperedge: 64/LPS slots stride over its pins, then a
// fixed xor tree across slots.
template <int B>
__device__ __forceinline__ void
csr_big(int bx, int nbx, const int32_t *__restrict__ list, const int32_t *__restrict__ count,
        const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins,
        const float *__restrict__ U, const float *__restrict__ alpha,
        const float *__restrict__ beta, const float *__restrict__ xE,
        float *__restrict__ yE, float *__restrict__ W, int on_mask) {
  using G = Geo<B>;
  constexpr int SLOTS = 64 / G::LPS;
  const int lane = threadIdx.x & 63;
  const int slot = lane / G::LPS;
  const int sub = lane % G::LPS;
  const bool on = (on_mask >> (sub / G::NCH)) & 1;
  const int32_t cnt = *count;
  for (int32_t bi = bx * kWaves + (threadIdx.x >> 6); bi < cnt; bi += nbx * kWaves) {
    const int32_t e = list[bi];
    const int32_t a = eptr[e], b = eptr[e + 1];
    CsrIn<B> in;
    if (slot == 0 && on) in.load(e, sub, alpha, beta, xE);
    float acc[G::CH];
#pragma unroll
    for (int c = 0; c < G::CH; ++c) acc[c] = 0.0f;
    if (on) {
      // 8 incidences per slot in flight: ids first, then rows
      for (int32_t j0 = a + slot; j0 < b; j0 += 8 * SLOTS) {
        int32_t pp[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) pp[q] = (j0 + q * SLOTS < b) ? pins[j0 + q * SLOTS] : -1;
        float v[8][G::CH];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (pp[q] >= 0) {
            load_ch<G::CH>(U + int64_t(pp[q]) * G::RW + sub * G::CH, v[q]);
          } else {
#pragma unroll
            for (int c = 0; c < G::CH; ++c) v[q][c] = 0.0f;
          }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
          for (int c = 0; c < G::CH; ++c) acc[c] += v[q][c];
      }
    }
#pragma unroll
    for (int off = 32; off >= G::LPS; off >>= 1)
#pragma unroll
      for (int c = 0; c < G::CH; ++c) acc[c] += __shfl_xor(acc[c], off, 64);
    if (slot == 0 && on) csr_finish<B>(e, sub, acc, in, yE, W);
  }
}

// ---- CSC pass: per node u ---------------------------------------------------
//   star:   yV[u] = s_u * sum_{e ∋ u} W_star[e]
//   clique: yc[u] = s_u * sum_{e ∋ u} W_T[e] - gam_u xc[u]
// The per-node inputs of the finish (s_u, and gamma_u with this lane's chunk
// of xc[u] for the clique half), loaded before the gather.
template <int B>
struct CscIn {
  float su, gu;
  float own[Geo<B>::CH];
  __device__ __forceinline__ void load(int64_t u, int sub, const float *__restrict__ s,
                                       const float *__restrict__ gam,
                                       const float *__restrict__ xc) {
    using G = Geo<B>;
    const int vec = sub / G::NCH, ch = sub % G::NCH;
    su = s[u];
    if (vec == 0) {
      gu = 0.0f;
#pragma unroll
      for (int c = 0; c < G::CH; ++c) own[c] = 0.0f;
    } else {
      gu = gam[u];
      load_ch<G::CH>(xc + u * B + ch * G::CH, own);
    }
  }
};

template <int B>
__device__ __forceinline__ void csc_finish(int64_t u, int sub, const float (&acc)[Geo<B>::CH],
                                           const CscIn<B> &in, float *__restrict__ yV,
                                           float *__restrict__ yc) {
  using G = Geo<B>;
  const int vec = sub / G::NCH, ch = sub % G::NCH;
  const float su = in.su;
  float out[G::CH];
  if (vec == 0) {
#pragma unroll
    for (int c = 0; c < G::CH; ++c) out[c] = su * acc[c];
    store_ch<G::CH>(yV + u * B + ch * G::CH, out);
  } else {
    const float gu = in.gu;
#pragma unroll
    for (int c = 0; c < G::CH; ++c) out[c] = su * acc[c] - gu * in.own[c];
    store_ch<G::CH>(yc + u * B + ch * G::CH, out);
  }
}

template <int B>
__device__ __forceinline__ void
csc_small(int64_t blk, const int32_t *__restrict__ vptr, const int32_t *__restrict__ eids,
          const float *__restrict__ W, const float *__restrict__ s,
          const float *__restrict__ gam, const float *__restrict__ xc,
          float *__restrict__ yV, float *__restrict__ yc, int32_t n, int on_mask) {
  using G = Geo<B>;
  const int64_t g = blk * kThreads + threadIdx.x;
  const int64_t u = g / G::LPS;
  const int sub = int(g % G::LPS);
  if (u >= n) return;
  if (!((on_mask >> (sub / G::NCH)) & 1)) return;
  const int32_t a = vptr[u], b = vptr[u + 1];
  if (b - a > kSmallSeg) return;
  CscIn<B> in;
  in.load(u, sub, s, gam, xc);
  float acc[G::CH];
#pragma unroll
  for (int c = 0; c < G::CH; ++c) acc[c] = 0.0f;
  // chunks of 8 hyperedges: all ids first, then all rows
  for (int32_t j0 = a; j0 < b; j0 += 8) {
    int32_t ee[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) ee[q] = (j0 + q < b) ? eids[j0 + q] : -1;
    float v[8][G::CH];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (ee[q] >= 0) {
        load_ch<G::CH>(W + int64_t(ee[q]) * G::RW + sub * G::CH, v[q]);
      } else {
#pragma unroll
        for (int c = 0; c < G::CH; ++c) v[q][c] = 0.0f;
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int c = 0; c < G::CH; ++c) acc[c] += v[q][c];
  }
  csc_finish<B>(u, sub, acc, in, yV, yc);
}

template <int B>
__device__ __forceinline__ void
csc_big(int bx, int nbx, const int32_t *__restrict__ list, const int32_t *__restrict__ count,
        const int32_t *__restrict__ vptr, const int32_t *__restrict__ eids,
        const float *__restrict__ W, const float *__restrict__ s,
        const float *__restrict__ gam, const float *__restrict__ xc,
        float *__restrict__ yV, float *__restrict__ yc, int on_mask) {
  using G = Geo<B>;
  constexpr int SLOTS = 64 / G::LPS;
  const int lane = threadIdx.x & 63;
  const int slot = lane / G::LPS;
  const int sub = lane % G::LPS;
  const bool on = (on_mask >> (sub / G::NCH)) & 1;
  const int32_t cnt = *count;
  for (int32_t bi = bx * kWaves + (threadIdx.x >> 6); bi < cnt; bi += nbx * kWaves) {
    const int32_t u = list[bi];
    const int32_t a = vptr[u], b = vptr[u + 1];
    CscIn<B> in;
    if (slot == 0 && on) in.load(u, sub, s, gam, xc);
    float acc[G::CH];
#pragma unroll
    for (int c = 0; c < G::CH; ++c) acc[c] = 0.0f;
    if (on) {
      for (int32_t j0 = a + slot; j0 < b; j0 += 8 * SLOTS) {
        int32_t ee[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) ee[q] = (j0 + q * SLOTS < b) ? eids[j0 + q * SLOTS] : -1;
        float v[8][G::CH];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (ee[q] >= 0) {
            load_ch<G::CH>(W + int64_t(ee[q]) * G::RW + sub * G::CH, v[q]);
          } else {
#pragma unroll
            for (int c = 0; c < G::CH; ++c) v[q][c] = 0.0f;
          }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
          for (int c = 0; c < G::CH; ++c) acc[c] += v[q][c];
      }
    }
#pragma unroll
    for (int off = 32; off >= G::LPS; off >>= 1)
#pragma unroll
      for (int c = 0; c < G::CH; ++c) acc[c] += __shfl_xor(acc[c], off, 64);
    if (slot == 0 && on) csc_finish<B>(u, sub, acc, in, yV, yc);
  }
}

// One launch per pass: workgroups [0, kBigGrid) walk the long segments (one
// wave each), the rest take the short ones (kBigGrid is a multiple of 8, so
// a workgroup's XCD is the same in both numberings).  Up to b = 8 the pass
// is held to 64 VGPRs, i.e. 8 waves per SIMD for its gathers (one register
// more would leave 7).
template <int B>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(B <= 8 ? 8 : 1, 8)))
k_csr(const int32_t *__restrict__ big_e, const int32_t *__restrict__ n_big,
      const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins,
      const float *__restrict__ U, const float *__restrict__ alpha,
      const float *__restrict__ beta, const float *__restrict__ xE, float *__restrict__ yE,
      float *__restrict__ W, int32_t m, int on_mask) {
  if (int(blockIdx.x) < kBigGrid) {
    csr_big<B>(int(blockIdx.x), kBigGrid, big_e, n_big, eptr, pins, U, alpha, beta, xE, yE, W,
               on_mask);
  } else {
    const int64_t nsmall = int64_t(gridDim.x) - kBigGrid;
    csr_small<B>(xcd_block(int64_t(blockIdx.x) - kBigGrid, nsmall), eptr, pins, U, alpha, beta,
                 xE, yE, W, m, on_mask);
  }
}

template <int B>
__global__ void __launch_bounds__(kThreads)
k_csc(const int32_t *__restrict__ big_v, const int32_t *__restrict__ n_big_v,
      const int32_t *__restrict__ vptr, const int32_t *__restrict__ eids,
      const float *__restrict__ W, const float *__restrict__ s, const float *__restrict__ gam,
      const float *__restrict__ xc, float *__restrict__ yV, float *__restrict__ yc, int32_t n,
      int on_mask) {
  if (int(blockIdx.x) < kBigGrid) {
    csc_big<B>(int(blockIdx.x), kBigGrid, big_v, n_big_v, vptr, eids, W, s, gam, xc, yV, yc,
               on_mask);
  } else {
    const int64_t nsmall = int64_t(gridDim.x) - kBigGrid;
    csc_small<B>(xcd_block(int64_t(blockIdx.x) - kBigGrid, nsmall), vptr, eids, W, s, gam, xc,
                 yV, yc, n, on_mask);
  }
}

static_assert(kBigGrid % 8 == 0, "the XCD of a workgroup must not depend on its role");

template <int B>
hef_status spmm_t(const Level &L, const Structure &st, const float *xs, float *ys,
                  const float *xc, float *yc, float *scratch, hipStream_t s) {
  using G = Geo<B>;
  const int64_t n = L.n, m = L.m;
  const float *xE = xs ? xs + n * B : nullptr;
  float *yE = ys ? ys + n * B : nullptr;
  float *W = scratch;
  float *U = scratch + m * G::RW;
  const int on = (xs ? 1 : 0) | (xc ? 2 : 0);
  TimedScope step(kStSpmmStep, s);
  if (n > 0) {
    TimedScope ts(kStSpmmPrep, s);
    k_prep<B><<<cdiv(n * G::LPS, kThreads), kThreads, 0, s>>>(n, st.s, xs, xc, U);
    HEF_LAUNCH_CHECK();
  }
  if (m > 0) {
    const int64_t nb = cdiv(m * G::LPS, kThreads);
    TimedScope ts(kStSpmmCsr, s);
    k_csr<B><<<kBigGrid + nb, kThreads, 0, s>>>(st.big_e, st.n_big, L.eptr, L.pins, U, st.alpha,
                                                st.beta, xE, yE, W, int32_t(m), on);
    HEF_LAUNCH_CHECK();
  }
  if (n > 0) {
    const int64_t nb = cdiv(n * G::LPS, kThreads);
    TimedScope ts(kStSpmmCsc, s);
    k_csc<B><<<kBigGrid + nb, kThreads, 0, s>>>(st.big_v, st.n_big + 1, st.vptr, st.eids, W, st.s,
                                                st.gam, xc, ys, yc, int32_t(n), on);
    HEF_LAUNCH_CHECK();
  }
  return HEF_OK;
}

}  // namespace

hef_status spmm_apply(const Level &L, const Structure &st, int B, const float *xs, float *ys,
                      const float *xc, float *yc, float *scratch, hipStream_t s) {
  switch (B) {
    case 1: return spmm_t<1>(L, st, xs, ys, xc, yc, scratch, s);
    case 2: return spmm_t<2>(L, st, xs, ys, xc, yc, scratch, s);
    case 4: return spmm_t<4>(L, st, xs, ys, xc, yc, scratch, s);
    case 8: return spmm_t<8>(L, st, xs, ys, xc, yc, scratch, s);
    case 16: return spmm_t<16>(L, st, xs, ys, xc, yc, scratch, s);
    default: set_error("block width %d is not a power of two in 1..16", B);
             return HEF_ERR_UNSUPPORTED;
  }
}

}  // namespace hef

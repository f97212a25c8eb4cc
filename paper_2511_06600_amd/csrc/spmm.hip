// Fused implicit SpMM of the normalised star and clique adjacencies
// (Section III-A: G_b with z_b(e,p) = w_e/|e|, G_c with
// z_c(u,v) = sum_e w_e / C(|e|,2); A = D^-1/2 W D^-1/2).  Neither expansion
// is materialised: a CSR pass over hyperedges gathers node rows, a CSC pass
// over nodes gathers hyperedge rows.  Segments up to kSmallSeg pins go to
// lane groups (one group of 2*B/CH lanes per segment, one lane per CH-float
// chunk of a row); longer segments get a whole workgroup.
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
  static constexpr int NCH = B / CH;        // lanes per vector row
  static constexpr int LPS = 2 * NCH;       // lanes per segment (2 vectors)
};

constexpr int kThreads = 256;
constexpr int kBigGrid = 1024;

// ---- CSR pass: per hyperedge e ------------------------------------------
// vec 0 (star):   yE[e] = alpha_e * sum_{p in e} s_p xs[p]
// vec 1 (clique): tb[e] = beta_e  * sum_{p in e} s_p xc[p]
template <int B>
__global__ void __launch_bounds__(kThreads)
k_csr_small(const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins,
            const float *__restrict__ s, const float *__restrict__ alpha,
            const float *__restrict__ beta, const float *__restrict__ xs,
            const float *__restrict__ xc, float *__restrict__ yE, float *__restrict__ tb,
            int32_t m) {
  using G = Geo<B>;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t g = blk * kThreads + threadIdx.x;
  const int64_t e = g / G::LPS;
  const int sub = int(g % G::LPS);
  if (e >= m) return;
  const int vec = sub / G::NCH;
  const int ch = sub % G::NCH;
  const float *x = vec == 0 ? xs : xc;
  if (x == nullptr) return;
  const int32_t a = eptr[e], b = eptr[e + 1];
  if (b - a > kSmallSeg) return;
  float acc[G::CH];
#pragma unroll
  for (int c = 0; c < G::CH; ++c) acc[c] = 0.0f;
  // chunks of 8 pins: all ids first, then all rows, so the loads overlap
  for (int32_t j0 = a; j0 < b; j0 += 8) {
    int32_t pp[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) pp[u] = (j0 + u < b) ? pins[j0 + u] : -1;
    float sp[8], v[8][G::CH];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (pp[u] >= 0) {
        sp[u] = s[pp[u]];
        load_ch<G::CH>(x + int64_t(pp[u]) * B + ch * G::CH, v[u]);
      } else {
        sp[u] = 0.0f;
#pragma unroll
        for (int c = 0; c < G::CH; ++c) v[u][c] = 0.0f;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int c = 0; c < G::CH; ++c) acc[c] = fmaf(sp[u], v[u][c], acc[c]);
  }
  const float f = vec == 0 ? alpha[e] : beta[e];
#pragma unroll
  for (int c = 0; c < G::CH; ++c) acc[c] *= f;
  store_ch<G::CH>((vec == 0 ? yE : tb) + e * B + ch * G::CH, acc);
}

template <int B>
__global__ void __launch_bounds__(kThreads)
k_csr_big(const int32_t *__restrict__ list, const int32_t *__restrict__ count,
          const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins,
          const float *__restrict__ s, const float *__restrict__ alpha,
          const float *__restrict__ beta, const float *__restrict__ xs,
          const float *__restrict__ xc, float *__restrict__ yE, float *__restrict__ tb) {
  using G = Geo<B>;
  constexpr int SLOTS = kThreads / G::LPS;
  __shared__ float red[kThreads * G::CH];
  const int tid = threadIdx.x;
  const int slot = tid / G::LPS;
  const int sub = tid % G::LPS;
  const int vec = sub / G::NCH;
  const int ch = sub % G::NCH;
  const float *x = vec == 0 ? xs : xc;
  const int32_t cnt = *count;
  for (int32_t bi = blockIdx.x; bi < cnt; bi += gridDim.x) {
    const int32_t e = list[bi];
    const int32_t a = eptr[e], b = eptr[e + 1];
    float acc[G::CH];
#pragma unroll
    for (int c = 0; c < G::CH; ++c) acc[c] = 0.0f;
    if (x != nullptr) {
      for (int32_t j = a + slot; j < b; j += SLOTS) {
        const int32_t p = pins[j];
        const float sp = s[p];
        float v[G::CH];
        load_ch<G::CH>(x + int64_t(p) * B + ch * G::CH, v);
#pragma unroll
        for (int c = 0; c < G::CH; ++c) acc[c] = fmaf(sp, v[c], acc[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < G::CH; ++c) red[tid * G::CH + c] = acc[c];
    __syncthreads();
    for (int stride = SLOTS / 2; stride > 0; stride >>= 1) {
      if (slot < stride) {
#pragma unroll
        for (int c = 0; c < G::CH; ++c)
          red[tid * G::CH + c] += red[(tid + stride * G::LPS) * G::CH + c];
      }
      __syncthreads();
    }
    if (slot == 0 && x != nullptr) {
      float out[G::CH];
      const float f = vec == 0 ? alpha[e] : beta[e];
#pragma unroll
      for (int c = 0; c < G::CH; ++c) out[c] = red[tid * G::CH + c] * f;
      store_ch<G::CH>((vec == 0 ? yE : tb) + int64_t(e) * B + ch * G::CH, out);
    }
    __syncthreads();
  }
}

// ---- CSC pass: per node u -----------------------------------------------
// vec 0 (star):   yV[u] = s_u * sum_{e ∋ u} alpha_e xE[e]
// vec 1 (clique): yc[u] = s_u * sum_{e ∋ u} tb[e] - gam_u xc[u]
template <int B>
__global__ void __launch_bounds__(kThreads)
k_csc_small(const int32_t *__restrict__ vptr, const int32_t *__restrict__ eids,
            const float *__restrict__ s, const float *__restrict__ gam,
            const float *__restrict__ alpha, const float *__restrict__ xE,
            const float *__restrict__ tb, const float *__restrict__ xc,
            float *__restrict__ yV, float *__restrict__ yc, int32_t n) {
  using G = Geo<B>;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t g = blk * kThreads + threadIdx.x;
  const int64_t u = g / G::LPS;
  const int sub = int(g % G::LPS);
  if (u >= n) return;
  const int vec = sub / G::NCH;
  const int ch = sub % G::NCH;
  if (vec == 0 ? (xE == nullptr) : (xc == nullptr)) return;
  const int32_t a = vptr[u], b = vptr[u + 1];
  if (b - a > kSmallSeg) return;
  float acc[G::CH];
#pragma unroll
  for (int c = 0; c < G::CH; ++c) acc[c] = 0.0f;
  // chunks of 8 hyperedges: all ids first, then all rows
  for (int32_t j0 = a; j0 < b; j0 += 8) {
    int32_t ee[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) ee[u] = (j0 + u < b) ? eids[j0 + u] : -1;
    float f[8], v[8][G::CH];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (ee[u] >= 0) {
        f[u] = vec == 0 ? alpha[ee[u]] : 1.0f;
        load_ch<G::CH>((vec == 0 ? xE : tb) + int64_t(ee[u]) * B + ch * G::CH, v[u]);
      } else {
        f[u] = 0.0f;
#pragma unroll
        for (int c = 0; c < G::CH; ++c) v[u][c] = 0.0f;
      }
    }
    if (vec == 0) {
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int c = 0; c < G::CH; ++c) acc[c] = fmaf(f[u], v[u][c], acc[c]);
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int c = 0; c < G::CH; ++c) acc[c] += v[u][c];
    }
  }
  const float su = s[u];
  float out[G::CH];
  if (vec == 0) {
#pragma unroll
    for (int c = 0; c < G::CH; ++c) out[c] = su * acc[c];
    store_ch<G::CH>(yV + u * B + ch * G::CH, out);
  } else {
    const float gu = gam[u];
    float own[G::CH];
    load_ch<G::CH>(xc + u * B + ch * G::CH, own);
#pragma unroll
    for (int c = 0; c < G::CH; ++c) out[c] = su * acc[c] - gu * own[c];
    store_ch<G::CH>(yc + u * B + ch * G::CH, out);
  }
}

template <int B>
__global__ void __launch_bounds__(kThreads)
k_csc_big(const int32_t *__restrict__ list, const int32_t *__restrict__ count,
          const int32_t *__restrict__ vptr, const int32_t *__restrict__ eids,
          const float *__restrict__ s, const float *__restrict__ gam,
          const float *__restrict__ alpha, const float *__restrict__ xE,
          const float *__restrict__ tb, const float *__restrict__ xc,
          float *__restrict__ yV, float *__restrict__ yc) {
  using G = Geo<B>;
  constexpr int SLOTS = kThreads / G::LPS;
  __shared__ float red[kThreads * G::CH];
  const int tid = threadIdx.x;
  const int slot = tid / G::LPS;
  const int sub = tid % G::LPS;
  const int vec = sub / G::NCH;
  const int ch = sub % G::NCH;
  const bool on = vec == 0 ? (xE != nullptr) : (xc != nullptr);
  const int32_t cnt = *count;
  for (int32_t bi = blockIdx.x; bi < cnt; bi += gridDim.x) {
    const int32_t u = list[bi];
    const int32_t a = vptr[u], b = vptr[u + 1];
    float acc[G::CH];
#pragma unroll
    for (int c = 0; c < G::CH; ++c) acc[c] = 0.0f;
    if (on) {
      for (int32_t j = a + slot; j < b; j += SLOTS) {
        const int32_t e = eids[j];
        float v[G::CH];
        if (vec == 0) {
          const float f = alpha[e];
          load_ch<G::CH>(xE + int64_t(e) * B + ch * G::CH, v);
#pragma unroll
          for (int c = 0; c < G::CH; ++c) acc[c] = fmaf(f, v[c], acc[c]);
        } else {
          load_ch<G::CH>(tb + int64_t(e) * B + ch * G::CH, v);
#pragma unroll
          for (int c = 0; c < G::CH; ++c) acc[c] += v[c];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < G::CH; ++c) red[tid * G::CH + c] = acc[c];
    __syncthreads();
    for (int stride = SLOTS / 2; stride > 0; stride >>= 1) {
      if (slot < stride) {
#pragma unroll
        for (int c = 0; c < G::CH; ++c)
          red[tid * G::CH + c] += red[(tid + stride * G::LPS) * G::CH + c];
      }
      __syncthreads();
    }
    if (slot == 0 && on) {
      const float su = s[u];
      float out[G::CH];
      if (vec == 0) {
#pragma unroll
        for (int c = 0; c < G::CH; ++c) out[c] = su * red[tid * G::CH + c];
        store_ch<G::CH>(yV + int64_t(u) * B + ch * G::CH, out);
      } else {
        const float gu = gam[u];
        float own[G::CH];
        load_ch<G::CH>(xc + int64_t(u) * B + ch * G::CH, own);
#pragma unroll
        for (int c = 0; c < G::CH; ++c) out[c] = su * red[tid * G::CH + c] - gu * own[c];
        store_ch<G::CH>(yc + int64_t(u) * B + ch * G::CH, out);
      }
    }
    __syncthreads();
  }
}

template <int B>
hef_status spmm_t(const Level &L, const Structure &st, const float *xs, float *ys,
                  const float *xc, float *yc, float *tb, hipStream_t s) {
  using G = Geo<B>;
  const int64_t n = L.n, m = L.m;
  const float *xE = xs ? xs + n * B : nullptr;
  float *yE = ys ? ys + n * B : nullptr;
  if (m > 0) {
    const int64_t nb = cdiv(m * G::LPS, kThreads);
    {
      TimedScope ts(kStSpmmCsr, s);
      k_csr_small<B><<<nb, kThreads, 0, s>>>(L.eptr, L.pins, st.s, st.alpha, st.beta, xs, xc,
                                             yE, tb, int32_t(m));
    }
    {
      TimedScope ts(kStSpmmCsrBig, s);
      k_csr_big<B><<<kBigGrid, kThreads, 0, s>>>(st.big_e, st.n_big, L.eptr, L.pins, st.s,
                                                 st.alpha, st.beta, xs, xc, yE, tb);
    }
    HEF_LAUNCH_CHECK();
  }
  if (n > 0) {
    const int64_t nb = cdiv(n * G::LPS, kThreads);
    {
      TimedScope ts(kStSpmmCsc, s);
      k_csc_small<B><<<nb, kThreads, 0, s>>>(st.vptr, st.eids, st.s, st.gam, st.alpha, xE, tb,
                                             xc, ys, yc, int32_t(n));
    }
    {
      TimedScope ts(kStSpmmCscBig, s);
      k_csc_big<B><<<kBigGrid, kThreads, 0, s>>>(st.big_v, st.n_big + 1, st.vptr, st.eids, st.s,
                                                 st.gam, st.alpha, xE, tb, xc, ys, yc);
    }
    HEF_LAUNCH_CHECK();
  }
  return HEF_OK;
}

}  // namespace

hef_status spmm_apply(const Level &L, const Structure &st, int B, const float *xs, float *ys,
                      const float *xc, float *yc, float *tbuf, hipStream_t s) {
  switch (B) {
    case 1: return spmm_t<1>(L, st, xs, ys, xc, yc, tbuf, s);
    case 2: return spmm_t<2>(L, st, xs, ys, xc, yc, tbuf, s);
    case 4: return spmm_t<4>(L, st, xs, ys, xc, yc, tbuf, s);
    case 8: return spmm_t<8>(L, st, xs, ys, xc, yc, tbuf, s);
    case 16: return spmm_t<16>(L, st, xs, ys, xc, yc, tbuf, s);
    default: set_error("block width %d is not a power of two in 1..16", B);
             return HEF_ERR_UNSUPPORTED;
  }
}

}  // namespace hef

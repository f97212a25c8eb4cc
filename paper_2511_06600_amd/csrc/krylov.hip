// Block Krylov bases of both expansions (Eq. (12), Alg. 1 steps 1-4).
//
// Per expansion, b start vectors and k steps of the block three-term
// recurrence: Y = A V_j, then V_{j+1} is the Gram-Schmidt of Y against
// [V_{j-1}, V_j] and within itself.  The Gram-Schmidt is carried out in the
// Gram metric of M = [V_{j-1} | V_j | Y]: G = M^T M is accumulated with
// FP32 matrix cores in row chunks and summed across chunks in float64, its
// Cholesky factor R (float64) gives V_{j+1} = M R^-1[:, Y columns].  A
// column whose Gram-Schmidt residual falls below tau times its length is a
// breakdown and becomes zero.  V_0 = X R^-1 starts the sequence and is not
// part of the pool; V_1..V_k are (star: node rows only).
#include <cmath>

#include "krylov.hpp"

namespace hef {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kGramBlocks = 512;   // workgroups of the Gram partial pass
constexpr int kFlushSteps = 128;   // FP32 accumulation length (MFMA steps)

__device__ __forceinline__ float load_m(const float *v0, const float *v1, const float *y,
                                        int64_t r, int c, int B) {
  if (c < B) return v0 ? v0[r * B + c] : 0.0f;
  if (c < 2 * B) return v1 ? v1[r * B + c - B] : 0.0f;
  if (c < 3 * B) return y[r * B + c - 2 * B];
  return 0.0f;
}

// Gram partials of M = [v0 | v1 | y] (rows x 3B, column c of tile t is
// 32t + c).  Each workgroup (4 waves) covers a contiguous row range; FP32
// MFMA accumulators are flushed to float64 every kFlushSteps steps; the 4
// waves are combined in LDS in wave order.  partial[blk][p][32*32] for tile
// pair p = (I <= J).
template <int T>
__global__ void __launch_bounds__(256)
k_lgram(const float *__restrict__ v0, const float *__restrict__ v1,
        const float *__restrict__ y, int64_t rows, int B, int64_t rows_per_blk,
        double *__restrict__ partial) {
  constexpr int TP = T * (T + 1) / 2;
  __shared__ double comb[TP * 1024];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int C = 3 * B;
  const int64_t r0 = int64_t(blockIdx.x) * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < rows ? r0 + rows_per_blk : rows;
  floatx16 acc[TP];
  double dacc[TP][16];
#pragma unroll
  for (int p = 0; p < TP; ++p) {
    for (int v = 0; v < 16; ++v) { acc[p][v] = 0.0f; dacc[p][v] = 0.0; }
  }
  int steps = 0;
  // wave wv takes row pairs r0 + 2*(wv + 4*i)
  for (int64_t r = r0 + 2 * wv; r < r1; r += 8) {
    const int64_t rr = r + (lane >> 5);
    float a[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int c = 32 * t + (lane & 31);
      a[t] = (rr < r1 && c < C) ? load_m(v0, v1, y, rr, c, B) : 0.0f;
    }
    int p = 0;
#pragma unroll
    for (int I = 0; I < T; ++I) {
#pragma unroll
      for (int J = I; J < T; ++J) {
        acc[p] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[I], a[J], acc[p], 0, 0, 0);
        ++p;
      }
    }
    if (++steps == kFlushSteps) {
      steps = 0;
#pragma unroll
      for (int q = 0; q < TP; ++q)
        for (int v = 0; v < 16; ++v) { dacc[q][v] += double(acc[q][v]); acc[q][v] = 0.0f; }
    }
  }
#pragma unroll
  for (int q = 0; q < TP; ++q)
    for (int v = 0; v < 16; ++v) dacc[q][v] += double(acc[q][v]);
  // combine waves in order 0,1,2,3
  for (int w = 0; w < 4; ++w) {
    if (wv == w) {
#pragma unroll
      for (int q = 0; q < TP; ++q)
        for (int v = 0; v < 16; ++v) {
          const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          const int j = lane & 31;
          double &dst = comb[q * 1024 + i * 32 + j];
          dst = (w == 0) ? dacc[q][v] : dst + dacc[q][v];
        }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < TP * 1024; e += 256)
    partial[int64_t(blockIdx.x) * TP * 1024 + e] = comb[e];
}

// Sum partials over blocks in block order; write the full symmetric C x C.
__global__ void k_lgram_reduce(const double *__restrict__ partial, int nblk, int T, int C,
                               double *__restrict__ G) {
  const int TP = T * (T + 1) / 2;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= TP * 1024) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[int64_t(b) * TP * 1024 + e];
  const int p = e / 1024, ij = e % 1024, i = ij / 32, j = ij % 32;
  int I = 0, J = 0, q = 0;
  for (int a = 0; a < T; ++a)
    for (int b = a; b < T; ++b) {
      if (q == p) { I = a; J = b; }
      ++q;
    }
  const int gi = 32 * I + i, gj = 32 * J + j;
  if (gi < C && gj < C) {
    G[gi * C + gj] = s;
    G[gj * C + gi] = s;
  }
}

// Cholesky of G with column dropping, then the Y-block columns of R^-1.
// One 64-thread workgroup per expansion.  Column c is dropped when its
// reference length is 0 or its Schur pivot d_c <= tau^2 * G_cc.
__global__ void __launch_bounds__(64)
k_lsolve(const double *__restrict__ Gall, int C, int B, double tau,
         double *__restrict__ Tall, int32_t *__restrict__ drops) {
  __shared__ double A[48 * 48];
  __shared__ double Lm[48 * 48];
  __shared__ int keep[48];
  const double *G = Gall + blockIdx.x * C * C;
  double *T = Tall + blockIdx.x * C * B;
  const int t = threadIdx.x;
  for (int e = t; e < C * C; e += 64) { A[e] = G[e]; Lm[e] = 0.0; }
  __syncthreads();
  for (int k = 0; k < C; ++k) {
    if (t == 0) {
      const double d = A[k * C + k];
      const double ref = G[k * C + k];
      keep[k] = (ref > 0.0 && d > tau * tau * ref) ? 1 : 0;
      if (keep[k]) Lm[k * C + k] = sqrt(d);
    }
    __syncthreads();
    if (keep[k] && t > k && t < C) Lm[t * C + k] = A[t * C + k] / Lm[k * C + k];
    __syncthreads();
    if (keep[k] && t > k && t < C) {
      const double lik = Lm[t * C + k];
      for (int j = k + 1; j <= t; ++j) A[t * C + j] -= lik * Lm[j * C + k];
    }
    __syncthreads();
  }
  // column c of R^-1 (R = L^T) = row c of L^-1: L^T x = e_c by back substitution
  if (t < B) {
    const int c = 2 * B + t;
    double x[48];
    for (int i = 0; i < C; ++i) x[i] = 0.0;
    if (keep[c]) {
      x[c] = 1.0 / Lm[c * C + c];
      for (int i = c - 1; i >= 0; --i) {
        if (!keep[i]) continue;
        double acc = 0.0;
        for (int l = i + 1; l <= c; ++l) acc += Lm[l * C + i] * x[l];
        x[i] = -acc / Lm[i * C + i];
      }
    }
    for (int i = 0; i < C; ++i) T[i * B + t] = x[i];
    if (!keep[c]) atomicAdd(&drops[blockIdx.x], 1);
  }
}

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

// V_next = [v0 | v1 | y] T (float64 arithmetic, one row per thread); the
// first pool_rows rows also go to the pool at column col0.
template <int B>
__global__ void __launch_bounds__(256)
k_lapply(const float *__restrict__ v0, const float *__restrict__ v1,
         const float *__restrict__ y, const double *__restrict__ Tm, float *__restrict__ vn,
         int64_t rows, void *__restrict__ pool, int pool_type, int64_t pool_rows, int K,
         int col0) {
  constexpr int C = 3 * B;
  __shared__ double Ts[C * B];
  for (int e = threadIdx.x; e < C * B; e += 256) Ts[e] = Tm[e];
  __syncthreads();
  const int64_t r = int64_t(xcd_block(blockIdx.x, gridDim.x)) * 256 + threadIdx.x;
  if (r >= rows) return;
  double out[B];
#pragma unroll
  for (int i = 0; i < B; ++i) out[i] = 0.0;
#pragma unroll
  for (int q = 0; q < C; ++q) {
    float mv;
    if (q < B) mv = v0 ? v0[r * B + q] : 0.0f;
    else if (q < 2 * B) mv = v1 ? v1[r * B + q - B] : 0.0f;
    else mv = y[r * B + q - 2 * B];
    const double md = double(mv);
#pragma unroll
    for (int i = 0; i < B; ++i) out[i] = fma(md, Ts[q * B + i], out[i]);
  }
  float of[B];
#pragma unroll
  for (int i = 0; i < B; ++i) of[i] = float(out[i]);
#pragma unroll
  for (int i = 0; i < B; ++i) vn[r * B + i] = of[i];
  if (pool && r < pool_rows) {
    if (pool_type == kPoolF32) {
      float *pp = reinterpret_cast<float *>(pool) + r * K + col0;
#pragma unroll
      for (int i = 0; i < B; ++i) pp[i] = of[i];
    } else {
      uint16_t *pp = reinterpret_cast<uint16_t *>(pool) + r * K + col0;
#pragma unroll
      for (int i = 0; i < B; ++i) pp[i] = f2bf(of[i]);
    }
  }
}

__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// N(0,1) element i of stream (seed, level, expansion): splitmix64 counter and
// Box-Muller, float64.
__global__ void k_start(uint64_t h, int64_t total, float *out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const uint64_t a = splitmix64(h + 2ull * uint64_t(i));
  const uint64_t c = splitmix64(h + 2ull * uint64_t(i) + 1ull);
  const double u1 = (double((a >> 11)) + 1.0) * 0x1.0p-53;
  const double u2 = double(c >> 11) * 0x1.0p-53;
  out[i] = float(sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2));
}

template <int B>
hef_status apply_t(const float *v0, const float *v1, const float *y, const double *T, float *vn,
                   int64_t rows, void *pool, int pool_type, int64_t pool_rows, int K, int col0,
                   hipStream_t s) {
  if (rows == 0) return HEF_OK;
  k_lapply<B><<<cdiv(rows, 256), 256, 0, s>>>(v0, v1, y, T, vn, rows, pool, pool_type,
                                               pool_rows, K, col0);
  HEF_LAUNCH_CHECK();
  return HEF_OK;
}

hef_status lapply(int B, const float *v0, const float *v1, const float *y, const double *T,
                  float *vn, int64_t rows, void *pool, int pool_type, int64_t pool_rows, int K,
                  int col0, hipStream_t s) {
  switch (B) {
    case 1: return apply_t<1>(v0, v1, y, T, vn, rows, pool, pool_type, pool_rows, K, col0, s);
    case 2: return apply_t<2>(v0, v1, y, T, vn, rows, pool, pool_type, pool_rows, K, col0, s);
    case 4: return apply_t<4>(v0, v1, y, T, vn, rows, pool, pool_type, pool_rows, K, col0, s);
    case 8: return apply_t<8>(v0, v1, y, T, vn, rows, pool, pool_type, pool_rows, K, col0, s);
    case 16: return apply_t<16>(v0, v1, y, T, vn, rows, pool, pool_type, pool_rows, K, col0, s);
    default: return HEF_ERR_UNSUPPORTED;
  }
}

int tiles_for(int B) { return (3 * B + 31) / 32; }

hef_status lgram(const float *v0, const float *v1, const float *y, int64_t rows, int B,
                 double *partial, double *G, hipStream_t s) {
  const int T = tiles_for(B);
  const int C = 3 * B;
  const int64_t per = std::max<int64_t>(8, cdiv(cdiv(rows, kGramBlocks), 8) * 8);
  const int nblk = int(std::max<int64_t>(1, cdiv(rows, per)));
  if (T == 1)
    k_lgram<1><<<nblk, 256, 0, s>>>(v0, v1, y, rows, B, per, partial);
  else
    k_lgram<2><<<nblk, 256, 0, s>>>(v0, v1, y, rows, B, per, partial);
  const int TP = T * (T + 1) / 2;
  k_lgram_reduce<<<cdiv(TP * 1024, 256), 256, 0, s>>>(partial, nblk, T, C, G);
  HEF_LAUNCH_CHECK();
  return HEF_OK;
}

}  // namespace

size_t krylov_ws_bytes(int64_t n, int64_t m, int B) {
  Arena a;
  for (int i = 0; i < 4; ++i) a.take<float>((n + m) * B);
  for (int i = 0; i < 4; ++i) a.take<float>(n * B);
  a.take<float>(m * B);
  const int T = tiles_for(B);
  a.take<double>(size_t(2) * kGramBlocks * (T * (T + 1) / 2) * 1024);
  a.take<double>(2 * 48 * 48);
  a.take<double>(2 * 48 * 16);
  a.take<int32_t>(2);
  return a.mark();
}

hef_status start_block(uint64_t seed, int level, int expansion, int64_t rows, int B,
                       float *out, hipStream_t s) {
  const uint64_t base = splitmix64(seed);
  const uint64_t h = splitmix64(base + 2ull * uint64_t(level) + uint64_t(expansion));
  const int64_t total = rows * B;
  if (total == 0) return HEF_OK;
  k_start<<<cdiv(total, 256), 256, 0, s>>>(h, total, out);
  HEF_LAUNCH_CHECK();
  return HEF_OK;
}

hef_status krylov_pool(const Level &L, const Structure &st, int B, int k, double tau,
                       const float *start_star, const float *start_clique, bool use_star,
                       bool use_clique, KrylovOut &out, Arena &ws, hipStream_t s) {
  const int64_t n = L.n, m = L.m;
  const int64_t Ns = n + m;
  const size_t mk = ws.mark();
  float *sb[4], *cb[4];
  for (int i = 0; i < 4; ++i) sb[i] = ws.take<float>(Ns * B);
  for (int i = 0; i < 4; ++i) cb[i] = ws.take<float>(n * B);
  float *tb = ws.take<float>(m * B);
  const int T = tiles_for(B);
  double *partial = ws.take<double>(size_t(2) * kGramBlocks * (T * (T + 1) / 2) * 1024);
  double *G = ws.take<double>(2 * 48 * 48);
  double *Tm = ws.take<double>(2 * 48 * 16);
  int32_t *drops = ws.take<int32_t>(2);
  if (ws.overflow) return HEF_ERR_WORKSPACE_TOO_SMALL;
  const int C = 3 * B;
  double *Gs = G, *Gc = G + C * C;
  double *Ts = Tm, *Tc = Tm + C * B;
  double *ps = partial, *pc = partial + size_t(kGramBlocks) * (T * (T + 1) / 2) * 1024;
  HEF_HIP(hipMemsetAsync(drops, 0, 2 * sizeof(int32_t), s));
  HEF_HIP(hipMemsetAsync(G, 0, 2 * 48 * 48 * sizeof(double), s));

  // indices into the rolling buffers: prev, cur, y, next
  int ip = 0, ic = 1, iy = 2, in = 3;
  const int K = out.K;
  const int64_t bk = int64_t(B) * k;
  // V_0 = X R^-1 (no pool write)
  if (use_star) {
    HEF_HIP(hipMemcpyAsync(sb[iy], start_star, Ns * B * sizeof(float), hipMemcpyDeviceToDevice, s));
    HEF_TRY(lgram(nullptr, nullptr, sb[iy], Ns, B, ps, Gs, s));
  }
  if (use_clique) {
    HEF_HIP(hipMemcpyAsync(cb[iy], start_clique, n * B * sizeof(float), hipMemcpyDeviceToDevice, s));
    HEF_TRY(lgram(nullptr, nullptr, cb[iy], n, B, pc, Gc, s));
  }
  k_lsolve<<<2, 64, 0, s>>>(G, C, B, tau, Tm, drops);
  HEF_LAUNCH_CHECK();
  if (use_star) HEF_TRY(lapply(B, nullptr, nullptr, sb[iy], Ts, sb[in], Ns, nullptr, 0, 0, K, 0, s));
  if (use_clique) HEF_TRY(lapply(B, nullptr, nullptr, cb[iy], Tc, cb[in], n, nullptr, 0, 0, K, 0, s));
  // rotate: cur <- next; prev stays "absent" for step 1
  std::swap(ic, in);
  bool have_prev = false;

  for (int j = 1; j <= k; ++j) {
    HEF_TRY(spmm_apply(L, st, B, use_star ? sb[ic] : nullptr, use_star ? sb[iy] : nullptr,
                       use_clique ? cb[ic] : nullptr, use_clique ? cb[iy] : nullptr, tb, s));
    if (use_star)
      HEF_TRY(lgram(have_prev ? sb[ip] : nullptr, sb[ic], sb[iy], Ns, B, ps, Gs, s));
    if (use_clique)
      HEF_TRY(lgram(have_prev ? cb[ip] : nullptr, cb[ic], cb[iy], n, B, pc, Gc, s));
    k_lsolve<<<2, 64, 0, s>>>(G, C, B, tau, Tm, drops);
    HEF_LAUNCH_CHECK();
    const int64_t col_s = (j - 1) * int64_t(B);
    const int64_t col_c = (use_star ? bk : 0) + (j - 1) * int64_t(B);
    if (use_star)
      HEF_TRY(lapply(B, have_prev ? sb[ip] : nullptr, sb[ic], sb[iy], Ts, sb[in], Ns, out.pool,
                     out.pool_type, n, K, int(col_s), s));
    if (use_clique)
      HEF_TRY(lapply(B, have_prev ? cb[ip] : nullptr, cb[ic], cb[iy], Tc, cb[in], n, out.pool,
                     out.pool_type, n, K, int(col_c), s));
    // rotate prev <- cur <- next, next <- old prev
    const int old_prev = ip;
    ip = ic;
    ic = in;
    in = old_prev;
    have_prev = true;
  }
  ws.reset(mk);
  return HEF_OK;
}

}  // namespace hef

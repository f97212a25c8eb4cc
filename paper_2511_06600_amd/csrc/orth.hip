// Joint orthonormalisation of the Krylov pool (Alg. 1 step 4: Gram-Schmidt
// of the unified [star | clique] list), as Cholesky QR:
//   G = V^T V      FP32 matrix-core tiles over 32-row LDS slabs, FP32
//                  accumulation flushed to float64 every 128 rows, float64
//                  across row chunks (fixed order);
//   G = R^T R      float64 Cholesky, one workgroup, with the drop rule;
//   V <- V R^-1    FP32 matrix cores, in place, one 32-row slab per workgroup.
// Cholesky QR produces the same Q as Gram-Schmidt (positive diag(R)).
#include <cmath>

#include "krylov.hpp"
#include "orth.hpp"

namespace hef {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kSB = 128;        // super-block width (4 MFMA tiles)
constexpr int kSlab = 32;       // rows per LDS slab
constexpr int kFlushSlabs = 4;  // FP32 accumulation over 128 rows

__device__ __forceinline__ float pool_at(const void *pool, int pool_type, int64_t idx) {
  if (pool_type == kPoolF32) return reinterpret_cast<const float *>(pool)[idx];
  const uint16_t h = reinterpret_cast<const uint16_t *>(pool)[idx];
  return __uint_as_float(uint32_t(h) << 16);
}

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

// Loads rows [r, r+32) x cols [c0, c0+128) into sh[32][128] (zeros outside).
__device__ __forceinline__ void load_slab(float *sh, const void *pool, int pool_type,
                                          int64_t r, int64_t r_end, int c0, int K) {
  const int col = threadIdx.x & 127;
  const int rsub = threadIdx.x >> 7;  // 0..1
#pragma unroll
  for (int i = 0; i < kSlab / 2; ++i) {
    const int rr = rsub + 2 * i;
    const int64_t row = r + rr;
    const int c = c0 + col;
    sh[rr * kSB + col] = (row < r_end && c < K) ? pool_at(pool, pool_type, row * K + c) : 0.0f;
  }
}

// Gram partials.  Block = (chunk, pair); pair p = (a <= b) of super blocks.
// Wave w owns tile row w of the 128x128 super tile and its 4 column tiles.
__device__ __forceinline__ int2 pair_of(int p, int nsb) {
  for (int a = 0; a < nsb; ++a) {
    if (p < nsb - a) return make_int2(a, a + p);
    p -= nsb - a;
  }
  return make_int2(0, 0);
}

__global__ void __launch_bounds__(256)
k_jgram(const void *__restrict__ pool, int pool_type, int64_t n, int K, int nsb,
        int npairs, int64_t rows_per_chunk, double *__restrict__ partial) {
  __shared__ float As[kSlab * kSB];
  __shared__ float Bs[kSlab * kSB];
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int pair = int(lb % npairs);
  const int64_t chunk = lb / npairs;
  const int2 ab = pair_of(pair, nsb);
  const bool diag = ab.x == ab.y;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int64_t r0 = chunk * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < n ? r0 + rows_per_chunk : n;
  floatx16 acc[4];
  double dacc[4][16];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) { acc[t][v] = 0.0f; dacc[t][v] = 0.0; }
  const float *Bsrc = diag ? As : Bs;
  int slabs = 0;
  for (int64_t r = r0; r < r1; r += kSlab) {
    __syncthreads();
    load_slab(As, pool, pool_type, r, r1, ab.x * kSB, K);
    if (!diag) load_slab(Bs, pool, pool_type, r, r1, ab.y * kSB, K);
    __syncthreads();
#pragma unroll 4
    for (int s = 0; s < kSlab / 2; ++s) {
      const int row = 2 * s + (lane >> 5);
      const float a_op = As[row * kSB + 32 * w + (lane & 31)];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (!diag || t >= w) {
          const float b_op = Bsrc[row * kSB + 32 * t + (lane & 31)];
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a_op, b_op, acc[t], 0, 0, 0);
        }
      }
    }
    if (++slabs == kFlushSlabs) {
      slabs = 0;
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) { dacc[t][v] += double(acc[t][v]); acc[t][v] = 0.0f; }
    }
  }
  double *out = partial + (chunk * npairs + pair) * (16 * 1024);
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      const int j = lane & 31;
      out[(w * 4 + t) * 1024 + i * 32 + j] = dacc[t][v] + double(acc[t][v]);
    }
}

// G[gi][gj] = sum over chunks (in order) of the partial tiles.
__global__ void k_jgram_reduce(const double *__restrict__ partial, int nchunks, int nsb,
                               int npairs, int K, double *__restrict__ G) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(npairs) * 16 * 1024) return;
  const int pair = int(e / (16 * 1024));
  const int rem = int(e % (16 * 1024));
  const int wt = rem / 1024, ij = rem % 1024;
  const int w = wt / 4, t = wt % 4, i = ij / 32, j = ij % 32;
  const int2 ab = pair_of(pair, nsb);
  if (ab.x == ab.y && t < w) return;
  const int gi = ab.x * kSB + 32 * w + i;
  const int gj = ab.y * kSB + 32 * t + j;
  if (gi >= K || gj >= K) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += partial[(int64_t(c) * npairs + pair) * (16 * 1024) + rem];
  G[int64_t(gi) * K + gj] = s;
  G[int64_t(gj) * K + gi] = s;
}

// Blocked left-looking Cholesky G = L L^T (float64) with the drop rule, one
// 1024-thread workgroup.  L is kept column-major in global memory
// (LT[c*K + r] = L[r][c]); each 32-column panel is updated by a 4x4
// register-blocked product with the finished columns, then factored in LDS.
// A column whose Schur pivot is <= tau^2 G_jj (or that `force_keep` marks 0)
// is dropped: its column of L is zero.
constexpr int kPW = 32;
constexpr int kPS = kPW + 1;  // LDS row stride of a panel

__global__ void __launch_bounds__(1024)
k_jchol(const double *__restrict__ G, int K, double tau, double *__restrict__ LT,
        int32_t *__restrict__ keep, const int32_t *__restrict__ force_keep) {
  extern __shared__ double pan[];  // [K][kPS]
  __shared__ int s_keep;
  const int t = threadIdx.x;
  for (int64_t e = t; e < int64_t(K) * K; e += 1024) LT[e] = 0.0;
  __syncthreads();
  for (int c0 = 0; c0 < K; c0 += kPW) {
    const int w = K - c0 < kPW ? K - c0 : kPW;
    const int nr = K - c0;
    // panel rows [c0, K) x cols [c0, c0+w): G minus the finished columns
    const int nbi = (nr + 3) / 4, nbj = (w + 3) / 4;
    for (int blk = t; blk < nbi * nbj; blk += 1024) {
      const int bi = blk / nbj, bj = blk % nbj;
      const int r0 = c0 + 4 * bi, q0 = c0 + 4 * bj;
      if (4 * bi + 3 < 4 * bj) continue;  // strictly above the diagonal
      double acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int r = r0 + a, q = q0 + b;
          acc[a][b] = (r < K && q < c0 + w) ? G[int64_t(r) * K + q] : 0.0;
        }
      for (int l = 0; l < c0; ++l) {
        const double *col = LT + int64_t(l) * K;
        double x[4], y[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) x[a] = (r0 + a < K) ? col[r0 + a] : 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b) y[b] = (q0 + b < K) ? col[q0 + b] : 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] -= x[a] * y[b];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int i = 4 * bi + a, j = 4 * bj + b;
          if (i < nr && j < w) pan[i * kPS + j] = acc[a][b];
        }
    }
    __syncthreads();
    for (int jj = 0; jj < w; ++jj) {
      if (t == 0) {
        const double d = pan[jj * kPS + jj];
        const double ref = G[int64_t(c0 + jj) * K + c0 + jj];
        int kp = (ref > 0.0 && d > tau * tau * ref) ? 1 : 0;
        if (force_keep && !force_keep[c0 + jj]) kp = 0;
        keep[c0 + jj] = kp;
        s_keep = kp;
        pan[jj * kPS + jj] = kp ? sqrt(d) : 0.0;
      }
      __syncthreads();
      const int kp = s_keep;
      const double piv = pan[jj * kPS + jj];
      for (int i = jj + 1 + t; i < nr; i += 1024)
        pan[i * kPS + jj] = kp ? pan[i * kPS + jj] / piv : 0.0;
      __syncthreads();
      if (kp) {
        const int wc = w - jj - 1;
        if (wc > 0) {
          for (int e = t; e < (nr - jj - 1) * wc; e += 1024) {
            const int i = jj + 1 + e / wc, q = jj + 1 + e % wc;
            if (q <= i) pan[i * kPS + q] -= pan[i * kPS + jj] * pan[q * kPS + jj];
          }
        }
      }
      __syncthreads();
    }
    for (int e = t; e < nr * w; e += 1024) {
      const int i = e / w, j = e % w;
      if (i >= j) LT[int64_t(c0 + j) * K + c0 + i] = pan[i * kPS + j];
    }
    __syncthreads();
  }
}

// X = L^-1 by 32-column blocks, one workgroup per block J (independent):
// X_JJ = L_JJ^-1, then X_IJ = -L_II^-1 sum_{M=J}^{I-1} L_IM X_MJ for I > J.
// Rows and columns of dropped pivots are zero.  Writes Rinv = X^T
// (row-major, Kp x Kp, float64 and float32; entries outside stay as set).
__global__ void __launch_bounds__(1024)
k_jtrinv(const double *__restrict__ LT, const int32_t *__restrict__ keep, int K, int Kp,
         double *__restrict__ Rinv, float *__restrict__ Rinv32) {
  extern __shared__ double X[];  // [K][kPS]: rows of the column block J
  __shared__ double T[kPW * kPS];
  const int t = threadIdx.x;
  const int J = blockIdx.x;
  const int j0 = J * kPW;
  const int wj = K - j0 < kPW ? K - j0 : kPW;
  const int nb = (K + kPW - 1) / kPW;
  for (int e = t; e < K * kPS; e += 1024) X[e] = 0.0;
  __syncthreads();
  for (int I = J; I < nb; ++I) {
    const int i0 = I * kPW;
    const int wi = K - i0 < kPW ? K - i0 : kPW;
    // T = -sum_{m in [j0, i0)} L[i0+i][m] X[m][j]   (zero for I == J)
    {
      const int i = t / kPW, j = t % kPW;
      double acc = (I == J && i == j) ? 1.0 : 0.0;
      if (i < wi && j < wj) {
        for (int m = j0; m < i0; ++m) acc -= LT[int64_t(m) * K + i0 + i] * X[m * kPS + j];
      }
      T[i * kPS + j] = acc;
    }
    __syncthreads();
    // solve L_II X_IJ = T by forward substitution, one column per thread
    if (t < wj) {
      const int j = t;
      const bool colkeep = keep[j0 + j] != 0;
      for (int i = 0; i < wi; ++i) {
        double x = 0.0;
        if (colkeep && keep[i0 + i]) {
          double acc = T[i * kPS + j];
          for (int l = 0; l < i; ++l) acc -= LT[int64_t(i0 + l) * K + i0 + i] * X[(i0 + l) * kPS + j];
          x = acc / LT[int64_t(i0 + i) * K + i0 + i];
        }
        X[(i0 + i) * kPS + j] = x;
      }
    }
    __syncthreads();
  }
  // Rinv[j0+j][i] = X[i][j]
  for (int e = t; e < wj * K; e += 1024) {
    const int j = e / K, i = e % K;
    const double x = X[i * kPS + j];
    Rinv[int64_t(j0 + j) * Kp + i] = x;
    Rinv32[int64_t(j0 + j) * Kp + i] = float(x);
  }
}


// In-place V <- V Rinv on 32-row slabs (LDS row stride K+1 avoids bank
// conflicts of the column-wise A-operand reads).
__global__ void __launch_bounds__(256)
k_japply(void *__restrict__ pool, int pool_type, int64_t n, int K, int Kp,
         const float *__restrict__ Rinv32) {
  extern __shared__ float slab[];
  const int ld = K + 1;
  const int64_t r0 = int64_t(xcd_block(blockIdx.x, gridDim.x)) * kSlab;
  for (int e = threadIdx.x; e < kSlab * K; e += 256) {
    const int i = e / K, c = e % K;
    const int64_t row = r0 + i;
    slab[i * ld + c] = row < n ? pool_at(pool, pool_type, row * K + c) : 0.0f;
  }
  for (int i = threadIdx.x; i < kSlab; i += 256) slab[i * ld + K] = 0.0f;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int ntile = (K + 31) / 32;
  for (int J = w; J < ntile; J += 4) {
    floatx16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
    const int kend = (32 * J + 32 < K) ? 32 * J + 32 : K;
    const int c = 32 * J + (lane & 31);
    for (int k0 = 0; k0 < kend; k0 += 2) {
      const int k = k0 + (lane >> 5);
      const float a_op = k < K ? slab[(lane & 31) * ld + k] : 0.0f;
      const float b_op = k < K ? Rinv32[int64_t(k) * Kp + c] : 0.0f;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a_op, b_op, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      const int64_t row = r0 + i;
      if (row < n && c < K) {
        if (pool_type == kPoolF32)
          reinterpret_cast<float *>(pool)[row * K + c] = acc[v];
        else
          reinterpret_cast<uint16_t *>(pool)[row * K + c] = f2bf(acc[v]);
      }
    }
  }
}

struct GramPlan {
  int nsb = 0, npairs = 0, nchunks = 0;
  int64_t rows_per_chunk = 0;
};

GramPlan gram_plan(int64_t n, int K) {
  GramPlan p;
  p.nsb = (K + kSB - 1) / kSB;
  p.npairs = p.nsb * (p.nsb + 1) / 2;
  int64_t want = std::max<int64_t>(1, 768 / p.npairs);
  int64_t per = cdiv(std::max<int64_t>(n, 1), want);
  per = std::max<int64_t>(kSlab, cdiv(per, kSlab) * kSlab);
  p.rows_per_chunk = per;
  p.nchunks = int(std::max<int64_t>(1, cdiv(n, per)));
  return p;
}

hef_status gram_run(const void *pool, int pool_type, int64_t n, int K, double *G, Arena &ws,
                    hipStream_t s) {
  const GramPlan p = gram_plan(n, K);
  const size_t mk = ws.mark();
  double *partial = ws.take<double>(size_t(p.nchunks) * p.npairs * 16 * 1024);
  if (ws.overflow) return HEF_ERR_WORKSPACE_TOO_SMALL;
  HEF_HIP(hipMemsetAsync(G, 0, sizeof(double) * K * K, s));
  TimedScope ts(kStOrthGram, s);
  k_jgram<<<int64_t(p.npairs) * p.nchunks, 256, 0, s>>>(pool, pool_type, n, K, p.nsb, p.npairs,
                                                        p.rows_per_chunk, partial);
  const int64_t tot = int64_t(p.npairs) * 16 * 1024;
  k_jgram_reduce<<<cdiv(tot, 256), 256, 0, s>>>(partial, p.nchunks, p.nsb, p.npairs, K, G);
  HEF_LAUNCH_CHECK();
  ws.reset(mk);
  return HEF_OK;
}

}  // namespace

size_t orth_ws_bytes(int64_t n, int K) {
  const int Kp = (K + 31) / 32 * 32;
  const GramPlan p = gram_plan(n, K);
  Arena a;
  a.take<double>(int64_t(K) * K);    // G
  a.take<double>(int64_t(K) * K);    // A
  a.take<double>(int64_t(K) * K);    // LT
  a.take<double>(int64_t(Kp) * Kp);  // Rinv
  a.take<float>(int64_t(Kp) * Kp);   // Rinv32
  a.take<int32_t>(K);                // keep
  a.take<double>(size_t(p.nchunks) * p.npairs * 16 * 1024);
  return a.mark() + 1024;
}

hef_status gram_f32(const float *X, int64_t n, int K, double *G, Arena &ws, hipStream_t s) {
  if (K <= 0 || K > 512) return HEF_ERR_UNSUPPORTED;
  return gram_run(X, kPoolF32, n, K, G, ws, s);
}

hef_status orthonormalize_pool(void *pool, int pool_type, int64_t n, int K, double tau,
                               int passes, int32_t *keep_out, Arena &ws, hipStream_t s) {
  if (K <= 0) return HEF_OK;
  if (K > 512) {
    set_error("pool width %d exceeds 512", K);
    return HEF_ERR_UNSUPPORTED;
  }
  const int Kp = (K + 31) / 32 * 32;
  const size_t mk = ws.mark();
  double *G = ws.take<double>(int64_t(K) * K);
  double *A = ws.take<double>(int64_t(K) * K);
  double *LT = ws.take<double>(int64_t(K) * K);
  double *Rinv = ws.take<double>(int64_t(Kp) * Kp);
  float *Rinv32 = ws.take<float>(int64_t(Kp) * Kp);
  int32_t *keep = ws.take<int32_t>(K);
  if (ws.overflow) return HEF_ERR_WORKSPACE_TOO_SMALL;
  const size_t lds = size_t(kSlab) * (K + 1) * sizeof(float);
  for (int pass = 0; pass < passes; ++pass) {
    HEF_TRY(gram_run(pool, pool_type, n, K, G, ws, s));
    {
      TimedScope ts(kStOrthChol, s);
      const size_t lds_c = size_t(K) * kPS * sizeof(double);
      HEF_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_jchol),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_c)));
      HEF_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_jtrinv),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_c)));
      HEF_HIP(hipMemsetAsync(Rinv, 0, sizeof(double) * Kp * Kp, s));
      HEF_HIP(hipMemsetAsync(Rinv32, 0, sizeof(float) * Kp * Kp, s));
      k_jchol<<<1, 1024, lds_c, s>>>(G, K, tau, LT, keep, pass == 0 ? nullptr : keep);
      k_jtrinv<<<(K + kPW - 1) / kPW, 1024, lds_c, s>>>(LT, keep, K, Kp, Rinv, Rinv32);
    }
    HEF_LAUNCH_CHECK();
    if (n > 0) {
      HEF_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_japply),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
      TimedScope ts(kStOrthApply, s);
      k_japply<<<cdiv(n, kSlab), 256, lds, s>>>(pool, pool_type, n, K, Kp, Rinv32);
      HEF_LAUNCH_CHECK();
    }
  }
  if (keep_out) HEF_HIP(hipMemcpyAsync(keep_out, keep, K * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  ws.reset(mk);
  return HEF_OK;
}

}  // namespace hef

// Joint orthonormalisation of the Krylov pool (Alg. 1: Gram-Schmidt
// of the unified [star | clique] list), as Cholesky QR:
//   G = V^T V      FP32 matrix-core tiles over 32-row LDS slabs, FP32
//                  accumulation flushed to float64 every 128 rows, float64
//                  across row chunks (fixed order);
//   G = R^T R      blocked float64 Cholesky with the drop rule, and R^-1;
//   Q = V R^-1     FP32 matrix-core GEMM into the second pool buffer.
// Cholesky QR produces the same Q as Gram-Schmidt (positive diag(R)).
#include <cmath>

#include "krylov.hpp"
#include "orth.hpp"
#include "prims.hpp"

namespace hef {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));


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

// Blocked Cholesky G = L L^T (float64) with the drop rule.  L is kept
// column-major in global memory (LT[c*K + r] = L[r][c]).  A column whose
// Schur pivot is <= tau^2 G_jj (or that `force_keep` marks 0) is dropped:
// its column of L is zero.
constexpr int kPW = 32;
constexpr int kPS = kPW + 1;  // LDS row stride of a panel
constexpr int kMaxPB = 16;    // 32-column blocks of the widest pool (K <= 512)

// Right-looking: A holds G minus the contributions of the finished panels
// (lower triangle).  Panel [c0, c0+w) is factored by k_chol_panel;
// k_chol_update then subtracts its columns from the trailing matrix, tile
// by tile, so every entry sees its subtractions in ascending column order.
//
// k_chol_panel: the first wave of every workgroup factors the w x w
// diagonal block in registers (lane r holds row r; the pivot and the
// normalised column entries reach the other lanes by readlane), which fixes
// the drop decisions and pivots; the other three waves carry one panel row
// below the block each through the same column steps (divide by the pivot,
// subtract the row's multiple of every later column), so each entry of L
// sees the same operations in the same order as a column-by-column
// factorisation of the whole panel.  The two run as a pipeline: the first
// wave publishes column j of the block (multiples, pivot, keep) in LDS while
// the rows below take column j - 1, one barrier per column.  Workgroup 0
// also writes the diagonal block, keep and rho.
constexpr int kCT = 256;        // panel threads
constexpr int kCR = kCT - 64;   // rows below the block per workgroup

// FULL: the panel has kPW columns (every panel but a narrower last one), so
// the column bounds are compile-time and the unrolled steps carry no tests.
template <bool FULL>
__global__ void __launch_bounds__(kCT)
k_chol_panel(const double *__restrict__ A, const double *__restrict__ G, int K, int c0,
             double tau, double *__restrict__ LT, int32_t *__restrict__ keep,
             const int32_t *__restrict__ force_keep, double *__restrict__ rho) {
  __shared__ double Ln[kPW][kPS];  // the block's L (pivot on the diagonal)
  __shared__ double s_piv[kPW];
  __shared__ int s_kp[kPW];
  const int t = threadIdx.x;
  const int w = FULL ? kPW : (K - c0 < kPW ? K - c0 : kPW);
  const int nr = K - c0;
  const bool dw = t < 64;  // the diagonal block's wave (wave-uniform)
  const int r = t & (kPW - 1);
  // diagonal wave: lane r holds row r of the block; other waves: one row below
  const int i = w + int(blockIdx.x) * kCR + (t - 64);
  const bool row_ok = !dw && i < nr;
  double x[kPW];
  double ref = 0.0;
  int frc = 0;
  if (dw) {
#pragma unroll
    for (int j = 0; j < kPW; ++j)
      x[j] = (r < w && j <= r) ? A[int64_t(c0 + r) * K + c0 + j] : 0.0;
    ref = r < w ? G[int64_t(c0 + r) * K + c0 + r] : 0.0;
    frc = r < w ? (force_keep ? force_keep[c0 + r] : 1) : 0;
  } else if (row_ok) {
    const double *ar = A + int64_t(c0 + i) * K + c0;
#pragma unroll
    for (int j = 0; j < kPW; ++j) x[j] = j < w ? ar[j] : 0.0;
  }
  double dkeep = 0.0, pkeep = 0.0;  // lane r: column r's Schur pivot and L_rr
  int kkeep = 0;
  // column jj of the diagonal block (first wave)
  auto diag_step = [&](int jj) __attribute__((always_inline)) {
    const double d = readlane_f64(x[jj], jj);
    const double rf = readlane_f64(ref, jj);
    int kp = (rf > 0.0 && d > tau * tau * rf) ? 1 : 0;
    if (!__builtin_amdgcn_readlane(frc, jj)) kp = 0;
    const double piv = kp ? sqrt(d) : 0.0;
    const double lv = (kp && r > jj && r < w) ? x[jj] / piv : 0.0;
    if (r == jj) {
      dkeep = d;
      pkeep = piv;
      kkeep = kp;
    }
    // column jj of L below the pivot (entries above the diagonal of the
    // block are never read)
    x[jj] = r == jj ? piv : lv;
    if (t < kPW) Ln[t][jj] = t >= jj ? x[jj] : 0.0;
    if (t == 0) {
      s_piv[jj] = piv;
      s_kp[jj] = kp;
    }
    if (kp) {
#pragma unroll
      for (int tc = jj + 1; tc < kPW; ++tc)
        if (FULL || tc < w) x[tc] = __builtin_fma(-lv, readlane_f64(lv, tc), x[tc]);
    }
  };
  // column jj for a row below the block (the other waves)
  auto row_step = [&](int jj) __attribute__((always_inline)) {
    const int kp = s_kp[jj];
    x[jj] = kp ? x[jj] / s_piv[jj] : 0.0;
    if (kp) {
#pragma unroll
      for (int tc = jj + 1; tc < kPW; ++tc)
        if (FULL || tc < w) x[tc] = __builtin_fma(-x[jj], Ln[tc][jj], x[tc]);
    }
  };
#pragma unroll
  for (int jj = 0; jj <= kPW; ++jj) {
    if (FULL || jj <= w) {
      if (dw) {
        if (jj < w) diag_step(jj);
      } else if (row_ok && jj > 0) {
        row_step(jj - 1);
      }
      __syncthreads();
    }
  }
  if (dw && t < kPW && blockIdx.x == 0 && t < w) {
#pragma unroll
    for (int j = 0; j < kPW; ++j)
      if (j <= t) LT[int64_t(c0 + j) * K + c0 + t] = x[j];
    keep[c0 + t] = kkeep;
    // relative Gram-Schmidt residual |R_jj| / ||V_j|| of a kept column
    if (rho) rho[c0 + t] = kkeep ? sqrt(dkeep / ref) : 0.0;
  }
  if (row_ok) {
#pragma unroll
    for (int j = 0; j < kPW; ++j)
      if (j < w) LT[int64_t(c0 + j) * K + c0 + i] = x[j];
  }
}

// A[i][q] -= sum_{l in [c0, c0+w)} L[i][l] L[q][l] for c0+w <= q <= i < K:
// one workgroup per 32 x 32 tile of the trailing lower triangle.
__global__ void __launch_bounds__(256)
k_chol_update(double *__restrict__ A, const double *__restrict__ LT, int K, int c0, int w) {
  __shared__ double Li[kPW][kPS];
  __shared__ double Lq[kPW][kPS];
  const int r0 = c0 + w;
  int tile = blockIdx.x, ti = 0;
  while (tile > ti) { tile -= ti + 1; ++ti; }
  const int tj = tile;
  const int i0 = r0 + kPW * ti, q0 = r0 + kPW * tj;
  const int t = threadIdx.x;
  for (int e = t; e < kPW * w; e += 256) {
    const int l = e / kPW, a = e % kPW;
    Li[a][l] = i0 + a < K ? LT[int64_t(c0 + l) * K + i0 + a] : 0.0;
    Lq[a][l] = q0 + a < K ? LT[int64_t(c0 + l) * K + q0 + a] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = t + 256 * u;
    const int a = e / kPW, b = e % kPW;
    const int i = i0 + a, q = q0 + b;
    if (i < K && q <= i) {
      double acc = A[int64_t(i) * K + q];
      for (int l = 0; l < w; ++l) acc -= Li[a][l] * Lq[b][l];
      A[int64_t(i) * K + q] = acc;
    }
  }
}

// X = L^-1 by 32-column blocks, one workgroup per block J (independent):
// X_JJ = L_JJ^-1, then X_IJ = -L_II^-1 sum_{M=J}^{I-1} L_IM X_MJ for I > J.
// Rows and columns of dropped pivots are zero.  Writes Rinv = X^T
// (row-major, Kp x Kp, float64 and float32; entries outside stay as set).
//
// The block sum runs on the float64 matrix cores: wave w takes the 16 x 16
// tile w & 3 of the 32 x 32 sum over the k quarter w >> 2 of [j0, i0) (A
// operands straight from L in global memory, 16 at a time ahead of their
// products; B operands from the finished rows of X in LDS), and the four
// quarters are added in a fixed order.  The solve with L_II is a forward
// substitution: thread (i, j) keeps row i of column j (a column's 32 rows in
// half a wave); at step l the lane of row l scales its entry by the pivot's
// reciprocal and the other lanes take it by readlane.
constexpr int kTK = 16;  // k steps (of 4) whose A operands are loaded together

__device__ __forceinline__ double half_readlane_f64(double v, int l, int lane) {
  return lane < 32 ? readlane_f64(v, l) : readlane_f64(v, l + 32);
}

__global__ void __launch_bounds__(1024)
k_jtrinv(const double *__restrict__ LT, const int32_t *__restrict__ keep, int K, int Kp,
         double *__restrict__ Rinv, float *__restrict__ Rinv32, float *__restrict__ RinvT32) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  extern __shared__ double X[];  // [K][kPS]: rows of the column block J
  __shared__ double T[kPW * kPS];
  __shared__ double Lb[kPW * kPS];
  __shared__ int kr[kPW], kc[kPW];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int J = blockIdx.x;
  const int j0 = J * kPW;
  const int wj = K - j0 < kPW ? K - j0 : kPW;
  const int nb = (K + kPW - 1) / kPW;
  for (int e = t; e < K * kPS; e += 1024) X[e] = 0.0;
  if (t < kPW) kc[t] = t < wj ? keep[j0 + t] : 0;
  for (int I = J; I < nb; ++I) {
    const int i0 = I * kPW;
    const int wi = K - i0 < kPW ? K - i0 : kPW;
    // L_II and the keep flags are loaded here and stored to LDS after the
    // block sum, so their latency overlaps that of the A operands
    const int lmm = t / kPW, lii = t % kPW;
    const int lcl = lii < wi && lmm < wi;
    const double lbv = LT[int64_t(i0 + (lcl ? lmm : 0)) * K + i0 + (lcl ? lii : 0)];
    const int krv = t < kPW ? keep[i0 + (t < wi ? t : 0)] : 0;
    // S = sum_{m in [j0, i0)} L[i0+i][m] X[m][j]; T = delta_IJ - S
    const int tile = wv & 3, ks = wv >> 2;
    const int ti = tile >> 1, tj = tile & 1;
    const int r16 = lane & 15, k4 = lane >> 4;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    {
      const int S = (i0 - j0) / 4;  // k steps of 4
      const int s0 = S * ks / 4, s1 = S * (ks + 1) / 4;
      const int gi = i0 + 16 * ti + r16;
      const int gc = gi < K ? gi : K - 1;  // rows past K: clamped load, zero operand
      const bool rok = gi < K;
      for (int sb = s0; sb < s1; sb += kTK) {
        double a[kTK];
#pragma unroll
        for (int u = 0; u < kTK; ++u) {
          const int ss = sb + u < s1 ? sb + u : s1 - 1;
          a[u] = LT[int64_t(j0 + 4 * ss + k4) * K + gc];
        }
#pragma unroll
        for (int u = 0; u < kTK; ++u) {
          if (sb + u < s1) {
            const double b = X[(j0 + 4 * (sb + u) + k4) * kPS + 16 * tj + r16];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(rok ? a[u] : 0.0, b, acc, 0, 0, 0);
          }
        }
      }
    }
    // quarters added in order ks = 0, 1, 2, 3 (accumulator r of a lane is
    // tile row 4 r + (lane >> 4), column lane & 15)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      __syncthreads();
      if (q == 0) {
        Lb[lii * kPS + lmm] = lcl ? lbv : 0.0;
        if (t < kPW) kr[t] = t < wi ? krv : 0;
      }
      if (ks == q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * ti + 4 * r + k4, j = 16 * tj + r16;
          const double v = q == 0 ? acc[r] : T[i * kPS + j] + acc[r];
          T[i * kPS + j] = q < 3 ? v : (I == J && i == j ? 1.0 : 0.0) - v;
        }
      }
    }
    __syncthreads();
    // solve L_II X_IJ = T
    {
      const int j = t / kPW, i = t % kPW;
      double a = T[i * kPS + j];
      const double dinv = (kc[j] && kr[i]) ? 1.0 / Lb[i * kPS + i] : 0.0;
      double xi = 0.0;
#pragma unroll
      for (int l = 0; l < kPW; ++l) {
        if (l < wi) {
          const double own = a * dinv;  // x_l on the lane of row l
          if (i == l) xi = own;
          const double xl = half_readlane_f64(own, l, lane);
          if (i > l) a = __builtin_fma(-Lb[i * kPS + l], xl, a);
        }
      }
      if (j < wj && i < wi) X[(i0 + i) * kPS + j] = xi;
    }
    __syncthreads();
  }
  // Rinv[j0+j][i] = X[i][j]
  for (int e = t; e < wj * K; e += 1024) {
    const int j = e / K, i = e % K;
    const double x = X[i * kPS + j];
    Rinv[int64_t(j0 + j) * Kp + i] = x;
    Rinv32[int64_t(j0 + j) * Kp + i] = float(x);
    if (RinvT32) RinvT32[int64_t(i) * Kp + j0 + j] = float(x);
  }
}


// ---------------------------------------------------------------- Gram
// G = V^T V.  Block = (row chunk, super-tile pair (a <= b) of 128-column
// super blocks).  FP32 pool: 16 waves, one 32x32 tile of the 128x128 super
// tile each (tiles below the diagonal of a diagonal super tile are skipped).
// BF16 pool: 8 waves of two tiles each.  Row slabs of both super blocks are
// double-buffered in LDS (64 rows, column-major, for the FP32 pool); FP32
// MFMA accumulators are flushed to float64 registers every 128 rows.
constexpr int kSB = 128;        // super-block width (4 MFMA tiles)
constexpr int kSlab = 64;       // rows per LDS slab
constexpr int kSLd = kSlab + 4; // LDS column stride (floats) of a slab
constexpr int kFlushSlabs = 2;  // FP32 accumulation over 128 rows
constexpr int kGT = 512;        // BF16 Gram workgroup size
constexpr int kGT32 = 1024;     // FP32 Gram workgroup size: one wave per tile

__device__ __forceinline__ int2 pair_of(int p, int nsb) {
  for (int a = 0; a < nsb; ++a) {
    if (p < nsb - a) return make_int2(a, a + p);
    p -= nsb - a;
  }
  return make_int2(0, 0);
}

// 8 consecutive pool values (columns c..c+7 of row `row`) as floats; zeros
// past the matrix.  Vector loads when the row stride allows.
__device__ __forceinline__ void load8(const void *pool, int pool_type, int64_t row, int64_t rows,
                                      int c, int K, float (&v)[8]) {
  if (row >= rows || c >= K) {
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = 0.0f;
    return;
  }
  const int64_t off = row * K + c;
  if (pool_type == kPoolF32) {
    const float *p = reinterpret_cast<const float *>(pool) + off;
    if ((K & 3) == 0 && c + 8 <= K) {
      const float4 a = *reinterpret_cast<const float4 *>(p);
      const float4 b = *reinterpret_cast<const float4 *>(p + 4);
      v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
      v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = (c + q < K) ? p[q] : 0.0f;
    }
  } else {
    const uint16_t *p = reinterpret_cast<const uint16_t *>(pool) + off;
    if ((K & 7) == 0 && c + 8 <= K) {
      const uint4 a = *reinterpret_cast<const uint4 *>(p);
      const uint32_t u[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        v[2 * q] = __uint_as_float(u[q] << 16);
        v[2 * q + 1] = __uint_as_float(u[q] & 0xFFFF0000u);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q)
        v[q] = (c + q < K) ? __uint_as_float(uint32_t(p[q]) << 16) : 0.0f;
    }
  }
}

// The 8 rows rb..rb+7 (rb a multiple of 8) of column c of a pool in the
// row-octet layout (element (r, c) at ((r >> 3) K + c) 8 + (r & 7)), as
// floats; zeros past column K or row `rows`.
__device__ __forceinline__ void load8oct(const void *pool, int pool_type, int64_t rb,
                                         int64_t rows, int c, int K, float (&v)[8]) {
  if (rb >= rows || c >= K) {
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = 0.0f;
    return;
  }
  const int64_t off = ((rb >> 3) * K + c) * 8;
  if (pool_type == kPoolF32) {
    const float4 a = *reinterpret_cast<const float4 *>(reinterpret_cast<const float *>(pool) + off);
    const float4 b = *reinterpret_cast<const float4 *>(reinterpret_cast<const float *>(pool) + off + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
    const uint4 a = *reinterpret_cast<const uint4 *>(reinterpret_cast<const uint16_t *>(pool) + off);
    const uint32_t u[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[2 * q] = __uint_as_float(u[q] << 16);
      v[2 * q + 1] = __uint_as_float(u[q] & 0xFFFF0000u);
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (rb + q >= rows) v[q] = 0.0f;
}

// 32 rows of a 128-column super block of an FP32 pool into registers:
// row-octet input (thread -> octet of rows, 1 column) or row-major input
// (thread -> row, 8 columns).  The loads are unconditional (addresses
// clamped into the chunk and the row), so nothing waits on them until the
// values go to LDS; slab_put applies the row and column masks there and
// stores the block column-major (column c at S + c * kSLd), an octet as two
// 16-byte stores.  Within column c the groups of 4 rows are permuted: slab
// row r sits at r ^ slab_swz(c).  The transposed stores of row-major input
// (16 columns 8 apart, whose starts share a bank since 8 kSLd is a multiple
// of 32) then spread over all banks, while each 4-row group stays
// contiguous for the 16-byte operand reads.  Row-major input takes 16-byte
// loads when K % 8 == 0 and single floats otherwise.
template <bool OCT>
__device__ __forceinline__ void slab_get(const float *pool, int64_t r, int64_t r1, int cbase,
                                         int K, int tid, float (&v)[8]) {
  if (OCT) {
    const int64_t rb = r + 8 * (tid >> 7);
    const int64_t rr = rb < r1 ? rb : ((r1 - 1) & ~int64_t(7));
    const int c = cbase + (tid & 127);
    const float *p = pool + ((rr >> 3) * K + (c < K ? c : K - 1)) * 8;
    const float4 a = *reinterpret_cast<const float4 *>(p);
    const float4 b = *reinterpret_cast<const float4 *>(p + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
    const int64_t row = r + (tid >> 4);
    const float *p = pool + (row < r1 ? row : r1 - 1) * int64_t(K);
    const int c = cbase + (tid & 15) * 8;
    if ((K & 7) == 0) {
      const float *q = p + (c < K ? c : K - 8);
      const float4 a = *reinterpret_cast<const float4 *>(q);
      const float4 b = *reinterpret_cast<const float4 *>(q + 4);
      v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
      v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = p[c + q < K ? c + q : K - 1];
    }
  }
}

// the row permutation of slab column c (c < kSB): an XOR of whole 4-row groups
__device__ __forceinline__ int slab_swz(int c) { return ((c >> 3) & 15) << 2; }

// Stores the 32 rows h * 32 ... of a slab (r is the first of them).
template <bool OCT>
__device__ __forceinline__ void slab_put(float *S, int h, int64_t r, int64_t r1, int cbase, int K,
                                         int tid, const float (&v)[8]) {
  float m[8];
  if (OCT) {
    const int64_t rb = r + 8 * (tid >> 7);
    const int c = tid & 127;
    const bool cok = cbase + c < K;
#pragma unroll
    for (int q = 0; q < 8; ++q) m[q] = (cok && rb + q < r1) ? v[q] : 0.0f;
    const int row = 32 * h + 8 * (tid >> 7);
    float *d = S + c * kSLd;
    *reinterpret_cast<float4 *>(d + (row ^ slab_swz(c))) = make_float4(m[0], m[1], m[2], m[3]);
    *reinterpret_cast<float4 *>(d + ((row + 4) ^ slab_swz(c))) =
        make_float4(m[4], m[5], m[6], m[7]);
  } else {
    const bool rok = r + (tid >> 4) < r1;
    const int c0 = (tid & 15) * 8;
    const int c = cbase + c0;
#pragma unroll
    for (int q = 0; q < 8; ++q) m[q] = (rok && c + q < K) ? v[q] : 0.0f;
    const int row = (32 * h + (tid >> 4)) ^ slab_swz(c0);  // (the 8 columns share slab_swz)
#pragma unroll
    for (int q = 0; q < 8; ++q) S[(c0 + q) * kSLd + row] = m[q];
  }
}

// The 32x32 tile (ti, tj) of one LDS slab's products.  The slab's rows are
// split between the two lane halves (half h takes rows h kSlab/2 ...), so
// that each lane reads four consecutive rows of its column at once.
__device__ __forceinline__ void gram_tile(const float *A, const float *Bm, int lane, int ti, int tj,
                                          floatx16 &acc) {
  const int ca = 32 * ti + (lane & 31), cb = 32 * tj + (lane & 31);
  const int h = (lane >> 5) * (kSlab / 2);
  const float *pa = A + ca * kSLd;
  const float *pb = Bm + cb * kSLd;
  const int sa = slab_swz(ca), sb = slab_swz(cb);
#pragma unroll
  for (int s = 0; s < kSlab / 2; s += 4) {
    const float4 a = *reinterpret_cast<const float4 *>(pa + ((h + s) ^ sa));
    const float4 b = *reinterpret_cast<const float4 *>(pb + ((h + s) ^ sb));
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b.w, acc, 0, 0, 0);
  }
}

template <bool OCT>
__global__ void __launch_bounds__(kGT32)
k_jgram(const float *__restrict__ pool, const float *__restrict__ poolB, int64_t n, int K, int nsb,
        int npairs, int64_t rows_per_chunk, double *__restrict__ partial) {
  __shared__ __attribute__((aligned(16))) float As[2][kSB * kSLd];
  __shared__ __attribute__((aligned(16))) float Bs[2][kSB * kSLd];
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int pair = int(lb % npairs);
  const int64_t chunk = lb / npairs;
  // symmetric (poolB null): super-tile pairs a <= b of V^T V;
  // cross: every (a, b) of V^T W with W = poolB
  const bool cross = poolB != nullptr;
  const int2 ab = cross ? make_int2(pair / nsb, pair % nsb) : pair_of(pair, nsb);
  const bool diag = !cross && ab.x == ab.y;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  // Off-diagonal and cross pairs: wave w owns tile (w / 4, (w - w / 4) % 4),
  // so that the tiles of one row or one column of the super tile sit on the
  // four SIMDs (wave w runs on SIMD w % 4) and tiles past column K, which are
  // skipped, leave every SIMD the same share.  Diagonal pairs: waves 0..9
  // own the ten tiles on or above the diagonal, row by row, and waves 10..15
  // only write zeros for the six tiles below it.
  int ti = w >> 2, tj = ((w & 3) - (w >> 2)) & 3;
  bool on = true;
  if (diag) {
    const int t = w < 10 ? w : w - 10;
    const int r = w < 10 ? (t < 4 ? 0 : t < 7 ? 1 : t < 9 ? 2 : 3)
                         : (t < 1 ? 1 : t < 3 ? 2 : 3);
    const int first = w < 10 ? (r == 0 ? 0 : r == 1 ? 4 : r == 2 ? 7 : 9)
                             : (r == 1 ? 0 : r == 2 ? 1 : 3);
    ti = r;
    tj = w < 10 ? r + (t - first) : t - first;
    on = w < 10;
  }
  on = on && ab.x * kSB + 32 * ti < K && ab.y * kSB + 32 * tj < K;
  // the first half of the block stages super block a, the second half b
  // (a diagonal pair stages one super block)
  const bool loader = !diag || tid < kGT32 / 2;
  const float *src = tid < kGT32 / 2 ? pool : (cross ? poolB : pool);
  const int cb = (tid < kGT32 / 2 ? ab.x : ab.y) * kSB;
  const int lt = tid & (kGT32 / 2 - 1);
  const int64_t r0 = chunk * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < n ? r0 + rows_per_chunk : n;
  floatx16 acc;
  double d[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) { acc[v] = 0.0f; d[v] = 0.0; }
  // a slab is staged as 32-row halves.  Slab t + 1 goes to LDS at the start
  // of iteration t (its loads were issued one iteration earlier), then the
  // loads of slab t + 2 are issued, then slab t's products run: the LDS
  // writes overlap other waves' products and the loads have a whole
  // iteration to arrive.
  float rv[kSlab / 32][8];
  auto fetch = [&](int64_t r) __attribute__((always_inline)) {
#pragma unroll
    for (int h = 0; h < kSlab / 32; ++h) slab_get<OCT>(src, r + 32 * h, r1, cb, K, lt, rv[h]);
  };
  auto stash = [&](int b, int64_t r) __attribute__((always_inline)) {
    float *S = tid < kGT32 / 2 ? As[b] : Bs[b];
#pragma unroll
    for (int h = 0; h < kSlab / 32; ++h) slab_put<OCT>(S, h, r + 32 * h, r1, cb, K, lt, rv[h]);
  };
  if (loader && r0 < r1) {  // (an empty chunk has nothing to stage)
    fetch(r0);
    stash(0, r0);
    if (r0 + kSlab < r1) fetch(r0 + kSlab);
  }
  __syncthreads();
  int buf = 0, slabs = 0;
  for (int64_t r = r0; r < r1; r += kSlab) {
    if (loader && r + kSlab < r1) {
      stash(buf ^ 1, r + kSlab);
      if (r + 2 * kSlab < r1) fetch(r + 2 * kSlab);
    }
    const float *A = As[buf];
    const float *Bm = diag ? As[buf] : Bs[buf];
    if (on) gram_tile(A, Bm, lane, ti, tj, acc);
    if (++slabs == kFlushSlabs) {
      slabs = 0;
#pragma unroll
      for (int v = 0; v < 16; ++v) { d[v] += double(acc[v]); acc[v] = 0.0f; }
    }
    __syncthreads();
    buf ^= 1;
  }
  double *out = partial + (chunk * npairs + pair) * (16 * 1024);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int j = lane & 31;
    out[(ti * 4 + tj) * 1024 + i * 32 + j] = on ? d[v] + double(acc[v]) : 0.0;
  }
}

// The symmetric Gram of an FP32 pool in the row-octet layout, with the slabs
// staged by direct global-to-LDS loads (global_load_lds_dwordx4): block,
// wave and output layout as k_jgram.  A slab of a super block is kept as
// [octet (8)][column (128)][8 rows], i.e. the pool's own layout; one wave
// load fills 32 columns of one octet.  The 16-byte halves of column c sit
// swapped when bit 3 of c is set, so that the operand reads of 16
// consecutive columns hit distinct banks.  Slab t + 1 loads into the other
// buffer during slab t's products; one barrier per slab.  Octets past the
// last row are written as zeros instead (the pool's padding rows inside the
// last octet are zero).
constexpr int kGO = 8 * kSB * 8;  // floats of one staged slab of a super block

__device__ __forceinline__ void gram_tile_oct(const float *A, const float *Bm, int lane, int ti,
                                              int tj, floatx16 &acc) {
  const int li = lane & 31, h = lane >> 5;
  const int sw = (li >> 3) & 1;
  const float *pa = A + (32 * ti + li) * 8;
  const float *pb = Bm + (32 * tj + li) * 8;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int off = (4 * h + (q >> 1)) * (kSB * 8) + 4 * ((q & 1) ^ sw);
    const float4 a = *reinterpret_cast<const float4 *>(pa + off);
    const float4 b = *reinterpret_cast<const float4 *>(pb + off);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b.w, acc, 0, 0, 0);
  }
}

__global__ void __launch_bounds__(kGT32)
k_jgram_dma(const float *__restrict__ pool, int64_t n, int K, int nsb, int npairs,
            int64_t rows_per_chunk, double *__restrict__ partial) {
  // buffers 0 and 1 of both super blocks as separate LDS objects (the loads
  // into one buffer are then disjoint from the reads of the other)
  __shared__ __attribute__((aligned(1024))) float A0[kGO];
  __shared__ __attribute__((aligned(1024))) float A1[kGO];
  __shared__ __attribute__((aligned(1024))) float B0[kGO];
  __shared__ __attribute__((aligned(1024))) float B1[kGO];
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int pair = int(lb % npairs);
  const int64_t chunk = lb / npairs;
  const int2 ab = pair_of(pair, nsb);
  const bool diag = ab.x == ab.y;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  int ti = w >> 2, tj = ((w & 3) - (w >> 2)) & 3;  // (tiles of a row or column on 4 SIMDs)
  bool on = true;
  if (diag) {
    const int t = w < 10 ? w : w - 10;
    const int r = w < 10 ? (t < 4 ? 0 : t < 7 ? 1 : t < 9 ? 2 : 3)
                         : (t < 1 ? 1 : t < 3 ? 2 : 3);
    const int first = w < 10 ? (r == 0 ? 0 : r == 1 ? 4 : r == 2 ? 7 : 9)
                             : (r == 1 ? 0 : r == 2 ? 1 : 3);
    ti = r;
    tj = w < 10 ? r + (t - first) : t - first;
    on = w < 10;
  }
  on = on && ab.x * kSB + 32 * ti < K && ab.y * kSB + 32 * tj < K;  // tiles past K skipped
  const int64_t r0 = chunk * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < n ? r0 + rows_per_chunk : n;
  const int64_t olast = (n - 1) >> 3;
  // wave w stages the pieces 4w..4w+3 of a slab: piece = (super block,
  // octet, 32-column group); a diagonal pair stages one super block
  // (waves 0..7 fill super block a, waves 8..15 super block b: each branch
  // writes one known LDS object)
  auto piece_load = [&](int64_t r, float *S, int cb, int piece) __attribute__((always_inline)) {
    const int o = (piece >> 2) & 7, cg = piece & 3;
    float *dst = S + o * (kSB * 8) + cg * 256;
    const int64_t og = (r >> 3) + o;
    if (og <= olast) {
      const int cl = 32 * cg + (lane >> 1);  // column within the super block
      const int hf = (lane & 1) ^ ((cl >> 3) & 1);
      const int col = cb + cl < K ? cb + cl : K - 1;
      __builtin_amdgcn_global_load_lds(pool + (og * K + col) * 8 + 4 * hf, dst, 16, 0, 0);
    } else {
      *reinterpret_cast<float4 *>(dst + 4 * lane) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
  };
  auto dma = [&](int64_t r, float *SA, float *SB) __attribute__((always_inline)) {
    if (w < 8) {
#pragma unroll
      for (int u = 0; u < 4; ++u) piece_load(r, SA, ab.x * kSB, 4 * w + u);
    } else if (!diag) {
#pragma unroll
      for (int u = 0; u < 4; ++u) piece_load(r, SB, ab.y * kSB, 4 * (w - 8) + u);
    }
  };
  floatx16 acc;
  double d[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) { acc[v] = 0.0f; d[v] = 0.0; }
  auto mul = [&](const float *SA, const float *SB) __attribute__((always_inline)) {
    // (two copies, so that each reads known LDS objects)
    if (!on) return;
    if (diag) gram_tile_oct(SA, SA, lane, ti, tj, acc);
    else gram_tile_oct(SA, SB, lane, ti, tj, acc);
  };
  if (r0 < r1) {
    dma(r0, A0, B0);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  }
  __syncthreads();
  int slabs = 0;
  auto flush = [&]() __attribute__((always_inline)) {
    if (++slabs == 2) {  // float32 sums over 128 rows, then float64
      slabs = 0;
#pragma unroll
      for (int v = 0; v < 16; ++v) { d[v] += double(acc[v]); acc[v] = 0.0f; }
    }
  };
  for (int64_t r = r0; r < r1; r += 128) {
    if (r + 64 < r1) dma(r + 64, A1, B1);
    mul(A0, B0);
    flush();
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    if (r + 64 >= r1) break;
    if (r + 128 < r1) dma(r + 128, A0, B0);
    mul(A1, B1);
    flush();
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
  }
  double *out = partial + (chunk * npairs + pair) * (16 * 1024);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int j = lane & 31;
    out[(ti * 4 + tj) * 1024 + i * 32 + j] = on ? d[v] + double(acc[v]) : 0.0;
  }
}

// G[gi][gj] from the chunk-summed tiles (mirrored unless `cross`).
__global__ void k_jgram_scatter(const double *__restrict__ sums, int nsb, int npairs, int K,
                                int cross, double *__restrict__ G) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(npairs) * 16 * 1024) return;
  const int pair = int(e / (16 * 1024));
  const int rem = int(e % (16 * 1024));
  const int wt = rem / 1024, ij = rem % 1024;
  const int ti = wt / 4, tj = wt % 4, i = ij / 32, j = ij % 32;
  const int2 ab = cross ? make_int2(pair / nsb, pair % nsb) : pair_of(pair, nsb);
  if (!cross && ab.x == ab.y && tj < ti) return;
  const int gi = ab.x * kSB + 32 * ti + i;
  const int gj = ab.y * kSB + 32 * tj + j;
  if (gi >= K || gj >= K) return;
  const double s = sums[e];
  G[int64_t(gi) * K + gj] = s;
  if (!cross) G[int64_t(gj) * K + gi] = s;
}

// The Gram of a float64 pool in the row-octet layout (the float64 debug
// basis): workgroup = (row chunk, super-block pair a <= b), its partial in
// the layout k_jgram_scatter reads (16 tiles of 32 x 32 per pair).  Thread
// (ty, tx) accumulates rows 8 ty .. 8 ty + 7 of block a against columns
// 8 tx .. 8 tx + 7 of block b in float64, over the chunk's rows staged 16 at
// a time in LDS.
constexpr int kG64Rows = 16;

__global__ void __launch_bounds__(256)
k_jgram_f64(const double *__restrict__ P, int64_t n, int K, int nsb, int npairs, int64_t rpc,
            double *__restrict__ partial) {
  __shared__ double As[kG64Rows][kSB + 1];
  __shared__ double Bs[kG64Rows][kSB + 1];
  const int pair = int(blockIdx.x % npairs);
  const int64_t chunk = int64_t(blockIdx.x) / npairs;
  const int2 ab = pair_of(pair, nsb);
  const int64_t r0 = chunk * rpc;
  const int64_t r1 = r0 + rpc < n ? r0 + rpc : n;
  const int t = threadIdx.x, ty = t / 16, tx = t % 16;
  double acc[8][8];
#pragma unroll
  for (int u = 0; u < 8; ++u)
#pragma unroll
    for (int v = 0; v < 8; ++v) acc[u][v] = 0.0;
  for (int64_t r = r0; r < r1; r += kG64Rows) {
    for (int e = t; e < kG64Rows * kSB; e += 256) {
      const int rr = e % kG64Rows, cc = e / kG64Rows;
      const int64_t row = r + rr;
      const int ca = ab.x * kSB + cc, cb = ab.y * kSB + cc;
      As[rr][cc] = (row < r1 && ca < K) ? P[((row >> 3) * K + ca) * 8 + (row & 7)] : 0.0;
      Bs[rr][cc] = (row < r1 && cb < K) ? P[((row >> 3) * K + cb) * 8 + (row & 7)] : 0.0;
    }
    __syncthreads();
    for (int rr = 0; rr < kG64Rows; ++rr) {
      double av[8], bv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        av[u] = As[rr][8 * ty + u];
        bv[u] = Bs[rr][8 * tx + u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int v = 0; v < 8; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
    }
    __syncthreads();
  }
  double *out = partial + int64_t(blockIdx.x) * 16 * 1024;
#pragma unroll
  for (int u = 0; u < 8; ++u)
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int i = 8 * ty + u, j = 8 * tx + v;
      out[((i / 32) * 4 + j / 32) * 1024 + (i % 32) * 32 + (j % 32)] = acc[u][v];
    }
}

// Q = V Rinv in float64 for the float64 debug basis: V in the row-octet
// layout, Rinv upper triangular (Kp x Kp, row-major), Q row-major n x K.
// Workgroup = 64 x 64 output tile, thread (ty, tx) = 4 x 4 outputs; the k
// loop stops at the tile's last column, 16 k at a time staged in LDS.
__global__ void __launch_bounds__(256)
k_japply_f64(const double *__restrict__ V, double *__restrict__ Q, int64_t n, int K, int Kp,
             const double *__restrict__ Rinv) {
  __shared__ double Vs[16][65];
  __shared__ double Rs[16][65];
  const int ncb = (K + 63) / 64;
  const int64_t r0 = int64_t(blockIdx.x / ncb) * 64;
  const int c0 = int(blockIdx.x % ncb) * 64;
  const int t = threadIdx.x, ty = t / 16, tx = t % 16;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  const int kend = K < c0 + 64 ? K : c0 + 64;
  for (int k0 = 0; k0 < kend; k0 += 16) {
    for (int e = t; e < 16 * 64; e += 256) {
      const int kk = e / 64, rr = e % 64;
      const int64_t row = r0 + rr;
      const int k = k0 + kk;
      Vs[kk][rr] = (row < n && k < K) ? V[((row >> 3) * K + k) * 8 + (row & 7)] : 0.0;
      Rs[kk][rr] = (k < K && c0 + rr < K) ? Rinv[int64_t(k) * Kp + c0 + rr] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = Vs[kk][4 * ty + u];
        b[u] = Rs[kk][4 * tx + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + 4 * ty + u;
      const int col = c0 + 4 * tx + v;
      if (row < n && col < K) Q[row * K + col] = acc[u][v];
    }
}

// ---------------------------------------------------------------- apply
// Q = V Rinv (n x K times upper-triangular K x K), out of place.  Block =
// 128 x 128 output tile; 8 waves of 64 x 32 (2 x 1 MFMA tiles) for the FP32
// pool, 4 waves of 64 x 64 for the BF16 pool.  The k loop runs over 32-wide
// chunks up to the tile's last column (Rinv is zero below its diagonal);
// both operand chunks are staged in LDS, the next one fetched into
// registers during the current chunk's products.
constexpr int kAT = 256;         // BF16 apply workgroup size
constexpr int kAT32 = 512;       // FP32 apply workgroup size
constexpr int kAM = 128, kAN = 128, kAK = 32;
constexpr int kALDA = kAK + 1;   // A chunk [128][33]
constexpr int kALDB = kAN + 1;   // B chunk [32][129]

template <bool RAW>
__global__ void __launch_bounds__(kAT32)
k_japply(const void *__restrict__ V, void *__restrict__ Q, int pool_type, int oct, int64_t n,
         int K, int Kp, const float *__restrict__ Rinv32, int ncb, int full, int accumulate) {
  __shared__ float As[kAM * kALDA];
  __shared__ float Bs[kAK * kALDB];
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int cb = int(lb % ncb);
  const int64_t rt = lb / ncb;
  const int64_t row0 = rt * kAM;
  const int col0 = cb * kAN;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  // the column quarter of wave w rotates with the block, so that the waves
  // which stop early (below) fall on every SIMD in turn
  const int wr = (w >> 2) * 64, wc = int(((w & 3) + lb) & 3) * 32;
  const bool won = col0 + wc < K;  // a wave whose columns are all past K idles
  floatx16 acc[2][1];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 1; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.0f;
  // Rinv is upper triangular: rows past the tile's last column are zero
  const int kend = (!full && col0 + kAN < K) ? col0 + kAN : K;
  // ... and the wave's own columns need rows k < col0 + wc + 32 only
  const int kw = (!full && col0 + wc + 32 < kend) ? col0 + wc + 32 : kend;
  // the next k chunk is fetched into registers while the current one is
  // multiplied: A = 128 rows x 32 columns of V (2 groups of 8 values per
  // thread), B = 32 rows x 128 columns of Rinv32 (4 float4 per thread)
  float ra[1][8];
  float4 rb[2];
  // RAW (an FP32 row-major V, K % 8 == 0): loads at clamped addresses,
  // masked in stash, which keeps them in flight during the products
  auto fetch = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int h = 0; h < 1; ++h) {
      const int g = tid + kAT32 * h;
      if (RAW) {
        const int r = g / (kAK / 8), c8 = (g % (kAK / 8)) * 8;
        const int64_t row = row0 + r < n ? row0 + r : n - 1;
        const int c = k0 + c8 < K ? k0 + c8 : K - 8;
        const float *p = reinterpret_cast<const float *>(V) + row * K + c;
        const float4 x = *reinterpret_cast<const float4 *>(p);
        const float4 y = *reinterpret_cast<const float4 *>(p + 4);
        ra[h][0] = x.x; ra[h][1] = x.y; ra[h][2] = x.z; ra[h][3] = x.w;
        ra[h][4] = y.x; ra[h][5] = y.y; ra[h][6] = y.z; ra[h][7] = y.w;
      } else if (oct) {
        const int o = g / kAK, c = g % kAK;
        load8oct(V, pool_type, row0 + 8 * o, n, k0 + c, K, ra[h]);
      } else {
        const int r = g / (kAK / 8), c8 = (g % (kAK / 8)) * 8;
        load8(V, pool_type, row0 + r, n, k0 + c8, K, ra[h]);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int g = tid + kAT32 * h;
      const int r = g / (kAN / 4), c4 = (g % (kAN / 4)) * 4;
      const int kk = k0 + r < kend ? k0 + r : kend - 1, cc = col0 + c4 < Kp ? col0 + c4 : Kp - 4;
      rb[h] = *reinterpret_cast<const float4 *>(Rinv32 + int64_t(kk) * Kp + cc);
    }
  };
  auto stash = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int h = 0; h < 1; ++h) {
      const int g = tid + kAT32 * h;
      if (oct) {
        const int o = g / kAK, c = g % kAK;
#pragma unroll
        for (int q = 0; q < 8; ++q) As[(8 * o + q) * kALDA + c] = (k0 + c < kend) ? ra[h][q] : 0.0f;
      } else {
        const int r = g / (kAK / 8), c8 = (g % (kAK / 8)) * 8;
#pragma unroll
        for (int q = 0; q < 8; ++q) As[r * kALDA + c8 + q] = (k0 + c8 + q < kend) ? ra[h][q] : 0.0f;
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int g = tid + kAT32 * h;
      const int r = g / (kAN / 4), c4 = (g % (kAN / 4)) * 4;
      const bool ok = k0 + r < kend && col0 + c4 < Kp;
      float *d = Bs + r * kALDB + c4;
      d[0] = ok ? rb[h].x : 0.0f; d[1] = ok ? rb[h].y : 0.0f;
      d[2] = ok ? rb[h].z : 0.0f; d[3] = ok ? rb[h].w : 0.0f;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < kend; k0 += kAK) {
    __syncthreads();
    stash(k0);
    __syncthreads();
    if (k0 + kAK < kend) fetch(k0 + kAK);
    if (k0 >= kw || !won) continue;
#pragma unroll 4
    for (int s = 0; s < kAK / 2; ++s) {
      const int kk = 2 * s + (lane >> 5);
      float a_op[2], b_op[1];
#pragma unroll
      for (int a = 0; a < 2; ++a) a_op[a] = As[(wr + 32 * a + (lane & 31)) * kALDA + kk];
#pragma unroll
      for (int b = 0; b < 1; ++b) b_op[b] = Bs[kk * kALDB + wc + 32 * b + (lane & 31)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 1; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a_op[a], b_op[b], acc[a][b], 0, 0, 0);
    }
  }
  if (accumulate) {  // float32 only: the tile's old values are read first, all at once
    float *Qf = reinterpret_cast<float *>(Q);
    const int col = col0 + wc + (lane & 31);
    const int cc = col < K ? col : K - 1;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      float old[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = row0 + wr + 32 * a + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        old[v] = Qf[(row < n ? row : n - 1) * K + cc];
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = row0 + wr + 32 * a + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (row < n && col < K) Qf[row * K + col] = old[v] + acc[a][0][v];
      }
    }
    return;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 1; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = row0 + wr + 32 * a + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int col = col0 + wc + 32 * b + (lane & 31);
        if (row < n && col < K) {
          if (pool_type == kPoolF32)
            reinterpret_cast<float *>(Q)[row * K + col] = acc[a][b][v];
          else
            reinterpret_cast<uint16_t *>(Q)[row * K + col] = f2bf(acc[a][b][v]);
        }
      }
}

// Q = V Rinv for the float32 pool, Rinv upper triangular (Kp x Kp, zero
// outside K x K), read through its transpose RT (RT[c][k] = Rinv[k][c]): no
// LDS and no barriers.  A workgroup of four waves takes 64 rows; the
// 32-column output tiles are dealt to the waves in snake order of their work
// (tile c needs the c + 1 leading 32-row chunks of Rinv), so the waves'
// shares of the triangle are about equal, at most 4 tiles each.  Operands
// come straight from global memory into registers, kA2G k steps at a time,
// the next group loaded while the current one is multiplied:
//  * MFMA step s of a 32-wide k chunk pairs k = 32 kc + s (lanes 0-31) with
//    32 kc + 16 + s (lanes 32-63), so a lane's B values for kA2G steps are
//    kA2G consecutive entries of one row of RT (one 16-byte load);
//  * the wave's two row tiles interleave: lane i of row tile r holds local
//    row 2i + r, so in the row-octet layout one 8-byte load gives a lane its
//    A values of both row tiles;
//  * a row-major pool with K % 4 == 0 (VEC) gives a lane its kA2G k values
//    of one row as one 16-byte load (a group's first k is a multiple of 4,
//    so the group lies wholly inside or wholly past column K).
constexpr int kA2T = 256;
constexpr int kA2Rows = 64;
constexpr int kA2G = 4;  // k steps per register group (4 groups per 32-wide chunk)

template <bool OCT, bool VEC, int NA>
__device__ __forceinline__ void tri_chunks(const float *__restrict__ Vw,
                                           const float *__restrict__ RT, uint32_t vo,
                                           uint32_t vo1, int K, int Kp,
                                           const uint32_t (&rb)[4], int h, int kc0, int kc1,
                                           floatx16 (&acc)[2][4]) {
  constexpr int GPC = 16 / kA2G;  // register groups per 32-wide chunk
  const int g0 = kc0 * GPC, g1 = kc1 * GPC;
  if (g0 >= g1) return;
  // The loads are unconditional (k clamped into the row, rows clamped in the
  // caller) and their values are masked only where the products use them,
  // so the next group's loads stay in flight during the current products.
  // A clamped row's products land in output rows that are never stored; a
  // clamped k is zeroed here.
  float a[2][kA2G][2];
  bool kin[2][kA2G];
  float4 b[2][NA];
  const char *vb = reinterpret_cast<const char *>(Vw);
  const char *rt = reinterpret_cast<const char *>(RT);
  auto load = [&](int g, int buf) __attribute__((always_inline)) {
    const int kb = 32 * (g / GPC) + 16 * h + kA2G * (g % GPC);  // first k of the group
    if constexpr (VEC) {
      const bool in = kb < K;
      const uint32_t kk = in ? uint32_t(kb) : 0u;
      const float4 t0 = *reinterpret_cast<const float4 *>(vb + 4u * (vo + kk));
      const float4 t1 = *reinterpret_cast<const float4 *>(vb + 4u * (vo1 + kk));
      a[buf][0][0] = t0.x; a[buf][1][0] = t0.y; a[buf][2][0] = t0.z; a[buf][3][0] = t0.w;
      a[buf][0][1] = t1.x; a[buf][1][1] = t1.y; a[buf][2][1] = t1.z; a[buf][3][1] = t1.w;
#pragma unroll
      for (int s = 0; s < kA2G; ++s) kin[buf][s] = in;
    } else {
#pragma unroll
      for (int s = 0; s < kA2G; ++s) {
        const int k = kb + s;
        kin[buf][s] = k < K;
        const uint32_t kk = k < K ? uint32_t(k) : 0u;
        if constexpr (OCT) {
          // rows 2i and 2i + 1 sit side by side in their octet
          const float2 t = *reinterpret_cast<const float2 *>(vb + 4u * (vo + 8u * kk));
          a[buf][s][0] = t.x;
          a[buf][s][1] = t.y;
        } else {
          a[buf][s][0] = *reinterpret_cast<const float *>(vb + 4u * (vo + kk));
          a[buf][s][1] = *reinterpret_cast<const float *>(vb + 4u * (vo1 + kk));
        }
      }
    }
#pragma unroll
    for (int j = 0; j < NA; ++j)
      b[buf][j] = *reinterpret_cast<const float4 *>(rt + 4u * (rb[j] + uint32_t(kb)));
  };
  auto mul = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < kA2G; ++s)
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        const float bv = s == 0 ? b[buf][j].x : s == 1 ? b[buf][j].y : s == 2 ? b[buf][j].z
                                                                              : b[buf][j].w;
#pragma unroll
        for (int r = 0; r < 2; ++r)
          acc[r][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(kin[buf][s] ? a[buf][s][r] : 0.0f, bv,
                                                           acc[r][j], 0, 0, 0);
      }
  };
  // two register groups in flight: the next group's loads are issued before
  // the current group's products
  load(g0, 0);
  int g = g0;
  for (; g + 2 <= g1; g += 2) {
    load(g + 1, 1);
    mul(0);
    if (g + 2 < g1) load(g + 2, 0);
    mul(1);
  }
  if (g < g1) mul(0);
}

template <bool OCT, bool VEC>
__global__ void __launch_bounds__(kA2T) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_japply_tri(const float *__restrict__ V, float *__restrict__ Q, int64_t n, int K, int Kp,
             const float *__restrict__ RT) {
  static_assert(kA2G == 4, "a group's B values (and VEC's A values) are one float4");
  static_assert(!(OCT && VEC), "VEC is the row-major layout");
  const int64_t row0 = int64_t(xcd_block(blockIdx.x, gridDim.x)) * kA2Rows;
  // the wave index and everything derived from it are wave-uniform (scalar)
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int li = lane & 31, h = lane >> 5;
  const int nct = Kp / 32;
  // this wave's tiles, in descending order of their column (and work): in
  // the snake, wave w takes positions t with t % 8 in {w, 7 - w}
  int ct[4] = {0, 0, 0, 0};
  int nt = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int t = 8 * (q >> 1) + ((q & 1) ? 7 - w : w);
    if (t < nct) ct[nt++] = nct - 1 - t;
  }
  if (nt == 0) return;
  // the workgroup's rows of V from a uniform base (row0 is a multiple of 8)
  const float *Vw = OCT ? V + (row0 >> 3) * int64_t(K) * 8 : V + row0 * int64_t(K);
  const int64_t last = n - 1 - row0;  // the last valid local row
  // a valid row pair to read (masked out above when past the end)
  const uint32_t r0 = uint32_t(2 * li <= last ? 2 * li : (last & ~int64_t(1)));
  const uint32_t r1 = uint32_t(2 * li + 1 <= last ? 2 * li + 1 : last);
  const uint32_t vo = OCT ? ((r0 >> 3) * uint32_t(K)) * 8u + (r0 & 7u) : r0 * uint32_t(K);
  const uint32_t vo1 = r1 * uint32_t(K);
  uint32_t rb[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) rb[j] = uint32_t(32 * ct[j] + li) * uint32_t(Kp);
  floatx16 acc[2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[r][j][v] = 0.0f;
  // k chunks 0 .. ct[nt-1] with all nt tiles, then one tile fewer after each
  // tile's diagonal chunk
  const int e3 = nt >= 4 ? ct[3] + 1 : 0;
  const int e2 = nt >= 3 ? ct[2] + 1 : 0;
  const int e1 = nt >= 2 ? ct[1] + 1 : 0;
  const int e0 = ct[0] + 1;
  if (nt >= 4) tri_chunks<OCT, VEC, 4>(Vw, RT, vo, vo1, K, Kp, rb, h, 0, e3, acc);
  if (nt >= 3) tri_chunks<OCT, VEC, 3>(Vw, RT, vo, vo1, K, Kp, rb, h, e3, e2, acc);
  if (nt >= 2) tri_chunks<OCT, VEC, 2>(Vw, RT, vo, vo1, K, Kp, rb, h, e2, e1, acc);
  tri_chunks<OCT, VEC, 1>(Vw, RT, vo, vo1, K, Kp, rb, h, e1, e0, acc);
  float *Qw = Q + row0 * int64_t(K);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (j >= nt) continue;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rl = 2 * (8 * (v >> 2) + 4 * h + (v & 3)) + r;
        const int col = 32 * ct[j] + li;
        if (rl <= last && col < K) Qw[uint32_t(rl) * uint32_t(K) + uint32_t(col)] = acc[r][j][v];
      }
  }
}

// Q = V R^-1 for an FP32 pool in the row-octet layout, operands staged in
// LDS by direct global-to-LDS loads (global_load_lds_dwordx4).  A workgroup
// of 16 waves takes a panel of 256 rows and one of two column sets: set g
// holds the 32-column tiles j with (nct - 1 - j) % 2 == g, in descending
// order (at most 8 slots), which gives the two sets nearly equal triangular
// work (tile j takes the k chunks 0..j, R^-1 being upper triangular).  Wave
// w owns rows 32 (w % 8) .. 32 (w % 8) + 31 of the panel and the slots
// w / 8, w / 8 + 2, w / 8 + 4, w / 8 + 6 (one 32x32 FP32 accumulator each;
// alternate slots keep the two halves' triangular work even).  Per 32-wide
// k chunk, two LDS buffers:
//   A [k][256 rows]: one wave load is one k of the panel (lane i: rows
//     4i..4i+3, a half octet); the k rows 16..31 sit 32 floats further
//     on, so that the two lane halves (k and k + 16) read distinct banks;
//   B [slot][32 columns][32 k] from the transposed copy RT[col][k], the
//     16-byte k group x of column c stored at slot x ^ ((c >> 1) & 7), so
//     that the operand reads of 16 consecutive columns hit distinct banks.
// Chunk c + 1 is loaded into the other buffer during chunk c's products;
// one barrier per chunk.  MFMA k-step s of lane half h is k = 16h + s of the
// chunk, in A and B alike.  Tiles past their last chunk drop out (loads and
// products).  Rows past n and k past K read clamped addresses: such rows
// are never stored and R^-1 is zero in rows k >= K.
constexpr int kDR = 256;   // rows per panel
constexpr int kDT = 1024;  // threads: 16 waves
constexpr int kPMaxTiles = 8;
constexpr int kWT = 4;     // slots per wave
typedef float f32x4 __attribute__((ext_vector_type(4)));  // (register-friendly float4)

__global__ void __launch_bounds__(kDT)
k_japply_dma(const float *__restrict__ V, float *__restrict__ Q, int64_t n, int K, int Kp,
             const float *__restrict__ RT) {
  // two buffers as four separate LDS objects, so that the compiler sees
  // the loads into one buffer as disjoint from the reads of the other
  __shared__ __attribute__((aligned(1024))) float As0[32 * kDR + 32];
  __shared__ __attribute__((aligned(1024))) float As1[32 * kDR + 32];
  __shared__ __attribute__((aligned(1024))) float Bs0[kPMaxTiles * 32 * 32];
  __shared__ __attribute__((aligned(1024))) float Bs1[kPMaxTiles * 32 * 32];
  const auto aoff = [](int kk) { return kk * kDR + ((kk >> 4) << 5); };
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t r0 = (lb >> 1) * kDR;
  const int set = int(lb & 1);
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int rt = w & 7, tg = w >> 3;
  const int lane = threadIdx.x & 63, li = lane & 31, h = lane >> 5;
  const int nct = Kp / 32;
  const int top = nct - 1 - set;  // this set's tiles: slot ts is tile top - 2 ts
  const int ntile = top >= 0 ? top / 2 + 1 : 0;
  if (ntile == 0) return;
  const int nch = top + 1;  // chunks 0..top
  const int64_t olast = (n - 1) >> 3;
  int64_t og = (r0 >> 3) + (lane >> 1);
  og = og <= olast ? og : olast;
  const float *va = V + og * int64_t(K) * 8 + 4 * (lane & 1);
  // each wave loads k rows 2w, 2w + 1 of A and the (slot, 8-column) pieces
  // 2w, 2w + 1 of B
  auto dma = [&](int c, float *A, float *B) __attribute__((always_inline)) {
    const int k0 = 32 * c;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int kk = 2 * w + u;
      const int k = k0 + kk < K ? k0 + kk : K - 1;
      __builtin_amdgcn_global_load_lds(va + int64_t(k) * 8, A + aoff(kk), 16, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int piece = 2 * w + u;
      const int ts = piece >> 2, t8 = piece & 3;
      if (ts < ntile && top - 2 * ts >= c) {
        const int cl = 8 * t8 + (lane >> 3);  // column within the tile
        const int col = 32 * (top - 2 * ts) + cl;
        const int x = (lane & 7) ^ ((cl >> 1) & 7);
        __builtin_amdgcn_global_load_lds(RT + int64_t(col) * Kp + k0 + 4 * x,
                                         B + (32 * ts + 8 * t8) * 32, 16, 0, 0);
      }
    }
  };
  floatx16 acc[kWT];
#pragma unroll
  for (int u = 0; u < kWT; ++u)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[u][v] = 0.0f;
  auto mul = [&](int c, const float *A, const float *B) __attribute__((always_inline)) {
    const int na = ntile < (top - c) / 2 + 1 ? ntile : (top - c) / 2 + 1;  // active slots
    const float *pa = A + aoff(16 * h) + 32 * rt + li;
    const float *pb = B + li * 32;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float a[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) a[t] = pa[(4 * q + t) * kDR];
      const int xo = 4 * ((4 * h + q) ^ ((li >> 1) & 7));
      f32x4 bv[kWT];
#pragma unroll
      for (int u = 0; u < kWT; ++u)
        bv[u] = *reinterpret_cast<const f32x4 *>(pb + (tg + 2 * u) * 32 * 32 + xo);
#pragma unroll
      for (int u = 0; u < kWT; ++u) {
        if (tg + 2 * u < na) {
          acc[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0], bv[u].x, acc[u], 0, 0, 0);
          acc[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1], bv[u].y, acc[u], 0, 0, 0);
          acc[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[2], bv[u].z, acc[u], 0, 0, 0);
          acc[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[3], bv[u].w, acc[u], 0, 0, 0);
        }
      }
    }
  };
  dma(0, As0, Bs0);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's loads are in LDS
  __syncthreads();
  // chunk c in buffer c % 2 while chunk c + 1 loads into the other; after
  // each chunk every wave waits for its loads, then the barrier
  for (int c = 0; c < nch; c += 2) {
    if (c + 1 < nch) dma(c + 1, As1, Bs1);
    mul(c, As0, Bs0);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    if (c + 1 >= nch) break;
    if (c + 2 < nch) dma(c + 2, As0, Bs0);
    mul(c + 1, As1, Bs1);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
  }
  // D[i][j] of a 32x32 tile: lane holds column li, rows 8 (v >> 2) + 4 h + (v & 3)
#pragma unroll
  for (int u = 0; u < kWT; ++u) {
    const int ts = tg + 2 * u;
    if (ts >= ntile) continue;
    const int col = 32 * (top - 2 * ts) + li;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t row = r0 + 32 * rt + 8 * (v >> 2) + 4 * h + (v & 3);
      if (row < n && col < K) Q[row * K + col] = acc[u][v];
    }
  }
}

// ---------------------------------------------------------------- bf16 pool
// With the pool stored as bfloat16 its values are exact bf16 numbers, so the
// Gram runs on bf16 matrix cores (v_mfma_f32_32x32x16_bf16: exact products,
// float32 sums) with the same float64 flush every 128 rows, and the apply
// multiplies by R^-1 split into bf16 high and low parts (two products,
// relative error about 2^-17 before the bf16 rounding of Q).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int kBSlab = 64;           // rows per LDS slab
constexpr int kBLd = kBSlab + 8;     // LDS column stride (bf16 elements)

// 8 consecutive bf16 of row `row` from column c (zeros past the matrix)
__device__ __forceinline__ uint4 load8_bf16(const uint16_t *pool, int64_t row, int64_t rows,
                                            int c, int K) {
  if (row >= rows || c >= K) return make_uint4(0u, 0u, 0u, 0u);
  const uint16_t *p = pool + row * K + c;
  if ((K & 7) == 0 && c + 8 <= K) return *reinterpret_cast<const uint4 *>(p);
  uint32_t w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t lo = (c + 2 * q < K) ? p[2 * q] : 0u;
    const uint32_t hi = (c + 2 * q + 1 < K) ? p[2 * q + 1] : 0u;
    w[q] = lo | (hi << 16);
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

__device__ __forceinline__ void store_t8(uint16_t *T, int c8, int row, uint4 v) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    T[(c8 + 2 * q) * kBLd + row] = uint16_t(w[q] & 0xFFFFu);
    T[(c8 + 2 * q + 1) * kBLd + row] = uint16_t(w[q] >> 16);
  }
}

// G partials of V^T V for a bf16 pool; block / wave / output layout as k_jgram.
// Slabs of 64 rows are stored transposed in LDS ([column][row]) so that the
// 8 consecutive rows an MFMA lane needs are one 16-byte read.
__global__ void __launch_bounds__(kGT)
k_jgram_bf16(const uint16_t *__restrict__ pool, int oct, int64_t n, int K, int nsb, int npairs,
             int64_t rows_per_chunk, double *__restrict__ partial) {
  __shared__ __attribute__((aligned(16))) uint16_t As[kSB * kBLd];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[kSB * kBLd];
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int pair = int(lb % npairs);
  const int64_t chunk = lb / npairs;
  const int2 ab = pair_of(pair, nsb);
  const bool diag = ab.x == ab.y;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int ti = w >> 1;
  const int tj0 = 2 * (w & 1);
  const bool on0 = !diag || tj0 >= ti;
  const bool on1 = !diag || tj0 + 1 >= ti;
  const int64_t r0 = chunk * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < n ? r0 + rows_per_chunk : n;
  floatx16 acc0, acc1;
  double d0[16], d1[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) { acc0[v] = 0.0f; acc1[v] = 0.0f; d0[v] = 0.0; d1[v] = 0.0; }
  const uint16_t *Bm = diag ? As : Bs;
  int slabs = 0;
  if (oct) {
    // row-octet layout: the 8 rows of a column an MFMA lane needs are one
    // 16-byte load; 4 k-steps (64 rows) are loaded before they are used
    const int ca = ab.x * kSB + 32 * ti + (lane & 31);
    const int cb0 = ab.y * kSB + 32 * tj0 + (lane & 31);
    const int cb1 = cb0 + 32;
    // loads at addresses clamped into the chunk and the row, masked where
    // the products use them; the next 64 rows are loaded during the
    // current rows' products
    const int64_t rlast = r1 > r0 ? ((r1 - 1) & ~int64_t(7)) : 0;
    auto ld = [&](int64_t rb, int c) -> uint4 {
      return *reinterpret_cast<const uint4 *>(
          pool + (((rb < r1 ? rb : rlast) >> 3) * K + (c < K ? c : K - 1)) * 8);
    };
    auto use = [&](const uint4 &u, int64_t rb, int c) -> bf16x8 {
      const uint32_t m = uint32_t(rb < r1) & uint32_t(c < K) ? 0xFFFFFFFFu : 0u;
      const uint4 z = make_uint4(u.x & m, u.y & m, u.z & m, u.w & m);
      return *reinterpret_cast<const bf16x8 *>(&z);
    };
    uint4 ua[2][4], ub0[2][4], ub1[2][4];
    auto fetch = [&](int64_t r, int q) __attribute__((always_inline)) {
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int64_t rb = r + 16 * st + 8 * (lane >> 5);
        ua[q][st] = ld(rb, ca);  // (unconditional, also where a tile is off)
        ub0[q][st] = ld(rb, cb0);
        ub1[q][st] = ld(rb, cb1);
      }
    };
    auto mul = [&](int64_t r, int q) __attribute__((always_inline)) {
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int64_t rb = r + 16 * st + 8 * (lane >> 5);
        const bf16x8 av = use(ua[q][st], rb, ca);
        if (on0)
          acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, use(ub0[q][st], rb, cb0), acc0, 0, 0, 0);
        if (on1)
          acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, use(ub1[q][st], rb, cb1), acc1, 0, 0, 0);
      }
    };
    // two 64-row steps per trip (register buffers 0 and 1 by name), each
    // buffer refilled as soon as its products are issued, so the loads of
    // one step are in flight during the other's products; float32 sums
    // over the trip's 128 rows, then float64
    // (loads past the chunk read clamped addresses and are never used)
    if (r0 < r1) {
      fetch(r0, 0);
      fetch(r0 + 64, 1);
    }
    for (int64_t r = r0; r < r1; r += 128) {
      mul(r, 0);
      fetch(r + 128, 0);
      if (r + 64 < r1) mul(r + 64, 1);
      fetch(r + 192, 1);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        d0[v] += double(acc0[v]); acc0[v] = 0.0f;
        d1[v] += double(acc1[v]); acc1[v] = 0.0f;
      }
    }
  }
  for (int64_t r = r0; r < (oct ? r0 : r1); r += kBSlab) {
    uint4 ra[2], rb[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int g = tid + kGT * h;  // 64 rows x 16 groups of 8 columns
      const int row = g >> 4, c8 = (g & 15) * 8;
      ra[h] = load8_bf16(pool, r + row, r1, ab.x * kSB + c8, K);
      if (!diag) rb[h] = load8_bf16(pool, r + row, r1, ab.y * kSB + c8, K);
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int g = tid + kGT * h;
      const int row = g >> 4, c8 = (g & 15) * 8;
      store_t8(As, c8, row, ra[h]);
      if (!diag) store_t8(Bs, c8, row, rb[h]);
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < kBSlab / 16; ++st) {
      const int kk = 16 * st + 8 * (lane >> 5);
      const bf16x8 a_op = *reinterpret_cast<const bf16x8 *>(As + (32 * ti + (lane & 31)) * kBLd + kk);
      if (on0) {
        const bf16x8 b0 = *reinterpret_cast<const bf16x8 *>(Bm + (32 * tj0 + (lane & 31)) * kBLd + kk);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_op, b0, acc0, 0, 0, 0);
      }
      if (on1) {
        const bf16x8 b1 = *reinterpret_cast<const bf16x8 *>(Bm + (32 * (tj0 + 1) + (lane & 31)) * kBLd + kk);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_op, b1, acc1, 0, 0, 0);
      }
    }
    if (++slabs == 2) {  // float32 sums over 128 rows, then float64
      slabs = 0;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        d0[v] += double(acc0[v]); acc0[v] = 0.0f;
        d1[v] += double(acc1[v]); acc1[v] = 0.0f;
      }
    }
  }
  double *out = partial + (chunk * npairs + pair) * (16 * 1024);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int j = lane & 31;
    out[(ti * 4 + tj0) * 1024 + i * 32 + j] = on0 ? d0[v] + double(acc0[v]) : 0.0;
    out[(ti * 4 + tj0 + 1) * 1024 + i * 32 + j] = on1 ? d1[v] + double(acc1[v]) : 0.0;
  }
}

// RhT[j][k] = bf16(R^-1[k][j]), RlT[j][k] = bf16(R^-1[k][j] - RhT[j][k])
// (transposed, row stride Kp; zero outside K x K)
__global__ void k_split_rinv(const double *__restrict__ Rinv, int K, int Kp,
                             uint16_t *__restrict__ RhT, uint16_t *__restrict__ RlT) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(Kp) * Kp) return;
  const int j = int(idx / Kp), k = int(idx % Kp);
  uint16_t h = 0, l = 0;
  if (j < K && k < K) {
    const float r = float(Rinv[int64_t(k) * Kp + j]);
    h = f2bf(r);
    l = f2bf(r - __uint_as_float(uint32_t(h) << 16));
  }
  RhT[idx] = h;
  RlT[idx] = l;
}

// Q (bf16) = V (bf16) (Rh + Rl): 128 x 128 output tiles, 4 waves of 64 x 64,
// k chunks of 32 (two bf16 MFMA steps) staged in LDS; the k loop stops at the
// tile's last column (R^-1 is upper triangular).
constexpr int kALd = 32 + 8;  // LDS row stride of the bf16 apply chunks
__global__ void __launch_bounds__(kAT)
k_japply_bf16(const uint16_t *__restrict__ V, uint16_t *__restrict__ Q, int oct, int64_t n, int K,
              int Kp, const uint16_t *__restrict__ RhT, const uint16_t *__restrict__ RlT,
              int ncb) {
  __shared__ __attribute__((aligned(16))) uint16_t As[kAM * kALd];
  __shared__ __attribute__((aligned(16))) uint16_t Bh[kAN * kALd];
  __shared__ __attribute__((aligned(16))) uint16_t Bl[kAN * kALd];
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int cb = int(lb % ncb);
  const int64_t rt = lb / ncb;
  const int64_t row0 = rt * kAM;
  const int col0 = cb * kAN;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  floatx16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.0f;
  const int kend = (col0 + kAN < K) ? col0 + kAN : K;
  for (int k0 = 0; k0 < kend; k0 += 32) {
    __syncthreads();
    // A chunk: 128 rows x 32 columns of V = 512 groups of 8 (2 per thread)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int g = tid + kAT * h;
      if (oct) {
        // 8 rows of one column, transposed into the row-major chunk
        const int o = g >> 5, c = g & 31;
        uint4 u = make_uint4(0u, 0u, 0u, 0u);
        const int64_t rb = row0 + 8 * o;
        if (rb < n && k0 + c < kend)
          u = *reinterpret_cast<const uint4 *>(V + ((rb >> 3) * K + k0 + c) * 8);
        const uint32_t wv[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          As[(8 * o + 2 * q) * kALd + c] = uint16_t(wv[q] & 0xFFFFu);
          As[(8 * o + 2 * q + 1) * kALd + c] = uint16_t(wv[q] >> 16);
        }
      } else {
        const int r = g >> 2, k8 = (g & 3) * 8;
        uint4 v = load8_bf16(V, row0 + r, n, k0 + k8, K);
        if (k0 + k8 + 8 > kend) {  // columns past kend are zero in R^-1 anyway
          uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int q = 0; q < 8; ++q)
            if (k0 + k8 + q >= kend) wv[q >> 1] &= (q & 1) ? 0x0000FFFFu : 0xFFFF0000u;
          v = make_uint4(wv[0], wv[1], wv[2], wv[3]);
        }
        *reinterpret_cast<uint4 *>(As + r * kALd + k8) = v;
      }
    }
    // B chunks: columns col0..col0+127 (rows of the transposed split), k0..k0+31
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int g = tid + kAT * h;
      const int j = g >> 2, k8 = (g & 3) * 8;
      uint4 vh = make_uint4(0u, 0u, 0u, 0u), vl = vh;
      if (col0 + j < Kp && k0 + k8 < Kp) {
        vh = *reinterpret_cast<const uint4 *>(RhT + int64_t(col0 + j) * Kp + k0 + k8);
        vl = *reinterpret_cast<const uint4 *>(RlT + int64_t(col0 + j) * Kp + k0 + k8);
      }
      *reinterpret_cast<uint4 *>(Bh + j * kALd + k8) = vh;
      *reinterpret_cast<uint4 *>(Bl + j * kALd + k8) = vl;
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      const int kk = 16 * st + 8 * (lane >> 5);
      bf16x8 a_op[2], bh[2], bl[2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
        a_op[a] = *reinterpret_cast<const bf16x8 *>(As + (wr + 32 * a + (lane & 31)) * kALd + kk);
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        bh[b] = *reinterpret_cast<const bf16x8 *>(Bh + (wc + 32 * b + (lane & 31)) * kALd + kk);
        bl[b] = *reinterpret_cast<const bf16x8 *>(Bl + (wc + 32 * b + (lane & 31)) * kALd + kk);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_op[a], bh[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_op[a], bl[b], acc[a][b], 0, 0, 0);
        }
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = row0 + wr + 32 * a + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int col = col0 + wc + 32 * b + (lane & 31);
        if (row < n && col < K) Q[row * K + col] = f2bf(acc[a][b][v]);
      }
}

// Workgroups a Gram launch aims for.  The FP32 kernels hold 128 KB of LDS,
// one workgroup per CU, and super-tile pairs differ in work (a diagonal pair
// has 10 of the 16 tiles, and tiles past K are skipped); about eight
// workgroups per CU even that out, where two left the CUs that drew two
// large pairs running alone at the end.
constexpr int kGramWG = 2048;

struct GramPlan {
  int nsb = 0, npairs = 0, nchunks = 0;
  int64_t rows_per_chunk = 0;
};

GramPlan gram_plan(int64_t n, int K, bool cross = false) {
  GramPlan p;
  p.nsb = (K + kSB - 1) / kSB;
  p.npairs = cross ? p.nsb * p.nsb : p.nsb * (p.nsb + 1) / 2;
  int64_t want = std::max<int64_t>(1, kGramWG / p.npairs);
  int64_t per = cdiv(std::max<int64_t>(n, 1), want);
  per = std::max<int64_t>(128, cdiv(per, 128) * 128);  // whole slabs of both kernels
  p.rows_per_chunk = per;
  p.nchunks = int(std::max<int64_t>(1, cdiv(n, per)));
  return p;
}

hef_status gram_run(const void *pool, const void *poolB, int pool_type, int64_t n, int K,
                    double *G, Arena &ws, hipStream_t s, bool oct = false) {
  const GramPlan p = gram_plan(n, K, poolB != nullptr);
  const size_t mk = ws.mark();
  double *partial = ws.take<double>(size_t(p.nchunks) * p.npairs * 16 * 1024);
  const int64_t tot = int64_t(p.npairs) * 16 * 1024;
  double *sums = ws.take<double>(tot);
  HEF_WS_CHECK(ws);
  HEF_TRY(zero_async(G, sizeof(double) * K * K, s));
  {
  TimedScope ts(kStOrthGram, s);
  if (pool_type == kPoolF64) {
    if (poolB || !oct) {
      set_error("the float64 pool takes the row-octet Gram only");
      return HEF_ERR_UNSUPPORTED;
    }
    k_jgram_f64<<<int64_t(p.npairs) * p.nchunks, 256, 0, s>>>(
        reinterpret_cast<const double *>(pool), n, K, p.nsb, p.npairs, p.rows_per_chunk, partial);
  } else if (pool_type == kPoolBF16 && !poolB)
    k_jgram_bf16<<<int64_t(p.npairs) * p.nchunks, kGT, 0, s>>>(
        reinterpret_cast<const uint16_t *>(pool), oct, n, K, p.nsb, p.npairs, p.rows_per_chunk,
        partial);
  else if (pool_type != kPoolF32) {
    set_error("cross Gram of a BF16 pool is not supported");
    return HEF_ERR_UNSUPPORTED;
  } else if (oct && !poolB)
    k_jgram_dma<<<int64_t(p.npairs) * p.nchunks, kGT32, 0, s>>>(
        reinterpret_cast<const float *>(pool), n, K, p.nsb, p.npairs, p.rows_per_chunk, partial);
  else if (oct)
    k_jgram<true><<<int64_t(p.npairs) * p.nchunks, kGT32, 0, s>>>(
        reinterpret_cast<const float *>(pool), reinterpret_cast<const float *>(poolB), n, K, p.nsb,
        p.npairs, p.rows_per_chunk, partial);
  else
    k_jgram<false><<<int64_t(p.npairs) * p.nchunks, kGT32, 0, s>>>(
        reinterpret_cast<const float *>(pool), reinterpret_cast<const float *>(poolB), n, K, p.nsb,
        p.npairs, p.rows_per_chunk, partial);
  HEF_LAUNCH_CHECK();
  }
  TimedScope ts(kStOrthReduce, s);
  HEF_TRY(reduce_cols_f64(partial, p.nchunks, tot, sums, s));
  k_jgram_scatter<<<cdiv(tot, 256), 256, 0, s>>>(sums, p.nsb, p.npairs, K, poolB != nullptr, G);
  HEF_LAUNCH_CHECK();
  ws.reset(mk);
  return HEF_OK;
}

hef_status apply_run(const void *V, void *Q, int pool_type, int64_t n, int K, int Kp,
                     const float *Rinv32, hipStream_t s, bool full = false,
                     bool accumulate = false, bool oct = false, const float *RinvT32 = nullptr,
                     const double *Rinv64 = nullptr) {
  if (n == 0) return HEF_OK;
  TimedScope ts(kStOrthApply, s);
  if (pool_type == kPoolF64) {
    if (!oct || full || accumulate || !Rinv64) {
      set_error("the float64 pool takes the row-octet apply only");
      return HEF_ERR_UNSUPPORTED;
    }
    k_japply_f64<<<cdiv(n, 64) * ((K + 63) / 64), 256, 0, s>>>(
        reinterpret_cast<const double *>(V), reinterpret_cast<double *>(Q), n, K, Kp, Rinv64);
    HEF_LAUNCH_CHECK();
    return HEF_OK;
  }
  if (!full && !accumulate && pool_type == kPoolF32 && RinvT32) {
    if (oct)  // (Kp <= 512: at most 8 tiles per column set)
      k_japply_dma<<<2 * cdiv(n, kDR), kDT, 0, s>>>(reinterpret_cast<const float *>(V),
                                                   reinterpret_cast<float *>(Q), n, K, Kp,
                                                   RinvT32);
    else if ((K & 3) == 0)
      k_japply_tri<false, true><<<cdiv(n, kA2Rows), kA2T, 0, s>>>(
          reinterpret_cast<const float *>(V), reinterpret_cast<float *>(Q), n, K, Kp, RinvT32);
    else
      k_japply_tri<false, false><<<cdiv(n, kA2Rows), kA2T, 0, s>>>(
          reinterpret_cast<const float *>(V), reinterpret_cast<float *>(Q), n, K, Kp, RinvT32);
    HEF_LAUNCH_CHECK();
    return HEF_OK;
  }
  const int ncb = (K + kAN - 1) / kAN;
  if (!oct && pool_type == kPoolF32 && (K & 7) == 0)
    k_japply<true><<<cdiv(n, kAM) * ncb, kAT32, 0, s>>>(V, Q, pool_type, oct, n, K, Kp, Rinv32,
                                                      ncb, full, accumulate);
  else
    k_japply<false><<<cdiv(n, kAM) * ncb, kAT32, 0, s>>>(V, Q, pool_type, oct, n, K, Kp, Rinv32,
                                                       ncb, full, accumulate);
  HEF_LAUNCH_CHECK();
  return HEF_OK;
}

}  // namespace

// The most row chunks the Gram plan takes for any row count up to n: a
// chunk holds at least 128 rows and the plan never exceeds `want` chunks,
// but the count is not monotone in n, so a coarser level (fewer rows) can
// need more partials than the finest.
int64_t gram_max_chunks(int64_t n, int K, bool cross) {
  const GramPlan p = gram_plan(n, K, cross);
  const int64_t want = std::max<int64_t>(1, kGramWG / p.npairs);
  return std::max<int64_t>(1, std::min<int64_t>(want, cdiv(std::max<int64_t>(n, 1), 128)));
}

size_t orth_ws_bytes(int64_t n, int K) {
  const int Kp = (K + 31) / 32 * 32;
  GramPlan p = gram_plan(n, K);
  p.nchunks = int(gram_max_chunks(n, K, false));
  Arena a;
  a.take<double>(int64_t(K) * K);    // G
  a.take<double>(int64_t(K) * K);    // LT
  a.take<double>(int64_t(K) * K);    // trailing matrix of the Cholesky
  a.take<double>(int64_t(Kp) * Kp);  // Rinv
  a.take<float>(int64_t(Kp) * Kp);   // Rinv32
  a.take<float>(int64_t(Kp) * Kp);   // its transpose
  a.take<uint16_t>(int64_t(Kp) * Kp);  // RhT
  a.take<uint16_t>(int64_t(Kp) * Kp);  // RlT
  a.take<int32_t>(K);                // keep
  a.take<double>(size_t(p.nchunks) * p.npairs * 16 * 1024);
  a.take<double>(size_t(p.npairs) * 16 * 1024);
  return a.mark() + 1024;
}

hef_status gram_f32(const float *X, int64_t n, int K, double *G, Arena &ws, hipStream_t s) {
  if (K <= 0 || K > 512) return HEF_ERR_UNSUPPORTED;
  return gram_run(X, nullptr, kPoolF32, n, K, G, ws, s);
}

size_t gram_cross_ws_bytes(int64_t n, int K) {
  GramPlan p = gram_plan(n, K, true);
  p.nchunks = int(gram_max_chunks(n, K, true));
  Arena a;
  a.take<double>(size_t(p.nchunks) * p.npairs * 16 * 1024);
  a.take<double>(size_t(p.npairs) * 16 * 1024);
  return a.mark() + 1024;
}

hef_status gram_cross_f32(const float *X, const float *W, int64_t n, int K, double *G, Arena &ws,
                          hipStream_t s) {
  if (K <= 0 || K > 512) return HEF_ERR_UNSUPPORTED;
  return gram_run(X, W, kPoolF32, n, K, G, ws, s);
}

hef_status gemm_f32(const float *X, int64_t n, int K, const float *W, int Kp, float *out,
                    bool accumulate, hipStream_t s) {
  if (K <= 0 || K > 512) return HEF_ERR_UNSUPPORTED;
  return apply_run(X, out, kPoolF32, n, K, Kp, W, s, true, accumulate);
}

hef_status orthonormalize_pool(void *P, void *out, int pool_type, int64_t n, int K, double tau,
                               int passes, int32_t *keep_out, Arena &ws, hipStream_t s,
                               double *rinv_out, double *rho_out) {
  if (K <= 0) return HEF_OK;
  if (K > 512) {
    set_error("pool width %d exceeds 512", K);
    return HEF_ERR_UNSUPPORTED;
  }
  const int Kp = (K + 31) / 32 * 32;
  const size_t mk = ws.mark();
  double *G = ws.take<double>(int64_t(K) * K);
  double *LT = ws.take<double>(int64_t(K) * K);
  double *A = ws.take<double>(int64_t(K) * K);
  double *Rinv = ws.take<double>(int64_t(Kp) * Kp);
  float *Rinv32 = ws.take<float>(int64_t(Kp) * Kp);
  float *RinvT32 = ws.take<float>(int64_t(Kp) * Kp);
  uint16_t *RhT = ws.take<uint16_t>(int64_t(Kp) * Kp);
  uint16_t *RlT = ws.take<uint16_t>(int64_t(Kp) * Kp);
  int32_t *keep = ws.take<int32_t>(K);
  HEF_WS_CHECK(ws);
  for (int pass = 0; pass < passes; ++pass) {
    // pass 0: P (row-octet layout) -> out; pass 1: out -> P (reused,
    // row-major), copied back to out
    const bool oct = pass == 0;
    const void *src = pass == 0 ? P : out;
    void *dst = pass == 0 ? out : P;
    HEF_TRY(gram_run(src, nullptr, pool_type, n, K, G, ws, s, oct));
    {
      TimedScope ts(kStOrthChol, s);
      const size_t lds_c = size_t(K) * kPS * sizeof(double);
      HEF_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_jtrinv),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_c)));
      HEF_TRY(zero_async(Rinv, sizeof(double) * Kp * Kp, s));
      HEF_TRY(zero_async(Rinv32, sizeof(float) * Kp * Kp, s));
      HEF_TRY(zero_async(RinvT32, sizeof(float) * Kp * Kp, s));
      HEF_HIP(hipMemcpyAsync(A, G, sizeof(double) * K * K, hipMemcpyDeviceToDevice, s));
      HEF_TRY(zero_async(LT, sizeof(double) * K * K, s));
      for (int c0 = 0; c0 < K; c0 += kPW) {
        const int w = K - c0 < kPW ? K - c0 : kPW;
        const int nb = K - c0 - w > 0 ? int(cdiv(K - c0 - w, kCR)) : 1;
        if (w == kPW)
          k_chol_panel<true><<<nb, kCT, 0, s>>>(A, G, K, c0, tau, LT, keep,
                                                pass == 0 ? nullptr : keep,
                                                pass == 0 ? rho_out : nullptr);
        else
          k_chol_panel<false><<<nb, kCT, 0, s>>>(A, G, K, c0, tau, LT, keep,
                                                 pass == 0 ? nullptr : keep,
                                                 pass == 0 ? rho_out : nullptr);
        const int nt = (K - c0 - w + kPW - 1) / kPW;
        if (nt > 0) k_chol_update<<<nt * (nt + 1) / 2, 256, 0, s>>>(A, LT, K, c0, w);
      }
      k_jtrinv<<<(K + kPW - 1) / kPW, 1024, lds_c, s>>>(LT, keep, K, Kp, Rinv, Rinv32, RinvT32);
      HEF_LAUNCH_CHECK();
    }
    if (pool_type == kPoolBF16) {
      {
        TimedScope ts(kStOrthChol, s);
        k_split_rinv<<<cdiv(int64_t(Kp) * Kp, 256), 256, 0, s>>>(Rinv, K, Kp, RhT, RlT);
      }
      TimedScope ts(kStOrthApply, s);
      const int ncb = (K + kAN - 1) / kAN;
      if (n > 0)
        k_japply_bf16<<<cdiv(n, kAM) * ncb, kAT, 0, s>>>(
            reinterpret_cast<const uint16_t *>(src), reinterpret_cast<uint16_t *>(dst), oct, n, K,
            Kp, RhT, RlT, ncb);
      HEF_LAUNCH_CHECK();
    } else {
      HEF_TRY(apply_run(src, dst, pool_type, n, K, Kp, Rinv32, s, false, false, oct, RinvT32,
                        Rinv));
    }
    if (pass == 1)
      HEF_HIP(hipMemcpyAsync(out, P,
                             size_t(n) * K * (pool_type == kPoolBF16 ? 2 : pool_type == kPoolF64 ? 8 : 4),
                             hipMemcpyDeviceToDevice, s));
  }
  if (keep_out) HEF_HIP(hipMemcpyAsync(keep_out, keep, K * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  if (rinv_out)
    HEF_HIP(hipMemcpyAsync(rinv_out, Rinv, sizeof(double) * Kp * Kp, hipMemcpyDeviceToDevice, s));
  ws.reset(mk);
  return HEF_OK;
}

}  // namespace hef

// Block Krylov bases of both expansions (Eq. (12), Alg. 1).
//
// Per expansion, b start vectors and k steps of the block three-term
// recurrence: Y = A V_j, then V_{j+1} is the Gram-Schmidt of Y against
// [V_{j-1}, V_j] and within itself.  The Gram-Schmidt is carried out in the
// Gram metric of M = [V_{j-1} | V_j | Y]: G = M^T M is accumulated in FP32
// register blocks over row chunks and summed across chunks in float64, its
// Cholesky factor R (float64) gives V_{j+1} = M R^-1[:, Y columns].  A
// column whose Gram-Schmidt residual falls below tau times its length is a
// breakdown and becomes zero.  V_0 = X R^-1 starts the sequence and is not
// part of the pool; V_1..V_k are (star: node rows only).
#include <cmath>

#include "krylov.hpp"
#include "prims.hpp"

namespace hef {
namespace {

constexpr int kGramBlocks = 1024;  // workgroups of the Gram partial pass

// Register staging of one Gram slab of M = [v0 | v1 | y] (SLAB rows).
// LDS row stride (floats) of a Gram slab of C = 3B columns.  The products
// read, per half-wave, 6-column blocks of about four consecutive rows; at
// B = 8 a stride of C + 1 = 25 maps some of those (row, block) pairs to one
// bank (measured: a third of the kernel's cycles in bank conflicts), C + 4 =
// 28 spreads them (7 % faster, same values).
template <int B>
__host__ __device__ constexpr int gram_ld() { return B == 8 ? 3 * B + 4 : 3 * B + 1; }

template <int B, int SLAB>
struct GramSlab {
  static constexpr int C = 3 * B;
  static constexpr int LD = gram_ld<B>();
  static constexpr int Q = B >= 4 ? B / 4 : 1;  // float4 per row per array
  static constexpr int TOT = B >= 4 ? SLAB * 3 * Q : SLAB * C;
  static constexpr int NPT = (TOT + 255) / 256;
  static __device__ __forceinline__ void fetch(float4 (&pre)[NPT], int tid, int64_t base,
                                               int64_t r1, const float *v0, const float *v1,
                                               const float *y) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int e = tid + 256 * i;
      float4 t = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (e < TOT) {
        if constexpr (B >= 4) {
          const int a = e / (SLAB * Q);
          const int rem = e % (SLAB * Q);
          const int r = rem / Q, q = rem % Q;
          const int64_t row = base + r;
          const float *src = a == 0 ? v0 : (a == 1 ? v1 : y);
          if (row < r1 && src) t = *reinterpret_cast<const float4 *>(src + row * B + 4 * q);
        } else {
          const int r = e / C, c = e % C;
          const int64_t row = base + r;
          if (row < r1) {
            if (c < B) t.x = v0 ? v0[row * B + c] : 0.0f;
            else if (c < 2 * B) t.x = v1 ? v1[row * B + c - B] : 0.0f;
            else t.x = y[row * B + c - 2 * B];
          }
        }
      }
      pre[i] = t;
    }
  }
  static __device__ __forceinline__ void stash(const float4 (&pre)[NPT], int tid, float *sh) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int e = tid + 256 * i;
      if (e < TOT) {
        if constexpr (B >= 4) {
          const int a = e / (SLAB * Q);
          const int rem = e % (SLAB * Q);
          const int r = rem / Q, q = rem % Q;
          float *d = sh + r * LD + a * B + 4 * q;
          d[0] = pre[i].x; d[1] = pre[i].y; d[2] = pre[i].z; d[3] = pre[i].w;
        } else {
          const int r = e / C, c = e % C;
          sh[r * LD + c] = pre[i].x;
        }
      }
    }
  }
};

// Gram partials of M = [v0 | v1 | y] (rows x C, C = 3B), FP32 register
// blocks: the C x C Gram is cut into S x S blocks, one thread per block on or
// above the diagonal; a workgroup stages 64-row slabs in LDS and its RG row
// groups split each slab's rows.  Per-thread FP32 sums (a few hundred rows)
// are combined in float64 in row-group order; partial[blk][C*C].  The next
// slab is loaded into registers while the current one is consumed.
// Operands of one expansion's Gram.  A launch covers two expansions:
// workgroups [0, nb0) take side 0, the rest side 1.
struct GramSide {
  const float *v0, *v1, *y;
  int64_t rows, rows_per_blk;
  double *partial;
};
struct GramPair {
  GramSide s[2];
  int nb0;
};

template <int B>
__global__ void __launch_bounds__(256)
k_lgram(const GramPair P) {
  const bool second = int(blockIdx.x) >= P.nb0;
  const int bid = int(blockIdx.x) - (second ? P.nb0 : 0);
  const float *__restrict__ v0 = second ? P.s[1].v0 : P.s[0].v0;
  const float *__restrict__ v1 = second ? P.s[1].v1 : P.s[0].v1;
  const float *__restrict__ y = second ? P.s[1].y : P.s[0].y;
  const int64_t rows = second ? P.s[1].rows : P.s[0].rows;
  const int64_t rows_per_blk = second ? P.s[1].rows_per_blk : P.s[0].rows_per_blk;
  double *__restrict__ partial = second ? P.s[1].partial : P.s[0].partial;
  constexpr int C = 3 * B;
  constexpr int S = (C % 6 == 0) ? 6 : 3;
  constexpr int NB = C / S;
  constexpr int NT = NB * (NB + 1) / 2;
  constexpr int RG = 256 / NT;
  constexpr int SLAB = 128;
  constexpr int LD = gram_ld<B>();
  // slab buffer, reused for the row groups' sums at the end
  constexpr int SH = SLAB * LD > RG * NT * S * S ? SLAB * LD : RG * NT * S * S;
  __shared__ float sh[SH];
  const int tid = threadIdx.x;
  const int g = tid / NT;
  const int blk = tid % NT;
  const bool active = g < RG;
  int bi = 0, bj = 0;
  {
    int q = blk;
    for (int a = 0; a < NB; ++a) {
      if (q < NB - a) { bi = a; bj = a + q; break; }
      q -= NB - a;
    }
  }
  float acc[S][S];
#pragma unroll
  for (int a = 0; a < S; ++a)
#pragma unroll
    for (int b = 0; b < S; ++b) acc[a][b] = 0.0f;
  const int64_t r0 = int64_t(bid) * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < rows ? r0 + rows_per_blk : rows;
  // the next slab is fetched into registers while the current one is used
  using SL = GramSlab<B, SLAB>;
  float4 pre[SL::NPT];
  if (r0 < r1) SL::fetch(pre, tid, r0, r1, v0, v1, y);
  for (int64_t base = r0; base < r1; base += SLAB) {
    __syncthreads();
    SL::stash(pre, tid, sh);
    __syncthreads();
    if (base + SLAB < r1) SL::fetch(pre, tid, base + SLAB, r1, v0, v1, y);
    if (active) {
      for (int r = g; r < SLAB; r += RG) {
        float xa[S], xb[S];
#pragma unroll
        for (int a = 0; a < S; ++a) xa[a] = sh[r * LD + bi * S + a];
#pragma unroll
        for (int b = 0; b < S; ++b) xb[b] = sh[r * LD + bj * S + b];
#pragma unroll
        for (int a = 0; a < S; ++a)
#pragma unroll
          for (int b = 0; b < S; ++b) acc[a][b] = fmaf(xa[a], xb[b], acc[a][b]);
      }
    }
  }
  // every row group's sums go to LDS (the slab buffer is free now); each
  // entry is then summed over the row groups in ascending order, in float64
  __syncthreads();
  float *red = sh;
  if (active) {
#pragma unroll
    for (int a = 0; a < S; ++a)
#pragma unroll
      for (int b = 0; b < S; ++b) red[(g * NT + blk) * S * S + a * S + b] = acc[a][b];
  }
  __syncthreads();
  for (int e = tid; e < C * C; e += 256) {
    const int i = e / C, j = e % C;
    const int ri = i / S, rj = j / S;
    double t = 0.0;
    if (ri <= rj) {
      int id = rj - ri;
      for (int a = 0; a < ri; ++a) id += NB - a;
      const int off = id * S * S + (i % S) * S + (j % S);
      for (int gg = 0; gg < RG; ++gg) t += double(red[gg * NT * S * S + off]);
    }
    partial[int64_t(bid) * C * C + e] = t;
  }
}

// G = the column sums of the partials (float64: 32 row lanes of eight
// accumulators each, then a fixed tree), written for the entries in blocks
// on or above the diagonal and mirrored into the blocks below it.
// 256 threads = 8 columns x 32 row lanes.
// Two expansions per launch: workgroups [0, nbh) reduce (in0, nrows0) into
// G0, the rest (in1, nrows1) into G1.
__global__ void __launch_bounds__(256)
k_gram_reduce(const double *__restrict__ in0, int64_t nrows0, double *__restrict__ G0,
              const double *__restrict__ in1, int64_t nrows1, double *__restrict__ G1, int nbh,
              int C, int S) {
  __shared__ double red[32][9];
  const bool second = int(blockIdx.x) >= nbh;
  const double *__restrict__ in = second ? in1 : in0;
  const int64_t nrows = second ? nrows1 : nrows0;
  double *__restrict__ G = second ? G1 : G0;
  const int cl = threadIdx.x & 7, rl = threadIdx.x >> 3;
  const int64_t c = int64_t(int(blockIdx.x) - (second ? nbh : 0)) * 8 + cl;
  const int64_t ncols = int64_t(C) * C;
  const int i = int(c / C), j = int(c % C);
  const bool upper = c < ncols && i / S <= j / S;
  double acc[8] = {};
  if (upper) {
    int64_t r = rl;
    for (; r + 7 * 32 < nrows; r += 8 * 32) {
      double t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = in[(r + 32 * q) * ncols + c];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += t[q];
    }
#pragma unroll
    for (int q = 0; q < 7; ++q)
      if (r + 32 * q < nrows) acc[q] += in[(r + 32 * q) * ncols + c];
  }
  red[rl][cl] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  for (int off = 16; off > 0; off >>= 1) {
    if (rl < off) red[rl][cl] += red[rl + off][cl];
    __syncthreads();
  }
  if (rl == 0 && upper) {
    G[int64_t(i) * C + j] = red[0][cl];
    if (i / S < j / S) G[int64_t(j) * C + i] = red[0][cl];
  }
}

// Cholesky of G with column dropping, then the Y-block columns of R^-1.
// One wave per expansion; lane t holds row t of the C x C Gram (registers),
// so the factorisation needs no barriers: column k's pivot and the entries
// L_jk reach the other lanes by readlane.  Column c is dropped when its reference
// length is 0 or its Schur pivot d_c <= tau^2 * G_cc.  L goes to LDS; lane c
// then forms column c of R^-1 = L^-T by back substitution.
template <int C>
__global__ void __launch_bounds__(64)
k_lsolve(const double *__restrict__ Gall, int B, double tau, double *__restrict__ Tall,
         int32_t *__restrict__ drops, double *__restrict__ Rall) {
  __shared__ double Ls[C * C];
  const double *G = Gall + blockIdx.x * C * C;
  double *T = Tall + blockIdx.x * C * B;
  const int t = threadIdx.x;
  double a[C], l[C];
#pragma unroll
  for (int j = 0; j < C; ++j) {
    a[j] = t < C ? G[t * C + j] : 0.0;
    l[j] = 0.0;
  }
  double gref = 0.0;
#pragma unroll
  for (int j = 0; j < C; ++j)
    if (j == t) gref = a[j];
  uint64_t keep = 0;
#pragma unroll
  for (int k = 0; k < C; ++k) {
    const double d = readlane_f64(a[k], k);
    const double ref = readlane_f64(gref, k);
    if (ref > 0.0 && d > tau * tau * ref) {
      keep |= uint64_t(1) << k;
      const double lkk = sqrt(d);
      const double lk = t == k ? lkk : (t > k ? a[k] / lkk : 0.0);
      l[k] = lk;
      // (also the entries right of lane t's diagonal, which are never read:
      // an unpredicated update; lk is zero on the rows above the pivot)
#pragma unroll
      for (int j = k + 1; j < C; ++j) {
        const double ljk = readlane_f64(lk, j);
        a[j] -= lk * ljk;
      }
    }
  }
  if (t < C) {
#pragma unroll
    for (int j = 0; j < C; ++j) Ls[t * C + j] = l[j];
  }
  __syncthreads();
  // column c of R^-1 (R = L^T): L^T x = e_c, rows c, c-1, ..., 0
  const int c = t;
  const bool kc = c < C && ((keep >> c) & 1);
  double x[C];
#pragma unroll
  for (int i = C - 1; i >= 0; --i) {
    double acc = 0.0;
#pragma unroll
    for (int q = i + 1; q < C; ++q) acc += Ls[q * C + i] * x[q];
    const bool ki = (keep >> i) & 1;
    double xi = 0.0;
    if (kc && ki) xi = i == c ? 1.0 / Ls[i * C + i] : (i < c ? -acc / Ls[i * C + i] : 0.0);
    x[i] = xi;
  }
  if (c >= 2 * B && c < C) {
#pragma unroll
    for (int i = 0; i < C; ++i) T[i * B + (c - 2 * B)] = x[i];
  }
  if (t < B && !((keep >> (2 * B + t)) & 1)) atomicAdd(&drops[blockIdx.x], 1);
  // optionally the whole R^-1 (row-major C x C), zero rows/columns for drops
  if (Rall && c < C) {
    double *Rf = Rall + blockIdx.x * C * C;
#pragma unroll
    for (int i = 0; i < C; ++i) Rf[i * C + c] = x[i];
  }
}

// the solve for C = 3B columns (B in {1, 2, 4, 8, 16})
hef_status lsolve_launch(const double *G, int B, double tau, double *T, int32_t *drops,
                         double *R, hipStream_t s) {
  switch (B) {
    case 1: k_lsolve<3><<<2, 64, 0, s>>>(G, B, tau, T, drops, R); break;
    case 2: k_lsolve<6><<<2, 64, 0, s>>>(G, B, tau, T, drops, R); break;
    case 4: k_lsolve<12><<<2, 64, 0, s>>>(G, B, tau, T, drops, R); break;
    case 8: k_lsolve<24><<<2, 64, 0, s>>>(G, B, tau, T, drops, R); break;
    case 16: k_lsolve<48><<<2, 64, 0, s>>>(G, B, tau, T, drops, R); break;
    default: return HEF_ERR_UNSUPPORTED;
  }
  HEF_LAUNCH_CHECK();
  return HEF_OK;
}

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

// V_next = [v0 | v1 | y] T in float64 arithmetic.  A workgroup stages its
// rows of the three inputs in LDS with coalesced float4 loads, one thread per
// row (two for B = 16) forms the outputs, which leave through LDS as
// coalesced stores.  The first pool_rows rows also go to the pool (row-octet
// layout, float32, bfloat16 or, for the float64 debug basis, float64) at
// column col0.
template <int CH>
__device__ __forceinline__ void ld(const float *p, float (&v)[CH]) {
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

// Operands of one expansion's apply.  A launch covers two expansions:
// logical workgroups [0, nb0) take side 0, the rest side 1.
struct ApplySide {
  const float *v0, *v1, *y;
  const double *T;
  float *vn;
  int64_t rows;
  int col0;
};
struct ApplyPair {
  ApplySide s[2];
  int64_t nb0;
};

template <int B>
__global__ void __launch_bounds__(256)
k_lapply(const ApplyPair P, void *__restrict__ pool, int pool_type, int64_t pool_rows, int K) {
  constexpr int C = 3 * B;
  constexpr int RB = B <= 8 ? 256 : 128;  // rows per workgroup
  constexpr int NSPL = 256 / RB;          // threads per row
  constexpr int OPT = B / NSPL;           // outputs per thread
  constexpr int LDR = B + 1;              // LDS row stride (odd: no bank conflicts)
  __shared__ double Ts[C * B];
  __shared__ float sm[3][RB * LDR];
  const int tid = threadIdx.x;
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const bool second = lb >= P.nb0;
  const float *__restrict__ v0 = second ? P.s[1].v0 : P.s[0].v0;
  const float *__restrict__ v1 = second ? P.s[1].v1 : P.s[0].v1;
  const float *__restrict__ y = second ? P.s[1].y : P.s[0].y;
  const double *__restrict__ Tm = second ? P.s[1].T : P.s[0].T;
  float *__restrict__ vn = second ? P.s[1].vn : P.s[0].vn;
  const int64_t rows = second ? P.s[1].rows : P.s[0].rows;
  const int col0 = second ? P.s[1].col0 : P.s[0].col0;
  const int64_t row0 = (lb - (second ? P.nb0 : 0)) * RB;
  const int nrow = int(rows - row0 < RB ? rows - row0 : RB);
  const float *src[3] = {v0, v1, y};
  // coalesced loads of the workgroup's rows into LDS, all of a thread's
  // loads issued before the first is stored
  if constexpr (B >= 4) {
    constexpr int NL = (RB * B / 4 + 255) / 256;  // float4 per thread and array
    float4 t[3][NL];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        const int i = tid + 256 * u;
        t[a][u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (src[a] != nullptr && i < nrow * B / 4)
          t[a][u] = reinterpret_cast<const float4 *>(src[a] + row0 * B)[i];
      }
    for (int e = tid; e < C * B; e += 256) Ts[e] = Tm[e];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        const int i = tid + 256 * u;
        if (src[a] != nullptr && i < nrow * B / 4) {
          float *d = &sm[a][(4 * i / B) * LDR + (4 * i) % B];
          d[0] = t[a][u].x; d[1] = t[a][u].y; d[2] = t[a][u].z; d[3] = t[a][u].w;
        }
      }
  } else {
    for (int e = tid; e < C * B; e += 256) Ts[e] = Tm[e];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (src[a] == nullptr) continue;
      const float *base = src[a] + row0 * B;
      for (int i = tid; i < nrow * B; i += 256) sm[a][(i / B) * LDR + i % B] = base[i];
    }
  }
  __syncthreads();
  const int r = tid / NSPL, h = tid % NSPL;
  float of[OPT];
  {
    double out[OPT];
#pragma unroll
    for (int c = 0; c < OPT; ++c) out[c] = 0.0;
    if (r < nrow) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (src[a] == nullptr) continue;
#pragma unroll
        for (int u = 0; u < B; ++u) {
          const double md = double(sm[a][r * LDR + u]);
          const double *trow = Ts + (a * B + u) * B + h * OPT;
#pragma unroll
          for (int c = 0; c < OPT; ++c) out[c] = fma(md, trow[c], out[c]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < OPT; ++c) of[c] = float(out[c]);
  }
  __syncthreads();
  if (r < nrow) {
#pragma unroll
    for (int c = 0; c < OPT; ++c) sm[0][r * LDR + h * OPT + c] = of[c];
  }
  __syncthreads();
  // coalesced stores of the new rows, then the pool columns
  float *vbase = vn + row0 * B;
  if constexpr (B >= 4) {
    for (int i = tid; i < nrow * B / 4; i += 256) {
      const float *d = &sm[0][(4 * i / B) * LDR + (4 * i) % B];
      reinterpret_cast<float4 *>(vbase)[i] = make_float4(d[0], d[1], d[2], d[3]);
    }
  } else {
    for (int i = tid; i < nrow * B; i += 256) vbase[i] = sm[0][(i / B) * LDR + i % B];
  }
  if (pool) {
    // pool rows in the row-octet layout: per (octet, column) 8 consecutive
    // values; rows at or past pool_rows are zero (row0 is a multiple of 8)
    const int noct = (nrow + 7) / 8;
    for (int i = tid; i < noct * B; i += 256) {
      const int o = i / B, c = i % B;
      const int64_t gr0 = row0 + 8 * o;
      if (gr0 >= pool_rows) continue;
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        v[u] = (8 * o + u < nrow && gr0 + u < pool_rows) ? sm[0][(8 * o + u) * LDR + c] : 0.0f;
      const int64_t off = ((gr0 >> 3) * K + col0 + c) * 8;
      if (pool_type == kPoolF32) {
        float4 *pp = reinterpret_cast<float4 *>(reinterpret_cast<float *>(pool) + off);
        pp[0] = make_float4(v[0], v[1], v[2], v[3]);
        pp[1] = make_float4(v[4], v[5], v[6], v[7]);
      } else if (pool_type == kPoolF64) {
        double2 *pp = reinterpret_cast<double2 *>(reinterpret_cast<double *>(pool) + off);
#pragma unroll
        for (int q = 0; q < 4; ++q) pp[q] = make_double2(double(v[2 * q]), double(v[2 * q + 1]));
      } else {
        uint32_t wv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          wv[q] = uint32_t(f2bf(v[2 * q])) | (uint32_t(f2bf(v[2 * q + 1])) << 16);
        *reinterpret_cast<uint4 *>(reinterpret_cast<uint16_t *>(pool) + off) =
            make_uint4(wv[0], wv[1], wv[2], wv[3]);
      }
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

// Sides with zero rows launch nothing.
template <int B>
hef_status apply_t(const ApplySide &a, const ApplySide &b, void *pool, int pool_type,
                   int64_t pool_rows, int K, hipStream_t s) {
  constexpr int RB = B <= 8 ? 256 : 128;
  ApplyPair P;
  P.s[0] = a;
  P.s[1] = b;
  P.nb0 = cdiv(a.rows, RB);
  const int64_t nblk = P.nb0 + cdiv(b.rows, RB);
  if (nblk == 0) return HEF_OK;
  TimedScope ts(kStLanczosApply, s);
  k_lapply<B><<<nblk, 256, 0, s>>>(P, pool, pool_type, pool_rows, K);
  HEF_LAUNCH_CHECK();
  return HEF_OK;
}

hef_status lapply2(int B, const ApplySide &a, const ApplySide &b, void *pool, int pool_type,
                   int64_t pool_rows, int K, hipStream_t s) {
  switch (B) {
    case 1: return apply_t<1>(a, b, pool, pool_type, pool_rows, K, s);
    case 2: return apply_t<2>(a, b, pool, pool_type, pool_rows, K, s);
    case 4: return apply_t<4>(a, b, pool, pool_type, pool_rows, K, s);
    case 8: return apply_t<8>(a, b, pool, pool_type, pool_rows, K, s);
    case 16: return apply_t<16>(a, b, pool, pool_type, pool_rows, K, s);
    default: return HEF_ERR_UNSUPPORTED;
  }
}

hef_status lapply(int B, const float *v0, const float *v1, const float *y, const double *T,
                  float *vn, int64_t rows, void *pool, int pool_type, int64_t pool_rows, int K,
                  int col0, hipStream_t s) {
  const ApplySide a{v0, v1, y, T, vn, rows, col0};
  const ApplySide none{nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0};
  return lapply2(B, a, none, pool, pool_type, pool_rows, K, s);
}

// The Grams of up to two expansions (a side with y == nullptr is skipped),
// each over its own rows, in one Gram launch and one reduce launch.
hef_status lgram2(int B, const float *v0a, const float *v1a, const float *ya, int64_t rowsa,
                  double *partiala, double *Ga, const float *v0b, const float *v1b,
                  const float *yb, int64_t rowsb, double *partialb, double *Gb, hipStream_t s) {
  const int C = 3 * B;
  const int S = (C % 6 == 0) ? 6 : 3;
  GramPair P;
  int nb[2] = {0, 0};
  const float *v0[2] = {v0a, v0b}, *v1[2] = {v1a, v1b}, *y[2] = {ya, yb};
  const int64_t rows[2] = {rowsa, rowsb};
  double *part[2] = {partiala, partialb};
  for (int i = 0; i < 2; ++i) {
    const int64_t per = std::max<int64_t>(64, cdiv(cdiv(rows[i], kGramBlocks), 64) * 64);
    nb[i] = y[i] ? int(std::max<int64_t>(1, cdiv(rows[i], per))) : 0;
    P.s[i] = GramSide{v0[i], v1[i], y[i], rows[i], per, part[i]};
  }
  P.nb0 = nb[0];
  const int nblk = nb[0] + nb[1];
  if (nblk == 0) return HEF_OK;
  {
  TimedScope ts(kStLanczosGram, s);
  switch (B) {
    case 1: k_lgram<1><<<nblk, 256, 0, s>>>(P); break;
    case 2: k_lgram<2><<<nblk, 256, 0, s>>>(P); break;
    case 4: k_lgram<4><<<nblk, 256, 0, s>>>(P); break;
    case 8: k_lgram<8><<<nblk, 256, 0, s>>>(P); break;
    case 16: k_lgram<16><<<nblk, 256, 0, s>>>(P); break;
    default: return HEF_ERR_UNSUPPORTED;
  }
  HEF_LAUNCH_CHECK();
  }
  TimedScope ts(kStLanczosReduce, s);
  const int nbh = int(cdiv(int64_t(C) * C, 8));
  if (nb[0] > 0 && nb[1] > 0)
    k_gram_reduce<<<2 * nbh, 256, 0, s>>>(partiala, nb[0], Ga, partialb, nb[1], Gb, nbh, C, S);
  else if (nb[0] > 0)
    k_gram_reduce<<<nbh, 256, 0, s>>>(partiala, nb[0], Ga, nullptr, 0, nullptr, nbh, C, S);
  else
    k_gram_reduce<<<nbh, 256, 0, s>>>(partialb, nb[1], Gb, nullptr, 0, nullptr, nbh, C, S);
  HEF_LAUNCH_CHECK();
  return HEF_OK;
}

hef_status lgram(const float *v0, const float *v1, const float *y, int64_t rows, int B,
                 double *partial, double *G, hipStream_t s) {
  return lgram2(B, v0, v1, y, rows, partial, G, nullptr, nullptr, nullptr, 0, nullptr, nullptr, s);
}

}  // namespace

size_t lanczos_partial_elems(int B) { return size_t(kGramBlocks) * 9 * B * B; }

hef_status lanczos_gram(const float *v0, const float *v1, const float *y, int64_t rows, int B,
                        double *partial, double *G, hipStream_t s) {
  return lgram(v0, v1, y, rows, B, partial, G, s);
}

hef_status lanczos_solve(const double *G2, int B, double tau, double *T2, int32_t *drops,
                         double *R2, hipStream_t s) {
  TimedScope ts(kStLanczosSolve, s);
  return lsolve_launch(G2, B, tau, T2, drops, R2, s);
}

hef_status lanczos_apply(int B, const float *v0, const float *v1, const float *y, const double *T,
                         float *vn, int64_t rows, void *pool, int pool_type, int64_t pool_rows,
                         int K, int col0, hipStream_t s) {
  return lapply(B, v0, v1, y, T, vn, rows, pool, pool_type, pool_rows, K, col0, s);
}

hef_status lanczos_apply_pair(int B, const float *v0a, const float *v1a, const float *ya,
                              const double *Ta, float *vna, int64_t rowsa, const float *v0b,
                              const float *v1b, const float *yb, const double *Tb, float *vnb,
                              int64_t rowsb, int K, hipStream_t s) {
  const ApplySide a{v0a, v1a, ya, Ta, vna, rowsa, 0};
  const ApplySide b{v0b, v1b, yb, Tb, vnb, rowsb, 0};
  return lapply2(B, a, b, nullptr, 0, 0, K, s);
}

size_t krylov_ws_bytes(int64_t n, int64_t m, int B) {
  Arena a;
  for (int i = 0; i < 4; ++i) a.take<float>((n + m) * B);
  for (int i = 0; i < 4; ++i) a.take<float>(n * B);
  a.take<float>(spmm_scratch_floats(n, m, B));
  a.take<double>(size_t(2) * kGramBlocks * 9 * B * B);
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
  TimedScope ts(kStStart, s);
  k_start<<<cdiv(total, 256), 256, 0, s>>>(h, total, out);
  HEF_LAUNCH_CHECK();
  return HEF_OK;
}

hef_status krylov_pool(const Level &L, const Structure &st, int B, int k, double tau,
                       const float *start_star, const float *start_clique, bool use_star,
                       bool use_clique, KrylovOut &out, Arena &ws, hipStream_t s,
                       const KrylovTape *tape) {
  const int64_t n = L.n, m = L.m;
  const int64_t Ns = n + m;
  const size_t mk = ws.mark();
  float *sb[4], *cb[4];
  for (int i = 0; i < 4; ++i) sb[i] = ws.take<float>(Ns * B);
  for (int i = 0; i < 4; ++i) cb[i] = ws.take<float>(n * B);
  float *tb = ws.take<float>(spmm_scratch_floats(n, m, B));
  double *partial = ws.take<double>(size_t(2) * kGramBlocks * 9 * B * B);
  double *G = ws.take<double>(2 * 48 * 48);
  double *Tm = ws.take<double>(2 * 48 * 16);
  int32_t *drops = ws.take<int32_t>(2);
  HEF_WS_CHECK(ws);
  const int C = 3 * B;
  double *Gs = G, *Gc = G + C * C;
  double *ps = partial, *pc = partial + size_t(kGramBlocks) * 9 * B * B;
  HEF_TRY(zero_async(drops, 2 * sizeof(int32_t), s));
  HEF_TRY(zero_async(G, 2 * 48 * 48 * sizeof(double), s));
  // per-step T (and R^-1 for the adjoint)
  auto t_of = [&](int j) { return tape ? tape->T + size_t(j) * 2 * C * B : Tm; };
  auto r_of = [&](int j) { return tape ? tape->Rinv + size_t(j) * 2 * C * C : nullptr; };
  const int seg = tape ? (tape->seg > 0 && tape->seg < k ? tape->seg : k) : 0;
  // checkpoint slot j/seg <- (V_{j-1}, V_j) at the start of each segment
  auto checkpoint = [&](int j, const float *vs_prev, const float *vs, const float *vc_prev,
                        const float *vc) -> hef_status {
    if (!tape || j % seg != 0 || j >= k) return HEF_OK;
    const size_t slot = size_t(j / seg);
    if (use_star) {
      float *d = tape->ck_star + slot * 2 * Ns * B;
      if (vs_prev) HEF_HIP(hipMemcpyAsync(d, vs_prev, Ns * B * sizeof(float), hipMemcpyDeviceToDevice, s));
      else HEF_TRY(zero_async(d, Ns * B * sizeof(float), s));
      HEF_HIP(hipMemcpyAsync(d + Ns * B, vs, Ns * B * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    if (use_clique) {
      float *d = tape->ck_clique + slot * 2 * n * B;
      if (vc_prev) HEF_HIP(hipMemcpyAsync(d, vc_prev, n * B * sizeof(float), hipMemcpyDeviceToDevice, s));
      else HEF_TRY(zero_async(d, n * B * sizeof(float), s));
      HEF_HIP(hipMemcpyAsync(d + n * B, vc, n * B * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    return HEF_OK;
  };

  // the rolling buffers: prev, cur, y, next (as pointers: with a full tape
  // Y_j and V_j live in the tape's step buffers instead)
  const bool full = tape && seg == k && tape->y_s;
  const size_t scr = spmm_scratch_floats(n, m, B);
  const int K = out.K;
  const int64_t bk = int64_t(B) * k;
  // V_0 = X R^-1 (no pool write)
  if (use_star)
    HEF_HIP(hipMemcpyAsync(sb[2], start_star, Ns * B * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (use_clique)
    HEF_HIP(hipMemcpyAsync(cb[2], start_clique, n * B * sizeof(float), hipMemcpyDeviceToDevice, s));
  HEF_TRY(lgram2(B, nullptr, nullptr, use_star ? sb[2] : nullptr, Ns, ps, Gs, nullptr, nullptr,
                 use_clique ? cb[2] : nullptr, n, pc, Gc, s));
  {
    TimedScope ts(kStLanczosSolve, s);
    HEF_TRY(lsolve_launch(G, B, tau, t_of(0), drops, r_of(0), s));
  }
  {
    const ApplySide as{nullptr, nullptr, sb[2], t_of(0), sb[3], use_star ? Ns : 0, 0};
    const ApplySide ac{nullptr, nullptr, cb[2], t_of(0) + C * B, cb[3], use_clique ? n : 0, 0};
    HEF_TRY(lapply2(B, as, ac, nullptr, 0, 0, K, s));
  }
  HEF_TRY(checkpoint(0, nullptr, sb[3], nullptr, cb[3]));
  float *sp = nullptr, *sc = sb[3], *cp = nullptr, *cc = cb[3];  // prev (absent), cur
  // the rolling buffer that is neither prev, cur nor y (non-full runs)
  auto spare = [&](float *const *buf, const float *p, const float *c, const float *y) {
    for (int i = 0; i < 4; ++i)
      if (buf[i] != p && buf[i] != c && buf[i] != y) return buf[i];
    return buf[0];
  };
  for (int j = 1; j <= k; ++j) {
    float *sy = full ? tape->y_s + size_t(j - 1) * Ns * B : sb[2];
    float *cy = full ? tape->y_c + size_t(j - 1) * n * B : cb[2];
    float *tj = full ? tape->t + size_t(j - 1) * scr : tb;
    HEF_TRY(spmm_apply(L, st, B, use_star ? sc : nullptr, use_star ? sy : nullptr,
                       use_clique ? cc : nullptr, use_clique ? cy : nullptr, tj, s));
    HEF_TRY(lgram2(B, sp, sc, use_star ? sy : nullptr, Ns, ps, Gs, cp, cc,
                   use_clique ? cy : nullptr, n, pc, Gc, s));
    double *Tj = t_of(j);
    {
      TimedScope ts(kStLanczosSolve, s);
      HEF_TRY(lsolve_launch(G, B, tau, Tj, drops, r_of(j), s));
    }
    // V_j: a tape step buffer (j < k, full tape) or the spare rolling buffer
    float *sn = (full && j < k) ? tape->v_s + size_t(j - 1) * Ns * B
                                : spare(sb, sp, sc, full ? sb[2] : sy);
    float *cn = (full && j < k) ? tape->v_c + size_t(j - 1) * n * B
                                : spare(cb, cp, cc, full ? cb[2] : cy);
    const int64_t col_s = (j - 1) * int64_t(B);
    const int64_t col_c = (use_star ? bk : 0) + (j - 1) * int64_t(B);
    {
      const ApplySide as{sp, sc, sy, Tj, sn, use_star ? Ns : 0, int(col_s)};
      const ApplySide ac{cp, cc, cy, Tj + C * B, cn, use_clique ? n : 0, int(col_c)};
      HEF_TRY(lapply2(B, as, ac, out.pool, out.pool_type, n, K, s));
    }
    HEF_TRY(checkpoint(j, sc, sn, cc, cn));
    sp = sc;
    sc = sn;
    cp = cc;
    cc = cn;
  }
  ws.reset(mk);
  return HEF_OK;
}

}  // namespace hef

// Adjoint of Alg. 1 with respect to the hyperedge weights: for
// L = sum_e c_e R_e (c = dL/dR given), dL/dw_e.
//
// The forward is recomputed exactly as hef_resistance computes it (same
// kernels, so the same floating-point function), keeping a tape: per
// Lanczos step the R^-1 of its Cholesky QR, and the two blocks at the start
// of every checkpoint segment.  The reverse sweep then runs
//   1. the ratios (Eqs. (9), (13), (14)): the largest ratio and the largest /
//      smallest pin are taken at fixed positions (lowest column, lowest CSR
//      position on ties), so R_e is smooth in chi on the branch they select;
//      Q_H also depends on w directly;
//   2. the joint Cholesky QR of the pool (Alg. 1): the adjoint of a
//      thin QR with positive diagonal, Vbar = (Qbar + Q sym(-Qbar^T Q)) R^-T,
//      sym() copying the lower triangle onto the upper;
//   3. every block-Lanczos step, a Cholesky QR of M = [V_{j-2} | V_{j-1} | Y]
//      with Y = A V_{j-1}, backwards: Mbar = M Z + Vbar_j T^T with
//      Z = R^-1 sym(S) R^-T, S holding -Vbar_j^T M R^-1 in its last b rows;
//      Mbar splits into Vbar_{j-2}, Vbar_{j-1} and Ybar, and
//      Vbar_{j-1} += A Ybar (A is symmetric);
//   4. the weights enter A only through alpha_e = sqrt(w_e)/|e|,
//      beta_e = w_e/(|e|(|e|-1)) and the node scales s_p = d_b(p)^-1/2,
//      d_b(p) = sum_{e ∋ p} w_e/|e| (Section III-A).  With u = Ybar and
//      x = V_{j-1}, d/dw_e of u^T A x is
//        star   (u_E.Y_E + x_E.(A u)_E)[e] / (2 w_e)
//               - 1/(2|e|) sum_{p in e} s_p^2 (x_V.(A u)_V + u_V.Y_V)[p]
//        clique (Tbar_e . T_e) / (w_e beta_e)
//               - beta_e/w_e sum_{p in e} s_p^2 (u.x)[p]
//               - 1/(2|e|) sum_{p in e} s_p^2 (u.Y + x.(A u))[p]
//      where T_e = beta_e sum_{p in e} s_p x_p and Tbar_e the same of u.
//      Node quantities are summed over the steps first and gathered per
//      hyperedge once at the end.
// All sums run in a fixed order (no floating-point atomics): the result is
// bitwise reproducible.
#include <cfloat>
#include <climits>
#include <cmath>

#include "cluster.hpp"
#include "krylov.hpp"
#include "orth.hpp"
#include "prims.hpp"
#include "score.hpp"
#include "structure.hpp"

namespace hef {
namespace {

constexpr int kThreads = 256;
constexpr int kEdgesPerBlk = 64;
constexpr int kXBlocks = 2048;  // workgroups of the step cross products

// ------------------------------------------------------------ pool loads
template <int CPL>
__device__ __forceinline__ void load_row(const float *__restrict__ X, int64_t row, int K, int c0,
                                         float (&v)[CPL]) {
  const float *p = X + row * K + c0;
  if ((K & 3) == 0 && c0 + CPL <= K) {
#pragma unroll
    for (int q = 0; q < CPL; q += 4) {
      const float4 t = *reinterpret_cast<const float4 *>(p + q);
      v[q] = t.x; v[q + 1] = t.y; v[q + 2] = t.z; v[q + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int q = 0; q < CPL; ++q) v[q] = (c0 + q < K) ? p[q] : 0.0f;
  }
}

template <int CPL>
__device__ __forceinline__ void load_row_i(const int32_t *__restrict__ X, int64_t row, int K,
                                           int c0, int32_t (&v)[CPL]) {
  const int32_t *p = X + row * K + c0;
  if ((K & 3) == 0 && c0 + CPL <= K) {
#pragma unroll
    for (int q = 0; q < CPL; q += 4) {
      const int4 t = *reinterpret_cast<const int4 *>(p + q);
      v[q] = t.x; v[q + 1] = t.y; v[q + 2] = t.z; v[q + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int q = 0; q < CPL; ++q) v[q] = (c0 + q < K) ? p[q] : -1;
  }
}

// ------------------------------------------------------------ 1. ratios
// Pass A: per hyperedge the spreads s_e^(i), the ratio s * (1/Q_H) as the
// forward forms it, the first column i* of the maximum; per workgroup the
// column sums of c_e s_e^(i*) / Q_H(i*)^2 (fixed order).
template <int CPL>
__global__ void __launch_bounds__(kThreads)
k_sadj_a(const float *__restrict__ sfwd, int K, int LPR, int64_t m, const double *__restrict__ qh,
         const float *__restrict__ dR, int32_t *__restrict__ istar, double *__restrict__ partial) {
  __shared__ double comb[512];
  const int tid = threadIdx.x;
  const int ngrp = kThreads / LPR;
  const int grp = tid / LPR;
  const int c0 = (tid % LPR) * CPL;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t e0 = blk * kEdgesPerBlk;
  const int64_t e1 = e0 + kEdgesPerBlk < m ? e0 + kEdgesPerBlk : m;
  double inv[CPL], acc[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const double qv = (c0 + q < K) ? qh[c0 + q] : 0.0;
    inv[q] = qv > 0.0 ? 1.0 / qv : 0.0;
    acc[q] = 0.0;
  }
  for (int64_t e = e0 + grp; e < e1; e += ngrp) {
    // the numerators the forward ratios were formed from
    double s[CPL];
    {
      float v[CPL];
      load_row<CPL>(sfwd, e, K, c0, v);
#pragma unroll
      for (int q = 0; q < CPL; ++q) s[q] = double(v[q]);
    }
    double best = 0.0;
    int bi = INT_MAX;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const double r = s[q] * inv[q];
      if (c0 + q < K && r > best) { best = r; bi = c0 + q; }
    }
    for (int off = LPR / 2; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, LPR);
      const int oi = __shfl_xor(bi, off, LPR);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (tid % LPR == 0) istar[e] = best > 0.0 ? bi : -1;
    if (best > 0.0) {
      const double ce = double(dR[e]);
#pragma unroll
      for (int q = 0; q < CPL; ++q)
        if (c0 + q == bi) acc[q] += ce * s[q] * inv[q] * inv[q];
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

// Pass B: with qbar_i = -qsum_i (dL/dQ_H(i)), per (e, i) the spread's
// adjoint sbar = [i = i*] c_e / Q_H(i) + w_e qbar_i, the positions of the
// largest / smallest pin (first in CSR order) and dbar = 2 (max - min) sbar;
// per hyperedge the direct term sum_i qbar_i s_e^(i).
template <int CPL>
__global__ void __launch_bounds__(kThreads)
k_sadj_b(const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins,
         const float *__restrict__ chi, int K, int LPR, int64_t m, const double *__restrict__ qh,
         const float *__restrict__ dR, const float *__restrict__ w,
         const int32_t *__restrict__ istar, const double *__restrict__ qsum,
         int32_t *__restrict__ slot_a, int32_t *__restrict__ slot_b, float *__restrict__ dbar,
         double *__restrict__ wdirect) {
  const int tid = threadIdx.x;
  const int ngrp = kThreads / LPR;
  const int grp = tid / LPR;
  const int c0 = (tid % LPR) * CPL;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t e0 = blk * kEdgesPerBlk;
  const int64_t e1 = e0 + kEdgesPerBlk < m ? e0 + kEdgesPerBlk : m;
  double inv[CPL], qb[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const double qv = (c0 + q < K) ? qh[c0 + q] : 0.0;
    inv[q] = qv > 0.0 ? 1.0 / qv : 0.0;
    qb[q] = (c0 + q < K) ? -qsum[c0 + q] : 0.0;
  }
  for (int64_t e = e0 + grp; e < e1; e += ngrp) {
    const int32_t a = eptr[e], b = eptr[e + 1];
    float mx[CPL], mn[CPL];
    int32_t ja[CPL], jb[CPL];
    {
      float v[CPL];
      load_row<CPL>(chi, pins[a], K, c0, v);
#pragma unroll
      for (int q = 0; q < CPL; ++q) { mx[q] = v[q]; mn[q] = v[q]; ja[q] = a; jb[q] = a; }
    }
    // pins in chunks of 4 in CSR order (ids first, then rows); a chunk past
    // the end repeats the last pin, which never beats it strictly
    for (int32_t j0 = a + 1; j0 < b; j0 += 4) {
      int32_t pp[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) pp[u] = pins[j0 + u < b ? j0 + u : b - 1];
      float v[4][CPL];
#pragma unroll
      for (int u = 0; u < 4; ++u) load_row<CPL>(chi, pp[u], K, c0, v[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int32_t j = j0 + u < b ? j0 + u : b - 1;
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
          if (v[u][q] > mx[q]) { mx[q] = v[u][q]; ja[q] = j; }
          if (v[u][q] < mn[q]) { mn[q] = v[u][q]; jb[q] = j; }
        }
      }
    }
    const int is = istar[e];
    const double ce = double(dR[e]);
    const double we = w ? double(w[e]) : 1.0;
    double wd = 0.0;
    if (c0 < K) {
      const int64_t off = e * K + c0;
#pragma unroll
      for (int q = 0; q < CPL; ++q) {
        if (c0 + q < K) {
          const double d = double(mx[q]) - double(mn[q]);
          const double sbar = we * qb[q] + (c0 + q == is ? ce * inv[q] : 0.0);
          wd += qb[q] * (d * d);
          slot_a[off + q] = ja[q];
          slot_b[off + q] = jb[q];
          dbar[off + q] = float(2.0 * d * sbar);
        }
      }
    }
    for (int o = LPR / 2; o > 0; o >>= 1) wd += __shfl_xor(wd, o, LPR);
    if (tid % LPR == 0) wdirect[e] = wd;
  }
}

// Pass C: chibar[p, i] = sum over the hyperedges e ∋ p (ascending) of
// +dbar(e, i) where p is e's largest pin and -dbar(e, i) where it is the
// smallest; cslot[t] is the CSR position of the t-th CSC entry.
template <int CPL>
__global__ void __launch_bounds__(kThreads)
k_sadj_c(const int32_t *__restrict__ vptr, const int32_t *__restrict__ eids,
         const int32_t *__restrict__ cslot, const int32_t *__restrict__ slot_a,
         const int32_t *__restrict__ slot_b, const float *__restrict__ dbar, int K, int LPR,
         int64_t n, float *__restrict__ chibar) {
  const int tid = threadIdx.x;
  const int ngrp = kThreads / LPR;
  const int64_t p = int64_t(xcd_block(blockIdx.x, gridDim.x)) * ngrp + tid / LPR;
  const int c0 = (tid % LPR) * CPL;
  if (p >= n || c0 >= K) return;
  double acc[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q] = 0.0;
  for (int32_t t = vptr[p]; t < vptr[p + 1]; ++t) {
    const int64_t e = eids[t];
    const int32_t pos = cslot[t];
    int32_t sa[CPL], sb[CPL];
    float d[CPL];
    load_row_i<CPL>(slot_a, e, K, c0, sa);
    load_row_i<CPL>(slot_b, e, K, c0, sb);
    load_row<CPL>(dbar, e, K, c0, d);
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      if (sa[q] == pos) acc[q] += double(d[q]);
      if (sb[q] == pos) acc[q] -= double(d[q]);
    }
  }
  float *dst = chibar + p * K + c0;
#pragma unroll
  for (int q = 0; q < CPL; ++q)
    if (c0 + q < K) dst[q] = float(acc[q]);
}

__global__ void k_pos_pairs(const int32_t *__restrict__ pins, uint32_t *__restrict__ keys,
                            uint32_t *__restrict__ vals, int64_t nnz) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j < nnz) { keys[j] = uint32_t(pins[j]); vals[j] = uint32_t(j); }
}

// ------------------------------------------------------------ 2. joint QR
// W1 = R^-T and W2 = sym(-Mq) R^-T (float32, Kp x Kp, zero outside K x K),
// Mq = chibar^T chi, sym(X)[i][l] = X[max(i,l)][min(i,l)].
__global__ void k_qradj_w(const double *__restrict__ Rinv, const double *__restrict__ Mq, int K,
                          int Kp, float *__restrict__ W1, float *__restrict__ W2) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(Kp) * Kp) return;
  const int i = int(idx / Kp), j = int(idx % Kp);
  if (i >= K || j >= K) { W1[idx] = 0.0f; W2[idx] = 0.0f; return; }
  W1[idx] = float(Rinv[int64_t(j) * Kp + i]);
  double acc = 0.0;
  const double *rj = Rinv + int64_t(j) * Kp;
  for (int l = j; l < K; ++l) {
    const double z = i >= l ? Mq[int64_t(i) * K + l] : Mq[int64_t(l) * K + i];
    acc -= z * rj[l];
  }
  W2[idx] = float(acc);
}

// ------------------------------------------------------------ 3. Lanczos steps
// X3 = [v0 | v1 | y]^T vbar (3B x B, float64): per workgroup a row range in
// 64-row LDS slabs, one output entry (or a few) per thread, FP32 per slab,
// float64 across slabs; partial[blk][3B*B].
// vbar = abar + pbar[:, col .. col + B) on the first pool_rows rows, formed
// while the cross products read it; abar is cleared for the next step.
struct VbarIn {
  float *abar;
  const float *pbar;
  int K, col;
  int64_t pool_rows;
  float *vbar;
};

// One expansion's operands of the step cross products; a launch covers two.
struct XgramSide {
  const float *v0, *v1, *y;
  VbarIn vi;
  int64_t rows, rows_per_blk;
  double *partial;
};
struct XgramPair {
  XgramSide s[2];
  int nb0;
};

// One SL-row slab of [v0 | v1 | y | vbar] into registers (element g of the
// slab: row g / (C + B), column g % (C + B)); zeros past r1.
template <int B, int SL, int PF>
__device__ __forceinline__ void xgram_fetch(float (&pre)[PF], int tid, int64_t rs, int64_t r1,
                                            const float *v0, const float *v1, const float *y,
                                            const VbarIn &vi) {
  constexpr int C = 3 * B;
#pragma unroll
  for (int i = 0; i < PF; ++i) {
    const int g = tid + i * kThreads;
    const int r = g / (C + B), c = g % (C + B);
    const int64_t row = rs + r;
    float v = 0.0f;
    if (g < SL * (C + B) && row < r1) {
      if (c < C) {
        const float *sp = c < B ? v0 : (c < 2 * B ? v1 : y);
        v = sp ? sp[row * B + (c % B)] : 0.0f;
      } else {
        // vbar = abar + the pool adjoint's columns, written out (and abar
        // cleared) here: every row is fetched exactly once
        const int64_t gi = row * B + (c - C);
        v = vi.abar[gi];
        if (row < vi.pool_rows) v += vi.pbar[row * vi.K + vi.col + (c - C)];
        vi.vbar[gi] = v;
        vi.abar[gi] = 0.0f;
      }
    }
    pre[i] = v;
  }
}

template <int B>
__global__ void __launch_bounds__(kThreads)
k_xgram(const XgramPair P) {
  // workgroups [0, nb0) take side 0, the rest side 1
  const bool second = int(blockIdx.x) >= P.nb0;
  const XgramSide &S = second ? P.s[1] : P.s[0];
  const float *__restrict__ v0 = S.v0;
  const float *__restrict__ v1 = S.v1;
  const float *__restrict__ y = S.y;
  const VbarIn vi = S.vi;
  const int64_t rows = S.rows, rows_per_blk = S.rows_per_blk;
  double *__restrict__ partial = S.partial;
  const int bid = int(blockIdx.x) - (second ? P.nb0 : 0);
  constexpr int C = 3 * B;
  constexpr int NE = C * B;
  constexpr int EPT = (NE + kThreads - 1) / kThreads;
  // with few entries, RG row groups split each slab's rows (entry e of group
  // g takes rows g, g + RG, ...); their float64 sums are added in group order
  constexpr int RG = NE >= kThreads ? 1 : kThreads / NE;
  constexpr int SL = 64;
  __shared__ float sm[SL][C + 1];
  __shared__ float sv[SL][B + 1];
  __shared__ double gsum[RG > 1 ? RG * NE : 1];
  const int tid = threadIdx.x;
  const int grp = RG > 1 ? tid / NE : 0;
  const int64_t r0 = int64_t(bid) * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < rows ? r0 + rows_per_blk : rows;
  double acc[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) acc[u] = 0.0;
  // the next slab is fetched into registers while the current one is used
  constexpr int PF = (SL * (C + B) + kThreads - 1) / kThreads;
  float pre[PF];
  if (r0 < r1) xgram_fetch<B, SL, PF>(pre, tid, r0, r1, v0, v1, y, vi);
  for (int64_t rs = r0; rs < r1; rs += SL) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int g = tid + i * kThreads;
      if (g < SL * (C + B)) {
        const int r = g / (C + B), c = g % (C + B);
        if (c < C) sm[r][c] = pre[i]; else sv[r][c - C] = pre[i];
      }
    }
    __syncthreads();
    if (rs + SL < r1) xgram_fetch<B, SL, PF>(pre, tid, rs + SL, r1, v0, v1, y, vi);
    if (RG > 1) {
      if (grp < RG) {
        const int e = tid - grp * NE;
        const int a = e / B, c = e % B;
        float sacc = 0.0f;
        for (int r = grp; r < SL; r += RG) sacc = fmaf(sm[r][a], sv[r][c], sacc);
        acc[0] += double(sacc);
      }
    } else {
#pragma unroll
      for (int u = 0; u < EPT; ++u) {
        const int e = tid + u * kThreads;
        if (e < NE) {
          const int a = e / B, c = e % B;
          float sacc = 0.0f;
          for (int r = 0; r < SL; ++r) sacc = fmaf(sm[r][a], sv[r][c], sacc);
          acc[u] += double(sacc);
        }
      }
    }
  }
  if (RG > 1) {
    if (grp < RG) gsum[tid] = acc[0];
    __syncthreads();
    if (tid < NE) {
      double t = gsum[tid];
      for (int g = 1; g < RG; ++g) t += gsum[g * NE + tid];
      partial[int64_t(bid) * NE + tid] = t;
    }
  } else {
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = tid + u * kThreads;
      if (e < NE) partial[int64_t(bid) * NE + e] = acc[u];
    }
  }
}

// The step's adjoint coefficients, one workgroup per expansion:
//   S = -X3^T R^-1 (B x C) in the last B rows of an otherwise zero C x C
//   matrix, Zr = R^-1 sym(.) R^-T, and Tadj = [Zr ; T^T] ((C + B) x C) with
//   T = R^-1[:, 2B:3B].
__global__ void __launch_bounds__(kThreads)
k_tadj(const double *__restrict__ X3all, const double *__restrict__ Rall, int B, int mask,
       double *__restrict__ Tall) {
  if (!((mask >> blockIdx.x) & 1)) return;
  const int C = 3 * B;
  const double *X3 = X3all + blockIdx.x * C * B;
  const double *Rg = Rall + blockIdx.x * C * C;
  double *Tadj = Tall + blockIdx.x * (C + B) * C;
  __shared__ double Rs[48 * 48];
  __shared__ double Zs[48 * 48];
  __shared__ double Z1[48 * 48];
  const int t = threadIdx.x;
  for (int e = t; e < C * C; e += kThreads) { Rs[e] = Rg[e]; Zs[e] = 0.0; }
  __syncthreads();
  // S[c][q] = -sum_a X3[a][c] R^-1[a][q]  -> row 2B + c
  for (int e = t; e < B * C; e += kThreads) {
    const int c = e / C, q = e % C;
    double acc = 0.0;
    for (int a = 0; a < C; ++a) acc -= X3[a * B + c] * Rs[a * C + q];
    Zs[(2 * B + c) * C + q] = acc;
  }
  __syncthreads();
  // sym: copy the lower triangle onto the upper (entries above stay as
  // mirrors of those below the diagonal)
  for (int e = t; e < C * C; e += kThreads) {
    const int i = e / C, j = e % C;
    Z1[e] = i >= j ? Zs[e] : Zs[j * C + i];
  }
  __syncthreads();
  // Zs = R^-1 Z1
  for (int e = t; e < C * C; e += kThreads) {
    const int i = e / C, j = e % C;
    double acc = 0.0;
    for (int l = 0; l < C; ++l) acc += Rs[i * C + l] * Z1[l * C + j];
    Zs[e] = acc;
  }
  __syncthreads();
  // Tadj[0:C] = Zs R^-T ; Tadj[C + c][q] = R^-1[q][2B + c]
  for (int e = t; e < C * C; e += kThreads) {
    const int i = e / C, j = e % C;
    double acc = 0.0;
    for (int l = 0; l < C; ++l) acc += Zs[i * C + l] * Rs[j * C + l];
    Tadj[e] = acc;
  }
  for (int e = t; e < B * C; e += kThreads) {
    const int c = e / C, q = e % C;
    Tadj[(C + c) * C + q] = Rs[q * C + 2 * B + c];
  }
}

// Mbar = [v0 | v1 | y | vbar] Tadj; one thread per (row, output block g):
// g = 0 -> accP += (Vbar_{j-2}), g = 1 -> accC += (Vbar_{j-1}), g = 2 -> ybar.
// Both expansions in one launch: logical workgroups [0, nb0) take side 0,
// the rest side 1.
struct AapplySide {
  const float *v0, *v1, *y, *vb;
  const double *Tadj;
  int64_t rows;
  float *accP, *accC, *ybar;
};
struct AapplyPair {
  AapplySide s[2];
  int64_t nb0;
};

template <int B>
__global__ void __launch_bounds__(kThreads)
k_aapply(const AapplyPair P) {
  constexpr int C = 3 * B;
  __shared__ float Ts[(C + B) * C];
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const bool second = lb >= P.nb0;
  const float *__restrict__ v0 = second ? P.s[1].v0 : P.s[0].v0;
  const float *__restrict__ v1 = second ? P.s[1].v1 : P.s[0].v1;
  const float *__restrict__ y = second ? P.s[1].y : P.s[0].y;
  const float *__restrict__ vb = second ? P.s[1].vb : P.s[0].vb;
  const double *__restrict__ Tadj = second ? P.s[1].Tadj : P.s[0].Tadj;
  const int64_t rows = second ? P.s[1].rows : P.s[0].rows;
  float *__restrict__ accP = second ? P.s[1].accP : P.s[0].accP;
  float *__restrict__ accC = second ? P.s[1].accC : P.s[0].accC;
  float *__restrict__ ybar = second ? P.s[1].ybar : P.s[0].ybar;
  for (int e = threadIdx.x; e < (C + B) * C; e += kThreads) Ts[e] = float(Tadj[e]);
  __syncthreads();
  const int64_t gid = (lb - (second ? P.nb0 : 0)) * kThreads + threadIdx.x;
  const int64_t r = gid / 3;
  const int g = int(gid % 3);
  if (r >= rows) return;
  float *dst = g == 0 ? accP : (g == 1 ? accC : ybar);
  if (!dst) return;
  float out[B];
#pragma unroll
  for (int c = 0; c < B; ++c) out[c] = 0.0f;
  const float *src[4] = {v0, v1, y, vb};
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    if (!src[a]) continue;
    const float *row = src[a] + r * B;
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const float x = row[u];
      const float *tr = Ts + (a * B + u) * C + g * B;
#pragma unroll
      for (int c = 0; c < B; ++c) out[c] = fmaf(x, tr[c], out[c]);
    }
  }
  float *d = dst + r * B;
  if (g == 2) {
#pragma unroll
    for (int c = 0; c < B; ++c) d[c] = out[c];
  } else {
#pragma unroll
    for (int c = 0; c < B; ++c) d[c] += out[c];
  }
}

// Node part of the weight terms of one step (both expansions), and
// Vbar_{j-1} += A ybar on node rows.
template <int B>
__global__ void __launch_bounds__(kThreads)
k_wnode(int64_t n, const float *__restrict__ s, const float *__restrict__ ybs,
        const float *__restrict__ ys, const float *__restrict__ xs, const float *__restrict__ ays,
        const float *__restrict__ ybc, const float *__restrict__ yc, const float *__restrict__ xc,
        const float *__restrict__ ayc, float *__restrict__ accs, float *__restrict__ accc,
        double *__restrict__ znode, double *__restrict__ hnode) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double z = 0.0, h = 0.0;
  if (ybs) {
    for (int c = 0; c < B; ++c) {
      const int64_t i = p * B + c;
      z += double(xs[i]) * double(ays[i]) + double(ybs[i]) * double(ys[i]);
      if (accs) accs[i] += ays[i];
    }
  }
  if (ybc) {
    for (int c = 0; c < B; ++c) {
      const int64_t i = p * B + c;
      z += double(ybc[i]) * double(yc[i]) + double(xc[i]) * double(ayc[i]);
      h += double(ybc[i]) * double(xc[i]);
      if (accc) accc[i] += ayc[i];
    }
  }
  const double s2 = double(s[p]) * double(s[p]);
  znode[p] += s2 * z;
  hnode[p] += s2 * h;
}

// Hyperedge part of one step: star hyperedge rows (offset n) and the clique
// products T . Tbar; Vbar_{j-1} += A ybar on star hyperedge rows.
template <int B>
__global__ void __launch_bounds__(kThreads)
k_wedge(int64_t n, int64_t m, const int32_t *__restrict__ eptr, const float *__restrict__ w,
        const float *__restrict__ ybs, const float *__restrict__ ys, const float *__restrict__ xs,
        const float *__restrict__ ays, const float *__restrict__ tbar, const float *__restrict__ tf,
        float *__restrict__ accs, double *__restrict__ eacc) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const double we = w ? double(w[e]) : 1.0;
  double acc = 0.0;
  if (ybs) {
    double es = 0.0;
    for (int c = 0; c < B; ++c) {
      const int64_t i = (n + e) * B + c;
      es += double(ybs[i]) * double(ys[i]) + double(xs[i]) * double(ays[i]);
      if (accs) accs[i] += ays[i];
    }
    acc += es / (2.0 * we);
  }
  if (tbar) {
    double ec = 0.0;
    // T_e lives in the SpMM scratch at row stride 2B, offset B
    for (int c = 0; c < B; ++c)
      ec += double(tbar[e * 2 * B + B + c]) * double(tf[e * 2 * B + B + c]);
    const double k = double(eptr[e + 1] - eptr[e]);
    acc += ec * (k * (k - 1.0)) / (we * we);  // = ec / (w_e beta_e)
  }
  eacc[e] += acc;
}

// dw_e = eacc_e - 1/(2|e|) sum_{p in e} znode_p - 1/(|e|(|e|-1)) sum_{p in e} hnode_p
//        + wdirect_e   (beta_e / w_e = 1/(|e|(|e|-1)))
__global__ void k_wfinal(const int32_t *__restrict__ eptr, const int32_t *__restrict__ pins,
                         int64_t m, const double *__restrict__ eacc,
                         const double *__restrict__ znode, const double *__restrict__ hnode,
                         const double *__restrict__ wdirect, float *__restrict__ dw) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int32_t a = eptr[e], b = eptr[e + 1];
  double gz = 0.0, gh = 0.0;
  // pins in chunks of 8 (loads first), added in CSR order
  for (int32_t j0 = a; j0 < b; j0 += 8) {
    int32_t pp[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) pp[u] = pins[j0 + u < b ? j0 + u : b - 1];
    double z[8], hv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      z[u] = znode[pp[u]];
      hv[u] = hnode[pp[u]];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (j0 + u < b) {
        gz += z[u];
        gh += hv[u];
      }
  }
  const double k = double(b - a);
  dw[e] = float(eacc[e] - gz / (2.0 * k) - gh / (k * (k - 1.0)) + wdirect[e]);
}

int lanes_for(int K, int CPL) {
  int need = (K + CPL - 1) / CPL;
  int l = 1;
  while (l < need) l <<= 1;
  return l;
}

// ------------------------------------------------------------ workspace
struct BwdWs {
  Structure st;
  int32_t *flags = nullptr;
  float *xs = nullptr, *xc = nullptr;   // generated start blocks
  float *P = nullptr, *chi = nullptr;   // pool before (row-octet) / after the joint QR
  double *qh = nullptr;
  float *R = nullptr;
  double *rinvJ = nullptr;
  KrylovTape tape;
  int32_t *istar = nullptr;
  double *qsum = nullptr, *wdirect = nullptr, *spart = nullptr;
  float *sfwd = nullptr;                // the forward's numerators (m x K)
  int32_t *cslot = nullptr;
  float *chibar = nullptr;
  char *big = nullptr;                  // slot_a | slot_b | dbar, later pbar
  double *Mq = nullptr;
  float *W1 = nullptr, *W2 = nullptr;
  float *vseg_s = nullptr, *vseg_c = nullptr, *yseg_s = nullptr, *yseg_c = nullptr;
  float *tseg = nullptr;
  float *abar_s = nullptr, *abar_c = nullptr;
  float *vb_s = nullptr, *vb_c = nullptr, *yb_s = nullptr, *yb_c = nullptr;
  float *ay_s = nullptr, *ay_c = nullptr, *tbar = nullptr;
  double *xpart = nullptr, *X3 = nullptr, *Tadj = nullptr;
  double *znode = nullptr, *hnode = nullptr, *eacc = nullptr;
};

int seg_of(const hef_params &p) { return (p.ckpt_every > 0 && p.ckpt_every < p.k) ? p.ckpt_every : p.k; }

void carve(Arena &a, int64_t n, int64_t m, int64_t nnz, const hef_params &p, BwdWs &w) {
  const int B = p.b, k = p.k, K = pool_width_of(p), C = 3 * B;
  const int Kp = (K + 31) / 32 * 32;
  const int64_t Ns = n + m;
  const int seg = seg_of(p);
  const int nseg = (k + seg - 1) / seg;
  structure_carve(a, n, m, nnz, w.st);
  w.flags = a.take<int32_t>(4);
  w.xs = a.take<float>(Ns * B);
  w.xc = a.take<float>(n * B);
  w.P = a.take<float>(oct_rows(n) * K);
  w.chi = a.take<float>(n * K);
  w.qh = a.take<double>(K);
  w.R = a.take<float>(m);
  w.rinvJ = a.take<double>(int64_t(Kp) * Kp);
  w.tape.seg = seg;
  w.tape.T = a.take<double>(int64_t(k + 1) * 2 * C * B);
  w.tape.Rinv = a.take<double>(int64_t(k + 1) * 2 * C * C);
  w.tape.ck_star = a.take<float>(int64_t(nseg) * 2 * Ns * B);
  w.tape.ck_clique = a.take<float>(int64_t(nseg) * 2 * n * B);
  w.istar = a.take<int32_t>(m);
  w.qsum = a.take<double>(K);
  w.wdirect = a.take<double>(m);
  w.spart = a.take<double>(cdiv(std::max<int64_t>(m, 1), kEdgesPerBlk) * K);
  w.sfwd = a.take<float>(std::max<int64_t>(m, 1) * K);
  w.cslot = a.take<int32_t>(nnz);
  w.chibar = a.take<float>(n * K);
  w.big = a.take<char>(std::max<int64_t>(m * K * 12, n * K * 4));
  w.Mq = a.take<double>(int64_t(K) * K);
  w.W1 = a.take<float>(int64_t(Kp) * Kp);
  w.W2 = a.take<float>(int64_t(Kp) * Kp);
  w.vseg_s = a.take<float>(int64_t(seg) * Ns * B);
  w.vseg_c = a.take<float>(int64_t(seg) * n * B);
  w.yseg_s = a.take<float>(int64_t(seg) * Ns * B);
  w.yseg_c = a.take<float>(int64_t(seg) * n * B);
  w.tseg = a.take<float>(int64_t(seg) * spmm_scratch_floats(n, m, B));
  if (seg == k) {
    // one segment: the taped forward fills the step buffers itself (Y_j,
    // its clique sums, V_j), so the reverse sweep recomputes nothing
    w.tape.v_s = w.vseg_s;
    w.tape.v_c = w.vseg_c;
    w.tape.y_s = w.yseg_s;
    w.tape.y_c = w.yseg_c;
    w.tape.t = w.tseg;
  }
  w.abar_s = a.take<float>(3 * Ns * B);
  w.abar_c = a.take<float>(3 * n * B);
  w.vb_s = a.take<float>(Ns * B);
  w.vb_c = a.take<float>(n * B);
  w.yb_s = a.take<float>(Ns * B);
  w.yb_c = a.take<float>(n * B);
  w.ay_s = a.take<float>(Ns * B);
  w.ay_c = a.take<float>(n * B);
  w.tbar = a.take<float>(spmm_scratch_floats(n, m, B));
  w.xpart = a.take<double>(int64_t(2) * kXBlocks * C * B);
  w.X3 = a.take<double>(2 * C * B);
  w.Tadj = a.take<double>(2 * (C + B) * C);
  w.znode = a.take<double>(n);
  w.hnode = a.take<double>(n);
  w.eacc = a.take<double>(m);
}

size_t transient_bytes(int64_t n, int64_t m, int64_t nnz, const hef_params &p) {
  const int K = pool_width_of(p);
  size_t need = structure_build_ws(n, m, nnz);
  need = std::max(need, krylov_ws_bytes(n, m, p.b));
  need = std::max(need, orth_ws_bytes(n, K));
  need = std::max(need, score_ws_bytes(m, K));
  need = std::max(need, gram_cross_ws_bytes(n, K));
  Arena a;
  a.take<uint32_t>(nnz);
  a.take<uint32_t>(nnz);
  a.take<uint32_t>(nnz);
  need = std::max(need, a.mark() + radix_ws_bytes(nnz));
  return need + 4096;
}

// The step cross products X3 of both expansions (a side with zero rows
// contributes a zero X3), in one launch and one reduce.
struct StepSide {
  int64_t rows, pool_rows;
  float *abar;
  int col;
  float *vbar;
  const float *v0, *v1, *y;
  double *xpart, *X3;
};

template <int B>
hef_status step_kernels_t(const StepSide &a, const StepSide &b, const float *pbar, int K,
                          hipStream_t s) {
  constexpr int C = 3 * B;
  XgramPair P;
  int nb[2];
  const StepSide *sd[2] = {&a, &b};
  for (int i = 0; i < 2; ++i) {
    const StepSide &t = *sd[i];
    const int64_t per = std::max<int64_t>(64, cdiv(cdiv(t.rows, kXBlocks), 64) * 64);
    nb[i] = int(std::max<int64_t>(1, cdiv(t.rows, per)));
    P.s[i] = XgramSide{t.v0, t.v1, t.y, VbarIn{t.abar, pbar, K, t.col, t.pool_rows, t.vbar},
                       t.rows, per, t.xpart};
  }
  P.nb0 = nb[0];
  k_xgram<B><<<nb[0] + nb[1], kThreads, 0, s>>>(P);
  HEF_LAUNCH_CHECK();
  return reduce_cols_f64_pair(a.xpart, nb[0], a.X3, b.xpart, nb[1], b.X3, int64_t(C) * B, s);
}

hef_status step_kernels(int B, const StepSide &a, const StepSide &b, const float *pbar, int K,
                        hipStream_t s) {
  switch (B) {
    case 1: return step_kernels_t<1>(a, b, pbar, K, s);
    case 2: return step_kernels_t<2>(a, b, pbar, K, s);
    case 4: return step_kernels_t<4>(a, b, pbar, K, s);
    case 8: return step_kernels_t<8>(a, b, pbar, K, s);
    case 16: return step_kernels_t<16>(a, b, pbar, K, s);
    default: return HEF_ERR_UNSUPPORTED;
  }
}

template <int B>
hef_status aapply_t(const AapplySide &a, const AapplySide &b, hipStream_t s) {
  AapplyPair P;
  P.s[0] = a;
  P.s[1] = b;
  P.nb0 = cdiv(a.rows * 3, kThreads);
  const int64_t nblk = P.nb0 + cdiv(b.rows * 3, kThreads);
  if (nblk == 0) return HEF_OK;
  k_aapply<B><<<nblk, kThreads, 0, s>>>(P);
  HEF_LAUNCH_CHECK();
  return HEF_OK;
}

hef_status aapply(int B, const AapplySide &a, const AapplySide &b, hipStream_t s) {
  switch (B) {
    case 1: return aapply_t<1>(a, b, s);
    case 2: return aapply_t<2>(a, b, s);
    case 4: return aapply_t<4>(a, b, s);
    case 8: return aapply_t<8>(a, b, s);
    case 16: return aapply_t<16>(a, b, s);
    default: return HEF_ERR_UNSUPPORTED;
  }
}

template <int B>
hef_status weights_t(const Level &L, const Structure &st, const float *ybs, const float *ys,
                     const float *xs, const float *ays, const float *ybc, const float *yc,
                     const float *xc, const float *ayc, const float *tbar, const float *tf,
                     float *accs, float *accc, double *znode, double *hnode, double *eacc,
                     hipStream_t s) {
  if (L.n > 0)
    k_wnode<B><<<cdiv(L.n, 256), 256, 0, s>>>(L.n, st.s, ybs, ys, xs, ays, ybc, yc, xc, ayc, accs,
                                             accc, znode, hnode);
  if (L.m > 0)
    k_wedge<B><<<cdiv(L.m, 256), 256, 0, s>>>(L.n, L.m, L.eptr, L.w, ybs, ys, xs, ays, tbar, tf,
                                             accs, eacc);
  HEF_LAUNCH_CHECK();
  return HEF_OK;
}

hef_status weights(int B, const Level &L, const Structure &st, const float *ybs, const float *ys,
                   const float *xs, const float *ays, const float *ybc, const float *yc,
                   const float *xc, const float *ayc, const float *tbar, const float *tf,
                   float *accs, float *accc, double *znode, double *hnode, double *eacc,
                   hipStream_t s) {
  switch (B) {
    case 1: return weights_t<1>(L, st, ybs, ys, xs, ays, ybc, yc, xc, ayc, tbar, tf, accs, accc, znode, hnode, eacc, s);
    case 2: return weights_t<2>(L, st, ybs, ys, xs, ays, ybc, yc, xc, ayc, tbar, tf, accs, accc, znode, hnode, eacc, s);
    case 4: return weights_t<4>(L, st, ybs, ys, xs, ays, ybc, yc, xc, ayc, tbar, tf, accs, accc, znode, hnode, eacc, s);
    case 8: return weights_t<8>(L, st, ybs, ys, xs, ays, ybc, yc, xc, ayc, tbar, tf, accs, accc, znode, hnode, eacc, s);
    case 16: return weights_t<16>(L, st, ybs, ys, xs, ays, ybc, yc, xc, ayc, tbar, tf, accs, accc, znode, hnode, eacc, s);
    default: return HEF_ERR_UNSUPPORTED;
  }
}

template <int CPL>
hef_status score_adjoint_t(const Level &L, const Structure &st, const float *chi, int K,
                           const double *qh, const float *dR, BwdWs &w, hipStream_t s) {
  const int LPR = lanes_for(K, CPL);
  const int64_t nblk = cdiv(L.m, kEdgesPerBlk);
  k_sadj_a<CPL><<<nblk, kThreads, 0, s>>>(w.sfwd, K, LPR, L.m, qh, dR, w.istar,
                                          w.spart);
  HEF_LAUNCH_CHECK();
  HEF_TRY(reduce_cols_f64(w.spart, nblk, K, w.qsum, s));
  int32_t *slot_a = reinterpret_cast<int32_t *>(w.big);
  int32_t *slot_b = slot_a + int64_t(L.m) * K;
  float *dbar = reinterpret_cast<float *>(slot_b + int64_t(L.m) * K);
  k_sadj_b<CPL><<<nblk, kThreads, 0, s>>>(L.eptr, L.pins, chi, K, LPR, L.m, qh, dR, L.w, w.istar,
                                          w.qsum, slot_a, slot_b, dbar, w.wdirect);
  HEF_LAUNCH_CHECK();
  const int ngrp = kThreads / LPR;
  if (L.n > 0) {
    k_sadj_c<CPL><<<cdiv(L.n, ngrp), kThreads, 0, s>>>(st.vptr, st.eids, w.cslot, slot_a, slot_b,
                                                      dbar, K, LPR, L.n, w.chibar);
    HEF_LAUNCH_CHECK();
  }
  return HEF_OK;
}

}  // namespace

size_t backward_bytes(int64_t n, int64_t m, int64_t nnz, const hef_params &p) {
  Arena a;
  BwdWs w;
  carve(a, n, m, nnz, p, w);
  return a.mark() + transient_bytes(n, m, nnz, p) + 1024;
}

// The forward with tape (the computation of hef_resistance, FP32 pool): the
// structure, pool, orthonormal pool, Q_H, R and the Krylov tape stay in the
// carved part of the workspace (arguments already checked; n, m > 0).
hef_status taped_forward(const Level &L, const hef_params &p, const float *start_star,
                         const float *start_clique, BwdWs &w, Arena &a, hipStream_t s) {
  const int64_t n = L.n, m = L.m;
  const int B = p.b, k = p.k, K = pool_width_of(p);
  const int64_t Ns = n + m;
  const bool use_star = !(p.flags & HEF_FLAG_CLIQUE_ONLY);
  const bool use_clique = !(p.flags & HEF_FLAG_STAR_ONLY);
  const Structure &st = w.st;
  HEF_TRY(structure_build(L, w.st, a, s));
  if (use_star && !start_star) {
    HEF_TRY(start_block(p.seed, 0, 0, Ns, B, w.xs, s));
    start_star = w.xs;
  }
  if (use_clique && !start_clique) {
    HEF_TRY(start_block(p.seed, 0, 1, n, B, w.xc, s));
    start_clique = w.xc;
  }
  KrylovOut ko;
  ko.pool = w.P;
  ko.K = K;
  ko.pool_type = kPoolF32;
  HEF_TRY(krylov_pool(L, st, B, k, double(p.drop_tol), start_star, start_clique, use_star,
                      use_clique, ko, a, s, &w.tape));
  HEF_TRY(orthonormalize_pool(w.P, w.chi, kPoolF32, n, K, double(p.drop_tol), 1, nullptr, a, s,
                              w.rinvJ));
  HEF_TRY(score_pool(L, w.chi, kPoolF32, K, w.qh, w.R, a, s, w.sfwd));
  return HEF_OK;
}

// The reverse sweep from the tape left by taped_forward in the same workspace.
hef_status reverse_sweep(const Level &L, const hef_params &p, const float *dR, float *dw,
                         BwdWs &w, Arena &a, hipStream_t s) {
  const int64_t n = L.n, m = L.m, nnz = L.nnz;
  const int B = p.b, k = p.k, K = pool_width_of(p), C = 3 * B;
  const int Kp = (K + 31) / 32 * 32;
  const int64_t Ns = n + m;
  const bool use_star = !(p.flags & HEF_FLAG_CLIQUE_ONLY);
  const bool use_clique = !(p.flags & HEF_FLAG_STAR_ONLY);
  const int64_t bk = int64_t(B) * k;
  const Structure &st = w.st;
  TimedScope ts(kStAdjoint, s);
  // ---- 1. ratios -> chibar
  {
    const size_t mk = a.mark();
    uint32_t *keys = a.take<uint32_t>(nnz);
    uint32_t *vals = a.take<uint32_t>(nnz);
    uint32_t *keys_out = a.take<uint32_t>(nnz);
    HEF_WS_CHECK(a);
    k_pos_pairs<<<cdiv(nnz, 256), 256, 0, s>>>(L.pins, keys, vals, nnz);
    HEF_LAUNCH_CHECK();
    HEF_TRY(radix_sort_pairs(keys, vals, keys_out, reinterpret_cast<uint32_t *>(w.cslot), nnz,
                             bits_for(n > 0 ? n - 1 : 0), a, s));
    a.reset(mk);
  }
  if (K > 256) HEF_TRY(score_adjoint_t<8>(L, st, w.chi, K, w.qh, dR, w, s));
  else HEF_TRY(score_adjoint_t<4>(L, st, w.chi, K, w.qh, dR, w, s));

  // ---- 2. joint QR: pbar = chibar R^-T + chi sym(-chibar^T chi) R^-T
  float *pbar = reinterpret_cast<float *>(w.big);
  HEF_TRY(gram_cross_f32(w.chibar, w.chi, n, K, w.Mq, a, s));
  k_qradj_w<<<cdiv(int64_t(Kp) * Kp, 256), 256, 0, s>>>(w.rinvJ, w.Mq, K, Kp, w.W1, w.W2);
  HEF_LAUNCH_CHECK();
  HEF_TRY(gemm_f32(w.chibar, n, K, w.W1, Kp, pbar, false, s));
  HEF_TRY(gemm_f32(w.chi, n, K, w.W2, Kp, pbar, true, s));

  // ---- 3. Lanczos steps in reverse, segment by segment
  HEF_TRY(zero_async(w.abar_s, sizeof(float) * 3 * Ns * B, s));
  HEF_TRY(zero_async(w.abar_c, sizeof(float) * 3 * n * B, s));
  HEF_TRY(zero_async(w.znode, sizeof(double) * n, s));
  HEF_TRY(zero_async(w.hnode, sizeof(double) * n, s));
  HEF_TRY(zero_async(w.eacc, sizeof(double) * m, s));
  HEF_TRY(zero_async(w.X3, sizeof(double) * 2 * C * B, s));
  const int seg = w.tape.seg;
  const int nseg = (k + seg - 1) / seg;
  const int mask = (use_star ? 1 : 0) | (use_clique ? 2 : 0);
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int j0 = sg * seg;
    const int j1 = std::min(j0 + seg, k);
    const float *cks = w.tape.ck_star + size_t(sg) * 2 * Ns * B;
    const float *ckc = w.tape.ck_clique + size_t(sg) * 2 * n * B;
    // V_j of this segment: j0-1 and j0 from the checkpoint, the rest cached
    auto vs = [&](int j) -> const float * {
      if (j < 0) return nullptr;
      if (j == j0 - 1) return cks;
      if (j == j0) return cks + Ns * B;
      return w.vseg_s + size_t(j - j0 - 1) * Ns * B;
    };
    auto vc = [&](int j) -> const float * {
      if (j < 0) return nullptr;
      if (j == j0 - 1) return ckc;
      if (j == j0) return ckc + n * B;
      return w.vseg_c + size_t(j - j0 - 1) * n * B;
    };
    // recompute: Y_j = A V_{j-1} (with the clique sums T) and V_j, j < j1
    // (nothing to do when the taped forward kept every step)
    for (int j = j0 + 1; j <= j1 && !w.tape.y_s; ++j) {
      const int t = j - j0 - 1;
      float *ysj = w.yseg_s + size_t(t) * Ns * B;
      float *ycj = w.yseg_c + size_t(t) * n * B;
      float *tj = w.tseg + size_t(t) * spmm_scratch_floats(n, m, B);
      HEF_TRY(spmm_apply(L, st, B, use_star ? vs(j - 1) : nullptr, use_star ? ysj : nullptr,
                         use_clique ? vc(j - 1) : nullptr, use_clique ? ycj : nullptr, tj, s));
      if (j < j1) {
        const double *Tj = w.tape.T + size_t(j) * 2 * C * B;
        HEF_TRY(lanczos_apply_pair(B, j >= 2 ? vs(j - 2) : nullptr, vs(j - 1), ysj, Tj,
                                   w.vseg_s + size_t(t) * Ns * B, use_star ? Ns : 0,
                                   j >= 2 ? vc(j - 2) : nullptr, vc(j - 1), ycj, Tj + C * B,
                                   w.vseg_c + size_t(t) * n * B, use_clique ? n : 0, K, s));
      }
    }
    for (int j = j1; j > j0; --j) {
      const int t = j - j0 - 1;
      const float *ysj = w.yseg_s + size_t(t) * Ns * B;
      const float *ycj = w.yseg_c + size_t(t) * n * B;
      const float *tj = w.tseg + size_t(t) * spmm_scratch_floats(n, m, B);
      const float *ps = j >= 2 ? vs(j - 2) : nullptr, *pc = j >= 2 ? vc(j - 2) : nullptr;
      float *as_j = w.abar_s + size_t(j % 3) * Ns * B;
      float *as_1 = j >= 2 ? w.abar_s + size_t((j - 1) % 3) * Ns * B : nullptr;
      float *as_2 = j >= 3 ? w.abar_s + size_t((j - 2) % 3) * Ns * B : nullptr;
      float *ac_j = w.abar_c + size_t(j % 3) * n * B;
      float *ac_1 = j >= 2 ? w.abar_c + size_t((j - 1) % 3) * n * B : nullptr;
      float *ac_2 = j >= 3 ? w.abar_c + size_t((j - 2) % 3) * n * B : nullptr;
      const int col_s = int((j - 1) * int64_t(B));
      const int col_c = int((use_star ? bk : 0) + (j - 1) * int64_t(B));
      {
        const StepSide ss{use_star ? Ns : 0, n, as_j, col_s, w.vb_s, ps, vs(j - 1), ysj,
                          w.xpart, w.X3};
        const StepSide sc{use_clique ? n : 0, n, ac_j, col_c, w.vb_c, pc, vc(j - 1), ycj,
                          w.xpart + size_t(kXBlocks) * C * B, w.X3 + C * B};
        HEF_TRY(step_kernels(B, ss, sc, pbar, K, s));
      }
      k_tadj<<<2, kThreads, 0, s>>>(w.X3, w.tape.Rinv + size_t(j) * 2 * C * C, B, mask, w.Tadj);
      HEF_LAUNCH_CHECK();
      {
        const AapplySide sa{ps, vs(j - 1), ysj, w.vb_s, w.Tadj, use_star ? Ns : 0, as_2, as_1,
                            w.yb_s};
        const AapplySide sc{pc, vc(j - 1), ycj, w.vb_c, w.Tadj + (C + B) * C, use_clique ? n : 0,
                            ac_2, ac_1, w.yb_c};
        HEF_TRY(aapply(B, sa, sc, s));
      }
      HEF_TRY(spmm_apply(L, st, B, use_star ? w.yb_s : nullptr, use_star ? w.ay_s : nullptr,
                         use_clique ? w.yb_c : nullptr, use_clique ? w.ay_c : nullptr, w.tbar, s));
      HEF_TRY(weights(B, L, st, use_star ? w.yb_s : nullptr, ysj, vs(j - 1), w.ay_s,
                      use_clique ? w.yb_c : nullptr, ycj, vc(j - 1), w.ay_c,
                      use_clique ? w.tbar : nullptr, tj, as_1, ac_1, w.znode, w.hnode, w.eacc,
                      s));
    }
  }

  // ---- 4. gather per hyperedge
  k_wfinal<<<cdiv(m, 256), 256, 0, s>>>(L.eptr, L.pins, m, w.eacc, w.znode, w.hnode, w.wdirect,
                                        dw);
  HEF_LAUNCH_CHECK();
  return HEF_OK;
}

}  // namespace hef

using namespace hef;

extern "C" {

hef_status hef_resistance_backward(const hef_hypergraph *hg, const hef_params *p,
                                   const float *start_star, const float *start_clique,
                                   const float *dR, float *dw, void *ws, size_t ws_bytes,
                                   hipStream_t stream) {
  if (!hg || !p) { set_error("NULL argument"); return HEF_ERR_INVALID_ARGUMENT; }
  size_t need = 0;
  HEF_TRY(hef_workspace_size(hg, p, HEF_OP_BACKWARD, &need));
  if (!ws) { set_error("workspace is NULL"); return HEF_ERR_INVALID_ARGUMENT; }
  if (ws_bytes < need) {
    set_error("workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    return HEF_ERR_WORKSPACE_TOO_SMALL;
  }
  if (hg->m > 0 && (!dR || !dw)) { set_error("dR or dw is NULL"); return HEF_ERR_INVALID_ARGUMENT; }
  if (p->orth_passes != 1) {
    set_error("the adjoint supports orth_passes = 1");
    return HEF_ERR_UNSUPPORTED;
  }
  Arena a;
  a.base = static_cast<char *>(ws);
  a.cap = ws_bytes;
  Level L;
  L.n = hg->n; L.m = hg->m; L.nnz = hg->nnz; L.eptr = hg->eptr; L.pins = hg->pins; L.w = hg->w;
  if (!(p->flags & (HEF_FLAG_ASSUME_VALID | HEF_FLAG_TAPED))) {
    Arena t = a;
    Structure st;
    structure_carve(t, L.n, L.m, L.nnz, st);
    int32_t *flags = t.take<int32_t>(4);
    int32_t bad = 0;
    HEF_TRY(validate_device(L, flags, &bad, stream));
    if (bad) { set_error("invalid hypergraph (code %d)", bad); return HEF_ERR_INVALID_HYPERGRAPH; }
  }
  if (L.m == 0) return HEF_OK;
  if (L.n == 0) {
    HEF_TRY(zero_async(dw, sizeof(float) * L.m, stream));
    return HEF_OK;
  }
  BwdWs w;
  carve(a, L.n, L.m, L.nnz, *p, w);
  HEF_WS_CHECK(a);
  if (!(p->flags & HEF_FLAG_TAPED))
    HEF_TRY(taped_forward(L, *p, start_star, start_clique, w, a, stream));
  return reverse_sweep(L, *p, dR, dw, w, a, stream);
}

hef_status hef_resistance_taped(const hef_hypergraph *hg, const hef_params *p,
                                const float *start_star, const float *start_clique, float *R,
                                void *ws, size_t ws_bytes, hipStream_t stream) {
  if (!hg || !p) { set_error("NULL argument"); return HEF_ERR_INVALID_ARGUMENT; }
  size_t need = 0;
  HEF_TRY(hef_workspace_size(hg, p, HEF_OP_BACKWARD, &need));
  if (!ws) { set_error("workspace is NULL"); return HEF_ERR_INVALID_ARGUMENT; }
  if (ws_bytes < need) {
    set_error("workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    return HEF_ERR_WORKSPACE_TOO_SMALL;
  }
  if (hg->m > 0 && !R) { set_error("R is NULL"); return HEF_ERR_INVALID_ARGUMENT; }
  if (p->orth_passes != 1) {
    set_error("the adjoint supports orth_passes = 1");
    return HEF_ERR_UNSUPPORTED;
  }
  Arena a;
  a.base = static_cast<char *>(ws);
  a.cap = ws_bytes;
  Level L;
  L.n = hg->n; L.m = hg->m; L.nnz = hg->nnz; L.eptr = hg->eptr; L.pins = hg->pins; L.w = hg->w;
  if (!(p->flags & HEF_FLAG_ASSUME_VALID)) {
    Arena t = a;
    Structure st;
    structure_carve(t, L.n, L.m, L.nnz, st);
    int32_t *flags = t.take<int32_t>(4);
    int32_t bad = 0;
    HEF_TRY(validate_device(L, flags, &bad, stream));
    if (bad) { set_error("invalid hypergraph (code %d)", bad); return HEF_ERR_INVALID_HYPERGRAPH; }
  }
  if (L.m == 0) return HEF_OK;
  if (L.n == 0) {
    HEF_TRY(zero_async(R, sizeof(float) * L.m, stream));
    return HEF_OK;
  }
  BwdWs w;
  carve(a, L.n, L.m, L.nnz, *p, w);
  HEF_WS_CHECK(a);
  HEF_TRY(taped_forward(L, *p, start_star, start_clique, w, a, stream));
  HEF_HIP(hipMemcpyAsync(R, w.R, sizeof(float) * L.m, hipMemcpyDeviceToDevice, stream));
  return HEF_OK;
}

}  // extern "C"

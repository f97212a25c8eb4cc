// Block Krylov sequences of the normalised star and clique adjacencies.
#pragma once

#include "common.hpp"
#include "structure.hpp"

namespace hef {

// Row-major blocks with row stride B (= b: 1, 2, 4, 8 or 16):
//   star   block: (n+m) x B, node rows [0,n) then hyperedge rows [n, n+m)
//   clique block: n x B
struct Blocks {
  float *star = nullptr;
  float *clique = nullptr;
};

// One application of both normalised adjacencies (Section III-A: star
// expansion with z_b(e,p) = w_e/|e|, clique expansion with
// z_c(u,v) = sum_e w_e / C(|e|,2)), y = A x, implicit through CSR and CSC:
//   star   y_E[e] = alpha_e sum_{p in e} s_p x_V[p]
//          y_V[u] = s_u sum_{e ∋ u} alpha_e x_E[e]
//   clique T_e    = beta_e sum_{p in e} s_p x_c[p]
//          y_c[u] = s_u sum_{e ∋ u} T_e - gam_u x_c[u]
// `scratch` (spmm_scratch_floats) holds W (m x 2B, [alpha_e x_E | T_e]) then
// U (n x 2B, [s_p x_V | s_p x_c]); after the call T_e is at
// scratch[e * 2B + B + c].  Either expansion may be skipped (null pointers).
inline int64_t spmm_scratch_floats(int64_t n, int64_t m, int B) { return 2 * int64_t(B) * (n + m); }
hef_status spmm_apply(const Level &L, const Structure &st, int B, const float *xs,
                      float *ys, const float *xc, float *yc, float *scratch, hipStream_t s);

// Pool column storage.
enum PoolType { kPoolF32 = 0, kPoolBF16 = 1, kPoolF64 = 2 };

struct KrylovOut {
  void *pool = nullptr;  // oct_rows(n) x K, row-octet layout (fp32 or bf16)
  int K = 0;
  int pool_type = kPoolF32;
};

size_t krylov_ws_bytes(int64_t n, int64_t m, int B);

// What the adjoint keeps of a forward run (all device memory, caller-owned):
//  * T[j]    (j = 0..k): the two C x B matrices R^-1[:, y columns] of step j
//    (star then clique, C = 3B), float64;
//  * Rinv[j] (j = 0..k): the two whole C x C matrices R^-1, float64;
//  * ck_star / ck_clique: checkpoint pairs (V_{sc-1}, V_{sc}) for segments
//    s = 0..nseg-1 of `seg` steps (nseg = ceil(k/seg)); slot s holds
//    2 blocks of (n+m) x B (star) or n x B (clique); V_{-1} is zero;
//  * with one segment (seg = k) and the five step buffers set, every step
//    itself: y_s / y_c[j-1] = Y_j = A V_{j-1} (steps 1..k), t[j-1] its SpMM
//    scratch (the clique sums), v_s / v_c[j-1] = V_j (steps 1..k-1).  The
//    forward then writes its blocks there and the reverse sweep recomputes
//    nothing.
struct KrylovTape {
  int seg = 0;
  double *T = nullptr;
  double *Rinv = nullptr;
  float *ck_star = nullptr;
  float *ck_clique = nullptr;
  float *v_s = nullptr, *v_c = nullptr, *y_s = nullptr, *y_c = nullptr, *t = nullptr;
};

// k steps of block Lanczos per expansion (three-term recurrence; each new
// block is orthonormalised against the previous two in a float64 Gram
// metric, with the drop rule for breakdowns); writes the pool columns
// [star steps 1..k | clique steps 1..k], b columns per step, star node rows
// only.  `start_star` ((n+m) x B) and `start_clique` (n x B) are consumed.
// `use_star` / `use_clique` select the expansions (the pool then holds
// b*k columns of the one selected).  `tape` (nullable) records what the
// adjoint needs.
hef_status krylov_pool(const Level &L, const Structure &st, int B, int k, double tau,
                       const float *start_star, const float *start_clique, bool use_star,
                       bool use_clique, KrylovOut &out, Arena &ws, hipStream_t s,
                       const KrylovTape *tape = nullptr);

// The steps of one block-Lanczos iteration, for callers that drive the
// recurrence themselves (the adjoint):
//  * lanczos_gram: G (3B x 3B, float64) of M = [v0 | v1 | y] (null = zero
//    block) over `rows` rows; `partial` holds lanczos_partial_elems(B);
//  * lanczos_solve: for two expansions' Grams G2 = [G_star | G_clique]
//    (C x C each, C = 3B, consecutive), Cholesky with the drop rule and
//    T2 = [T_star | T_clique], T = R^-1[:, y columns] (C x B each); R2
//    (nullable) receives both whole R^-1 (C x C each, consecutive);
//  * lanczos_apply: vn = M T (float64 arithmetic), optional pool write;
//  * lanczos_apply_pair: two lanczos_apply without pool writes (sides a and
//    b, a side with zero rows skipped) in one launch.
size_t lanczos_partial_elems(int B);
hef_status lanczos_gram(const float *v0, const float *v1, const float *y, int64_t rows, int B,
                        double *partial, double *G, hipStream_t s);
hef_status lanczos_solve(const double *G2, int B, double tau, double *T2, int32_t *drops,
                         double *R2, hipStream_t s);
hef_status lanczos_apply(int B, const float *v0, const float *v1, const float *y, const double *T,
                         float *vn, int64_t rows, void *pool, int pool_type, int64_t pool_rows,
                         int K, int col0, hipStream_t s);
hef_status lanczos_apply_pair(int B, const float *v0a, const float *v1a, const float *ya,
                              const double *Ta, float *vna, int64_t rowsa, const float *v0b,
                              const float *v1b, const float *yb, const double *Tb, float *vnb,
                              int64_t rowsb, int K, hipStream_t s);

// Counter-based N(0,1) start block (splitmix64 + Box-Muller in float64).
hef_status start_block(uint64_t seed, int level, int expansion, int64_t rows, int B,
                       float *out, hipStream_t s);

}  // namespace hef

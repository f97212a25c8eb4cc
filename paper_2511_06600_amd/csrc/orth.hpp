// Joint block orthonormalisation of the pool (Cholesky QR on matrix cores).
#pragma once

#include "common.hpp"

namespace hef {

size_t orth_ws_bytes(int64_t n, int K);

// Orthonormalises the Krylov pool (Alg. 1, the joint Gram-Schmidt
// of [star | clique]): G = V^T V (matrix-core tiles, float64 across row
// chunks), Cholesky G = R^T R in float64 with the drop rule (column j
// dropped when its Schur pivot <= tau^2 G_jj), Q = V R^-1.  `P` holds V in
// the row-octet layout (oct_rows(n) x K); Q goes to `out` (n x K row-major).
// `passes` = 2 repeats the factorisation on Q (keeping the first pass's
// drops), using P as scratch.  `keep_out` (device int32 [K], may be null)
// receives 1 for kept and 0 for dropped columns; `rinv_out` (device float64
// [Kp x Kp], Kp = K rounded up to 32, may be null) the last pass's R^-1
// (row-major, upper triangular, zero rows and columns for drops); `rho_out`
// (device float64 [K], may be null) the first pass's relative residuals
// rho_j = |R_jj| / ||V_j|| (0 for dropped columns).
hef_status orthonormalize_pool(void *P, void *out, int pool_type, int64_t n, int K, double tau,
                               int passes, int32_t *keep_out, Arena &ws, hipStream_t s,
                               double *rinv_out = nullptr, double *rho_out = nullptr);

// Test hook: G = X^T X (float64, K x K) of a row-major n x K float32 matrix,
// through the same matrix-core Gram kernels.
hef_status gram_f32(const float *X, int64_t n, int K, double *G, Arena &ws, hipStream_t s);

// G = X^T W (float64, K x K, not symmetric) of two row-major n x K float32
// matrices, through the same kernels; scratch gram_cross_ws_bytes(n, K).
size_t gram_cross_ws_bytes(int64_t n, int K);
hef_status gram_cross_f32(const float *X, const float *W, int64_t n, int K, double *G, Arena &ws,
                          hipStream_t s);

// out (n x K) = X W, or out += X W if `accumulate`, for a general K x K
// float32 matrix W (row-major, row stride Kp), on the matrix cores.
hef_status gemm_f32(const float *X, int64_t n, int K, const float *W, int Kp, float *out,
                    bool accumulate, hipStream_t s);

}  // namespace hef

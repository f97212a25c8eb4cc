/*
 * hyperef.h -- C ABI of the MI355X (gfx950) HyperEF 2.0 hot path.
 *
 * The calls follow the paper's problem statement:
 *   Alg. 1 ("Effective resistance estimation"): hypergraph H = (V, E, w) in,
 *          the vector R of hyperedge effective resistances out;
 *   Alg. 2 ("Resistance-Based Hypergraph Local Clustering"): H in, a
 *          coarsened hypergraph and the vertex clusters C out.
 *
 * Conventions shared by every call
 * --------------------------------
 * Ownership.  The library never allocates or frees device memory.  Every
 *   pointer marked DEVICE is caller-owned device memory on the current HIP
 *   device; scratch memory comes from the caller's workspace `ws` of
 *   `ws_bytes` bytes (256-byte aligned), sized by hef_workspace_size().
 * Streams.  Calls enqueue their work on `stream` and return; device outputs
 *   are valid once the stream is synchronised.  Calls with a HOST output
 *   (n_clusters) synchronise `stream` before returning.
 * Errors.  Every call returns an hef_status.  Argument checks run on the host
 *   before any launch; when one fails nothing is written.  Unless
 *   HEF_FLAG_ASSUME_VALID is set, the hypergraph is validated on the device
 *   first (one stream synchronisation); an invalid hypergraph returns
 *   HEF_ERR_INVALID_HYPERGRAPH with no output written.  HIP runtime failures
 *   return HEF_ERR_DEVICE.  hef_last_error() gives a text for the last
 *   non-OK status of the calling thread.
 * Determinism.  Identical inputs, parameters and device give bitwise-
 *   identical outputs: floating-point reductions use fixed orders and the
 *   clustering stage uses integer atomics only.
 * Concurrency.  Calls are reentrant; two calls may run concurrently if they
 *   use different workspaces.
 *
 * Hypergraph layout (CSR over hyperedges)
 * ---------------------------------------
 *   eptr[m+1]  int32, eptr[0] = 0, non-decreasing, eptr[m] = nnz;
 *   pins[nnz]  int32, 0 <= pin < n, strictly increasing within a hyperedge
 *              (so pins of a hyperedge are distinct), every |e| >= 2;
 *   w[m]       float32, finite and > 0 (NULL means all 1).
 * Nodes of degree 0 are allowed.
 */
#ifndef HYPEREF_H
#define HYPEREF_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HEF_OK = 0,
  HEF_ERR_INVALID_ARGUMENT = 1,   /* bad scalar or NULL pointer            */
  HEF_ERR_INVALID_HYPERGRAPH = 2, /* structure or weights violate layout   */
  HEF_ERR_WORKSPACE_TOO_SMALL = 3,
  HEF_ERR_DEVICE = 4,             /* a HIP runtime call failed             */
  HEF_ERR_NUMERICAL = 5,          /* every quadratic form vanished / NaN   */
  HEF_ERR_UNSUPPORTED = 6
} hef_status;

/* Storage type of the Krylov pool chi^(1..K). */
/* Pool storage.  HEF_BASIS_FP64 is a debug basis of hef_resistance and
 * hef_resistance_static only: the Krylov pool is stored in float64 (the
 * float32 Krylov blocks widened exactly), the joint Gram, R^-1 apply and the
 * resistance ratios run in float64, and chi is returned as float64; every
 * other entry point rejects it with HEF_ERR_UNSUPPORTED, and it takes
 * orth_passes = 1. */
typedef enum { HEF_BASIS_FP32 = 0, HEF_BASIS_BF16 = 1, HEF_BASIS_FP64 = 2 } hef_basis;

/* Which operation a workspace is sized for. */
typedef enum {
  HEF_OP_RESISTANCE = 0,
  HEF_OP_COARSEN = 1,
  HEF_OP_CLUSTER_LEVEL = 2,
  HEF_OP_BACKWARD = 3,
  HEF_OP_APPLY = 4,
  HEF_OP_CONDUCTANCE = 5, /* sized for n_clusters up to n; ignores params  */
  HEF_OP_REBUILD = 6,     /* hef_rebuild; ignores params                    */
  HEF_OP_RATING = 7       /* hef_rating; ignores params                     */
} hef_op;

/* Flags for hef_params.flags. */
#define HEF_FLAG_ASSUME_VALID 1u  /* skip the device validation (no sync)  */
#define HEF_FLAG_STAR_ONLY 2u     /* pool from the star expansion only     */
#define HEF_FLAG_CLIQUE_ONLY 4u   /* pool from the clique expansion only   */
#define HEF_FLAG_TAPED 8u         /* backward: the tape of a preceding
                                     hef_resistance_taped is in `ws`        */

typedef struct {
  int32_t n, m;          /* nodes, hyperedges                               */
  int64_t nnz;           /* pins; must equal eptr[m]                        */
  const int32_t *eptr;   /* DEVICE [m+1]                                    */
  const int32_t *pins;   /* DEVICE [nnz]                                    */
  const float *w;        /* DEVICE [m], or NULL for unit weights            */
} hef_hypergraph;

typedef struct {
  int32_t k;             /* Krylov steps per expansion (>= 1)               */
  int32_t b;             /* start vectors per expansion, 1..16              */
  int32_t levels;        /* coarsening levels for hef_coarsen (>= 1)        */
  float percentile;      /* merge threshold delta as a percentile of R, (0,1] */
  int32_t local_clustering; /* 0/1: attach isolated nodes (Alg. 2's local clustering) */
  int32_t basis;         /* hef_basis of the pool                           */
  uint64_t seed;         /* counter-generator seed for start blocks         */
  float drop_tol;        /* tau: relative Gram-Schmidt residual below which
                            a pool column is dropped (1e-3)                 */
  int32_t orth_passes;   /* joint Cholesky-QR passes, 1 or 2                */
  int32_t ckpt_every;    /* adjoint tape: 0 (default) or >= k keeps every
                            Krylov step of the forward, so the reverse sweep
                            recomputes nothing (about 8 (k-1)(2n+m)b bytes of
                            workspace); 1..k-1 keeps checkpoints every
                            ckpt_every steps and recomputes each segment    */
  uint32_t flags;        /* HEF_FLAG_*                                      */
  float target_nr;       /* node-reduction target of the level loop (Section
                            IV: NR = 60 % is a 2.5x reduction): with
                            target_nr > 0 coarsening stops before a level
                            once n_l <= (1 - target_nr) n_0, or after a level
                            that merged nothing; `levels` stays the cap.
                            0 = run exactly `levels` levels.  In [0, 1).   */
} hef_params;

/* Fills *p with the defaults: k=10, b=1, levels=1, percentile=0.5,
 * local_clustering=1, basis=FP32, seed=7, drop_tol=1e-3, orth_passes=1,
 * ckpt_every=0, flags=0, target_nr=0. */
void hef_params_default(hef_params *p);

/* Pool width K = 2*b*k (b*k with a single-expansion flag). */
int32_t hef_pool_width(const hef_params *p);

/* Bytes of workspace the operation `op` needs for this hypergraph and these
 * parameters.  Host only; reads no device memory.  The bound covers every
 * coarsening level, whose hypergraphs are never larger than level 0's. */
hef_status hef_workspace_size(const hef_hypergraph *hg, const hef_params *p,
                              int32_t op, size_t *bytes);

/* Validates a hypergraph held in HOST arrays against the layout above
 * (CPU only; no device needed).  Returns HEF_OK or
 * HEF_ERR_INVALID_HYPERGRAPH / HEF_ERR_INVALID_ARGUMENT. */
hef_status hef_validate_host(int32_t n, int32_t m, const int32_t *eptr,
                             const int32_t *pins, const float *w);

/* Alg. 1 (Section III-A, Eqs. (12)-(14)): per-hyperedge effective-resistance
 * estimates.  Builds the b-column block Krylov sequences of the normalised
 * star and clique adjacencies implicitly from the incidence, orthonormalises
 * them into a pool chi^(1..K) (star columns first, star-node entries only),
 * and returns R_e = max_i (max_{p in e} chi_p^(i) - min_{p in e} chi_p^(i))^2
 * / Q_H(chi^(i)) with Q_H of Eq. (9).
 *   start_star   DEVICE [(n+m) x b] float32 row-major start block of the star
 *                expansion (node rows first, then hyperedge rows), or NULL to
 *                draw it from the counter generator (seed, level 0, expansion 0);
 *   start_clique DEVICE [n x b] float32, or NULL (expansion 1);
 *   R            DEVICE [m] float32 output;
 *   qh           DEVICE [K] float64 output Q_H(chi^(i)), or NULL; a dropped
 *                column reports 0;
 *   chi          DEVICE [n x K] row-major output pool (float32, bfloat16 when
 *                basis = BF16, float64 when basis = FP64), or NULL; dropped
 *                columns are zero.
 * Unless HEF_FLAG_ASSUME_VALID is set, the results are checked on the device
 * (one more stream synchronisation) and HEF_ERR_NUMERICAL is returned if
 * every Q_H vanished or a value is not finite.  With HEF_FLAG_ASSUME_VALID
 * the call synchronises nothing and checks neither the input nor the
 * results: the caller vouches for both. */
hef_status hef_resistance(const hef_hypergraph *hg, const hef_params *p,
                          const float *start_star, const float *start_clique,
                          float *R, double *qh, void *chi,
                          void *ws, size_t ws_bytes, hipStream_t stream);

/* hef_resistance for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * It takes no workspace; its scratch is a static device array of
 * HEF_STATIC_SCRATCH_BYTES bytes that every device the library runs on holds
 * until the process ends, and the call itself calls no hipMalloc, hipFree or
 * allocating library routine.  Arguments, outputs, errors and results are
 * those of hef_resistance (bitwise identical for identical inputs); the
 * caller still provides every input and output.  A hypergraph whose
 * workspace (hef_workspace_size with HEF_OP_RESISTANCE, or with chi given,
 * that size less the n x K pool) exceeds HEF_STATIC_SCRATCH_BYTES returns
 * HEF_ERR_WORKSPACE_TOO_SMALL with nothing written.  All calls on one device
 * share that device's scratch, which keeps the last call's contents (every
 * call initialises what it reads): calls that overlap on one device -- on
 * two streams or from two threads -- race and give undefined results.  With
 * HEF_FLAG_ASSUME_VALID the call synchronises nothing and enqueues only
 * kernels and device-to-device copies (buffers are cleared by kernels, not
 * hipMemsetAsync), so it can be captured into a HIP graph; every replay
 * recomputes the result.  Make one call before capturing: the first call on
 * a device looks up the scratch array's address. */
#define HEF_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
hef_status hef_resistance_static(const hef_hypergraph *hg, const hef_params *p,
                                 const float *start_star, const float *start_clique, float *R,
                                 double *qh, void *chi, hipStream_t stream);

/* Alg. 2 (Section III-A "Multilevel Effective Resistance Clustering",
 * Eq. (15); Section III-B, Eq. (16)): `levels` rounds of resistance
 * estimation, Eq. (15) update, threshold contraction in ascending resistance
 * order, resistance-based local clustering of isolated nodes and coarse
 * rebuild.  Start blocks come from the counter generator.
 *   cluster     DEVICE [n] int32 output: original node -> final cluster label
 *               (labels are ranks of each cluster's smallest node id);
 *   n_clusters  HOST int32 output;
 *   R0          DEVICE [m] float32 output: level-0 resistances, or NULL;
 *   eta         DEVICE [n] float32 output: eta of each final cluster in
 *               entries [0, n_clusters), or NULL.
 * Synchronises `stream`. */
hef_status hef_coarsen(const hef_hypergraph *hg, const hef_params *p,
                       int32_t *cluster, int32_t *n_clusters, float *R0,
                       float *eta, void *ws, size_t ws_bytes, hipStream_t stream);

/* What hef_coarsen_levels records of every level l < cap it runs (any
 * pointer may be NULL; n0, m0 are the sizes of the input hypergraph and K
 * the pool width):
 *   n, m, nnz  HOST [cap]: sizes of level l's hypergraph (level 0 = input);
 *   R          DEVICE [cap x m0] float32: level l's resistances (Alg. 1, before
 *              Eq. (15)) at offset l*m0, first m_l entries;
 *   qh         DEVICE [cap x K] float64: level l's Q_H per pool column;
 *   rho        DEVICE [cap x K] float64: level l's relative Gram-Schmidt
 *              residuals |R_jj| / ||V_j|| of the joint orthonormalisation
 *              (Alg. 1's orthonormalisation; 0 for a dropped column); min over j is the
 *              pool's conditioning margin;
 *   label      DEVICE [cap x n0] int32: level-l node -> level-(l+1) node at
 *              offset l*n0, first n_l entries;
 *   eta        DEVICE [cap x n0] float32: eta of the level-(l+1) nodes (the
 *              clusters level l formed) at offset l*n0, first n_{l+1} entries;
 *   levels_run HOST output: the number of levels run. */
typedef struct {
  int32_t cap;
  int32_t levels_run;
  int32_t *n, *m;
  int64_t *nnz;
  float *R;
  double *qh;
  double *rho;
  int32_t *label;
  float *eta;
} hef_level_trace;

/* hef_coarsen with a per-level record (`trace` may be NULL): the level-l
 * resistances and eta serve the partitioner integration of Section III-E
 * (its Eq. (15) node weights and per-level ratings), and the per-level
 * labels compose to the final map. */
hef_status hef_coarsen_levels(const hef_hypergraph *hg, const hef_params *p, int32_t *cluster,
                              int32_t *n_clusters, float *R0, float *eta,
                              hef_level_trace *trace, void *ws, size_t ws_bytes,
                              hipStream_t stream);

/* Sizes (n, m, nnz; HOST arrays of `cap` entries, any may be NULL) of the
 * levels whose resistances the calling thread's last hef_coarsen call
 * estimated; returns the number of such levels. */
int32_t hef_last_coarsen_levels(int32_t *n, int32_t *m, int64_t *nnz, int32_t cap);

/* Work of the local clustering's best-neighbour search (Section III-B,
 * Eq. (16)) in the calling thread's last hef_coarsen call, per level (HOST
 * array of `cap` entries, may be NULL): the number of (isolated node,
 * candidate cluster) pairs it screened, one per co-pin occurrence of every
 * isolated node, i.e. sum over isolated p of sum_{e ∋ p} (|e| - 1); 0 for a
 * level without local clustering.  Counted on the device with integer sums;
 * returns the number of levels. */
int32_t hef_last_coarsen_work(int64_t *best_candidates, int32_t cap);

/* One level of Alg. 2 (steps 4-10) from GIVEN inputs, so that a caller can
 * feed the same resistances to two implementations:
 *   R        DEVICE [m] float32 resistances of this level;
 *   eta_in   DEVICE [n] float32 node weights eta (Eq. (15)), NULL = zeros;
 *   chi      DEVICE [n x K] pool, K = hef_pool_width(p): float32, or
 *            bfloat16 when p->basis = HEF_BASIS_BF16 (as hef_resistance
 *            writes it); with local clustering every value must be finite
 *            and below 65504 in magnitude (the best-neighbour screen keeps
 *            float16 copies), else HEF_ERR_INVALID_ARGUMENT;
 *   qh       DEVICE [K] float64 quadratic forms (<= 0 marks an unusable column);
 *   cluster  DEVICE [n] int32 output: node -> cluster label;
 *   n_clusters HOST int32 output;
 *   eta_out  DEVICE [n] float32 output, entries [0, n_clusters) valid.
 * Synchronises `stream`. */
hef_status hef_cluster_level(const hef_hypergraph *hg, const hef_params *p,
                             const float *R, const float *eta_in,
                             const float *chi, const double *qh,
                             int32_t *cluster, int32_t *n_clusters,
                             float *eta_out, void *ws, size_t ws_bytes,
                             hipStream_t stream);

/* Alg. 2's coarse hypergraph H' of a clustering: each pin p
 * becomes label[p], the labels of a hyperedge are sorted and deduplicated,
 * hyperedges left with fewer than 2 pins are removed, and the kept ones keep
 * their order and weight (w' = w).
 *   label      DEVICE [n] int32: node -> cluster in [0, n_clusters) (a pin
 *              whose label lies outside gives HEF_ERR_INVALID_ARGUMENT);
 *   eptr_out   DEVICE [m+1] int32, pins_out DEVICE [nnz] int32, w_out
 *              DEVICE [m] float32: H' in CSR (first m' + 1, nnz', m'
 *              entries written);
 *   kept_out   DEVICE [m] int32 or NULL: the input id of each kept hyperedge;
 *   m_out, nnz_out  HOST: m' and nnz';
 *   ws         DEVICE workspace of hef_workspace_size(hg, NULL, HEF_OP_REBUILD).
 * The hypergraph is validated on the device.  Synchronises `stream`. */
hef_status hef_rebuild(const hef_hypergraph *hg, const int32_t *label, int32_t n_clusters,
                       int32_t *eptr_out, int32_t *pins_out, float *w_out, int32_t *kept_out,
                       int32_t *m_out, int64_t *nnz_out, void *ws, size_t ws_bytes,
                       hipStream_t stream);

/* Resistance-based vertex-pair rating for multilevel partitioning
 * (Section III-E, Eq. (17); Alg. 3): for nodes p != q sharing
 * hyperedges,  r(p, q) = sum over the hyperedges e holding both of
 * w(e) / (R_e - shift), summed in float64 in ascending hyperedge order; a
 * hyperedge with R_e - shift == 0 adds nothing.  Eq. (17) prints the
 * denominator as R_e - 1, i.e. Eq. (7)'s cardinality term |e| - 1 with |e|
 * replaced by R_e; since R_e <= 1/w(e) that form is negative for every
 * hyperedge with w(e) >= 1 and rates heavy hyperedges lowest, against the
 * stated aim (heavy, low-resistance hyperedges).  shift = 0 replaces the
 * whole term |e| - 1 by R_e (heavy, low-resistance hyperedges rate high);
 * shift = 1 evaluates the printed form.  With R_e = |e| and shift = 1 this is
 * Eq. (7) itself.
 *   R       DEVICE [m] float32 resistances (finite, else
 *           HEF_ERR_INVALID_ARGUMENT), e.g. a level's Eq. (15) values;
 *   best    DEVICE [n] int32 output: the neighbour q of largest r(p, q), ties
 *           to the smallest q; -1 for a node without neighbours;
 *   rating  DEVICE [n] float64 output: r(p, best[p]) (0 without neighbours);
 *   ws      DEVICE workspace of hef_workspace_size(hg, NULL, HEF_OP_RATING).
 * Work and memory are proportional to sum_e |e| (|e| - 1).  The hypergraph is
 * validated on the device.  Synchronises `stream`. */
hef_status hef_rating(const hef_hypergraph *hg, const float *R, float shift, int32_t *best,
                      double *rating, void *ws, size_t ws_bytes, hipStream_t stream);

/* Cluster quality of a partition (Section II-A, Eq. (3); Section IV,
 * Eq. (18)).  With d_v the summed weight of v's hyperedges and vol(S) the
 * summed degree of S, a cluster S gets cut(S) = the summed weight of the
 * hyperedges with pins both in S and outside it (each counted once), and
 * phi(S) = cut(S) / min(vol(S), vol(V) - vol(S)), or 0 when cut(S) = 0.
 * phi_avg is the mean of phi over the n_clusters clusters.  All in float64,
 * deterministic (fixed summation order, no atomics).
 *   label      DEVICE [n] int32: node -> cluster in [0, n_clusters) (a label
 *              outside on a pin gives HEF_ERR_INVALID_ARGUMENT after the run;
 *              nodes without hyperedges add nothing and are not read);
 *   n_clusters 1 <= n_clusters <= max(n, 1); clusters without nodes get 0s;
 *   cut, vol, phi  DEVICE [n_clusters] float64 outputs;
 *   phi_avg    DEVICE [1] float64 output;
 *   ws         DEVICE workspace of hef_workspace_size(hg, NULL,
 *              HEF_OP_CONDUCTANCE, .) bytes.
 * The hypergraph is validated on the device.  Synchronises `stream`. */
hef_status hef_conductance(const hef_hypergraph *hg, const int32_t *label, int32_t n_clusters,
                           double *cut, double *vol, double *phi, double *phi_avg, void *ws,
                           size_t ws_bytes, hipStream_t stream);

/* Adjoint of hef_resistance with respect to the hyperedge weights (the
 * derivative of Eqs. (9), (13), (14) through the Krylov bases of
 * Section III-B, serving the resistance-based hyperedge weighting of
 * Section I): given dR = dL/dR (DEVICE [m] float32), writes dw = dL/dw
 * (DEVICE [m] float32).  Unless p->flags has HEF_FLAG_TAPED it first
 * recomputes the forward pass with the same start blocks (which must be the
 * ones the forward used; NULL = counter generator), keeping the Krylov
 * tape p->ckpt_every asks for; with HEF_FLAG_TAPED it uses the
 * tape that hef_resistance_taped left in `ws` (same hypergraph, params and
 * workspace, untouched in between).  Ties in a maximum take the lowest
 * column index and the lowest CSR position.  The derivative is that of the
 * FP32-pool computation (a BF16 request differentiates the FP32 path);
 * orth_passes must be 1 (else HEF_ERR_UNSUPPORTED).  Workspace:
 * hef_workspace_size(..., HEF_OP_BACKWARD, ...). */
hef_status hef_resistance_backward(const hef_hypergraph *hg, const hef_params *p,
                                   const float *start_star, const float *start_clique,
                                   const float *dR, float *dw,
                                   void *ws, size_t ws_bytes, hipStream_t stream);

/* The forward pass of hef_resistance (FP32 pool) writing R (DEVICE [m]
 * float32) and keeping in `ws` (sized for HEF_OP_BACKWARD) the tape that a
 * following hef_resistance_backward with HEF_FLAG_TAPED reverses, so that
 * forward + backward costs one forward and one reverse sweep. */
hef_status hef_resistance_taped(const hef_hypergraph *hg, const hef_params *p,
                                const float *start_star, const float *start_clique, float *R,
                                void *ws, size_t ws_bytes, hipStream_t stream);

/* Test hook: y = A x for one normalised expansion adjacency
 * (expansion 0 = star, x and y DEVICE [(n+m) x b]; 1 = clique, [n x b]),
 * row-major float32, b in 1..16. */
hef_status hef_debug_apply(const hef_hypergraph *hg, int32_t expansion, int32_t b,
                           const float *x, float *y, void *ws, size_t ws_bytes,
                           hipStream_t stream);

/* Test hook: G = X^T X (DEVICE [cols x cols] float64 output, row-major) of a
 * DEVICE [rows x cols] row-major float32 matrix X (cols <= 512), through the
 * matrix-core Gram kernels of the joint orthonormalisation.  The workspace
 * must hold hef_debug_gram_ws(rows, cols) bytes. */
hef_status hef_debug_gram(const float *X, int64_t rows, int32_t cols, double *G,
                          void *ws, size_t ws_bytes, hipStream_t stream);
size_t hef_debug_gram_ws(int64_t rows, int32_t cols);

/* The counter generator of the start blocks on the device: writes the
 * rows x b float32 block for (seed, level, expansion) to DEVICE `out`
 * (element (r, c) is element r*b + c of the stream). */
hef_status hef_start_block(uint64_t seed, int32_t level, int32_t expansion,
                           int64_t rows, int32_t b, float *out, hipStream_t stream);

const char *hef_status_string(hef_status s);
const char *hef_last_error(void);

/* Profiling aid.  While enabled (process-wide), every stage of the calls
 * above records a pair of HIP events on its launch stream around its
 * kernels.  hef_timing_read() waits for the recorded events, adds their
 * elapsed times to per-stage totals, copies the totals (milliseconds) and
 * launch counts of the first `nstages` stages to the HOST arrays `ms` and
 * `counts` (either may be NULL), and clears them if `reset` is non-zero.
 * Stage names come from hef_timing_stage_name(0 .. count-1).
 * hef_timing_stages(mask) limits the event pairs to the stages whose bit is
 * set (bit i for stage i), so that a timed run pays for the events of the
 * stages it measures only.  Until it is called every stage is timed except
 * "spmm_step", one span over the fused SpMM's three kernels (which the
 * stages spmm_prep, spmm_csr and spmm_csc also cover). */
void hef_timing_enable(int32_t on);
void hef_timing_stages(uint32_t mask);
int32_t hef_timing_stage_count(void);
const char *hef_timing_stage_name(int32_t stage);
hef_status hef_timing_read(double *ms, int64_t *counts, int32_t nstages, int32_t reset);

#ifdef __cplusplus
}
#endif
#endif /* HYPEREF_H */

// Host-side checks of the C ABI under AddressSanitizer and UBSan (no GPU):
// the host validator, workspace planning for every operation, parameter
// checks, and the argument errors every entry point returns before it
// touches the device.  Prints one line per check; exits non-zero on a
// wrong status.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "hyperef.h"

static int failures = 0;

static void expect(const char *what, int got, int want) {
  std::printf("%-58s %d%s\n", what, got, got == want ? "" : "  <-- unexpected");
  if (got != want) ++failures;
}

int main() {
  // ---- host validator
  std::vector<int32_t> eptr = {0, 2, 5}, pins = {0, 3, 1, 2, 4};
  std::vector<float> w = {1.0f, 2.0f};
  expect("validate: valid", hef_validate_host(5, 2, eptr.data(), pins.data(), w.data()), HEF_OK);
  expect("validate: unit weights", hef_validate_host(5, 2, eptr.data(), pins.data(), nullptr), HEF_OK);
  expect("validate: empty", hef_validate_host(0, 0, eptr.data(), nullptr, nullptr), HEF_OK);
  {
    auto p = pins; p[1] = 7;
    expect("validate: pin out of range", hef_validate_host(5, 2, eptr.data(), p.data(), w.data()),
           HEF_ERR_INVALID_HYPERGRAPH);
    p = pins; p[1] = 0;
    expect("validate: repeated pin", hef_validate_host(5, 2, eptr.data(), p.data(), w.data()),
           HEF_ERR_INVALID_HYPERGRAPH);
    p = pins; std::swap(p[2], p[3]);
    expect("validate: unsorted pins", hef_validate_host(5, 2, eptr.data(), p.data(), w.data()),
           HEF_ERR_INVALID_HYPERGRAPH);
    std::vector<int32_t> e1 = {0, 1, 5};
    expect("validate: |e| < 2", hef_validate_host(5, 2, e1.data(), pins.data(), w.data()),
           HEF_ERR_INVALID_HYPERGRAPH);
    std::vector<int32_t> e2 = {1, 2, 5};
    expect("validate: eptr[0] != 0", hef_validate_host(5, 2, e2.data(), pins.data(), w.data()),
           HEF_ERR_INVALID_HYPERGRAPH);
    auto ww = w; ww[1] = -1.0f;
    expect("validate: negative weight", hef_validate_host(5, 2, eptr.data(), pins.data(), ww.data()),
           HEF_ERR_INVALID_HYPERGRAPH);
    ww[1] = std::nanf("");
    expect("validate: NaN weight", hef_validate_host(5, 2, eptr.data(), pins.data(), ww.data()),
           HEF_ERR_INVALID_HYPERGRAPH);
    expect("validate: NULL eptr", hef_validate_host(5, 2, nullptr, pins.data(), w.data()),
           HEF_ERR_INVALID_ARGUMENT);
    expect("validate: NULL pins", hef_validate_host(5, 2, eptr.data(), nullptr, w.data()),
           HEF_ERR_INVALID_ARGUMENT);
    expect("validate: negative size", hef_validate_host(-1, 2, eptr.data(), pins.data(), w.data()),
           HEF_ERR_INVALID_ARGUMENT);
  }
  // ---- parameters and workspace planning (host only)
  hef_params p;
  hef_params_default(&p);
  p.k = 30; p.b = 8; p.levels = 3;
  expect("pool width 2 b k", hef_pool_width(&p), 480);
  hef_hypergraph big{2000000, 2200000, 7907430, (const int32_t *)8, (const int32_t *)8, nullptr};
  hef_hypergraph none{0, 0, 0, (const int32_t *)8, nullptr, nullptr};
  for (int op = 0; op < 8; ++op) {
    size_t b1 = 0, b0 = 0;
    char name[64];
    std::snprintf(name, sizeof(name), "workspace op %d at 2M nodes (status)", op);
    expect(name, hef_workspace_size(&big, &p, op, &b1), HEF_OK);
    std::snprintf(name, sizeof(name), "workspace op %d empty (status)", op);
    expect(name, hef_workspace_size(&none, &p, op, &b0), HEF_OK);
    std::snprintf(name, sizeof(name), "workspace op %d grows with the input", op);
    expect(name, b1 > b0, 1);
  }
  {
    size_t b = 0;
    expect("workspace: unknown op", hef_workspace_size(&big, &p, 99, &b), HEF_ERR_INVALID_ARGUMENT);
    expect("workspace: NULL out", hef_workspace_size(&big, &p, 0, nullptr), HEF_ERR_INVALID_ARGUMENT);
    hef_hypergraph huge = big;
    huge.nnz = int64_t(1) << 32;
    expect("workspace: nnz beyond int32", hef_workspace_size(&huge, &p, 0, &b), HEF_ERR_UNSUPPORTED);
    hef_hypergraph neg = big;
    neg.n = -5;
    expect("workspace: negative n", hef_workspace_size(&neg, &p, 0, &b), HEF_ERR_INVALID_ARGUMENT);
    struct Bad { const char *what; void (*set)(hef_params &); int want; } bad[] = {
        {"params: k = 0", [](hef_params &q) { q.k = 0; }, HEF_ERR_INVALID_ARGUMENT},
        {"params: b = 3", [](hef_params &q) { q.b = 3; }, HEF_ERR_UNSUPPORTED},
        {"params: pool width 544", [](hef_params &q) { q.b = 16; q.k = 17; }, HEF_ERR_UNSUPPORTED},
        {"params: basis 7", [](hef_params &q) { q.basis = 7; }, HEF_ERR_INVALID_ARGUMENT},
        {"params: drop_tol 1", [](hef_params &q) { q.drop_tol = 1.0f; }, HEF_ERR_INVALID_ARGUMENT},
        {"params: orth_passes 3", [](hef_params &q) { q.orth_passes = 3; }, HEF_ERR_INVALID_ARGUMENT},
        {"params: star and clique only", [](hef_params &q) { q.flags = HEF_FLAG_STAR_ONLY | HEF_FLAG_CLIQUE_ONLY; }, HEF_ERR_INVALID_ARGUMENT},
        {"params: levels 0 (coarsen)", [](hef_params &q) { q.levels = 0; }, HEF_ERR_INVALID_ARGUMENT},
        {"params: percentile 0 (coarsen)", [](hef_params &q) { q.percentile = 0.0f; }, HEF_ERR_INVALID_ARGUMENT},
        {"params: target_nr 1 (coarsen)", [](hef_params &q) { q.target_nr = 1.0f; }, HEF_ERR_INVALID_ARGUMENT},
        {"params: target_nr NaN (coarsen)", [](hef_params &q) { q.target_nr = std::nanf(""); }, HEF_ERR_INVALID_ARGUMENT},
    };
    for (const Bad &c : bad) {
      hef_params q = p;
      c.set(q);
      expect(c.what, hef_workspace_size(&big, &q, HEF_OP_COARSEN, &b), c.want);
    }
    // the float64 basis: Alg. 1 only, one orthonormalisation pass
    hef_params f = p;
    f.basis = HEF_BASIS_FP64;
    expect("params: fp64 basis (resistance)", hef_workspace_size(&big, &f, HEF_OP_RESISTANCE, &b), HEF_OK);
    expect("params: fp64 basis (coarsen)", hef_workspace_size(&big, &f, HEF_OP_COARSEN, &b), HEF_ERR_UNSUPPORTED);
    expect("params: fp64 basis (backward)", hef_workspace_size(&big, &f, HEF_OP_BACKWARD, &b), HEF_ERR_UNSUPPORTED);
    f.orth_passes = 2;
    expect("params: fp64 basis, two passes", hef_workspace_size(&big, &f, HEF_OP_RESISTANCE, &b), HEF_ERR_UNSUPPORTED);
  }
  // ---- argument errors returned before any device work
  float R[2];
  double qh[480];
  int32_t lab[8], nc = 0, m2 = 0;
  int64_t nnz2 = 0;
  char ws[256];
  expect("resistance: NULL hypergraph",
         hef_resistance(nullptr, &p, nullptr, nullptr, R, qh, nullptr, ws, sizeof(ws), nullptr),
         HEF_ERR_INVALID_ARGUMENT);
  expect("resistance: NULL params",
         hef_resistance(&big, nullptr, nullptr, nullptr, R, qh, nullptr, ws, sizeof(ws), nullptr),
         HEF_ERR_INVALID_ARGUMENT);
  expect("resistance: workspace too small",
         hef_resistance(&big, &p, nullptr, nullptr, R, qh, nullptr, ws, sizeof(ws), nullptr),
         HEF_ERR_WORKSPACE_TOO_SMALL);
  expect("resistance_static: beyond the static scratch",
         hef_resistance_static(&big, &p, nullptr, nullptr, R, qh, nullptr, nullptr),
         HEF_ERR_WORKSPACE_TOO_SMALL);
  expect("coarsen: NULL count",
         hef_coarsen(&big, &p, lab, nullptr, nullptr, nullptr, ws, sizeof(ws), nullptr),
         HEF_ERR_INVALID_ARGUMENT);
  expect("coarsen: workspace too small",
         hef_coarsen(&big, &p, lab, &nc, nullptr, nullptr, ws, sizeof(ws), nullptr),
         HEF_ERR_WORKSPACE_TOO_SMALL);
  hef_level_trace tr;
  std::memset(&tr, 0, sizeof(tr));
  tr.cap = -1;
  expect("coarsen_levels: negative trace capacity",
         hef_coarsen_levels(&big, &p, lab, &nc, nullptr, nullptr, &tr, ws, sizeof(ws), nullptr),
         HEF_ERR_INVALID_ARGUMENT);
  expect("cluster_level: workspace too small",
         hef_cluster_level(&big, &p, R, nullptr, R, qh, lab, &nc, R, ws, sizeof(ws), nullptr),
         HEF_ERR_WORKSPACE_TOO_SMALL);
  expect("rebuild: NULL outputs",
         hef_rebuild(&big, lab, 4, nullptr, nullptr, nullptr, nullptr, &m2, &nnz2, ws, sizeof(ws), nullptr),
         HEF_ERR_INVALID_ARGUMENT);
  expect("rebuild: n_clusters above n",
         hef_rebuild(&big, lab, 2000001, lab, lab, R, nullptr, &m2, &nnz2, ws, sizeof(ws), nullptr),
         HEF_ERR_INVALID_ARGUMENT);
  expect("rating: NULL outputs",
         hef_rating(&big, R, 0.0f, nullptr, nullptr, ws, sizeof(ws), nullptr), HEF_ERR_INVALID_ARGUMENT);
  expect("rating: infinite shift",
         hef_rating(&big, R, INFINITY, lab, qh, ws, sizeof(ws), nullptr), HEF_ERR_INVALID_ARGUMENT);
  expect("rating: workspace too small",
         hef_rating(&big, R, 0.0f, lab, qh, ws, sizeof(ws), nullptr), HEF_ERR_WORKSPACE_TOO_SMALL);
  expect("conductance: NULL label",
         hef_conductance(&big, nullptr, 3, qh, qh, qh, qh, ws, sizeof(ws), nullptr),
         HEF_ERR_INVALID_ARGUMENT);
  expect("backward: workspace too small",
         hef_resistance_backward(&big, &p, nullptr, nullptr, R, R, ws, sizeof(ws), nullptr),
         HEF_ERR_WORKSPACE_TOO_SMALL);
  expect("debug_apply: b = 3",
         hef_debug_apply(&big, 0, 3, R, R, ws, sizeof(ws), nullptr), HEF_ERR_UNSUPPORTED);
  expect("debug_gram: 600 columns", hef_debug_gram(R, 10, 600, qh, ws, sizeof(ws), nullptr),
         HEF_ERR_INVALID_ARGUMENT);
  for (int s = 0; s <= 7; ++s) std::printf("status %d: %s\n", s, hef_status_string(hef_status(s)));
  std::printf("last error: %s\n", hef_last_error());
  std::printf("%d unexpected\n", failures);
  return failures == 0 ? 0 : 1;
}

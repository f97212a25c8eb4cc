"""Plain FP64 CPU oracle for HyperEF 2.0's resistance estimate and coarsening.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls or links
this package; only the tests, the smoke check and the benchmark's CPU-baseline
leg do.  It shares no code with the HIP library and is written to be checked
against the paper by eye: every function cites the passage it follows, and
there is no blocking, fusion or reordering beyond what that passage states.

Modules:
  resistance  -- Alg. 1: expansions, Krylov pools, orthonormalisation,
                 resistance ratios (Eqs. (9), (12)-(14)).
  clustering  -- Alg. 2: Eq. (15) update, threshold contraction, resistance-
                 based local clustering (Eq. (16)), coarse rebuild.
  gradient    -- derivative of sum_e c_e R_e with respect to hyperedge weights,
                 by float64 autograd through the same definitions.
  exact       -- exact quantities the estimate is pinned against: pseudo-
                 inverse resistances and the convex program of Eq. (8).

Parity status: every function here is pinned by a CPU test except the
estimate's quality against the exact R* at large n and the cluster quality
(conductance, cut), which are "parity unpinned" -- the paper's own numbers
for them need the ISPD98 netlists.
"""
from . import resistance  # noqa: F401

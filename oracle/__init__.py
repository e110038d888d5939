"""FP64 CPU oracle for the biasing-force path of PySAGES (arXiv 2301.04835).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this
package.  It shares no code with the HIP implementation in
``paper_2301_04835_amd`` and never imports it; the two meet only through the
seeded input generators, which hold none of the method's arithmetic.

The heavy primitives (dihedral, radius of gyration, coordination number,
Gaussian hill sums, the well-tempered height sequence) are plain C in
``oracle.c`` (FP64, sequential sums, no fast-math).  The composition of a
biasing step (chain rule, ABF bookkeeping, the surrogate network) is plain
NumPy in FP64 in the submodules.  Each function cites the passage of the
paper it follows.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants, finite differences or brute force; none is
"parity unpinned".
"""
from ._clib import (  # noqa: F401
    KB,
    coordination,
    dihedral,
    gyration,
    hillsum,
    hillsum_batch,
    switch,
    wt_height,
    wt_sequence,
)
from .methods import (  # noqa: F401
    TWO_PI,
    AbfGrid,
    abf_bin,
    abf_step,
    abf_step_momentum,
    abf_momentum_wp,
    abf_theta,
    cv_eval,
    cv_periods,
    metad_step,
    chain_rule,
)

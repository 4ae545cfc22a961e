"""Plain CPU FP64 oracle of the TLR quasi-Monte Carlo estimator.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import or run anything in this package;
the library (the HIP path and its host setup) never does, and this package
imports nothing from the library.

It computes, slowly and plainly, what the paper defines:

* the separation-of-variables (SOV) integrand of an MVN probability
  (Section 2.1, Eq. 2 and Algorithm "QMC for MVN probabilities"), one dense
  row product per variable, in log space;
* the Student-t probability as a chi scale mixture of MVN probabilities
  (Section 2.2, Eq. 4 and the "mvt" algorithm based on it);
* the tile-low-rank factor as input (Section 3.4, TLR QMC algorithms): the
  oracle expands it to dense rows, since the TLR recursion computes the same
  row sums re-associated;
* the Richtmyer lattice with random shifts (Section 2.1, the remark after
  the MVN algorithm) and the estimate with its standard error (Section 4,
  last paragraph: relative error = standard error / mean);
* block reordering by univariate conditioning (Section 3.3, "Block
  reordering" algorithm), and the factor by dense Cholesky plus per-tile
  truncation (Section 3.3: fixed absolute truncation of the TLR tiles).

Readings of passages where the paper is silent or garbled are listed in the
module that takes them.  Every function is pinned by tests in
``tests/test_oracle_*.py``; none is "parity unpinned".
"""

from . import lattice, special, sov, estimate, factor, reorder, skewnormal  # noqa: F401
from .api import sample_logp, probability  # noqa: F401

"""MI355X-native tile-low-rank quasi-Monte Carlo estimator of MVN / MVT probabilities.

The estimator runs in HIP kernels behind the C ABI of include/tlrqmc.h
(libtlrqmc.so, built by ``python -m paper_2003_11183_amd.build``); the
``tlrqmc`` module is its ctypes binding.
"""

from . import tlrqmc  # noqa: F401
from .tlrqmc import (  # noqa: F401
    Context, Factor, TLRQMCError, block_reorder, geometric_order, mvn_prob, mvt_prob, probability,
    sample_logp,
)

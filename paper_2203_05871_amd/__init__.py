"""MI355X-native MPO-TEBD step for the Lindblad master equation of qubit chains
(Landa & Misguich, arXiv:2203.05871).  The compute path is the HIP library
liblmpo.so behind the C ABI in include/lmpo.h; `lmpo.Chain` is its binding."""
from .lmpo import (Batch, Chain, Gradient, LmpoError, arena_bytes, expectation,  # noqa: F401
                   expectation_series, load_library, osee, renyi2)

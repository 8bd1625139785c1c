"""FP64 CPU oracle of the 2-D lattice Boltzmann hot path (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The HIP library never does.
"""
from .oracle import Oracle, build, BUDGET_NAMES  # noqa: F401

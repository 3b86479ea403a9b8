"""FP64 CPU oracle of the Shan-Chen foam step with the film barrier (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the GPU library.
"""
from .oracle import OracleSim, p0, splitmix64, uniform, lattice, match_labels  # noqa: F401

"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only *describes* inputs: random grid circuits of the kind the
paper verifies (single-qubit sqrt(X)/sqrt(Y)/sqrt(W) layers plus fSim couplers
in an ABCD tiling, section "Verification of Google's experiment") and seeded
bitstring batches.  It holds none of the contraction method's arithmetic:
nothing here builds tensors, contracts, or reduces amplitudes.
"""

from .circuits import (  # noqa: F401
    Circuit,
    grid_circuit,
    worked_example_circuit,
    CONFIGS,
    config_circuit,
    batch_spec,
    batch_circuit,
)
from .bitstrings import (  # noqa: F401
    uniform_bitstrings,
    prefix_bitstrings,
    config_bitstrings,
    bits_to_str,
)

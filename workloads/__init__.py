"""Seeded synthetic workloads for the FGIM merge path.

This package generates inputs only: base vectors, queries and the pre-built
input proximity graphs that the merge consumes.  It holds none of the merge
method's arithmetic and is shared by the oracle-side tests and the GPU path's
tests and benchmark, which is the only code the two sides share.
"""

from .configs import CONFIGS, WorkloadConfig, get_config  # noqa: F401
from .synth import make_vectors, make_queries, split_sizes  # noqa: F401
from .input_pg import build_input_pg, InputPG, reach_fraction  # noqa: F401

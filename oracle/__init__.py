"""FP64 CPU oracle for the PEPS-VMC hot path.

Test infrastructure: only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it.  The product path never does.
"""
from .peps_oracle import *  # noqa: F401,F403

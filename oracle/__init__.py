"""FP64 CPU oracle for the decorated-particle Vlasov-Poisson cycle.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU-baseline leg
may import this package.  The HIP product path never imports, links or runs it.
"""
from .vp_oracle import *  # noqa: F401,F403
from .vp_oracle import __all__  # noqa: F401

"""FP64 CPU oracle for the decorated-particle Vlasov-Poisson cycle and its initialisation.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU-baseline leg
may import this package.  The HIP product path never imports, links or runs it.
"""
from .vp_oracle import *  # noqa: F401,F403
from .vp_oracle import __all__ as _cycle_all
from .cluster_oracle import *  # noqa: F401,F403
from .cluster_oracle import __all__ as _cluster_all
from .k3_oracle import *  # noqa: F401,F403
from .k3_oracle import __all__ as _k3_all

__all__ = list(_cycle_all) + list(_cluster_all) + list(_k3_all)

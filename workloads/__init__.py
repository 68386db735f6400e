"""Seeded synthetic inputs shared by the tests, the benchmark and the examples.

Holds input generation only (lattice initial states and workload presets); none of the
per-step method arithmetic lives here.
"""
from .lattice import (make_lattice, landau_profile, two_stream_profile,  # noqa: F401
                      bump_on_tail_profile, cast_state)
from .configs import (Workload, landau_linear, two_stream, landau_nonlinear,  # noqa: F401
                      landau_sweep, served_jobs, landau_strong, random_markers)

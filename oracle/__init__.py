"""FP64 CPU oracle for IFNSO (test infrastructure only).

This package is the reference against which the GPU library is checked. Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import it;
the library itself never does, and this package imports nothing from the library.
"""
from .ifnso import *  # noqa: F401,F403
from .coeffs import *  # noqa: F401,F403
from .mlp import *  # noqa: F401,F403
from . import fp8  # noqa: F401
from .muon import *  # noqa: F401,F403
from . import baselines  # noqa: F401

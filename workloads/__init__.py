"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package generates matrices only. It holds none of the orthogonalisation
arithmetic: neither the oracle nor the HIP path is imported here, and both
consume the bytes produced by these generators.
"""
from .gen import *  # noqa: F401,F403
from .configs import *  # noqa: F401,F403
from .spectra import *  # noqa: F401,F403

"""FP64 CPU oracle of the range-only tracking environment.

TEST INFRASTRUCTURE ONLY: loaded by the test suite, the package smoke check and
the benchmark's CPU-baseline leg, never by the product path.
"""
from .oracle import *  # noqa: F401,F403

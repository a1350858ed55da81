"""CPU oracle for fragment-history volumes.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark. The product path never imports it.
"""
from .oracle import *  # noqa: F401,F403

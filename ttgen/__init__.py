"""Seeded synthetic inputs shared by the tests and the benchmark.

Holds only random-number generation and workload shapes; no contraction
arithmetic lives here.
"""
from . import rng, configs  # noqa: F401

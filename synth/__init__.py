"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

Holds only random-number generation and parameter screening; no step arithmetic.
"""
from .philox import philox4x32, u24, u53, action_value  # noqa: F401
from .workloads import *  # noqa: F401,F403

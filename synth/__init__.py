"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package draws random numbers and assembles inputs; it holds none of the
tracking method's arithmetic (no orbit propagation, light time, projection,
matched filter or stacking).  Geometry that needs the method -- where each
exposure points and where an injected source lands -- is read from the
stored workload files under ``tests/golden/`` that the oracle wrote.
"""
from .gen import *  # noqa: F401,F403

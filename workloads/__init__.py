"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only draws random fields and lays them out; it holds none of the
radiative-transfer arithmetic (no opacity law, no tree, no rays).
"""
from .synth import *  # noqa: F401,F403

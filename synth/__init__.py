"""Seeded synthetic VELO-like events and their generator truth.

This package is input infrastructure shared by the tests and the benchmark.
It simulates particles crossing a planar pixel detector and emits packed
raw pixel words; it holds none of the reconstruction arithmetic (no
clustering, no track finding, no fitting).
"""
from .gen import CONFIGS, EventBatch, generate, make_config  # noqa: F401

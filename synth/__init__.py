"""Seeded synthetic tight-binding inputs shared by the tests, the benchmark and
the oracle's golden-value scripts.

This module only draws random matrices and lays them out as CSR; it performs
none of the density-matrix arithmetic, so neither the GPU library nor the
oracle depends on the other through it.
"""
from .lattice import lattice, with_long_tail, CONFIGS, BETA, KT_EV, config_system  # noqa: F401

"""Seeded synthetic workloads shared by the oracle and the HIP path.

This package holds configuration records and random draws only: lattice
sites, charges, vacancies and the sketch matrix.  It performs none of the
arithmetic of the ACP method or of the physical model; both the CPU oracle and
the GPU workload builder consume what it returns.
"""
from .seeds import Config, CONFIGS, get_config, draw_sites, draw_sketch, small_config  # noqa: F401

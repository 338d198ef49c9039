"""Seeded synthetic workloads for the VQ-NQS local-energy path.

This package holds only data: the model/lattice configurations, the flat
parameter layout (names and shapes, in storage order) and the seeded
generators for spin configurations and parameter buffers.  It contains none
of the method's arithmetic, so both the CPU oracle and the GPU tests/bench can
draw their inputs from it without sharing any computation.
"""
from .configs import (ModelConfig, CONFIGS, MULTI_LATTICE, config_by_name,
                      with_batch)
from .layout import param_layout, param_count
from .generate import make_spins, make_params, scale_codebooks, bf16_round

__all__ = ["ModelConfig", "CONFIGS", "MULTI_LATTICE", "config_by_name",
           "with_batch", "param_layout", "param_count", "make_spins",
           "make_params", "scale_codebooks", "bf16_round"]

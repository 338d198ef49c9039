"""VQ-NQS local energy on MI355X: Python binding of libvqnqs.so.

Argument marshalling only: every step of the computation runs in the HIP
library (see include/vqnqs.h for the contract).  PyTorch supplies device
memory and the current stream.  Importing this package does not load the
library; the first call does, and fails loudly if it has not been built.
"""
from .api import (Config, PLAIN, DEDUP, F64, F32, BF16, FLAG_CERTIFIED_VQ,
                  NCOUNTERS, CTR, VQNQSError, library_path, load_library,
                  exported_symbols, param_count, workspace_size, neighbours,
                  forward_logpsi, local_energy, grad_logpsi, logpsi,
                  make_config, profile_enable, profile_reset, profile_read,
                  WS_FORWARD, WS_GRAD, MULTI_CONCURRENT, MULTI_GRAPH,
                  local_energy_multi, workspace_size_multi, autotune,
                  set_tuning, local_energy_static, STATIC_SCRATCH_BYTES,
                  forward_activations, probe_exp_rate, probe_gelu, sample,
                  WS_SAMPLE,
                  vmc_step, WS_VMC, n_sites, n_tokens)

__all__ = ["Config", "PLAIN", "DEDUP", "F64", "F32", "BF16",
           "FLAG_CERTIFIED_VQ", "NCOUNTERS", "CTR", "VQNQSError",
           "library_path", "load_library", "exported_symbols", "param_count",
           "workspace_size", "neighbours", "forward_logpsi", "local_energy",
           "grad_logpsi", "logpsi", "make_config", "profile_enable",
           "profile_reset", "profile_read", "WS_FORWARD", "WS_GRAD",
           "MULTI_CONCURRENT", "MULTI_GRAPH", "local_energy_multi",
           "workspace_size_multi", "autotune", "set_tuning",
           "local_energy_static", "STATIC_SCRATCH_BYTES",
           "forward_activations", "probe_exp_rate", "probe_gelu", "sample",
           "WS_SAMPLE",
           "vmc_step", "WS_VMC", "n_sites", "n_tokens"]

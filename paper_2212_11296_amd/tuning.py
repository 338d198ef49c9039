"""Persistent cache of the autotuner's launch choices, as JSON.

vqnqs_autotune times the rows-per-wave variants of the matrix-core products
and keeps the fastest for the process; the library keys its choices by the
model width d and the quantizer segment width d/H.  This module stores
them per device name and key in a JSON file, so a later process sets them
with vqnqs_set_tuning instead of timing again:

    {"<device>|d=<d>|seg=<d/H>": {"qkv_mb": 1, "mlp_mb": 2, "vq_mb": 2}, ...}
"""
import json
import os

from . import api

DEFAULT_PATH = os.path.join(os.path.expanduser("~"), ".cache",
                            "vqnqs_tuning.json")


def cache_key(cfg, device_name):
    return f"{device_name}|d={cfg.d_model}|seg={cfg.d_model // cfg.vq_heads}"


def load(path):
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return {}
    return data if isinstance(data, dict) else {}


def save(path, data):
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune_cached(cfg, params, spins, path=DEFAULT_PATH, mode=api.DEDUP,
                    ws=None, device_name=None):
    """Launch choices [qkv, mlp, vq] for this model: from the cache file
    when it holds them for this device (set in the library with
    vqnqs_set_tuning), else timed by vqnqs_autotune and written to the
    file.  Returns (choices, True if they came from the cache)."""
    if device_name is None:
        import torch
        device_name = torch.cuda.get_device_name(0)
    key = cache_key(cfg, device_name)
    data = load(path)
    ent = data.get(key)
    if ent is not None:
        choices = [int(ent["qkv_mb"]), int(ent["mlp_mb"]), int(ent["vq_mb"])]
        api.set_tuning(cfg, choices)
        return choices, True
    choices = api.autotune(cfg, params, spins, mode, ws=ws)
    data[key] = {"qkv_mb": choices[0], "mlp_mb": choices[1],
                 "vq_mb": choices[2]}
    save(path, data)
    return choices, False

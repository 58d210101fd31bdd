"""Cached autotuning of the engine's launch choices.

The search itself runs in the library (nf_autotune: device-timed sweeps of
work-item size, fold workgroup size, bin-stage threads, and for batched
launches the fit tile of the batched fold and its bin-stage threads). This module keys
its result by model, event counts, precision mode and device, stores it in a
JSON file, and applies a stored choice to new engines without re-timing.
"""
from __future__ import annotations

import hashlib
import json
import os

OPTIONS = ("chunk", "fold_block", "tail_threads", "batch_threads", "batch_fit_tile")


def default_cache_path():
    return os.path.join(os.path.expanduser("~"), ".cache", "nufold", "autotune.json")


def device_name():
    import torch
    p = torch.cuda.get_device_properties(0)
    return f"{p.name}/{getattr(p, 'gcnArchName', '')}/{p.multi_processor_count}"


def tuning_key(desc, event_counts, mode, device, batch=0):
    h = hashlib.sha256()
    h.update(json.dumps(desc, sort_keys=True).encode())
    h.update(json.dumps([int(n) for n in event_counts]).encode())
    h.update(f"{mode}|{device}|{int(batch)}".encode())
    return h.hexdigest()[:24]


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(engine, desc, event_counts, theta, cache_path=None, evals=50, batch=0, force=False):
    """Apply the cached choice for this (model, events, mode, device) or run
    the library's autotuner and cache its choice. Returns the record."""
    path = cache_path or default_cache_path()
    mode = "m64" if engine.mode == 0 else "m32"
    key = tuning_key(desc, event_counts, mode, device_name(), batch)
    cache = _load(path)
    rec = cache.get(key)
    if rec is not None and not force:
        for k in OPTIONS:
            if k in rec["options"]:
                engine.set_option(k, rec["options"][k])
        return dict(rec, cached=True)
    options, (us, us_batch) = engine.autotune(theta, evals=evals, batch=batch)
    rec = dict(options=options, us_per_eval=us, us_per_batched_eval=us_batch, batch=batch)
    cache[key] = rec
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return dict(rec, cached=False)

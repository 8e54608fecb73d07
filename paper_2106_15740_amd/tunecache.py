"""Tuning cache: the tile shapes the library's autotuners chose for a plan,
keyed by (GPU architecture, element type, plan signature).

An entry holds the global tuning (qtn_autotune: workgroup shape, split
thresholds, merging, the LDS-resident kernel) and the per-band tiles of the
wide buckets (qtn_autotune_bands), with the persistent sweep's time when they
were chosen.  The file is JSON; the default is ``tuning_cache.json`` beside
this module, or the path in the environment variable QTN_TUNE_CACHE.
"""
from __future__ import annotations

import json
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PATH = os.path.join(HERE, "tuning_cache.json")


def cache_path(path: Optional[str] = None) -> str:
    return path or os.environ.get("QTN_TUNE_CACHE") or DEFAULT_PATH


def arch(device: int) -> str:
    """The GPU's architecture name without feature flags (e.g. gfx950)."""
    import torch

    name = getattr(torch.cuda.get_device_properties(device), "gcnArchName", "") or "unknown"
    return name.split(":")[0]


# the planner's step structure (merging rules); entries of another version
# were tuned for different programs
PLAN_VERSION = 2


def key(net) -> str:
    return f"{arch(net.device)}|{net.dtype}|{net.signature()}|plan{PLAN_VERSION}"


def load(path: Optional[str] = None) -> dict:
    try:
        with open(cache_path(path)) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store(entries: dict, path: Optional[str] = None) -> bool:
    """Writes the cache (whole file, replaced atomically); False if the path
    is not writable."""
    p = cache_path(path)
    tmp = p + ".tmp"
    try:
        os.makedirs(os.path.dirname(os.path.abspath(p)), exist_ok=True)
        with open(tmp, "w") as fh:
            json.dump(entries, fh, indent=1, sort_keys=True)
        os.replace(tmp, p)
        return True
    except OSError:
        return False


def tuned(net, with_grad: bool = True, path: Optional[str] = None, search: bool = True, retune: bool = False,
          reps: int = 2) -> Optional[dict]:
    """Applies this plan's cached tuning; without an entry (or with retune)
    runs the global autotuner from the net's current tuning, then the per-band
    one, and stores the result.  Returns the entry with 'source' ('cache' or
    'search'), or None when there is no entry and search is off."""
    entries = load(path)
    k = key(net)
    if k in entries and not retune:
        e = entries[k]
        net.set_tuning(**e["tuning"])
        net.set_band_tuning(e["bands"])
        return dict(e, key=k, source="cache")
    if not search:
        return None
    net.autotune(with_grad=with_grad, reps=max(reps, 1))
    bands, ms = net.autotune_bands(with_grad=with_grad, reps=reps)
    e = {"tuning": net.tuning(), "bands": bands, "sweep_ms": ms}
    entries = load(path)
    entries[k] = e
    stored = store(entries, path)
    return dict(e, key=k, source="search", stored=stored)

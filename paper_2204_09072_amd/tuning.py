"""Persistent autotune cache of the batched trace.

tr_batch_tune searches segments per pass, waves per block and the work-queue chunk on a
sample of the batch.  The setting it finds depends on the GPU and on the batch's shape, not
on its values, so it is stored in a JSON file keyed by (GPU architecture, N_side values,
radial points, instance count, grid class = total cells to the nearest power of two) and
applied with tr_batch_set_tuning the next time a batch of that key is built.
"""
from __future__ import annotations

import json
import math
import os

_FIELDS = ("bins_per_pass", "waves_per_block", "chunk", "sample_ms", "widest_pass", "waves_used")


def cache_key(arch: str, trees, params) -> str:
    n_sides = sorted({int(p.n_side) for p in params})
    n_bins = max(int(t.n_bins) for t in trees)
    cells = sum(int(t.n_cells) for t in trees)
    cls = int(round(math.log2(max(cells, 1))))
    return (f"{arch.split(':')[0]}|n_side={','.join(map(str, n_sides))}|n_bins={n_bins}"
            f"|instances={len(trees)}|cells~2^{cls}")


def device_arch(device: int = 0) -> str:
    import torch
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def load(path) -> dict:
    """The cache's entries (an empty dict if the file does not exist)."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    if data.get("version") != 1:
        raise ValueError(f"{path}: not a version-1 tuning cache")
    return data["entries"]


def store(path, key: str, tuning) -> None:
    entries = load(path)
    entries[key] = {k: (round(float(getattr(tuning, k)), 3) if k == "sample_ms" else int(getattr(tuning, k)))
                    for k in _FIELDS}
    tmp = str(path) + ".tmp"
    with open(tmp, "w") as f:
        json.dump({"version": 1, "entries": entries}, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_cached(batch, path, key: str, sample_stride: int = 16):
    """Apply the cached setting for `key` if there is one, else tune and store the result.
    Returns (the batch's setting, True if it came from the cache)."""
    hit = load(path).get(key)
    if hit is not None:
        batch.set_tuning(hit["bins_per_pass"], hit["waves_per_block"], hit["chunk"])
        return batch.get_tuning(), True
    t = batch.tune(sample_stride)
    store(path, key, t)
    return t, False

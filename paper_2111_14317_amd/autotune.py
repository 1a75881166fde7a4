"""Work-item size autotuner for the batched tracker.

The batched form (one persistent launch over many systems) hands out work items of
`tile x 4 waves x (64 / N)` paths of one system at a time: small items balance the uneven path
lengths at the end of the launch, large items stage each system's tables into LDS fewer times.
The best size depends on the mix of systems and on the precision, so it is measured: `tune`
tracks an evenly strided sample of the paths once per candidate size, times the launch with the
library's own kernel events, and remembers the fastest size in a JSON cache keyed by the batch's
shape.  The chosen size goes into `hom_track_params.tile`.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

CANDIDATES = (1, 2, 4, 8, 16)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2111_14317_amd",
                             "tiles.json")


def signature(batch, sys_idx, precision, device_name: str) -> str:
    """Key of a tuning result: device, precision, each system's (n, largest m_k) and its path count
    rounded to two significant digits."""
    counts = np.bincount(np.asarray(sys_idx, np.int64), minlength=batch.num_sys)
    shape = [(int(n), int(m), float(f"{int(p):.2g}")) for n, m, p in
             zip(batch.ns, batch.mmax, counts)]
    blob = json.dumps([device_name, int(precision), shape])
    return hashlib.sha1(blob.encode()).hexdigest()


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_tile(hom, batch, c, z0, s0, sys_idx, precision, tile, reps=1) -> float:
    """Milliseconds of the batched tracking kernel for this sample at this work-item size (the
    mean over `reps` launches after one untimed launch)."""
    import torch
    params = hom.default_params(precision, tile=int(tile))
    hom.track(batch, c, z0, s0, params, sys_idx=sys_idx)  # untimed: first-touch effects
    torch.cuda.synchronize()
    hom.profile_read()
    hom.set_profiling(True)
    try:
        for _ in range(reps):
            hom.track(batch, c, z0, s0, params, sys_idx=sys_idx)
        torch.cuda.synchronize()
    finally:
        hom.set_profiling(False)
    ms = [t for name, t, _ in hom.profile_read() if name.startswith("k_track_batch")]
    return sum(ms) / max(len(ms), 1)


def tune(hom, batch, c, z0, s0, sys_idx, precision, candidates=CANDIDATES, sample_every=8,
         cache_path: str | None = DEFAULT_CACHE, refresh=False):
    """Return (best tile, {tile: ms}) for tracking these paths on this batch handle.  The sample is
    every `sample_every`-th path (so every system keeps its share and sys_idx stays sorted)."""
    import torch
    sys_idx = np.asarray(sys_idx, np.int32)
    dev = torch.cuda.get_device_name()
    key = signature(batch, sys_idx, precision, dev)
    table = _load(cache_path) if cache_path else {}
    if not refresh and key in table:
        hit = table[key]
        return int(hit["tile"]), {int(k): v for k, v in hit["ms"].items()}
    pick = np.arange(0, len(sys_idx), max(int(sample_every), 1))
    zs = np.asarray(z0)[pick]
    ss = np.asarray(s0)[pick] if np.ndim(s0) else s0
    times = {}
    for t in candidates:
        times[int(t)] = time_tile(hom, batch, c, zs, ss, sys_idx[pick], precision, t)
    best = min(times, key=times.get)
    if cache_path:
        table[key] = {"tile": best, "ms": {str(k): v for k, v in times.items()},
                      "device": dev, "precision": int(precision), "sample_every": int(sample_every)}
        _store(cache_path, table)
    return best, times

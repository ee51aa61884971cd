"""Cache of collide tilings chosen by the library's autotuner.

`mpc_autotune` times a coordinate search over tilings on the live state;
results do not depend on the tiling, only the speed does.  This module keeps
the chosen tiling (cells per tile, persistent grid, rows per block, tile
order) in a JSON file keyed by the device (architecture name and compute-unit
count), the storage form, the feature flags and the box shapes, so that a
later handle of the same kind skips the timing runs.

The file is `$MPC_TUNE_CACHE` if set, else `tuning_cache.json` beside this
module.  Entries are plain JSON; a corrupt or unreadable file is treated as
empty, and a file that cannot be written leaves the cache in memory only.
"""
from __future__ import annotations

import json
import math
import os
import tempfile

DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")
FIELDS = ("tile_cells", "grid", "yblock", "order")


def cache_path(path: str | None = None) -> str:
    return path or os.environ.get("MPC_TUNE_CACHE") or DEFAULT_PATH


def device_tag() -> str:
    """Architecture name and compute-unit count of the current device."""
    import torch
    prop = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(prop, "gcnArchName", "") or prop.name
    return f"{arch.split(':')[0]}/{prop.multi_processor_count}cu"


def cache_key(device: str, params) -> str:
    """Key of a set of boxes: device, form, flags, and the box shapes -- every
    (L, density) for up to four boxes, else the box count with the particle
    total and the mean density rounded to a power of two."""
    p0 = params[0]
    head = f"{device}|form{p0.form}|flags{p0.flags}"
    if len(params) <= 4:
        shapes = ";".join(f"{q.L[0]}x{q.L[1]}x{q.L[2]}@{q.density:g}" for q in params)
        return f"{head}|{shapes}"
    cells = [q.L[0] * q.L[1] * q.L[2] for q in params]
    ntot = sum(round(q.density * c) for q, c in zip(params, cells))
    dens = ntot / max(1, sum(cells))
    return (f"{head}|{len(params)}boxes|n2^{round(math.log2(max(ntot, 1)))}"
            f"|d2^{round(math.log2(max(dens, 1e-9)))}")


def load(path: str | None = None) -> dict:
    try:
        with open(cache_path(path)) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save(data: dict, path: str | None = None) -> bool:
    """Write the cache atomically; False if the location is not writable."""
    p = cache_path(path)
    tmp = None
    try:
        fd, tmp = tempfile.mkstemp(prefix=".tuning", dir=os.path.dirname(p) or ".")
        with os.fdopen(fd, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
        return True
    except OSError:
        if tmp is not None and os.path.exists(tmp):
            try:
                os.unlink(tmp)
            except OSError:
                pass
        return False


def autotune_cached(sim, trial_steps: int = 3, path: str | None = None,
                    device: str | None = None):
    """Apply the cached tiling for `sim` or, on a miss, run the autotuner and
    store its choice.  Returns (tiling dict, hit)."""
    key = cache_key(device or device_tag(), sim.params)
    data = load(path)
    hit = data.get(key)
    if isinstance(hit, dict) and all(k in hit for k in FIELDS):
        sim.set_tiling(*(int(hit[k]) for k in FIELDS))
        return {k: int(hit[k]) for k in FIELDS}, True
    sim.autotune(trial_steps)
    t = sim.get_tiling()
    entry = {k: int(t[k]) for k in FIELDS}
    data[key] = entry
    save(data, path)
    return entry, False

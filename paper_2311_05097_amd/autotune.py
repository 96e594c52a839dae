"""Tile-shape autotuner for the fused step kernel.

The step kernel is compiled for 64 x TY tiles with TY in {4, 8, 16} (and 32
outside FP64 storage).  Small TY
gives more blocks (better load balance on 256 CUs) but recomputes a larger
share of halo; large TY amortises the 3-node halo of the order parameter.  The
best choice depends on the grid and on the storage mode, so it is measured:
each candidate runs a few milliseconds of steps on a scratch domain of the
same size and storage (HIP-event kernel time, best of two interleaved
rounds), and the fastest is cached in a JSON file keyed by (nx, ny,
storage).

Cache: $LBMGLS_TUNE_CACHE or ~/.cache/lbmgls/tiles.json.
"""
from __future__ import annotations

import json
import os

import numpy as np

CANDIDATES = (4, 8, 16)
CANDIDATES_32 = CANDIDATES + (32,)  # 64 x 32 tiles are built for FP32 and 16-bit storage


def cache_path() -> str:
    p = os.environ.get("LBMGLS_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "lbmgls", "tiles.json")


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(c: dict):
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + ".tmp"
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass


def key(nx: int, ny: int, storage: str) -> str:
    return f"{nx}x{ny}:{storage}"


def measure(params: dict, storage: str, ty: int, steps: int = 40, warmup: int = 5) -> float:
    """Average step-kernel time (ms) of tile shape 64 x ty on a scratch domain."""
    from . import lbmgls
    nx, ny = int(params["nx"]), int(params["ny"])
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    phi = np.tanh((min(nx, ny) / 4.0 - np.hypot(x - nx / 2.0, y - ny / 2.0)) / 2.0)
    d = lbmgls.Domain(params, phi, np.zeros_like(phi), storage=storage, tile=ty)
    d.step(warmup)
    d.step(steps)
    ms = d.last_step_ms
    d.close()
    return ms


def best_tile(params: dict, storage: str, retune: bool = False) -> int:
    nx, ny = int(params["nx"]), int(params["ny"])
    k = key(nx, ny, storage)
    cache = _load()
    if not retune and k in cache:
        return int(cache[k]["tile"])
    # enough steps for a few milliseconds per measurement, two interleaved
    # rounds, the better of the two per candidate (near-ties are common)
    steps = max(40, min(400, int(2e8 // (nx * ny))))
    times = {}
    for _ in range(2):
        for ty in (CANDIDATES if storage == "fp64" else CANDIDATES_32):
            t = measure(params, storage, ty, steps=steps)
            times[ty] = min(t, times.get(ty, t))
    best = min(times, key=times.get)
    cache[k] = {"tile": best, "ms": {str(t): round(v, 5) for t, v in times.items()}}
    _save(cache)
    return best

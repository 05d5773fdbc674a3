"""Launch-shape autotuner for batched replicas.

For a loaded ``Batch`` it times whole batched steps (replayed as the cached
HIP graph, so launch overhead is what a production loop sees) for every
candidate ``Tiles``, keeps the fastest, and caches the choice on disk keyed
by the batch's shape and the device.  Every candidate gives bitwise the same
trajectory (the tiles only change how work is spread over workgroups), so
tuning never changes results; the state is restored after each trial.

The timing uses HIP events on the current stream; the library does the
work, this module only orders the calls.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Iterable, List, Optional, Tuple

import numpy as np
import torch

from .dpd import Batch, Tiles

FORCE_GRIDS = (0, 512, 1024, 2048, 4096)
NLIST_WAVES = (1, 2, 4)
NLIST_KINDS = (0, 1, 2)


def builder_candidates() -> List[Tiles]:
    """List builders with the default force grid.  The tile builder (kind 0)
    sizes its workgroups from the density and ignores nlist_waves, so it is
    one candidate; the block and lane builders take 1, 2 or 4 waves."""
    return [Tiles(force_grid=0, nlist_waves=w, nlist_kind=k)
            for k in NLIST_KINDS for w in ((4,) if k == 0 else NLIST_WAVES)]


def force_candidates(builder: Tiles) -> List[Tiles]:
    """Force grids with a chosen list builder."""
    return [Tiles(force_grid=g, nlist_waves=builder.nlist_waves, nlist_kind=builder.nlist_kind)
            for g in FORCE_GRIDS]


def default_candidates() -> List[Tiles]:
    """Every combination (the staged search of ``tune`` times a subset)."""
    return [Tiles(force_grid=g, nlist_waves=w, nlist_kind=k)
            for k in NLIST_KINDS for g in FORCE_GRIDS for w in ((4,) if k == 0 else NLIST_WAVES)]


def cache_path() -> str:
    root = os.environ.get("DPD_AUTOTUNE_CACHE")
    if root:
        return root
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "libdpd", "autotune.json")


def batch_key(b: Batch) -> str:
    """Shape of the work: particle counts, boxes, precision and device."""
    h = hashlib.sha256()
    h.update(np.asarray(b.sizes, dtype=np.int64).tobytes())
    h.update(np.asarray([p.box for p in b.params], dtype=np.float64).tobytes())
    h.update(np.asarray([b.params[0].r_c, b.params[0].skin], dtype=np.float64).tobytes())
    h.update(str(b.precision).encode())
    h.update(torch.cuda.get_device_name(b.state.x.device).encode())
    return h.hexdigest()[:32]


def _load_cache(path: str) -> Dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store_cache(path: str, data: Dict) -> None:
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass                                   # a read-only home only loses the cache


def _snapshot(b: Batch):
    st = b.state
    return [t.clone() for t in (st.x, st.v, st.f, st.tag, st.type, b.d_step, b.status)]


def _restore(b: Batch, snap) -> None:
    st = b.state
    for dst, src in zip((st.x, st.v, st.f, st.tag, st.type, b.d_step, b.status), snap):
        dst.copy_(src)


def time_tiles(b: Batch, tiles: Tiles, steps: int = 5, warmup: int = 2, repeats: int = 3) -> float:
    """Median milliseconds per graph-replayed step with these tiles."""
    b.set_tiles(tiles)
    b.step(warmup, use_graph=True)
    times = []
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.step(steps, use_graph=True)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / steps)
    return float(np.median(times))


def tune(b: Batch, candidates: Optional[Iterable[Tiles]] = None, *, use_cache: bool = True,
         steps: int = 5) -> Tuple[Tiles, Dict[str, float]]:
    """Pick and apply the fastest tiles for ``b``; returns (tiles, timings).

    Without explicit candidates the search is staged: the list builder
    first (default force grid), then the force grid with that builder.  The
    two are separate kernels of a step whose times add, so the stages find
    the joint optimum with 7 + 4 trials instead of 35.  The batch state
    (and step counter) is restored after every trial, so the caller
    continues from where it was."""
    path = cache_path()
    key = batch_key(b)
    if use_cache:
        hit = _load_cache(path).get(key)
        if hit is not None:
            t = Tiles(int(hit["force_grid"]), int(hit["nlist_waves"]), int(hit.get("nlist_kind", 0)))
            b.set_tiles(t)
            return t, {k: float(v) for k, v in hit.get("timings", {}).items()}
    snap = _snapshot(b)
    timings: Dict[str, float] = {}
    best, best_ms = None, float("inf")

    def trial(cands):
        nonlocal best, best_ms
        for t in cands:
            name = f"{t.force_grid}/{t.nlist_waves}/{t.nlist_kind}"
            if name in timings:
                continue
            ms = time_tiles(b, t, steps=steps)
            _restore(b, snap)
            timings[name] = ms
            if ms < best_ms:
                best, best_ms = t, ms

    if candidates is not None:
        trial(list(candidates))
    else:
        trial(builder_candidates())
        trial(force_candidates(best))
    torch.cuda.synchronize()
    b.set_tiles(best)
    if use_cache:
        data = _load_cache(path)
        data[key] = {"force_grid": best.force_grid, "nlist_waves": best.nlist_waves,
                     "nlist_kind": best.nlist_kind, "ms_per_step": best_ms, "timings": timings}
        _store_cache(path, data)
    return best, timings

"""Autotuner for batched launches: picks the tile geometry and the
time-chunk length of a batch.

A batch's work list cuts every (instance, channel, tile group) into time
chunks; short chunks balance the persistent grid but cost a partial-sum
round trip through HBM each, long chunks leave compute units idle at the
tail.  Instances with N <= 128 run either as padded 256-input super-blocks
or in the halves geometry (the 10 tiles of a 4-block triangle over pairs of
32-sample steps).  The tuner times every feasible (geometry, chunk length)
candidate on scratch accumulators of the batch's own shapes (the caller's
sums are never touched), keeps the fastest, and caches the choice in a
JSON file keyed by the device architecture and the batch's shape
signature.

Cache file: ``$XE_TUNE_CACHE`` if set, else ``~/.cache/xengine/tune.json``.
"""

from __future__ import annotations

import hashlib
import json
import os
import threading
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

from . import xengine

_lock = threading.Lock()

#: cache entries written by this version (older entries carry no geometry)
CACHE_VERSION = 2


@dataclass(frozen=True)
class Choice:
    """A batch's tuned launch: chunk length in 32-sample steps and the tile
    geometry of its N <= 128 instances ("super" or "halves"; "auto" when
    the batch has none)."""
    chunk_steps: int
    geometry: str


def cache_path() -> str:
    return os.environ.get("XE_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "xengine", "tune.json")


def signature(shapes: Sequence[Tuple[int, int, int, int]]) -> str:
    """Order-free digest of the instances' (N, F, T, B)."""
    text = ";".join(f"{n},{f},{t},{b}" for n, f, t, b in sorted(shapes))
    return hashlib.sha256(text.encode()).hexdigest()[:20]


def _arch(device: int) -> str:
    import torch
    p = torch.cuda.get_device_properties(device)
    return f"{getattr(p, 'gcnArchName', 'unknown')}/{p.multi_processor_count}cu"


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    try:
        with open(path or cache_path()) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(key: str, entry: dict, path: Optional[str] = None) -> None:
    path = path or cache_path()
    with _lock:
        data = load_cache(path)
        data[key] = entry
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = f"{path}.{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)


def candidates(shapes: Sequence[Tuple[int, int, int, int]], n_cu: int) -> List[int]:
    """Feasible chunk lengths around the automatic one, plus 'never split'."""
    auto = xengine.batch_query(shapes, n_cu=n_cu).chunk_steps
    out = []
    for c in sorted({max(32, int(auto * r)) for r in (0.5, 0.7, 1.0, 1.4, 2.0, 3.0)} |
                    {1 << 18}):
        try:
            xengine.batch_query(shapes, n_cu=n_cu, chunk_steps=c)
        except xengine.XEngineError:
            continue   # time-chunk sums would not fit the workspace
        out.append(c)
    return out


def geometries(shapes: Sequence[Tuple[int, int, int, int]]) -> List[str]:
    """Tile geometries worth timing: both when an instance has N <= 128."""
    return ["super", "halves"] if any(n <= 128 for n, _, _, _ in shapes) else ["auto"]


def _key(items: Sequence[Tuple]) -> Tuple[str, List[Tuple[int, int, int, int]]]:
    dev = items[0][0].device
    shapes = [(int(p.shape[2]), int(p.shape[1]), int(p.shape[0]), int(B))
              for p, m, B, v, c in items]
    return f"{_arch(dev.index)}|{signature(shapes)}", shapes


def lookup(items: Sequence[Tuple], path: Optional[str] = None) -> Optional[dict]:
    """The cached tuning entry of this batch (its choice and every timing),
    or None."""
    if not items:
        return None
    hit = load_cache(path).get(_key(items)[0])
    return hit if hit is not None and hit.get("version") == CACHE_VERSION else None


def best_by_geometry(entry: dict) -> Dict[str, float]:
    """Fastest timing (ms) per geometry of a cached tuning entry."""
    best: Dict[str, float] = {}
    for name, ms in entry.get("timings_ms", {}).items():
        geom = name.split("/")[0]
        best[geom] = min(best.get(geom, float("inf")), float(ms))
    return best


def tune(items: Sequence[Tuple], handle: Optional[xengine.Handle] = None,
         reps: int = 5, use_cache: bool = True, path: Optional[str] = None) -> Choice:
    """Best (chunk length, geometry) for a batch of (packed, mask, B, vis,
    count) items; runs on scratch accumulators."""
    import torch
    if not items:
        return Choice(0, "auto")
    dev = items[0][0].device
    key, shapes = _key(items)
    if use_cache:
        hit = load_cache(path).get(key)
        if hit is not None and hit.get("version") == CACHE_VERSION:
            return Choice(int(hit["chunk_steps"]), str(hit["geometry"]))
    n_cu = torch.cuda.get_device_properties(dev.index).multi_processor_count
    h = handle or xengine.default_handle(dev.index)
    scratch = [(p, m, B, torch.zeros_like(v), torch.zeros_like(c)) for p, m, B, v, c in items]
    timings = {}
    stream = torch.cuda.current_stream(dev)
    for geom in geometries(shapes):
        for cs in candidates(shapes, n_cu):
            for _, _, _, v, _ in scratch:     # every candidate integrates afresh
                xengine.reset_integration(v)
            plan = xengine.BatchPlan(scratch, chunk_steps=cs, handle=h, geometry=geom)
            try:
                plan.run(stream)   # warm-up
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(reps):
                    plan.run(stream)
                e1.record(stream)
                e1.synchronize()
                timings[(geom, cs)] = e0.elapsed_time(e1) / reps
            finally:
                plan.release()
    del scratch
    geom, cs = min(timings, key=timings.get)
    _store(key, {"version": CACHE_VERSION, "chunk_steps": cs, "geometry": geom,
                 "ms": timings[(geom, cs)],
                 "timings_ms": {f"{g}/{c}": round(v, 5) for (g, c), v in timings.items()},
                 "instances": len(shapes)}, path)
    return Choice(cs, geom)

"""Autotuner for the launch shape of mesh and mesh-batch plans.

It builds one plan per candidate (workgroup size, elements per thread), times
`reps` gradient calls of each with HIP events on the current stream, and keeps
the fastest.  Results are cached in a JSON file keyed by plan kind, dtype,
nodes per element and a size class, so a workload class is tuned once.
Cache path: $PGRAD_TUNE_CACHE, else ~/.cache/pgrad/tune.json.
"""
from __future__ import annotations

import json
import math
import os
from typing import Callable, Dict, Iterable, List, Optional, Tuple

import torch

from . import pgrad

CANDIDATES: Tuple[Tuple[int, int], ...] = ((256, 1), (512, 1), (1024, 1), (256, 2), (512, 2),
                                           (128, 4))


def _cache_path() -> str:
    p = os.environ.get("PGRAD_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "pgrad", "tune.json")


def _load() -> Dict[str, dict]:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db: Dict[str, dict]) -> None:
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home directory only loses the cache


def size_class(n_elems: int) -> int:
    return int(math.log2(max(n_elems, 1)))


def time_calls(fn: Callable[[], object], reps: int, warmup: int) -> float:
    """Average milliseconds of fn() over reps calls, after warmup calls."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(key: str, make: Callable[[int, int], pgrad._Plan], run: Callable[[pgrad._Plan], object],
         candidates: Iterable[Tuple[int, int]] = CANDIDATES, reps: int = 10, warmup: int = 2,
         use_cache: bool = True) -> dict:
    """Return {"block", "tile", "ms", "table"} for the fastest candidate."""
    db = _load() if use_cache else {}
    if use_cache and key in db:
        return db[key]
    table: List[dict] = []
    for block, tile in candidates:
        try:
            plan = make(block, tile)
        except pgrad.PgError:
            continue
        ms = time_calls(lambda: run(plan), reps, warmup)
        table.append({"block": block, "tile": tile, "ms": round(ms, 5)})
        plan.close()
    if not table:
        raise pgrad.PgError(pgrad.EINVAL, "autotune", "no candidate could be planned")
    best = min(table, key=lambda r: r["ms"])
    res = {"block": best["block"], "tile": best["tile"], "ms": best["ms"], "table": table}
    if use_cache:
        db[key] = res
        _store(db)
    return res


def tune_mesh(conn, B, w, n_nodes: int, x, adjoint: str = "atomic", ckpt: str = "recompute",
              candidates=CANDIDATES, reps: int = 10, use_cache: bool = True) -> dict:
    key = f"mesh:{adjoint}:{B.dtype}:k{conn.shape[1]}:e{size_class(conn.shape[0])}"
    g = torch.empty_like(x)

    def make(block, tile):
        return pgrad.MeshObjective(conn, B, w, n_nodes, adjoint=adjoint, ckpt=ckpt, block=block,
                                   tile=tile)

    return tune(key, make, lambda p: p.gradient(x, out=g), candidates, reps, 2, use_cache)


def tune_batch(inst, conn, B, w, x, ckpt: str = "recompute", candidates=CANDIDATES,
               reps: int = 5, use_cache: bool = True) -> dict:
    n_el = int(sum(int(r[1]) for r in inst))
    key = f"batch:{B.dtype}:k{conn.shape[1]}:i{len(inst)}:e{size_class(n_el)}"
    g = torch.empty_like(x)

    def make(block, tile):
        return pgrad.MeshBatch(inst, conn, B, w, ckpt=ckpt, block=block, tile=tile)

    return tune(key, make, lambda p: p.gradient(x, out=g), candidates, reps, 2, use_cache)

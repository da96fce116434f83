"""Measured choice of a plan's chunk schedule.

A plan cuts every problem into chunks of about rows / target_chunks rows (at
least 32 and 2k + 2 rows, at most 64^2 chunks per problem).  Few long chunks
leave lanes idle and make each lane's row chain long; many short ones add
summary and scan work.  The best target depends on the batch's sizes and
bandwidths and on the operation, so it is measured: each candidate plan runs
the caller's step a few times on the device and the fastest is kept.
Results can be cached in a JSON file keyed by the batch's shape.
"""
from __future__ import annotations

import json
import math
import os
from typing import Callable, Dict, Iterable, Optional

import torch

DEFAULT_CANDIDATES = (16384, 32768, 65536, 131072, 196608, 262144)


def device_arch() -> str:
    """The current device's architecture name (gfx950 on MI355X), or "cpu"."""
    if not torch.cuda.is_available():
        return "cpu"
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def shape_key(ns, ks, op: str, prec: int, arch: Optional[str] = None) -> str:
    """Batch signature: device architecture, problem count, total rows (2
    significant digits) and the set of bandwidths, plus the operation and
    storage format."""
    arch = device_arch() if arch is None else arch
    rows = sum(int(n) for n in ns)
    mag = 10 ** max(int(math.log10(rows)) - 1, 0) if rows > 0 else 1
    return (f"{arch}|{op}|p{prec}|np{len(ns)}|rows{round(rows / mag) * mag}"
            f"|k{','.join(map(str, sorted(set(ks))))}")


def time_step(step: Callable[[], None], reps: int = 3) -> float:
    """Mean milliseconds of step() over reps runs after one warm-up."""
    step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        step()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(ns, ks, make_step: Callable[[int], Callable[[], None]], op: str, prec: int,
         candidates: Iterable[int] = DEFAULT_CANDIDATES, reps: int = 3,
         cache_path: Optional[str] = None) -> Dict:
    """Pick the target chunk count with the fastest step.  make_step(target)
    builds a plan for that target and returns its step.  Returns
    {"target_chunks": best, "ms": {target: ms}, "cached": bool}."""
    key = shape_key(ns, ks, op, prec)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return dict(cache[key], cached=True)
    ms = {}
    for t in candidates:
        ms[int(t)] = time_step(make_step(int(t)), reps)
    best = min(ms, key=ms.get)
    res = {"target_chunks": best, "ms": ms}
    if cache_path:
        cache[key] = res
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return dict(res, cached=False)

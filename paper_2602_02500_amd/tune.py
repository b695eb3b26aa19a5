"""Autotuner of the 256-tile schedules: per stage (Gram, squaring, product) it times candidate
schedules (tile order blocks, XCD queue groups, grid) on the caller's real
inputs, keeps the fastest, and caches the choice in a JSON file keyed by device and plan.

Timing uses the library's per-launch-slot events: a call records an event before every slot, so
the time of one stage is the sum of its slots. Results do not depend on the schedule (each tile
is computed the same way in any order), so tuning changes only speed.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Iterable, List

from . import STAGE_GRAM, STAGE_PRODUCT, STAGE_SQUARE

__all__ = ["STAGES", "candidates", "tune", "plan_key", "load_cache", "save_cache", "apply"]

STAGES = {"gram": STAGE_GRAM, "square": STAGE_SQUARE, "product": STAGE_PRODUCT}


def candidates(stage: int) -> List[dict]:
    """Schedules tried for a stage: XCD queues with three group sizes and four block shapes, and
    plain striding. The same list serves every stage."""
    out = []
    for group in (16, 32, 64):
        for br, bc in ((4, 8), (8, 8), (2, 16), (8, 4)):
            out.append(dict(xcd_sched=1, group=group, block_rows=br, block_cols=bc, wg_per_xcd=32))
    out.append(dict(xcd_sched=0, group=32, block_rows=4, block_cols=8, wg_per_xcd=32))
    return out


def _stage_ms(plan, Ms, Ys, ws, stage: int, reps: int, torch) -> float:
    n = plan.num_launches
    slots = [i for i in range(n) if plan.launch_info(i)[0] == stage]
    total = 0.0
    for _ in range(reps):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
        for e in evs:
            e.record()
        torch.cuda.synchronize()
        plan.launch_events([e.cuda_event for e in evs])
        plan.orthogonalize_batched(Ms, Ys, ws)
        torch.cuda.synchronize()
        total += sum(evs[i].elapsed_time(evs[i + 1]) for i in slots)
    return total / reps


def tune(plan, Ms, Ys, ws, stages: Iterable[str] = ("gram", "square", "product"), reps: int = 2,
         log=None) -> Dict[str, dict]:
    """Tunes the listed stages of `plan` on the batch (Ms, Ys, ws) in turn and leaves the best
    schedule of each set on the plan. Returns {stage name: {"config": ..., "ms": ..., "default_ms": ...}}."""
    import torch
    plan.orthogonalize_batched(Ms, Ys, ws)  # warm-up
    torch.cuda.synchronize()
    result = {}
    for name in stages:
        st = STAGES[name]
        base = plan.get_config(st)
        base_ms = _stage_ms(plan, Ms, Ys, ws, st, reps, torch)
        best, best_ms = base, base_ms
        for c in candidates(st):
            if c == base:
                continue
            plan.set_config(st, c)
            ms = _stage_ms(plan, Ms, Ys, ws, st, reps, torch)
            if log:
                log(f"tune {name}: {c} -> {ms:.3f} ms")
            if ms < best_ms:
                best, best_ms = c, ms
        plan.set_config(st, best)
        result[name] = {"config": best, "ms": round(best_ms, 4), "default_ms": round(base_ms, 4)}
        if log:
            log(f"tune {name}: best {best} {best_ms:.3f} ms (default {base_ms:.3f} ms)")
    return result


def plan_key(device_name: str, shapes, compute: str, exponents) -> str:
    """Cache key: device (architecture and compute-unit count), compute type, exponents and the
    multiset of problem shapes."""
    sig = json.dumps({"compute": compute, "exponents": list(map(int, exponents)),
                      "shapes": sorted([list(map(int, s)) for s in shapes])})
    return f"{device_name}|{hashlib.sha1(sig.encode()).hexdigest()[:16]}"


def load_cache(path: str) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save_cache(path: str, key: str, result: Dict[str, dict], note: str = ""):
    cache = load_cache(path)
    cache[key] = {"stages": {k: v["config"] for k, v in result.items()}, "timing_ms": result, "note": note}
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def apply(plan, entry: dict):
    """Sets the cached schedules of an entry written by save_cache on `plan`."""
    for name, cfg in entry["stages"].items():
        plan.set_config(STAGES[name], cfg)

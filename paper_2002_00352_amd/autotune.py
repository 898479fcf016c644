"""Autotuner for the sweep's tile shape: users per tile and grid size per
problem shape class, chosen by timing the sweep kernel with HIP events on the
caller's instance, cached as JSON.

Shape class: (gfx arch, M, K, b_format, local-constraint signature, N bucket).
The cache lives at $KP_AUTOTUNE_CACHE (default ~/.cache/kp_autotune.json).
Tuning changes only speed: decisions, multipliers and consumption are the
same for every choice (g and P may differ in the last bits, being FP64 sums
grouped by block)."""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

from . import Context, Problem, default_context, kp_eval_dual, kp_scd_sweep

USERS_PER_TILE = (4, 8, 16, 32, 48, 64)
GRIDS = (512, 1024, 2048, 4096)


def cache_path() -> str:
    return os.environ.get("KP_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "kp_autotune.json"))


def _arch() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "gfx950"


def shape_key(prob: Problem) -> str:
    tree = ",".join(f"{p}/{c}" for p, c in zip(prob.parent.tolist(), prob.cap.tolist()))
    leaf = ",".join(str(v) for v in prob.leaf.tolist())
    fmt = "dense" if prob.b is not None else "csr"
    nb = int(math.log2(max(prob.N, 1)))
    return f"{_arch()}|M{prob.M}|K{prob.K}|{fmt}|{tree}|{leaf}|N2^{nb}"


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    path = path or cache_path()
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: Dict[str, dict], path: Optional[str] = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(ctx: Context, prob: Problem, choice: Tuple[int, int]) -> None:
    fmt = 0 if prob.b is not None else 1
    ctx.set_tuning(prob.M, prob.K, fmt, int(choice[0]), int(choice[1]))


def _time(ctx: Context, prob: Problem, lam, scd: bool, reps: int) -> float:
    import torch
    ctx.set_timing(True)
    for _ in range(reps):
        if scd:
            kp_scd_sweep(prob, lam, ctx=ctx)
        else:
            kp_eval_dual(prob, lam, ctx=ctx)
    torch.cuda.synchronize()
    ms, n, _ = ctx.timing()
    ctx.set_timing(False)
    return ms / max(n, 1)


def tune(prob: Problem, ctx: Optional[Context] = None, scd: bool = True, lam=None, reps: int = 2,
         candidates: Optional[Sequence[Tuple[int, int]]] = None, use_cache: bool = True,
         path: Optional[str] = None) -> Tuple[int, int]:
    """Best (users_per_tile, grid) for this problem's shape class; measured on
    this instance unless cached, then applied to the context."""
    import torch
    ctx = ctx or default_context()
    key = shape_key(prob) + ("|scd" if scd else "|eval")
    cache = load_cache(path) if use_cache else {}
    if key in cache:
        choice = tuple(cache[key]["choice"])
        apply(ctx, prob, choice)
        return choice
    if lam is None:
        lam = torch.full((prob.K,), 0.5 / prob.K, dtype=torch.float64, device="cuda")
    cands = list(candidates) if candidates else [(u, g) for u in USERS_PER_TILE for g in GRIDS]
    results = []
    for u, g in cands:
        apply(ctx, prob, (u, g))
        try:
            _time(ctx, prob, lam, scd, 1)            # warm
            results.append((_time(ctx, prob, lam, scd, reps), u, g))
        except Exception:
            continue
    if not results:
        apply(ctx, prob, (0, 0))
        return (0, 0)
    results.sort()
    best = (results[0][1], results[0][2])
    apply(ctx, prob, best)
    if use_cache:
        cache = load_cache(path)
        cache[key] = {"choice": list(best), "ms": results[0][0],
                      "tried": [[u, g, ms] for ms, u, g in results]}
        save_cache(cache, path)
    return best

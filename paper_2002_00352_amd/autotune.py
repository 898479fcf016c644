"""Autotuner for the sweep's tile shape: users per tile and grid size per
problem shape class (the grid alone for the uniform-row kernel), chosen by
timing the sweep kernel with HIP events on the caller's instance, cached as
JSON; and the batched plan's LDS budget and block split, timed over whole
iterations.

Shape class: (gfx arch, M, K, b_format, local-constraint signature, N bucket).
The cache lives at $KP_AUTOTUNE_CACHE (default ~/.cache/kp_autotune.json).
Tuning changes only speed: decisions, multipliers and consumption are the
same for every choice (g and P may differ in the last bits, being FP64 sums
grouped by block)."""
from __future__ import annotations

import json
import math
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import (KP_ERR_UNSUPPORTED, Context, KPError, Problem, default_context, kp_eval_dual,
               kp_scd_sweep)

USERS_PER_TILE = (4, 8, 16, 32, 48, 64)
GRIDS = (512, 1024, 2048, 4096)
ELL_GRIDS = (128, 256, 512, 768, 1024)          # the uniform-row kernel: grid only
BATCHED = ((32768, 64), (40960, 32), (40960, 64), (40960, 128), (65536, 64))   # (LDS bytes, block multiple)
KERNEL_NAMES = {0: "general", 1: "uniform-row", 2: "dense-lane", 3: "dense-lane window pass"}


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
    fmt = "dense" if prob.b is not None else f"csr{prob.row_nnz}"
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


def _run(ctx: Context, prob: Problem, lam, scd: bool):
    if scd:
        return kp_scd_sweep(prob, lam, ctx=ctx)
    return kp_eval_dual(prob, lam, ctx=ctx)


def _time(ctx: Context, prob: Problem, lam, scd: bool, reps: int) -> float:
    import torch
    ctx.set_timing(True)
    for _ in range(reps):
        _run(ctx, prob, lam, scd)
    torch.cuda.synchronize()
    ms, n, _ = ctx.timing()
    ctx.set_timing(False)
    return ms / max(n, 1)


def candidates_for(kernel: int) -> List[Tuple[int, int]]:
    """(users per tile, grid) candidates of a kernel: the uniform-row kernel
    tunes its grid only; for the lane-per-user dense evaluation, its grids
    and the general kernel's tiles (a users-per-tile choice selects the
    general kernel)."""
    if kernel == 1:
        return [(0, g) for g in ELL_GRIDS]
    general = [(u, g) for u in USERS_PER_TILE for g in GRIDS]
    if kernel == 2:
        return [(0, g) for g in ELL_GRIDS] + general
    return general


def tune(prob: Problem, ctx: Optional[Context] = None, scd: bool = True, lam=None, reps: int = 2,
         candidates: Optional[Sequence[Tuple[int, int]]] = None, use_cache: bool = True,
         path: Optional[str] = None) -> Tuple[int, int]:
    """Best (users_per_tile, grid) for this problem's shape class; measured on
    this instance unless cached, then applied to the context.  Candidates
    that launch the same shape as an earlier one (a grid capped at the
    resident blocks) are timed once; a candidate the library refuses as
    unsupported is skipped, any other error is raised."""
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
    apply(ctx, prob, (0, 0))
    _run(ctx, prob, lam, scd)
    kernel = ctx.launch_shape()[0]
    cands = list(candidates) if candidates else candidates_for(kernel)
    results, seen = [], set()
    for u, g in cands:
        apply(ctx, prob, (u, g))
        try:
            _run(ctx, prob, lam, scd)                   # warm
        except KPError as e:
            if e.status == KP_ERR_UNSUPPORTED:
                continue
            raise
        shape = ctx.launch_shape()
        if shape in seen:
            continue
        seen.add(shape)
        results.append((_time(ctx, prob, lam, scd, reps), u, g, shape))
    if not results:
        apply(ctx, prob, (0, 0))
        return (0, 0)
    results.sort()
    best = (results[0][1], results[0][2])
    apply(ctx, prob, best)
    if use_cache:
        cache = load_cache(path)
        cache[key] = {"choice": list(best), "ms": results[0][0], "kernel": KERNEL_NAMES.get(kernel, kernel),
                      "tried": [[u, g, ms, list(sh)] for ms, u, g, sh in results]}
        save_cache(cache, path)
    return best


def tune_batched(probs: Sequence[Problem], candidates: Sequence[Tuple[int, int]] = BATCHED,
                 steps: int = 2, warmup: int = 1):
    """Best (LDS bytes per block, block multiple) of the batched plan for this
    batch, timed over the same SCD iterations from lambda = 0 (a new plan per
    candidate).  Returns (choice, table of (choice, ms per iteration, plan
    shape))."""
    import time
    import torch
    from . import BatchedSCD
    table = []
    for lds, mult in candidates:
        ctx = Context()
        ctx.set_batched_tuning(lds, mult)
        try:
            bs = BatchedSCD(probs, ctx=ctx)
        except KPError as e:
            if e.status == KP_ERR_UNSUPPORTED:
                continue
            raise
        for _ in range(warmup):
            bs.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            bs.step()
        torch.cuda.synchronize()
        table.append(((lds, mult), (time.perf_counter() - t0) * 1e3 / steps, bs.shape()))
        bs.close()
        ctx.close()
    best = min(table, key=lambda r: r[1])[0] if table else (0, 0)
    return best, table

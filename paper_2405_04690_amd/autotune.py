"""Autotuner of the launch shapes (the gbl_tuning knobs of include/gbl.h):
times each candidate setting on the caller's own workload with HIP events on
the context's stream and keeps the fastest.  Results can be cached in a JSON
file keyed by device, precision and a workload tag.

Knobs: the bucket group size (uneven widths and the mixed-precision FP64
re-evaluation), the launch order of the width buckets, exact grids from
host-read bucket sizes (a stream synchronisation per call), and the grid cap
of the flow inference launches."""
from __future__ import annotations

import itertools
import json
import os

import torch

from .gbl import Context

__all__ = ["time_call", "tune", "tune_delta_var", "tune_flow", "load_cached", "store_cached"]

CHUNKS = (1 << 14, 1 << 16, 1 << 18, 1 << 20)
FLOW_GRIDS = (512, 1024, 2048, 4096, 8192, 16384)


def time_call(ctx: Context, fn, reps: int = 5) -> float:
    """mean milliseconds per call of fn() on the context's current stream (one warm-up call)"""
    stream = torch.cuda.current_stream(ctx.device)
    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / reps


def tune(ctx: Context, fn, space: dict, reps: int = 5):
    """exhaustive search over the product of the knob lists in `space`;
    sets and returns the best knobs with the timing table"""
    base = ctx.get_tuning().as_dict()
    names = list(space)
    table = []
    for vals in itertools.product(*(space[n] for n in names)):
        knobs = dict(zip(names, vals))
        ctx.set_tuning(**knobs)
        table.append((time_call(ctx, fn, reps), knobs))
    table.sort(key=lambda x: x[0])
    best = dict(base)
    best.update(table[0][1])
    ctx.set_tuning(**best)
    return best, [(round(ms, 4), k) for ms, k in table]


def tune_delta_var(ctx: Context, args: tuple, kwargs: dict | None = None, reps: int = 5):
    """knobs of gb_delta_loglike_var on the given call (bucket group size, launch order)"""
    kwargs = dict(kwargs or {})
    out = torch.empty(args[2].shape[0], dtype=torch.float64, device=ctx.device)
    kwargs["out"] = out
    space = {"bucket_chunk": list(CHUNKS), "widest_first": [1, 0], "exact_grids": [0, 1]}
    return tune(ctx, lambda: ctx.gb_delta_loglike_var(*args, **kwargs), space, reps)


def tune_flow(ctx: Context, flow, u, band, reps: int = 5):
    """grid cap of the flow inference launches on the given batch"""
    return tune(ctx, lambda: flow.log_prob(u, band), {"flow_grid": list(FLOW_GRIDS)}, reps)


def _key(ctx: Context, tag: str) -> str:
    name = torch.cuda.get_device_properties(ctx.device).name
    return f"{name}|precision={ctx.cfg.precision}|{tag}"


def load_cached(ctx: Context, tag: str, path: str) -> bool:
    """apply cached knobs for (device, precision, tag) if present"""
    if not os.path.exists(path):
        return False
    rec = json.load(open(path)).get(_key(ctx, tag))
    if rec is None:
        return False
    ctx.set_tuning(**rec)
    return True


def store_cached(ctx: Context, tag: str, path: str):
    data = json.load(open(path)) if os.path.exists(path) else {}
    data[_key(ctx, tag)] = ctx.get_tuning().as_dict()
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)

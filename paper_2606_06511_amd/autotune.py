"""Autotuner for the library's launch parameters.

The launch shapes and work budgets of the kernels (``ttie.PARAM_*``) change only the speed of a
step, never its results.  ``tune`` times a caller-supplied step on its real inputs and picks,
one parameter at a time and for a few passes (coordinate descent), the value with the shortest
step.  It only sets parameters and reads the clock; the step itself runs in library kernels.
"""

from __future__ import annotations

import time

import torch

from . import ttie

# candidate values per parameter (the library's defaults are 4096, 2048, 128, 64 and 0)
SPACE = {
    "screen_blocks": (ttie.PARAM_SCREEN_BLOCKS, (512, 1024, 2048, 4096, 8192)),
    "row_blocks": (ttie.PARAM_ROW_BLOCKS, (256, 512, 1024, 2048, 4096)),
    "trav_budget": (ttie.PARAM_TRAV_BUDGET, (16, 24, 32, 64, 128, 256, 1024)),
    # 0: one contiguous chunk of the candidate list per wave; otherwise tiles from a queue
    "screen_tile": (ttie.PARAM_SCREEN_TILE, (0, 1024, 4096, 16384)),
}


def time_step(step, reps: int = 10, warmup: int = 3) -> float:
    """Milliseconds per call of ``step`` (device-synchronized)."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def tune(ctx: ttie.Context, step, space=SPACE, reps: int = 10, rounds: int = 2):
    """Coordinate descent over ``space``.  Leaves the best values set on ``ctx`` and returns
    ({name: value}, ms with them, ms with the defaults)."""
    for pid, _ in space.values():
        ctx.set_param(pid, 0)
    ms_default = time_step(step, reps)
    best = {name: ctx.get_param(pid) for name, (pid, _) in space.items()}
    for _ in range(rounds):
        for name, (pid, values) in space.items():
            times = {}
            for v in values:
                ctx.set_param(pid, v)
                times[v] = time_step(step, reps)
            best[name] = min(times, key=times.get)
            ctx.set_param(pid, best[name])
    return best, time_step(step, reps), ms_default

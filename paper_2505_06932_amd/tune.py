"""Autotuner of the launch shapes (ftc_tuning) for a given front: the whole
coupling step is captured in a HIP graph for each candidate shape and timed
by replays; the fastest shape is kept.  The knobs are searched one after
another (lanes per cell in the fast PPIC shape, z-chunks per column block,
the fast PPIC shape's grid), each with the others at their best so far.  Every
shape gives the same cell lists, decisions and curvatures, so the choice is
a matter of time only."""
from __future__ import annotations

import dataclasses

import torch

from . import ftc

CANDIDATES = {
    "ring_lanes": (4, 8, 16),
    "column_chunks": (4, 8, 16),
    "ring_blocks": (0, 2048, 8192),
}


def time_step(step, reps: int = 20, warmup: int = 3) -> float:
    """Milliseconds per step of graph replays of step.run()."""
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step.run(stream=s)  # warm the shapes outside the capture
        with torch.cuda.graph(g, stream=s):
            step.run(stream=s)
    torch.cuda.synchronize()
    for _ in range(warmup):
        g.replay()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune(step, reps: int = 20, warmup: int = 3, candidates=None, log=None):
    """Choose and set the launch shapes of step's workspace.  Returns the
    chosen ftc.Tuning and the table of (tuning, ms per step) tried."""
    cand = dict(CANDIDATES if candidates is None else candidates)
    best = ftc.get_tuning(step.cells)
    table = []
    timed = {}

    def measure(t):
        if t not in timed:
            ftc.set_tuning(step.cells, t)
            timed[t] = time_step(step, reps, warmup)
            table.append((t, timed[t]))
            if log:
                log(f"[tune] {t}: {timed[t] * 1e3:.1f} us/step")
        return timed[t]

    best_ms = measure(best)
    for knob, values in cand.items():
        for v in values:
            t = dataclasses.replace(best, **{knob: v})
            ms = measure(t)
            if ms < best_ms:
                best, best_ms = t, ms
    ftc.set_tuning(step.cells, best)
    return best, table

"""Autotuner of the launch shapes (ftc_tuning) for a given front: the whole
coupling step is captured in a HIP graph for each candidate shape and timed
by replays; the fastest shape is kept.

The PPIC knobs that interact are searched jointly: lanes per cell in the fast
shape (4 to 64) times the work-queue chunk (0: the static split of the cell
groups over the XCDs; else groups taken from per-XCD queues that many at a
time).  Then the fast shape's grid and the column pass's z-chunks are
searched one after the other, each with the others at their best so far.
Every shape gives the same cell lists, decisions and curvatures, so the
choice is a matter of time only."""
from __future__ import annotations

import dataclasses
import itertools

import torch

from . import ftc

# Knob groups in search order; a group of several knobs is searched over
# the product of its values.
CANDIDATES = (
    {"ring_lanes": (4, 8, 16, 32, 64), "queue_chunk": (0, 1, 2, 4, 8)},
    {"ring_blocks": (0, 2048, 8192)},
    {"column_chunks": (4, 8, 16)},
)


def shapes_of(group: dict, base: ftc.Tuning):
    """The tunings of one knob group around base."""
    keys = list(group)
    for vals in itertools.product(*(group[k] for k in keys)):
        yield dataclasses.replace(base, **dict(zip(keys, vals)))


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
    chosen ftc.Tuning and the table of (tuning, ms per step) tried, in the
    order tried."""
    groups = CANDIDATES if candidates is None else candidates
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
    for group in groups:
        base = best
        for t in shapes_of(group, base):
            ms = measure(t)
            if ms < best_ms:
                best, best_ms = t, ms
    ftc.set_tuning(step.cells, best)
    return best, table

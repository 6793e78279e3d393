"""Autotuner of the solve's configuration per ROM size (n, m).

Candidates: the execution form (fused: the whole Newton loop in one kernel,
launched with one workgroup per point or as a persistent grid of k
workgroups per compute unit pulling points from a work list; phased, n <= 75:
the first evaluations as separate material and contraction launches), and
how the four waves of a workgroup share the contraction (split the ECM
points, or the tiles of K; the point split keeps every tile in registers:
FP64 for n <= 75, the reduced forms for n <= 123).  Each candidate is timed
with HIP events on the same sample load step from the same state; the
fastest is kept in a table keyed by (n, m, contraction) that can be saved as
JSON.
"""
import json

import numpy as np
import torch

from . import (DT_F64, MODE_FUSED, MODE_PHASED, rom_default_opts, rom_homogenized_stress_tangent, rom_state_init,
               rom_step, rom_fused_tiles)
from .batch import RomBatch

GRIDS = (0, 1, 2, 4)


def candidates(n, contraction=DT_F64, graph=False):
    """(mode, split, grid_per_cu): point split (FP64 up to five column tiles,
    reduced forms up to eight) and tile split, each with every launch form of
    the fused kernel, and the phased form up to five column tiles (not for
    steps captured in a graph, which it does not support)."""
    T = rom_fused_tiles(n)
    splits = (0, 1) if (T <= 5 or contraction != DT_F64) else (1,)
    out = [(MODE_FUSED, s, g) for s in splits for g in GRIDS]
    if T <= 5 and not graph:
        out += [(MODE_PHASED, s, 2) for s in splits]
    return out


def time_config(rb, Fb, contraction, mode, split, grid, reps=3, warm=1):
    s = rb.stream
    o = rom_default_opts(mode=mode, contraction=contraction, split=split, grid_per_cu=grid)
    best = np.inf
    for r in range(warm + reps):
        rom_state_init(rb.h, rb.P, rb.mu.data_ptr(), rb.state.data_ptr(), s.cuda_stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        rom_step(rb.h, rb.P, Fb.data_ptr(), rb.state.data_ptr(), o, rb.status.data_ptr(), rb.iters.data_ptr(),
                 rb.resnorm.data_ptr(), s.cuda_stream)
        e1.record(s)
        e1.synchronize()
        if r >= warm:
            best = min(best, e0.elapsed_time(e1))
    return best


def tune(rom_path, mu, Fbar, contraction, reps=3, graph=False):
    """Time every candidate on one load step of the batch (mu, Fbar (P, 2, 2));
    graph: only the configurations that can be captured in a graph."""
    rb = RomBatch(rom_path, mu)
    Fb = torch.as_tensor(np.ascontiguousarray(Fbar), dtype=torch.float64).reshape(rb.P, 4).to(rb.device)
    n, m = rb.info['n'], rb.info['m']
    times = {}
    for cfg in candidates(n, contraction, graph):
        times[cfg] = time_config(rb, Fb, contraction, *cfg, reps=reps)
    rb.close()
    best = min(times, key=times.get)
    return dict(n=n, m=m, contraction=contraction, mode=best[0], split=best[1], grid_per_cu=best[2],
                ms=times[best], trials={f"mode{md}_split{s}_grid{g}": t for (md, s, g), t in times.items()})


class Table:
    def __init__(self, entries=None):
        self.entries = {(e['n'], e['m'], e['contraction']): e for e in (entries or [])}

    def lookup(self, n, m, contraction):
        return self.entries.get((n, m, contraction))

    def add(self, e):
        self.entries[(e['n'], e['m'], e['contraction'])] = e

    def save(self, path):
        with open(path, 'w') as fh:
            json.dump(list(self.entries.values()), fh, indent=1)

    @classmethod
    def load(cls, path):
        with open(path) as fh:
            return cls(json.load(fh))

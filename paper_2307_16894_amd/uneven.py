"""Uneven persistent batches over several ROMs, driven from a captured graph.

Each ROM of the batch is a group: its points follow their own load paths
with their own step counts.  One load step of every group is a device-side
sequence -- rom_path_gather (next Fbar and the active mask), rom_step on the
active points (persistent fused kernel, or the phased form with its side
stream forked and joined inside the step), rom_homogenized_stress_tangent,
rom_path_advance -- so the whole step is captured once as a HIP graph whose
branches (one per group) run concurrently, and replayed until every point has
finished its path.  Kernel configurations per (n, m) come from the
autotuner.
"""
import numpy as np
import torch

from . import (DT_F64, MODE_FUSED, rom_default_opts, rom_homogenized_stress_tangent, rom_path_advance,
               rom_path_gather, rom_state_init, rom_step)
from .batch import RomBatch


class Group:
    def __init__(self, rom_path, mu, paths, nsteps, contraction=DT_F64, split=-1, grid_per_cu=2, max_iter=15,
                 max_substeps=4, mode=MODE_FUSED, device='cuda:0'):
        self.rb = RomBatch(rom_path, mu, device)
        dev = self.rb.device
        self.P = self.rb.P
        self.Kmax = int(paths.shape[1])
        self.paths = torch.from_numpy(np.ascontiguousarray(paths.reshape(self.P, self.Kmax, 4))).to(dev)
        self.nsteps = torch.as_tensor(np.asarray(nsteps), dtype=torch.int32, device=dev).contiguous()
        self.step = torch.zeros(self.P, dtype=torch.int32, device=dev)
        self.Fbar = torch.eye(2, dtype=torch.float64, device=dev).reshape(1, 4).repeat(self.P, 1).contiguous()
        self.active = torch.zeros(self.P, dtype=torch.int32, device=dev)
        self.evals = torch.zeros(self.P, dtype=torch.int64, device=dev)
        self.solved = torch.zeros(self.P, dtype=torch.int64, device=dev)
        self.failed = torch.zeros(self.P, dtype=torch.int64, device=dev)
        self.opts = rom_default_opts(mode=mode, contraction=contraction, split=split, grid_per_cu=grid_per_cu,
                                     max_iter=max_iter, max_substeps=max_substeps)
        self.opts.active = self.active.data_ptr()

    def enqueue(self, stream):
        """One load step of the group on `stream` (no host synchronisation)."""
        rb, s = self.rb, stream.cuda_stream
        rom_path_gather(self.P, self.paths.data_ptr(), self.Kmax, self.nsteps.data_ptr(), self.step.data_ptr(),
                        self.Fbar.data_ptr(), self.active.data_ptr(), s)
        rom_step(rb.h, self.P, self.Fbar.data_ptr(), rb.state.data_ptr(), self.opts, rb.status.data_ptr(),
                 rb.iters.data_ptr(), rb.resnorm.data_ptr(), s)
        rom_homogenized_stress_tangent(rb.h, self.P, rb.state.data_ptr(), rb.Pbar.data_ptr(), rb.Abar.data_ptr(), s)
        with torch.cuda.stream(stream):
            act = self.active.to(torch.int64)
            self.evals += act * rb.iters.to(torch.int64)
            self.solved += act
            self.failed += act * ((rb.status != 0) & (rb.status != 3)).to(torch.int64)
        rom_path_advance(self.P, self.active.data_ptr(), self.step.data_ptr(), s)

    def reset(self):
        """Back to the virgin state at step 0 (outside any capture)."""
        rb = self.rb
        rom_state_init(rb.h, self.P, rb.mu.data_ptr(), rb.state.data_ptr(), rb.stream.cuda_stream)
        for t in (self.step, self.active, self.evals, self.solved, self.failed):
            t.zero_()

    def close(self):
        self.rb.close()


class UnevenBatch:
    def __init__(self, groups):
        self.groups = groups
        self.graph = None
        self.streams = [torch.cuda.Stream() for _ in groups]  # default priority

    @property
    def max_steps(self):
        return max(int(g.nsteps.max()) for g in self.groups)

    def step_eager(self):
        main = torch.cuda.current_stream()
        for g, s in zip(self.groups, self.streams):
            s.wait_stream(main)
            g.enqueue(s)
        for s in self.streams:
            main.wait_stream(s)

    def capture(self):
        """Capture one load step of all groups as a graph with one branch per group."""
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream()
        with torch.cuda.graph(self.graph, stream=cap):
            for g, s in zip(self.groups, self.streams):
                s.wait_stream(cap)
                g.enqueue(s)
            for s in self.streams:
                cap.wait_stream(s)
        torch.cuda.synchronize()
        return self.graph

    def run(self, use_graph=True):
        for _ in range(self.max_steps):
            if use_graph:
                self.graph.replay()
            else:
                self.step_eager()

    def reset(self):
        torch.cuda.synchronize()
        for g in self.groups:
            g.reset()
        torch.cuda.synchronize()

    def totals(self):
        return dict(point_steps=int(sum(int(g.solved.sum()) for g in self.groups)),
                    evaluations=int(sum(int(g.evals.sum()) for g in self.groups)),
                    failed=int(sum(int(g.failed.sum()) for g in self.groups)))

    def close(self):
        for g in self.groups:
            g.close()

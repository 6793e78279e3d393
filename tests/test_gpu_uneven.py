"""Uneven persistent batch: several ROMs, per-point step counts, one load
step of everything captured as a graph and replayed.  Every replay is checked
against the same sequence run eagerly, and the final states against the FP64
oracle on each point's own path; the autotuner's pick must reproduce the
results of the default configuration."""
import os

import numpy as np
import pytest
import torch

import workloads
from oracle.rom import ROM
from tests.conftest import rom_path

import paper_2307_16894_amd as L
from paper_2307_16894_amd import autotune
from paper_2307_16894_amd.uneven import Group, UnevenBatch

pytestmark = pytest.mark.gpu


def _groups(specs, grid):
    out = []
    for name, P, seed in specs:
        ns = workloads.uneven_steps(seed, P, 6, 14)
        mu = workloads.one_void_mu(seed, P)
        paths = workloads.uneven_cyclic_paths(seed, P, ns, (0.005, 0.015))
        out.append((name, mu, paths, ns, Group(rom_path(name), mu, paths, ns, grid_per_cu=grid)))
    return out


def test_graph_replays_match_eager_and_oracle(gpu):
    specs = [('onevoid_n20_m120', 96, 31)]
    if os.path.exists(rom_path("onevoid_n40_m400")):
        specs.append(('onevoid_n40_m400', 64, 32))
    eager = _groups(specs, grid=2)
    graph = _groups(specs, grid=2)
    be = UnevenBatch([g for *_, g in eager])
    bg = UnevenBatch([g for *_, g in graph])
    bg.capture()
    for k in range(bg.max_steps):
        print(f"[gpu] uneven step {k}", flush=True)
        be.step_eager()
        bg.graph.replay()
        torch.cuda.synchronize()
        for (_, _, _, _, ge), (_, _, _, _, gg) in zip(eager, graph):
            assert torch.equal(ge.step, gg.step) and torch.equal(ge.active, gg.active)
            assert torch.equal(ge.rb.status, gg.rb.status)
            assert torch.equal(ge.rb.Pbar, gg.rb.Pbar) and torch.equal(ge.rb.r(), gg.rb.r())
    tot = bg.totals()
    assert tot['failed'] == 0
    assert tot['point_steps'] == sum(int(ns.sum()) for _, _, _, ns, _ in graph)
    # last-step effective stress of every point against the oracle on its own path
    for name, mu, paths, ns, g in graph:
        rom = ROM(rom_path(name))
        Pb = g.rb.Pbar.cpu().numpy()
        for p in range(0, g.P, 7):
            ref = rom.run_path(mu[p], paths[p, :ns[p]], max_iter=15, max_substeps=4)[-1]
            assert np.abs(Pb[p] - ref['Pbar']).max() < 1e-6 * np.abs(ref['Pbar']).max()
    be.close()
    bg.close()


def test_autotuner_pick_reproduces_default(gpu):
    name = 'onevoid_n20_m120'
    P = 256
    mu = workloads.one_void_mu(41, P)
    F = workloads.monotone_paths(41, P, 10)[:, 2]
    res = autotune.tune(rom_path(name), mu, F, L.DT_F64, reps=2)
    assert (res['split'], res['grid_per_cu']) in autotune.candidates(20)
    assert len(res['trials']) == len(autotune.candidates(20))
    out = {}
    pick = (res['split'], res['grid_per_cu'])
    for split, grid in ((-1, 0), (pick[0], 0), pick):
        g = Group(rom_path(name), mu, F[:, None], np.ones(P, dtype=np.int32), split=split, grid_per_cu=grid)
        g.opts.fixed_iters, g.opts.max_iter = 1, 6  # same Newton map on every side
        b = UnevenBatch([g])
        b.step_eager()
        torch.cuda.synchronize()
        out[(split, grid)] = g.rb.Pbar.cpu().numpy().copy()
        b.close()
    # the launch form (one workgroup per point or the persistent grid) leaves
    # every point's arithmetic unchanged: bit-identical
    assert np.array_equal(out[(pick[0], 0)], out[pick])
    # the split changes the summation order of K and f only
    ref = out[(-1, 0)]
    assert np.abs(out[pick] - ref).max() <= 1e-10 * np.abs(ref).max()

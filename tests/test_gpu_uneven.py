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


def _groups(specs, grid, mode):
    out = []
    for name, P, seed in specs:
        ns = workloads.uneven_steps(seed, P, 6, 14)
        mu = workloads.one_void_mu(seed, P)
        paths = workloads.uneven_cyclic_paths(seed, P, ns, (0.005, 0.015))
        out.append((name, mu, paths, ns, Group(rom_path(name), mu, paths, ns, grid_per_cu=grid, mode=mode)))
    return out


@pytest.mark.parametrize("mode", [L.MODE_FUSED, pytest.param(L.MODE_PHASED, marks=pytest.mark.skip(
    reason="graph capture of the phased step (side-stream fork and join) crashed the runtime's end of capture; "
           "the phased form now refuses capture (test_phased_form_refuses_graph_capture)"))])
def test_graph_replays_match_eager_and_oracle(gpu, mode):
    """Fused form captured as a graph; the phased form runs eagerly only."""
    specs = [('onevoid_n20_m120', 96, 31)]
    if os.path.exists(rom_path("onevoid_n40_m400")):
        specs.append(('onevoid_n40_m400', 64, 32))
    eager = _groups(specs, grid=2, mode=mode)
    graph = _groups(specs, grid=2, mode=mode)
    be = UnevenBatch([g for *_, g in eager])
    bg = UnevenBatch([g for *_, g in graph])
    bg.capture()
    for k in range(bg.max_steps):
        print(f"[gpu] uneven mode {mode} step {k}", flush=True)
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
    pick = (res['mode'], res['split'], res['grid_per_cu'])
    assert pick in autotune.candidates(20)
    assert len(res['trials']) == len(autotune.candidates(20))
    out = {}
    for cfg in ((L.MODE_FUSED, -1, 0), (L.MODE_FUSED, pick[1], 0), pick):
        mode, split, grid = cfg
        g = Group(rom_path(name), mu, F[:, None], np.ones(P, dtype=np.int32), split=split, grid_per_cu=grid,
                  mode=mode)
        g.opts.fixed_iters, g.opts.max_iter = 1, 6  # same Newton map on every side
        b = UnevenBatch([g])
        b.step_eager()
        torch.cuda.synchronize()
        out[cfg] = g.rb.Pbar.cpu().numpy().copy()
        b.close()
    # the execution form (one workgroup per point, the persistent grid, the
    # phased launches) leaves every point's arithmetic unchanged: bit-identical
    assert np.array_equal(out[(L.MODE_FUSED, pick[1], 0)], out[pick])
    # the split changes the summation order of K and f only
    ref = out[(L.MODE_FUSED, -1, 0)]
    assert np.abs(out[pick] - ref).max() <= 1e-10 * np.abs(ref).max()


def test_phased_form_refuses_graph_capture(gpu):
    """rom_step in the phased form returns ROM_EUNSUPPORTED inside a stream
    capture (checked before anything is enqueued); the capture is then ended
    with only a trivial kernel in it."""
    from paper_2307_16894_amd.batch import RomBatch
    name = 'onevoid_n20_m120'
    P = 8
    rb = RomBatch(rom_path(name), workloads.one_void_mu(3, P))
    Fb = torch.eye(2, dtype=torch.float64, device='cuda').reshape(1, 4).repeat(P, 1).contiguous()
    o = L.rom_default_opts(mode=L.MODE_PHASED)
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    torch.cuda.synchronize()
    code = None
    with torch.cuda.graph(g, stream=cap):
        try:
            L.rom_step(rb.h, P, Fb.data_ptr(), rb.state.data_ptr(), o, rb.status.data_ptr(), rb.iters.data_ptr(),
                       rb.resnorm.data_ptr(), cap.cuda_stream)
        except L.RomError as e:
            code = e.code
        Fb.add_(0.0)
    torch.cuda.synchronize()
    assert code == L.ROM_EUNSUPPORTED
    rb.close()


def test_full_uneven_workload_against_oracle(gpu):
    """The benchmark's uneven workload at full size: five ROMs (n = 20 ... 120,
    m = 120 ... 2000), 32768 points, per-point step counts U[5, 40], Newton
    cap 15, cutting depth 4, one captured step replayed until every path is
    done.  Every point-step converges, and in every ROM group the points with
    the two shortest paths and one of median length end at the oracle's Pbar
    and Abar on their own paths."""
    from bench import SUBSTEPS, UNEVEN
    u = UNEVEN['uneven_mixed_P32768']
    groups, specs = [], []
    for i, (name, P) in enumerate(u['roms']):
        seed = u['seed'] + i
        mu = workloads.one_void_mu(seed, P) if name.startswith('onevoid') else workloads.four_void_mu(seed, P)
        ns = workloads.uneven_steps(seed, P, *u['steps'])
        paths = workloads.uneven_cyclic_paths(seed, P, ns, u['rho'])
        groups.append(Group(rom_path(name), mu, paths, ns, max_iter=u['max_iter'], max_substeps=SUBSTEPS))
        specs.append((name, mu, paths, ns))
    b = UnevenBatch(groups)
    b.capture()
    for k in range(b.max_steps):
        if k % 10 == 0:
            print(f"[gpu] uneven full size replay {k} of {b.max_steps}", flush=True)
        b.graph.replay()
    torch.cuda.synchronize()
    tot = b.totals()
    assert tot['failed'] == 0
    assert tot['point_steps'] == sum(int(ns.sum()) for *_, ns in specs)
    for (name, mu, paths, ns), g in zip(specs, groups):
        rom = ROM(rom_path(name))
        Pb, Ab = g.rb.Pbar.cpu().numpy(), g.rb.Abar.cpu().numpy()
        order = np.argsort(ns, kind='stable')
        for p in (order[0], order[1], order[len(order) // 2]):
            print(f"[oracle] {name} point {p}, {ns[p]} steps", flush=True)
            ref = rom.run_path(mu[p], paths[p, :ns[p]], max_iter=u['max_iter'], max_substeps=SUBSTEPS)[-1]
            assert ref['status'] == 0
            assert np.abs(Pb[p] - ref['Pbar']).max() < 1e-6 * np.abs(ref['Pbar']).max(), (name, p)
            assert np.abs(Ab[p] - ref['Abar'].reshape(-1)).max() < 1e-6 * np.abs(ref['Abar']).max(), (name, p)
    b.close()

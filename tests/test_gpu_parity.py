"""GPU parity: the HIP solve against the FP64 oracle on the same seeded inputs.

Parity runs in fixed-iteration mode (both sides make the same number of
Newton evaluations, so they follow the same Newton map to rounding) and
compares, after every load step, the trial reduced coordinates, the status,
the effective stress and stiffness, and the committed history.  Tolerance:
1e-10 relative to the largest entry of each compared quantity (FP64 path).
"""
import numpy as np
import pytest
import torch

import workloads
from oracle.rom import ROM
from tests.conftest import rom_path

pytestmark = pytest.mark.gpu

TOL = 1e-10


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / scale)


def oracle_path(rom, mu, path, max_iter, fixed, tol=1e-8):
    return rom.run_path(mu, path, tol=tol, max_iter=max_iter, fixed=fixed)


def _run_gpu(name, mu, paths, mode, max_iter, fixed, record_hist=True, **extra):
    from paper_2307_16894_amd import batch as B
    from paper_2307_16894_amd import rom_default_opts
    rb = B.RomBatch(rom_path(name), mu)
    P, K = paths.shape[0], paths.shape[1]
    out = []
    for k in range(K):
        print(f"[gpu] {name} mode={mode} {extra} step {k}", flush=True)
        o = rom_default_opts(max_iter=max_iter, fixed_iters=int(fixed), mode=mode, **extra)
        st, it, rn = rb.step(torch.from_numpy(np.ascontiguousarray(paths[:, k])).cuda(), o)
        torch.cuda.synchronize()
        rec = dict(status=st.cpu().numpy().copy(), iters=it.cpu().numpy().copy(), res=rn.cpu().numpy().copy(),
                   r=rb.r(trial=True).cpu().numpy().copy(), Pbar=rb.Pbar.cpu().numpy().copy(),
                   Abar=rb.Abar.cpu().numpy().copy())
        if record_hist:
            rec['hist'] = rb.history().cpu().numpy().copy()
        out.append(rec)
    rb.close()
    return out


# staged form; fused form with the automatic layout, with the tile split, and
# launched as a persistent grid pulling points from the work list; phased form
# (its evaluations, then the fused kernel resuming the points from their state)
FORMS = {'staged': dict(mode=0), 'fused': dict(mode=1), 'fused_tilesplit': dict(mode=1, split=1),
         'fused_queue': dict(mode=1, grid_per_cu=2), 'fused_tilesplit_queue': dict(mode=1, split=1, grid_per_cu=1),
         'phased': dict(mode=2), 'phased_tilesplit_k2': dict(mode=2, split=1, phased_evals=2),
         # slow points after two evaluations to the side stream
         'phased_early2': dict(mode=2, phased_evals=5, phased_early=2),
         # every evaluation of the first attempt phased: a failed attempt is redone by the fused kernel
         'phased_all': dict(mode=2, phased_evals=1000, phased_early=-1)}


@pytest.mark.parametrize("form", sorted(FORMS))
def test_fixed_iteration_parity_onevoid_n20(gpu, form):
    name = 'onevoid_n20_m120'
    P, K = 16, 10
    mu = workloads.one_void_mu(0, 64)[:P]
    paths = workloads.monotone_paths(0, 64, 10)[:P]
    g = _run_gpu(name, mu, paths, max_iter=6, fixed=True, **FORMS[form])
    rom = ROM(rom_path(name))
    for p in range(P):
        ref = oracle_path(rom, mu[p], paths[p], max_iter=6, fixed=True)
        hist = rom.virgin()
        for k in range(K):
            s = ref[k]
            assert g[k]['status'][p] == s['status'], (p, k)
            assert g[k]['iters'][p] == s['iters']
            assert rel_err(g[k]['r'][p], s['r']) < TOL, (p, k, rel_err(g[k]['r'][p], s['r']))
            assert rel_err(g[k]['Pbar'][p], s['Pbar']) < TOL, (p, k)
            assert rel_err(g[k]['Abar'][p], s['Abar'].reshape(-1)) < TOL, (p, k)
            if s['status'] == 0:
                hist = s['hist']
            Fp, Fp33, xi = hist
            gh = g[k]['hist'][p]
            assert rel_err(gh[0:4].T.reshape(-1, 2, 2), Fp) < TOL
            assert rel_err(gh[4], Fp33) < TOL
            if np.abs(xi).max() > 0:
                assert rel_err(gh[5], xi) < TOL
            else:
                assert np.abs(gh[5]).max() == 0.0


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_converged_path_onevoid_n20(gpu, mode):
    """Plain Newton to 1e-8: every step converges, same iteration counts and
    effective stress as the oracle (to the Newton tolerance)."""
    name = 'onevoid_n20_m120'
    P = 64
    mu = workloads.one_void_mu(0, P)
    paths = workloads.monotone_paths(0, P, 10)
    g = _run_gpu(name, mu, paths, mode, max_iter=15, fixed=False, record_hist=False)
    rom = ROM(rom_path(name))
    for p in range(0, P, 8):
        ref = oracle_path(rom, mu[p], paths[p], max_iter=15, fixed=False)
        for k in range(10):
            assert g[k]['status'][p] == 0 and ref[k]['status'] == 0
            assert abs(int(g[k]['iters'][p]) - ref[k]['iters']) <= 1
            assert rel_err(g[k]['Pbar'][p], ref[k]['Pbar']) < 1e-6
    assert all((rec['status'] == 0).all() for rec in g)


def test_active_mask_skips_points(gpu):
    """Points with active[p] == 0 keep their state and outputs; the others
    match a run without the mask (fixed iterations, bit-identical)."""
    import paper_2307_16894_amd as L
    from paper_2307_16894_amd.batch import RomBatch
    name = 'onevoid_n20_m120'
    P = 40
    mu = workloads.one_void_mu(5, P)
    paths = workloads.monotone_paths(5, P, 4)
    act = torch.tensor([(p % 3) != 1 for p in range(P)], dtype=torch.int32, device='cuda')
    for mode, grid in ((1, 0), (1, 2), (2, 0)):
        full, masked = RomBatch(rom_path(name), mu), RomBatch(rom_path(name), mu)
        for k in range(4):
            print(f"[gpu] active mask mode={mode} grid={grid} step {k}", flush=True)
            Fb = torch.from_numpy(np.ascontiguousarray(paths[:, k])).cuda()
            o = L.rom_default_opts(mode=mode, fixed_iters=1, max_iter=5, grid_per_cu=grid)
            full.step(Fb, o)
            torch.cuda.synchronize()  # the batches run on their own streams
            r_before = masked.r().clone()
            masked.iters.fill_(-7)
            torch.cuda.synchronize()
            o.active = act.data_ptr()
            masked.step(Fb, o)
            torch.cuda.synchronize()
            on = act.bool()
            assert torch.equal(masked.r()[on], full.r()[on])
            assert torch.equal(masked.Pbar[on], full.Pbar[on])
            assert torch.equal(masked.r()[~on], r_before[~on])
            assert (masked.iters[~on] == -7).all()
        full.close()
        masked.close()


@pytest.mark.parametrize("form", ['fused', 'fused_tilesplit_queue', 'phased', 'phased_early2', 'phased_all'])
def test_load_step_cutting_parity(gpu, form):
    """Large increments from the virgin state, where the plain step fails:
    with cutting depth 4 (fixed evaluations per attempt, so both sides take
    the same attempts) the kernel follows the oracle's sequence of sub-steps
    and commits the same state."""
    from paper_2307_16894_amd import batch as B
    import paper_2307_16894_amd as L
    name = 'onevoid_n20_m120'
    P, K, D, it = 16, 2, 4, 8
    mu = workloads.one_void_mu(7, 40)[:P]
    paths = workloads.monotone_paths(7, 40, K, rho=(0.06, 0.1))[:P]
    rb = B.RomBatch(rom_path(name), mu)
    rom = ROM(rom_path(name))
    refs = [rom.run_path(mu[p], paths[p], max_iter=it, fixed=True, max_substeps=D) for p in range(P)]
    assert sum(len(refs[p][k]['targets']) for p in range(P) for k in range(K)) > 0
    for k in range(K):
        print(f"[gpu] cutting {form} step {k}", flush=True)
        o = L.rom_default_opts(max_iter=it, fixed_iters=1, max_substeps=D, **FORMS[form])
        st, its, _ = rb.step(torch.from_numpy(np.ascontiguousarray(paths[:, k])).cuda(), o)
        torch.cuda.synchronize()
        st, its = st.cpu().numpy(), its.cpu().numpy()
        Pb, Ab, rc, fbc = (rb.Pbar.cpu().numpy(), rb.Abar.cpu().numpy(), rb.r().cpu().numpy(),
                           rb.fbar_committed().cpu().numpy())
        hc = rb.history().cpu().numpy()
        sub = rb.substeps().cpu().numpy().view(np.uint32)
        for p in range(P):
            s = refs[p][k]
            assert st[p] == s['status'] and its[p] == s['iters'], (p, k, st[p], s['status'], its[p], s['iters'])
            # converged sub-step ends t / 16 on the 1/32 grid: bit 2t - 1
            assert sub[p] == sum(1 << (2 * t - 1) for t in s['ends']), (p, k, hex(sub[p]), s['ends'])
            assert rel_err(Pb[p], s['Pbar']) < TOL and rel_err(Ab[p], s['Abar'].reshape(-1)) < TOL, (p, k)
            r_c, h_c, F_c = ((s['r'], s['hist'], paths[p, k]) if s['status'] == 0
                             else (s['r_c'], s['hist_c'], s['Fbar_c']))
            assert rel_err(rc[p], r_c) < TOL and rel_err(fbc[p], np.asarray(F_c).reshape(-1)) < 1e-15, (p, k)
            assert rel_err(hc[p][0:4].T.reshape(-1, 2, 2), h_c[0]) < TOL, (p, k)
    rb.close()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_commit_trial_equals_committing_step(gpu, mode):
    """A trial step (commit = 0) followed by rom_commit_trial leaves the state
    a committing step to the same Fbar leaves, bit for bit, over three load
    steps; points that did not converge keep their committed state."""
    from paper_2307_16894_amd import batch as B
    from paper_2307_16894_amd import rom_default_opts
    P, K = 64, 3
    mu = workloads.one_void_mu(31, P)
    paths = workloads.monotone_paths(31, P, K, (0.01, 0.03))
    a, b = B.RomBatch(rom_path('onevoid_n20_m120'), mu), B.RomBatch(rom_path('onevoid_n20_m120'), mu)
    for k in range(K):
        print(f"[gpu] commit_trial mode={mode} step {k}", flush=True)
        F = torch.from_numpy(np.ascontiguousarray(paths[:, k])).cuda()
        # a low cap leaves some points unconverged at the larger increments
        o = dict(mode=mode, tol=1e-10, max_iter=4)
        st_a, _, _ = a.step(F, rom_default_opts(commit=1, **o))
        b.step(F, rom_default_opts(commit=0, **o))
        b.commit_trial(F)
        torch.cuda.synchronize()
        assert np.array_equal(st_a.cpu().numpy(), b.status.cpu().numpy())
        for view in (lambda x: x.r(), lambda x: x.history(), lambda x: x._view(B.FIELD_FBAR_COMMITTED, (P, 4))):
            assert torch.equal(view(a), view(b)), k
    a.close()
    b.close()

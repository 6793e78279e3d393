"""Parity at the benchmark's full size: the one-void ROM with n = 40 modes and
371 ECM points, 4096 macro points on 20-step load / unload paths, launched as
the benchmark launches it (fused form, automatic layout, one workgroup per
point).  The oracle recomputes a sample of the points one by one, spread over
the batch (first, last and points in between)."""
import functools

import numpy as np
import pytest
import torch

import paper_2307_16894_amd as L
from bench import WORKLOADS, inputs
from oracle.rom import ROM
from paper_2307_16894_amd.batch import RomBatch
from tests.conftest import rom_path

pytestmark = pytest.mark.gpu

W = WORKLOADS['onevoid_n40_m400_P4096_cyclic20']
# spread over the batch, plus points whose plain Newton step fails somewhere
# on their path (they converge with load-step cutting)
SAMPLE = np.unique(np.r_[np.linspace(0, W['P'] - 1, 12).astype(int), 1, 255, 256, 2047, 27, 83, 122, 145])


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


def run_gpu(opts, K):
    mu, paths = inputs(W)
    rb = RomBatch(rom_path(W['rom']), mu)
    out = []
    for k in range(K):
        print(f"[gpu] full size P={W['P']} contraction={opts.contraction} fixed={opts.fixed_iters} step {k}",
              flush=True)
        st, it, rn = rb.step(torch.from_numpy(np.ascontiguousarray(paths[:, k])).cuda(), opts)
        torch.cuda.synchronize()
        out.append(dict(status=st.cpu().numpy().copy(), iters=it.cpu().numpy().copy(),
                        r=rb.r(trial=True).cpu().numpy().copy(), Pbar=rb.Pbar.cpu().numpy().copy(),
                        Abar=rb.Abar.cpu().numpy().copy(), sub=rb.substeps().cpu().numpy().view(np.uint32).copy()))
    rb.close()
    return out


@functools.lru_cache(maxsize=None)
def oracle(p, K, fixed, max_iter, max_substeps=0):
    mu, paths = inputs(W)
    return ROM(rom_path(W['rom'])).run_path(mu[p], paths[p, :K], tol=1e-8, max_iter=max_iter, fixed=fixed,
                                            max_substeps=max_substeps)


def test_fixed_iteration_parity_full_size(gpu):
    K = 6
    g = run_gpu(L.rom_default_opts(mode=L.MODE_FUSED, fixed_iters=1, max_iter=4), K)
    for p in SAMPLE:
        ref = oracle(int(p), K, True, 4)
        for k in range(K):
            assert g[k]['status'][p] == ref[k]['status'], (p, k)
            assert rel(g[k]['r'][p], ref[k]['r']) < 1e-10, (p, k)
            assert rel(g[k]['Pbar'][p], ref[k]['Pbar']) < 1e-10, (p, k)
            assert rel(g[k]['Abar'][p], ref[k]['Abar'].reshape(-1)) < 1e-10, (p, k)


# BF16 with abar_f64: K*, C and sum w|J| A of Abar from an FP64 evaluation at
# the returned state, so Abar differs from the oracle's only as far as the two
# converged states do (BF16 Newton takes other iterates than FP64 and stops at
# another point within the tolerance: the bound of Pbar)
@pytest.mark.parametrize("dt,abar,tol_P,tol_A", [(L.DT_F64, 0, 1e-6, 1e-6), (L.DT_BF16, 0, 1e-5, 3e-2),
                                                 (L.DT_BF16, 1, 1e-5, 1e-5)])
def test_converged_paths_full_size(gpu, dt, abar, tol_P, tol_A):
    """Plain Newton with load-step cutting (depth 4), as the benchmark runs it:
    every point-step of the batch converges, and the sampled points agree with
    the oracle to the Newton tolerance on every step of the same loading path
    (the same converged sub-steps since the start of the path).  FP64 takes
    the oracle's sub-steps everywhere; the BF16 tangent may let a sampled
    point (several of them are chosen because their plain step fails) cut a
    step differently, after which it integrates its plastic flow over other
    increments: those point-steps are counted, not compared."""
    K = W['steps']
    g = run_gpu(L.rom_default_opts(mode=L.MODE_FUSED, contraction=dt, max_substeps=4, abar_f64=abar), K)
    conv = np.mean([(rec['status'] == 0).mean() for rec in g])
    print(f"contraction {dt}: converged fraction {conv:.6f}")
    assert conv > 0.9995
    other = 0
    for p in SAMPLE:
        ref = oracle(int(p), K, False, 15, 4)
        same = True
        for k in range(K):
            assert g[k]['status'][p] == ref[k]['status'] == 0, (p, k)
            rec = sum(1 << (2 * t - 1) for t in ref[k]['ends'])  # converged sub-step ends t / 16: bit 2t - 1
            if dt == L.DT_F64:
                assert g[k]['sub'][p] == rec, (p, k)
                assert abs(int(g[k]['iters'][p]) - ref[k]['iters']) <= 2, (p, k)
            same = same and g[k]['sub'][p] == rec
            if not same:
                other += 1
                continue
            assert rel(g[k]['Pbar'][p], ref[k]['Pbar']) < tol_P, (p, k)
            assert rel(g[k]['Abar'][p], ref[k]['Abar'].reshape(-1)) < tol_A, (p, k)
    print(f"contraction {dt}: {other} of {len(SAMPLE) * K} sampled point-steps on another loading path")
    assert other <= 0.1 * len(SAMPLE) * K


def test_plain_step_failures_keep_committed_state(gpu):
    """Without cutting some steps of the workload fail; a failed point keeps
    its committed state, and the sampled failing points fail on the oracle too."""
    K = 4
    g = run_gpu(L.rom_default_opts(mode=L.MODE_FUSED), K)
    failed = np.flatnonzero(np.any([rec['status'] != 0 for rec in g], axis=0))
    print(f"points with a failed plain step in the first {K} steps: {failed.size}")
    assert failed.size > 0
    for p in failed[:6]:
        ref = oracle(int(p), K, False, 15)
        assert [g[k]['status'][p] for k in range(K)] == [ref[k]['status'] for k in range(K)], p


@pytest.mark.parametrize("dt", [L.DT_F64, L.DT_BF16])
def test_phased_matches_fused_bitwise_full_size(gpu, dt):
    """The phased form (material and contraction launches for the first
    evaluations, the fused kernel resuming the rest) gives the fused form's
    results bit for bit: same statuses (cut steps included), iteration counts,
    residuals, r, history, Pbar and Abar."""
    K = 6
    mu, paths = inputs(W)
    fu, ph = RomBatch(rom_path(W['rom']), mu), RomBatch(rom_path(W['rom']), mu)
    for k in range(K):
        print(f"[gpu] phased vs fused P={W['P']} contraction={dt} step {k}", flush=True)
        Fb = torch.from_numpy(np.ascontiguousarray(paths[:, k])).cuda()
        a = fu.step(Fb, L.rom_default_opts(mode=L.MODE_FUSED, contraction=dt, max_substeps=4))
        torch.cuda.synchronize()
        b = ph.step(Fb, L.rom_default_opts(mode=L.MODE_PHASED, contraction=dt, max_substeps=4))
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert torch.equal(x, y), k
        assert torch.equal(fu.Pbar, ph.Pbar) and torch.equal(fu.Abar, ph.Abar)
        assert torch.equal(fu.r(), ph.r()) and torch.equal(fu.r(trial=True), ph.r(trial=True))
        assert torch.equal(fu.history(), ph.history()) and torch.equal(fu.fbar_committed(), ph.fbar_committed())
    print(f"iterations in the last step: mean {b[1].double().mean().item():.3f}, max {b[1].max().item()}")
    fu.close()
    ph.close()


W4 = WORKLOADS['fourvoid_n100_m1500_P16384_cyclic20']
SAMPLE4 = [0, 5461, 10922, W4['P'] - 1, 1, 2047, 8191, 13000, 4095, 12288]


def run_gpu4(opts, K):
    mu, paths = inputs(W4)
    rb = RomBatch(rom_path(W4['rom']), mu)
    out = []
    for k in range(K):
        print(f"[gpu] four-void P={W4['P']} contraction={opts.contraction} fixed={opts.fixed_iters} step {k}",
              flush=True)
        st, it, rn = rb.step(torch.from_numpy(np.ascontiguousarray(paths[:, k])).cuda(), opts)
        torch.cuda.synchronize()
        out.append(dict(status=st.cpu().numpy()[SAMPLE4].copy(), iters=it.cpu().numpy()[SAMPLE4].copy(),
                        all_status=st.cpu().numpy().copy(),
                        r=rb.r(trial=True).cpu().numpy()[SAMPLE4].copy(), Pbar=rb.Pbar.cpu().numpy()[SAMPLE4].copy(),
                        Abar=rb.Abar.cpu().numpy()[SAMPLE4].copy()))
    rb.close()
    return out


@functools.lru_cache(maxsize=None)
def oracle4(p, K, fixed, max_iter):
    mu, paths = inputs(W4)
    return ROM(rom_path(W4['rom'])).run_path(mu[p], paths[p, :K], tol=1e-8, max_iter=max_iter, fixed=fixed)


def test_fourvoid_fixed_iteration_parity_full_size(gpu):
    """n = 100 (seven column tiles, the tile split of the waves), 16384 points."""
    K = 3
    g = run_gpu4(L.rom_default_opts(mode=L.MODE_FUSED, fixed_iters=1, max_iter=4), K)
    for i, p in enumerate(SAMPLE4):
        ref = oracle4(p, K, True, 4)
        for k in range(K):
            assert g[k]['status'][i] == ref[k]['status'], (p, k)
            assert rel(g[k]['r'][i], ref[k]['r']) < 1e-10, (p, k)
            assert rel(g[k]['Pbar'][i], ref[k]['Pbar']) < 1e-10, (p, k)
            assert rel(g[k]['Abar'][i], ref[k]['Abar'].reshape(-1)) < 1e-10, (p, k)


@pytest.mark.parametrize("dt,abar,tol_A", [(L.DT_F32, 0, 1e-4), (L.DT_BF16, 0, 3e-2), (L.DT_BF16, 1, 1e-5)])
def test_fourvoid_reduced_precision_full_size(gpu, dt, abar, tol_A):
    """FP32 / BF16 contraction at n = 100: converged to the same 1e-8 residual,
    Pbar within 1e-5 of the FP64 oracle, Abar within the dtype's bound (with
    abar_f64, the FP64 evaluation at the returned state runs the tile split)."""
    K = 3
    g = run_gpu4(L.rom_default_opts(mode=L.MODE_FUSED, contraction=dt, max_substeps=4, abar_f64=abar), K)
    assert all((rec['all_status'] == 0).mean() > 0.999 for rec in g)
    eP, eA = [], []
    for i, p in enumerate(SAMPLE4[:2]):
        ref = oracle4(p, K, False, 15)
        for k in range(K):
            assert g[k]['status'][i] == 0 and ref[k]['status'] == 0, (p, k)
            eP.append(rel(g[k]['Pbar'][i], ref[k]['Pbar']))
            eA.append(rel(g[k]['Abar'][i], ref[k]['Abar'].reshape(-1)))
    print(f"four-void contraction {dt}: max rel err Pbar {max(eP):.2e}, Abar {max(eA):.2e}")
    assert max(eP) < 1e-5
    assert max(eA) < tol_A


@pytest.mark.parametrize("mode", [L.MODE_FUSED, L.MODE_PHASED])
def test_abar_f64_refinement_full_size(gpu, mode):
    """abar_f64 changes Abar only: against the same BF16 step without it the
    statuses, evaluation counts, sub-step records, r and the committed state
    are equal bit for bit and Pbar to rounding.  Abar is then the FP64 one at
    the state the BF16 Newton loop returned: the oracle evaluated once at that
    r, from the committed history the step started from, agrees to 1e-10 at
    the sampled points whose full step converged (Abar of the plain BF16 step
    differs there by its contraction precision)."""
    K = 6
    mu, paths = inputs(W)
    rom = ROM(rom_path(W['rom']))
    a, b = RomBatch(rom_path(W['rom']), mu), RomBatch(rom_path(W['rom']), mu)
    plain = L.rom_default_opts(mode=mode, contraction=L.DT_BF16, max_substeps=4)
    refined = L.rom_default_opts(mode=mode, contraction=L.DT_BF16, max_substeps=4, abar_f64=1)
    worst, worst_plain, checked = 0.0, 0.0, 0
    for k in range(K):
        print(f"[gpu] abar_f64 mode={mode} P={W['P']} step {k}", flush=True)
        Fb = torch.from_numpy(np.ascontiguousarray(paths[:, k])).cuda()
        hist0 = b.history().cpu().numpy()[SAMPLE].copy()
        sa = [t.clone() for t in a.step(Fb, plain)]
        torch.cuda.synchronize()
        sb = [t.clone() for t in b.step(Fb, refined)]
        torch.cuda.synchronize()
        for x, y in zip(sa, sb):
            assert torch.equal(x, y), k
        assert torch.equal(a.substeps(), b.substeps())
        assert torch.equal(a.r(), b.r()) and torch.equal(a.r(trial=True), b.r(trial=True))
        assert torch.equal(a.history(), b.history()) and torch.equal(a.fbar_committed(), b.fbar_committed())
        assert torch.allclose(a.Pbar, b.Pbar, rtol=0, atol=1e-13 * a.Pbar.abs().max().item())
        st, sub = sb[0].cpu().numpy(), b.substeps().cpu().numpy().view(np.uint32)
        rt, Ab, Ap = b.r(trial=True).cpu().numpy(), b.Abar.cpu().numpy(), a.Abar.cpu().numpy()
        for i, p in enumerate(SAMPLE):
            if st[p] != 0 or sub[p] != 1 << 31:  # the full step converged: it started from hist0
                continue
            Finv, J = rom.transformation(mu[p])
            h = hist0[i]
            ref = rom.step(rt[p], (h[0:4].T.reshape(-1, 2, 2), h[4], h[5]), paths[p, k], Finv, J, max_iter=1,
                           fixed=True)['Abar'].reshape(-1)
            worst = max(worst, rel(Ab[p], ref))
            worst_plain = max(worst_plain, rel(Ap[p], ref))
            checked += 1
    print(f"Abar against the oracle at the returned state, {checked} point-steps: refined {worst:.2e}, "
          f"plain BF16 {worst_plain:.2e}")
    assert checked >= 0.5 * K * len(SAMPLE)
    assert worst < 1e-10
    assert worst_plain > 1e-6  # the comparison sees the BF16 contraction
    a.close()
    b.close()


def test_abar_f64_fused_equals_phased(gpu):
    K = 3
    mu, paths = inputs(W)
    fu, ph = RomBatch(rom_path(W['rom']), mu), RomBatch(rom_path(W['rom']), mu)
    for k in range(K):
        print(f"[gpu] abar_f64 fused vs phased step {k}", flush=True)
        Fb = torch.from_numpy(np.ascontiguousarray(paths[:, k])).cuda()
        fu.step(Fb, L.rom_default_opts(mode=L.MODE_FUSED, contraction=L.DT_BF16, max_substeps=4, abar_f64=1))
        ph.step(Fb, L.rom_default_opts(mode=L.MODE_PHASED, contraction=L.DT_BF16, max_substeps=4, abar_f64=1))
        torch.cuda.synchronize()
        assert torch.equal(fu.Pbar, ph.Pbar) and torch.equal(fu.Abar, ph.Abar), k
        assert torch.equal(fu.history(), ph.history()), k
    fu.close()
    ph.close()

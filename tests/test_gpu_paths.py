"""Every point of the benchmark's timed run, reduced-precision and learned
forms against plain FP64: the one-void ROM with n = 40 modes, 4096 macro
points, 20-step load / unload paths, load-step cutting depth 4, phased form,
as the benchmark times them.

A point-step that followed the plain FP64 loading path (the same converged
sub-steps since the start of the path) solves the same discrete problems as
the FP64 run: its Pbar must agree to 1e-5 of max |Pbar| (the reduced-precision
bound).  A point whose load steps are cut differently integrates the plastic
flow over other increments from then on; for a sample of those the oracle
solves the same sequence of increments (the sub-step targets the form
converged on, each solved from the previous one) and must agree with the form
at the end of every load step.  Where plain Newton from the committed state
does not reach an increment's solution (the learned start converged a full
step that the plain start cuts), the oracle reaches the same solution by
continuation: the load moved towards the target in quarters with the
committed history held fixed, nothing committed on the way, so the equations
solved at the end are the increment's own."""
import functools

import numpy as np
import pytest
import torch

import paper_2307_16894_amd as L
from bench import SUBSTEPS, WORKLOADS, inputs, same_path
from oracle.rom import ROM
from paper_2307_16894_amd.batch import RomBatch
from paper_2307_16894_amd.warmstart import WarmStart, generate
from tests.conftest import rom_path

pytestmark = pytest.mark.gpu

W = WORKLOADS['onevoid_n40_m400_P4096_cyclic20']
TOL_P = 1e-5


def run(opts):
    mu, paths = inputs(W)
    P, K = W['P'], W['steps']
    rb = RomBatch(rom_path(W['rom']), mu)
    Pb, sub, st = [], [], []
    for k in range(K):
        print(f"[gpu] paths P={P} contraction={opts.contraction} warm={opts.warm_start} step {k}", flush=True)
        s, _, _ = rb.step(torch.from_numpy(np.ascontiguousarray(paths[:, k])).cuda(), opts)
        torch.cuda.synchronize()
        Pb.append(rb.Pbar.cpu().numpy().copy())
        sub.append(rb.substeps().cpu().numpy().copy())
        st.append(s.cpu().numpy().copy())
    rb.close()
    return dict(Pbar=np.stack(Pb), sub=np.stack(sub), status=np.stack(st), K=K)


@functools.lru_cache(maxsize=None)
def plain_fp64():
    return run(L.rom_default_opts(mode=L.MODE_PHASED, max_substeps=SUBSTEPS))


@functools.lru_cache(maxsize=None)
def warm_start():
    """A network trained as the benchmark trains it, on fewer paths and epochs."""
    w = dict(W, P=4096)
    mu, paths = inputs(w, seed=W['train_seed'], P=4096)
    rb = RomBatch(rom_path(W['rom']), mu)
    X, Y = generate(rb, paths)
    rb.close()
    ws = WarmStart(X.shape[1], Y.shape[1], max_batch=4096, seed=0)
    ws.fit_scaling(X, Y)
    ws.train(X, Y, epochs=60, batch=2048, lr=4e-3, precision=L.DT_BF16)
    torch.cuda.synchronize()
    return ws


def solve_increment(rom, r_c, h_c, F_c, F_t, Finv, J):
    """The oracle's solution of one increment from the committed (r_c, h_c) at
    Fbar_c to Fbar_t: plain Newton, else continuation in the load with the
    committed history fixed."""
    s = rom.step(r_c, h_c, F_t, Finv, J, max_iter=40)
    if s['status'] == 0:
        return s
    r = r_c
    for t in (0.25, 0.5, 0.75, 1.0):
        s = rom.step(r, h_c, F_c + t * (F_t - F_c), Finv, J, max_iter=40)
        if s['status'] != 0:
            return s
        r = s['r']
    return s


def targets_of(path, subs):
    """The increments a run converged on for one point: per load step, the
    sub-step ends t / 16 of the segment from the committed Fbar (bit 2t - 1 of
    the record), the last one the step's own Fbar."""
    out, Fc = [], np.eye(2)
    full = 2 ** SUBSTEPS
    for k, rec in enumerate(subs):
        ends = [t for t in range(1, full + 1) if (int(rec) >> (2 * t - 1)) & 1]
        assert ends and ends[-1] == full, (k, hex(int(rec)))
        F = np.asarray(path[k])
        out += [F if t == full else Fc + (t / full) * (F - Fc) for t in ends]
        Fc = F
    return out


@pytest.mark.parametrize("form", ['bf16_phased', 'bf16_mlp_phased'])
def test_every_point_against_plain_fp64(gpu, form):
    ref = plain_fp64()
    assert (ref['status'] == 0).all()
    if '_mlp' in form:
        opts = warm_start().opts(contraction=L.DT_BF16, max_substeps=SUBSTEPS, mode=L.MODE_PHASED)
    else:
        opts = L.rom_default_opts(mode=L.MODE_PHASED, contraction=L.DT_BF16, max_substeps=SUBSTEPS)
    g = run(opts)
    assert np.isin(g['status'], (L.ST_CONVERGED, L.ST_FALLBACK)).all()
    same = same_path(g, ref)
    scale = np.abs(ref['Pbar']).max()
    dev = np.abs(g['Pbar'] - ref['Pbar']).max(axis=-1) / scale
    other = np.flatnonzero((~same).any(axis=0))
    print(f"{form}: same-path max {dev[same].max():.2e} median {np.median(dev[same]):.2e}; "
          f"other path {(~same).mean():.4f} of point-steps, {other.size} points, max {dev.max():.2e}")
    assert dev[same].max() <= TOL_P
    assert (~same).mean() < 0.05
    # points on another path: the oracle along the increments the form converged on
    mu, paths = inputs(W)
    rom = ROM(rom_path(W['rom']))
    checked, sampled = 0, other[:6]
    for p in sampled:
        k1 = min(g['K'], int(np.flatnonzero(~same[:, p])[0]) + 3)
        T = targets_of(paths[p, :k1], g['sub'][:k1, p])
        Finv, J = rom.transformation(mu[p])
        r, h, Fc = np.zeros(rom.n), rom.virgin(), np.eye(2)
        refs, solved = [], True
        for Ft in T:
            st = solve_increment(rom, r, h, Fc, np.asarray(Ft), Finv, J)
            if st['status'] != 0:
                solved = False
                break
            refs.append(st)
            r, h, Fc = st['r'], st['hist'], np.asarray(Ft)
        if not solved:
            print(f"point {p}: the oracle does not reach every increment's solution; not checked")
            continue
        ends = np.cumsum([bin(int(rec) & 0xFFFFFFFF).count('1') for rec in g['sub'][:k1, p]]) - 1
        for k, e in enumerate(ends):
            d = np.abs(g['Pbar'][k, p] - refs[e]['Pbar']).max() / scale
            assert d <= TOL_P, (p, k, d)
        checked += 1
    print(f"{form}: {checked} of {sampled.size} points on another path checked against the oracle")
    assert 2 * checked >= sampled.size

"""Parity at the tile counts the benchmark ROMs leave out: n = 50 (four column
tiles) and n = 80 (six) as the leading modes of the four-void n = 100 ROM (a
truncated POD basis keeps the same ECM rule, which integrates the smaller
span as well), and the full four-void n = 60 (five tiles) and n = 120 (eight,
the widest the kernels are built for) ROMs, and n = 28, 44, 45, 60, 63, 95
(n mod 16 >= 12, where the rows and columns carrying the residual, the
effective stress and stiffness start at the next tile boundary, so that they
lie in the last tile).  Fixed-iteration FP64 parity with the oracle for the
fused form with each wave split it supports and for the phased form (up to
five tiles); at n = 120, 28, 44, 45, 60 and 63 also the reduced-precision
contractions, solved to 1e-8 and compared on the effective stress."""
import functools
import os

import numpy as np
import pytest
import torch

import workloads
from oracle import artifact
from oracle.rom import ROM
from tests.conftest import rom_path

import paper_2307_16894_amd as L
from paper_2307_16894_amd.batch import RomBatch

pytestmark = pytest.mark.gpu

P, K, IT = 2, 2, 3
CASES = [('fourvoid_n100_m1500', 50), ('fourvoid_n60_m800', None), ('fourvoid_n100_m1500', 80),
         ('fourvoid_n120_m2000', None),
         # n mod 16 >= 12: the padding block starts at the next tile boundary
         ('fourvoid_n100_m1500', 45), ('fourvoid_n100_m1500', 63), ('fourvoid_n100_m1500', 95),
         ('fourvoid_n100_m1500', 28), ('fourvoid_n100_m1500', 44)]


@pytest.fixture(scope='module')
def roms(tmp_path_factory):
    tmp = tmp_path_factory.mktemp('roms')
    out = {}
    for name, n in CASES:
        if n is None:
            out[(name, n)] = rom_path(name)
            continue
        a = artifact.read(rom_path(name))
        path = str(tmp / f'{name}_first{n}.rom')
        artifact.write(path, n, a['m'], a['c'], a['kind'], a['n_mu'], a['mat'], a['r0'], a['void_area'],
                       a['cell_area'], a['w'], np.ascontiguousarray(a['G'][:, :, :n]), a['Gd'], a['src'])
        out[(name, n)] = path
    return out


def inputs(seed):
    # small monotone increments: every plain Newton step converges from the virgin state
    return workloads.four_void_mu(seed, P), workloads.monotone_paths(seed, P, K, (0.01, 0.02))


@functools.lru_cache(maxsize=None)
def oracle_run(path, seed, fixed, max_iter):
    mu, paths = inputs(seed)
    rom = ROM(path)
    return [rom.run_path(mu[p], paths[p], tol=1e-8, max_iter=max_iter, fixed=fixed) for p in range(P)]


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


def forms(n):
    T = L.rom_fused_tiles(n)
    out = [('fused', dict(mode=L.MODE_FUSED))]
    if T <= 5:  # the point split is the automatic one here; the tile split on request
        out.append(('fused_tilesplit', dict(mode=L.MODE_FUSED, split=1)))
        out.append(('phased', dict(mode=L.MODE_PHASED, phased_evals=2)))
    return out


@pytest.mark.parametrize("case", range(len(CASES)))
def test_fixed_iteration_parity_every_tile_count(gpu, roms, case):
    path = roms[CASES[case]]
    seed = 60 + case
    mu, paths = inputs(seed)
    refs = oracle_run(path, seed, True, IT)
    n = artifact.read(path)['n']
    for form, kw in forms(n):
        rb = RomBatch(path, mu)
        for k in range(K):
            print(f"[gpu] tiles n={n} form={form} step {k}", flush=True)
            st, it, _ = rb.step(torch.from_numpy(np.ascontiguousarray(paths[:, k])).cuda(),
                                L.rom_default_opts(fixed_iters=1, max_iter=IT, **kw))
            torch.cuda.synchronize()
            st, r, Pb, Ab = st.cpu().numpy(), rb.r(trial=True).cpu().numpy(), rb.Pbar.cpu().numpy(), \
                rb.Abar.cpu().numpy()
            for p in range(P):
                s = refs[p][k]
                assert st[p] == s['status'], (n, form, p, k)
                assert rel(r[p], s['r']) < 1e-10, (n, form, p, k, rel(r[p], s['r']))
                assert rel(Pb[p], s['Pbar']) < 1e-10, (n, form, p, k)
                assert rel(Ab[p], s['Abar'].reshape(-1)) < 1e-10, (n, form, p, k)
        rb.close()


@pytest.mark.parametrize("case,prec", [(3, L.DT_BF16), (4, L.DT_BF16), (4, L.DT_F32), (5, L.DT_BF16),
                                       (1, L.DT_BF16), (7, L.DT_BF16), (7, L.DT_F32), (8, L.DT_BF16)])
def test_reduced_precision_contraction(gpu, roms, case, prec):
    """n = 120 (the widest) and n = 28, 44, 45, 60, 63 (padding at the next
    tile boundary): the BF16 / FP32 contraction (point split, FP32
    accumulators) solved to 1e-8 like the oracle; effective stress within
    1e-5.  Where the FP64 oracle's plain Newton step fails (the n = 120 ROM,
    point 0, second step: the residual grows from 4e-3 to 1.2e-2 over the 15
    evaluations) the reduced-precision step must fail too."""
    path = roms[CASES[case]]
    n = artifact.read(path)['n']
    seed = 70 + case
    mu, paths = inputs(seed)
    refs = oracle_run(path, seed, False, 15)
    rb = RomBatch(path, mu)
    converged = 0
    for k in range(K):
        print(f"[gpu] tiles n={n} precision {prec} step {k}", flush=True)
        st, it, _ = rb.step(torch.from_numpy(np.ascontiguousarray(paths[:, k])).cuda(),
                            L.rom_default_opts(mode=L.MODE_FUSED, contraction=prec))
        torch.cuda.synchronize()
        st, Pb = st.cpu().numpy(), rb.Pbar.cpu().numpy()
        for p in range(P):
            if refs[p][k]['status'] != 0:
                assert st[p] != 0, (p, k)
                continue
            converged += 1
            assert st[p] == 0, (p, k)
            assert rel(Pb[p], refs[p][k]['Pbar']) < 1e-5, (p, k, rel(Pb[p], refs[p][k]['Pbar']))
    rb.close()
    assert converged >= P * K - 1

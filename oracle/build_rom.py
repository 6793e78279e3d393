"""Offline stage of Algorithm 1: build ROM artifacts from full-order solves.

    python -m oracle.build_rom <name> [--workers K]

Steps (Algorithm 1, offline): parent mesh; auxiliary transformation modes;
training parameters from a scrambled Sobol design and seeded load paths;
full-order solves collecting fluctuation and weighted-stress snapshots; POD of
both; ECM on the products of the two bases; the artifact.  A JSON report
beside the artifact records the settings, the POD spectra, the ECM residual
and the ROM-vs-FOM error on held-out paths (eps_P of Sec. 4).

Settings that the paper leaves open and that are chosen here: the number of
weighted-stress modes L and the ECM stop rule (tolerance or a target point
count m, whichever comes first), listed per ROM below.
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

import workloads
from . import artifact, auxiliary, ecm, fem, fom, mesh as meshmod, pod
from .rom import ROM

MAT = (1.0, 0.3, 0.01, 0.05)  # E, nu, sigma_y0, H

ROMS = {
    # one centred void, mu = (a, b) in [0.15, 0.35]^2, ~1.2k T6
    'onevoid_n20_m120': dict(kind=0, r0=0.25, nt=15, nr=10, n=20, L=7, m=120, eps=1e-3,
                             n_mu=8, per_mu=3, path='monotone', steps=10, rho=(0.02, 0.05),
                             seed=1000),
    # same family, ~8k T6
    'onevoid_n40_m400': dict(kind=0, r0=0.25, nt=40, nr=25, n=40, L=11, m=400, eps=1e-3,
                             n_mu=16, per_mu=3, path='cyclic', steps=20, rho=(0.02, 0.08),
                             seed=2000),
}

# two phases: the one-void cell whose void is lined with a stiff elastic
# coating (every point of the parent cell within `coating` of the void
# boundary), ten times the matrix modulus and no yield in range
ROMS['coatvoid_n20_m120'] = dict(ROMS['onevoid_n20_m120'], coating=0.06, mat2=(10.0, 0.3, 1.0e3, 0.0), seed=1500)

# four elliptical voids of fixed area 0.075 each (porosity 0.3), parent circles
# of equal area; mu = (kappa_i, theta_i) per void; ~30k T6.  The three ROMs
# share mesh and training data (so they can share a snapshot cache).
_FOUR = dict(kind=1, r0=float(np.sqrt(0.075 / np.pi)), void_area=0.075, nt=32, nr=29, n_mu=16, per_mu=3,
             path='cyclic', steps=20, rho=(0.02, 0.08), seed=3000, eps=1e-4)
ROMS['fourvoid_n100_m1500'] = dict(_FOUR, n=100, L=16, m=1500)
ROMS['fourvoid_n60_m800'] = dict(_FOUR, n=60, L=15, m=800)
ROMS['fourvoid_n120_m2000'] = dict(_FOUR, n=120, L=19, m=2000)

# the composite cell of Sec. 4.1: 23 random elliptical inclusions (23.4 % of
# the cell at zeta = 1) ten times stiffer than the matrix and elastic in
# range, mu = (zeta) in [0.5, 1.2] scaling every inclusion about its centre;
# structured 40 x 40 mesh (3200 T6), inclusions resolved to the element size;
# 16 training zeta x 3 cyclic paths
ROMS['inclusions_n30_m250'] = dict(kind=2, nx=40, layout_seed=5, r0=0.0, n=30, L=12, m=250, eps=1e-4, n_mu=16,
                                   per_mu=3, path='cyclic', steps=20, rho=(0.02, 0.05), seed=4100,
                                   mat2=(10.0, 0.3, 1.0e3, 0.0))

_G = {}


def _geometry(spec):
    if spec['kind'] == 0:
        m = meshmod.one_void_cell(spec['r0'], spec['nt'], spec['nr'])
    elif spec['kind'] == 1:
        m = meshmod.four_void_cell(spec['r0'], spec['nt'], spec['nr'])
    else:
        m = meshmod.inclusion_cell(spec['nx'], workloads.inclusion_layout(spec['layout_seed']))
    space = fem.PeriodicSpace(m)
    ax = auxiliary.AuxiliaryProblem(m, spec['kind'])
    grad_modes = ax.gradients(ax.modes())  # (c, nq, 2, 2)
    return m, space, grad_modes


def phases(spec, m):
    """Phase of every quadrature point of the parent mesh: 1 in the coating
    around the (centred) void or in an inclusion, 0 in the matrix."""
    if spec['kind'] == 2:
        return m.qphase.copy()
    if 'coating' not in spec:
        return np.zeros(m.nq, dtype=np.int64)
    d = np.hypot(m.qX[:, 0] - 0.5, m.qX[:, 1] - 0.5)
    return (d < spec['r0'] + spec['coating']).astype(np.int64)


def material(spec, m):
    """Material constants at every quadrature point (scalars for one phase)."""
    ph = phases(spec, m)
    if not ph.any():
        return MAT
    return tuple(np.where(ph == 1, b, a) for a, b in zip(MAT, spec['mat2']))


def _mu_coeff(spec, mu):
    return auxiliary.coefficients(spec['kind'], mu, spec['r0'], spec.get('void_area'))


def _fom_job(args):
    spec, mu, path = args
    m, space, grad_modes = _G['geom']
    Fmu = auxiliary.transformation(grad_modes, _mu_coeff(spec, mu))
    pr = fem.Problem(m, space, Fmu, material(spec, m))
    res = fom.solve_path(pr, path, tol=1e-10 * max(1.0, 1.0), want_W=True)
    return np.array(res.w), np.array(res.W), np.array(res.Pbar), res.iters


def _paths(spec, seed, count):
    if spec['path'] == 'monotone':
        return workloads.monotone_paths(seed, count, spec['steps'], spec['rho'])
    return workloads.cyclic_paths(seed, count, spec['steps'], spec['rho'])


def _training_mu(spec, seed, count):
    if spec['kind'] == 0:
        return workloads.one_void_training_mu(seed, count)
    if spec['kind'] == 2:
        return workloads.inclusion_training_mu(seed, count)
    return workloads.four_void_training_mu(seed, count)


def _test_mu(spec, seed, count):
    return {0: workloads.one_void_mu, 1: workloads.four_void_mu, 2: workloads.inclusion_mu}[spec['kind']](seed, count)


def build(name, outdir, workers, snapshot_cache=None, overrides=None, pod_fn=None, ecm_fn=None, heldout=True):
    """Offline stage of Algorithm 1 for the ROM `name`: training FOM solves,
    POD of the fluctuations and of the weighted stress, the ECM rule, the
    artifact, and (heldout) the ROM's error on held-out FOM paths.  pod_fn and
    ecm_fn stand in for pod.pod and ecm.greedy (same arguments and results),
    so that a caller can build the same ROM with another implementation of
    those two steps; by default the ones of this package."""
    pod_fn = pod_fn or pod.pod
    ecm_fn = ecm_fn or ecm.greedy
    spec = dict(ROMS[name])
    spec.update(overrides or {})
    t0 = time.time()
    geom = _geometry(spec)
    _G['geom'] = geom
    m, space, grad_modes = geom
    print(f"[{name}] mesh: {m.nn} nodes, {m.ne} T6, {m.nq} points, {space.ndof} dofs", flush=True)
    mus = _training_mu(spec, spec['seed'], spec['n_mu'])
    paths = _paths(spec, spec['seed'] + 1, spec['n_mu'] * spec['per_mu'])
    jobs = [(spec, mus[i // spec['per_mu']], paths[i]) for i in range(len(paths))]
    if snapshot_cache and os.path.exists(snapshot_cache):
        z = np.load(snapshot_cache)
        Sw, SW, fom_iters = z['Sw'], z['SW'], float(z['fom_iters'])
    else:
        with mp.get_context('fork').Pool(workers) as pool:
            results = pool.map(_fom_job, jobs, chunksize=1)
        Sw = np.concatenate([r[0] for r in results]).T  # (ndof, ns)
        SW = np.concatenate([r[1] for r in results]).T  # (4 nq, ns)
        fom_iters = float(np.mean([np.mean(r[3]) for r in results]))
        if snapshot_cache:
            np.savez(snapshot_cache, Sw=Sw, SW=SW, fom_iters=fom_iters)
    print(f"[{name}] {len(jobs)} training solves done in {time.time() - t0:.1f}s", flush=True)
    # POD of the fluctuations in V^p and of the weighted stress in L^2(parent)
    Fid = auxiliary.transformation(grad_modes, np.zeros(grad_modes.shape[0]))
    pr0 = fem.Problem(m, space, Fid, MAT)
    MV = pod.v_gram(pr0)
    Phi, lam_w = pod_fn(Sw, MV, spec['n'])
    B, lam_W = pod_fn(SW, np.repeat(m.qw, 4), spec['L'])
    Gfull = (pr0.Gop @ Phi).reshape(m.nq, 4, spec['n'])
    Bq = B.reshape(m.nq, 4, spec['L'])
    J = ecm.integrand_matrix(Gfull, Bq, spec['n'], spec['L'])
    J = np.vstack([J, np.ones((1, m.nq))])  # constant integrand: parent area (build's addition)
    idx, wq, hist = ecm_fn(J, m.qw, spec['eps'], spec['m'])
    print(f"[{name}] ECM: {idx.size} points, relative residual {hist[-1]:.3e}", flush=True)
    order = np.argsort(idx)
    idx, wq = idx[order], wq[order]
    Gd = np.stack([g.reshape(m.nq, 4)[idx] for g in grad_modes], axis=-1)  # (m, 4, c)
    path = os.path.join(outdir, name + '.rom')
    n_mu = {0: 2, 1: 8, 2: 1}[spec['kind']]
    ph = phases(spec, m)
    two = bool(ph.any())
    artifact.write(path, spec['n'], idx.size, grad_modes.shape[0], spec['kind'], n_mu, MAT,
                   spec['r0'], spec.get('void_area', 0.0), 1.0, wq, Gfull[idx], Gd, idx,
                   mat2=spec['mat2'] if two else None, phase=ph[idx] if two else None)
    # ROM quality on held-out paths (not a parity check)
    rom = ROM(path)
    test_mu = _test_mu(spec, spec['seed'] + 7, 4)
    test_paths = _paths(spec, spec['seed'] + 8, 4)
    ref = []
    if heldout:
        with mp.get_context('fork').Pool(workers) as pool:
            ref = pool.map(_fom_job, [(spec, test_mu[i], test_paths[i]) for i in range(4)])
    errs = []
    for i in range(len(ref)):
        out = rom.run_path(test_mu[i], test_paths[i])
        Pr = np.array([o['Pbar'] for o in out])
        Pf = ref[i][2].reshape(-1, 4)
        errs.append(float(np.sum(np.linalg.norm(Pr - Pf, axis=1)) / np.sum(np.linalg.norm(Pf, axis=1))))
    report = dict(name=name, spec={k: (list(v) if isinstance(v, tuple) else v) for k, v in spec.items()},
                  mesh=dict(nodes=m.nn, elements=m.ne, points=m.nq, dofs=space.ndof),
                  snapshots=int(Sw.shape[1]), pod_w_energy_kept=float(lam_w[:spec['n']].sum() / lam_w[lam_w > 0].sum()),
                  pod_W_energy_kept=float(lam_W[:spec['L']].sum() / lam_W[lam_W > 0].sum()),
                  ecm_points=int(idx.size), ecm_residual=float(hist[-1]), ecm_weight_sum=float(wq.sum()),
                  parent_area=float(m.qw.sum()), heldout_eps_P=errs,
                  fom_iters_mean=fom_iters,
                  build_seconds=time.time() - t0)
    with open(os.path.join(outdir, name + '.json'), 'w') as fh:
        json.dump(report, fh, indent=1)
    print(json.dumps(report, indent=1), flush=True)
    return path


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument('names', nargs='+')
    ap.add_argument('--out', default=os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), 'roms'))
    ap.add_argument('--workers', type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument('--snapshots', default=None, help='npz file caching the training snapshots')
    ap.add_argument('--L', type=int, default=None, help='override the number of weighted-stress modes')
    a = ap.parse_args(argv)
    os.makedirs(a.out, exist_ok=True)
    for n in a.names:
        build(n, a.out, a.workers, a.snapshots, {'L': a.L} if a.L else None)


if __name__ == '__main__':
    sys.exit(main())

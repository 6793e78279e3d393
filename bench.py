#!/usr/bin/env python3
"""Throughput of the batched hyper-reduced RVE solve on one MI355X.

One step = one load step of every macro point of the batch: rom_step (Newton
on the reduced coordinates to ||f||_2 <= 1e-8, then effective stress and
stiffness) and rom_homogenized_stress_tangent.  The metric is macro-point load
steps per second with all inputs resident in device memory, for the
learned + mixed-precision form (BF16 contraction of the reduced tangent, FP64
everywhere else, learned Newton warm start) next to the plain FP64 form at
the same 1e-8 residual; the other forms are reported beside them.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--variants a,b]

Prints one JSON line.  The dominant kernel is reported against the MI355X
FP64 peak (timed with HIP events on the stream the kernel runs on), and the
plain FP64 CPU oracle is timed on a bounded sample of the same workload on the
host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402


WORKLOADS = {
    # one elliptical void, n = 40 modes, m ~ 400 ECM points, 4096 points,
    # 20-step load / unload paths of amplitude <= 0.08
    'onevoid_n40_m400_P4096_cyclic20': dict(rom='onevoid_n40_m400', cell='onevoid', P=4096, steps=20,
                                            path='cyclic', rho=(0.02, 0.08), seed=0, train_points=25000,
                                            train_seed=1, timed=20, warm=20,
                                            variants=['fp64', 'fp64_phased', 'fp64_staged', 'fp32_phased', 'bf16',
                                                      'bf16_phased', 'fp64_mlp_phased', 'fp32_mlp_phased',
                                                      'bf16_mlp', 'bf16_mlp_phased', 'bf16_mlp_a64_phased']),
    # small case: n = 20, m = 120, 64 points, 10-step monotone paths
    'onevoid_n20_m120_P64_monotone10': dict(rom='onevoid_n20_m120', cell='onevoid', P=64, steps=10,
                                            path='monotone', rho=(0.02, 0.05), seed=0, train_points=4096,
                                            train_seed=1, timed=20, warm=20,
                                            variants=['fp64', 'fp64_phased', 'fp64_staged', 'fp32_phased',
                                                      'bf16_phased']),
    # four elliptical voids (mu in R^8), n = 100 modes, m ~ 1500 ECM points,
    # 16384 points, 20-step load / unload paths: the reduced-precision contraction
    'fourvoid_n100_m1500_P16384_cyclic20': dict(rom='fourvoid_n100_m1500', cell='fourvoid', P=16384, steps=20,
                                                path='cyclic', rho=(0.02, 0.08), seed=0, timed=3, warm=1,
                                                variants=['fp64', 'fp32', 'bf16', 'bf16_a64']),
    # two phases: the n = 20 one-void cell lined with a stiff elastic coating,
    # 16384 points, 10-step monotone paths; beside it the single-phase cell
    # at the same size (the cost of a material per ECM point)
    'coatvoid_n20_m120_P16384_monotone10': dict(rom='coatvoid_n20_m120', cell='onevoid', P=16384, steps=10,
                                                path='monotone', rho=(0.02, 0.05), seed=0, timed=10, warm=10,
                                                variants=['fp64', 'fp64_phased', 'bf16_phased']),
    'onevoid_n20_m120_P16384_monotone10': dict(rom='onevoid_n20_m120', cell='onevoid', P=16384, steps=10,
                                               path='monotone', rho=(0.02, 0.05), seed=0, timed=10, warm=10,
                                               variants=['fp64', 'fp64_phased', 'bf16_phased']),
}
# uneven persistent batch: several ROMs in one captured step, per-point step
# counts U[5, 40], Newton cap 15 per step; the points are shared out by cost
UNEVEN = {'uneven_mixed_P32768': dict(
    roms=[('onevoid_n20_m120', 12288), ('onevoid_n40_m400', 10240), ('fourvoid_n60_m800', 6144),
          ('fourvoid_n100_m1500', 2048), ('fourvoid_n120_m2000', 2048)],
    steps=(5, 40), rho=(0.01, 0.04), seed=0, max_iter=15, tune_points=1024)}
DEFAULT = 'onevoid_n40_m400_P4096_cyclic20'
EXTRA_N100, EXTRA_UNEVEN = 'fourvoid_n100_m1500_P16384_cyclic20', 'uneven_mixed_P32768'
VARIANTS = WORKLOADS[DEFAULT]['variants']
# warm-start training: 160 epochs of minibatch Adam, cosine-decayed from 4e-3
# (measured on the n = 40 workload: 3.20 Newton evaluations per point-step,
# 3.24 after 80 epochs, 3.29 after 40; training is set-up, not timed)
WS_EPOCHS = 160
PBAR_TOL = 1e-5  # reduced-precision forms: largest admitted |Pbar - Pbar_FP64| / max |Pbar_FP64|
# counted floating-point operations per ECM point and evaluation
# (paper_2307_16894_amd/flop_count.py, the smallest over the return map's
# branches; each transcendental call counted once): the return map with its
# consistent tangent, and the weighting D = w|J| T^T A T, W = w|J| P F_mu^-T
C_CM, C_W = 559, 144
PEAK = {'f64': 78.6, 'f32': 157.3, 'bf16': 2500.0}  # MI355X dense TFLOP/s: FP64 (vector = matrix), FP32 MFMA, BF16
HBM_TBS = 8.0
SUBSTEPS = 4  # load-step cutting depth of the fused forms: a failed step is retried in up to 1/16 strides
MAX_ITER = 15  # Newton evaluations per attempt (the library's default cap)


def inputs(w, seed=None, P=None):
    P = w['P'] if P is None else P
    seed = w['seed'] if seed is None else seed
    K = w['steps']
    mu = workloads.one_void_mu(seed, P) if w['cell'] == 'onevoid' else workloads.four_void_mu(seed, P)
    if w['path'] == 'cyclic':
        paths = workloads.cyclic_paths(seed, P, K, w['rho'])
    else:
        paths = workloads.monotone_paths(seed, P, K, w['rho'])
    return mu, paths


def train_warm_start(w, rom_file, log):
    """Samples from FP64 ROM trajectories, then the library's own training kernels."""
    import torch
    from paper_2307_16894_amd.batch import RomBatch
    from paper_2307_16894_amd.warmstart import WarmStart, generate
    import paper_2307_16894_amd as L
    t0 = time.perf_counter()
    mu, paths = inputs(w, seed=w['train_seed'], P=w['train_points'])
    rb = RomBatch(rom_file, mu)
    X, Y = generate(rb, paths)
    rb.close()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ws = WarmStart(X.shape[1], Y.shape[1], max_batch=4096, seed=0)
    ws.fit_scaling(X, Y)
    hist = ws.train(X, Y, epochs=WS_EPOCHS, batch=2048, lr=4e-3, precision=L.DT_BF16)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    log(f"warm start: {X.shape[0]} samples in {t1 - t0:.1f}s, trained in {t2 - t1:.1f}s, "
        f"loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    return ws, dict(samples=int(X.shape[0]), params=int(ws.param_count), epochs=WS_EPOCHS,
                    loss_first=hist[0], loss_last=hist[-1], gen_s=t1 - t0, train_s=t2 - t1)


def gpu_run(w, steps, warmup, opts, rom_file):
    import torch
    import paper_2307_16894_amd as L
    from paper_2307_16894_amd.batch import RomBatch
    mu, paths = inputs(w)
    P, K = w['P'], w['steps']
    dev = torch.device('cuda:0')
    Fb = torch.from_numpy(np.ascontiguousarray(paths.reshape(P, K, 4).transpose(1, 0, 2))).to(dev)  # [K][P][4]
    rb = RomBatch(rom_file, mu, dev)
    n, m = rb.info['n'], rb.info['m']

    def run(nsteps, record):
        k = 0
        rec = []
        for _ in range(nsteps):
            if k == K:  # the path is cycled from the virgin state
                L.rom_state_init(rb.h, P, rb.mu.data_ptr(), rb.state.data_ptr(), rb.stream.cuda_stream)
                k = 0
            rb.step(Fb[k], opts)
            if record:  # device-side copies, no synchronisation
                rec.append((rb.iters.clone(), (rb.status == 0).sum() + (rb.status == 3).sum(), rb.Pbar.clone(),
                            rb.substeps().clone(), rb.Abar.clone()))
            k += 1
        return rec

    L.rom_state_init(rb.h, P, rb.mu.data_ptr(), rb.state.data_ptr(), rb.stream.cuda_stream)
    # the warm-up records too, so that the timed steps find the memory of their
    # device-side copies in torch's cache instead of allocating it
    run(warmup, True)
    torch.cuda.synchronize()
    L.rom_state_init(rb.h, P, rb.mu.data_ptr(), rb.state.data_ptr(), rb.stream.cuda_stream)
    L.rom_timing_enable(rb.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rec = run(steps, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, launches = L.rom_timing_read(rb.h)
    L.rom_timing_enable(rb.h, False)
    evals = int(sum(int(r[0].sum()) for r in rec))
    conv = int(sum(int(r[1]) for r in rec))
    max_it = int(max(int(r[0].max()) for r in rec))
    Pbars = torch.stack([r[2] for r in rec]).cpu().numpy()
    subs = torch.stack([r[3] for r in rec]).cpu().numpy()
    Abars = torch.stack([r[4] for r in rec]).cpu().numpy()
    rb.close()
    return dict(elapsed=t1 - t0, evals=evals, converged=conv, max_iter=max_it, kern_ms=kern_ms,
                launches=launches, n=n, m=m, Pbar=Pbars, Abar=Abars, sub=subs, K=K)


def same_path(g, ref):
    """[steps][P] mask of the point-steps whose loading path so far equals the
    reference run's: every (sub-)step of the point since the start of its path
    ended at the same fractions of its load steps (the sub-step records agree),
    so both runs solved the same sequence of discrete problems."""
    agree = g['sub'] == ref['sub']
    same = np.empty_like(agree)
    for k in range(agree.shape[0]):
        same[k] = agree[k] if k % g['K'] == 0 else (same[k - 1] & agree[k])
    return same


def sensitivity_rate(w, rom_file, at_step=5, reps=5):
    """Shape sensitivities dPbar/dmu of the whole batch after a trial step:
    the batch is driven (fused FP64, cutting) through the first at_step load
    steps, then a trial step (no commit) to the next one; the sensitivity call
    is timed with HIP events on its stream."""
    import torch
    import paper_2307_16894_amd as L
    from paper_2307_16894_amd.batch import RomBatch
    mu, paths = inputs(w)
    rb = RomBatch(rom_file, mu)
    for k in range(at_step + 1):
        o = L.rom_default_opts(mode=L.MODE_FUSED, max_substeps=SUBSTEPS if k < at_step else 0, commit=int(k < at_step))
        rb.step(torch.from_numpy(np.ascontiguousarray(paths[:, k])).cuda(), o)
    Fb = torch.from_numpy(np.ascontiguousarray(paths[:, at_step])).cuda()
    S = rb.shape_sensitivity(Fb)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(rb.stream)
        S = rb.shape_sensitivity(Fb)
        e1.record(rb.stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    finite = bool(torch.isfinite(S).all())
    rb.close()
    ms = float(np.median(times))
    return dict(value=w['P'] / (ms * 1e-3), unit="macro points/s", ms_per_call=ms, n_mu=int(S.shape[2]),
                after_steps=at_step, all_finite=finite)


FE2_MESH, FE2_STEPS, FE2_PEAK = (20, 10), 50, 0.012


def fe2_compliance_error(mode):
    """The compliance error of the GPU two-scale loop with the n = 20 ROM
    against the full-order two-scale reference stored in
    tests/golden/fe2_fom_4x2.json (4 x 2 block, eight load steps up to the
    peak and back; Sec. 4.2): eps_C,k = |C_k - C_k^ref| / |C_k^ref| per
    loaded step and its mean."""
    from paper_2307_16894_amd.fe2 import Fe2Solver
    with open(os.path.join(ROOT, 'tests', 'golden', 'fe2_fom_4x2.json')) as fh:
        ref = json.load(fh)
    mesh = workloads.fe2_mesh(*ref['macro_mesh'])
    loads = workloads.fe2_loads(ref['load_steps'], ref['peak_traction'])
    sol = Fe2Solver(os.path.join(ROOT, 'roms', ref['cell'] + '.rom'), mesh,
                    lambda X: workloads.fe2_shape(X[:, 0], X[:, 1]), mode=mode)
    out = sol.run(loads)
    sol.close()
    C, Cr = np.array([o['C'] for o in out]), np.array(ref['compliance'])
    loaded = np.asarray(loads) > 0
    eps = np.abs(C[loaded] - Cr[loaded]) / np.abs(Cr[loaded])
    return dict(workload=f"fe2_q8_{ref['macro_mesh'][0]}x{ref['macro_mesh'][1]}_K{ref['load_steps']}",
                rom=ref['cell'], reference="full-order RVE at every macro point (oracle, stored)",
                converged_steps=int(sum(o['status'] == 0 for o in out)), eps_C=[float(e) for e in eps],
                eps_C_mean=float(eps.mean()))


def fe2_rate(rom_file, mode):
    """The two-scale example: a 2 x 1 block of 20 x 10 eight-node elements
    (800 RVE points, 1322 dofs), bottom fixed, parabolic top traction up to
    FE2_PEAK over 25 steps and back to zero over 25; void shape fields over
    the block.  Whole-run wall time of the macro Newton loop (trial and
    commit RVE solves, assembly, banded solves, one host read-back per macro
    iteration)."""
    import torch
    import workloads
    from paper_2307_16894_amd.fe2 import Fe2Solver
    mesh = workloads.fe2_mesh(*FE2_MESH)
    sol = Fe2Solver(rom_file, mesh, lambda X: workloads.fe2_shape(X[:, 0], X[:, 1]), mode=mode)
    loads = workloads.fe2_loads(FE2_STEPS, FE2_PEAK)
    sol.load_step(0.0)  # warm-up: one converged step at zero load (the virgin state)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = sol.run(loads)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    info = sol.info
    sol.close()
    ok = sum(r['status'] == 0 for r in res)
    C = [r['C'] for r in res]
    return dict(workload=f"fe2_q8_{FE2_MESH[0]}x{FE2_MESH[1]}_P{info['points']}_K{FE2_STEPS}",
                value=len(res) / dt, unit="macro load steps/s", seconds=dt, load_steps=len(res),
                converged_steps=ok, macro_iters=sum(r['macro_iters'] for r in res),
                rve_point_evals=sum(r['rve_evals'] for r in res), dofs=info['dofs'], points=info['points'],
                band_kl=info['kl'], peak_traction=FE2_PEAK, max_compliance=max(C))


POD_SIZE = (32316, 960, 40)   # dofs of the n = 40 cell, snapshots (16 mu x 3 paths x 20 steps), modes
ECM_SIZE = (441, 155, 154)    # integrands (n L + 1 for n = 40, L = 11), grid of about 24000 points


def offline_rates():
    """The offline stage on the GPU at the n = 40 ROM's sizes: POD of 960
    snapshots of 32316 dofs with a sparse SPD weight (40 modes), and the
    empirical cubature of 441 smooth integrands over 23870 points
    (tolerance 1e-4).  Wall time of each call (inputs resident in HBM),
    after one untimed call of the same size: the library routines load
    size-dependent code on first use."""
    import torch
    import workloads
    from paper_2307_16894_amd.offline import ecm, pod
    nrow, ns, n = POD_SIZE
    S = workloads.pod_snapshots(7, nrow, ns, 200, 0.8, 1e-12)
    M = workloads.banded_spd(8, nrow, 8)
    pod(S, M, n)  # warm-up (library handles, code objects)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    modes, lam = pod(S, M, n)
    torch.cuda.synchronize()
    t_pod = time.perf_counter() - t0
    R, nx, ny = ECM_SIZE
    pts, w = workloads.grid_points(nx, ny)
    J = workloads.cos_integrands(4, pts, R)
    ecm(J, w, 1e-4, 1024)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx, wq, hist, rank, code = ecm(J, w, 1e-4, 1024)
    torch.cuda.synchronize()
    t_ecm = time.perf_counter() - t0
    gram_flops = 2.0 * ns * ns * nrow + 2.0 * n * ns * nrow + 2.0 * n * n * nrow
    return dict(pod=dict(rows=nrow, snapshots=ns, modes=n, seconds=t_pod, gemm_gflop=gram_flops / 1e9,
                         lambda_ratio=float(lam[n - 1] / lam[0])),
                ecm=dict(integrands=R, points=nx * ny, rank=rank, selected=int(len(idx)), iterations=len(hist) - 1,
                         final_residual=float(hist[-1]), seconds=t_ecm, code=code))


_ORACLE = {}


def _oracle_init(rom_file):
    """Pool worker set-up, outside the timed map: one BLAS thread, the ROM loaded once."""
    from threadpoolctl import threadpool_limits
    from oracle.rom import ROM
    _ORACLE['limit'] = threadpool_limits(1)
    _ORACLE['rom'] = ROM(rom_file)


def _oracle_worker(args):
    mu, path = args
    out = _ORACLE['rom'].run_path(mu, path, max_iter=MAX_ITER, max_substeps=SUBSTEPS)
    return sum(o['iters'] for o in out), sum(o['status'] == 0 for o in out)


def cpu_model():
    try:
        with open('/proc/cpuinfo') as fh:
            for line in fh:
                if line.startswith('model name'):
                    return line.split(':', 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, rom_file, budget_s=20.0):
    """The FP64 oracle on a bounded sample of the workload, one process per
    core, with the GPU forms' options (Newton cap MAX_ITER, load-step cutting
    depth SUBSTEPS); the rate counts converged point-steps only."""
    import multiprocessing as mp
    mu, paths = inputs(w)
    cores = min(len(os.sched_getaffinity(0)), 16)
    _oracle_init(rom_file)
    t0 = time.perf_counter()
    _oracle_worker((mu[0], paths[0]))
    t1 = time.perf_counter() - t0
    S = int(np.clip(budget_s * cores / max(t1, 1e-3), cores, w['P']))
    S = max(cores, (S // cores) * cores)
    jobs = [(mu[i], paths[i]) for i in range(S)]
    with mp.get_context('fork').Pool(cores, initializer=_oracle_init, initargs=(rom_file,)) as pool:
        pool.map(_oracle_worker, jobs[:cores], chunksize=1)  # every worker has loaded the ROM
        t0 = time.perf_counter()
        res = pool.map(_oracle_worker, jobs, chunksize=1)
        wall = time.perf_counter() - t0
    steps = S * w['steps']
    conv = int(sum(r[1] for r in res))
    return dict(value=conv / wall, unit='macro-point load steps/s', cores=cores, kind='oracle',
                cpu=cpu_model(),
                sample=f"first {S} of {w['P']} macro points, all {w['steps']} load steps ({steps} point-steps, "
                       f"{conv} converged, {wall:.1f}s wall); Newton cap {MAX_ITER}, cutting depth {SUBSTEPS} "
                       f"as on the GPU; the rate counts converged point-steps",
                mean_iters=float(sum(r[0] for r in res) / steps),
                converged_fraction=float(conv / steps))


def uneven_run(workload, log):
    """The uneven persistent batch: autotuned launch per ROM, one load step of
    every ROM captured as a graph (a branch per ROM), replayed until every
    point has finished its own path; the timed run starts from the virgin
    state after an untimed run of the same replays."""
    import torch
    import paper_2307_16894_amd as L
    from paper_2307_16894_amd import autotune
    from paper_2307_16894_amd.uneven import Group, UnevenBatch
    u = UNEVEN[workload]
    groups, tuned = [], {}
    for i, (name, P) in enumerate(u['roms']):
        seed = u['seed'] + i
        mu = workloads.one_void_mu(seed, P) if name.startswith('onevoid') else workloads.four_void_mu(seed, P)
        ns = workloads.uneven_steps(seed, P, *u['steps'])
        paths = workloads.uneven_cyclic_paths(seed, P, ns, u['rho'])
        rom_file = os.path.join(ROOT, 'roms', name + '.rom')
        tp = min(P, u['tune_points'])
        t = autotune.tune(rom_file, mu[:tp], paths[:tp, 0], L.DT_F64, reps=2, graph=True)
        tuned[name] = dict(n=t['n'], m=t['m'], mode={L.MODE_FUSED: 'fused', L.MODE_PHASED: 'phased'}[t['mode']],
                           split=t['split'], grid_per_cu=t['grid_per_cu'], trials_ms=t['trials'])
        log(f"[bench] {name}: P={P}, n={t['n']}, m={t['m']}, tuned {tuned[name]['mode']} split={t['split']} "
            f"grid_per_cu={t['grid_per_cu']}")
        groups.append(Group(rom_file, mu, paths, ns, split=t['split'], grid_per_cu=t['grid_per_cu'],
                            max_iter=u['max_iter'], max_substeps=SUBSTEPS, mode=t['mode']))
    ub = UnevenBatch(groups)
    ub.capture()
    K = ub.max_steps
    for rep in range(2):  # untimed run, then the timed one, each from the virgin state
        ub.reset()
        t0 = time.perf_counter()
        for _ in range(K):
            ub.graph.replay()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        log(f"[bench] uneven run {rep}: {elapsed:.3f}s")
    tot = ub.totals()
    ub.close()
    P = sum(P for _, P in u['roms'])
    out = dict(metric="ROM macro-point load steps/s at 1e-8 residual; learned+mixed vs plain FP64",
               value=tot['point_steps'] / elapsed, unit="macro-point load steps/s", n_gpus=1, steps=K, warmup=K,
               ms_per_step=1e3 * elapsed / K, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
               data="synthetic",
               config=dict(workload=workload, roms=[dict(rom=n, points=p) for n, p in u['roms']], batch=P,
                           steps_per_point=list(u['steps']), newton_cap=u['max_iter'], tol=1e-8, form='fp64',
                           graph=True, tuned=tuned),
               point_steps=tot['point_steps'], evaluations=tot['evaluations'],
               mean_evaluations=tot['evaluations'] / max(tot['point_steps'], 1),
               failed_point_steps=tot['failed'], replays=K, elapsed_s=elapsed)
    return out


def flops_per_eval(n, m):
    """Algorithmic flops of one Newton evaluation of one macro point: per ECM
    point the contraction K = sum_q G_q^T (D_q G_q) (8 n^2 + 32 n), the
    residual f (8 n), the tangent right-hand sides C (32 n), the kinematics
    (8 n), the return map with tangent (C_CM) and the weighting (C_W); per
    point the elimination (2/3 n^3) and five right-hand sides (forward and
    back substitution, 2 n^2 each)."""
    return m * (8.0 * n * n + 80.0 * n + C_CM + C_W) + 2.0 / 3.0 * n ** 3 + 10.0 * n * n


def stage_roofline(n, m, evals, point_steps, contraction, kern_ms, refine_evals=0):
    """Sum over the stages of max(flops / peak of the stage's unit, bytes /
    HBM bandwidth) for a run of `evals` point-evaluations, against its kernel
    time: the contraction of K and C (8 n^2 + 32 n per ECM point) at the peak
    of its precision, everything else at the FP64 peak; the history read and
    committed once per point-step (2 x 48 m bytes) is the algorithmic HBM
    traffic.  `refine_evals` FP64 evaluations more (abar_f64) count whole at
    the FP64 peak."""
    c_flops = evals * m * (8.0 * n * n + 32.0 * n)
    r_flops = (evals + refine_evals) * flops_per_eval(n, m) - c_flops
    t_c = c_flops / (PEAK[contraction] * 1e12)
    t_r = r_flops / (PEAK['f64'] * 1e12)
    t_b = point_steps * 2 * 48.0 * m / (HBM_TBS * 1e12)
    t_roof = t_c + max(t_r, t_b)
    return dict(t_roofline_ms=1e3 * t_roof, t_kernels_ms=kern_ms, frac=1e3 * t_roof / kern_ms if kern_ms > 0 else 0.0,
                stages=dict(contraction=dict(flops=c_flops, peak_tflops=PEAK[contraction], ms=1e3 * t_c),
                            fp64_rest=dict(flops=r_flops, peak_tflops=PEAK['f64'], ms=1e3 * t_r),
                            history_bytes=dict(bytes=point_steps * 2 * 48.0 * m, ms=1e3 * t_b)))


def kernel_source_digest():
    """SHA-256 over the sources of the fused and phased kernels (a recorded
    traffic measurement is reported only while they are unchanged)."""
    import hashlib
    csrc = os.path.join(ROOT, 'paper_2307_16894_amd', 'csrc')
    h = hashlib.sha256()
    for f in sorted(os.listdir(csrc)):
        if (f.startswith(('rom_fused', 'rom_phased')) and f.endswith(('.hip', '.h'))) or f in ('j2_device.h',
                                                                                              'rom_common.h'):
            with open(os.path.join(csrc, f), 'rb') as fh:
                h.update(f.encode() + b'\0' + fh.read())
    return h.hexdigest()


def measured_traffic(workload, form):
    """HBM bytes per timed unit (fused form: one kernel launch; phased form:
    the launches of one step) from the committed counter summary (FETCH_SIZE +
    WRITE_SIZE, scaled by a copy of known size), or None."""
    name = 'k_fused_fp64' if form == 'fused' else 'phased_fp64'
    path = os.path.join(ROOT, 'profiles', f'{name}_{workload}_traffic.json')
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get('kernel_source_sha256') != kernel_source_digest():
        return None
    return t.get('hbm_bytes_per_launch')


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=None, help='timed steps (default: per workload)')
    ap.add_argument('--warmup', type=int, default=None, help='untimed steps (default: per workload)')
    ap.add_argument('--workload', default=DEFAULT, choices=sorted(WORKLOADS) + sorted(UNEVEN))
    ap.add_argument('--variants', default=None, help='comma-separated forms (default: per workload)')
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--no-fe2', action='store_true', help='skip the two-scale example')
    ap.add_argument('--no-extra', action='store_true',
                    help='skip the four-void n = 100 and uneven workloads reported beside the default one')
    ap.add_argument('--calibrate-copy', type=int, default=0, metavar='MIB',
                    help='first copy MIB MiB device to device (a known-size reference for HBM counters)')
    ap.add_argument('--offline-only', action='store_true',
                    help='time only the offline stage (POD and cubature) at the n = 40 sizes and print it')
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(json.dumps(dict(error="this benchmark runs on one GPU: the macro points of a batch are "
                                    "independent and a single MI355X holds the whole workload; "
                                    "run with --gpus 1")))
        return 2
    import paper_2307_16894_amd as L
    log = lambda s: print(s, file=sys.stderr, flush=True)  # noqa: E731
    if a.calibrate_copy > 0:
        import torch
        nel = a.calibrate_copy * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device='cuda:0')
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {a.calibrate_copy} MiB done")
        del src, dst
    if a.offline_only:
        print(json.dumps(dict(offline=offline_rates())), flush=True)
        return 0
    if a.workload in UNEVEN:
        print(json.dumps(uneven_run(a.workload, log)), flush=True)
        return 0
    w = WORKLOADS[a.workload]
    steps = w['timed'] if a.steps is None else a.steps
    warmup = w['warm'] if a.warmup is None else a.warmup
    variants = [v for v in (a.variants or ','.join(w['variants'])).split(',') if v]
    r = run_forms(a.workload, variants, steps, warmup, log)
    out_var, head, plain_best, n, m = r['variants'], r['head'], r['plain'], r['n'], r['m']
    rf = r['res'][plain_best] if plain_best else r['res'][head]
    rf_form = 'phased' if (plain_best or '').endswith('_phased') else 'fused'
    fpe = flops_per_eval(n, m)
    achieved = fpe * rf['evals'] / (rf['kern_ms'] * 1e-3) / 1e12 if rf['kern_ms'] > 0 else 0.0
    P = w['P']
    out = dict(
        metric="ROM macro-point load steps/s at 1e-8 residual; learned+mixed vs plain FP64",
        value=out_var[head]['value'], unit="macro-point load steps/s", n_gpus=1, steps=steps, warmup=warmup,
        ms_per_step=out_var[head]['ms_per_step'], higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype={'bf16': 'bf16+f64', 'fp32': 'f32+f64'}.get(head.split('_')[0], 'f64'),
        data="synthetic",
        config=dict(workload=a.workload, rom=w['rom'], n=n, m=m, batch=P, load_steps=w['steps'], tol=1e-8,
                    form=head, contraction=head.split('_')[0], warm_start='_mlp' in head),
        plain_fp64=dict(out_var[plain_best], form=plain_best) if plain_best else None,
        speedup_vs_plain_fp64=(out_var[head]['value'] / out_var[plain_best]['value']) if plain_best else None,
        head_rule=f"learned+reduced-precision form (else reduced-precision form) of highest throughput with every "
                  f"timed point-step converged and max |Pbar - Pbar_fp64| / max |Pbar_fp64| <= {PBAR_TOL:g} over all "
                  f"timed point-steps that followed the plain FP64 loading path (same converged sub-steps); the "
                  f"fraction on another path is reported per form (other_path_fraction)",
        variants=out_var,
        warm_start=r['warm_start'],
        # the plain FP64 step against the FP64 peak (its kernels: the fused
        # kernel, or the phased step's kinematics, material, contraction,
        # solve and finishing launches on both streams); algorithmic flops
        # per point-evaluation as in flops_per_eval
        roofline=dict(bound="mfma",
                      kernel=("k_fused<fp64>" if rf_form == 'fused' else
                              "phased step <fp64>: k_ph_kin + k_ph_mat + k_ph_cs + k_ph_s + k_fused_queue"),
                      achieved=achieved, peak=PEAK['f64'],
                      unit="TFLOP/s", frac=achieved / PEAK['f64'],
                      traffic=measured_traffic(a.workload, rf_form),
                      launches=rf['launches'], avg_launch_ms=rf['kern_ms'] / max(rf['launches'], 1),
                      flops_per_point_eval=fpe, point_evals=rf['evals'], c_cm=C_CM, c_w=C_W),
        roofline_head=dict(form=head, **out_var[head]['stage_roofline']),
    )
    rom_file = os.path.join(ROOT, 'roms', w['rom'] + '.rom')
    log("[bench] shape sensitivities")
    out['shape_sensitivity'] = sensitivity_rate(w, rom_file)
    if not a.no_fe2 and w['rom'] == 'onevoid_n40_m400':
        log("[bench] two-scale example")
        out['fe2'] = fe2_rate(rom_file, L.MODE_PHASED)
        out['fe2']['compliance_error'] = fe2_compliance_error(L.MODE_PHASED)
        log("[bench] offline stage")
        out['offline'] = offline_rates()
    if not a.no_extra and a.workload == DEFAULT:
        # the four-void n = 100 workload (reduced-precision contraction at a
        # large n) and the uneven batch over five ROMs, each with its own rates
        log("[bench] four-void n = 100")
        r4 = run_forms(EXTRA_N100, WORKLOADS[EXTRA_N100]['variants'], WORKLOADS[EXTRA_N100]['timed'],
                       WORKLOADS[EXTRA_N100]['warm'], log)
        out[EXTRA_N100] = dict(head=r4['head'], n=r4['n'], m=r4['m'], batch=WORKLOADS[EXTRA_N100]['P'],
                               variants=r4['variants'])
        log("[bench] uneven batch")
        out[EXTRA_UNEVEN] = uneven_run(EXTRA_UNEVEN, log)
    if not a.no_cpu_baseline:
        out['cpu_baseline'] = cpu_baseline(w, os.path.join(ROOT, 'roms', w['rom'] + '.rom'))
    print(json.dumps(out), flush=True)
    return 0


def run_forms(workload, variants, steps, warmup, log):
    """Every form of `variants` on a standard workload (warm-up steps, then
    the timed steps), compared with plain FP64; returns the per-form rates
    and accuracy, the head form and the plain FP64 form of highest rate."""
    import paper_2307_16894_amd as L
    w = WORKLOADS[workload]
    rom_file = os.path.join(ROOT, 'roms', w['rom'] + '.rom')
    ws, wsinfo = (None, None)
    if any('_mlp' in v for v in variants):
        ws, wsinfo = train_warm_start(w, rom_file, log)
    P = w['P']
    res = {}
    n = m = 0
    for v in variants:
        # <precision>[_mlp][_a64][_phased[K[eE]] | _staged]  (a64: Abar from an FP64 evaluation at the
        # returned state; K: phased evaluations, E: early hand-over, -1 none; library defaults when left out)
        vb = v
        dt = {'fp64': L.DT_F64, 'fp32': L.DT_F32, 'bf16': L.DT_BF16}[vb.split('_')[0]]
        last = vb.split('_')[-1]
        mode = L.MODE_PHASED if last.startswith('phased') else L.MODE_FUSED
        kph, kearly = 0, 0
        if mode == L.MODE_PHASED and last[6:]:
            ks, _, es = last[6:].partition('e')
            kph, kearly = int(ks or 0), int(es or 0)
        ph = dict(mode=mode, phased_evals=kph, phased_early=kearly)
        if '_mlp' in vb:
            opts = ws.opts(contraction=dt, max_substeps=SUBSTEPS, **ph)
        elif vb.endswith('_staged'):  # the staged form has no load-step cutting
            opts = L.rom_default_opts(mode=L.MODE_STAGED, contraction=dt)
        else:
            opts = L.rom_default_opts(contraction=dt, max_substeps=SUBSTEPS, **ph)
        if '_a64' in vb:
            opts.abar_f64 = 1
        log(f"[bench] {workload}: {v}")
        g = gpu_run(w, steps, warmup, opts, rom_file)
        n, m = g['n'], g['m']
        res[v] = g
    if ws is not None:
        ws.close()
    ref = res.get('fp64')
    out_var = {}
    for v, g in res.items():
        d = dict(value=P * steps / g['elapsed'], ms_per_step=1e3 * g['elapsed'] / steps,
                 mean_iters=g['evals'] / (P * steps), max_iters=g['max_iter'],
                 converged_fraction=g['converged'] / (P * steps),
                 kernel_ms_per_step=g['kern_ms'] / steps)
        prec = {'fp64': 'f64', 'fp32': 'f32', 'bf16': 'bf16'}[v.split('_')[0]]
        d['stage_roofline'] = stage_roofline(n, m, g['evals'], P * steps, prec, g['kern_ms'],
                                             refine_evals=g['converged'] if '_a64' in v else 0)
        if ref is not None and v != 'fp64':
            # Deviation from plain FP64 over every timed point-step that followed the
            # same loading path (the same converged sub-steps since the start of the
            # path), where both runs solve the same discrete problems and differ by
            # precision and Newton's stopping point alone.  A point whose steps are
            # cut differently (the warm start or a reduced-precision tangent changes
            # whether the full step converges) integrates the plastic flow over other
            # increments from then on: those point-steps are counted, and their
            # deviation is reported apart.
            scale = np.abs(ref['Pbar']).max()
            dev = np.abs(g['Pbar'] - ref['Pbar']).max(axis=-1) / scale  # [steps][P]
            same = same_path(g, ref)
            d['max_rel_diff_Pbar_vs_fp64_step1'] = float(dev[0].max())
            d['max_rel_diff_Pbar_vs_fp64_same_path'] = float(dev[same].max()) if same.any() else None
            d['median_rel_diff_Pbar_vs_fp64_same_path'] = float(np.median(dev[same])) if same.any() else None
            d['other_path_fraction'] = float(1.0 - same.mean())
            d['other_path_points'] = int((~same).any(axis=0).sum())
            d['max_rel_diff_Pbar_vs_fp64_other_path'] = float(dev[~same].max()) if (~same).any() else None
            d['max_rel_diff_Pbar_vs_fp64'] = float(dev.max())
            adev = np.abs(g['Abar'] - ref['Abar']).max(axis=-1) / np.abs(ref['Abar']).max()
            d['max_rel_diff_Abar_vs_fp64_same_path'] = float(adev[same].max()) if same.any() else None
            d['median_rel_diff_Abar_vs_fp64_same_path'] = float(np.median(adev[same])) if same.any() else None
            d['p999_rel_diff_Abar_vs_fp64_same_path'] = float(np.quantile(adev[same], 0.999)) if same.any() else None
        out_var[v] = d

    # head: the learned + reduced-precision form (else the reduced-precision
    # form) of highest throughput whose Pbar stays within PBAR_TOL of plain FP64
    # on every timed point-step of the same loading path, all of them converged
    def admitted(v):
        d = out_var.get(v, {})
        dm = d.get('max_rel_diff_Pbar_vs_fp64_same_path')
        return dm is not None and dm <= PBAR_TOL and d['converged_fraction'] == 1.0
    reduced = [v for v in out_var if v.split('_')[0] in ('fp32', 'bf16')]
    cands = [v for v in reduced if '_mlp' in v and admitted(v)] or [v for v in reduced if admitted(v)]
    head = max(cands, key=lambda v: out_var[v]['value']) if cands else ('fp64' if 'fp64' in out_var else variants[0])
    # plain FP64 Newton: the faster of its fused and phased executions (the same
    # arithmetic, the same results bit for bit)
    plain = [v for v in ('fp64', 'fp64_phased') if v in out_var]
    plain_best = max(plain, key=lambda v: out_var[v]['value']) if plain else None
    return dict(variants=out_var, head=head, plain=plain_best, res=res, n=n, m=m, warm_start=wsinfo)


if __name__ == '__main__':
    sys.exit(main())

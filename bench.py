#!/usr/bin/env python3
"""Throughput of the batched hyper-reduced RVE solve on one MI355X.

One step = one load step of every macro point of the batch: rom_step (Newton
on the reduced coordinates to ||f||_2 <= 1e-8, then effective stress and
stiffness) followed by rom_homogenized_stress_tangent.  The metric is macro-
point load steps per second with all inputs resident in device memory.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--mode fused|staged]

Prints one JSON line.  Also reports the dominant kernel against the MI355X
FP64 peak (measured with HIP events on the stream the kernel runs on) and the
plain FP64 CPU oracle timed on a bounded sample of the same workload on the
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

PEAK_FP64_TFLOPS = 78.6  # MI355X dense FP64 (vector and matrix)

WORKLOADS = {
    # one elliptical void, n = 40 modes, m ~ 400 ECM points, 4096 points,
    # 20-step load / unload paths of amplitude <= 0.08
    'onevoid_n40_m400_P4096_cyclic20': dict(rom='onevoid_n40_m400', P=4096, steps=20, path='cyclic',
                                            rho=(0.02, 0.08), seed=0),
    # small case: n = 20, m = 120, 64 points, 10-step monotone paths
    'onevoid_n20_m120_P64_monotone10': dict(rom='onevoid_n20_m120', P=64, steps=10, path='monotone',
                                            rho=(0.02, 0.05), seed=0),
}
DEFAULT = 'onevoid_n40_m400_P4096_cyclic20'


def inputs(w):
    P, K = w['P'], w['steps']
    mu = workloads.one_void_mu(w['seed'], P)
    if w['path'] == 'cyclic':
        paths = workloads.cyclic_paths(w['seed'], P, K, w['rho'])
    else:
        paths = workloads.monotone_paths(w['seed'], P, K, w['rho'])
    return mu, paths


def gpu_run(w, steps, warmup, mode, rom_file):
    import torch
    import paper_2307_16894_amd as L
    from paper_2307_16894_amd.batch import RomBatch
    mu, paths = inputs(w)
    P, K = w['P'], w['steps']
    dev = torch.device('cuda:0')
    Fb = torch.from_numpy(np.ascontiguousarray(paths.reshape(P, K, 4).transpose(1, 0, 2))).to(dev)  # [K][P][4]
    rb = RomBatch(rom_file, mu, dev)
    n, m = rb.info['n'], rb.info['m']
    opts = L.rom_default_opts(mode=mode)

    def run(nsteps, record):
        k = 0
        rec = []
        for _ in range(nsteps):
            if k == K:  # the path is cycled from the virgin state
                L.rom_state_init(rb.h, P, rb.mu.data_ptr(), rb.state.data_ptr(), rb.stream.cuda_stream)
                k = 0
            rb.step(Fb[k], opts)
            if record:  # device-side copies, no synchronisation
                rec.append((rb.iters.clone(), (rb.status == 0).sum()))
            k += 1
        return rec

    L.rom_state_init(rb.h, P, rb.mu.data_ptr(), rb.state.data_ptr(), rb.stream.cuda_stream)
    run(warmup, False)
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
    evals = int(sum(int(it.sum()) for it, _ in rec))
    conv = int(sum(int(c) for _, c in rec))
    max_it = int(max(int(it.max()) for it, _ in rec))
    rb.close()
    return dict(elapsed=t1 - t0, evals=evals, converged=conv, max_iter=max_it, kern_ms=kern_ms,
                launches=launches, n=n, m=m)


def _oracle_worker(args):
    rom_file, mu, path = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        from oracle.rom import ROM
        rom = ROM(rom_file)
        out = rom.run_path(mu, path)
    return sum(o['iters'] for o in out), sum(o['status'] == 0 for o in out)


def cpu_baseline(w, rom_file, budget_s=20.0):
    """The FP64 oracle on a bounded sample of the workload, one process per core."""
    import multiprocessing as mp
    mu, paths = inputs(w)
    cores = min(len(os.sched_getaffinity(0)), 16)
    t0 = time.perf_counter()
    _oracle_worker((rom_file, mu[0], paths[0]))
    t1 = time.perf_counter() - t0
    S = int(np.clip(budget_s * cores / max(t1, 1e-3), cores, w['P']))
    S = max(cores, (S // cores) * cores)
    jobs = [(rom_file, mu[i], paths[i]) for i in range(S)]
    with mp.get_context('fork').Pool(cores) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_worker, jobs, chunksize=1)
        wall = time.perf_counter() - t0
    steps = S * w['steps']
    return dict(value=steps / wall, unit='macro-point load steps/s', cores=cores, kind='oracle',
                sample=f"first {S} of {w['P']} macro points, all {w['steps']} load steps "
                       f"({steps} point-steps, {wall:.1f}s wall)",
                mean_iters=float(sum(r[0] for r in res) / steps),
                converged_fraction=float(sum(r[1] for r in res) / steps))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=20)
    ap.add_argument('--warmup', type=int, default=20)
    ap.add_argument('--workload', default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument('--mode', default='staged', choices=['staged', 'fused'])
    ap.add_argument('--no-cpu-baseline', action='store_true')
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(json.dumps(dict(error="this benchmark runs on one GPU: the macro points of a batch are "
                                    "independent and a single MI355X holds the whole workload; "
                                    "run with --gpus 1")))
        return 2
    w = WORKLOADS[a.workload]
    rom_file = os.path.join(ROOT, 'roms', w['rom'] + '.rom')
    mode = 1 if a.mode == 'fused' else 0
    g = gpu_run(w, a.steps, a.warmup, mode, rom_file)
    P = w['P']
    value = P * a.steps / g['elapsed']
    n, m = g['n'], g['m']
    # dominant kernel: the reduced-tangent contraction K = sum_q G_q^T D_q G_q
    # with H = D_q G_q and f = sum_q G_q^T W_q: m (8 n^2 + 40 n) flops per
    # point-evaluation
    flops_per_eval = m * (8.0 * n * n + 40.0 * n)
    per_launch_ms = g['kern_ms'] / max(g['launches'], 1)
    achieved = flops_per_eval * g['evals'] / (g['kern_ms'] * 1e-3) / 1e12 if g['kern_ms'] > 0 else 0.0
    out = dict(
        metric="ROM macro-point load steps/s at 1e-8 residual",
        value=value, unit="macro-point load steps/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
        ms_per_step=1e3 * g['elapsed'] / a.steps, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64", data="synthetic",
        config=dict(workload=a.workload, rom=w['rom'], n=n, m=m, batch=P, load_steps=w['steps'],
                    mode=a.mode, contraction="f64", tol=1e-8),
        newton=dict(mean_iters=g['evals'] / (P * a.steps), max_iters=g['max_iter'],
                    converged_fraction=g['converged'] / (P * a.steps)),
        roofline=dict(bound="mfma", kernel="k_assemble" if mode == 0 else "k_fused",
                      achieved=achieved, peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                      frac=achieved / PEAK_FP64_TFLOPS, traffic=None,
                      launches=g['launches'], avg_launch_ms=per_launch_ms,
                      flops_per_point_eval=flops_per_eval, point_evals=g['evals']),
    )
    if not a.no_cpu_baseline:
        out['cpu_baseline'] = cpu_baseline(w, rom_file)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == '__main__':
    sys.exit(main())

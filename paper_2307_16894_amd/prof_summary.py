"""Summaries of rocprofv3 CSV output for the profiles directory.

    python -m paper_2307_16894_amd.prof_summary stats KERNEL_STATS_CSV OUT.md --command "..."
    python -m paper_2307_16894_amd.prof_summary counters OUT.md PMC_CSV [PMC_CSV ...] --command "..." [--command ...]
    python -m paper_2307_16894_amd.prof_summary traffic FETCH_CSV WRITE_CSV OUT_PREFIX \\
        --workload W --copy-mib N --command-fetch "..." --command-write "..."

`stats` keeps the kernel table of a --kernel-trace --stats run (with
--unit-kernel K also the summed duration per call of K, e.g. per phased step).
`counters` adds up the counters of --pmc runs per kernel and derives the
MFMA-busy fraction and per-wave instruction counts.
`traffic` takes the FETCH_SIZE and WRITE_SIZE counter runs (KiB per
dispatch), scales each by the reading of the same counter for the calibration
copy of known size (bench.py --calibrate-copy), and writes the HBM bytes per
launch of the kernel (--kernel: comma-separated name parts; with --unit-kernel
the bytes of all matching dispatches per call of that kernel, e.g. per phased
step) together with the digest of the kernel sources.
"""
import argparse
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rows(path):
    with open(path, newline='') as fh:
        return list(csv.DictReader(fh))


def stats(args):
    rows = _rows(args.csv)
    rows.sort(key=lambda r: -float(r['TotalDurationNs']))
    total = sum(float(r['TotalDurationNs']) for r in rows)
    lines = [f"# rocprofv3 kernel statistics: {args.title}", "", "Command:", "", "```", args.command, "```", "",
             "| kernel | calls | total ms | average us | min us | max us | share |", "|---|---|---|---|---|---|---|"]
    for r in rows[:args.top]:
        name = r['Name']
        if len(name) > 90:
            name = name[:87] + '...'
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {100 * float(r['TotalDurationNs']) / total:.1f}% |")
    if args.unit_kernel:
        units = sum(int(r['Calls']) for r in rows if args.unit_kernel in r['Name'])
        parts = [k for k in args.kernels.split(',') if k] if args.kernels else None
        sel = [r for r in rows if parts is None or any(k in r['Name'] for k in parts)]
        if units:
            tot = sum(float(r['TotalDurationNs']) for r in sel)
            lines += ["", f"Per call of `{args.unit_kernel}` ({units} calls): {tot / units / 1e3:.1f} us of "
                      f"{'the kernels ' + ', '.join(parts) if parts else 'all kernels'}."]
    with open(args.out, 'w') as fh:
        fh.write('\n'.join(lines) + '\n')


def _per_dispatch(path, counter):
    out = {}
    for r in _rows(path):
        if r.get('Counter_Name') != counter:
            continue
        key = r['Dispatch_Id']
        out.setdefault(key, [r['Kernel_Name'], 0.0])
        out[key][1] += float(r['Counter_Value'])
    return list(out.values())


def _split(disp, kernel_subs, copy_sub):
    ker = [v for name, v in disp if any(k in name for k in kernel_subs)]
    cpy = [v for name, v in disp if copy_sub in name]
    if not ker or not cpy:
        raise SystemExit(f"kernel or calibration copy not found ({len(ker)} / {len(cpy)} dispatches)")
    return ker, max(cpy)


def traffic(args):
    sys.path.insert(0, ROOT)
    from bench import kernel_source_digest
    copy_bytes = args.copy_mib * (1 << 20)
    res = {}
    parts = [k for k in args.kernel.split(',') if k]
    for counter, path in (('FETCH_SIZE', args.fetch_csv), ('WRITE_SIZE', args.write_csv)):
        disp = _per_dispatch(path, counter)
        ker, cpy_kib = _split(disp, parts, args.copy)
        units = len(ker)
        if args.unit_kernel:
            units = sum(1 for name, _ in disp if args.unit_kernel in name)
        factor = copy_bytes / (cpy_kib * 1024.0)
        res[counter] = dict(dispatches=len(ker), units=units, mean_kib=sum(ker) / units, copy_kib=cpy_kib,
                            factor=factor, bytes_per_launch=factor * 1024.0 * sum(ker) / units)
    hbm = res['FETCH_SIZE']['bytes_per_launch'] + res['WRITE_SIZE']['bytes_per_launch']
    out = dict(kernel=args.kernel, workload=args.workload, kernel_source_sha256=kernel_source_digest(),
               copy_mib=args.copy_mib, counters=res, hbm_bytes_per_launch=hbm,
               commands=dict(fetch=args.command_fetch, write=args.command_write))
    with open(args.out_prefix + '.json', 'w') as fh:
        json.dump(out, fh, indent=1)
    per = f"per call of `{args.unit_kernel}`" if args.unit_kernel else "per dispatch"
    lines = [f"# HBM traffic of `{args.kernel}` ({args.workload})", "",
             f"Counters in KiB {per}, scaled by a {args.copy_mib} MiB calibration copy.", ""]
    for c in ('FETCH_SIZE', 'WRITE_SIZE'):
        r = res[c]
        lines.append(f"- {c}: {r['dispatches']} dispatches over {r['units']} units, mean {r['mean_kib']:.1f} KiB; copy read "
                     f"{r['copy_kib']:.1f} KiB for {args.copy_mib * 1024} KiB -> factor {r['factor']:.4f}; "
                     f"{r['bytes_per_launch'] / 1e6:.3f} MB per launch")
    lines += [f"- HBM bytes per launch: {hbm / 1e6:.3f} MB", "", "Commands:", "", "```", args.command_fetch,
              args.command_write, "```"]
    with open(args.out_prefix + '.md', 'w') as fh:
        fh.write('\n'.join(lines) + '\n')


def counters(args):
    """Per-kernel sums of the counters of one or more --pmc runs (every
    dispatch of a kernel added), with the derived ratios: MFMA-busy fraction
    SQ_VALU_MFMA_BUSY_CYCLES / (4 SQ_BUSY_CU_CYCLES) (four SIMDs per compute
    unit), instructions per wave, LDS bank-conflict cycles per LDS
    instruction."""
    tot = {}
    for path in args.csvs:
        for r in _rows(path):
            name = r['Kernel_Name']
            if args.kernels and not any(k in name for k in args.kernels.split(',')):
                continue
            d = tot.setdefault(name, {})
            key = r['Counter_Name']
            d[key] = d.get(key, 0.0) + float(r['Counter_Value'])
            d.setdefault('_dispatches_' + os.path.basename(path), set()).add(r['Dispatch_Id'])
    lines = [f"# rocprofv3 counters: {args.title}", "", "Commands:", "", "```"] + args.command + ["```", ""]
    for name, d in sorted(tot.items(), key=lambda kv: -kv[1].get('SQ_BUSY_CU_CYCLES', kv[1].get('SQ_WAVES', 0))):
        disp = max(len(v) for k, v in d.items() if k.startswith('_dispatches_'))
        lines.append(f"## `{name[:110]}` ({disp} dispatches)")
        lines.append("")
        lines.append("| counter | sum over dispatches |")
        lines.append("|---|---|")
        for k in sorted(k for k in d if not k.startswith('_')):
            lines.append(f"| {k} | {d[k]:.6g} |")
        derived = []
        if 'SQ_VALU_MFMA_BUSY_CYCLES' in d and d.get('SQ_BUSY_CU_CYCLES'):
            derived.append(f"MFMA busy: {d['SQ_VALU_MFMA_BUSY_CYCLES'] / (4.0 * d['SQ_BUSY_CU_CYCLES']):.3f} "
                           f"of the SIMD cycles while the compute units were busy")
        if d.get('SQ_WAVES'):
            for k in ('SQ_INSTS_VALU', 'SQ_INSTS_MFMA', 'SQ_INSTS_LDS', 'SQ_INSTS_SALU', 'SQ_INSTS_VMEM_RD'):
                if k in d:
                    derived.append(f"{k} per wave: {d[k] / d['SQ_WAVES']:.1f}")
        if d.get('SQ_INSTS_LDS') and 'SQ_LDS_BANK_CONFLICT' in d:
            derived.append(f"LDS bank-conflict cycles per LDS instruction: {d['SQ_LDS_BANK_CONFLICT'] / d['SQ_INSTS_LDS']:.3f}")
        if derived:
            lines += [""] + [f"- {x}" for x in derived]
        lines.append("")
    with open(args.out, 'w') as fh:
        fh.write('\n'.join(lines) + '\n')


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest='what', required=True)
    s = sub.add_parser('stats')
    s.add_argument('csv')
    s.add_argument('out')
    s.add_argument('--command', required=True)
    s.add_argument('--title', default='')
    s.add_argument('--top', type=int, default=15)
    s.add_argument('--unit-kernel', default='')
    s.add_argument('--kernels', default='')
    t = sub.add_parser('traffic')
    t.add_argument('fetch_csv')
    t.add_argument('write_csv')
    t.add_argument('out_prefix')
    t.add_argument('--workload', required=True)
    t.add_argument('--copy-mib', type=int, required=True)
    t.add_argument('--kernel', default='k_fused<3, 0, 0>')
    t.add_argument('--copy', default='copyBuffer')
    t.add_argument('--unit-kernel', default='')
    t.add_argument('--command-fetch', required=True)
    t.add_argument('--command-write', required=True)
    c = sub.add_parser('counters')
    c.add_argument('out')
    c.add_argument('csvs', nargs='+')
    c.add_argument('--command', action='append', required=True)
    c.add_argument('--title', default='')
    c.add_argument('--kernels', default='')
    a = ap.parse_args(argv)
    {'stats': stats, 'traffic': traffic, 'counters': counters}[a.what](a)


if __name__ == '__main__':
    main()

"""Writes fe2_fom_4x2.json: the reference two-scale solution with the
full-order RVE at every macro point (Sec. 4.2: the compliance C_k of every
load step, against which the reduced model's compliance error
eps_C,k = |C_k - C_k^ref| / |C_k^ref| is measured).

The macro problem is the 4 x 2 block of eight-node quadrilaterals (32 Gauss
points) of the two-scale tests, bottom edge fixed, the parabolic top traction
rising to its peak over four steps and back over four; the cell is the one
void cell of the n = 20 ROM (its parent mesh, transformation modes and
material), the void shapes those of the shape fields over the block.  Every
value comes from the oracle (oracle/fe2.py, oracle/fom.py).

    python tests/golden/make_fe2_fom.py [--workers K]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402
from oracle import build_rom, fe2  # noqa: E402

MESH, STEPS, PEAK, CELL = (4, 2), 8, 0.01, 'onevoid_n20_m120'
OUT = os.path.join(HERE, 'fe2_fom_4x2.json')


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument('--workers', type=int, default=min(8, os.cpu_count() or 1))
    a = ap.parse_args(argv)
    mesh = workloads.fe2_mesh(*MESH)
    Xg = fe2.geometry(mesh)['Xg']
    mu = workloads.fe2_shape(Xg[:, 0], Xg[:, 1])
    loads = workloads.fe2_loads(STEPS, PEAK)
    rve = fe2.FomRve(build_rom.ROMS[CELL], workers=a.workers)
    t0 = time.time()
    out = fe2.run(rve, mesh, mu, loads)
    rve.close()
    res = dict(cite="Sec. 4.2 (two-scale example; compliance and its relative error per load step)",
               macro_mesh=list(MESH), load_steps=STEPS, peak_traction=PEAK, cell=CELL, rve="full order",
               dofs_per_rve=int(rve.n), gauss_points=int(Xg.shape[0]),
               loads=[float(x) for x in loads], status=[int(o['status']) for o in out],
               macro_iters=[int(o['macro_iters']) for o in out], compliance=[float(o['C']) for o in out],
               seconds=time.time() - t0)
    with open(OUT, 'w') as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res))
    return 0


if __name__ == '__main__':
    sys.exit(main())

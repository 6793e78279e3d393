"""ROM artifact file: the output of the offline stage of Algorithm 1.

Everything the online hyper-reduced solve needs, for one parent domain:
the ECM rule (weights w_q > 0 at the selected points), the parent gradients
of the POD modes at those points, the parent gradients of the auxiliary
transformation modes at those points, the material constants and the map
from shape parameters mu to the affine transformation coefficients.

Layout (little-endian), 256-byte header then FP64 / int64 arrays:

  off  type       field
    0  char[8]    magic "PODECMR1"
    8  uint32     version (1)
   12  uint32     n        reduced displacement modes
   16  uint32     m        ECM points
   20  uint32     c        affine transformation coefficients
   24  uint32     kind     mu -> c map (0: one void (a, b); 1: four voids; 2: inclusions scaled by zeta)
   28  uint32     n_mu     shape parameters per macro point
   32  f64[4]     E, nu, sigma_y0, H
   64  f64        r0        parent void radius
   72  f64        void_area area of each mapped void (kind 1)
   80  f64        cell_area |cell| used to normalise effective quantities
   88  f64[4]     E, nu, sigma_y0, H of the second phase (version 2)
  120  ...        zero padding to 256
  256  f64[m]          w        ECM weights
       f64[m][4][n]    G        G[q][2 i + J][k] = d(phi_k)_i / dX^p_J at point q
       f64[m][4][c]    Gd       Gd[q][2 i + J][k] = d(dhat_k)_i / dX^p_J
       int64[m]        src      index of the point in the full rule
       int64[m]        phase    material of the point, 0 or 1 (version 2)

Version 1 is a single-phase cell (the material at offset 32 everywhere);
version 2 adds a second phase for multi-phase cells.
"""
import numpy as np

MAGIC = b"PODECMR1"
VERSION = 1
VERSION_PHASES = 2
HEADER = 256


def write(path, n, m, c, kind, n_mu, mat, r0, void_area, cell_area, w, G, Gd, src, mat2=None, phase=None):
    hdr = bytearray(HEADER)
    hdr[0:8] = MAGIC
    two = phase is not None
    np.frombuffer(hdr, dtype='<u4', count=6, offset=8)[:] = [VERSION_PHASES if two else VERSION, n, m, c, kind, n_mu]
    np.frombuffer(hdr, dtype='<f8', count=7, offset=32)[:] = list(mat) + [r0, void_area, cell_area]
    if two:
        np.frombuffer(hdr, dtype='<f8', count=4, offset=88)[:] = list(mat2)
    w = np.ascontiguousarray(w, dtype='<f8')
    G = np.ascontiguousarray(G, dtype='<f8')
    Gd = np.ascontiguousarray(Gd, dtype='<f8')
    src = np.ascontiguousarray(src, dtype='<i8')
    assert w.shape == (m,) and G.shape == (m, 4, n) and Gd.shape == (m, 4, c) and src.shape == (m,)
    arrays = [w, G, Gd, src]
    if two:
        phase = np.ascontiguousarray(phase, dtype='<i8')
        assert phase.shape == (m,) and np.all((phase == 0) | (phase == 1))
        arrays.append(phase)
    with open(path, 'wb') as fh:
        fh.write(bytes(hdr))
        for a in arrays:
            fh.write(a.tobytes())


def read(path):
    raw = open(path, 'rb').read()
    if raw[:8] != MAGIC:
        raise ValueError("not a ROM artifact")
    version, n, m, c, kind, n_mu = np.frombuffer(raw, dtype='<u4', count=6, offset=8)
    if version not in (VERSION, VERSION_PHASES):
        raise ValueError("unsupported artifact version")
    E, nu, sy0, H, r0, void_area, cell_area = np.frombuffer(raw, dtype='<f8', count=7, offset=32)
    off = HEADER
    n, m, c = int(n), int(m), int(c)

    def take(count, dt):
        nonlocal off
        a = np.frombuffer(raw, dtype=dt, count=count, offset=off).copy()
        off += count * 8
        return a

    w = take(m, '<f8')
    G = take(m * 4 * n, '<f8').reshape(m, 4, n)
    Gd = take(m * 4 * c, '<f8').reshape(m, 4, c)
    src = take(m, '<i8')
    if version == VERSION_PHASES:
        mat2 = tuple(np.frombuffer(raw, dtype='<f8', count=4, offset=88))
        phase = take(m, '<i8')
    else:
        mat2, phase = None, np.zeros(m, dtype=np.int64)
    return dict(n=n, m=m, c=c, kind=int(kind), n_mu=int(n_mu), mat=(E, nu, sy0, H), r0=r0,
                void_area=void_area, cell_area=cell_area, w=w, G=G, Gd=Gd, src=src, mat2=mat2, phase=phase)

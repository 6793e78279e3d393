"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module generates random inputs only (shape parameters and macroscopic
deformation-gradient paths); it contains none of the method's arithmetic.
Every draw uses numpy.random.Generator(PCG64(seed)).

Load paths follow the paper's practice of sampling the symmetric stretch
Ubar (Sec. 4: Fbar = Rbar Ubar, only Ubar needs sampling) and applying it with
an amplitude function beta(k):

* monotone: Fbar_k = I + (k / K) E, k = 1..K;
* cyclic:   beta rises 0 -> 1 over K/2 steps and falls back to 0
            (load / unload, as in the paper's training paths).

E is symmetric with a uniformly random direction in (E_xx, E_yy, E_xy)
space, normalised to the Frobenius norm rho of the 2x2 tensor.
"""
import numpy as np
from scipy.stats import qmc

ONE_VOID_MU = (0.15, 0.35)          # semi-axes a, b of the elliptical void
FOUR_VOID_KAPPA = (1.0, 1.5)        # aspect ratio b/a per void
FOUR_VOID_THETA = (0.0, np.pi)      # orientation per void


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _directions(g, P):
    d = g.uniform(-1.0, 1.0, size=(P, 3))
    E = np.zeros((P, 2, 2))
    E[:, 0, 0] = d[:, 0]
    E[:, 1, 1] = d[:, 1]
    E[:, 0, 1] = E[:, 1, 0] = d[:, 2]
    E /= np.linalg.norm(E.reshape(P, 4), axis=1)[:, None, None]
    return E


def monotone_paths(seed, P, steps=10, rho=(0.02, 0.05)):
    """(P, steps, 2, 2) monotone paths with |Fbar - I|_F <= rho_max."""
    g = rng(seed)
    E = _directions(g, P) * g.uniform(*rho, size=P)[:, None, None]
    beta = np.arange(1, steps + 1) / steps
    return np.eye(2)[None, None] + beta[None, :, None, None] * E[:, None]


def cyclic_paths(seed, P, steps=20, rho=(0.02, 0.08)):
    """(P, steps, 2, 2) load / unload paths with amplitude <= rho_max."""
    g = rng(seed)
    E = _directions(g, P) * g.uniform(*rho, size=P)[:, None, None]
    half = steps // 2
    beta = np.concatenate([np.arange(1, half + 1) / half,
                           1.0 - np.arange(1, steps - half + 1) / (steps - half)])
    return np.eye(2)[None, None] + beta[None, :, None, None] * E[:, None]


def one_void_mu(seed, P):
    return rng(seed).uniform(*ONE_VOID_MU, size=(P, 2))


def four_void_mu(seed, P):
    g = rng(seed)
    mu = np.empty((P, 8))
    mu[:, 0::2] = g.uniform(*FOUR_VOID_KAPPA, size=(P, 4))
    mu[:, 1::2] = g.uniform(*FOUR_VOID_THETA, size=(P, 4))
    return mu


def sobol_points(seed, count, lo, hi):
    """Scrambled Sobol samples in the box [lo, hi] (training designs)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    s = qmc.Sobol(d=lo.size, scramble=True, seed=rng(seed))
    return qmc.scale(s.random(count), lo, hi)


def one_void_training_mu(seed, count):
    return sobol_points(seed, count, [ONE_VOID_MU[0]] * 2, [ONE_VOID_MU[1]] * 2)


def four_void_training_mu(seed, count):
    lo = [FOUR_VOID_KAPPA[0], FOUR_VOID_THETA[0]] * 4
    hi = [FOUR_VOID_KAPPA[1], FOUR_VOID_THETA[1]] * 4
    return sobol_points(seed, count, lo, hi)


def inclusion_layout(seed, count=23, fraction=0.234, grow=1.2, gap=0.012, aspect=(0.6, 1.0), spread=(0.75, 1.25),
                     tries=20000):
    """Random non-overlapping elliptical inclusions in the unit cell (the
    composite cell of Sec. 4.1): `count` ellipses of total area `fraction`,
    semi-axis ratio U[aspect], orientation U[0, pi), sizes spread by U[spread]
    around the mean, placed one after another (largest first) at uniform
    random centres, rejected unless the ellipse grown by `grow` (the largest
    shape parameter) and a `gap` keeps clear of the cell boundary and of the
    grown earlier ones.  Returns (count, 5): cx, cy, a, b, theta."""
    g = rng(seed)
    s = g.uniform(*spread, size=count)
    kap = g.uniform(*aspect, size=count)          # b / a
    th = g.uniform(0.0, np.pi, size=count)
    area = fraction * s ** 2 / np.sum(s ** 2)      # pi a b each
    a = np.sqrt(area / (np.pi * kap))
    b = kap * a
    order = np.argsort(-area)
    t = np.linspace(0.0, 2.0 * np.pi, 96, endpoint=False)
    placed = []

    def boundary(c, aa, bb, tt, f):
        R = np.array([[np.cos(tt), -np.sin(tt)], [np.sin(tt), np.cos(tt)]])
        return c + (R @ np.stack([f * aa * np.cos(t), f * bb * np.sin(t)])).T

    def inside(pts, c, aa, bb, tt, f):
        R = np.array([[np.cos(tt), -np.sin(tt)], [np.sin(tt), np.cos(tt)]])
        q = (pts - c) @ R
        return (q[:, 0] / (f * aa)) ** 2 + (q[:, 1] / (f * bb)) ** 2 <= 1.0

    for i in order:
        for _ in range(tries):
            c = g.uniform(0.0, 1.0, size=2)
            f = grow * (1.0 + gap / max(a[i], 1e-12))
            B = boundary(c, a[i], b[i], th[i], f)
            if B.min() < gap or B.max() > 1.0 - gap:
                continue
            ok = True
            for (cj, aj, bj, tj) in placed:
                fj = grow * (1.0 + gap / aj)
                if inside(B, cj, aj, bj, tj, fj).any() or inside(boundary(cj, aj, bj, tj, fj), c, a[i], b[i], th[i], f).any():
                    ok = False
                    break
            if ok:
                placed.append((c, a[i], b[i], th[i]))
                break
        else:
            raise RuntimeError("inclusion layout: no room left")
    return np.array([[c[0], c[1], aa, bb, tt] for c, aa, bb, tt in placed])


def inclusion_mu(seed, P, lo=0.5, hi=1.2):
    """Inclusion scale zeta ~ U[lo, hi] (Sec. 4.1: 0.5 to 1.2), one per point."""
    return rng(seed).uniform(lo, hi, size=(P, 1))


def inclusion_training_mu(seed, count, lo=0.5, hi=1.2):
    return sobol_points(seed, count, [lo], [hi])


def uneven_steps(seed, P, lo=5, hi=40):
    """Per-point step counts, uniform in [lo, hi]."""
    return rng(seed).integers(lo, hi + 1, size=P)


def uneven_cyclic_paths(seed, P, nsteps, rho=(0.02, 0.08)):
    """Per-point load / unload paths of their own lengths nsteps[p]: beta rises
    to 1 over the first half of the point's steps and falls back.  Returned
    as (P, max(nsteps), 2, 2), padded with the last target."""
    g = rng(seed)
    E = _directions(g, P) * g.uniform(*rho, size=P)[:, None, None]
    Kmax = int(np.max(nsteps))
    out = np.empty((P, Kmax, 2, 2))
    for p in range(P):
        K = int(nsteps[p])
        half = max(K // 2, 1)
        beta = np.concatenate([np.arange(1, half + 1) / half, 1.0 - np.arange(1, K - half + 1) / max(K - half, 1)])
        beta = np.concatenate([beta, np.full(Kmax - K, beta[-1])])
        out[p] = np.eye(2)[None] + beta[:, None, None] * E[p][None]
    return out


# ---------------------------------------------------------------------------
# Two-scale workload (Sec. 4.2 setting, rescaled to the ROMs' material):
# a W x H block meshed with nx x ny eight-node quadrilaterals, fixed at the
# bottom, loaded on the top edge by a downward parabolic traction of peak
# Tbar_k; the void shape varies smoothly over the block.

FE2_WIDTH, FE2_HEIGHT = 2.0, 1.0
FE2_KAPPA = (1.4, 1.01)     # kappa(x, y) = KAPPA[0] - (KAPPA[0] - KAPPA[1]) y / H
FE2_VOID = (0.12, 0.20)     # v(x, y) = VOID[0] + (VOID[1] - VOID[0]) (1 - x / (W / 2))^2


def fe2_mesh(nx, ny, width=FE2_WIDTH, height=FE2_HEIGHT):
    """Structured Q8 mesh of [0, width] x [0, height].

    Nodes are numbered column by column in x (corner columns carry 2 ny + 1
    nodes, the columns between them ny + 1), which keeps the bandwidth of
    the stiffness small.  Element nodes: corners counterclockwise from
    (-1, -1), then the midsides of the edges bottom, right, top, left.
    Returns X (nodes, 2), conn (elements, 8), bottom (nodes on y = 0) and
    top (elements, 3: nodes of each top edge from left to right)."""
    dx, dy = width / nx, height / ny
    X, full, mid = [], {}, {}
    for c in range(2 * nx + 1):
        x = 0.5 * c * dx
        for j in range(2 * ny + 1):
            if c % 2 == 1 and j % 2 == 1:
                continue
            (full if c % 2 == 0 else mid)[(c, j)] = len(X)
            X.append((x, 0.5 * j * dy))
    node = {**full, **mid}
    conn, top = [], []
    for i in range(nx):
        for j in range(ny):
            c0, c1, j0, j1 = 2 * i, 2 * i + 2, 2 * j, 2 * j + 2
            e = [node[(c0, j0)], node[(c1, j0)], node[(c1, j1)], node[(c0, j1)],
                 node[(c0 + 1, j0)], node[(c1, j0 + 1)], node[(c0 + 1, j1)], node[(c0, j0 + 1)]]
            conn.append(e)
            if j == ny - 1:
                top.append((e[3], e[6], e[2]))
    X = np.array(X)
    bottom = np.flatnonzero(X[:, 1] == 0.0)
    return dict(X=X, conn=np.array(conn, dtype=np.int32), bottom=bottom.astype(np.int32),
                top=np.array(top, dtype=np.int32), width=width, height=height)


def fe2_shape(x, y, width=FE2_WIDTH, height=FE2_HEIGHT):
    """Semi-axes (a, b) of the one-void cell at reference position (x, y):
    aspect ratio kappa = b / a and void fraction v = pi a b of the unit cell
    vary linearly in y and quadratically in x."""
    kappa = FE2_KAPPA[0] - (FE2_KAPPA[0] - FE2_KAPPA[1]) * np.asarray(y) / height
    v = FE2_VOID[0] + (FE2_VOID[1] - FE2_VOID[0]) * (1.0 - np.asarray(x) / (0.5 * width)) ** 2
    a = np.sqrt(v / (np.pi * kappa))
    return np.stack([a, kappa * a], axis=-1)


def fe2_loads(steps, peak):
    """Peak traction per load step: up linearly to `peak` over steps / 2
    steps, then back to zero."""
    half = steps // 2
    beta = np.concatenate([np.arange(1, half + 1) / half,
                           1.0 - np.arange(1, steps - half + 1) / (steps - half)])
    return peak * beta


# ---------------------------------------------------------------------------
# Offline-stage inputs: snapshot sets with a prescribed spectrum and sparse
# SPD weights with the pattern of a mass-plus-stiffness matrix (POD), and
# smooth integrands at the points of a uniform grid (cubature).

def pod_snapshots(seed, nrow, ns, rank, decay, noise):
    """(nrow, ns): rank-`rank` snapshots with singular values decay**k plus
    Gaussian noise of size `noise`."""
    g = rng(seed)
    U = np.linalg.qr(g.standard_normal((nrow, rank)))[0]
    V = np.linalg.qr(g.standard_normal((ns, rank)))[0]
    return (U * decay ** np.arange(rank)) @ V.T + noise * g.standard_normal((nrow, ns))


def banded_spd(seed, nrow, bw):
    """Sparse symmetric positive definite (nrow, nrow) matrix with bw off-
    diagonals on each side (diagonally dominant)."""
    import scipy.sparse as sp
    g = rng(seed)
    diags = [g.uniform(-0.1, 0.1, nrow - k) for k in range(1, bw + 1)]
    A = sp.diags(diags, list(range(1, bw + 1)), shape=(nrow, nrow))
    return (A + A.T + sp.diags(np.full(nrow, 1.0 + 0.2 * bw))).tocsr()


def grid_points(nx, ny):
    """Cell centres of an nx x ny grid on the unit square and equal weights."""
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y, indexing='ij')
    return np.stack([X.ravel(), Y.ravel()], axis=1), np.full(nx * ny, 1.0 / (nx * ny))


def cos_integrands(seed, pts, R):
    """(R, points): cos(pi k x + a_k) cos(pi l y + b_l) for the first R pairs
    (k, l) of a K x K table, random phases."""
    g = rng(seed)
    K = int(np.ceil(np.sqrt(R)))
    x, y = pts[:, 0], pts[:, 1]
    ph, ps = g.uniform(0, 2 * np.pi, K), g.uniform(0, 2 * np.pi, K)
    return np.array([np.cos(np.pi * k * x + ph[k]) * np.cos(np.pi * l * y + ps[l])
                     for k in range(K) for l in range(K)][:R])

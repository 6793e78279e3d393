"""Parent-domain meshes: six-node triangles with three interior Gauss points.

The paper discretises its RVEs with 6-node quadratic triangles and three
quadrature points per element (Sec. 4.1 and 4.2 problem descriptions).  It
does not say which three-point rule; the one used here is the degree-2
interior rule with points (1/6, 1/6), (2/3, 1/6), (1/6, 2/3) and weight 1/6
each on the reference triangle.

Parent geometry is the unit cell [0, 1]^2 (Sec. 4: RVEs of size [0, 1]^2),
optionally with circular voids.  Meshes are built by a mapped (transfinite)
block mesher: each void sits in a square sub-cell split into four blocks that
join one side of the sub-cell to a quarter of the circle.  Opposite cell sides
carry the same node distribution, so boundary nodes pair periodically.
Mid-side nodes are placed by the block map, so edges on a void follow the
circle.

The composite cell (Sec. 4.1: stiff elliptical inclusions in a plastic
matrix) is meshed without fitting the inclusions: a structured mesh of the
cell, the phase of every quadrature point decided by whether it lies in an
ellipse, and the nodes inside an ellipse marked as carrying that inclusion's
transformation data (the auxiliary problem prescribes them; see
auxiliary.py).  The interface is thus resolved to the element size.
"""
import numpy as np

# reference 3-point rule (area coordinates L2 = xi, L3 = eta)
QP_REF = np.array([[1.0 / 6.0, 1.0 / 6.0], [2.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 2.0 / 3.0]])
QW_REF = np.array([1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0])


def t6_shape(xi, eta):
    """Shape functions and reference gradients of the 6-node triangle.

    Node order: corners 0, 1, 2 then mid-sides 01, 12, 20.
    Returns N (6,), dN (6, 2) with dN[a, k] = dN_a / d(xi, eta)_k.
    """
    L1 = 1.0 - xi - eta
    L2 = xi
    L3 = eta
    N = np.array([L1 * (2 * L1 - 1), L2 * (2 * L2 - 1), L3 * (2 * L3 - 1),
                  4 * L1 * L2, 4 * L2 * L3, 4 * L3 * L1])
    dL = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
    Ls = (L1, L2, L3)
    dN = np.zeros((6, 2))
    for a in range(3):
        dN[a] = (4 * Ls[a] - 1) * dL[a]
    pairs = [(0, 1), (1, 2), (2, 0)]
    for k, (a, b) in enumerate(pairs):
        dN[3 + k] = 4 * (Ls[a] * dL[b] + Ls[b] * dL[a])
    return N, dN


class Mesh:
    """T6 mesh with quadrature data.

    Attributes
    ----------
    X      : (nn, 2) node coordinates.
    T      : (ne, 6) connectivity.
    void_of_node : (nn,) index of the void whose boundary carries the node,
                   -1 otherwise.
    voids  : list of (cx, cy, r0).
    qX     : (nq, 2) quadrature point coordinates, nq = 3 ne, q = 3 e + g.
    qw     : (nq,) physical quadrature weights w_ref * det J.
    qN     : (nq, 6) shape-function values.
    qdN    : (nq, 6, 2) physical shape-function gradients dN_a / dX_k.
    """

    def __init__(self, X, T, void_of_node, voids):
        self.X = np.asarray(X, dtype=np.float64)
        self.T = np.asarray(T, dtype=np.int64)
        self.void_of_node = np.asarray(void_of_node, dtype=np.int64)
        self.voids = list(voids)
        self._orient()
        self._quadrature()

    @property
    def nn(self):
        return self.X.shape[0]

    @property
    def ne(self):
        return self.T.shape[0]

    @property
    def nq(self):
        return 3 * self.ne

    def _orient(self):
        # make every element counter-clockwise (positive corner area)
        x = self.X[self.T[:, :3]]
        area2 = ((x[:, 1, 0] - x[:, 0, 0]) * (x[:, 2, 1] - x[:, 0, 1])
                 - (x[:, 2, 0] - x[:, 0, 0]) * (x[:, 1, 1] - x[:, 0, 1]))
        flip = area2 < 0
        T = self.T.copy()
        # swap corners 1 and 2: mid-sides 01 <-> 20, 12 stays
        T[flip] = self.T[flip][:, [0, 2, 1, 5, 4, 3]]
        self.T = T

    def _quadrature(self):
        ne = self.ne
        Xe = self.X[self.T]  # (ne, 6, 2)
        qX = np.zeros((ne, 3, 2))
        qw = np.zeros((ne, 3))
        qN = np.zeros((ne, 3, 6))
        qdN = np.zeros((ne, 3, 6, 2))
        for g in range(3):
            N, dN = t6_shape(*QP_REF[g])
            Jm = np.einsum('eak,al->ekl', Xe, dN)  # dX_k / dxi_l
            det = Jm[:, 0, 0] * Jm[:, 1, 1] - Jm[:, 0, 1] * Jm[:, 1, 0]
            if np.any(det <= 0):
                raise ValueError("non-positive element Jacobian")
            Jinv = np.empty_like(Jm)
            Jinv[:, 0, 0] = Jm[:, 1, 1] / det
            Jinv[:, 1, 1] = Jm[:, 0, 0] / det
            Jinv[:, 0, 1] = -Jm[:, 0, 1] / det
            Jinv[:, 1, 0] = -Jm[:, 1, 0] / det
            qX[:, g] = np.einsum('eak,a->ek', Xe, N)
            qw[:, g] = QW_REF[g] * det
            qN[:, g] = N
            # dN_a/dX_k = dN_a/dxi_l * dxi_l/dX_k
            qdN[:, g] = np.einsum('al,elk->eak', dN, Jinv)
        self.qX = qX.reshape(-1, 2)
        self.qw = qw.reshape(-1)
        self.qN = qN.reshape(-1, 6)
        self.qdN = qdN.reshape(-1, 6, 2)
        self.qelem = np.repeat(np.arange(ne), 3)

    def outer_boundary_nodes(self, tol=1e-12):
        x, y = self.X[:, 0], self.X[:, 1]
        return np.nonzero((np.abs(x) < tol) | (np.abs(x - 1) < tol)
                          | (np.abs(y) < tol) | (np.abs(y - 1) < tol))[0]


class _NodeMerger:
    """Collect points, merging coordinates equal to within a tolerance."""

    def __init__(self, scale=1e11):
        self.scale = scale
        self.index = {}
        self.pts = []
        self.void = []

    def add(self, p, void=-1):
        key = (int(round(p[0] * self.scale)), int(round(p[1] * self.scale)))
        i = self.index.get(key)
        if i is None:
            i = len(self.pts)
            self.index[key] = i
            self.pts.append((float(p[0]), float(p[1])))
            self.void.append(void)
        elif void >= 0:
            self.void[i] = void
        return i


def _add_quad_grid(merger, elems, P, void_row):
    """Triangulate a (2a+1) x (2b+1) grid of mapped points into T6 elements.

    P[i, j] are points on the fine grid (i along the block side, j radial);
    row j = 0 lies on a void if void_row >= 0.
    """
    n1, n2 = P.shape[0], P.shape[1]
    ids = np.empty((n1, n2), dtype=np.int64)
    for i in range(n1):
        for j in range(n2):
            ids[i, j] = merger.add(P[i, j], void_row if j == 0 else -1)
    for I in range(0, n1 - 1, 2):
        for J in range(0, n2 - 1, 2):
            a, b = ids[I, J], ids[I + 2, J]
            c, d = ids[I + 2, J + 2], ids[I, J + 2]
            # alternate the diagonal for a symmetric pattern
            if ((I // 2) + (J // 2)) % 2 == 0:
                elems.append([a, b, c, ids[I + 1, J], ids[I + 2, J + 1], ids[I + 1, J + 1]])
                elems.append([a, c, d, ids[I + 1, J + 1], ids[I + 1, J + 2], ids[I, J + 1]])
            else:
                elems.append([a, b, d, ids[I + 1, J], ids[I + 1, J + 1], ids[I, J + 1]])
                elems.append([b, c, d, ids[I + 2, J + 1], ids[I + 1, J + 2], ids[I + 1, J + 1]])


def _void_subcell(merger, elems, cx, cy, hw, r0, nt, nr, void_index, grading=1.0):
    """Four mapped blocks between the square [c-hw, c+hw]^2 and a circle."""
    t = np.linspace(0.0, 1.0, 2 * nt + 1)
    rho = np.linspace(0.0, 1.0, 2 * nr + 1) ** grading
    corners = np.array([[cx - hw, cy - hw], [cx + hw, cy - hw], [cx + hw, cy + hw], [cx - hw, cy + hw]])
    theta0 = [-0.75 * np.pi, -0.25 * np.pi, 0.25 * np.pi, 0.75 * np.pi]
    for k in range(4):
        c0, c1 = corners[k], corners[(k + 1) % 4]
        P = np.zeros((t.size, rho.size, 2))
        for i, ti in enumerate(t):
            side = c0 + ti * (c1 - c0)
            th = theta0[k] + ti * 0.5 * np.pi
            arc = np.array([cx + r0 * np.cos(th), cy + r0 * np.sin(th)])
            for j, rj in enumerate(rho):
                P[i, j] = (1.0 - rj) * arc + rj * side
        _add_quad_grid(merger, elems, P, void_index)


def mesh_voids(voids, nt, nr, grading=1.0):
    """Unit cell with circular voids, each centred in its own square sub-cell.

    voids : list of (cx, cy, r0); sub-cells tile [0, 1]^2 (1 void: the whole
            cell, 4 voids: the 2x2 sub-cells).
    nt, nr: element-pair counts along each block side and radially.
    """
    nv = len(voids)
    if nv == 1:
        hw = 0.5
    elif nv == 4:
        hw = 0.25
    else:
        raise ValueError("1 or 4 voids supported")
    merger = _NodeMerger()
    elems = []
    for v, (cx, cy, r0) in enumerate(voids):
        _void_subcell(merger, elems, cx, cy, hw, r0, nt, nr, v, grading)
    return Mesh(np.array(merger.pts), np.array(elems), np.array(merger.void), voids)


def mesh_square(nx):
    """Void-free unit cell, structured: nx x nx quads, two T6 each."""
    merger = _NodeMerger()
    elems = []
    s = np.linspace(0.0, 1.0, 2 * nx + 1)
    P = np.zeros((s.size, s.size, 2))
    P[..., 0] = s[:, None]
    P[..., 1] = s[None, :]
    _add_quad_grid(merger, elems, P, -1)
    return Mesh(np.array(merger.pts), np.array(elems), np.array(merger.void), [])


def one_void_cell(r0, nt, nr, grading=1.0):
    return mesh_voids([(0.5, 0.5, r0)], nt, nr, grading)


def four_void_cell(r0, nt, nr, grading=1.0):
    c = [0.25, 0.75]
    return mesh_voids([(c[i], c[j], r0) for j in range(2) for i in range(2)], nt, nr, grading)


def in_ellipses(P, inclusions):
    """Index of the ellipse (cx, cy, a, b, theta) containing each point of
    P (k, 2) (boundary included), -1 outside all."""
    P = np.asarray(P, dtype=np.float64)
    out = np.full(P.shape[0], -1, dtype=np.int64)
    for i, (cx, cy, a, b, th) in enumerate(np.asarray(inclusions, dtype=np.float64)):
        c, sn = np.cos(th), np.sin(th)
        dx, dy = P[:, 0] - cx, P[:, 1] - cy
        u = c * dx + sn * dy    # coordinates in the ellipse's axes
        v = -sn * dx + c * dy
        out[(u / a) ** 2 + (v / b) ** 2 <= 1.0] = i
    return out


def inclusion_cell(nx, inclusions):
    """Structured nx x nx cell with elliptical inclusions (cx, cy, a, b,
    theta): nodes inside inclusion i carry void_of_node = i and voids[i] =
    (cx, cy, 0) holds its centre (the point its transformation scales about);
    qphase gives 1 at the quadrature points inside an inclusion."""
    m = mesh_square(nx)
    m.inclusions = np.asarray(inclusions, dtype=np.float64)
    m.void_of_node = in_ellipses(m.X, m.inclusions)
    m.voids = [(float(c[0]), float(c[1]), 0.0) for c in m.inclusions]
    m.qphase = (in_ellipses(m.qX, m.inclusions) >= 0).astype(np.int64)
    return m

"""Finite-element operators of the mapped RVE problem (Sec. 2.1).

The unknown is the periodic fluctuation w^p on the parent domain (space V^p,
eq. weakform-dep-mapped).  Periodicity is imposed by identifying each node on
the sides x = 1 and y = 1 with its partner on x = 0 and y = 0 (all four
corners become one node).  The paper does not say how the rigid translation
of w is removed; here the corner node is fixed to w = 0, which leaves the
effective stress unchanged.

Gradients are stored as 4-vectors in the component order
[11, 12, 21, 22] = index 2 i + J of dw_i / dX_J.
"""
import numpy as np
import scipy.sparse as sp


class PeriodicSpace:
    """Independent DOFs of the periodic fluctuation field with the corner fixed."""

    def __init__(self, mesh, tol=1e-9):
        X = mesh.X
        key = np.round(np.mod(X + tol, 1.0) - tol, 9)
        key[np.abs(key) < tol] = 0.0
        # master node: the node carrying the key, preferring x < 1 and y < 1
        order = np.lexsort((X[:, 1], X[:, 0]))
        master_of_key = {}
        for i in order:
            k = (key[i, 0], key[i, 1])
            if k not in master_of_key:
                master_of_key[k] = i
        masters = np.array([master_of_key[(key[i, 0], key[i, 1])] for i in range(mesh.nn)])
        uniq = np.unique(masters)
        corner = master_of_key[(0.0, 0.0)]
        free = uniq[uniq != corner]
        node_index = -np.ones(mesh.nn, dtype=np.int64)
        node_index[free] = np.arange(free.size)
        self.mesh = mesh
        self.master = masters
        self.free_nodes = free
        self.node_dof = node_index[masters]  # -1 for the fixed corner
        self.ndof = 2 * free.size

    def expand(self, w):
        """Nodal fluctuation (nn, 2) from the reduced DOF vector."""
        out = np.zeros((self.mesh.nn, 2))
        idx = self.node_dof
        ok = idx >= 0
        out[ok, 0] = w[2 * idx[ok]]
        out[ok, 1] = w[2 * idx[ok] + 1]
        return out


def gradient_operator(mesh, node_dof, ndof):
    """Sparse map from DOFs to parent gradients at all quadrature points.

    Row 4 q + 2 i + J holds d w_i / d X_J at point q.  node_dof[a] is the
    DOF block of node a (DOFs 2 k, 2 k + 1) or -1 for a fixed node.
    """
    nq = mesh.nq
    rows, cols, vals = [], [], []
    Tq = mesh.T[mesh.qelem]  # (nq, 6)
    for a in range(6):
        blk = node_dof[Tq[:, a]]
        ok = blk >= 0
        q = np.nonzero(ok)[0]
        for i in range(2):
            for J in range(2):
                rows.append(4 * q + 2 * i + J)
                cols.append(2 * blk[ok] + i)
                vals.append(mesh.qdN[q, a, J])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(4 * nq, ndof))


def value_operator(mesh, node_dof, ndof):
    """Sparse map from DOFs to values w_i at all quadrature points (row 2 q + i)."""
    nq = mesh.nq
    rows, cols, vals = [], [], []
    Tq = mesh.T[mesh.qelem]
    for a in range(6):
        blk = node_dof[Tq[:, a]]
        ok = blk >= 0
        q = np.nonzero(ok)[0]
        for i in range(2):
            rows.append(2 * q + i)
            cols.append(2 * blk[ok] + i)
            vals.append(mesh.qN[q, a])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(2 * nq, ndof))


def block_diag4(D):
    """Sparse block-diagonal matrix from (nq, 4, 4) blocks."""
    nq = D.shape[0]
    base = 4 * np.arange(nq)
    r = (base[:, None, None] + np.arange(4)[None, :, None]) + 0 * np.arange(4)[None, None, :]
    c = (base[:, None, None] + np.arange(4)[None, None, :]) + 0 * np.arange(4)[None, :, None]
    return sp.csr_matrix((D.reshape(-1), (r.reshape(-1), c.reshape(-1))), shape=(4 * nq, 4 * nq))


def right_map(Finv):
    """T with vec(H F_mu^-1) = T vec(H): T[(i j), (i r)] = (F_mu^-1)_{r j}.

    Finv: (..., 2, 2).  Returns (..., 4, 4).
    """
    T = np.zeros(Finv.shape[:-2] + (4, 4))
    for i in range(2):
        for j in range(2):
            for r in range(2):
                T[..., 2 * i + j, 2 * i + r] = Finv[..., r, j]
    return T


class Problem:
    """The discrete mapped RVE problem for one transformation F_mu.

    Holds the parent gradient operator, quadrature weights and the
    transformation at the quadrature points; evaluates the residual
    f (eq. full_system) and stiffness K (linearisation eq. Dweakform-dep).
    """

    def __init__(self, mesh, space, Fmu, mat, cell_area=1.0):
        self.mesh = mesh
        self.space = space
        self.Gop = gradient_operator(mesh, space.node_dof, space.ndof)
        self.GopT = self.Gop.T.tocsr()
        self.Fmu = Fmu
        self.Finv = np.linalg.inv(Fmu)
        self.J = np.linalg.det(Fmu)
        if np.any(self.J <= 0):
            raise ValueError("transformation not invertible (det F_mu <= 0)")
        self.T = right_map(self.Finv)
        self.mat = mat
        self.qw = mesh.qw
        self.cell_area = cell_area

    def deformation(self, w, Fbar):
        Hp = (self.Gop @ w).reshape(-1, 2, 2)
        return Fbar[None] + Hp @ self.Finv

    def evaluate(self, w, Fbar, hist, material_point):
        """Residual, stiffness and point data at fluctuation DOFs w."""
        F = self.deformation(w, Fbar)
        P, A, Fp, Fp33, xi, gam = material_point(F, *hist, self.mat)
        wJ = self.qw * np.abs(self.J)
        # weighted stress W = P F_mu^-T |det F_mu| (eq. forcevector_rewritten)
        W = P @ np.swapaxes(self.Finv, -1, -2) * np.abs(self.J)[:, None, None]
        f = self.GopT @ (self.qw[:, None, None] * W).reshape(-1)
        A4 = A.reshape(-1, 4, 4)
        D = np.einsum('qab,qbc,qcd->qad', np.swapaxes(self.T, -1, -2), A4, self.T) * wJ[:, None, None]
        K = (self.GopT @ block_diag4(D) @ self.Gop).tocsc()
        return dict(f=f, K=K, F=F, P=P, A=A, W=W, hist=(Fp, Fp33, xi), gamma=gam, wJ=wJ)

    def effective_stress(self, ev):
        """eq. eff_stress_full, normalised by the cell area."""
        return np.einsum('q,qij->ij', ev['wJ'], ev['P']) / self.cell_area

    def effective_stiffness(self, ev, solve):
        """eq. eff_stiffness_full with the tangent problems eq. tangentproblem.

        solve(K, B) returns K^-1 B.  Returns Abar (2, 2, 2, 2).
        """
        wJ = ev['wJ']
        A4 = ev['A'].reshape(-1, 4, 4)
        # right-hand sides: -int (grad dw F^-1) : A |J| : E_kl
        TA = np.einsum('qba,qbc->qac', self.T, A4) * wJ[:, None, None]  # T^T A
        B = -(self.GopT @ TA.reshape(-1, 4))  # (ndof, 4)
        Q = solve(ev['K'], B)  # q_kl for the 4 components
        dH = (self.Gop @ Q).reshape(-1, 4, 4)  # parent gradient of q_kl, column kl
        dF = np.einsum('qab,qbk->qak', self.T, dH)  # mapped
        Abar = np.einsum('q,qab,qbk->ak', wJ, A4, np.eye(4)[None] + dF) / self.cell_area
        return Abar.reshape(2, 2, 2, 2)

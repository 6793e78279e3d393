"""Proper orthogonal decomposition of snapshot sets (Sec. 3.1, 3.2).

Fluctuation modes phi_n (eq. pod_disp) are orthonormal in the V^p inner
product (eq. Vdotproduct taken on the parent domain, as the basis lives
there): (u, v)_V = int u . v + grad u : grad v dX^p, whose Gram matrix on the
DOFs is M_V = M + K_H1.  Weighted-stress modes B_l (eq. weighted_stress_pod)
are orthonormal in L^2 of the parent domain (eq. pod_P_orthonormal), with the
full quadrature rule.

Both use the method of snapshots: eigen-decompose the snapshot Gram matrix
S^T M S = V diag(lambda) V^T and take S V lambda^(-1/2) for the leading
eigenvalues, then re-orthonormalise once in the M inner product.
"""
import numpy as np
import scipy.sparse as sp

from .fem import value_operator


def v_gram(problem):
    """M_V = M + K_H1 on the periodic DOFs (parent domain)."""
    mesh = problem.mesh
    Nop = value_operator(mesh, problem.space.node_dof, problem.space.ndof)
    w2 = np.repeat(mesh.qw, 2)
    w4 = np.repeat(mesh.qw, 4)
    M = Nop.T @ sp.diags(w2) @ Nop
    KH = problem.Gop.T @ sp.diags(w4) @ problem.Gop
    return (M + KH).tocsr()


def pod(S, M, n):
    """n leading POD modes of snapshot columns S, orthonormal in <., .>_M.

    M is a sparse/dense matrix or a 1-D array of diagonal weights.
    Returns (modes, eigenvalues of the snapshot Gram matrix, descending).
    """
    def Mv(X):
        if np.ndim(M) == 1:
            return M[:, None] * X
        return M @ X

    C = S.T @ Mv(S)
    C = 0.5 * (C + C.T)
    lam, V = np.linalg.eigh(C)
    order = np.argsort(lam)[::-1]
    lam, V = lam[order], V[:, order]
    if n > np.sum(lam > lam[0] * 1e-13):  # below this the Gram eigenvalues are rounding noise
        raise ValueError("requested more modes than the snapshot rank")
    Phi = S @ (V[:, :n] / np.sqrt(lam[:n]))
    # one re-orthonormalisation pass (Cholesky of the Gram matrix)
    Gm = Phi.T @ Mv(Phi)
    L = np.linalg.cholesky(0.5 * (Gm + Gm.T))
    Phi = np.linalg.solve(L, Phi.T).T
    return Phi, lam

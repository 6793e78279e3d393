"""Auxiliary problem for the geometrical transformation (Sec. 3.4).

Phi_mu(X^p) = X^p + d(X^p), with d solving linear elasticity on the parent
domain (eq. auxiliary_problem), E_aux = 1 and nu_aux = 0.25 as in the paper.
d = 0 on the outer cell boundary and is prescribed on the void boundaries.

The paper does not say whether the auxiliary problem is plane strain or plane
stress (it reports that the choice of auxiliary constants matters little);
plane strain is used here.

Boundary data.  A circular parent void of radius r0 centred at X_c is mapped
to the ellipse of the parameters by d = (S(mu) - I)(X - X_c) on its
boundary, with S symmetric.  d is linear in the entries of S - I, so
d = sum_k c_k(mu) dhat_k exactly, where dhat_k solves the auxiliary problem
for unit boundary data.  This is the reduced auxiliary system
A_hat d_hat = b_hat(mu) of eq. reduced_aux_problem with one unknown per affine
coefficient; the paper's POD + DEIM construction of it is unnecessary when
the boundary data are affine in c(mu).

Parameter maps (kind):
  0  one axis-aligned elliptical void, mu = (a, b) semi-axes:
     S = diag(a, b) / r0, c = (a/r0 - 1, b/r0 - 1).
  1  four voids of equal area A_v, mu = (kappa_1, theta_1, ..., kappa_4,
     theta_4): a = sqrt(A_v / (pi kappa)), b = kappa a (as in the paper's
     second example), S = R(theta) diag(a, b) R(theta)^T / r0,
     c = (S_xx - 1, S_yy - 1, S_xy) per void.
  2  inclusions all scaled about their centres by one factor, mu = (zeta)
     (the paper's first example): S = zeta I for every inclusion, one
     coefficient c = zeta - 1 and one mode, the response to
     d = X - X_c,i on the nodes of every inclusion i at once.  The
     inclusion meshes do not fit the ellipses; the data are prescribed on
     all nodes inside an inclusion, so the map is exactly the scaling there.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import gradient_operator, block_diag4

E_AUX = 1.0
NU_AUX = 0.25


def _plane_strain_D(E, nu):
    """Isotropic elasticity as a 4x4 map on full gradient components.

    sigma = lam tr(eps) I + 2 G eps with eps = sym(grad d); acting on grad d
    the map is D[(ij),(kl)] = lam d_ij d_kl + G (d_ik d_jl + d_il d_jk).
    """
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    G = E / (2 * (1 + nu))
    D = np.zeros((4, 4))
    for i in range(2):
        for j in range(2):
            for k in range(2):
                for l in range(2):
                    D[2 * i + j, 2 * k + l] = (lam * (i == j) * (k == l)
                                               + G * ((i == k) * (j == l) + (i == l) * (j == k)))
    return D


def n_coeff(kind):
    return {0: 2, 1: 12, 2: 1}[kind]


def unit_patterns(kind):
    """Symmetric 2x2 patterns E_k of S - I, and the void each belongs to."""
    if kind == 0:
        return [(np.array([[1.0, 0.0], [0.0, 0.0]]), 0), (np.array([[0.0, 0.0], [0.0, 1.0]]), 0)]
    if kind == 1:
        out = []
        for v in range(4):
            out.append((np.array([[1.0, 0.0], [0.0, 0.0]]), v))
            out.append((np.array([[0.0, 0.0], [0.0, 1.0]]), v))
            out.append((np.array([[0.0, 1.0], [1.0, 0.0]]), v))
        return out
    if kind == 2:
        return [(np.eye(2), -1)]  # every inclusion (void index -1: all of them)
    raise ValueError(kind)


def coefficients(kind, mu, r0, void_area=None):
    """Affine coefficients c(mu) of the boundary data."""
    mu = np.asarray(mu, dtype=np.float64)
    if kind == 0:
        return np.array([mu[0] / r0 - 1.0, mu[1] / r0 - 1.0])
    if kind == 1:
        c = []
        for v in range(4):
            kappa, theta = mu[2 * v], mu[2 * v + 1]
            a = np.sqrt(void_area / (np.pi * kappa))
            b = kappa * a
            R = np.array([[np.cos(theta), -np.sin(theta)], [np.sin(theta), np.cos(theta)]])
            S = R @ np.diag([a, b]) @ R.T / r0
            c += [S[0, 0] - 1.0, S[1, 1] - 1.0, S[0, 1]]
        return np.array(c)
    if kind == 2:
        return np.array([mu[0] - 1.0])
    raise ValueError(kind)


def coefficient_jacobian(kind, mu, r0, void_area=None):
    """d c / d mu, shape (c, n_mu), of coefficients(): kind 0 is linear in
    (a, b); kind 1 per void from S = R(theta) diag(a, b) R(theta)^T / r0 with
    a = sqrt(A_v / (pi kappa)), da/dkappa = -a / (2 kappa), b = kappa a,
    db/dkappa = a / 2."""
    mu = np.asarray(mu, dtype=np.float64)
    if kind == 0:
        return np.eye(2) / r0
    if kind == 1:
        Jc = np.zeros((12, 8))
        for v in range(4):
            kappa, theta = mu[2 * v], mu[2 * v + 1]
            a = np.sqrt(void_area / (np.pi * kappa))
            b = kappa * a
            da, db = -a / (2.0 * kappa), a / 2.0
            cs, sn = np.cos(theta), np.sin(theta)
            # S11 = (a c^2 + b s^2) / r0, S22 = (a s^2 + b c^2) / r0, S12 = (a - b) s c / r0
            Jc[3 * v + 0, 2 * v] = (da * cs * cs + db * sn * sn) / r0
            Jc[3 * v + 1, 2 * v] = (da * sn * sn + db * cs * cs) / r0
            Jc[3 * v + 2, 2 * v] = (da - db) * sn * cs / r0
            Jc[3 * v + 0, 2 * v + 1] = 2.0 * sn * cs * (b - a) / r0
            Jc[3 * v + 1, 2 * v + 1] = 2.0 * sn * cs * (a - b) / r0
            Jc[3 * v + 2, 2 * v + 1] = (a - b) * (cs * cs - sn * sn) / r0
        return Jc
    if kind == 2:
        return np.ones((1, 1))
    raise ValueError(kind)


class AuxiliaryProblem:
    """Linear-elastic transformation problem on a parent mesh."""

    def __init__(self, mesh, kind):
        self.mesh = mesh
        self.kind = kind
        nn = mesh.nn
        node_dof = np.arange(nn)
        self.Gall = gradient_operator(mesh, node_dof, 2 * nn)
        D = _plane_strain_D(E_AUX, NU_AUX)
        Dq = np.broadcast_to(D, (mesh.nq, 4, 4)) * mesh.qw[:, None, None]
        self.K = (self.Gall.T @ block_diag4(np.ascontiguousarray(Dq)) @ self.Gall).tocsr()
        outer = mesh.outer_boundary_nodes()
        inner = np.nonzero(mesh.void_of_node >= 0)[0]
        fixed_nodes = np.union1d(outer, inner)
        self.fixed = np.sort(np.concatenate([2 * fixed_nodes, 2 * fixed_nodes + 1]))
        self.free = np.setdiff1d(np.arange(2 * nn), self.fixed)
        self.inner = inner
        Kff = self.K[self.free][:, self.free].tocsc()
        self._lu = spla.splu(Kff)

    def solve_boundary_data(self, dB):
        """Solve with nodal boundary values dB (nn, 2) on the fixed nodes."""
        d = np.zeros(2 * self.mesh.nn)
        d[self.fixed] = dB.reshape(-1)[self.fixed]
        rhs = -(self.K[self.free][:, self.fixed] @ d[self.fixed])
        d[self.free] = self._lu.solve(rhs)
        return d.reshape(-1, 2)

    def void_data(self, patterns):
        """Nodal boundary data sum over (S_v - I)(X - X_c,v) on each void."""
        mesh = self.mesh
        dB = np.zeros((mesh.nn, 2))
        for Ev, v in patterns:
            for u in (range(len(mesh.voids)) if v < 0 else (v,)):
                nodes = self.inner[mesh.void_of_node[self.inner] == u]
                cx, cy, _ = mesh.voids[u]
                dX = mesh.X[nodes] - np.array([cx, cy])
                dB[nodes] += dX @ Ev.T
        return dB

    def modes(self):
        """dhat_k for every affine coefficient, as nodal fields (c, nn, 2)."""
        return np.stack([self.solve_boundary_data(self.void_data([p]))
                         for p in unit_patterns(self.kind)])

    def gradients(self, fields):
        """Parent gradients of nodal fields at all quadrature points (.., nq, 2, 2)."""
        return np.stack([(self.Gall @ f.reshape(-1)).reshape(-1, 2, 2) for f in fields])


def transformation(grad_modes, c):
    """F_mu = I + sum_k c_k grad dhat_k at the given points: (..., 2, 2)."""
    F = np.einsum('k,kqij->qij', np.asarray(c), grad_modes)
    F[:, 0, 0] += 1.0
    F[:, 1, 1] += 1.0
    return F

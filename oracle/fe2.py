"""Two-scale (FE^2) macro solve driven by the reduced RVE model (Sec. 4.2).

TEST INFRASTRUCTURE ONLY (see the package header): plain numpy, dense
matrices, one RVE solve at a time.

The macro problem is the quasi-static finite-strain balance of the first
Piola-Kirchhoff stress on the reference block, discretised with eight-node
quadrilaterals and 2 x 2 Gauss points (four quadrature points per element,
as in the paper's macro mesh).  At every quadrature point the constitutive
response is the RVE's: Pbar and Abar = dPbar/dFbar of the reduced model
(Sec. 3.3, Algorithm 1 online), with the point's own shape parameters and
committed history.

Readings (the paper describes the example, not the macro solver):
* total Lagrangian, plane strain, the traction a dead load per unit
  reference length acting downward with magnitude T(x);
* at a load step, Newton on the free displacements: every iteration solves
  each RVE from its committed state to the current Fbar (a trial solve),
  assembles f_int and K = sum B^T Abar B, and stops when
  ||f_ext - f_int||_2 (free dofs) <= max(tol_rel ||f_ext||_2, tol_abs);
  the state of that last evaluation is committed;
* a change of the prescribed displacements enters through the tangent of
  the current state: the first iteration of a step evaluates the RVEs at the
  previous displacements and solves K_ff du_f = r_f - K_fd du_d, with du_d
  the change of the prescribed values (the usual lifting; the RVE solves
  then see a predicted Fbar instead of a jump at the boundary); a step has
  converged once the prescribed values are in place and the residual test
  holds;
* the compliance is the work of the load, C = int_top T(x) (-u_y) dx, so it
  is positive under compression (the paper writes T u_y with T signed).

Components are stored in the order [11, 12, 21, 22] = 2 i + J (Pbar, Fbar)
and Abar[2 i + J, 2 k + L] = dP_iJ / dF_kL, as the RVE model returns them.
"""
import numpy as np

# corner nodes counterclockwise from (-1, -1), then the midsides of the
# bottom, right, top and left edges
Q8_NODES = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1], [0, -1], [1, 0], [0, 1], [-1, 0]], dtype=np.float64)
GAUSS_2 = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], dtype=np.float64) / np.sqrt(3.0)


def q8_shape(xi, eta):
    """Serendipity shape functions N (8,) and their derivatives dN/d(xi, eta)
    (8, 2) at one parent point."""
    N = np.zeros(8)
    dN = np.zeros((8, 2))
    for a, (xa, ea) in enumerate(Q8_NODES):
        if xa != 0 and ea != 0:   # corner
            N[a] = 0.25 * (1 + xi * xa) * (1 + eta * ea) * (xi * xa + eta * ea - 1)
            dN[a, 0] = 0.25 * xa * (1 + eta * ea) * (2 * xi * xa + eta * ea)
            dN[a, 1] = 0.25 * ea * (1 + xi * xa) * (xi * xa + 2 * eta * ea)
        elif xa == 0:             # midside of a horizontal edge
            N[a] = 0.5 * (1 - xi * xi) * (1 + eta * ea)
            dN[a, 0] = -xi * (1 + eta * ea)
            dN[a, 1] = 0.5 * ea * (1 - xi * xi)
        else:                     # midside of a vertical edge
            N[a] = 0.5 * (1 + xi * xa) * (1 - eta * eta)
            dN[a, 0] = 0.5 * xa * (1 - eta * eta)
            dN[a, 1] = -eta * (1 + xi * xa)
    return N, dN


def geometry(mesh):
    """Per quadrature point p = 4 e + g: dN/dX (P, 8, 2), weight * det J (P,)
    and position (P, 2)."""
    X, conn = mesh['X'], mesh['conn']
    P = 4 * conn.shape[0]
    dNdX = np.zeros((P, 8, 2))
    wJ = np.zeros(P)
    Xg = np.zeros((P, 2))
    for e, nodes in enumerate(conn):
        Xe = X[nodes]
        for g, (xi, eta) in enumerate(GAUSS_2):
            N, dN = q8_shape(xi, eta)
            Jm = Xe.T @ dN                 # dX_I / dxi_j
            p = 4 * e + g
            dNdX[p] = dN @ np.linalg.inv(Jm)
            wJ[p] = np.linalg.det(Jm)      # Gauss weights are 1
            Xg[p] = N @ Xe
    return dict(dNdX=dNdX, wJ=wJ, Xg=Xg)


def deformation_gradient(mesh, geo, u):
    """Fbar (P, 2, 2) = I + sum_a u_a (x) dN_a/dX at every quadrature point."""
    ue = u.reshape(-1, 2)[np.repeat(mesh['conn'], 4, axis=0)]   # (P, 8, 2)
    return np.eye(2)[None] + np.einsum('pai,paJ->piJ', ue, geo['dNdX'])


def internal_force(mesh, geo, Pbar):
    """f_int (ndof,): f[2 n + i] = sum_p P_iJ dN_a/dX_J w|J| over the points
    whose element holds node n as its node a."""
    f = np.zeros(2 * mesh['X'].shape[0])
    contrib = np.einsum('piJ,paJ,p->pai', Pbar.reshape(-1, 2, 2), geo['dNdX'], geo['wJ'])
    nodes = np.repeat(mesh['conn'], 4, axis=0)
    for i in range(2):
        np.add.at(f, 2 * nodes + i, contrib[:, :, i])
    return f


def stiffness(mesh, geo, Abar):
    """Dense K (ndof, ndof) = sum_p B_p^T Abar_p B_p w|J|."""
    ndof = 2 * mesh['X'].shape[0]
    K = np.zeros((ndof, ndof))
    A = Abar.reshape(-1, 2, 2, 2, 2)
    for p, nodes in enumerate(np.repeat(mesh['conn'], 4, axis=0)):
        ke = np.einsum('aJ,iJkL,bL->aibk', geo['dNdX'][p], A[p], geo['dNdX'][p]) * geo['wJ'][p]
        dofs = (2 * nodes[:, None] + np.arange(2)[None]).reshape(-1)
        K[np.ix_(dofs, dofs)] += ke.reshape(16, 16)
    return K


GAUSS_3 = (np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)]), np.array([5.0, 8.0, 5.0]) / 9.0)


def _edge_shape(s):
    return np.array([0.5 * s * (s - 1), 1 - s * s, 0.5 * s * (s + 1)]), np.array([s - 0.5, -2 * s, s + 0.5])


def traction_profile(x, Tbar, width):
    """T(x) = Tbar (1 - (2 x / W - 1)^2)."""
    return Tbar * (1.0 - (2.0 * x / width - 1.0) ** 2)


def external_force(mesh, Tbar):
    """Consistent nodal forces of the downward traction T(x) on the top edge
    (three-point Gauss rule per quadratic edge, exact for this load)."""
    f = np.zeros(2 * mesh['X'].shape[0])
    for edge in mesh['top']:
        x = mesh['X'][edge, 0]
        for s, w in zip(*GAUSS_3):
            N, dN = _edge_shape(s)
            t = traction_profile(N @ x, Tbar, mesh['width'])
            f[2 * edge + 1] -= N * t * abs(dN @ x) * w
    return f


def compliance(mesh, Tbar, u):
    """C = int_top T(x) (-u_y(x)) dx by the same edge rule."""
    uy = u.reshape(-1, 2)[:, 1]
    C = 0.0
    for edge in mesh['top']:
        x = mesh['X'][edge, 0]
        for s, w in zip(*GAUSS_3):
            N, dN = _edge_shape(s)
            C -= traction_profile(N @ x, Tbar, mesh['width']) * (N @ uy[edge]) * abs(dN @ x) * w
    return C


def run(rom, mesh, mu, Tbars, fixed_dofs=None, fixed_values=None, tol_rel=1e-9, tol_abs=1e-12, max_macro=20,
        rve_tol=1e-10, rve_max_iter=25):
    """Load steps with peak traction Tbars[k] (and, if given, prescribed
    values fixed_values[k] on fixed_dofs; default: the bottom edge held at
    zero).  Returns a list of per-step dicts (u, C, macro iterations, RVE
    evaluations, status 0 / 1 macro cap / 2 an RVE solve failed)."""
    ndof = 2 * mesh['X'].shape[0]
    if fixed_dofs is None:
        fixed_dofs = np.sort(np.concatenate([2 * mesh['bottom'], 2 * mesh['bottom'] + 1]))
    fixed_dofs = np.asarray(fixed_dofs)
    free = np.setdiff1d(np.arange(ndof), fixed_dofs)
    geo = geometry(mesh)
    P = geo['wJ'].size
    trans = [rom.transformation(mu[p]) for p in range(P)]
    r_c = [np.zeros(rom.n) for _ in range(P)]
    h_c = [rom.virgin() for _ in range(P)]
    u = np.zeros(ndof)
    out = []
    for k, Tbar in enumerate(Tbars):
        fext = external_force(mesh, Tbar)
        target = np.zeros(fixed_dofs.size) if fixed_values is None else np.asarray(fixed_values[k], dtype=np.float64)
        status, evals, steps = 1, 0, None
        for it in range(max_macro):
            F = deformation_gradient(mesh, geo, u)
            if hasattr(rom, 'step_all'):  # RVE models that solve the points side by side
                steps = rom.step_all([(r_c[p], h_c[p], F[p], trans[p]) for p in range(P)], rve_tol, rve_max_iter)
            else:
                steps = [rom.step(r_c[p], h_c[p], F[p], *trans[p], tol=rve_tol, max_iter=rve_max_iter)
                         for p in range(P)]
            evals += sum(s['iters'] for s in steps)
            if any(s['status'] != 0 for s in steps):
                status = 2
                break
            Pbar = np.array([s['Pbar'] for s in steps])
            res = fext - internal_force(mesh, geo, Pbar)
            dud = target - u[fixed_dofs]
            if not dud.any() and np.linalg.norm(res[free]) <= max(tol_rel * np.linalg.norm(fext[free]), tol_abs):
                status = 0
                break
            Abar = np.array([s['Abar'] for s in steps])
            K = stiffness(mesh, geo, Abar)
            rhs = res[free] - K[np.ix_(free, fixed_dofs)] @ dud
            u[free] += np.linalg.solve(K[np.ix_(free, free)], rhs)
            u[fixed_dofs] = target
        if status == 0:
            r_c = [s['r'] for s in steps]
            h_c = [s['hist'] for s in steps]
        out.append(dict(u=u.copy(), C=compliance(mesh, Tbar, u), macro_iters=it + 1, rve_evals=evals,
                        status=status, Pbar=np.array([s['Pbar'] for s in steps])))
        if status != 0:
            break
    return out


_FOM = {}


def damped_newton(problem, w0, Fbar, hist, tol, max_iter=200):
    """Newton with backtracking on ||f||: the step -K^-1 f is halved until the
    residual norm drops (at most 30 halvings).  The same equations as plain
    Newton, reached from starts where the full step overshoots; used for the
    reference solution only when plain Newton fails."""
    from . import fom, material
    w = w0.copy()
    ev = problem.evaluate(w, Fbar, hist, material.j2_point)
    res = np.linalg.norm(ev['f'])
    for it in range(max_iter):
        if not np.isfinite(res):
            return None
        if res <= tol:
            return w, ev, it + 1
        d = fom._solve(ev['K'], ev['f'])
        a = 1.0
        for _ in range(30):
            wn = w - a * d
            evn = problem.evaluate(wn, Fbar, hist, material.j2_point)
            rn = np.linalg.norm(evn['f'])
            if np.isfinite(rn) and rn < res:
                break
            a *= 0.5
        else:
            return None
        w, ev, res = wn, evn, rn
    return None


def _fom_step(args):
    r0, hist, Fbar, mu, tol, max_iter = args
    return _FOM['rve'].step(r0, hist, Fbar, mu, tol=tol, max_iter=max_iter)


class FomRve:
    """The full-order RVE (Sec. 2: the periodic fluctuation on the mapped
    parent cell, Newton on the full system, eq. full_newton; effective stress
    and stiffness of eqs. eff_stress_full and eff_stiffness_full) with the
    interface run() uses for the reduced model, so the same macro loop gives
    the reference two-scale solution of the compliance error (Sec. 4.2).
    `spec` is the offline stage's description of the cell (its mesh,
    transformation modes and materials); the 'coordinates' are the
    fluctuation dofs.  With `workers` > 1 the points of a macro iteration are
    solved in a process pool."""

    def __init__(self, spec, workers=1):
        from . import build_rom
        self._br = build_rom
        self.spec = dict(spec)
        self.mesh, self.space, self.grad_modes = build_rom._geometry(self.spec)
        self.mat = build_rom.material(self.spec, self.mesh)
        self.n = self.space.ndof
        self.workers = workers
        self._pool = None

    def close(self):
        if self._pool is not None:
            self._pool.close()
            self._pool = None

    def transformation(self, mu):
        return (np.asarray(mu, dtype=np.float64),)

    def _problem(self, mu):
        from . import auxiliary, fem
        Fmu = auxiliary.transformation(self.grad_modes, self._br._mu_coeff(self.spec, mu))
        return fem.Problem(self.mesh, self.space, Fmu, self.mat)

    def virgin(self):
        from . import material
        return material.virgin_history((self.mesh.nq,))

    def step(self, r0, hist, Fbar, mu, tol=1e-10, max_iter=25):
        from . import fom
        pr = self._problem(mu)
        Fbar = np.asarray(Fbar, dtype=np.float64)
        sol = fom.newton(pr, r0, Fbar, hist, tol, max_iter)
        if sol is None:
            sol = damped_newton(pr, r0, Fbar, hist, tol)
        if sol is None:
            nan = np.full((2, 2), np.nan)
            return dict(r=r0, hist=hist, status=1, iters=max_iter, Pbar=nan, Abar=np.full((2, 2, 2, 2), np.nan))
        w, ev, its = sol
        return dict(r=w, hist=ev['hist'], status=0, iters=its, Pbar=pr.effective_stress(ev),
                    Abar=pr.effective_stiffness(ev, fom._solve))

    def step_all(self, jobs, tol, max_iter):
        args = [(r, h, F, t[0], tol, max_iter) for r, h, F, t in jobs]
        if self.workers <= 1:
            return [self.step(*a[:4], tol=tol, max_iter=max_iter) for a in args]
        if self._pool is None:
            import multiprocessing as mp
            _FOM['rve'] = self
            self._pool = mp.get_context('fork').Pool(self.workers)
        return self._pool.map(_fom_step, args, chunksize=1)

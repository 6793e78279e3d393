"""Hyper-reduced online solve (Sec. 3.2-3.3, Algorithm 1 online).

For one macro point with shape parameters mu and committed history:

1. c(mu) and, at every ECM point q, F_mu = I + sum_k c_k grad dhat_k,
   F_mu^-1 and det F_mu (eq. reduced_aux_problem and the text after it);
2. Newton on the reduced coordinates r (the paper's a), eq. red_newton, with
   the hyper-reduced force and stiffness of eqs. forcevector_ecm and
   stiffnessmatrix_ecm:
       f_i  = sum_q w_q (grad phi_i F_mu^-1) : P(F_q) |det F_mu|
       K_ij = sum_q w_q (grad phi_i F_mu^-1) : A(F_q) : (grad phi_j F_mu^-1) |det F_mu|
   with F_q = Fbar + (sum_n r_n grad phi_n) F_mu^-1;
3. effective stress by the ECM rule, eq. eff_stress_1;
4. the four tangent problems K* q = b, eq. tangent_problem_red, and the
   effective stiffness, eqs. eff_stiffness_1 and eff_stress_f11.

Readings taken (the paper is silent): the initial guess is the previous
converged r; no line search; convergence when ||f||_2 <= tol (absolute).
One Newton iteration is one evaluation of (f, K); the loop stops at the
first evaluation that satisfies the tolerance, so the returned state, stress
and K* belong to the returned r.  In fixed-iteration mode exactly max_iter
evaluations are made (updating r after all but the last) and the status is
decided by the last one; this mode exists so that two implementations can be
compared along the same Newton map.

Status codes: 0 converged, 1 iteration cap, 2 non-finite residual.

Load-step cutting (the appendix on the material model notes that the global
Newton solver sometimes needs much smaller load steps): with a depth D >= 1 a
step that fails is retried towards intermediate targets on the straight line
from the committed Fbar_c to the requested Fbar,
    Fbar(t) = Fbar_c + (t / 2^D) (Fbar - Fbar_c),  t = 1 .. 2^D,
halving the attempted stride on every failure and doubling it (within the
remaining distance) after every converged sub-step, whose state then becomes
the start of the next attempt.  The step fails when a stride of 1 / 2^D does
not converge; D = 0 is the plain method.
"""
import numpy as np

from . import artifact, auxiliary, material
from .fem import right_map


class ROM:
    def __init__(self, path=None, data=None):
        d = artifact.read(path) if data is None else data
        self.__dict__.update(d)
        # material per ECM point (a second phase where phase == 1)
        phase = np.asarray(d.get('phase', np.zeros(self.m, dtype=np.int64)))
        if d.get('mat2') is not None and np.any(phase == 1):
            self.mat_q = tuple(np.where(phase == 1, b, a) for a, b in zip(self.mat, d['mat2']))
        else:
            self.mat_q = self.mat

    # -- step 1 -------------------------------------------------------------
    def transformation(self, mu):
        c = auxiliary.coefficients(self.kind, mu, self.r0, self.void_area)
        Fmu = np.einsum('k,qak->qa', c, self.Gd).reshape(self.m, 2, 2)
        Fmu[:, 0, 0] += 1.0
        Fmu[:, 1, 1] += 1.0
        J = np.linalg.det(Fmu)
        return np.linalg.inv(Fmu), J

    # -- step 2 -------------------------------------------------------------
    def evaluate(self, r, Fbar, hist, Finv, J):
        H = (self.G @ r).reshape(self.m, 2, 2)  # sum_n r_n grad phi_n at the points
        F = Fbar[None] + H @ Finv
        P, A, Fp, Fp33, xi, gam = material.j2_point(F, *hist, self.mat_q)
        wJ = self.w * np.abs(J)
        T = right_map(Finv)  # vec(Hp F_mu^-1) = T vec(Hp)
        B = T @ self.G  # mapped mode gradients (m, 4, n)
        f = np.einsum('qai,qa->i', B, P.reshape(self.m, 4) * wJ[:, None])
        A4 = A.reshape(self.m, 4, 4)
        K = np.einsum('qai,qab,qbj->ij', B, A4 * wJ[:, None, None], B)
        return dict(f=f, K=K, P=P, A=A4, B=B, wJ=wJ, hist=(Fp, Fp33, xi), gamma=gam)

    def newton(self, r0, hist, Fbar, Finv, J, tol=1e-8, max_iter=25, fixed=False):
        r = np.array(r0, dtype=np.float64)
        status = 1
        for it in range(max_iter):
            ev = self.evaluate(r, Fbar, hist, Finv, J)
            res = np.linalg.norm(ev['f'])
            if not np.isfinite(res):
                return r, ev, 2, it + 1, res
            last = it == max_iter - 1
            if fixed:
                if last:
                    status = 0 if res <= tol else 1
                    return r, ev, status, it + 1, res
            elif res <= tol:
                return r, ev, 0, it + 1, res
            elif last:
                return r, ev, 1, it + 1, res
            r = r - np.linalg.solve(ev['K'], ev['f'])
        raise AssertionError("unreachable")

    # -- steps 3, 4 ---------------------------------------------------------
    def effective(self, ev):
        wJ, A4, B = ev['wJ'], ev['A'], ev['B']
        Pbar = np.einsum('q,qa->a', wJ, ev['P'].reshape(self.m, 4)) / self.cell_area
        Abar = np.zeros((4, 4))
        for kl in range(4):
            E = np.zeros(4)
            E[kl] = 1.0
            # right-hand side b_i = -(sum_q w_q (grad phi_i F^-1) : A |J|) : E_kl
            b = -np.einsum('qai,qab,b->i', B, A4 * wJ[:, None, None], E)
            q = np.linalg.solve(ev['K'], b)
            dF = E[None, :] + B @ q  # E_kl + grad q_kl F^-1 at each point
            Abar[:, kl] = np.einsum('q,qab,qb->a', wJ, A4, dF) / self.cell_area
        return Pbar, Abar

    # -- shape sensitivities -----------------------------------------------
    def shape_sensitivity(self, mu, r, Fbar, hist):
        """dPbar / dmu at the state r of load Fbar reached from the committed
        history hist, which is held fixed: eq. eff_sensitivities_full with the
        ECM rule, where d/dmu (dw/dX) = sum_i (dr_i/dmu) grad phi_i and dr/dmu
        follows from the reduced equilibrium, K dr/dmu = -df/dmu at fixed r
        (f of eq. forcevector_ecm, K of eq. stiffnessmatrix_ecm).  Returns
        (4, n_mu): component (i J) of Pbar by shape parameter."""
        Finv, J = self.transformation(mu)
        ev = self.evaluate(r, Fbar, hist, Finv, J)
        m, n = self.m, self.n
        dc = auxiliary.coefficient_jacobian(self.kind, mu, self.r0, self.void_area)  # (c, n_mu)
        n_mu = dc.shape[1]
        dFmu = np.einsum('qak,kj->jqa', self.Gd, dc).reshape(n_mu, m, 2, 2)  # dF_mu / dmu_j
        dFinv = -Finv[None] @ dFmu @ Finv[None]                              # d(F_mu^-1) / dmu_j
        dJ = J[None] * np.einsum('qab,jqba->jq', Finv, dFmu)                 # d det F_mu / dmu_j
        dwJ = self.w[None] * np.sign(J)[None] * dJ                           # d(w |det F_mu|) / dmu_j
        wJ, P4, A4, B = ev['wJ'], ev['P'].reshape(m, 4), ev['A'], ev['B']
        H = (self.G @ r).reshape(m, 2, 2)
        dFr = (H[None] @ dFinv).reshape(n_mu, m, 4)                          # dF / dmu_j at fixed r
        out = np.zeros((4, n_mu))
        for j in range(n_mu):
            Bd = right_map(dFinv[j]) @ self.G                                 # vec(grad phi_i dF_mu^-1/dmu_j)
            AdF = np.einsum('qab,qb->qa', A4, dFr[j])
            df = (np.einsum('qai,qa->i', B, P4 * dwJ[j][:, None]) + np.einsum('qai,qa->i', Bd, P4 * wJ[:, None])
                  + np.einsum('qai,qa->i', B, AdF * wJ[:, None]))
            dr = -np.linalg.solve(ev['K'], df)
            dF = B @ dr + dFr[j]                                              # total dF / dmu_j
            out[:, j] = (np.einsum('q,qab,qb->a', wJ, A4, dF) + np.einsum('q,qa->a', dwJ[j], P4)) / self.cell_area
        return out

    def step(self, r0, hist, Fbar, Finv, J, tol=1e-8, max_iter=25, fixed=False):
        r, ev, status, iters, res = self.newton(r0, hist, Fbar, Finv, J, tol, max_iter, fixed)
        Pbar, Abar = self.effective(ev)
        return dict(r=r, hist=ev['hist'], status=status, iters=iters, resnorm=res,
                    Pbar=Pbar, Abar=Abar)

    def cut_step(self, r_c, hist_c, Fbar_c, Fbar, Finv, J, tol=1e-8, max_iter=25, fixed=False, max_substeps=0):
        """One load step with cutting (see the module notes).  Returns the last
        attempt's step dict with 'iters' summed over all attempts, plus the
        start state of that attempt ('r_c', 'hist_c', 'Fbar_c': the committed
        state after the converged sub-steps), the converged intermediate
        targets in order ('targets') and the end points t / 2^D of every
        converged sub-step, the last one included ('ends', as integers t)."""
        full = 2 ** max_substeps
        t, dt = 0, full
        r0, h0, F0 = r_c, hist_c, np.asarray(Fbar_c, dtype=np.float64)
        Fbar = np.asarray(Fbar, dtype=np.float64)
        total, targets, ends = 0, [], []
        while True:
            target = Fbar if t + dt == full else Fbar_c + ((t + dt) / full) * (Fbar - Fbar_c)
            s = self.step(r0, h0, target, Finv, J, tol, max_iter, fixed)
            total += s['iters']
            if s['status'] == 0:
                t += dt
                ends.append(t)
                if t == full:
                    break
                r0, h0, F0 = s['r'], s['hist'], target
                targets.append(target)
                dt = min(2 * dt, full - t)
            else:
                if dt == 1:
                    break
                dt //= 2
        s.update(iters=total, r_c=r0, hist_c=h0, Fbar_c=F0, targets=targets, ends=ends)
        return s

    def virgin(self):
        return material.virgin_history((self.m,))

    def run_path(self, mu, Fbar_path, tol=1e-8, max_iter=25, fixed=False, commit=True, max_substeps=0):
        """Solve a whole load path from the virgin state; commit converged steps
        (with cutting: also the converged sub-steps of a failed step)."""
        Finv, J = self.transformation(mu)
        if np.any(J <= 0):
            raise ValueError("invalid shape parameters: det F_mu <= 0")
        hist = self.virgin()
        r = np.zeros(self.n)
        Fc = np.eye(2)
        out = []
        for Fb in Fbar_path:
            Fb = np.asarray(Fb, dtype=np.float64)
            if max_substeps == 0:
                s = self.step(r, hist, Fb, Finv, J, tol, max_iter, fixed)
            else:
                s = self.cut_step(r, hist, Fc, Fb, Finv, J, tol, max_iter, fixed, max_substeps)
            out.append(s)
            if commit and s['status'] == 0:
                hist, r, Fc = s['hist'], s['r'], Fb
            elif commit and max_substeps > 0:
                hist, r, Fc = s['hist_c'], s['r_c'], s['Fbar_c']
        return out

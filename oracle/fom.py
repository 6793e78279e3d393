"""Full-order RVE solve on the parent domain (Sec. 2, Algorithm 1 offline).

Newton's method (eq. full_newton) on the periodic fluctuation DOFs until
||f||_2 <= eps_newton, with the load applied in steps.  When Newton fails to
converge within the iteration cap the step is halved (the appendix notes that
very small load steps are sometimes needed); history is only committed for
converged steps.
"""
import numpy as np
import scipy.sparse.linalg as spla

from . import material


def _solve(K, B):
    # sparse LU; K is structurally symmetric, so order on the pattern of K^T + K
    lu = spla.splu(K.tocsc(), permc_spec='MMD_AT_PLUS_A')
    return lu.solve(np.asarray(B))


class FOMResult:
    def __init__(self):
        self.w = []
        self.Pbar = []
        self.Abar = []
        self.W = []
        self.iters = []
        self.Fbar = []


def newton(problem, w0, Fbar, hist, tol, max_iter=20, material_point=material.j2_point):
    """Newton iterations at fixed committed history.  Returns (w, ev, iters),
    or None when the iteration fails: non-finite residual, the iteration cap,
    or divergence (three residual increases in a row, or growth by 1e4 over
    the first residual), after which the caller sub-steps."""
    w = w0.copy()
    res0 = None
    prev = np.inf
    rises = 0
    for it in range(max_iter):
        ev = problem.evaluate(w, Fbar, hist, material_point)
        res = np.linalg.norm(ev['f'])
        if not np.isfinite(res):
            return None
        if res <= tol:
            return w, ev, it + 1
        res0 = res if res0 is None else res0
        rises = rises + 1 if res > prev else 0
        if rises >= 3 or res > 1e4 * res0:
            return None
        prev = res
        w = w - _solve(ev['K'], ev['f'])
    return None


def solve_path(problem, Fbar_path, tol=1e-10, max_iter=20, want_tangent=False,
               want_W=True, max_halvings=8):
    """Follow a macroscopic deformation-gradient path from the undeformed state.

    Fbar_path : (K, 2, 2) targets of the load steps.
    Returns FOMResult with per-step w, Pbar (and Abar, W when asked).
    """
    nq = problem.mesh.nq
    hist = material.virgin_history((nq,))
    w = np.zeros(problem.space.ndof)
    out = FOMResult()
    Fprev = np.eye(2)
    for Ft in Fbar_path:
        Ft = np.asarray(Ft, dtype=np.float64)
        # sub-stepping between Fprev and Ft
        s, ds = 0.0, 1.0
        halvings = 0
        while s < 1.0 - 1e-14:
            ds = min(ds, 1.0 - s)
            Fb = Fprev + (s + ds) * (Ft - Fprev)
            sol = newton(problem, w, Fb, hist, tol, max_iter)
            if sol is None:
                halvings += 1
                if halvings > max_halvings:
                    raise RuntimeError("FOM Newton failed after sub-stepping")
                ds *= 0.5
                continue
            w, ev, its = sol
            hist = ev['hist']
            s += ds
        Fprev = Ft
        out.w.append(w.copy())
        out.Fbar.append(Ft.copy())
        out.iters.append(its)
        out.Pbar.append(problem.effective_stress(ev))
        if want_tangent:
            out.Abar.append(problem.effective_stiffness(ev, _solve))
        if want_W:
            out.W.append(ev['W'].reshape(-1).copy())
    out.hist = hist  # committed history after the last step
    return out

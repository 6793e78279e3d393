"""Empirical cubature (Sec. 3.2, eqs. integralsbasis and integral_ecm).

The integrands are the N L functions grad_p phi_i : B_l sampled at the full
rule's points; their exact integrals are b = sum_q w_hat_q (...)|_q.  A subset
of points with positive weights (the paper stresses positivity) is chosen
greedily until the integrals are matched to a relative tolerance eps or a
target number of points is reached.

The greedy follows the published empirical cubature method (Hernandez et al.
2017), which the paper defers to and which is not reproduced there:

1. express the integrands through an orthonormal basis: with
   Jw = J diag(sqrt(w_hat)) = U Sigma V^T (rank r), the rows of
   Z = V^T diag(1 / sqrt(w_hat)) are discretely L^2-orthonormal functions
   spanning the integrands; their integrals are b = Z w_hat;
2. start from an empty set and residual res = b;
3. add the point q maximising the positive normalised correlation
   Z_q . res / ||Z_q|| (ties go to the lowest index);
4. weights on the selected set by non-negative least squares
   (Lawson-Hanson); points whose weight is zero leave the set;
5. res = b - Z_S w_S; stop when ||res|| <= eps ||b|| or |S| reaches the
   target.

Option (not in the paper): a constant integrand can be appended, so that the
rule also integrates the parent area; the paper notes the effective stress
is integrated with the same rule and may lose accuracy otherwise.
"""
import numpy as np
from scipy.optimize import nnls


def integrand_matrix(Gfull, B, n, L):
    """J[(i, l), q] = grad_p phi_i(X_q) : B_l(X_q).

    Gfull : (nq, 4, n) parent mode gradients at all points.
    B     : (nq, 4, L) weighted-stress modes at all points.
    """
    return np.einsum('qai,qal->ilq', Gfull, B).reshape(n * L, -1)


def greedy(J, w_hat, eps, m_max, svd_tol=1e-12):
    """Select points and positive weights.  Returns (idx, weights, history)."""
    sq = np.sqrt(w_hat)
    U, s, Vt = np.linalg.svd(J * sq[None, :], full_matrices=False)
    r = int(np.sum(s > svd_tol * s[0]))
    Z = Vt[:r] / sq[None, :]
    b = Z @ w_hat
    bn = np.linalg.norm(b)
    colnorm = np.linalg.norm(Z, axis=0)
    sel = []
    w = np.zeros(0)
    res = b.copy()
    hist = [1.0]
    n_iter = 0
    while np.linalg.norm(res) > eps * bn and len(sel) < m_max and n_iter < 10 * m_max:
        n_iter += 1
        score = (Z.T @ res) / colnorm
        if sel:
            score[np.array(sel)] = -np.inf
        q = int(np.argmax(score))  # argmax returns the first (lowest) index on ties
        if score[q] <= 0:
            break
        sel.append(q)
        # least squares on the selected set; Lawson-Hanson NNLS only when a
        # weight comes out non-positive (both give the same positive solution
        # when the unconstrained one is positive)
        w = np.linalg.lstsq(Z[:, sel], b, rcond=None)[0]
        if np.any(w <= 0):
            w, _ = nnls(Z[:, sel], b, maxiter=50 * len(sel) + 100)
        keep = w > 0
        sel = [s_ for s_, k in zip(sel, keep) if k]
        w = w[keep]
        res = b - Z[:, sel] @ w
        hist.append(np.linalg.norm(res) / bn)
    return np.array(sel, dtype=np.int64), w, np.array(hist)

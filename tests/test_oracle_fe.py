"""Pins of the oracle's discretisation, transformation and full-order solve
(Sec. 2, Sec. 3.4) against exact integrals, patch tests, superposition and
closed-form homogeneous solutions."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import auxiliary as aux
from oracle import fem, fom, material
from oracle import mesh as M

MAT = (1.0, 0.3, 0.01, 0.05)


def test_quadrature_integrates_quadratics_exactly():
    m = M.mesh_square(3)
    x, y = m.qX[:, 0], m.qX[:, 1]
    w = m.qw
    exact = {'1': 1.0, 'x': 0.5, 'y': 0.5, 'xy': 0.25, 'xx': 1 / 3, 'yy': 1 / 3}
    got = {'1': w.sum(), 'x': w @ x, 'y': w @ y, 'xy': w @ (x * y), 'xx': w @ (x * x), 'yy': w @ (y * y)}
    for k in exact:
        assert abs(got[k] - exact[k]) < 1e-14, k


def test_void_mesh_area_and_periodic_pairs():
    r0 = 0.25
    m = M.one_void_cell(r0, 8, 5)
    assert abs(m.qw.sum() - (1 - np.pi * r0 ** 2)) < 1e-5  # quadratic edges on the circle
    X = m.X
    for side in (0, 1):
        lo = np.sort(X[np.abs(X[:, side]) < 1e-12][:, 1 - side])
        hi = np.sort(X[np.abs(X[:, side] - 1) < 1e-12][:, 1 - side])
        assert lo.shape == hi.shape and np.abs(lo - hi).max() < 1e-12
    void_nodes = X[m.void_of_node == 0]
    assert np.abs(np.linalg.norm(void_nodes - 0.5, axis=1) - r0).max() < 1e-12
    sp = fem.PeriodicSpace(m)
    # every node maps to a master with coordinates equal modulo 1
    d = np.mod(X - X[sp.master] + 0.5, 1.0) - 0.5
    assert np.abs(d).max() < 1e-12


def test_four_void_mesh():
    m = M.four_void_cell(0.15, 4, 3)
    assert abs(m.qw.sum() - (1 - 4 * np.pi * 0.15 ** 2)) < 1e-4
    assert set(np.unique(m.void_of_node)) == {-1, 0, 1, 2, 3}


@pytest.fixture(scope='module')
def small_void():
    m = M.one_void_cell(0.25, 6, 4)
    return m, fem.PeriodicSpace(m), aux.AuxiliaryProblem(m, 0)


def test_auxiliary_patch_test(small_void):
    """An affine field imposed on every Dirichlet node is reproduced exactly."""
    m, _, ax = small_void
    A = np.array([[0.03, -0.02], [0.05, 0.01]])
    d = ax.solve_boundary_data(m.X @ A.T)
    grad = (ax.Gall @ d.reshape(-1)).reshape(-1, 2, 2)
    assert np.abs(grad - A).max() < 1e-12


def test_auxiliary_superposition_and_parent(small_void):
    m, _, ax = small_void
    modes = ax.modes()
    mu = np.array([0.31, 0.19])
    c = aux.coefficients(0, mu, 0.25)
    direct = ax.solve_boundary_data(ax.void_data([(np.diag(c), 0)]))
    assert np.abs(np.tensordot(c, modes, 1) - direct).max() < 1e-12
    # the void boundary is mapped onto the ellipse with semi-axes mu
    vb = m.void_of_node == 0
    Y = m.X[vb] + direct[vb] - 0.5
    assert np.abs((Y[:, 0] / mu[0]) ** 2 + (Y[:, 1] / mu[1]) ** 2 - 1).max() < 1e-12
    gm = ax.gradients(modes)
    Fmu = aux.transformation(gm, aux.coefficients(0, [0.25, 0.25], 0.25))
    assert np.abs(Fmu - np.eye(2)).max() == 0.0
    for corner in ([0.15, 0.15], [0.35, 0.35], [0.15, 0.35], [0.35, 0.15]):
        J = np.linalg.det(aux.transformation(gm, aux.coefficients(0, corner, 0.25)))
        assert J.min() > 0


def test_four_void_coefficients():
    mu = np.array([1.2, 0.3, 1.0, 0.0, 1.5, 1.0, 1.3, 2.5])
    A = 0.075
    r0 = np.sqrt(A / np.pi)
    c = aux.coefficients(1, mu, r0, A)
    for v in range(4):
        S = np.array([[1 + c[3 * v], c[3 * v + 2]], [c[3 * v + 2], 1 + c[3 * v + 1]]])
        kappa = mu[2 * v]
        ev = np.sort(np.linalg.eigvalsh(S)) * r0
        a = np.sqrt(A / (np.pi * kappa))
        assert np.allclose(ev, np.sort([a, kappa * a]), rtol=1e-14)
        assert abs(np.pi * ev[0] * ev[1] - A) < 1e-14  # void area is preserved


def _problem(m, space, mu=None, kind=0):
    ax = aux.AuxiliaryProblem(m, kind) if m.voids else None
    if ax is None:
        Fmu = np.tile(np.eye(2), (m.nq, 1, 1))
    else:
        Fmu = aux.transformation(ax.gradients(ax.modes()), aux.coefficients(kind, mu, 0.25))
    return fem.Problem(m, space, Fmu, MAT)


def test_homogeneous_rve_matches_material_point():
    m = M.mesh_square(3)
    sp = fem.PeriodicSpace(m)
    pr = _problem(m, sp)
    path = [np.eye(2) + k / 5 * np.array([[0.04, 0.015], [-0.01, -0.03]]) for k in range(1, 6)]
    res = fom.solve_path(pr, path, want_tangent=True)
    Fp, Fp33, xi = material.virgin_history(())
    for k, Fb in enumerate(path):
        P, A, Fp, Fp33, xi, g = material.j2_point(Fb, Fp, Fp33, xi, MAT)
        assert np.abs(res.w[k]).max() < 1e-12
        assert np.abs(res.Pbar[k] - P).max() < 1e-13
        assert np.abs(res.Abar[k] - A).max() < 1e-11
    assert xi > 0


def test_zero_load_gives_zero_stress(small_void):
    m, sp, _ = small_void
    pr = _problem(m, sp, [0.3, 0.2])
    res = fom.solve_path(pr, [np.eye(2)])
    assert np.abs(res.Pbar[0]).max() == 0.0 and np.abs(res.w[0]).max() == 0.0


def test_stiffness_is_derivative_of_residual(small_void):
    m, sp, _ = small_void
    pr = _problem(m, sp, [0.3, 0.2])
    rng = np.random.default_rng(0)
    w = 0.01 * rng.normal(size=sp.ndof)
    Fb = np.array([[1.03, 0.01], [0.0, 0.98]])
    hist = material.virgin_history((m.nq,))
    ev = pr.evaluate(w, Fb, hist, material.j2_point)
    v = rng.normal(size=sp.ndof)
    h = 1e-7
    fp = pr.evaluate(w + h * v, Fb, hist, material.j2_point)['f']
    fm = pr.evaluate(w - h * v, Fb, hist, material.j2_point)['f']
    assert np.abs((fp - fm) / (2 * h) - ev['K'] @ v).max() < 1e-6 * np.abs(ev['K'] @ v).max()
    K = ev['K'].toarray()
    assert np.abs(K - K.T).max() < 1e-12 * np.abs(K).max()


def test_effective_stiffness_is_derivative_of_effective_stress(small_void):
    m, sp, _ = small_void
    pr = _problem(m, sp, [0.28, 0.22])
    F1 = np.array([[1.02, 0.01], [0.005, 0.985]])
    F2 = F1 + 0.2 * np.array([[0.015, 0.005], [0.005, -0.01]])  # a step Newton takes without sub-stepping
    res = fom.solve_path(pr, [F1], tol=1e-12)
    # committed state after step 1, then step 2 and its finite differences
    w1, hist = res.w[0], res.hist
    w2, ev2, _ = fom.newton(pr, w1, F2, hist, 1e-13)
    Abar = pr.effective_stiffness(ev2, fom._solve)
    h = 1e-6
    Afd = np.zeros((2, 2, 2, 2))
    for k in range(2):
        for l in range(2):
            d = np.zeros((2, 2))
            d[k, l] = h
            Pp = pr.effective_stress(fom.newton(pr, w1, F2 + d, hist, 1e-13)[1])
            Pm = pr.effective_stress(fom.newton(pr, w1, F2 - d, hist, 1e-13)[1])
            Afd[..., k, l] = (Pp - Pm) / (2 * h)
    assert np.abs(Abar - Afd).max() < 1e-6 * np.abs(Afd).max()

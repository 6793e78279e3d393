"""Pins of the oracle's material point (Appendix A) against what the
mathematics fixes independently of the oracle's own code paths."""
import numpy as np
import pytest

from oracle import material as M

MAT = (1.0, 0.3, 0.01, 0.05)
MAT_EX1 = (10.0, 0.3, 0.2, 5.0)  # matrix material of the paper's first example


def spectral(C, f):
    w, V = np.linalg.eigh(C)
    return (V * f(w)[..., None, :]) @ np.swapaxes(V, -1, -2)


def random_spd(rng, n, spread=1.0):
    A = rng.normal(size=(n, 2, 2)) * spread
    return A @ np.swapaxes(A, -1, -2) + 0.3 * np.eye(2)


def test_logm_expm_match_spectral_definition():
    rng = np.random.default_rng(0)
    C = random_spd(rng, 200)
    # near-isotropic and exactly isotropic cases (coincident eigenvalues)
    C[:10] = 1.3 * np.eye(2) + 1e-9 * random_spd(rng, 10)
    C[10:15] = 0.7 * np.eye(2)
    L = M.logm_sym2(C)
    assert np.abs(L - spectral(C, np.log)).max() < 5e-15 * np.abs(L).max() + 1e-15
    S = 0.5 * (C - np.eye(2))
    assert np.abs(M.expm_sym2(S) - spectral(S, np.exp)).max() < 1e-14 * np.abs(spectral(S, np.exp)).max()


def test_identity_gives_zero_stress():
    Fp, Fp33, xi = M.virgin_history((3,))
    P, A, Fpn, Fp33n, xin, g = M.j2_point(np.tile(np.eye(2), (3, 1, 1)), Fp, Fp33, xi, MAT)
    assert np.abs(P).max() == 0.0
    assert np.all(g == 0) and np.all(xin == 0)
    # tangent at the origin: plane-strain isotropic elasticity on sym(dF) plus
    # the geometric term (-P dF^T F^-T vanishes at P = 0)
    lam, G = M.lame(*MAT[:2])
    D = np.zeros((2, 2, 2, 2))
    for i, j, k, l in np.ndindex(2, 2, 2, 2):
        D[i, j, k, l] = lam * (i == j) * (k == l) + G * ((i == k) * (j == l) + (i == l) * (j == k))
    assert np.abs(A[0] - D).max() < 1e-14


def principal_path(lams, mat):
    """Coaxial path F = diag(l1, l2): the model reduces to scalar radial
    return on the principal log strains (closed form, any number of steps)."""
    E, nu, sy0, H = mat
    lam, G = M.lame(E, nu)
    ep = np.zeros(3)  # principal plastic log strains ln F^pl_i
    xi = 0.0
    out = []
    for l1, l2 in lams:
        ee = np.array([np.log(l1), np.log(l2), 0.0]) - ep
        s = lam * ee.sum() + 2 * G * ee
        dev = s - s.mean()
        q = np.sqrt(1.5) * np.linalg.norm(dev)
        f = q - (sy0 + H * xi)
        if f > 0:
            g = f / (3 * G + H)
            r = np.sqrt(1.5) * dev / np.linalg.norm(dev)
            s = s - 2 * G * g * r
            ep = ep + g * r
            xi += g
        out.append((s[0] / l1, s[1] / l2, xi, np.exp(ep)))
    return out


@pytest.mark.parametrize("mat", [MAT, MAT_EX1])
def test_coaxial_path_closed_form(mat):
    lams = [(1 + 0.02 * k, 1 - 0.015 * k) for k in range(1, 8)] + [(1.1 - 0.03 * k, 0.9 + 0.01 * k) for k in range(6)]
    ref = principal_path(lams, mat)
    Fp, Fp33, xi = M.virgin_history(())
    for (l1, l2), (P11, P22, xr, fp) in zip(lams, ref):
        P, A, Fp, Fp33, xi, g = M.j2_point(np.diag([l1, l2]), Fp, Fp33, xi, mat)
        assert abs(P[0, 0] - P11) < 1e-13 * max(1, abs(P11))
        assert abs(P[1, 1] - P22) < 1e-13 * max(1, abs(P22))
        assert abs(P[0, 1]) < 1e-15 and abs(P[1, 0]) < 1e-15
        assert abs(xi - xr) < 1e-14
        assert np.allclose([Fp[0, 0], Fp[1, 1], Fp33], fp, rtol=1e-13, atol=0)
    assert xi > 0  # the path does yield


def _random_states(rng, N, amp=0.06, pre=0.05):
    Fp, Fp33, xi = M.virgin_history((N,))
    Fpre = np.eye(2) + pre * rng.normal(size=(N, 2, 2))
    _, _, Fp, Fp33, xi, _ = M.j2_point(Fpre, Fp, Fp33, xi, MAT)
    F = np.eye(2) + amp * rng.normal(size=(N, 2, 2))
    return F, Fp, Fp33, xi


def test_tangent_matches_central_differences():
    rng = np.random.default_rng(1)
    F, Fp, Fp33, xi = _random_states(rng, 300)
    # half of the points unload into the elastic range
    F[150:] = np.eye(2) + 0.002 * rng.normal(size=(150, 2, 2))
    Fp[150:], Fp33[150:], xi[150:] = M.virgin_history((150,))
    P, A, *_ , g = M.j2_point(F, Fp, Fp33, xi, MAT)
    h = 1e-6
    Afd = np.zeros_like(A)
    for k in range(2):
        for l in range(2):
            d = np.zeros((2, 2))
            d[k, l] = h
            Pp = M.j2_update(F + d, Fp, Fp33, xi, MAT)[0]
            Pm = M.j2_update(F - d, Fp, Fp33, xi, MAT)[0]
            Afd[..., k, l] = (Pp - Pm) / (2 * h)
    gp = M.j2_update(F + 1e-6, Fp, Fp33, xi, MAT)[4]
    same_branch = (np.sign(gp) == np.sign(g))
    err = np.abs(A - Afd).max(axis=(1, 2, 3, 4))[same_branch]
    assert (g > 0).sum() > 50 and (g == 0).sum() > 5
    assert err.max() < 1e-7 * np.abs(A).max()


def test_tangent_major_symmetry():
    rng = np.random.default_rng(2)
    F, Fp, Fp33, xi = _random_states(rng, 300)
    A = M.j2_point(F, Fp, Fp33, xi, MAT)[1].reshape(-1, 4, 4)
    assert np.abs(A - np.swapaxes(A, -1, -2)).max() < 1e-12 * np.abs(A).max()


def test_objectivity_and_angular_momentum():
    rng = np.random.default_rng(3)
    F, Fp, Fp33, xi = _random_states(rng, 100)
    t = rng.uniform(0, 2 * np.pi, size=100)
    Q = np.stack([np.stack([np.cos(t), -np.sin(t)], -1), np.stack([np.sin(t), np.cos(t)], -1)], -2)
    P = M.j2_update(F, Fp, Fp33, xi, MAT)[0]
    PQ = M.j2_update(Q @ F, Fp, Fp33, xi, MAT)[0]
    assert np.abs(PQ - Q @ P).max() < 1e-14
    tau = P @ np.swapaxes(F, -1, -2)  # Kirchhoff stress must be symmetric
    assert np.abs(tau - np.swapaxes(tau, -1, -2)).max() < 1e-15


def test_plastic_flow_is_isochoric_and_consistent():
    rng = np.random.default_rng(4)
    F, Fp, Fp33, xi = _random_states(rng, 200)
    P, A, Fpn, Fp33n, xin, g = M.j2_point(F, Fp, Fp33, xi, MAT)
    assert np.abs(np.linalg.det(Fpn) * Fp33n - 1).max() < 1e-14
    # re-evaluating at the same F from the updated history is elastic (the
    # returned state lies on the yield surface) and gives the same stress
    P2, g2 = M.j2_update(F, Fpn, Fp33n, xin, MAT)[0::4]
    assert np.abs(g2).max() < 1e-14
    assert np.abs(P2 - P).max() < 1e-14


def test_elastic_stress_is_gradient_of_hencky_energy():
    lam, G = M.lame(*MAT[:2])
    rng = np.random.default_rng(5)
    F = np.eye(2) + 0.002 * rng.normal(size=(50, 2, 2))  # stays elastic (yield strain ~ 1e-2)
    Fp, Fp33, xi = M.virgin_history((50,))

    def psi(F):
        C = np.swapaxes(F, -1, -2) @ F
        w, _ = np.linalg.eigh(C)
        e = 0.5 * np.log(w)  # principal Hencky strains (eps_33 = 0)
        return G * (e ** 2).sum(-1) + 0.5 * lam * e.sum(-1) ** 2

    P, g = M.j2_update(F, Fp, Fp33, xi, MAT)[0::4]
    assert np.all(g == 0)
    h = 1e-6
    Pfd = np.zeros_like(P)
    for k in range(2):
        for l in range(2):
            d = np.zeros((2, 2))
            d[k, l] = h
            Pfd[..., k, l] = (psi(F + d) - psi(F - d)) / (2 * h)
    assert np.abs(P - Pfd).max() < 1e-9


def test_small_strain_limit_recovers_young_modulus():
    lam, G = M.lame(*MAT[:2])
    Fp, Fp33, xi = M.virgin_history(())
    d = 1e-7
    H = np.array([[0.3, 0.2], [-0.1, -0.5]]) * d
    P = M.j2_update(np.eye(2) + H, Fp, Fp33, xi, MAT)[0]
    eps = 0.5 * (H + H.T)
    sig = lam * np.trace(eps) * np.eye(2) + 2 * G * eps
    assert np.abs(P - sig).max() < 1e-6 * np.abs(sig).max()


def test_intermediate_stress_contraction_identity():
    """S = 2 sigma : d eps/dC equals sigma C^-1 for coaxial sigma (used in j2_update)."""
    rng = np.random.default_rng(6)
    C = random_spd(rng, 20)
    sig = 0.3 * np.eye(2) + 0.7 * C + 0.1 * C @ C  # coaxial with C
    h = 1e-6
    S = np.zeros_like(C)
    for k in range(2):
        for l in range(2):
            d = np.zeros((2, 2))
            d[k, l] += 0.5 * h
            d[l, k] += 0.5 * h
            de = 0.25 * (M.logm_sym2(C + d) - M.logm_sym2(C - d)) / h  # eps = 1/2 ln C, central difference
            S[..., k, l] = 2 * np.einsum('nij,nij->n', sig, de)
    assert np.abs(S - sig @ np.linalg.inv(C)).max() < 1e-8

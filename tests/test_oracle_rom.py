"""Pins of the oracle's offline reduction and online hyper-reduced solve
(Sec. 3): POD orthonormality and reconstruction, ECM exactness and
positivity, and the reduced solve reproducing the full-order model when the
basis is the full FE basis and the cubature is the full rule."""
import os
import tempfile

import numpy as np
import pytest

from oracle import artifact, auxiliary as aux, ecm, fem, fom, pod
from oracle import mesh as M
from oracle.rom import ROM

MAT = (1.0, 0.3, 0.01, 0.05)


def full_basis_rom(nt=2, nr=1):
    """A 'ROM' whose modes are the FE basis functions and whose cubature is
    the full rule: hyper-reduction is then the identity and the reduced
    solve must equal the full-order solve."""
    m = M.one_void_cell(0.25, nt, nr)
    sp = fem.PeriodicSpace(m)
    ax = aux.AuxiliaryProblem(m, 0)
    gm = ax.gradients(ax.modes())
    Gop = fem.gradient_operator(m, sp.node_dof, sp.ndof).toarray().reshape(m.nq, 4, sp.ndof)
    Gd = np.stack([g.reshape(m.nq, 4) for g in gm], axis=-1)
    data = dict(n=sp.ndof, m=m.nq, c=2, kind=0, n_mu=2, mat=MAT, r0=0.25, void_area=0.0, cell_area=1.0,
                w=m.qw.copy(), G=Gop, Gd=Gd, src=np.arange(m.nq))
    return m, sp, gm, data


def test_full_basis_rom_reproduces_fom():
    m, sp, gm, data = full_basis_rom()
    rom = ROM(data=data)
    mu = np.array([0.3, 0.21])
    E = np.array([[0.003, 0.001], [0.001, -0.002]])
    path = [np.eye(2) + k * E for k in range(1, 9)]
    Fmu = aux.transformation(gm, aux.coefficients(0, mu, 0.25))
    pr = fem.Problem(m, sp, Fmu, MAT)
    ref = fom.solve_path(pr, path, tol=1e-11, want_tangent=True)
    out = rom.run_path(mu, path, tol=1e-11)
    assert sum(o['iters'] for o in out) > 10
    for k in range(len(path)):
        assert out[k]['status'] == 0
        assert np.abs(out[k]['r'] - ref.w[k]).max() < 1e-10 * np.abs(ref.w[k]).max()
        assert np.abs(out[k]['Pbar'] - ref.Pbar[k].reshape(-1)).max() < 1e-12
        assert np.abs(out[k]['Abar'] - ref.Abar[k].reshape(4, 4)).max() < 1e-10 * np.abs(ref.Abar[k]).max()
    assert out[-1]['hist'][2].max() > 0  # the path yields somewhere


def test_parent_parameters_give_identity_transformation():
    _, _, _, data = full_basis_rom()
    Finv, J = ROM(data=data).transformation([0.25, 0.25])
    assert np.abs(Finv - np.eye(2)).max() == 0.0 and np.abs(J - 1).max() == 0.0


def test_rom_stiffness_symmetric_and_tangent_fd():
    _, _, _, data = full_basis_rom()
    rom = ROM(data=data)
    mu = [0.22, 0.33]
    Finv, J = rom.transformation(mu)
    F1 = np.array([[1.006, 0.002], [0.0015, 0.996]])
    s1 = rom.step(np.zeros(rom.n), rom.virgin(), F1, Finv, J, tol=1e-12)
    F2 = F1 + np.array([[0.003, 0.001], [0.001, -0.002]])
    s2 = rom.step(s1['r'], s1['hist'], F2, Finv, J, tol=1e-12)
    ev = rom.evaluate(s2['r'], F2, s1['hist'], Finv, J)
    assert np.abs(ev['K'] - ev['K'].T).max() < 1e-12 * np.abs(ev['K']).max()
    h = 1e-6
    Afd = np.zeros((4, 4))
    for kl in range(4):
        d = np.zeros(4)
        d[kl] = h
        sp_ = rom.step(s1['r'], s1['hist'], F2 + d.reshape(2, 2), Finv, J, tol=1e-13)
        sm_ = rom.step(s1['r'], s1['hist'], F2 - d.reshape(2, 2), Finv, J, tol=1e-13)
        Afd[:, kl] = (sp_['Pbar'] - sm_['Pbar']) / (2 * h)
    assert np.abs(s2['Abar'] - Afd).max() < 1e-6 * np.abs(Afd).max()


def test_pod_orthonormal_and_reconstructs_snapshots():
    rng = np.random.default_rng(0)
    N = 60
    A = rng.normal(size=(N, N))
    Mv = A @ A.T + N * np.eye(N)
    S = rng.normal(size=(N, 5)) @ rng.normal(size=(5, 12))  # rank 5
    Phi, lam = pod.pod(S, Mv, 5)
    assert np.abs(Phi.T @ Mv @ Phi - np.eye(5)).max() < 1e-12
    proj = Phi @ (Phi.T @ Mv @ S)
    assert np.abs(proj - S).max() < 1e-10 * np.abs(S).max()
    # the POD error of the leading modes equals the discarded eigenvalues
    Phi3, lam3 = pod.pod(S, Mv, 3)
    R = S - Phi3 @ (Phi3.T @ Mv @ S)
    assert abs(np.trace(R.T @ Mv @ R) - lam3[3:5].sum()) < 1e-9 * lam3.sum()
    with pytest.raises(ValueError):
        pod.pod(S, Mv, 7)


def test_ecm_integrates_polynomials_with_few_positive_points():
    m = M.mesh_square(6)
    x, y = m.qX[:, 0], m.qX[:, 1]
    J = np.stack([np.ones_like(x), x, y, x * y, x * x, y * y])
    idx, w, hist = ecm.greedy(J, m.qw, 1e-14, 50)
    assert len(idx) <= 6 and np.all(w > 0)
    assert np.abs(J[:, idx] @ w - J @ m.qw).max() < 1e-13
    assert np.all(np.diff(hist) <= 1e-12)


def test_ecm_residual_monotone_and_all_points_exact():
    rng = np.random.default_rng(1)
    m = M.mesh_square(3)
    J = rng.normal(size=(30, m.nq))
    idx, w, hist = ecm.greedy(J, m.qw, 1e-3, 40)
    assert np.all(w > 0) and np.all(np.diff(hist) <= 1e-12)
    # with as many points as the full rule the original weights are a solution
    idx2, w2, hist2 = ecm.greedy(J, m.qw, 1e-12, m.nq)
    assert hist2[-1] < 1e-10


def test_artifact_round_trip():
    _, _, _, data = full_basis_rom()
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, 'x.rom')
        artifact.write(p, data['n'], data['m'], 2, 0, 2, MAT, 0.25, 0.0, 1.0, data['w'], data['G'], data['Gd'],
                       data['src'])
        back = artifact.read(p)
    for k in ('w', 'G', 'Gd', 'src'):
        assert np.array_equal(back[k], data[k])
    assert back['n'] == data['n'] and back['m'] == data['m'] and back['mat'] == MAT


def test_load_step_cutting_equals_plain_steps_along_its_targets():
    """A step cut into sub-steps is the plain solve along the sequence of
    converged intermediate targets: replaying that sequence as an ordinary
    load path reproduces the state bit for bit.  Targets lie on the segment
    from the committed to the requested Fbar at increasing dyadic fractions,
    and depth 0 is the plain step."""
    rom_file = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), 'roms',
                            'onevoid_n20_m120.rom')
    if not os.path.exists(rom_file):
        pytest.skip("ROM artifact not built")
    import workloads
    rom = ROM(rom_file)
    mu = workloads.one_void_mu(7, 40)[6]
    Fb = workloads.monotone_paths(7, 40, 1, rho=(0.03, 0.06))[6, 0]
    Finv, J = rom.transformation(mu)
    r0, h0 = np.zeros(rom.n), rom.virgin()
    plain = rom.step(r0, h0, Fb, Finv, J, max_iter=15)
    assert plain['status'] == 1  # the full increment does not converge
    d0 = rom.cut_step(r0, h0, np.eye(2), Fb, Finv, J, max_iter=15, max_substeps=0)
    assert d0['status'] == 1 and d0['iters'] == plain['iters'] and np.array_equal(d0['r'], plain['r'])
    D = 4
    cut = rom.cut_step(r0, h0, np.eye(2), Fb, Finv, J, max_iter=15, max_substeps=D)
    assert cut['status'] == 0 and len(cut['targets']) >= 1
    fr = []
    for T in cut['targets']:
        s = (T - np.eye(2)) / (Fb - np.eye(2))
        assert np.ptp(s) < 1e-12  # on the segment
        fr.append(s.mean() * 2 ** D)
    assert np.allclose(fr, np.round(fr), atol=1e-9) and all(np.diff(fr) > 0) and fr[-1] < 2 ** D
    # the reported end points are the intermediate targets' fractions, then the full step
    assert cut['ends'] == [int(round(f)) for f in fr] + [2 ** D]
    replay = rom.run_path(mu, cut['targets'] + [Fb], max_iter=15)
    assert all(s['status'] == 0 for s in replay)
    assert np.array_equal(replay[-1]['r'], cut['r'])
    assert all(np.array_equal(a, b) for a, b in zip(replay[-1]['hist'], cut['hist']))
    assert np.array_equal(replay[-1]['Pbar'], cut['Pbar'])
    assert cut['iters'] > sum(s['iters'] for s in replay)  # the failed attempts count too
    # a path through run_path with cutting commits the same state
    via = rom.run_path(mu, [Fb], max_iter=15, max_substeps=D)[-1]
    assert np.array_equal(via['r'], cut['r'])


def _graded_square(v):
    """Void-free unit cell on the vertex lines v (both directions), two T6 per
    quad: elements of unequal size, so a misplaced quadrature weight shows."""
    v = np.asarray(v, dtype=np.float64)
    s = np.empty(2 * v.size - 1)
    s[0::2] = v
    s[1::2] = 0.5 * (v[1:] + v[:-1])
    P = np.zeros((s.size, s.size, 2))
    P[..., 0] = s[:, None]
    P[..., 1] = s[None, :]
    merger = M._NodeMerger()
    elems = []
    M._add_quad_grid(merger, elems, P, -1)
    return M.Mesh(np.array(merger.pts), np.array(elems), np.array(merger.void), [])


def _square_problem(v):
    m = _graded_square(v)
    sp = fem.PeriodicSpace(m)
    pr = fem.Problem(m, sp, np.tile(np.eye(2), (m.nq, 1, 1)), MAT)
    return m, sp, pr


def _nodal_dofs(m, sp, fx, fy):
    """DOF vector of the periodic field (fx, fy) sampled at the master nodes."""
    w = np.zeros(sp.ndof)
    for a in sp.free_nodes:
        k = sp.node_dof[a]
        x, y = m.X[a]
        w[2 * k], w[2 * k + 1] = fx(x, y), fy(x, y)
    return w


def test_v_gram_exact_on_piecewise_linear_periodic_fields():
    """eq. Vdotproduct on the parent cell: (u, v)_V = int u.v + grad u : grad v.
    The triangle wave t(s) = 1 - |2 s - 1| is periodic, vanishes at the fixed
    corner and is linear on every element of a grid with a line at s = 1/2,
    so the degree-2 rule integrates both terms exactly:
    int t^2 = 1/3, int t'^2 = 4, int t(x) t(y) = 1/4, grad t(x) . grad t(y) = 0."""
    m, sp, pr = _square_problem([0.0, 0.12, 0.3, 0.5, 0.55, 0.8, 1.0])
    assert np.ptp(m.qw) > 0.1 * m.qw.max()  # unequal elements
    MV = pod.v_gram(pr)
    t = lambda s: 1.0 - abs(2.0 * s - 1.0)  # noqa: E731
    z = lambda x, y: 0.0  # noqa: E731
    ux = _nodal_dofs(m, sp, lambda x, y: t(x), z)      # (t(x), 0)
    uy = _nodal_dofs(m, sp, z, lambda x, y: t(y))      # (0, t(y))
    vx = _nodal_dofs(m, sp, lambda x, y: t(y), z)      # (t(y), 0): d/dy of the first component
    cx = _nodal_dofs(m, sp, z, lambda x, y: t(x))      # (0, t(x))
    s = _nodal_dofs(m, sp, lambda x, y: t(x) + t(y), z)
    ip = lambda a, b: float(a @ (MV @ b))  # noqa: E731
    assert abs(ip(ux, ux) - (1 / 3 + 4)) < 1e-12
    assert abs(ip(uy, uy) - (1 / 3 + 4)) < 1e-12
    assert abs(ip(vx, vx) - (1 / 3 + 4)) < 1e-12
    assert abs(ip(ux, vx) - 0.25) < 1e-12       # mass term only: the gradients are orthogonal
    assert abs(ip(ux, cx)) < 1e-12              # different components never couple
    assert abs(ip(s, s) - (2 * (1 / 3 + 4) + 2 * 0.25)) < 1e-12
    # symmetric, and positive on every non-zero field
    assert abs(MV - MV.T).max() < 1e-14
    rng = np.random.default_rng(3)
    for _ in range(3):
        v = rng.standard_normal(sp.ndof)
        assert ip(v, v) > 0


def test_integrand_matrix_integrals_of_affine_fields():
    """eq. integralsbasis: J[(i, l), q] = grad phi_i(X_q) : B_l(X_q), and
    J w_hat = int grad phi_i : B_l.  With affine fields
    G_i[a] = al + be x + ga y and B_l[a] = de + ep x + ze y the integrand is
    quadratic, integrated exactly by the degree-2 rule over the unit square:
    int = al de + (al ep + be de + al ze + ga de) / 2 + (be ep + ga ze) / 3 + (be ze + ga ep) / 4,
    summed over the four components a.  Random coefficients make a transposed
    contraction or a (l, i) row order fail."""
    m = _graded_square([0.0, 0.2, 0.45, 0.5, 0.9, 1.0])
    rng = np.random.default_rng(11)
    n, L = 3, 4
    cg = rng.standard_normal((3, n, 4))   # al, be, ga of G_i[a]
    cb = rng.standard_normal((3, L, 4))   # de, ep, ze of B_l[a]
    x, y = m.qX[:, 0], m.qX[:, 1]
    G = (cg[0][None] + cg[1][None] * x[:, None, None] + cg[2][None] * y[:, None, None]).transpose(0, 2, 1)
    B = (cb[0][None] + cb[1][None] * x[:, None, None] + cb[2][None] * y[:, None, None]).transpose(0, 2, 1)
    J = ecm.integrand_matrix(G, B, n, L)
    assert J.shape == (n * L, m.nq)
    al, be, ga = cg[:, :, None, :]
    de, ep, ze = cb[:, None, :, :]
    exact = (al * de + (al * ep + be * de + al * ze + ga * de) / 2 + (be * ep + ga * ze) / 3
             + (be * ze + ga * ep) / 4).sum(axis=-1).reshape(n * L)
    assert np.abs(J @ m.qw - exact).max() < 1e-12

"""Two-phase cells (multi-phase RVEs; here a one-void cell whose
void is lined with a stiff elastic coating) in the oracle, pinned by what
fixes them independently: the material routine with per-point constants
equals point-by-point calls with scalars (the tangent to rounding); a second phase with the matrix's
own constants reproduces the single-phase solve exactly; with the full FE
basis and the full rule, the two-phase reduced solve equals the two-phase
full-order solve (hyper-reduction is then the identity); and the artifact
keeps the phases (version 2) while version-1 files read as one phase."""
import os
import tempfile

import numpy as np

import workloads
from oracle import artifact, auxiliary as aux, build_rom, fem, fom, material
from oracle import mesh as M
from oracle.rom import ROM
from tests.test_oracle_rom import MAT, full_basis_rom

MAT2 = (10.0, 0.3, 1.0e3, 0.0)


def test_material_with_per_point_constants_equals_scalar_calls():
    g = workloads.rng(21)
    P = 12
    F = np.eye(2)[None] + 0.03 * g.standard_normal((P, 2, 2))
    hist = material.virgin_history((P,))
    ph = g.integers(0, 2, P)
    mats = tuple(np.where(ph == 1, b, a) for a, b in zip(MAT, MAT2))
    Pv, Av, Fpv, Fp33v, xiv, _ = material.j2_point(F, *hist, mats)
    for p in range(P):
        mp = MAT2 if ph[p] else MAT
        Ps, As, Fps, Fp33s, xis, _ = material.j2_point(F[p], hist[0][p], hist[1][p], hist[2][p], mp)
        assert np.array_equal(Pv[p], Ps)
        # complex-step tangent: batched and single-point complex arithmetic round differently
        assert np.abs(Av[p] - As).max() <= 1e-13 * np.abs(As).max()
        assert np.array_equal(Fpv[p], Fps) and Fp33v[p] == Fp33s and xiv[p] == xis
    assert np.any(xiv[ph == 0] > 0) and np.all(xiv[ph == 1] == 0)  # the matrix yields, the coating does not


def _path():
    E = np.array([[0.004, 0.001], [0.001, -0.003]])
    return [np.eye(2) + k * E for k in range(1, 7)]


def test_second_phase_with_matrix_constants_is_single_phase():
    m, sp, gm, data = full_basis_rom()
    spec = dict(build_rom.ROMS['coatvoid_n20_m120'])
    ph = build_rom.phases(spec, m)
    assert 0 < ph.sum() < m.nq
    mu = np.array([0.28, 0.22])
    Fmu = aux.transformation(gm, aux.coefficients(0, mu, 0.25))
    same = tuple(np.where(ph == 1, a, a) for a in MAT)
    r1 = fom.solve_path(fem.Problem(m, sp, Fmu, MAT), _path(), tol=1e-11)
    r2 = fom.solve_path(fem.Problem(m, sp, Fmu, same), _path(), tol=1e-11)
    assert np.array_equal(np.array(r1.Pbar), np.array(r2.Pbar))
    rom1 = ROM(data=data)
    rom2 = ROM(data=dict(data, mat2=MAT, phase=ph))
    o1, o2 = rom1.run_path(mu, _path(), tol=1e-11), rom2.run_path(mu, _path(), tol=1e-11)
    for a, b in zip(o1, o2):
        assert np.array_equal(a['Pbar'], b['Pbar']) and np.array_equal(a['Abar'], b['Abar'])


def test_full_basis_two_phase_rom_reproduces_two_phase_fom():
    m, sp, gm, data = full_basis_rom()
    spec = dict(build_rom.ROMS['coatvoid_n20_m120'])
    ph = build_rom.phases(spec, m)
    rom = ROM(data=dict(data, mat2=MAT2, phase=ph))
    mu = np.array([0.3, 0.21])
    Fmu = aux.transformation(gm, aux.coefficients(0, mu, 0.25))
    mats = tuple(np.where(ph == 1, b, a) for a, b in zip(MAT, MAT2))
    ref = fom.solve_path(fem.Problem(m, sp, Fmu, mats), _path(), tol=1e-11, want_tangent=True)
    out = rom.run_path(mu, _path(), tol=1e-11)
    for k in range(len(_path())):
        assert out[k]['status'] == 0
        assert np.abs(out[k]['Pbar'] - ref.Pbar[k].reshape(-1)).max() < 1e-12
        assert np.abs(out[k]['Abar'] - ref.Abar[k].reshape(4, 4)).max() < 1e-10 * np.abs(ref.Abar[k]).max()
    # the coating changes the answer
    single = ROM(data=data).run_path(mu, _path(), tol=1e-11)
    assert np.abs(single[-1]['Pbar'] - out[-1]['Pbar']).max() > 1e-3 * np.abs(out[-1]['Pbar']).max()


def test_artifact_keeps_phases():
    _, _, _, data = full_basis_rom()
    ph = (np.arange(data['m']) % 3 == 0).astype(np.int64)
    with tempfile.TemporaryDirectory() as d:
        p1, p2 = os.path.join(d, 'a.rom'), os.path.join(d, 'b.rom')
        args = (data['n'], data['m'], 2, 0, 2, MAT, 0.25, 0.0, 1.0, data['w'], data['G'], data['Gd'], data['src'])
        artifact.write(p1, *args)
        artifact.write(p2, *args, mat2=MAT2, phase=ph)
        one, two = artifact.read(p1), artifact.read(p2)
    assert one['mat2'] is None and not one['phase'].any()
    assert two['mat2'] == MAT2 and np.array_equal(two['phase'], ph)
    assert np.array_equal(two['G'], data['G'])


# the composite cell with stiff elliptical inclusions (Sec. 4.1)
def _small_inclusions():
    inc = np.array([[0.3, 0.3, 0.12, 0.08, 0.4], [0.7, 0.65, 0.1, 0.1, 0.0], [0.28, 0.74, 0.09, 0.06, 2.0]])
    return M.inclusion_cell(12, inc), inc


def test_inclusion_layout_and_phases():
    """The seeded layout holds the requested area fraction exactly, its
    ellipses grown by the largest scale (1.2) stay apart and inside the cell;
    the quadrature points' phases cover the inclusion area to the mesh
    resolution; the point-in-ellipse test at known points."""
    L = workloads.inclusion_layout(5)
    assert L.shape == (23, 5) and abs(np.sum(np.pi * L[:, 2] * L[:, 3]) - 0.234) < 1e-12
    t = np.linspace(0, 2 * np.pi, 400, endpoint=False)
    pts = []
    for cx, cy, a, b, th in L:
        R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        B = np.array([cx, cy]) + (R @ np.stack([1.2 * a * np.cos(t), 1.2 * b * np.sin(t)])).T
        assert B.min() > 0 and B.max() < 1
        pts.append(B)
    for i, B in enumerate(pts):
        grown = L.copy()
        grown[:, 2:4] *= 1.2
        hit = M.in_ellipses(B, np.delete(grown, i, axis=0))
        assert (hit < 0).all(), i
    m = M.inclusion_cell(40, L)
    assert abs(np.sum(m.qw * m.qphase) - 0.234) < 3e-3
    inc = np.array([[0.5, 0.5, 0.2, 0.1, np.pi / 2]])  # long axis along y
    assert list(M.in_ellipses(np.array([[0.5, 0.5], [0.5, 0.69], [0.69, 0.5], [0.5, 0.71]]), inc)) == [0, 0, -1, -1]


def test_inclusion_transformation_scales_every_inclusion():
    """kind 2: c = zeta - 1 with one mode; F_mu = I at zeta = 1, F_mu affine
    in zeta, exactly zeta I on the elements whose nodes all lie in one
    inclusion, zero displacement on the cell boundary, det F_mu > 0 over
    zeta in [0.5, 1.2]; dc/dzeta = 1."""
    m, inc = _small_inclusions()
    ax = aux.AuxiliaryProblem(m, 2)
    modes = ax.modes()
    assert modes.shape[0] == aux.n_coeff(2) == 1
    assert np.abs(modes[0][m.outer_boundary_nodes()]).max() == 0.0
    gm = ax.gradients(modes)
    assert np.array_equal(aux.transformation(gm, aux.coefficients(2, [1.0], 0.0)), np.broadcast_to(np.eye(2), (m.nq, 2, 2)))
    F07 = aux.transformation(gm, aux.coefficients(2, [0.7], 0.0))
    F12 = aux.transformation(gm, aux.coefficients(2, [1.2], 0.0))
    assert np.abs((F07 - np.eye(2)) / -0.3 - (F12 - np.eye(2)) / 0.2).max() < 1e-12
    idx = m.void_of_node[m.T]
    inside = np.repeat((idx.min(axis=1) >= 0) & (idx.max(axis=1) == idx.min(axis=1)), 3)
    assert inside.sum() > 0
    assert np.abs(F07[inside] - 0.7 * np.eye(2)).max() < 1e-12
    for z in (0.5, 1.2):
        assert np.linalg.det(aux.transformation(gm, aux.coefficients(2, [z], 0.0))).min() > 0
    h = 1e-6
    fd = (aux.coefficients(2, [0.9 + h], 0.0) - aux.coefficients(2, [0.9 - h], 0.0)) / (2 * h)
    assert np.allclose(aux.coefficient_jacobian(2, [0.9], 0.0), fd[:, None], atol=1e-9)


def test_full_basis_inclusion_rom_reproduces_fom():
    """With the full FE basis and the full rule, the reduced solve of the
    inclusion cell (kind 2, two phases; one inclusion on a 6 x 6 mesh, so
    that the dense full-basis reduced operators stay small) equals its
    full-order solve."""
    m = M.inclusion_cell(6, np.array([[0.45, 0.5, 0.22, 0.15, 0.3]]))
    assert 0 < m.qphase.sum() < m.nq
    sp = fem.PeriodicSpace(m)
    ax = aux.AuxiliaryProblem(m, 2)
    gm = ax.gradients(ax.modes())
    Gop = fem.gradient_operator(m, sp.node_dof, sp.ndof).toarray().reshape(m.nq, 4, sp.ndof)
    Gd = np.stack([g.reshape(m.nq, 4) for g in gm], axis=-1)
    data = dict(n=sp.ndof, m=m.nq, c=1, kind=2, n_mu=1, mat=MAT, r0=0.0, void_area=0.0, cell_area=1.0,
                w=m.qw.copy(), G=Gop, Gd=Gd, src=np.arange(m.nq), mat2=MAT2, phase=m.qphase)
    rom = ROM(data=data)
    mu = np.array([0.8])
    Fmu = aux.transformation(gm, aux.coefficients(2, mu, 0.0))
    mats = tuple(np.where(m.qphase == 1, b, a) for a, b in zip(MAT, MAT2))
    ref = fom.solve_path(fem.Problem(m, sp, Fmu, mats), _path(), tol=1e-11, want_tangent=True)
    out = rom.run_path(mu, _path(), tol=1e-11)
    for k in range(len(_path())):
        assert out[k]['status'] == 0
        assert np.abs(out[k]['Pbar'] - ref.Pbar[k].reshape(-1)).max() < 1e-12
        assert np.abs(out[k]['Abar'] - ref.Abar[k].reshape(4, 4)).max() < 1e-10 * np.abs(ref.Abar[k]).max()

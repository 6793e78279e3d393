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

"""Two-scale driver on the GPU against the oracle (Sec. 4.2 setting).

* the whole macro Newton loop on a 4 x 2 block (32 RVE points, four load
  steps up and down, plastic at the peak): same statuses and macro
  iteration counts, displacements and compliance within 1e-9 relative;
* the patch test (uniform deformation from boundary displacements);
* each macro kernel at the full size of the example (20 x 10 elements, 800
  points, 1322 dofs): deformation gradient, traction, residual and
  compliance against the oracle's operators, the banded LU solve against a
  dense solve of the oracle's stiffness with the same Abar;
* full-size load steps through the RVE solve: every step converges and
  sampled points reproduce the oracle's RVE solve at the GPU's Fbar.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import fe2 as ofe2
from oracle.rom import ROM
from tests.conftest import rom_path

import paper_2307_16894_amd as L
from paper_2307_16894_amd.fe2 import Fe2Solver

pytestmark = pytest.mark.gpu


def shape(Xg):
    return workloads.fe2_shape(Xg[:, 0], Xg[:, 1])


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def test_two_scale_loop_matches_oracle(gpu):
    name = 'onevoid_n20_m120'
    mesh = workloads.fe2_mesh(4, 2)
    loads = workloads.fe2_loads(4, 0.008)
    ref = ofe2.run(ROM(rom_path(name)), mesh, shape(ofe2.geometry(mesh)['Xg']), loads)
    for mode in (L.MODE_FUSED, L.MODE_PHASED):
        print(f"[gpu] fe2 small mesh mode {mode}", flush=True)
        sol = Fe2Solver(rom_path(name), mesh, shape, mode=mode)
        out = sol.run(loads)
        sol.close()
        assert len(out) == len(ref)
        for k, (g, o) in enumerate(zip(out, ref)):
            assert g['status'] == 0 and o['status'] == 0, k
            assert g['macro_iters'] == o['macro_iters'], (k, g['macro_iters'], o['macro_iters'])
            scale = max(np.abs(o['u']).max(), 1e-300)
            assert np.abs(g['u'] - o['u']).max() <= 1e-9 * scale, (k, rel(g['u'], o['u']))
            assert abs(g['C'] - o['C']) <= 1e-9 * max(abs(o['C']), 1e-300), (k, g['C'], o['C'])
        print(f"macro iterations {[g['macro_iters'] for g in out]}, RVE evaluations "
              f"{[g['rve_evals'] for g in out]} (oracle {[o['rve_evals'] for o in ref]})")


def test_patch_test(gpu):
    mesh = workloads.fe2_mesh(2, 2)
    X = mesh['X']
    on = (X[:, 0] == 0) | (X[:, 1] == 0) | np.isclose(X[:, 0], mesh['width']) | np.isclose(X[:, 1], mesh['height'])
    nodes = np.flatnonzero(on)
    fixed = np.sort(np.concatenate([2 * nodes, 2 * nodes + 1]))
    F0 = np.array([[1.006, 0.002], [-0.001, 0.995]])
    lin = ((F0 - np.eye(2)) @ X.T).T.reshape(-1)
    mu1 = workloads.one_void_mu(7, 1)
    sol = Fe2Solver(rom_path('onevoid_n20_m120'), mesh, lambda Xg: np.tile(mu1, (Xg.shape[0], 1)), fixed_dofs=fixed)
    out = sol.run([0.0], fixed_values=[lin[fixed]], tol_abs=1e-13)
    F = sol.F.cpu().numpy()
    sol.close()
    assert out[0]['status'] == 0
    assert np.abs(out[0]['u'] - lin).max() < 1e-11
    assert np.abs(F - F0.reshape(1, 4)).max() < 1e-11


@pytest.fixture(scope='module')
def full():
    mesh = workloads.fe2_mesh(20, 10)
    return mesh, ofe2.geometry(mesh)


@pytest.mark.parametrize("dims", [(20, 10), (3, 30)])
def test_macro_kernels_full_size(gpu, full, dims):
    """(20, 10): the example (half-bandwidth 65, the LDS-window solve);
    (3, 30): a tall block numbered across its long side (half-bandwidth
    above 95, the global-memory solve)."""
    mesh, geo = full if dims == (20, 10) else (lambda m: (m, ofe2.geometry(m)))(workloads.fe2_mesh(*dims))
    name = 'onevoid_n40_m400'
    sol = Fe2Solver(rom_path(name), mesh, shape)
    s = sol.stream.cuda_stream
    print(f"[gpu] fe2 operators {dims}: {sol.info}", flush=True)
    if dims == (20, 10):
        assert sol.info['dofs'] == 1322 and sol.info['points'] == 800 and sol.info['kl'] <= 95
    else:
        assert 95 < sol.info['kl'] <= 255
    ndof = sol.info['dofs']
    assert np.abs(sol.Xg.cpu().numpy() - geo['Xg']).max() < 1e-14
    x, y = mesh['X'][:, 0], mesh['X'][:, 1]
    u = np.stack([0.003 * x * y - 0.002 * y * y, -0.006 * y + 0.001 * x * y * (2 - x)], axis=1).reshape(-1)
    sol.u.copy_(torch.from_numpy(u))
    L.rom_fe2_gradient(sol.h, sol.u.data_ptr(), sol.F.data_ptr(), s)
    T = 0.011
    L.rom_fe2_traction(sol.h, T, sol.fext.data_ptr(), s)
    torch.cuda.synchronize()
    Fo = ofe2.deformation_gradient(mesh, geo, u).reshape(-1, 4)
    assert np.abs(sol.F.cpu().numpy() - Fo).max() < 1e-14
    fext_o = ofe2.external_force(mesh, T)
    assert np.abs(sol.fext.cpu().numpy() - fext_o).max() < 1e-15
    # the RVEs at that Fbar give Pbar, Abar; residual and solve against the oracle's operators
    st, _, _ = sol.rb.step(sol.F, L.rom_default_opts(commit=0, tol=1e-10, max_iter=25))
    L.rom_fe2_residual(sol.h, sol.rb.Pbar.data_ptr(), sol.fext.data_ptr(), sol.res.data_ptr(), sol.norms.data_ptr(), s)
    torch.cuda.synchronize()
    assert int((st != 0).sum()) == 0
    Pbar, Abar = sol.rb.Pbar.cpu().numpy(), sol.rb.Abar.cpu().numpy()
    res_o = fext_o - ofe2.internal_force(mesh, geo, Pbar)
    res = sol.res.cpu().numpy()
    assert np.abs(res - res_o).max() <= 1e-12 * np.abs(res_o).max()
    free = np.setdiff1d(np.arange(ndof), sol.fixed)
    nr, nf = sol.norms.cpu().numpy()
    assert abs(nr - np.linalg.norm(res_o[free])) <= 1e-12 * nr
    assert abs(nf - np.linalg.norm(fext_o[free])) <= 1e-12 * nf
    K = ofe2.stiffness(mesh, geo, Abar)
    du_o = np.linalg.solve(K[np.ix_(free, free)], res_o[free])
    L.rom_fe2_solve(sol.h, sol.rb.Abar.data_ptr(), sol.res.data_ptr(), None, sol.u.data_ptr(),
                    sol.solve_info.data_ptr(), s)
    torch.cuda.synchronize()
    assert int(sol.solve_info.item()) == 0
    du = sol.u.cpu().numpy() - u
    assert np.abs(du[sol.fixed]).max() == 0.0
    assert np.abs(du[free] - du_o).max() <= 1e-9 * np.abs(du_o).max(), rel(du[free], du_o)
    # -Abar: a negative definite tangent, so the Cholesky form gives way to
    # the LU form with row interchanges (same launch); the step is -du
    negA = (-sol.rb.Abar).contiguous()
    sol.u.copy_(torch.from_numpy(u))
    L.rom_fe2_solve(sol.h, negA.data_ptr(), sol.res.data_ptr(), None, sol.u.data_ptr(), sol.solve_info.data_ptr(), s)
    torch.cuda.synchronize()
    assert int(sol.solve_info.item()) == 0
    dn = sol.u.cpu().numpy() - u
    assert np.abs(dn[free] + du_o).max() <= 1e-9 * np.abs(du_o).max(), rel(-dn[free], du_o)
    sol.u.copy_(torch.from_numpy(u + du))
    L.rom_fe2_compliance(sol.h, T, sol.u.data_ptr(), sol.C.data_ptr(), s)
    torch.cuda.synchronize()
    Co = ofe2.compliance(mesh, T, sol.u.cpu().numpy())
    assert abs(float(sol.C.item()) - Co) <= 1e-13 * abs(Co)
    sol.close()


def test_full_size_load_steps(gpu, full):
    """Four load steps of the full-size example; after the first (from the
    virgin state) sampled points are solved by the oracle at the GPU's final
    Fbar and must give the same Pbar."""
    mesh, geo = full
    name = 'onevoid_n40_m400'
    loads = workloads.fe2_loads(50, 0.012)[:4]
    sol = Fe2Solver(rom_path(name), mesh, shape)
    rom = ROM(rom_path(name))
    mu = shape(geo['Xg'])
    out = []
    for k, T in enumerate(loads):
        print(f"[gpu] fe2 full size step {k}", flush=True)
        out.append(sol.load_step(T))
        assert out[-1]['status'] == 0, (k, out[-1])
        if k == 0:
            F, Pg = sol.F.cpu().numpy(), sol.rb.Pbar.cpu().numpy()
            for p in range(0, 800, 97):
                o = rom.step(np.zeros(rom.n), rom.virgin(), F[p].reshape(2, 2), *rom.transformation(mu[p]),
                             tol=1e-10, max_iter=25)
                assert o['status'] == 0, p
                assert rel(Pg[p], o['Pbar']) < 1e-9, (p, rel(Pg[p], o['Pbar']))
    sol.close()
    C = [r['C'] for r in out]
    assert all(c > 0 for c in C) and all(b > a for a, b in zip(C, C[1:]))
    print(f"full size: macro iterations {[r['macro_iters'] for r in out]}, compliance {C}")


def test_compliance_error_against_full_order_two_scale(gpu):
    """The GPU two-scale loop with the n = 20 ROM against the full-order
    two-scale reference of tests/golden/fe2_fom_4x2.json (Sec. 4.2): the
    compliance error per loaded step equals the oracle ROM's (the GPU loop
    reproduces the oracle's), and its mean lies in the paper's band."""
    import json
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    ref = json.load(open(os.path.join(here, 'golden', 'fe2_fom_4x2.json')))
    mesh = workloads.fe2_mesh(*ref['macro_mesh'])
    loads = workloads.fe2_loads(ref['load_steps'], ref['peak_traction'])
    rom_file = rom_path(ref['cell'])
    orc = ofe2.run(ROM(rom_file), mesh, shape(ofe2.geometry(mesh)['Xg']), loads)
    print("[gpu] fe2 compliance error", flush=True)
    sol = Fe2Solver(rom_file, mesh, shape, mode=L.MODE_PHASED)
    out = sol.run(loads)
    sol.close()
    Cr = np.array(ref['compliance'])
    loaded = np.asarray(loads) > 0
    C = np.array([o['C'] for o in out])
    Co = np.array([o['C'] for o in orc])
    assert all(o['status'] == 0 for o in out)
    eps = np.abs(C[loaded] - Cr[loaded]) / np.abs(Cr[loaded])
    eps_o = np.abs(Co[loaded] - Cr[loaded]) / np.abs(Cr[loaded])
    print("eps_C per loaded step", np.round(eps, 4), "mean", eps.mean())
    assert np.abs(eps - eps_o).max() < 1e-7
    assert eps.mean() < 0.06

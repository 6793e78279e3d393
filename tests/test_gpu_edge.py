"""GPU edge cases: empty batch, rejected shape parameters, non-finite input,
iteration cap without commit and caller-side sub-stepping, and the
full-basis / full-rule ROM reproducing the full-order model."""
import os
import tempfile

import numpy as np
import pytest
import torch

import workloads
from oracle import artifact, auxiliary as aux, fem, fom
from oracle.rom import ROM
from tests.conftest import rom_path
from tests.test_oracle_rom import MAT, full_basis_rom

import paper_2307_16894_amd as L
from paper_2307_16894_amd.batch import RomBatch

pytestmark = pytest.mark.gpu
NAME = 'onevoid_n20_m120'


def _bad_mu(rom):
    """Shape parameters for which the oracle finds det F_mu <= 0 at an ECM point."""
    for a in np.linspace(-0.3, 0.05, 36):
        J = rom.transformation([a, 0.25])[1]
        if J.min() <= 0:
            return np.array([a, 0.25])
    raise AssertionError("no invalid parameters found")


@pytest.mark.parametrize("mode", [0, 1])
def test_empty_batch_is_a_no_op(gpu, mode):
    h = L.rom_load_file(rom_path(NAME), 0)
    o = L.rom_default_opts(mode=mode)
    s = torch.cuda.current_stream().cuda_stream
    assert L.rom_state_bytes(h, 0) >= 0
    assert L.lib().rom_step(h, 0, None, None, None, None, None, None, s) == L.ROM_OK
    assert L.lib().rom_state_init(h, 0, None, None, s) == L.ROM_OK
    L.rom_free(h)


@pytest.mark.parametrize("mode", [0, 1])
def test_rejected_shape_parameters_and_nonfinite_load(gpu, mode):
    rom = ROM(rom_path(NAME))
    P = 6
    mu = workloads.one_void_mu(3, P)
    mu[2] = _bad_mu(rom)
    rb = RomBatch(rom_path(NAME), mu)
    assert rb.init_code == L.ROM_EINVAL_MU
    assert rb.mu_ok().cpu().tolist() == [1, 1, 0, 1, 1, 1]
    F = workloads.monotone_paths(3, P, 10)[:, 0].copy()
    F[4, 0, 0] = np.nan
    h0 = rb.history().clone()
    st, it, rn = rb.step(torch.from_numpy(F).cuda(), L.rom_default_opts(mode=mode))
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert st[2] == L.ST_BADMU and st[4] == L.ST_NONFINITE
    assert all(st[i] == L.ST_CONVERGED for i in (0, 1, 3, 5))
    assert torch.isnan(rb.Pbar[2]).all()
    # nothing committed for the failed points
    assert torch.equal(rb.history()[4], h0[4])
    for i in (0, 1, 3, 5):
        ref = rom.run_path(mu[i], F[i:i + 1])[-1]
        assert np.abs(rb.Pbar[i].cpu().numpy() - ref['Pbar']).max() < 1e-6 * np.abs(ref['Pbar']).max()
    rb.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_iteration_cap_keeps_committed_state_and_substepping_recovers(gpu, mode):
    P = 4
    mu = workloads.one_void_mu(5, P)
    rb = RomBatch(rom_path(NAME), mu)
    E = np.array([[0.06, 0.02], [0.02, -0.05]])
    F = np.broadcast_to(np.eye(2) + E, (P, 2, 2)).copy()
    r0 = rb.r().clone()
    h0 = rb.history().clone()
    st, it, _ = rb.step(torch.from_numpy(F).cuda(), L.rom_default_opts(mode=mode, max_iter=2))
    torch.cuda.synchronize()
    assert (st.cpu() == L.ST_MAXITER).all() and (it.cpu() == 2).all()
    assert torch.equal(rb.r(), r0) and torch.equal(rb.history(), h0)
    # the caller sub-steps: ten smaller increments converge
    for k in range(1, 11):
        st, it, _ = rb.step(torch.from_numpy(np.broadcast_to(np.eye(2) + 0.1 * k * E, (P, 2, 2)).copy()).cuda(),
                            L.rom_default_opts(mode=mode))
        torch.cuda.synchronize()
        assert (st.cpu() == L.ST_CONVERGED).all(), k
    rom = ROM(rom_path(NAME))
    path = [np.eye(2) + 0.1 * k * E for k in range(1, 11)]
    for i in range(P):
        ref = rom.run_path(mu[i], path)[-1]
        assert np.abs(rb.Pbar[i].cpu().numpy() - ref['Pbar']).max() < 1e-6 * np.abs(ref['Pbar']).max()
    rb.close()


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("blocks", [(2, 1), (3, 1)])  # n = 76 and 116: both contraction layouts
def test_full_basis_rom_on_gpu_reproduces_fom(gpu, mode, blocks):
    m, sp, gm, data = full_basis_rom(*blocks)
    assert data['n'] <= 123
    mu = np.array([[0.3, 0.21], [0.22, 0.31]])
    E = np.array([[0.003, 0.001], [0.001, -0.002]])
    path = np.array([np.eye(2) + k * E for k in range(1, 9)])
    with tempfile.TemporaryDirectory() as d:
        f = os.path.join(d, 'full.rom')
        artifact.write(f, data['n'], data['m'], 2, 0, 2, MAT, 0.25, 0.0, 1.0, data['w'], data['G'], data['Gd'],
                       data['src'])
        rb = RomBatch(f, mu)
    for p in range(2):
        Fmu = aux.transformation(gm, aux.coefficients(0, mu[p], 0.25))
        ref = fom.solve_path(fem.Problem(m, sp, Fmu, MAT), path, tol=1e-11, want_tangent=True)
        if p == 0:
            outs = []
            for k in range(len(path)):
                st, it, rn = rb.step(torch.from_numpy(np.broadcast_to(path[k], (2, 2, 2)).copy()).cuda(),
                                     L.rom_default_opts(mode=mode, tol=1e-11, max_iter=25))
                torch.cuda.synchronize()
                outs.append((st.cpu().numpy().copy(), rb.r(trial=True).cpu().numpy().copy(),
                             rb.Pbar.cpu().numpy().copy(), rb.Abar.cpu().numpy().copy()))
        for k in range(len(path)):
            st, r, Pb, Ab = outs[k]
            assert st[p] == 0
            assert np.abs(r[p] - ref.w[k]).max() < 1e-9 * np.abs(ref.w[k]).max()
            assert np.abs(Pb[p] - ref.Pbar[k].reshape(-1)).max() < 1e-12
            assert np.abs(Ab[p] - ref.Abar[k].reshape(-1)).max() < 1e-9 * np.abs(ref.Abar[k]).max()
    rb.close()

"""rom_step_noalloc (the persistent fused solve with its work list and queue
counters in the library's static device scratch) against rom_step in the
same form: identical results bit for bit, on two calls in a row, the second
with a smaller batch (the scratch keeps the first call's list and counters),
and the batch limit of the scratch."""
import numpy as np
import pytest
import torch

import paper_2307_16894_amd as L
import workloads
from paper_2307_16894_amd.batch import RomBatch
from tests.conftest import rom_path

pytestmark = pytest.mark.gpu


def _pair(name, P, seed):
    mu = workloads.one_void_mu(seed, P)
    return mu, RomBatch(rom_path(name), mu), RomBatch(rom_path(name), mu)


def _outputs(rb):
    return (rb.status.clone(), rb.iters.clone(), rb.resnorm.clone(), rb.r(trial=True).clone(), rb.r().clone(),
            rb.history().clone(), rb.substeps().clone())


@pytest.mark.parametrize("name,contraction", [('onevoid_n20_m120', L.DT_F64), ('onevoid_n40_m400', L.DT_BF16)])
def test_noalloc_matches_rom_step(gpu, name, contraction):
    s = torch.cuda.current_stream().cuda_stream
    for call, (P, seed) in enumerate(((300, 5), (77, 6))):
        mu, ref, got = _pair(name, P, seed)
        paths = workloads.cyclic_paths(seed, P, 6, (0.02, 0.08))
        act = torch.from_numpy((np.arange(P) % 5 != 3).astype(np.int32)).cuda()
        for k in range(4):
            print(f"[gpu] no-alloc {name} call {call} P={P} step {k}", flush=True)
            Fb = torch.from_numpy(np.ascontiguousarray(paths[:, k])).cuda()
            o = L.rom_default_opts(mode=L.MODE_FUSED, contraction=contraction, grid_per_cu=2, max_substeps=4)
            if k == 3:
                o.active = act.data_ptr()  # a masked step: the list holds the active points only
            ref.step(Fb, o)
            L.rom_step_noalloc(got.h, P, Fb.data_ptr(), got.state.data_ptr(), o, got.status.data_ptr(),
                               got.iters.data_ptr(), got.resnorm.data_ptr(), s)
            L.rom_homogenized_stress_tangent(got.h, P, got.state.data_ptr(), got.Pbar.data_ptr(),
                                             got.Abar.data_ptr(), s)
            torch.cuda.synchronize()
            for a, b in zip(_outputs(ref), _outputs(got)):
                assert torch.equal(a, b), (call, k)
            assert torch.equal(ref.Pbar, got.Pbar) and torch.equal(ref.Abar, got.Abar), (call, k)
            assert (got.status == 0).all()
        ref.close()
        got.close()


def test_noalloc_batch_limit(gpu):
    mu, rb, _ = _pair('onevoid_n20_m120', 4, 1)
    big = L.NOALLOC_MAX_BATCH + 1
    Fb = torch.eye(2, dtype=torch.float64, device='cuda').reshape(1, 4).repeat(4, 1).contiguous()
    code = L.lib().rom_step_noalloc(rb.h, big, Fb.data_ptr(), rb.state.data_ptr(), None, rb.status.data_ptr(),
                                    rb.iters.data_ptr(), rb.resnorm.data_ptr(), None)
    assert code == L.ROM_ESCRATCH
    o = L.rom_default_opts(mode=L.MODE_PHASED)
    with pytest.raises(L.RomError) as e:
        L.rom_step_noalloc(rb.h, 4, Fb.data_ptr(), rb.state.data_ptr(), o, rb.status.data_ptr(),
                           rb.iters.data_ptr(), rb.resnorm.data_ptr(), None)
    assert e.value.code == L.ROM_EUNSUPPORTED
    rb.close()

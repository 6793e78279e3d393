"""POD on the GPU (rom_pod: method of snapshots, Sec. 3.1 and 3.2) against
the oracle's pod.pod on the same snapshots and weight: the eigenvalues of
the snapshot Gram matrix and the modes (each up to the eigensolver's sign),
with a sparse (CSR) weight and a diagonal one, at ragged sizes (tails of
every tile), and at the size of the n = 40 ROM's fluctuation POD (32316
dofs, 960 snapshots, 40 modes).  Tolerance: the modes are well separated
(eigenvalue gaps of 20 % or more), so rounding moves them by about 1e-16
times the conditioning of the Gram matrix relative to the gap; 1e-8 leaves
ample room.  A request beyond the numerical rank is an error on both sides."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import workloads
from oracle import pod as opod

import paper_2307_16894_amd as L
from paper_2307_16894_amd.offline import pod as gpod

pytestmark = pytest.mark.gpu


def snapshots(seed, nrow, ns, rank, decay, noise):
    g = workloads.rng(seed)
    U = np.linalg.qr(g.standard_normal((nrow, rank)))[0]
    V = np.linalg.qr(g.standard_normal((ns, rank)))[0]
    S = (U * decay ** np.arange(rank)) @ V.T
    return S + noise * g.standard_normal((nrow, ns))


def banded_spd(seed, nrow, bw):
    """A sparse SPD weight with the sparsity of a mass-plus-stiffness matrix."""
    g = workloads.rng(seed)
    diags = [g.uniform(-0.1, 0.1, nrow - k) for k in range(1, bw + 1)]
    A = sp.diags(diags, list(range(1, bw + 1)), shape=(nrow, nrow))
    A = A + A.T + sp.diags(np.full(nrow, 1.0 + 0.2 * bw))
    return A.tocsr()


def compare(S, M, n, tol=1e-8):
    ref, lam_o = opod.pod(S, M, n)
    modes, lam = gpod(S, M, n)
    torch.cuda.synchronize()
    modes, lam = modes.cpu().numpy(), lam.cpu().numpy()
    assert modes.shape == ref.shape
    assert np.abs(lam[:n] - lam_o[:n]).max() <= 1e-11 * lam_o[0]
    for k in range(n):
        sgn = np.sign(modes[:, k] @ ref[:, k])
        assert np.abs(sgn * modes[:, k] - ref[:, k]).max() <= tol * np.abs(ref[:, k]).max(), k
    return modes, lam


@pytest.mark.parametrize("weight", ["csr", "diag"])
def test_pod_ragged_sizes(gpu, weight):
    nrow, ns, n = 1001, 37, 5
    S = snapshots(3, nrow, ns, 12, 0.6, 1e-9)
    M = banded_spd(4, nrow, 3) if weight == "csr" else workloads.rng(5).uniform(0.5, 2.0, nrow)
    modes, _ = compare(S, M, n)
    Mm = M @ modes if weight == "csr" else M[:, None] * modes
    assert np.abs(modes.T @ Mm - np.eye(n)).max() < 1e-12


def test_pod_rank_limit(gpu):
    S = snapshots(6, 200, 20, 4, 0.5, 0.0)
    with pytest.raises(ValueError):
        opod.pod(S, np.ones(200), 6)
    with pytest.raises(L.RomError) as e:
        gpod(S, np.ones(200), 6)
    assert e.value.code == L.ROM_EINVAL


def test_pod_full_size(gpu):
    nrow, ns, n = 32316, 960, 40
    print("[gpu] pod full size", flush=True)
    S = snapshots(7, nrow, ns, 200, 0.8, 1e-12)
    M = banded_spd(8, nrow, 8)
    compare(S, M, n)

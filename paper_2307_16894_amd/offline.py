"""Offline stage on the GPU: POD of snapshot sets (Sec. 3.1, 3.2) through
rom_pod.  Argument marshalling only: the weight is uploaded as given (a
diagonal or the CSR arrays of a sparse matrix) and every arithmetic step
runs in the library."""
import numpy as np
import torch

from . import rom_pod, rom_pod_workspace


def pod(S, M, n, device='cuda:0'):
    """n leading POD modes of the snapshot columns of S (nrow, ns), orthonormal
    in the M product; M is a 1-D array of diagonal weights or a scipy sparse
    matrix.  Returns (modes (nrow, n) as a device tensor, eigenvalues of the
    snapshot Gram matrix descending (ns,))."""
    dev = torch.device(device)
    nrow, ns = S.shape
    St = torch.as_tensor(np.ascontiguousarray(np.asarray(S, dtype=np.float64).T), device=dev)
    keep = []
    if np.ndim(M) == 1:
        md = torch.as_tensor(np.asarray(M, dtype=np.float64), device=dev).contiguous()
        keep.append(md)
        weight = (md.data_ptr(), None, None, None)
    else:
        Mc = M.tocsr()
        ptr = torch.as_tensor(Mc.indptr.astype(np.int32), device=dev)
        col = torch.as_tensor(Mc.indices.astype(np.int32), device=dev)
        val = torch.as_tensor(Mc.data.astype(np.float64), device=dev)
        keep += [ptr, col, val]
        weight = (None, ptr.data_ptr(), col.data_ptr(), val.data_ptr())
    modes = torch.empty(n, nrow, dtype=torch.float64, device=dev)
    lam = torch.empty(ns, dtype=torch.float64, device=dev)
    wb = rom_pod_workspace(nrow, ns, n)
    work = torch.empty(wb, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    rom_pod(nrow, ns, St.data_ptr(), *weight, n, modes.data_ptr(), lam.data_ptr(), work.data_ptr(), wb,
            stream.cuda_stream)
    return modes.T, lam


def ecm(J, w, eps, m_max, device='cuda:0'):
    """Empirical cubature of the integrands J (R, nq) with full-rule weights w
    (nq,): returns (selected points in selection order, their weights,
    |res| / |b| after each iteration, rank of the integrand matrix, the
    library's return code)."""
    from . import rom_ecm, rom_ecm_workspace
    dev = torch.device(device)
    R, nq = J.shape
    Jd = torch.as_tensor(np.ascontiguousarray(J, dtype=np.float64), device=dev)
    wd = torch.as_tensor(np.ascontiguousarray(w, dtype=np.float64), device=dev)
    idx = torch.zeros(m_max, dtype=torch.int32, device=dev)
    wts = torch.zeros(m_max, dtype=torch.float64, device=dev)
    wb = rom_ecm_workspace(R, nq, m_max)
    work = torch.empty(wb, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    m, hist, rank, code = rom_ecm(R, nq, Jd.data_ptr(), wd.data_ptr(), eps, m_max, idx.data_ptr(), wts.data_ptr(),
                                  work.data_ptr(), wb, stream.cuda_stream, hist_cap=10 * m_max + 1)
    return idx[:m].cpu().numpy().astype(np.int64), wts[:m].cpu().numpy(), np.array(hist), rank, code

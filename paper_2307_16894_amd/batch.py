"""Torch-owned device buffers for a batch of macro points.

A thin convenience over the C ABI: allocates the state and the per-call
buffers as torch CUDA tensors and passes their pointers.  No arithmetic of
the method happens here.
"""
import torch

from . import (FIELD_ABAR, FIELD_FBAR_COMMITTED, FIELD_H_COMMITTED, FIELD_H_TRIAL, FIELD_MU_OK, FIELD_PBAR, FIELD_R_COMMITTED,
               FIELD_R_TRIAL, FIELD_SUBSTEPS, FIELD_TRANSFORM, rom_commit_trial, rom_default_opts, rom_free,
               rom_homogenized_stress_tangent,
               rom_info, rom_load_file, rom_shape_sensitivity, rom_state_bytes, rom_state_init, rom_state_offsets,
               rom_step)


class RomBatch:
    def __init__(self, rom_path, mu, device='cuda:0', stream=None):
        """mu: (P, n_mu) array-like of shape parameters."""
        self.device = torch.device(device)
        idx = self.device.index or 0
        self.h = rom_load_file(rom_path, idx)
        self.info = rom_info(self.h)
        self.mu = torch.as_tensor(mu, dtype=torch.float64).to(self.device).contiguous()
        self.P = int(self.mu.shape[0])
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = rom_state_bytes(self.h, self.P)
        self.state = torch.zeros(max(nbytes, 1), dtype=torch.uint8, device=self.device)
        self.offsets = rom_state_offsets(self.h, self.P)
        self.status = torch.zeros(self.P, dtype=torch.int32, device=self.device)
        self.iters = torch.zeros(self.P, dtype=torch.int32, device=self.device)
        self.resnorm = torch.zeros(self.P, dtype=torch.float64, device=self.device)
        self.Pbar = torch.zeros(self.P, 4, dtype=torch.float64, device=self.device)
        self.Abar = torch.zeros(self.P, 16, dtype=torch.float64, device=self.device)
        self.init_code = rom_state_init(self.h, self.P, self.mu.data_ptr(), self.state.data_ptr(),
                                        self.stream.cuda_stream)

    def close(self):
        if self.h is not None:
            rom_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, Fbar, opts=None, **kw):
        """Fbar: (P, 2, 2) or (P, 4) device tensor (float64)."""
        Fb = torch.as_tensor(Fbar, dtype=torch.float64, device=self.device).reshape(self.P, 4).contiguous()
        o = opts if opts is not None else rom_default_opts(**kw)
        rom_step(self.h, self.P, Fb.data_ptr(), self.state.data_ptr(), o, self.status.data_ptr(),
                 self.iters.data_ptr(), self.resnorm.data_ptr(), self.stream.cuda_stream)
        rom_homogenized_stress_tangent(self.h, self.P, self.state.data_ptr(), self.Pbar.data_ptr(),
                                       self.Abar.data_ptr(), self.stream.cuda_stream)
        self._keep = Fb  # keep alive until the stream has consumed it
        return self.status, self.iters, self.resnorm

    def commit_trial(self, Fbar):
        """Commit the trial state of the last step (made with commit = 0 to
        the same Fbar) at the points its status reports converged."""
        Fb = torch.as_tensor(Fbar, dtype=torch.float64, device=self.device).reshape(self.P, 4).contiguous()
        rom_commit_trial(self.h, self.P, Fb.data_ptr(), self.state.data_ptr(), self.status.data_ptr(),
                         self.stream.cuda_stream)
        self._keep_c = Fb

    def shape_sensitivity(self, Fbar):
        """dPbar/dmu (P, 4, n_mu) at the returned state of the last step, which
        must have been a trial step (commit = 0) to the same Fbar."""
        Fb = torch.as_tensor(Fbar, dtype=torch.float64, device=self.device).reshape(self.P, 4).contiguous()
        out = torch.empty(self.P, 4, self.info['n_mu'], dtype=torch.float64, device=self.device)
        rom_shape_sensitivity(self.h, self.P, Fb.data_ptr(), self.state.data_ptr(), out.data_ptr(),
                              self.stream.cuda_stream)
        self._keep_s = Fb
        return out

    def _view(self, field, shape, dtype=torch.float64):
        off = self.offsets[field]
        count = 1
        for s in shape:
            count *= s
        nb = count * torch.tensor([], dtype=dtype).element_size()
        return self.state[off:off + nb].view(dtype).view(*shape)

    def r(self, trial=False):
        n = self.info['n']
        return self._view(FIELD_R_TRIAL if trial else FIELD_R_COMMITTED, (self.P, n))

    def history(self, trial=False):
        m = self.info['m']
        return self._view(FIELD_H_TRIAL if trial else FIELD_H_COMMITTED, (self.P, 6, m))

    def fbar_committed(self):
        return self._view(FIELD_FBAR_COMMITTED, (self.P, 4))

    def transform(self):
        return self._view(FIELD_TRANSFORM, (self.P, 5, self.info['m']))

    def mu_ok(self):
        return self._view(FIELD_MU_OK, (self.P,), torch.int32)

    def substeps(self):
        """Record of the converged (sub-)steps of the last step, one int32 per
        point (bit k: a sub-step ended at (k+1)/32 of the load step)."""
        return self._view(FIELD_SUBSTEPS, (self.P,), torch.int32)

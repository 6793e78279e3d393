"""Two-scale (FE^2) driver over the reduced RVE solve (Sec. 4.2 setting).

A macro block of eight-node quadrilaterals whose 4 x elements Gauss points
are one batch of rom_step.  Per load step, Newton on the free macro
displacements: every iteration forms Fbar at the points, solves every RVE
from its committed state to that Fbar (a trial step, commit = 0) and returns
Pbar and Abar, assembles the residual, and either stops (the prescribed
values are in place and ||f_ext - f_int||_2 <= max(tol_rel ||f_ext||_2,
tol_abs) over the free dofs) or solves the banded macro system; a change of
the prescribed values enters that solve through the tangent (K_ff du_f =
r_f - K_fd du_d).  A converged step commits the RVE trial states of its last
iteration, which were solved at the final Fbar (rom_commit_trial: the state a
solve with commit = 1 from the same start would leave).  All arithmetic runs
in the library's kernels;
this module moves pointers and reads back the two norms, the RVE status
and the solve's info flag once per macro iteration.
"""
import numpy as np
import torch

from . import (MODE_FUSED, rom_default_opts, rom_fe2_compliance, rom_fe2_create, rom_fe2_free, rom_fe2_gradient,
               rom_fe2_info, rom_fe2_points, rom_fe2_residual, rom_fe2_solve, rom_fe2_traction)
from .batch import RomBatch

ST_OK, ST_MACRO_CAP, ST_RVE_FAILED, ST_SINGULAR = 0, 1, 2, 3


class Fe2Solver:
    def __init__(self, rom_path, mesh, shape_fn, fixed_dofs=None, device='cuda:0', mode=MODE_FUSED):
        """mesh: dict with X (nodes, 2), conn (elements, 8), bottom, top
        (edges, 3), width; shape_fn maps the (points, 2) reference positions
        of the Gauss points to (points, n_mu) shape parameters; fixed_dofs
        defaults to both components at the bottom nodes."""
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        if fixed_dofs is None:
            b = np.asarray(mesh['bottom'])
            fixed_dofs = np.sort(np.concatenate([2 * b, 2 * b + 1]))
        self.fixed = np.asarray(fixed_dofs, dtype=np.int32)
        self.h = rom_fe2_create(mesh['X'], mesh['conn'], self.fixed, mesh['top'], mesh['width'],
                                self.device.index or 0)
        self.info = rom_fe2_info(self.h)
        P, nd = self.info['points'], self.info['dofs']
        f64 = dict(dtype=torch.float64, device=self.device)
        self.Xg = torch.empty(P, 2, **f64)
        rom_fe2_points(self.h, self.Xg.data_ptr(), self.stream.cuda_stream)
        self.stream.synchronize()
        self.rb = RomBatch(rom_path, shape_fn(self.Xg.cpu().numpy()), device=device, stream=self.stream)
        self.mode = mode
        self.u = torch.zeros(nd, **f64)
        self.F = torch.empty(P, 4, **f64)
        self.fext = torch.empty(nd, **f64)
        self.res = torch.empty(nd, **f64)
        self.norms = torch.empty(2, **f64)
        self.C = torch.empty(1, **f64)
        self.dud = torch.zeros(max(self.fixed.size, 1), **f64)
        self.solve_info = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.applied = np.zeros(self.fixed.size)

    def close(self):
        if getattr(self, 'h', None) is not None:
            rom_fe2_free(self.h)
            self.h = None
        if getattr(self, 'rb', None) is not None:
            self.rb.close()
            self.rb = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _rve(self, commit, tol, max_iter):
        o = rom_default_opts(mode=self.mode, commit=commit, tol=tol, max_iter=max_iter)
        return self.rb.step(self.F, o)

    def load_step(self, Tbar, fixed_values=None, tol_rel=1e-9, tol_abs=1e-12, max_macro=20, rve_tol=1e-10,
                  rve_max_iter=25):
        """One load step; returns dict(status, macro_iters, rve_evals, C)."""
        s = self.stream.cuda_stream
        rom_fe2_traction(self.h, Tbar, self.fext.data_ptr(), s)
        target = self.applied if fixed_values is None else np.asarray(fixed_values, dtype=np.float64)
        status, evals, it = ST_MACRO_CAP, 0, 0
        for it in range(max_macro):
            rom_fe2_gradient(self.h, self.u.data_ptr(), self.F.data_ptr(), s)
            st, iters, _ = self._rve(0, rve_tol, rve_max_iter)
            rom_fe2_residual(self.h, self.rb.Pbar.data_ptr(), self.fext.data_ptr(), self.res.data_ptr(),
                             self.norms.data_ptr(), s)
            flags = torch.stack([self.norms[0], self.norms[1], (st != 0).any().double(), iters.sum().double()])
            rn, fn, bad, ev = flags.cpu().tolist()
            evals += int(ev)
            if bad:
                status = ST_RVE_FAILED
                break
            dud = target - self.applied
            if not dud.any() and rn <= max(tol_rel * fn, tol_abs):
                status = ST_OK
                break
            dptr = None
            if dud.any():
                self.dud[:dud.size].copy_(torch.from_numpy(dud))
                dptr = self.dud.data_ptr()
            rom_fe2_solve(self.h, self.rb.Abar.data_ptr(), self.res.data_ptr(), dptr, self.u.data_ptr(),
                          self.solve_info.data_ptr(), s)
            if int(self.solve_info.item()) != 0:
                status = ST_SINGULAR
                break
            self.applied = target.copy()
        if status == ST_OK:
            self.rb.commit_trial(self.F)
        rom_fe2_compliance(self.h, Tbar, self.u.data_ptr(), self.C.data_ptr(), s)
        return dict(status=status, macro_iters=it + 1, rve_evals=evals, C=float(self.C.item()))

    def run(self, Tbars, fixed_values=None, **kw):
        """Load steps with peak tractions Tbars[k] (prescribed values
        fixed_values[k] if given); stops at the first step that fails."""
        out = []
        for k, T in enumerate(Tbars):
            r = self.load_step(T, None if fixed_values is None else fixed_values[k], **kw)
            r['u'] = self.u.cpu().numpy().copy()
            out.append(r)
            if r['status'] != ST_OK:
                break
        return out

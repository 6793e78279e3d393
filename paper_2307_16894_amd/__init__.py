"""Python binding of libpodecm (the HIP hyper-reduced RVE solve).

Argument marshalling only: every step of the solve runs in the library's
HIP kernels.  Device buffers are torch tensors (torch is used for device
memory and streams); the functions take and return raw pointers through the
C ABI declared in include/podecm.h, under the same names.

The library must be built (``python -m paper_2307_16894_amd.build``); there is
no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, 'libpodecm.so')

ROM_OK = 0
ROM_EINVAL = -1
ROM_EFORMAT = -2
ROM_EVERSION = -3
ROM_EHIP = -4
ROM_EINVAL_MU = -5
ROM_EUNSUPPORTED = -6
ROM_ESCRATCH = -7
NOALLOC_MAX_BATCH = 32768

ST_CONVERGED = 0
ST_MAXITER = 1
ST_NONFINITE = 2
ST_FALLBACK = 3
ST_BADMU = 4
WARM_PREV, WARM_MLP = 0, 1

DT_F64, DT_F32, DT_BF16 = 0, 1, 2
MODE_STAGED, MODE_FUSED, MODE_PHASED = 0, 1, 2

FIELD_R_COMMITTED, FIELD_R_TRIAL, FIELD_H_COMMITTED, FIELD_H_TRIAL = 0, 1, 2, 3
FIELD_TRANSFORM, FIELD_PBAR, FIELD_ABAR, FIELD_MU_OK = 4, 5, 6, 7
FIELD_FBAR_COMMITTED, FIELD_R_GUESS, FIELD_SUBSTEPS = 8, 9, 10
NFIELDS = 11

EXPORTS = ['rom_default_opts', 'rom_load', 'rom_load_file', 'rom_free', 'rom_info', 'rom_state_bytes',
           'rom_state_offsets', 'rom_state_init', 'rom_step', 'rom_step_noalloc', 'rom_homogenized_stress_tangent',
           'rom_commit_trial', 'rom_shape_sensitivity',
           'rom_timing_enable', 'rom_timing_read', 'rom_mlp_create', 'rom_mlp_free', 'rom_mlp_param_count',
           'rom_mlp_set_params', 'rom_mlp_get_params', 'rom_mlp_set_scaling', 'rom_mlp_forward',
           'rom_mlp_gradients', 'rom_mlp_train_step', 'rom_mlp_infer', 'rom_mlp_train_epoch', 'rom_mlp_fit_scaling',
           'rom_mlp_save', 'rom_mlp_load', 'rom_features', 'rom_warm_samples', 'rom_path_gather', 'rom_path_advance',
           'rom_fe2_create', 'rom_fe2_free', 'rom_fe2_info', 'rom_fe2_points', 'rom_fe2_gradient', 'rom_fe2_traction',
           'rom_fe2_residual', 'rom_fe2_solve', 'rom_fe2_compliance', 'rom_pod_workspace', 'rom_pod',
           'rom_ecm_workspace', 'rom_ecm']


_CODES = {ROM_EINVAL: 'ROM_EINVAL (bad argument)', ROM_EFORMAT: 'ROM_EFORMAT (malformed artifact)',
          ROM_EVERSION: 'ROM_EVERSION (artifact version)', ROM_EHIP: 'ROM_EHIP (HIP runtime call failed)',
          ROM_EINVAL_MU: 'ROM_EINVAL_MU (shape parameters give det F_mu <= 0)',
          ROM_EUNSUPPORTED: 'ROM_EUNSUPPORTED (option combination not built)',
          ROM_ESCRATCH: f'ROM_ESCRATCH (batch above the static scratch limit of {NOALLOC_MAX_BATCH} points)'}


class RomError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what} failed with code {code}: {_CODES.get(code, 'unknown')}")
        self.code = code


class rom_opts(ctypes.Structure):
    _fields_ = [('tol', ctypes.c_double), ('max_iter', ctypes.c_int32), ('fixed_iters', ctypes.c_int32),
                ('commit', ctypes.c_int32), ('contraction', ctypes.c_int32), ('mode', ctypes.c_int32),
                ('warm_start', ctypes.c_int32), ('split', ctypes.c_int32), ('grid_per_cu', ctypes.c_int32),
                ('max_substeps', ctypes.c_int32), ('phased_evals', ctypes.c_int32), ('phased_early', ctypes.c_int32),
                ('abar_f64', ctypes.c_int32),
                ('mlp', ctypes.c_void_p), ('active', ctypes.c_void_p)]


_lib = None


def _hip_runtimes():
    """Paths of the HIP runtime libraries mapped into this process."""
    try:
        with open('/proc/self/maps') as fh:
            return sorted({ln.split()[-1] for ln in fh if 'libamdhip64' in ln})
    except OSError:
        return []


def lib():
    """Load libpodecm.so; raises if it has not been built.

    The library takes device pointers and hipStream_t handles from PyTorch, so
    it must bind to the HIP runtime PyTorch uses: torch is imported first (its
    runtime then satisfies the library's dependency), and a process holding
    two HIP runtimes is rejected."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2307_16894_amd.build")
        import torch  # noqa: F401  (loads the HIP runtime the library must share)
        L = ctypes.CDLL(LIB_PATH)
        rts = _hip_runtimes()
        if len(rts) > 1:
            raise RuntimeError(f"two HIP runtimes are loaded ({rts}); import torch before loading libpodecm")
        vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        L.rom_default_opts.argtypes = [ctypes.POINTER(rom_opts)]
        L.rom_load.argtypes = [vp, sz, ctypes.c_int, ctypes.POINTER(vp)]
        L.rom_load_file.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(vp)]
        L.rom_free.argtypes = [vp]
        L.rom_info.argtypes = [vp] + [ctypes.POINTER(i32)] * 4
        L.rom_state_bytes.argtypes = [vp, i32, ctypes.POINTER(sz)]
        L.rom_state_offsets.argtypes = [vp, i32, ctypes.POINTER(sz)]
        L.rom_state_init.argtypes = [vp, i32, vp, vp, vp]
        L.rom_step.argtypes = [vp, i32, vp, vp, ctypes.POINTER(rom_opts), vp, vp, vp, vp]
        L.rom_step_noalloc.argtypes = [vp, i32, vp, vp, ctypes.POINTER(rom_opts), vp, vp, vp, vp]
        L.rom_shape_sensitivity.argtypes = [vp, i32, vp, vp, vp, vp]
        L.rom_homogenized_stress_tangent.argtypes = [vp, i32, vp, vp, vp, vp]
        L.rom_commit_trial.argtypes = [vp, i32, vp, vp, vp, vp]
        L.rom_timing_enable.argtypes = [vp, ctypes.c_int]
        L.rom_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        fp = ctypes.POINTER(ctypes.c_float)
        L.rom_mlp_create.argtypes = [i32, i32, i32, i32, ctypes.c_int, ctypes.POINTER(vp)]
        L.rom_mlp_free.argtypes = [vp]
        L.rom_mlp_param_count.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.rom_mlp_set_params.argtypes = [vp, fp, ctypes.c_int64]
        L.rom_mlp_get_params.argtypes = [vp, fp, ctypes.c_int64]
        L.rom_mlp_set_scaling.argtypes = [vp, fp, fp, fp, fp]
        L.rom_mlp_forward.argtypes = [vp, i32, vp, vp, i32, vp]
        L.rom_mlp_gradients.argtypes = [vp, i32, vp, vp, i32, vp, vp, vp]
        L.rom_mlp_train_step.argtypes = [vp, i32, vp, vp, ctypes.c_float, i32, vp, vp]
        L.rom_features.argtypes = [vp, i32, vp, vp, vp, vp]
        L.rom_mlp_infer.argtypes = [vp, i32, vp, vp, i32, vp]
        L.rom_mlp_train_epoch.argtypes = [vp, i32, vp, vp, vp, i32, ctypes.c_float, i32, vp, vp]
        L.rom_mlp_fit_scaling.argtypes = [vp, i32, vp, vp, vp]
        L.rom_mlp_save.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
        L.rom_mlp_load.argtypes = [vp, ctypes.c_size_t, i32, ctypes.c_int, ctypes.POINTER(vp)]
        L.rom_warm_samples.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.rom_path_gather.argtypes = [i32, vp, i32, vp, vp, vp, vp, vp]
        L.rom_path_advance.argtypes = [i32, vp, vp, vp]
        dbl = ctypes.c_double
        L.rom_fe2_create.argtypes = [i32, i32, vp, vp, i32, vp, i32, vp, dbl, ctypes.c_int, ctypes.POINTER(vp)]
        L.rom_fe2_free.argtypes = [vp]
        L.rom_fe2_info.argtypes = [vp] + [ctypes.POINTER(i32)] * 4
        L.rom_fe2_points.argtypes = [vp, vp, vp]
        L.rom_fe2_gradient.argtypes = [vp, vp, vp, vp]
        L.rom_fe2_traction.argtypes = [vp, dbl, vp, vp]
        L.rom_fe2_residual.argtypes = [vp, vp, vp, vp, vp, vp]
        L.rom_fe2_solve.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.rom_fe2_compliance.argtypes = [vp, dbl, vp, vp, vp]
        L.rom_pod_workspace.argtypes = [i32, i32, i32, ctypes.POINTER(sz)]
        L.rom_pod.argtypes = [i32, i32, vp, vp, vp, vp, vp, i32, vp, vp, vp, sz, vp]
        L.rom_ecm_workspace.argtypes = [i32, i32, i32, ctypes.POINTER(sz)]
        L.rom_ecm.argtypes = [i32, i32, vp, vp, dbl, i32, vp, vp, ctypes.POINTER(i32), ctypes.POINTER(dbl), i32,
                              ctypes.POINTER(i32), ctypes.POINTER(i32), vp, sz, vp]
        for name in EXPORTS:
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(code, what):
    if code != ROM_OK:
        raise RomError(code, what)
    return code


def rom_default_opts(**kw):
    o = rom_opts()
    _check(lib().rom_default_opts(ctypes.byref(o)), 'rom_default_opts')
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def rom_load(blob, device=0):
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(bytes(blob), len(blob))
    _check(lib().rom_load(buf, len(blob), device, ctypes.byref(h)), 'rom_load')
    return h


def rom_load_file(path, device=0):
    h = ctypes.c_void_p()
    _check(lib().rom_load_file(os.fsencode(path), device, ctypes.byref(h)), 'rom_load_file')
    return h


def rom_free(h):
    _check(lib().rom_free(h), 'rom_free')


def rom_info(h):
    v = [ctypes.c_int32() for _ in range(4)]
    _check(lib().rom_info(h, *[ctypes.byref(x) for x in v]), 'rom_info')
    return dict(n=v[0].value, m=v[1].value, c=v[2].value, n_mu=v[3].value)


def rom_state_bytes(h, batch):
    s = ctypes.c_size_t()
    _check(lib().rom_state_bytes(h, batch, ctypes.byref(s)), 'rom_state_bytes')
    return s.value


def rom_state_offsets(h, batch):
    arr = (ctypes.c_size_t * NFIELDS)()
    _check(lib().rom_state_offsets(h, batch, arr), 'rom_state_offsets')
    return list(arr)


def rom_state_init(h, batch, mu_ptr, state_ptr, stream):
    """Returns ROM_OK or ROM_EINVAL_MU (points with det F_mu <= 0 are flagged)."""
    code = lib().rom_state_init(h, batch, mu_ptr, state_ptr, stream)
    if code not in (ROM_OK, ROM_EINVAL_MU):
        raise RomError(code, 'rom_state_init')
    return code


def rom_step(h, batch, Fbar_ptr, state_ptr, opts, status_ptr, iters_ptr, res_ptr, stream):
    return _check(lib().rom_step(h, batch, Fbar_ptr, state_ptr, ctypes.byref(opts) if opts is not None else None,
                                 status_ptr, iters_ptr, res_ptr, stream), 'rom_step')


def rom_step_noalloc(h, batch, Fbar_ptr, state_ptr, opts, status_ptr, iters_ptr, res_ptr, stream):
    return _check(lib().rom_step_noalloc(h, batch, Fbar_ptr, state_ptr,
                                         ctypes.byref(opts) if opts is not None else None,
                                         status_ptr, iters_ptr, res_ptr, stream), 'rom_step_noalloc')


def rom_commit_trial(h, batch, Fbar_ptr, state_ptr, status_ptr, stream):
    return _check(lib().rom_commit_trial(h, batch, Fbar_ptr, state_ptr, status_ptr, stream), 'rom_commit_trial')


def rom_homogenized_stress_tangent(h, batch, state_ptr, Pbar_ptr, Abar_ptr, stream):
    return _check(lib().rom_homogenized_stress_tangent(h, batch, state_ptr, Pbar_ptr, Abar_ptr, stream),
                  'rom_homogenized_stress_tangent')


def rom_shape_sensitivity(h, batch, Fbar_ptr, state_ptr, dPdmu_ptr, stream):
    return _check(lib().rom_shape_sensitivity(h, batch, Fbar_ptr, state_ptr, dPdmu_ptr, stream),
                  'rom_shape_sensitivity')


def rom_timing_enable(h, enable=True):
    _check(lib().rom_timing_enable(h, int(bool(enable))), 'rom_timing_enable')


def rom_timing_read(h):
    """(summed milliseconds, launches) of the dominant kernel since enable."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().rom_timing_read(h, ctypes.byref(ms), ctypes.byref(n)), 'rom_timing_read')
    return ms.value, n.value


def _f32(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def rom_mlp_create(n_in, width, n_out, max_batch, device=0):
    h = ctypes.c_void_p()
    _check(lib().rom_mlp_create(n_in, width, n_out, max_batch, device, ctypes.byref(h)), 'rom_mlp_create')
    return h


def rom_mlp_free(m):
    _check(lib().rom_mlp_free(m), 'rom_mlp_free')


def rom_mlp_param_count(m):
    c = ctypes.c_int64()
    _check(lib().rom_mlp_param_count(m, ctypes.byref(c)), 'rom_mlp_param_count')
    return c.value


def rom_mlp_set_params(m, params):
    a, ptr = _f32(params)
    _check(lib().rom_mlp_set_params(m, ptr, a.size), 'rom_mlp_set_params')


def rom_mlp_get_params(m):
    import numpy as np
    out = np.zeros(rom_mlp_param_count(m), dtype=np.float32)
    _check(lib().rom_mlp_get_params(m, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), out.size),
           'rom_mlp_get_params')
    return out


def rom_mlp_set_scaling(m, x_mean, x_std, y_mean, y_std):
    arrs = [_f32(v) for v in (x_mean, x_std, y_mean, y_std)]
    _check(lib().rom_mlp_set_scaling(m, *[p for _, p in arrs]), 'rom_mlp_set_scaling')


def rom_mlp_forward(m, batch, X_ptr, Y_ptr, precision, stream):
    _check(lib().rom_mlp_forward(m, batch, X_ptr, Y_ptr, precision, stream), 'rom_mlp_forward')


def rom_mlp_gradients(m, batch, X_ptr, Y_ptr, precision, grads_ptr, loss_ptr, stream):
    _check(lib().rom_mlp_gradients(m, batch, X_ptr, Y_ptr, precision, grads_ptr, loss_ptr, stream),
           'rom_mlp_gradients')


def rom_mlp_train_step(m, batch, X_ptr, Y_ptr, lr, precision, loss_ptr, stream):
    _check(lib().rom_mlp_train_step(m, batch, X_ptr, Y_ptr, ctypes.c_float(lr), precision, loss_ptr, stream),
           'rom_mlp_train_step')


def rom_features(h, batch, Fbar_ptr, state_ptr, X_ptr, stream):
    _check(lib().rom_features(h, batch, Fbar_ptr, state_ptr, X_ptr, stream), 'rom_features')


def rom_mlp_infer(m, batch, X_ptr, Y_ptr, precision, stream):
    _check(lib().rom_mlp_infer(m, batch, X_ptr, Y_ptr, precision, stream), 'rom_mlp_infer')


def rom_mlp_train_epoch(m, N, X_ptr, Y_ptr, order_ptr, batch, lr, precision, loss_sum_ptr, stream):
    _check(lib().rom_mlp_train_epoch(m, N, X_ptr, Y_ptr, order_ptr, batch, ctypes.c_float(lr), precision,
                                     loss_sum_ptr, stream), 'rom_mlp_train_epoch')


def rom_mlp_fit_scaling(m, N, X_ptr, Y_ptr, stream):
    _check(lib().rom_mlp_fit_scaling(m, N, X_ptr, Y_ptr, stream), 'rom_mlp_fit_scaling')


def rom_mlp_save(m):
    need = ctypes.c_size_t()
    _check(lib().rom_mlp_save(m, None, 0, ctypes.byref(need)), 'rom_mlp_save')
    buf = ctypes.create_string_buffer(need.value)
    _check(lib().rom_mlp_save(m, buf, need.value, ctypes.byref(need)), 'rom_mlp_save')
    return buf.raw


def rom_mlp_load(blob, max_batch, device=0):
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(bytes(blob), len(blob))
    _check(lib().rom_mlp_load(buf, len(blob), max_batch, device, ctypes.byref(h)), 'rom_mlp_load')
    return h


def rom_warm_samples(h, batch, state_ptr, X_feat_ptr, r_before_ptr, status_ptr, X_out_ptr, Y_out_ptr, count_ptr,
                     stream):
    _check(lib().rom_warm_samples(h, batch, state_ptr, X_feat_ptr, r_before_ptr, status_ptr, X_out_ptr, Y_out_ptr,
                                  count_ptr, stream), 'rom_warm_samples')


def rom_path_gather(batch, paths_ptr, max_steps, nsteps_ptr, step_ptr, Fbar_ptr, active_ptr, stream):
    _check(lib().rom_path_gather(batch, paths_ptr, max_steps, nsteps_ptr, step_ptr, Fbar_ptr, active_ptr, stream),
           'rom_path_gather')


def rom_path_advance(batch, active_ptr, step_ptr, stream):
    _check(lib().rom_path_advance(batch, active_ptr, step_ptr, stream), 'rom_path_advance')


def rom_fused_tiles(n):
    """16-column blocks of the fused contraction for n modes (f and C ride in columns n .. n+4)."""
    return (n + 5 + 15) // 16


def rom_fe2_create(X, conn, fixed_dofs, top, width, device=0):
    """Macro mesh on the device (host numpy inputs are copied)."""
    import numpy as np
    X = np.ascontiguousarray(X, dtype=np.float64)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    fixed = np.ascontiguousarray(fixed_dofs, dtype=np.int32)
    top = np.ascontiguousarray(top, dtype=np.int32).reshape(-1, 3)
    h = ctypes.c_void_p()
    _check(lib().rom_fe2_create(X.shape[0], conn.shape[0], X.ctypes.data, conn.ctypes.data, fixed.size,
                                fixed.ctypes.data, top.shape[0], top.ctypes.data, float(width), device,
                                ctypes.byref(h)), 'rom_fe2_create')
    return h


def rom_fe2_free(h):
    _check(lib().rom_fe2_free(h), 'rom_fe2_free')


def rom_fe2_info(h):
    v = [ctypes.c_int32() for _ in range(4)]
    _check(lib().rom_fe2_info(h, *[ctypes.byref(x) for x in v]), 'rom_fe2_info')
    return dict(dofs=v[0].value, free_dofs=v[1].value, points=v[2].value, kl=v[3].value)


def rom_fe2_points(h, Xg_ptr, stream):
    _check(lib().rom_fe2_points(h, Xg_ptr, stream), 'rom_fe2_points')


def rom_fe2_gradient(h, u_ptr, Fbar_ptr, stream):
    _check(lib().rom_fe2_gradient(h, u_ptr, Fbar_ptr, stream), 'rom_fe2_gradient')


def rom_fe2_traction(h, Tbar, fext_ptr, stream):
    _check(lib().rom_fe2_traction(h, float(Tbar), fext_ptr, stream), 'rom_fe2_traction')


def rom_fe2_residual(h, Pbar_ptr, fext_ptr, res_ptr, norms_ptr, stream):
    _check(lib().rom_fe2_residual(h, Pbar_ptr, fext_ptr, res_ptr, norms_ptr, stream), 'rom_fe2_residual')


def rom_fe2_solve(h, Abar_ptr, res_ptr, dud_ptr, u_ptr, info_ptr, stream):
    _check(lib().rom_fe2_solve(h, Abar_ptr, res_ptr, dud_ptr, u_ptr, info_ptr, stream), 'rom_fe2_solve')


def rom_fe2_compliance(h, Tbar, u_ptr, C_ptr, stream):
    _check(lib().rom_fe2_compliance(h, float(Tbar), u_ptr, C_ptr, stream), 'rom_fe2_compliance')


def rom_pod_workspace(nrow, ns, n):
    b = ctypes.c_size_t()
    _check(lib().rom_pod_workspace(nrow, ns, n, ctypes.byref(b)), 'rom_pod_workspace')
    return b.value


def rom_pod(nrow, ns, S_ptr, mdiag_ptr, csr_ptr, csr_col, csr_val, n, modes_ptr, lambda_ptr, work_ptr, work_bytes,
            stream):
    _check(lib().rom_pod(nrow, ns, S_ptr, mdiag_ptr, csr_ptr, csr_col, csr_val, n, modes_ptr, lambda_ptr, work_ptr,
                         work_bytes, stream), 'rom_pod')


def rom_ecm_workspace(R, nq, m_max):
    b = ctypes.c_size_t()
    _check(lib().rom_ecm_workspace(R, nq, m_max, ctypes.byref(b)), 'rom_ecm_workspace')
    return b.value


def rom_ecm(R, nq, J_ptr, w_ptr, eps, m_max, idx_ptr, weights_ptr, work_ptr, work_bytes, stream, hist_cap=0):
    """Returns (count, history list, rank, code); code ROM_EUNSUPPORTED is not raised (partial result)."""
    m = ctypes.c_int32()
    hl = ctypes.c_int32()
    rk = ctypes.c_int32()
    hist = (ctypes.c_double * max(hist_cap, 1))()
    code = lib().rom_ecm(R, nq, J_ptr, w_ptr, float(eps), m_max, idx_ptr, weights_ptr, ctypes.byref(m), hist,
                         hist_cap, ctypes.byref(hl), ctypes.byref(rk), work_ptr, work_bytes, stream)
    if code not in (ROM_OK, ROM_EUNSUPPORTED):
        _check(code, 'rom_ecm')
    return m.value, list(hist[:hl.value]), rk.value, code

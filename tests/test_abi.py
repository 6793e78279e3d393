"""The C-ABI library loads and exports every symbol the header declares, and
rom_load rejects malformed artifacts before touching a device (no GPU
needed)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2307_16894_amd as L
from tests.conftest import ROOT, rom_path

HEADER = os.path.join(ROOT, 'include', 'podecm.h')


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r'^int (rom_\w+)\(', txt, flags=re.M)))


def test_header_and_binding_agree():
    assert declared() == sorted(L.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    out = subprocess.run(['nm', '-D', '--defined-only', L.LIB_PATH], capture_output=True, text=True, check=True)
    syms = set(re.findall(r' T (rom_\w+)', out.stdout))
    for name in declared():
        assert name in syms, name
        assert getattr(lib, name) is not None


def test_default_opts():
    o = L.rom_default_opts()
    assert o.tol == 1e-8 and o.max_iter == 15 and o.commit == 1 and o.fixed_iters == 0
    assert o.contraction == L.DT_F64


def _load_code(blob):
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(bytes(blob), max(len(blob), 1))
    return L.lib().rom_load(buf, len(blob), 0, ctypes.byref(h))


def test_rom_load_rejects_malformed_artifacts():
    good = open(rom_path('onevoid_n20_m120'), 'rb').read()
    assert _load_code(b'') == L.ROM_EFORMAT
    assert _load_code(b'NOTAROM!' + good[8:]) == L.ROM_EFORMAT
    assert _load_code(good[:-8]) == L.ROM_EFORMAT  # truncated
    bad = bytearray(good)
    bad[8:12] = np.array([3], dtype='<u4').tobytes()
    assert _load_code(bad) == L.ROM_EVERSION
    bad[8:12] = np.array([2], dtype='<u4').tobytes()  # two phases: the phase array is missing
    assert _load_code(bad) == L.ROM_EFORMAT
    bad = bytearray(good)
    bad[256:264] = np.array([-1.0]).tobytes()  # a non-positive ECM weight
    assert _load_code(bad) == L.ROM_EFORMAT
    bad = bytearray(good)
    bad[264 + 8 * 5:264 + 8 * 6] = np.array([np.nan]).tobytes()
    assert _load_code(bad) == L.ROM_EFORMAT
    bad = bytearray(good)
    bad[12:16] = np.array([1000], dtype='<u4').tobytes()  # n beyond the supported maximum
    assert _load_code(bad) == L.ROM_EFORMAT


def test_null_arguments():
    lib = L.lib()
    assert lib.rom_load(None, 0, 0, None) == L.ROM_EINVAL
    assert lib.rom_state_bytes(None, 4, None) == L.ROM_EINVAL
    assert lib.rom_step(None, 4, None, None, None, None, None, None, None) == L.ROM_EINVAL
    assert lib.rom_free(None) == L.ROM_EINVAL


def test_rom_load_two_phase_artifacts():
    """Version 2 (a second phase and the phase of every ECM point): the
    loader rejects a phase other than 0 or 1 and an invalid second material
    before touching a device."""
    good = open(rom_path('coatvoid_n20_m120'), 'rb').read()
    assert np.frombuffer(good[8:12], dtype='<u4')[0] == 2
    bad = bytearray(good)
    bad[-8:] = np.array([2], dtype='<i8').tobytes()  # phase of the last point
    assert _load_code(bad) == L.ROM_EFORMAT
    bad = bytearray(good)
    bad[88:96] = np.array([-1.0]).tobytes()  # E of the second phase
    assert _load_code(bad) == L.ROM_EFORMAT
    assert _load_code(good[:-8]) == L.ROM_EFORMAT  # phases truncated


def test_offline_and_two_scale_argument_checks():
    """Argument validation of the two-scale and offline entry points happens
    on the host, before any device memory is touched."""
    import ctypes
    lib = L.lib()
    X = np.zeros((4, 2))
    conn = np.array([[0, 1, 2, 3, 0, 1, 2, 3]], dtype=np.int32)
    top = np.array([[3, 2, 2]], dtype=np.int32)
    h = ctypes.c_void_p()

    def create(conn_, fixed_, top_=top):
        return lib.rom_fe2_create(4, conn_.shape[0], X.ctypes.data, conn_.ctypes.data, fixed_.size,
                                  fixed_.ctypes.data, top_.shape[0], top_.ctypes.data, 2.0, 0, ctypes.byref(h))
    bad_conn = conn.copy()
    bad_conn[0, 5] = 9                                   # node index out of range
    assert create(bad_conn, np.array([0, 1], dtype=np.int32)) == L.ROM_EINVAL
    assert create(conn, np.array([0, 0], dtype=np.int32)) == L.ROM_EINVAL       # a dof fixed twice
    assert create(conn, np.arange(8, dtype=np.int32)) == L.ROM_EINVAL           # no free dof
    assert create(conn, np.array([0, 9], dtype=np.int32)) == L.ROM_EINVAL       # dof out of range
    assert create(conn, np.array([0], dtype=np.int32), np.array([[3, 2, 7]], dtype=np.int32)) == L.ROM_EINVAL
    b = ctypes.c_size_t()
    assert lib.rom_pod_workspace(10, 4, 5, ctypes.byref(b)) == L.ROM_EINVAL     # more modes than snapshots
    assert lib.rom_pod_workspace(10, 4, 2, ctypes.byref(b)) == L.ROM_OK and b.value > 0
    assert lib.rom_ecm_workspace(5, 100, 2000, ctypes.byref(b)) == L.ROM_EINVAL  # point budget above 1024
    assert lib.rom_ecm_workspace(5, 100, 50, ctypes.byref(b)) == L.ROM_OK and b.value > 0
    dummy = ctypes.c_void_p(1)
    # neither or both weights given
    assert lib.rom_pod(10, 4, dummy, None, None, None, None, 2, dummy, dummy, dummy, 1 << 30, None) == L.ROM_EINVAL

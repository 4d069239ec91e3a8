"""C ABI checks that need no GPU: the library loads, exports every function the
header declares, and its host-side validation returns the documented
status codes before anything touches a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mudiff.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1409_8186_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1409_8186_amd.build import build
        build()
    return _lib.load()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mudiff_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_five_calls():
    names = header_functions()
    for core in ("mudiff_tables", "mudiff_matvec", "mudiff_gmres", "mudiff_farfield", "mudiff_grad"):
        assert core in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1409_8186_amd import _lib
    names = header_functions()
    assert names, "no declarations parsed"
    for n in names:
        assert hasattr(lib, n), n
    # the binding declares exactly the header's functions
    assert sorted(_lib.SIGNATURES) == names


def _sizes(lib, disk_off, n_modes, flags=0):
    d = np.ascontiguousarray(disk_off, np.int64)
    n = np.ascontiguousarray(n_modes, np.int32)
    return lib.mudiff_tables_workspace_size(len(d) - 1, d.ctypes.data, n.ctypes.data, flags)


def test_workspace_size_queries(lib):
    assert _sizes(lib, [0, 4], [15] * 4) > 0
    assert _sizes(lib, [0, 2, 5], [3, 4, 5, 6, 7]) > 0
    assert _sizes(lib, [0, 4], [15, 15, -1, 15]) == 0          # N_p < 0
    assert _sizes(lib, [0, 4], [15, 15, 201, 15]) == 0         # N_p > MUDIFF_MAX_NP
    assert _sizes(lib, [1, 4], [3] * 4) == 0                   # disk_off[0] != 0
    assert _sizes(lib, [0, 2, 2], [3] * 2) == 0                # empty instance
    # monotone in the number of modes
    assert _sizes(lib, [0, 4], [12] * 4) > _sizes(lib, [0, 4], [8] * 4)
    assert _sizes(lib, [0, 4], [30] * 4) > _sizes(lib, [0, 4], [20] * 4)
    # the circulant form adds sum_b L_b M_b^2 complex values: L_min = 2 (N' + N'') + 1
    # = 41 is raised to 48 = 2^4 3 (at most 1.2 L_min: fast transforms) ...
    base = _sizes(lib, [0, 40], [10] * 40)
    circ = _sizes(lib, [0, 40], [10] * 40, flags=1)
    assert circ - base >= 48 * 40 * 40 * 16
    assert circ - base < 48 * 40 * 40 * 16 + 48 * 16 + 40 * 39 // 2 + 8 * 256
    # ... while L_min = 2 (10 + 8) + 1 = 37 stays (48 would add 30% to the products)
    base = _sizes(lib, [0, 40], [10] + [8] * 39)
    circ = _sizes(lib, [0, 40], [10] + [8] * 39, flags=1)
    assert circ - base >= 37 * 40 * 40 * 16
    assert circ - base < 37 * 40 * 40 * 16 + 37 * 16 + 40 * 39 // 2 + 8 * 256
    assert _sizes(lib, [0, 4], [3] * 4, flags=2) == 0         # unknown flag


def _tables(lib, centers, radii, n_modes, k, ws_bytes=1 << 40, ws_ptr=256, flags=0):
    c = np.ascontiguousarray(centers, np.float64)
    r = np.ascontiguousarray(radii, np.float64)
    n = np.ascontiguousarray(n_modes, np.int32)
    kk = np.ascontiguousarray([k], np.float64)
    d = np.ascontiguousarray([0, len(r)], np.int64)
    h = ctypes.c_void_p()
    st = lib.mudiff_tables(1, d.ctypes.data, c.ctypes.data, r.ctypes.data, n.ctypes.data,
                           kk.ctypes.data, ctypes.c_void_p(ws_ptr), ws_bytes, flags, None,
                           ctypes.byref(h))
    return st, lib.mudiff_last_error().decode()


def test_validation_status_codes(lib):
    """Errors are detected on the host before any device work: the fake
    workspace pointer below is never dereferenced."""
    c = [[0, 0], [3, 0], [0, 3]]
    st, msg = _tables(lib, c, [1, 1, 1], [4, 4, 4], -1.0)
    assert st == 1 and "k" in msg                               # k <= 0
    st, _ = _tables(lib, c, [1, 1, 1], [4, 4, 4], float("nan"))
    assert st == 1
    st, _ = _tables(lib, c, [1, 0, 1], [4, 4, 4], 2.0)
    assert st == 1                                              # a <= 0
    st, _ = _tables(lib, [[0, 0], [float("inf"), 0], [0, 3]], [1, 1, 1], [4, 4, 4], 2.0)
    assert st == 1                                              # non-finite center
    st, msg = _tables(lib, c, [1, 1, 1], [4, -2, 4], 2.0)
    assert st == 1
    st, msg = _tables(lib, [[0, 0], [2, 0], [0, 3]], [1, 1, 1], [4, 4, 4], 2.0)
    assert st == 2 and "overlap" in msg                         # touching disks
    st, msg = _tables(lib, [[0, 0], [1.5, 0], [0, 3]], [1, 1, 1], [4, 4, 4], 2.0)
    assert st == 2                                              # intersecting disks
    st, msg = _tables(lib, c, [1, 1, 1], [4, 4, 4], 2.0, ws_bytes=1024)
    assert st == 3 and "workspace" in msg                       # too small


def test_null_handle_rejected(lib):
    st = lib.mudiff_matvec(None, 1, ctypes.c_void_p(256), ctypes.c_void_p(512), 1, None, 0, None)
    assert st == 1
    st = lib.mudiff_gmres(None, 1, None, None, None, 30, 1e-8, 10, 0, None, 0, None, None, None,
                          None, None)
    assert st == 1
    assert lib.mudiff_matvec_workspace_size(None, 1) == 0
    assert lib.mudiff_gmres_workspace_size(None, 1, 30, 0) == 0


def test_probe_validation(lib):
    rate = ctypes.c_double(-1.0)
    buf = ctypes.create_string_buffer(512)
    # unknown kind and NULL pointers are rejected before any device work
    assert lib.mudiff_probe(7, 0, buf, 512, ctypes.byref(rate), None) == 1
    assert lib.mudiff_probe(0, 0, None, 0, ctypes.byref(rate), None) == 1
    assert lib.mudiff_probe(0, 0, buf, 512, None, None) == 1
    assert lib.mudiff_probe(2, 8, buf, 512, ctypes.byref(rate), None) == 1   # copy < 16 bytes
    assert rate.value == -1.0
    assert lib.mudiff_probe_workspace_size(9, 0) == 0


def test_time_reversal_validation(lib):
    buf = ctypes.create_string_buffer(4096)
    sweeps = ctypes.c_int32(7)
    assert lib.mudiff_tro(0, 4, buf, buf, None) == 1
    assert lib.mudiff_tro(4, 4, None, buf, None) == 1
    assert lib.mudiff_tro_eigh_workspace_size(0, 3) == 0
    need = lib.mudiff_tro_eigh_workspace_size(8, 8)
    assert need >= 8 * 8 * 16
    assert lib.mudiff_tro_eigh(8, 8, buf, buf, buf, 0, 1e-13, buf, 4096, ctypes.byref(sweeps), None) == 1
    assert lib.mudiff_tro_eigh(8, 8, buf, buf, buf, 10, 0.0, buf, 4096, ctypes.byref(sweeps), None) == 1
    assert lib.mudiff_tro_eigh(8, 8, buf, buf, buf, 10, 1e-13, buf, need - 1, ctypes.byref(sweeps), None) == 3
    assert lib.mudiff_tro_eigh(8, 8, buf, buf, buf, 10, 1e-13, buf, 4096, None, None) == 1
    assert sweeps.value == 7
    assert lib.mudiff_herglotz(0, buf, 1, buf, ctypes.c_double(1.0), ctypes.c_double(0.1), 4, buf, buf, None) == 1
    assert lib.mudiff_herglotz(4, buf, 1, buf, ctypes.c_double(-1.0), ctypes.c_double(0.1), 4, buf, buf, None) == 1
    assert lib.mudiff_herglotz(4, buf, 1, buf, ctypes.c_double(1.0), ctypes.c_double(0.1), 4, None, buf, None) == 1


def test_set_operator_validation(lib):
    w = (ctypes.c_double * 10)()
    assert lib.mudiff_set_operator(None, w, w, w, None, 0, None) == 1
    assert lib.mudiff_operator_workspace_size(None) == 0
    k = (ctypes.c_double * 4)(1.0, 1.0, 1.0, 1.0)
    assert lib.mudiff_set_penetrable(None, k, None, w, 4096, None) == 1
    assert lib.mudiff_interior_field(None, 1, w, w, 0, 1, w, w, w, 4096, None) == 1
    assert lib.mudiff_interior_workspace_size(None, 1) == 0
    assert lib.mudiff_rhs_point(None, 1, w, w, 0, None) == 1
    assert lib.mudiff_set_formulation(None, 1, 0.5, 0.0, 1.0, w, 4096, None) == 1


def test_circulant_validation(lib):
    """The circulant flag: unknown flags and orders beyond the form's limit are
    rejected on the host; the pair classification and mode calls reject a
    NULL handle and bad modes."""
    c = [[0, 0], [3, 0], [0, 3]]
    st, msg = _tables(lib, c, [1, 1, 1], [4, 4, 4], 2.0, flags=4)
    assert st == 1 and "flag" in msg
    st, msg = _tables(lib, c, [1, 1, 1], [4, 32, 4], 2.0, flags=1)
    assert st == 1 and "31" in msg                              # beyond the MFMA tile range
    assert _sizes(lib, [0, 3], [4, 32, 4], flags=1) == 0
    assert _sizes(lib, [0, 3], [4, 31, 4], flags=1) > _sizes(lib, [0, 3], [4, 31, 4])
    far, near = ctypes.c_int64(-1), ctypes.c_int64(-1)
    assert lib.mudiff_circulant_info(None, ctypes.byref(far), ctypes.byref(near), None) == 1
    assert lib.mudiff_set_circulant(None, 8, 1) == 1

"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point that include/tfl.h declares, and rejects bad arguments in
the host logic before any device call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tfl.h")
LIB = os.environ.get("TFL_LIB") or os.path.join(ROOT, "paper_2305_13419_amd", "libtfl.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(tfl_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.fail("libtfl.so is not built (run __graft_entry__.build())")
    from paper_2305_13419_amd import _lib
    return _lib


def test_every_declared_symbol_is_exported(L):
    names = declared()
    assert len(names) >= 18
    lib = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares every one of them, under the same name
    bound = set(L.SIGNATURES) | set(L.OPTIONAL_SIGNATURES)
    assert set(names) <= bound, set(names) - bound


def good_config(L):
    c = L.tfl_config()
    c.nx, c.ny, c.nz = 20, 10, 8
    c.dx = c.dy = c.dz = 1e-8
    c.dt = 1e-18
    c.theta = 1.0
    c.dtype = L.TFL_F64
    c.pml_order, c.pml_scale, c.kappa_max, c.alpha_max = 3.0, 1.0, 1.0, 0.0
    return c


def create(L, c):
    h = ctypes.c_void_p()
    rc = L.lib().tfl_create(ctypes.byref(c), ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("field,value", [("nx", 0), ("dy", 0.0), ("dt", -1.0), ("theta", 0.3), ("theta", 1.2),
                                         ("dtype", 7), ("dz", float("nan"))])
def test_create_rejects_bad_config(L, field, value):
    c = good_config(L)
    setattr(c, field, value)
    rc, h = create(L, c)
    assert rc == L.TFL_E_INVAL
    assert not h.value
    assert L.lib().tfl_last_error(None)


def test_create_rejects_bad_pml(L):
    c = good_config(L)
    c.bc[0] = L.TFL_CPML
    c.pml_lo[0], c.pml_hi[0] = 15, 10  # more than nx
    assert create(L, c)[0] == L.TFL_E_INVAL
    c.pml_lo[0], c.pml_hi[0] = 4, 4
    c.kappa_max = 0.5
    assert create(L, c)[0] == L.TFL_E_INVAL


def test_buffer_sizes_and_call_order(L):
    c = good_config(L)
    c.bc[0] = L.TFL_CPML
    c.pml_lo[0], c.pml_hi[0] = 4, 3
    c.bc[2] = L.TFL_CPML
    c.pml_lo[2], c.pml_hi[2] = 2, 2
    rc, h = create(L, c)
    assert rc == 0
    ws, sc, st = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    assert L.lib().tfl_buffer_sizes(h, ctypes.byref(ws), ctypes.byref(sc), ctypes.byref(st)) == 0
    # tables (6 n per CPML axis) and 4 slab arrays per CPML axis, each 256-byte padded, FP64
    pad = lambda n: (n + 31) // 32 * 32  # noqa: E731
    expect = pad(6 * 20) + pad(6 * 8) + pad(4 * 8 * 10 * 7) + pad(4 * 4 * 10 * 20)
    assert ws.value == 8 * expect
    assert st.value == 9 * ((20 * 10 * 8 * 8 + 255) // 256 * 256) + ws.value
    assert sc.value >= 8 * 5 * 1024
    # stepping, binding materials and energy before binding are state errors
    assert L.lib().tfl_step(h, 1, None) == L.TFL_E_STATE
    assert L.lib().tfl_energy(h, None, None, None) == L.TFL_E_STATE
    assert L.lib().tfl_bind_materials(h, None, None, None, None) == L.TFL_E_STATE
    assert b"workspace" in L.lib().tfl_last_error(h)
    # null and misaligned state pointers
    arr = (ctypes.c_void_p * 3)(0, 0, 0)
    pp = ctypes.cast(arr, L.PP)
    assert L.lib().tfl_bind_state(h, pp, pp, pp) == L.TFL_E_INVAL
    arr2 = (ctypes.c_void_p * 3)(4096 + 8, 8192, 16384)
    pp2 = ctypes.cast(arr2, L.PP)
    assert L.lib().tfl_bind_state(h, pp2, pp2, pp2) == L.TFL_E_INVAL
    assert b"aligned" in L.lib().tfl_last_error(h)
    # sources and probes are validated on the host
    s = L.tfl_source()
    s.comp, s.waveform, s.amplitude = 1, L.TFL_WAVE_SIN, 1.0
    for q, v in enumerate((0, 1, 0, 10, 0, 8)):
        s.box[q] = v
    i = ctypes.c_int()
    assert L.lib().tfl_add_source(h, ctypes.byref(s), ctypes.byref(i)) == 0 and i.value == 0
    s.box[1] = 21
    assert L.lib().tfl_add_source(h, ctypes.byref(s), ctypes.byref(i)) == L.TFL_E_INVAL
    s.box[1] = 1
    s.waveform = L.TFL_WAVE_GAUSS
    s.tw = 0.0
    assert L.lib().tfl_add_source(h, ctypes.byref(s), ctypes.byref(i)) == L.TFL_E_INVAL
    p = L.tfl_probe()
    p.comp = 3
    assert L.lib().tfl_add_probe(h, ctypes.byref(p), ctypes.byref(i)) == L.TFL_E_INVAL
    p.comp = 0
    for q, v in enumerate((0, 1, 0, 1, 0, 1)):
        p.box[q] = v
    p.capacity = 10
    assert L.lib().tfl_add_probe(h, ctypes.byref(p), ctypes.byref(i)) == L.TFL_E_INVAL  # no series buffer
    p.capacity = 0
    p.nfreq = 17
    assert L.lib().tfl_add_probe(h, ctypes.byref(p), ctypes.byref(i)) == L.TFL_E_INVAL
    assert L.lib().tfl_set_step(h, -1) == L.TFL_E_INVAL
    n = ctypes.c_int64()
    assert L.lib().tfl_set_step(h, 5) == 0
    assert L.lib().tfl_get_step(h, ctypes.byref(n)) == 0 and n.value == 5
    assert L.lib().tfl_set_nonfinite_check(h, -1) == L.TFL_E_INVAL
    assert L.lib().tfl_set_nonfinite_check(h, 16) == 0 and L.lib().tfl_set_nonfinite_check(h, 0) == 0
    assert L.lib().tfl_set_nonfinite_check(None, 1) == L.TFL_E_INVAL
    assert L.lib().tfl_destroy(h) == 0


def test_fused_buffer_layout(L):
    """9 padded fields (E, H, Js); with a CPML axis also a second set of that axis's four auxiliary
    variables (two H-side, two E-side; y slabs: nz x (lo + hi) x nx each), padded to 256 bytes."""
    c = good_config(L)
    rc, h = create(L, c)
    assert rc == 0
    b = ctypes.c_size_t()
    field = (20 * 10 * 8 * 8 + 255) // 256 * 256
    assert L.lib().tfl_fused_buffer_bytes(h, ctypes.byref(b)) == 0
    assert b.value == 9 * field
    assert L.lib().tfl_bind_fused_buffer(h, ctypes.c_void_p(0x1001)) == L.TFL_E_INVAL  # misaligned
    assert L.lib().tfl_bind_fused_buffer(h, None) == 0
    L.lib().tfl_destroy(h)
    c.bc[1] = L.TFL_CPML
    c.pml_lo[1], c.pml_hi[1] = 2, 3
    rc, h = create(L, c)
    assert rc == 0
    assert L.lib().tfl_fused_buffer_bytes(h, ctypes.byref(b)) == 0
    assert b.value == 9 * field + (4 * 8 * 5 * 20 * 8 + 255) // 256 * 256
    assert L.lib().tfl_bind_fused_buffer(h, ctypes.c_void_p(0x1010)) == L.TFL_E_INVAL
    assert L.lib().tfl_bind_fused_buffer(h, None) == 0
    L.lib().tfl_destroy(h)
    # all three axes: x slabs nz x ny x P, y slabs nz x P x nx, z slabs P x ny x nx (P = lo + hi)
    c.bc[0], c.bc[2] = L.TFL_CPML, L.TFL_CPML
    c.pml_lo[0], c.pml_hi[0] = 3, 2
    c.pml_lo[2], c.pml_hi[2] = 1, 2
    rc, h = create(L, c)
    assert rc == 0
    assert L.lib().tfl_fused_buffer_bytes(h, ctypes.byref(b)) == 0
    r256 = lambda n: (n + 255) // 256 * 256
    assert b.value == 9 * field + r256(4 * 8 * 10 * 5 * 8) + r256(4 * 8 * 5 * 20 * 8) + r256(4 * 3 * 10 * 20 * 8)
    L.lib().tfl_destroy(h)


def test_edge_class_buffer_size_and_call_order(L):
    """Class buffer: three padded uint16 arrays, the table of TFL_MAX_EDGE_CLASSES four-value
    entries and the staging area (65536 cell materials of three values, one uint64 tuple per
    class); binding needs bound maps and an aligned buffer; NULL unbinds."""
    c = good_config(L)
    rc, h = create(L, c)
    assert rc == 0
    b = ctypes.c_size_t()
    assert L.lib().tfl_edge_class_bytes(h, ctypes.byref(b)) == 0
    r256 = lambda n: (n + 255) // 256 * 256  # noqa: E731
    n = 20 * 10 * 8
    assert b.value == (3 * r256(2 * n) + r256(L.TFL_MAX_EDGE_CLASSES * 4 * 8) + r256(65536 * 3 * 8)
                       + r256(L.TFL_MAX_EDGE_CLASSES * 8))
    k = ctypes.c_int(-1)
    assert L.lib().tfl_bind_edge_classes(h, ctypes.c_void_p(0x1001), ctypes.byref(k), None) == L.TFL_E_INVAL
    assert L.lib().tfl_bind_edge_classes(h, ctypes.c_void_p(0x1000), ctypes.byref(k), None) == L.TFL_E_STATE
    assert b"materials not bound" in L.lib().tfl_last_error(h)
    assert L.lib().tfl_bind_edge_classes(h, None, ctypes.byref(k), None) == 0 and k.value == 0
    L.lib().tfl_destroy(h)

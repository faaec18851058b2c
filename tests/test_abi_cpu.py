"""Host-side checks of the C-ABI library (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ebbx.h")
LIB = os.path.join(ROOT, "paper_1506_07577_amd", "libebbx.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ebbx_[a-z0-9_A-Z]+)\s*\(", text)))


def test_header_declares_the_named_calls():
    names = declared_functions()
    for n in ["ebbx_relation_create", "ebbx_field_bind", "ebbx_keyfield_bind", "ebbx_fem_forces",
              "ebbx_fem_Kmul", "ebbx_implicit_step"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libebbx.so not built")
def test_library_loads_and_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.ebbx_version.restype = ctypes.c_int32
    assert lib.ebbx_version() >= 100
    lib.ebbx_last_error.restype = ctypes.c_char_p
    assert lib.ebbx_last_error() == b""


@pytest.mark.skipif(not os.path.exists(LIB), reason="libebbx.so not built")
def test_host_validation_without_gpu():
    """Argument checks that fail before any device work."""
    lib = ctypes.CDLL(LIB)
    lib.ebbx_relation_create.argtypes = [ctypes.c_char_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p)]
    lib.ebbx_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    assert lib.ebbx_relation_create(b"bad", -5, ctypes.byref(h)) == -1
    assert h.value is None
    assert b"out of range" in lib.ebbx_last_error()
    assert lib.ebbx_relation_create(b"r", 10, ctypes.byref(h)) == 0
    lib.ebbx_field_bind.argtypes = [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int, ctypes.c_int32,
                                    ctypes.c_void_p]
    # misaligned pointer for a float64 field
    assert lib.ebbx_field_bind(h, b"x", 1, 3, ctypes.c_void_p(0x1003)) == -4
    assert lib.ebbx_field_bind(h, b"x", 1, 0, ctypes.c_void_p(0x1000)) == -3
    lib.ebbx_relation_destroy.argtypes = [ctypes.c_void_p]
    assert lib.ebbx_relation_destroy(h) == 0
    assert lib.ebbx_relation_destroy(h) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libebbx.so not built")
def test_invalid_handles_rejected_without_gpu():
    """The assembled-stiffness and spring-mass entry points reject unknown handles on the host."""
    lib = ctypes.CDLL(LIB)
    lib.ebbx_last_error.restype = ctypes.c_char_p
    bogus = ctypes.c_void_p(0x1234)
    n = ctypes.c_int64(-7)
    for name, args in [("ebbx_fem_assemble", (bogus, None, None)),
                       ("ebbx_fem_spmv", (bogus, None, None, 0, None)),
                       ("ebbx_fem_edge_count", (bogus, ctypes.byref(n))),
                       ("ebbx_fem_edges_get", (bogus, None, None, None, None)),
                       ("ebbx_springs_forces", (bogus, None, None, 0, None)),
                       ("ebbx_springs_apply", (bogus, None, ctypes.c_double(1e-4), None, None, None, None)),
                       ("ebbx_springs_kinetic_energy", (bogus, None, None, None, None)),
                       ("ebbx_springs_run", (bogus, None, ctypes.c_double(1e-4), 1, None, None, None, None)),
                       ("ebbx_springs_rest", (bogus, None, None)),
                       ("ebbx_springs_destroy", (bogus,))]:
        fn = getattr(lib, name)
        assert fn(*args) == -1, name
        assert b"invalid" in lib.ebbx_last_error(), name
    assert n.value == -7
    lib.ebbx_springs_create.argtypes = [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_char_p, ctypes.c_void_p,
                                        ctypes.c_char_p, ctypes.c_double, ctypes.POINTER(ctypes.c_void_p)]
    out = ctypes.c_void_p()
    assert lib.ebbx_springs_create(bogus, b"tail", b"head", bogus, b"X", 1.0, ctypes.byref(out)) == -1
    assert out.value is None


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1506_07577_amd import ebbx
    monkeypatch.setattr(ebbx, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(ebbx, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        ebbx.lib()

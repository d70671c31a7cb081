"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "feasm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"^\s*typedef[^;]*;", "", text, flags=re.M)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


@pytest.fixture(scope="module")
def lib():
    from paper_2012_00585_amd import _lib

    return _lib.load()


def test_header_declares_the_four_calls():
    names = _declared_functions()
    for f in ("pattern_build", "assemble_csr", "assemble_crac", "reassemble_values"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2012_00585_amd import _lib

    names = _declared_functions()
    assert set(names) == set(_lib.SIGNATURES), (names, sorted(_lib.SIGNATURES))
    for n in names:
        assert hasattr(lib, n), n


def test_set_allocator_needs_both_callbacks(lib):
    """Host-only: one callback without the other is rejected; none restores
    the default."""
    from paper_2012_00585_amd import _lib

    alloc = _lib.ALLOC_FN(lambda nbytes, stream, ctx: None)
    release = _lib.RELEASE_FN(lambda ptr, stream, ctx: None)
    assert lib.set_allocator(alloc, _lib.RELEASE_FN(), None) == -1
    assert b"both" in lib.last_error()
    assert lib.set_allocator(_lib.ALLOC_FN(), release, None) == -1
    assert lib.set_allocator(_lib.ALLOC_FN(), _lib.RELEASE_FN(), None) == 0


def _build(lib, conn, E, k, d, nn, flags):
    h = ctypes.c_void_p()
    rc = lib.pattern_build(conn, E, k, d, nn, flags, None, ctypes.byref(h))
    return rc, h


def test_pattern_build_rejects_bad_arguments(lib):
    from paper_2012_00585_amd._lib import STATUS_NAMES

    dummy = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    cases = [
        ((None, 4, 4, 1, 9, 1), "FEASM_EINVAL"),
        ((dummy, 0, 4, 1, 9, 1), "FEASM_EINVAL"),
        ((dummy, 4, 0, 1, 9, 1), "FEASM_EINVAL"),
        ((dummy, 4, 4, 0, 9, 1), "FEASM_EINVAL"),
        ((dummy, 4, 4, 1, 0, 1), "FEASM_EINVAL"),
        ((dummy, 4, 4, 1, 9, 0), "FEASM_EINVAL"),      # neither CSR nor CRAC
        ((dummy, 4, 4, 1, 9, 64), "FEASM_EINVAL"),     # unknown flag
        ((dummy, 2 ** 30, 4, 1, 9, 1), "FEASM_EOVERFLOW"),
        ((dummy, 4, 4, 3, 2 ** 30, 1), "FEASM_EOVERFLOW"),
        ((dummy, 4, 100, 50, 9, 1), "FEASM_ELIMIT"),
    ]
    for args, want in cases:
        rc, h = _build(lib, *args)
        assert STATUS_NAMES[rc] == want, (args, rc)
        assert not h.value
        assert lib.last_error()
    h = ctypes.c_void_p()
    assert lib.pattern_build(dummy, 4, 4, 1, 9, 1, None, None) == -1


def test_generate_ke_rejects_bad_arguments(lib):
    """Argument checks of the workload generator, all taken before any device
    call (an empty batch also returns before launching)."""
    from paper_2012_00585_amd._lib import STATUS_NAMES

    d = ctypes.c_void_p(0x1000)  # never dereferenced
    cases = [
        ((0, 4, 4, 1, 0, None), "FEASM_EINVAL"),   # null output
        ((2, 4, 4, 1, 0, d), "FEASM_EINVAL"),      # unknown recipe
        ((1, -1, 24, 1, 0, d), "FEASM_EINVAL"),    # negative count
        ((1, 4, 0, 1, 0, d), "FEASM_EINVAL"),      # empty matrices
        ((0, 4, 4, 1, -5, d), "FEASM_EINVAL"),     # negative element offset
        ((1, 4, 91, 1, 0, d), "FEASM_ELIMIT"),     # 91*92*8 bytes > 64 KiB
        ((0, 0, 4, 1, 0, d), "FEASM_OK"),          # nothing to generate
        ((1, 0, 24, 1, 0, d), "FEASM_OK"),
    ]
    for args, want in cases:
        rc = lib.generate_ke(*args, None)
        assert STATUS_NAMES[rc] == want, (args, rc)
        if want != "FEASM_OK":
            assert lib.last_error()


def test_numeric_calls_reject_null_handle(lib):
    d = ctypes.c_void_p(0x1000)
    assert lib.assemble_csr(None, d, d, 0, None) == -1
    assert b"null handle" in lib.last_error()
    assert lib.assemble_crac(None, d, d, 0, None) == -1
    assert lib.reassemble_values(None, 0, d, d, 0, None) == -1
    assert lib.pattern_info(None, None, None, None, None) == -1
    assert lib.pattern_arrays(None, None, None, None, None) == -1
    assert lib.pattern_colouring(None, None, None, None) == -1
    assert lib.pattern_tune(None, 1, 0) == -1
    assert lib.spmv_csr(None, d, d, d, None) == -1
    assert b"spmv_csr: null handle" in lib.last_error()
    assert lib.spmv_crac(None, d, d, d, None) == -1
    assert lib.hex8_element_matrices(None, d, d, d, None) == -1
    assert lib.assemble_hex8(None, 1, d, d, d, 0, None) == -1
    assert b"assemble_hex8: null handle" in lib.last_error()
    lib.pattern_free(None)  # ignored


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2012_00585_amd import _lib

    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()

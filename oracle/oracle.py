"""Python access to the serial CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg.  The device library never imports it.

The functions mirror the C routines one to one and take/return numpy
arrays.  Indices are 0-based int64; values are float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11"]
# FEASM_ORACLE_SANITIZE=1: a separate build under AddressSanitizer and
# UndefinedBehaviorSanitizer (the process must preload gcc's libasan and
# libubsan); the tests run the oracle's pins against it.
SANITIZE = os.environ.get("FEASM_ORACLE_SANITIZE", "") == "1"
SAN_CFLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=all"]
_LIB = os.path.join(_HERE, "liboracle_san.so" if SANITIZE else "liboracle.so")


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` with gcc into ``liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        flags = [*CFLAGS, *SAN_CFLAGS] if SANITIZE else CFLAGS
        subprocess.check_call(["gcc", *flags, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I32 = ctypes.c_int32
        L.orc_dof_map.argtypes = [P, I32, I32, P]
        L.orc_dof_runs.argtypes = [P, I32, P]
        L.orc_dof_runs.restype = I32
        L.orc_pattern_pairs.argtypes = [I64, P, P, I64, I64, P, ctypes.POINTER(P)]
        L.orc_pattern_pairs.restype = I64
        L.orc_pattern.argtypes = [P, I64, I32, I32, I64, P, ctypes.POINTER(P)]
        L.orc_pattern.restype = I64
        L.orc_csr_find.argtypes = [P, P, I64, I64]
        L.orc_csr_find.restype = I64
        L.orc_crac_count.argtypes = [P, P, I64]
        L.orc_crac_count.restype = I64
        L.orc_crac_fill.argtypes = [P, P, I64, I64, P, P]
        L.orc_crac_find.argtypes = [P, P, I64, I64]
        L.orc_crac_find.restype = I64
        L.orc_assemble.argtypes = [P, I64, I32, I32, P, P, P, I64, P, P]
        L.orc_assemble.restype = ctypes.c_int
        L.orc_assemble_pairs.argtypes = [I64, P, P, P, P, P, I64, P]
        L.orc_assemble_pairs.restype = ctypes.c_int
        L.orc_greedy_colour.argtypes = [P, I64, I32, I64, P]
        L.orc_greedy_colour.restype = I32
        L.orc_colouring_valid.argtypes = [P, I64, I32, I64, P, I32]
        L.orc_colouring_valid.restype = ctypes.c_int
        L.orc_rows.argtypes = [P, I64, I32, I32, I64, P, I64, P, I64, P, P, P, P]
        L.orc_rows.restype = ctypes.c_int
        L.orc_spmv_csr.argtypes = [P, P, I64, P, P, P, P]
        L.orc_spmv_crac.argtypes = [P, P, I64, P, P, P]
        L.orc_hex8_stiffness.argtypes = [P, I32, P, P, P]
        L.orc_hex8_stiffness.restype = ctypes.c_int
        L.orc_hex8_matrices.argtypes = [P, I64, P, I32, P, P, P]
        L.orc_hex8_matrices.restype = ctypes.c_int
        L.orc_free.argtypes = [P]
        _lib = L
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def dof_map(conn_e, d):
    conn_e = _c(conn_e, np.int32)
    D = np.empty(conn_e.size * d, dtype=np.int64)
    lib().orc_dof_map(_p(conn_e), conn_e.size, d, _p(D))
    return D


def dof_runs(D):
    D = _c(D, np.int64)
    pairs = np.empty(2 * max(D.size, 1), dtype=np.int64)
    nr = lib().orc_dof_runs(_p(D), D.size, _p(pairs))
    return pairs[: 2 * nr].copy()


def _take(ptr, nnz):
    buf = (ctypes.c_int64 * max(nnz, 1)).from_address(ptr.value)
    out = np.frombuffer(buf, dtype=np.int64, count=nnz).copy()
    lib().orc_free(ptr)
    return out


def pattern_pairs(rows, cols, n_rows, n_cols):
    rows = _c(rows, np.int64)
    cols = _c(cols, np.int64)
    row_ptr = np.empty(n_rows + 1, dtype=np.int64)
    ptr = ctypes.c_void_p()
    nnz = lib().orc_pattern_pairs(rows.size, _p(rows), _p(cols), n_rows, n_cols, _p(row_ptr),
                                  ctypes.byref(ptr))
    if nnz < 0:
        raise ValueError(f"orc_pattern_pairs failed: {nnz}")
    return row_ptr, _take(ptr, nnz)


def pattern(conn, d, n_nodes):
    """CSR pattern (row_ptr, col_idx) of the union of element cliques."""
    conn = _c(conn, np.int32)
    E, k = conn.shape
    row_ptr = np.empty(d * n_nodes + 1, dtype=np.int64)
    ptr = ctypes.c_void_p()
    nnz = lib().orc_pattern(_p(conn), E, k, d, n_nodes, _p(row_ptr), ctypes.byref(ptr))
    if nnz < 0:
        raise ValueError(f"orc_pattern failed: {nnz}")
    return row_ptr, _take(ptr, nnz)


def csr_find(row_ptr, col_idx, i, j):
    return lib().orc_csr_find(_p(row_ptr), _p(col_idx), int(i), int(j))


def crac(row_ptr, col_idx, n_cols):
    """CRAC arrays (crac_row_ptr, ca) built from a CSR pattern."""
    row_ptr = _c(row_ptr, np.int64)
    col_idx = _c(col_idx, np.int64)
    n_rows = row_ptr.size - 1
    B = lib().orc_crac_count(_p(row_ptr), _p(col_idx), n_rows)
    crp = np.empty(n_rows + 1, dtype=np.int64)
    ca = np.empty(2 * B + 2, dtype=np.int64)
    lib().orc_crac_fill(_p(row_ptr), _p(col_idx), n_rows, n_cols, _p(crp), _p(ca))
    return crp, ca


def crac_find(crac_row_ptr, ca, i, j):
    return lib().orc_crac_find(_p(crac_row_ptr), _p(ca), int(i), int(j))


def assemble(conn, d, ke, row_ptr, col_idx, with_abs=True):
    """Sequential assembly; returns (values, abssum or None)."""
    conn = _c(conn, np.int32)
    ke = _c(ke, np.float64)
    E, k = conn.shape
    n = k * d
    assert ke.shape == (E, n, n)
    n_rows = row_ptr.size - 1
    nnz = int(row_ptr[-1])
    values = np.empty(nnz, dtype=np.float64)
    absv = np.empty(nnz, dtype=np.float64) if with_abs else None
    rc = lib().orc_assemble(_p(conn), E, k, d, _p(ke), _p(row_ptr), _p(col_idx), n_rows,
                            _p(values), _p(absv) if with_abs else None)
    if rc != 0:
        raise ValueError(f"orc_assemble failed: {rc}")
    return values, absv


def assemble_pairs(rows, cols, vals, row_ptr, col_idx):
    rows = _c(rows, np.int64)
    cols = _c(cols, np.int64)
    vals = _c(vals, np.float64)
    values = np.empty(int(row_ptr[-1]), dtype=np.float64)
    rc = lib().orc_assemble_pairs(rows.size, _p(rows), _p(cols), _p(vals), _p(row_ptr),
                                  _p(col_idx), row_ptr.size - 1, _p(values))
    if rc != 0:
        raise ValueError(f"orc_assemble_pairs failed: {rc}")
    return values


def greedy_colour(conn, n_nodes):
    conn = _c(conn, np.int32)
    E, k = conn.shape
    colour = np.empty(E, dtype=np.int32)
    nc = lib().orc_greedy_colour(_p(conn), E, k, n_nodes, _p(colour))
    if nc < 0:
        raise ValueError(f"orc_greedy_colour failed: {nc}")
    return colour, nc


def colouring_valid(conn, n_nodes, colour, n_colours):
    conn = _c(conn, np.int32)
    colour = _c(colour, np.int32)
    E, k = conn.shape
    return bool(lib().orc_colouring_valid(_p(conn), E, k, n_nodes, _p(colour), int(n_colours)) == 1)


def rows(conn, d, n_nodes, ke, req_rows, cap=4096):
    """Selected rows: list of (cols, vals, abssum) per requested DOF row."""
    conn = _c(conn, np.int32)
    ke = _c(ke, np.float64)
    req = _c(req_rows, np.int64)
    E, k = conn.shape
    ln = np.empty(req.size, dtype=np.int64)
    cols = np.empty((req.size, cap), dtype=np.int64)
    vals = np.empty((req.size, cap), dtype=np.float64)
    absv = np.empty((req.size, cap), dtype=np.float64)
    rc = lib().orc_rows(_p(conn), E, k, d, n_nodes, _p(ke), req.size, _p(req), cap, _p(ln),
                        _p(cols), _p(vals), _p(absv))
    if rc != 0:
        raise ValueError(f"orc_rows failed: {rc}")
    return [(cols[q, : ln[q]].copy(), vals[q, : ln[q]].copy(), absv[q, : ln[q]].copy())
            for q in range(req.size)]


def spmv_csr(row_ptr, col_idx, values, x, with_abs=True):
    """y = G x through CSR, summed in column order; returns (y, yabs or None)."""
    row_ptr = _c(row_ptr, np.int64)
    col_idx = _c(col_idx, np.int64)
    values = _c(values, np.float64)
    x = _c(x, np.float64)
    n_rows = row_ptr.size - 1
    y = np.empty(n_rows, dtype=np.float64)
    ya = np.empty(n_rows, dtype=np.float64) if with_abs else None
    lib().orc_spmv_csr(_p(row_ptr), _p(col_idx), n_rows, _p(values), _p(x), _p(y),
                       _p(ya) if with_abs else None)
    return y, ya


def spmv_crac(crac_row_ptr, ca, values, x):
    """y = G x through the CRAC runs, summed in column order."""
    crac_row_ptr = _c(crac_row_ptr, np.int64)
    ca = _c(ca, np.int64)
    values = _c(values, np.float64)
    x = _c(x, np.float64)
    n_rows = crac_row_ptr.size - 1
    y = np.empty(n_rows, dtype=np.float64)
    lib().orc_spmv_crac(_p(crac_row_ptr), _p(ca), n_rows, _p(values), _p(x), _p(y))
    return y


def hex8_stiffness(x, d, mat):
    """Stiffness of one 8-node hexahedron: x [8, 3], d 1 or 3, mat (kappa,)
    or (lambda, mu).  Returns (K [8d, 8d], kabs)."""
    x = _c(x, np.float64)
    mat = _c(mat, np.float64)
    n = 8 * d
    K = np.empty((n, n))
    A = np.empty((n, n))
    rc = lib().orc_hex8_stiffness(_p(x), d, _p(mat), _p(K), _p(A))
    if rc != 0:
        raise ValueError(f"orc_hex8_stiffness failed: {rc}")
    return K, A


def hex8_matrices(conn, coords, d, mat, with_abs=True):
    """Element matrices [E, 8d, 8d] of a hexahedral mesh (and their term bounds)."""
    conn = _c(conn, np.int32)
    coords = _c(coords, np.float64)
    mat = _c(mat, np.float64)
    E = conn.shape[0]
    n = 8 * d
    K = np.empty((E, n, n))
    A = np.empty((E, n, n)) if with_abs else None
    rc = lib().orc_hex8_matrices(_p(conn), E, _p(coords), d, _p(mat), _p(K),
                                 _p(A) if with_abs else None)
    if rc != 0:
        raise ValueError(f"orc_hex8_matrices failed: {rc}")
    return K, A

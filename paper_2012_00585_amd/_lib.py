"""ctypes declarations of libfeasm.so (the C ABI in include/feasm.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfeasm.so")

FEASM_OK = 0
STATUS_NAMES = {
    0: "FEASM_OK",
    -1: "FEASM_EINVAL",
    -2: "FEASM_ERANGE",
    -3: "FEASM_ENOMEM",
    -4: "FEASM_EHIP",
    -5: "FEASM_EOVERFLOW",
    -6: "FEASM_ELIMIT",
    -7: "FEASM_EINCOMPLETE",
}
FEASM_EINCOMPLETE = -7

# Every function the header declares, with (restype, argtypes).
P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
U32 = ctypes.c_uint32
INT = ctypes.c_int
PP = ctypes.POINTER(ctypes.c_void_p)
PI64 = ctypes.POINTER(ctypes.c_int64)
PI32 = ctypes.POINTER(ctypes.c_int32)

class ServeMesh(ctypes.Structure):
    _fields_ = [("conn", ctypes.c_void_p), ("n_elem", ctypes.c_int64),
                ("nodes_per_elem", ctypes.c_int32), ("dofs_per_node", ctypes.c_int32),
                ("n_nodes", ctypes.c_int64), ("recipe", ctypes.c_int32),
                ("pool_size", ctypes.c_int32), ("ke_pool", ctypes.c_void_p),
                ("pattern", ctypes.c_void_p)]


class Request(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("mesh", ctypes.c_int32),
                ("n_reassembly", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("keep_values", ctypes.c_void_p)]


class RequestResult(ctypes.Structure):
    _fields_ = [("admitted_s", ctypes.c_double), ("assembled_s", ctypes.c_double),
                ("done_s", ctypes.c_double)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("fmt", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("hbm_budget", ctypes.c_int64), ("pattern_cache_bytes", ctypes.c_int64)]


class ServeStats(ctypes.Structure):
    _fields_ = [("pattern_hits", ctypes.c_int64), ("pattern_misses", ctypes.c_int64),
                ("pattern_evictions", ctypes.c_int64), ("pattern_cache_peak_bytes", ctypes.c_int64),
                ("patterns_resident_at_end", ctypes.c_int64), ("pattern_build_s", ctypes.c_double),
                ("generate_ms", ctypes.c_double), ("assemble_ms", ctypes.c_double),
                ("generated_bytes", ctypes.c_int64)]


# set_allocator callbacks: alloc(bytes, stream, ctx) -> ptr, release(ptr, stream, ctx)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

SIGNATURES = {
    "pattern_build": (INT, [P, I64, I32, I32, I64, U32, P, PP]),
    "assemble_csr": (INT, [P, P, P, INT, P]),
    "assemble_crac": (INT, [P, P, P, INT, P]),
    "reassemble_values": (INT, [P, INT, P, P, INT, P]),
    "spmv_csr": (INT, [P, P, P, P, P]),
    "spmv_crac": (INT, [P, P, P, P, P]),
    "hex8_element_matrices": (INT, [P, P, P, P, P]),
    "assemble_hex8": (INT, [P, INT, P, P, P, INT, P]),
    "pattern_info": (INT, [P, PI64, PI64, PI64, PI32]),
    "pattern_arrays": (INT, [P, PP, PP, PP, PP]),
    "pattern_colouring": (INT, [P, PP, PP, PP]),
    "pattern_tune": (INT, [P, INT, I64]),
    "pattern_free": (None, [P]),
    "generate_ke": (INT, [INT, I64, I32, ctypes.c_uint64, I64, P, P]),
    "batch_create": (INT, [P, I64, INT, U32, PP]),
    "assemble_batch": (INT, [P, P, P, P]),
    "batch_info": (INT, [P, PI32, PI64, PI64, P]),
    "batch_free": (None, [P]),
    "serve_run": (INT, [ctypes.POINTER(ServeMesh), I64, ctypes.POINTER(Request), I64,
                        ctypes.POINTER(ServeConfig), ctypes.POINTER(RequestResult), P,
                        ctypes.POINTER(ServeStats)]),
    "last_error": (ctypes.c_char_p, []),
    "set_allocator": (INT, [ALLOC_FN, RELEASE_FN, P]),
    "spin_aborts": (INT, [P, PI64]),
    "assemble_spin_noalloc": (INT, [P, INT, P, P, P, INT, P]),
}

_lib = None


def load():
    """Load libfeasm.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2012_00585_amd.build` "
            "(the HIP library is required; there is no fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class FeasmError(RuntimeError):
    def __init__(self, what, code):
        msg = load().last_error().decode(errors="replace")
        super().__init__(f"{what} failed with {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code, what):
    if code != FEASM_OK:
        raise FeasmError(what, code)


_hip = None


def hip():
    """The HIP runtime (for device-to-device copies of borrowed arrays)."""
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.restype = INT
        _hip.hipMemcpyAsync.argtypes = [P, P, ctypes.c_size_t, INT, P]
    return _hip

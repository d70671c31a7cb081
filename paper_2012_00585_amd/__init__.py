"""feasm: MI355X-native finite-element sparse-matrix assembly (CSR + CRAC).

Python binding of libfeasm.so.  It only marshals arguments: every step of
the symbolic and numeric phases runs in the library's HIP kernels.  Tensors
are torch CUDA (HIP) tensors; streams default to torch's current stream.

    p = pattern_build(conn, dofs_per_node=3, n_nodes=nn)          # symbolic
    values = assemble_csr(p, ke)                                  # numeric
    values = assemble_crac(p, ke, values)
    values = reassemble_values(p, FMT_CRAC, ke_new, values)       # values only
"""
from __future__ import annotations

import atexit
import ctypes
import weakref

import torch

from . import _lib
from ._lib import FeasmError

BUILD_CSR = 1
BUILD_CRAC = 2
BUILD_COLOUR = 4
BUILD_TILES = 8
BUILD_OWNER_MAP = 16
FMT_CSR = 0
FMT_CRAC = 1
SCATTER_AUTO = 0
SCATTER_ATOMIC = 1
SCATTER_COLOURED = 2
SCATTER_OWNER = 3
SCATTER_SPIN = 4
ACCUMULATE = 0x100  # or into `scatter`: add into values without resetting them

TUNE_OWNER_BLOCKS_PER_CU = 1
TUNE_THREADS_PER_ELEM = 2
TUNE_OWNER_ROWS = 3
TUNE_OWNER_BATCH = 4
TUNE_STRATEGY = 5
TUNE_OWNER_FLAT = 6
TUNE_OWNER_PREFETCH = 7
TUNE_SPMV_CHUNK = 8
TUNE_HEX8_PIPE = 9
TUNE_SPIN_LIMIT = 10
TUNE_TILE_CAP = 11
TUNE_COLOUR_BLOCKS = 12

_HIP_D2D = 3  # hipMemcpyDeviceToDevice


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _require(t, dtype, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor, got {t.device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Pattern:
    """Handle of a sparsity pattern built on the device (owns device arrays)."""

    def __init__(self, handle, n_elem, nodes_per_elem, dofs_per_node, n_nodes, flags):
        self._h = handle
        self.n_elem = n_elem
        self.nodes_per_elem = nodes_per_elem
        self.dofs_per_node = dofs_per_node
        self.n = nodes_per_elem * dofs_per_node
        self.n_nodes = n_nodes
        self.flags = flags
        n_rows, nnz, n_ca = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        n_col = ctypes.c_int32()
        _lib.check(_lib.load().pattern_info(handle, ctypes.byref(n_rows), ctypes.byref(nnz),
                                            ctypes.byref(n_ca), ctypes.byref(n_col)),
                   "pattern_info")
        self.n_rows = n_rows.value
        self.nnz = nnz.value
        self.n_ca = n_ca.value
        self.n_colours = n_col.value
        _track(self)

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("pattern was freed")
        return self._h

    def _copy(self, ptr, count, dtype, stream=None):
        out = torch.empty(count, dtype=dtype, device="cuda")
        if count:
            rc = _lib.hip().hipMemcpyAsync(_ptr(out), ptr, count * out.element_size(), _HIP_D2D,
                                          _stream(stream))
            if rc != 0:
                raise RuntimeError(f"hipMemcpyAsync failed: {rc}")
        return out

    def _arrays(self):
        ptrs = [ctypes.c_void_p() for _ in range(4)]
        _lib.check(_lib.load().pattern_arrays(self.handle, *[ctypes.byref(p) for p in ptrs]),
                   "pattern_arrays")
        return ptrs

    def csr(self, stream=None):
        """Copies of (row_ptr[n_rows+1], col_idx[nnz]) as int32 device tensors."""
        rp, ci, _, _ = self._arrays()
        if not rp.value:
            raise ValueError("pattern was built without CSR")
        return (self._copy(rp, self.n_rows + 1, torch.int32, stream),
                self._copy(ci, self.nnz, torch.int32, stream))

    def crac(self, stream=None):
        """Copies of (crac_row_ptr[n_rows+1], col_align[n_ca]) as int32 device tensors."""
        _, _, crp, ca = self._arrays()
        if not crp.value:
            raise ValueError("pattern was built without CRAC")
        return (self._copy(crp, self.n_rows + 1, torch.int32, stream),
                self._copy(ca, self.n_ca, torch.int32, stream))

    def colouring(self, stream=None):
        """(colour_ptr list[n_colours+1], colour_elems int32[n_elem], element_colour int32[n_elem])."""
        cp, ce, ec = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        _lib.check(_lib.load().pattern_colouring(self.handle, ctypes.byref(cp), ctypes.byref(ce),
                                                 ctypes.byref(ec)), "pattern_colouring")
        cp = ctypes.cast(cp, ctypes.POINTER(ctypes.c_int64))
        ptr = [cp[i] for i in range(self.n_colours + 1)]
        return (ptr, self._copy(ce, self.n_elem, torch.int32, stream),
                self._copy(ec, self.n_elem, torch.int32, stream))

    def tune(self, key: int, value: int):
        """Set a launch-shape knob of this handle (0 = library default)."""
        _lib.check(_lib.load().pattern_tune(self.handle, key, value), "pattern_tune")

    def spin_aborts(self) -> int:
        """Row-lock lanes that gave up since the last call (synchronises);
        the library reports a non-zero count with FEASM_EINCOMPLETE."""
        c = ctypes.c_int64()
        rc = _lib.load().spin_aborts(self.handle, ctypes.byref(c))
        if rc != _lib.FEASM_EINCOMPLETE:
            _lib.check(rc, "spin_aborts")
        return c.value

    def free(self):
        if self._h is not None:
            _lib.load().pattern_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def pattern_build(conn: torch.Tensor, dofs_per_node: int, n_nodes: int,
                  flags: int = BUILD_CSR | BUILD_CRAC, stream=None) -> Pattern:
    """Symbolic phase: CSR/CRAC pattern (and optional colouring) of a mesh.

    ``conn`` is an int32 device tensor [n_elem, nodes_per_elem].
    """
    _require(conn, torch.int32, "conn")
    if conn.dim() != 2:
        raise ValueError("conn must be [n_elem, nodes_per_elem]")
    E, k = conn.shape
    h = ctypes.c_void_p()
    _lib.check(_lib.load().pattern_build(_ptr(conn), E, k, dofs_per_node, n_nodes, flags,
                                         _stream(stream), ctypes.byref(h)), "pattern_build")
    return Pattern(h, E, k, dofs_per_node, n_nodes, flags)


def _numeric_args(p: Pattern, ke, values):
    _require(ke, torch.float64, "ke")
    if ke.numel() != p.n_elem * p.n * p.n:
        raise ValueError(f"ke must hold n_elem*n*n = {p.n_elem * p.n * p.n} values, "
                         f"got {ke.numel()}")
    if values is None:
        values = torch.empty(p.nnz, dtype=torch.float64, device=ke.device)
    _require(values, torch.float64, "values")
    if values.numel() < p.nnz:
        raise ValueError(f"values must hold nnz = {p.nnz} entries, got {values.numel()}")
    return values


def assemble_csr(p: Pattern, ke: torch.Tensor, values: torch.Tensor | None = None,
                 scatter: int = SCATTER_AUTO, stream=None) -> torch.Tensor:
    """values := sum_e scatter(K_e) through the CSR arrays (asynchronous)."""
    values = _numeric_args(p, ke, values)
    _lib.check(_lib.load().assemble_csr(p.handle, _ptr(ke), _ptr(values), scatter,
                                        _stream(stream)), "assemble_csr")
    return values


def assemble_crac(p: Pattern, ke: torch.Tensor, values: torch.Tensor | None = None,
                  scatter: int = SCATTER_AUTO, stream=None) -> torch.Tensor:
    """values := sum_e scatter(K_e) through the CRAC arrays (asynchronous)."""
    values = _numeric_args(p, ke, values)
    _lib.check(_lib.load().assemble_crac(p.handle, _ptr(ke), _ptr(values), scatter,
                                         _stream(stream)), "assemble_crac")
    return values


def reassemble_values(p: Pattern, fmt: int, ke: torch.Tensor, values: torch.Tensor | None = None,
                      scatter: int = SCATTER_AUTO, stream=None) -> torch.Tensor:
    """Value-only re-assembly on an existing pattern (asynchronous)."""
    values = _numeric_args(p, ke, values)
    _lib.check(_lib.load().reassemble_values(p.handle, fmt, _ptr(ke), _ptr(values), scatter,
                                             _stream(stream)), "reassemble_values")
    return values


def _spmv_args(p: Pattern, values, x, y):
    _require(values, torch.float64, "values")
    _require(x, torch.float64, "x")
    if values.numel() < p.nnz:
        raise ValueError(f"values must hold nnz = {p.nnz} entries, got {values.numel()}")
    if x.numel() != p.n_rows:
        raise ValueError(f"x must hold n_rows = {p.n_rows} entries, got {x.numel()}")
    if y is None:
        y = torch.empty(p.n_rows, dtype=torch.float64, device=x.device)
    _require(y, torch.float64, "y")
    if y.numel() != p.n_rows:
        raise ValueError(f"y must hold n_rows = {p.n_rows} entries, got {y.numel()}")
    return y


def spmv_csr(p: Pattern, values: torch.Tensor, x: torch.Tensor, y: torch.Tensor | None = None,
             stream=None) -> torch.Tensor:
    """y := G x through CSR (asynchronous)."""
    y = _spmv_args(p, values, x, y)
    _lib.check(_lib.load().spmv_csr(p.handle, _ptr(values), _ptr(x), _ptr(y), _stream(stream)),
               "spmv_csr")
    return y


def spmv_crac(p: Pattern, values: torch.Tensor, x: torch.Tensor, y: torch.Tensor | None = None,
              stream=None) -> torch.Tensor:
    """y := G x through the CRAC runs (asynchronous)."""
    y = _spmv_args(p, values, x, y)
    _lib.check(_lib.load().spmv_crac(p.handle, _ptr(values), _ptr(x), _ptr(y), _stream(stream)),
               "spmv_crac")
    return y


def _hex8_args(p: Pattern, coords, material):
    _require(coords, torch.float64, "coords")
    _require(material, torch.float64, "material")
    if coords.numel() != 3 * p.n_nodes:
        raise ValueError(f"coords must hold 3 * n_nodes = {3 * p.n_nodes} values")
    m = 1 if p.dofs_per_node == 1 else 2
    if material.numel() != m * p.n_elem:
        raise ValueError(f"material must hold {m} * n_elem = {m * p.n_elem} values")


def hex8_element_matrices(p: Pattern, coords: torch.Tensor, material: torch.Tensor,
                          ke: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Element stiffness matrices of 8-node hexahedra (Laplace for d = 1,
    elasticity for d = 3) into ke [n_elem, 8d, 8d] (asynchronous)."""
    _hex8_args(p, coords, material)
    if ke is None:
        ke = torch.empty((p.n_elem, p.n, p.n), dtype=torch.float64, device=coords.device)
    _require(ke, torch.float64, "ke")
    if ke.numel() < p.n_elem * p.n * p.n:
        raise ValueError("ke too small")
    _lib.check(_lib.load().hex8_element_matrices(p.handle, _ptr(coords), _ptr(material), _ptr(ke),
                                                 _stream(stream)), "hex8_element_matrices")
    return ke


def assemble_hex8(p: Pattern, fmt: int, coords: torch.Tensor, material: torch.Tensor,
                  values: torch.Tensor | None = None, accumulate: bool = False,
                  stream=None) -> torch.Tensor:
    """values := G with each hexahedron's stiffness computed inside the
    row-owned assembly (no element matrices in memory; asynchronous)."""
    _hex8_args(p, coords, material)
    if values is None:
        values = torch.empty(p.nnz, dtype=torch.float64, device=coords.device)
    _require(values, torch.float64, "values")
    if values.numel() < p.nnz:
        raise ValueError(f"values must hold nnz = {p.nnz} entries")
    _lib.check(_lib.load().assemble_hex8(p.handle, fmt, _ptr(coords), _ptr(material), _ptr(values),
                                         ACCUMULATE if accumulate else 0, _stream(stream)),
               "assemble_hex8")
    return values


RECIPE_LAPLACIAN = 0
RECIPE_SPD = 1


def generate_ke(recipe: int, n_elem: int, n: int, seed: int, elem_offset: int = 0,
                out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Reproducible element matrices on the device (workload generator)."""
    if out is None:
        out = torch.empty((n_elem, n, n), dtype=torch.float64, device="cuda")
    _require(out, torch.float64, "out")
    if out.numel() < n_elem * n * n:
        raise ValueError("out too small")
    _lib.check(_lib.load().generate_ke(recipe, n_elem, n, seed, elem_offset, _ptr(out),
                                       _stream(stream)), "generate_ke")
    return out


def load():
    """Load the native library (raises if it is not built)."""
    return _lib.load()


# ------------------------------------------------------------ device memory
# Objects that own device arrays (patterns, batches); freed at interpreter
# exit while the allocator that created their arrays is still usable.
_live = weakref.WeakSet()
_allocator_refs = None  # the ctypes callbacks installed last (kept alive)


def _track(obj):
    _live.add(obj)


@atexit.register
def _free_live_objects():
    for obj in list(_live):
        try:
            obj.free()
        except Exception:
            pass


def set_allocator(alloc=None, release=None, ctx=None):
    """Install device-allocation callbacks for the library's own arrays.

    ``alloc`` and ``release`` are ``_lib.ALLOC_FN`` / ``_lib.RELEASE_FN``
    ctypes callbacks (or both None for hipMalloc/hipFree).  Objects keep the
    allocator that created them."""
    global _allocator_refs
    if (alloc is None) != (release is None):
        raise ValueError("give both alloc and release, or neither")
    a = alloc if alloc is not None else _lib.ALLOC_FN()
    r = release if release is not None else _lib.RELEASE_FN()
    _lib.check(_lib.load().set_allocator(a, r, ctx), "set_allocator")
    if alloc is not None:
        # callbacks stay referenced while any object may still release through them
        _allocator_refs = (alloc, release, _allocator_refs)


def use_torch_allocator():
    """Take the library's device arrays from torch's caching allocator, on
    the stream of the call that needs them (the current device's)."""

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:
            return None

    def _release(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    set_allocator(_lib.ALLOC_FN(_alloc), _lib.RELEASE_FN(_release))


def use_default_allocator():
    """Back to hipMalloc / hipFree for arrays created from now on."""
    set_allocator()

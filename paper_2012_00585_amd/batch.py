"""Batched assembly of many meshes in one graph-captured launch.

    b = Batch(patterns, fmt=FMT_CRAC)        # patterns: list of Pattern
    b.assemble(kes, values)                  # lists of device tensors, one per mesh
    b.free()

Each mesh runs the strategy and launch shape its handle was tuned to (see
``autotune``).  Modes: one launch per kernel path with a workgroup per work
tile (default), persistent launches pulling tiles from device counters
(``persistent=True``), or every mesh's own kernels (``per_mesh_graph=True``).
Argument marshalling only; the work runs in libfeasm's batch kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import FMT_CRAC, Pattern, _lib, _require, _stream, _track

PATH_NAMES = ["own_g4", "own_g8", "own_g16", "own_g32", "own_g64_j1", "own_g64_j2", "own_g64_j4",
              "own_g64_j8", "own_g64_j16", "rows2_j1", "rows2_j2", "own_pipe24", "own_lanes3",
              "own_lanes4", "elem_atomic16",
              "elem_atomic32",
              "elem_atomic64", "elem_plain16", "elem_plain32", "elem_plain64"]


class Batch:
    def __init__(self, patterns: list[Pattern], fmt: int = FMT_CRAC, accumulate: bool = False,
                 per_mesh_graph: bool = False, persistent: bool = False):
        self.patterns = list(patterns)
        n = len(self.patterns)
        arr = (ctypes.c_void_p * n)(*[p.handle.value for p in self.patterns])
        h = ctypes.c_void_p()
        flags = ((0x100 if accumulate else 0) | (0x200 if per_mesh_graph else 0)
                 | (0x400 if persistent else 0))
        self.per_mesh_graph = per_mesh_graph
        self.persistent = persistent
        _lib.check(_lib.load().batch_create(arr, n, fmt, flags, ctypes.byref(h)), "batch_create")
        self._h = h
        self.fmt = fmt
        self._keep = None
        _track(self)

    def assemble(self, kes, values, stream=None):
        """Replay the batch graph; kes[i], values[i] are device float64 tensors."""
        n = len(self.patterns)
        if len(kes) != n or len(values) != n:
            raise ValueError("one ke and one values tensor per mesh")
        for p, k, v in zip(self.patterns, kes, values):
            _require(k, torch.float64, "ke")
            _require(v, torch.float64, "values")
            if k.numel() != p.n_elem * p.n * p.n or v.numel() < p.nnz:
                raise ValueError("ke/values size does not match its mesh")
        ka = (ctypes.c_void_p * n)(*[k.data_ptr() for k in kes])
        va = (ctypes.c_void_p * n)(*[v.data_ptr() for v in values])
        self._keep = (kes, values)
        _lib.check(_lib.load().assemble_batch(self._h, ka, va, _stream(stream)), "assemble_batch")
        return values

    def info(self):
        n = len(self.patterns)
        ph, nt, grid = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        paths = (ctypes.c_int32 * n)()
        _lib.check(_lib.load().batch_info(self._h, ctypes.byref(ph), ctypes.byref(nt),
                                          ctypes.byref(grid), paths), "batch_info")
        return {"phases": ph.value, "tiles": nt.value, "grid": grid.value,
                "paths": [PATH_NAMES[i] for i in paths]}

    def free(self):
        if self._h is not None:
            _lib.load().batch_free(self._h)
            self._h = None
        self._keep = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

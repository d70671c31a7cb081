"""Serving: assembly and Newton-style re-assembly requests as they arrive.

Each request names a registered mesh and asks for one assembly followed by
``n_reassembly`` value-only re-assemblies.  The loop itself is libfeasm's
native engine (``serve_run``): continuous batching into stream slots under
an HBM budget, each slot issuing its next iteration as soon as the previous
one completes.  A mesh is registered either with a resident pattern handle
(``register``) or with its connectivity only (``register_mesh``), in which
case the engine builds its pattern on first use and keeps it in a cache
bounded in bytes, evicting the least recently used idle patterns.  Element
matrices are generated on the device for every iteration, or read from a
pool the caller generated beforehand (``ke_pool``).  ``slots=1`` gives the
one-mesh-at-a-time FIFO baseline on one stream.  This module marshals the
tables and summarises the timings.

Completion times and re-assembly latencies are device times (timing events);
admission is host time.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import FMT_CRAC, _lib


@dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the run
    mesh: object            # key of a registered mesh
    seed: int
    n_reassembly: int = 10


@dataclass
class _Mesh:
    pattern: object         # Pattern or None (built by the engine's cache)
    conn: object            # device int32 tensor [n_elem][k] or None
    n_elem: int
    k: int
    d: int
    n_nodes: int
    recipe: int
    ke_pool: object = None  # device float64 tensor [pool][n_elem][n][n] or None
    nnz_bound: int = 0

    @property
    def n(self):
        return self.k * self.d

    def footprint(self):
        ke = 0 if self.ke_pool is not None else 2 * self.n_elem * self.n * self.n * 8
        nnz = self.pattern.nnz if self.pattern is not None else self.n_elem * self.n * self.n
        return ke + nnz * 8


def iteration_seed(seed: int, it: int) -> int:
    """64-bit generator key of iteration `it` of a request (0 = assembly)."""
    return (seed * 1000003 + it * 7919 + 1) & ((1 << 64) - 1)


def pool_block(seed: int, it: int, pool_size: int) -> int:
    """Block of a mesh's element-matrix pool read by iteration `it`."""
    return ((seed & ((1 << 64) - 1)) + it) % (1 << 64) % pool_size


class Server:
    """Request server over registered meshes.  Each mesh assembles with the
    strategy its handle is tuned to (``Pattern.tune``; AUTO = row-owned)."""

    def __init__(self, fmt=FMT_CRAC, slots=8, hbm_budget=None, keep=(), pattern_cache_bytes=None):
        self.fmt = fmt
        self.nslots = slots
        self.meshes = {}
        self.budget = hbm_budget
        self.cache_bytes = pattern_cache_bytes
        self.keep = set(keep)        # request ids whose final values are kept
        self.kept = {}
        self.last_stats = None

    def register(self, key, pattern, recipe, ke_pool=None):
        """A mesh with a resident pattern handle of the caller."""
        self.meshes[key] = _Mesh(pattern, None, pattern.n_elem, pattern.nodes_per_elem,
                                 pattern.dofs_per_node, pattern.n_nodes, recipe, ke_pool)

    def register_mesh(self, key, conn, dofs_per_node, n_nodes, recipe, ke_pool=None):
        """A mesh known by its connectivity (device int32 [n_elem][k]); its
        pattern is built by the engine on first use and cached."""
        conn = conn.contiguous()
        self.meshes[key] = _Mesh(None, conn, conn.shape[0], conn.shape[1], dofs_per_node, n_nodes,
                                 recipe, ke_pool)

    def footprint(self, req):
        return self.meshes[req.mesh].footprint()

    def run(self, requests, log=None):
        """Serve `requests` with the native engine; returns latency and throughput figures."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        keys = list(self.meshes)
        index = {k: i for i, k in enumerate(keys)}
        table = (_lib.ServeMesh * len(keys))()
        for i, k in enumerate(keys):
            m = self.meshes[k]
            table[i].conn = m.conn.data_ptr() if m.conn is not None else None
            table[i].n_elem = m.n_elem
            table[i].nodes_per_elem = m.k
            table[i].dofs_per_node = m.d
            table[i].n_nodes = m.n_nodes
            table[i].recipe = m.recipe
            if m.ke_pool is not None:
                assert m.ke_pool.dtype == torch.float64 and m.ke_pool.is_contiguous()
                assert m.ke_pool.numel() % (m.n_elem * m.n * m.n) == 0
                table[i].pool_size = m.ke_pool.numel() // (m.n_elem * m.n * m.n)
                table[i].ke_pool = m.ke_pool.data_ptr()
            table[i].pattern = m.pattern.handle.value if m.pattern is not None else None
        arr = (_lib.Request * len(reqs))()
        keep = {}
        for i, r in enumerate(reqs):
            arr[i].arrival_s = r.arrival
            arr[i].mesh = index[r.mesh]
            arr[i].n_reassembly = r.n_reassembly
            arr[i].seed = r.seed & ((1 << 64) - 1)
            if r.rid in self.keep:
                m = self.meshes[r.mesh]
                nnz = m.pattern.nnz if m.pattern is not None else m.n_elem * m.n * m.n
                keep[r.rid] = torch.empty(nnz, dtype=torch.float64, device="cuda")
                arr[i].keep_values = keep[r.rid].data_ptr()
        cfg = _lib.ServeConfig(self.fmt, self.nslots, int(self.budget or 0),
                               int(self.cache_bytes or 0))
        res = (_lib.RequestResult * len(reqs))()
        n_re = sum(r.n_reassembly for r in reqs)
        re_lat = np.zeros(max(n_re, 1))
        st = _lib.ServeStats()
        torch.cuda.synchronize()
        _lib.check(_lib.load().serve_run(table, len(keys), arr, len(reqs), ctypes.byref(cfg), res,
                                         re_lat.ctypes.data_as(ctypes.c_void_p),
                                         ctypes.byref(st)),
                   "serve_run")
        torch.cuda.synchronize()
        for rid, t in keep.items():
            self.kept[rid] = t.cpu().numpy()
        arrival = np.array([r.arrival for r in reqs])
        admitted = np.array([x.admitted_s for x in res])
        assembled = np.array([x.assembled_s for x in res])
        done = np.array([x.done_s for x in res])
        elements = sum(self.meshes[r.mesh].n_elem * (1 + r.n_reassembly) for r in reqs)
        wall = float(done.max()) if len(reqs) else 0.0
        span = float(arrival.max()) if len(reqs) else 0.0
        # in-flight concurrency from admission/completion times
        ev = sorted([(a, 1) for a in admitted] + [(d, -1) for d in done])
        level = peak = 0
        for _, x in ev:
            level += x
            peak = max(peak, level)

        def pct(a, q):
            return float(np.percentile(np.asarray(a) * 1e3, q)) if len(a) else None

        lat_asm = assembled - arrival
        wait = admitted - arrival
        re = re_lat[:n_re]
        stats = {f: getattr(st, f) for f, _ in _lib.ServeStats._fields_}
        self.last_stats = stats
        return {
            "requests": len(reqs),
            "wall_s": wall,
            "arrival_span_s": span,
            "offered_req_per_s": len(reqs) / span if span > 0 else None,
            "achieved_req_per_s": len(reqs) / wall if wall > 0 else None,
            "element_matrices_per_s": elements / wall if wall > 0 else None,
            "assembly_ms": {"p50": pct(lat_asm, 50), "p99": pct(lat_asm, 99),
                            "mean": float(lat_asm.mean() * 1e3) if len(reqs) else None},
            "reassembly_ms": {"p50": pct(re, 50), "p99": pct(re, 99),
                              "mean": float(re.mean() * 1e3) if n_re else None},
            "queue_wait_ms": {"p50": pct(wait, 50), "p99": pct(wait, 99)},
            "max_pending": int(_max_waiting(arrival, admitted)),
            "peak_in_flight": peak,
            "slots": self.nslots,
            "engine": stats,
        }


def _max_waiting(arrival, admitted):
    """Largest number of requests that had arrived but were not yet admitted."""
    ev = sorted([(a, 1) for a in arrival] + [(b, -1) for b in admitted])
    level = peak = 0
    for _, x in ev:
        level += x
        peak = max(peak, level)
    return peak

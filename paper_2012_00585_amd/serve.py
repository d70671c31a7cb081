"""Serving: assembly and Newton-style re-assembly requests as they arrive.

Each request names a registered mesh (whose pattern stays resident on the
device) and asks for one assembly followed by ``n_reassembly`` value-only
re-assemblies, each with fresh element matrices generated on the device.
The loop itself is libfeasm's native engine (``serve_run``): continuous
batching into stream slots under an HBM budget, each slot issuing its next
iteration as soon as the previous one completes, element matrices for the
next iteration generated on a side stream.  ``slots=1`` gives the
one-mesh-at-a-time FIFO baseline on one stream.  This module marshals the
request table and summarises the timings.

Latency is host time from arrival (assembly) or issue (re-assembly) to the
engine's first poll that sees the completion.
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
    pattern: object
    recipe: int
    bytes: int  # element matrices x2 + values


def iteration_seed(seed: int, it: int) -> int:
    """64-bit generator key of iteration `it` of a request (0 = assembly)."""
    return (seed * 1000003 + it * 7919 + 1) & ((1 << 64) - 1)


class Server:
    """Request server over registered meshes.  Each mesh assembles with the
    strategy its handle is tuned to (``Pattern.tune``; AUTO = row-owned)."""

    def __init__(self, fmt=FMT_CRAC, slots=8, hbm_budget=None, keep=()):
        self.fmt = fmt
        self.nslots = slots
        self.meshes = {}
        self.budget = hbm_budget
        self.keep = set(keep)        # request ids whose final values are kept
        self.kept = {}

    def register(self, key, pattern, recipe):
        """Make a mesh's resident pattern available to requests."""
        nbytes = 2 * pattern.n_elem * pattern.n * pattern.n * 8 + pattern.nnz * 8
        self.meshes[key] = _Mesh(pattern, recipe, nbytes)

    def footprint(self, req):
        return self.meshes[req.mesh].bytes

    def run(self, requests, log=None):
        """Serve `requests` with the native engine; returns latency and throughput figures."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        keys = list(self.meshes)
        index = {k: i for i, k in enumerate(keys)}
        handles = (ctypes.c_void_p * len(keys))(*[self.meshes[k].pattern.handle.value
                                                  for k in keys])
        recipes = (ctypes.c_int32 * len(keys))(*[self.meshes[k].recipe for k in keys])
        arr = (_lib.Request * len(reqs))()
        keep = {}
        for i, r in enumerate(reqs):
            arr[i].arrival_s = r.arrival
            arr[i].mesh = index[r.mesh]
            arr[i].n_reassembly = r.n_reassembly
            arr[i].seed = r.seed & ((1 << 64) - 1)
            if r.rid in self.keep:
                p = self.meshes[r.mesh].pattern
                keep[r.rid] = torch.empty(p.nnz, dtype=torch.float64, device="cuda")
                arr[i].keep_values = keep[r.rid].data_ptr()
        res = (_lib.RequestResult * len(reqs))()
        n_re = sum(r.n_reassembly for r in reqs)
        re_lat = np.zeros(max(n_re, 1))
        torch.cuda.synchronize()
        _lib.check(_lib.load().serve_run(handles, recipes, len(keys), arr, len(reqs), self.fmt,
                                         self.nslots, int(self.budget or 0), res,
                                         re_lat.ctypes.data_as(ctypes.c_void_p)),
                   "serve_run")
        torch.cuda.synchronize()
        for rid, t in keep.items():
            self.kept[rid] = t.cpu().numpy()
        arrival = np.array([r.arrival for r in reqs])
        admitted = np.array([x.admitted_s for x in res])
        assembled = np.array([x.assembled_s for x in res])
        done = np.array([x.done_s for x in res])
        elements = sum(self.meshes[r.mesh].pattern.n_elem * (1 + r.n_reassembly) for r in reqs)
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
        }


def _max_waiting(arrival, admitted):
    """Largest number of requests that had arrived but were not yet admitted."""
    ev = sorted([(a, 1) for a in arrival] + [(b, -1) for b in admitted])
    level = peak = 0
    for _, x in ev:
        level += x
        peak = max(peak, level)
    return peak

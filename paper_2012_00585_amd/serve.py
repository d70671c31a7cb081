"""Serving loop: assembly and Newton-style re-assembly requests as they arrive.

Each request names a registered mesh (whose pattern stays resident on the
device) and asks for one assembly followed by ``n_reassembly`` value-only
re-assemblies, each with fresh element matrices generated on the device.

Continuous batching: requests are admitted into free slots as soon as the
HBM budget allows (footprint = two element-matrix buffers + one values
buffer); every slot has its own stream, so the work of all admitted
requests overlaps on the GPU, and each slot issues its next iteration the
moment its previous one completes (a Newton loop with zero solver time).
Element matrices for iteration i+1 are generated on the slot's side stream
while iteration i assembles (ping-pong buffers).  ``slots=1`` gives the
one-mesh-at-a-time FIFO baseline on one stream.

Latency is host time from arrival (assembly) or issue (re-assembly) to the
first poll that sees the completion event.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import (FMT_CRAC, FMT_CSR, SCATTER_AUTO, assemble_crac, assemble_csr, generate_ke,
               reassemble_values)


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


@dataclass
class _Slot:
    stream: object
    side: object
    req: Request = None
    it: int = 0
    ke: list = field(default_factory=list)
    values: object = None
    done: object = None       # event of the iteration in flight
    gen_done: list = field(default_factory=list)
    issued: float = 0.0
    footprint: int = 0


def iteration_seed(seed: int, it: int) -> int:
    """64-bit generator key of iteration `it` of a request (0 = assembly)."""
    return (seed * 1000003 + it * 7919 + 1) & ((1 << 64) - 1)


class Server:
    def __init__(self, fmt=FMT_CRAC, slots=8, hbm_budget=None, scatter=SCATTER_AUTO,
                 keep=()):
        self.fmt = fmt
        self.nslots = slots
        self.scatter = scatter
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

    def _issue(self, s: _Slot, now):
        m = self.meshes[s.req.mesh]
        p = m.pattern
        buf = s.it % 2
        s.stream.wait_event(s.gen_done[buf])
        if s.it == 0:
            fn = assemble_csr if self.fmt == FMT_CSR else assemble_crac
            fn(p, s.ke[buf], s.values, self.scatter, stream=s.stream)
        else:
            reassemble_values(p, self.fmt, s.ke[buf], s.values, self.scatter, stream=s.stream)
        s.done = torch.cuda.Event()
        s.done.record(s.stream)
        s.issued = now
        # element matrices of the next iteration go into the other buffer; its
        # last reader (iteration it-1) completed before this one was issued
        nxt = s.it + 1
        if nxt <= s.req.n_reassembly:
            ob = nxt % 2
            generate_ke(m.recipe, p.n_elem, p.n, iteration_seed(s.req.seed, nxt), 0,
                        out=s.ke[ob], stream=s.side)
            ev = torch.cuda.Event()
            ev.record(s.side)
            s.gen_done[ob] = ev

    def _admit(self, s: _Slot, req: Request, now):
        m = self.meshes[req.mesh]
        p = m.pattern
        s.req = req
        s.it = 0
        s.footprint = m.bytes
        s.ke = [torch.empty((p.n_elem, p.n, p.n), dtype=torch.float64, device="cuda")
                for _ in range(2)]
        s.values = torch.empty(p.nnz, dtype=torch.float64, device="cuda")
        generate_ke(m.recipe, p.n_elem, p.n, iteration_seed(req.seed, 0), 0, out=s.ke[0],
                    stream=s.side)
        ev = torch.cuda.Event()
        ev.record(s.side)
        s.gen_done = [ev, None]
        self._issue(s, now)

    def run(self, requests, log=None):
        """Serve `requests` (sorted by arrival); returns latency and throughput figures."""
        reqs = collections.deque(sorted(requests, key=lambda r: r.arrival))
        pending = collections.deque()
        slots = [_Slot(torch.cuda.Stream(), torch.cuda.Stream()) for _ in range(self.nslots)]
        used = 0
        lat_asm, lat_re, finish = [], [], {}
        queue_wait = []
        elements = 0
        max_pending = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        busy = 0
        while reqs or pending or busy:
            now = time.perf_counter() - t0
            while reqs and reqs[0].arrival <= now:
                pending.append(reqs.popleft())
            max_pending = max(max_pending, len(pending))
            # completions
            for s in slots:
                if s.req is None or not s.done.query():
                    continue
                now = time.perf_counter() - t0
                p = self.meshes[s.req.mesh].pattern
                elements += p.n_elem
                if s.it == 0:
                    lat_asm.append(now - s.req.arrival)
                else:
                    lat_re.append(now - s.issued)
                if s.it < s.req.n_reassembly:
                    s.it += 1
                    self._issue(s, now)
                else:
                    if s.req.rid in self.keep:
                        self.kept[s.req.rid] = s.values.detach().cpu().numpy()
                    finish[s.req.rid] = now
                    used -= s.footprint
                    s.req = None
                    s.ke, s.values = [], None
                    busy -= 1
            # admissions: FIFO, as slots and memory free up
            for s in slots:
                if not pending:
                    break
                if s.req is not None:
                    continue
                req = pending[0]
                fp = self.footprint(req)
                if self.budget is not None and used + fp > self.budget and busy > 0:
                    break
                pending.popleft()
                now = time.perf_counter() - t0
                queue_wait.append(now - req.arrival)
                used += fp
                busy += 1
                self._admit(s, req, now)
            if not busy and reqs and not pending:
                time.sleep(max(0.0, min(1e-4, reqs[0].arrival - (time.perf_counter() - t0))))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        span = max(r.arrival for r in requests) if requests else 0.0

        def pct(a, q):
            return float(np.percentile(np.asarray(a) * 1e3, q)) if a else None

        return {
            "requests": len(finish),
            "wall_s": wall,
            "arrival_span_s": span,
            "offered_req_per_s": len(requests) / span if span > 0 else None,
            "achieved_req_per_s": len(finish) / wall if wall > 0 else None,
            "element_matrices_per_s": elements / wall if wall > 0 else None,
            "assembly_ms": {"p50": pct(lat_asm, 50), "p99": pct(lat_asm, 99),
                            "mean": float(np.mean(lat_asm) * 1e3) if lat_asm else None},
            "reassembly_ms": {"p50": pct(lat_re, 50), "p99": pct(lat_re, 99),
                              "mean": float(np.mean(lat_re) * 1e3) if lat_re else None},
            "queue_wait_ms": {"p50": pct(queue_wait, 50), "p99": pct(queue_wait, 99)},
            "max_pending": max_pending,
            "slots": self.nslots,
        }

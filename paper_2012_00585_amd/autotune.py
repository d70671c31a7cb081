"""Autotuner: scatter strategy and launch shape per mesh size class.

A size class is (nodes per element, DOFs per node, size bucket), the bucket
being floor(log2(n_elem) / 2).  For each class the tuner times every
candidate on the class's largest mesh with single-mesh calls -- row-owned
(rows per wavefront 1 or 2, batch 8 or 16), atomic and coloured (lanes per
element 16 ... 64) -- keeps the fastest and applies it to every handle of
the class with ``Pattern.tune``.  Results do not depend on the choice; only
time does.  Choices can be saved to and loaded from a JSON file.

``autotune_batch`` then re-times, for every class, the leading single-mesh
candidates inside the batched launch they configure (the batch runs its
own kernels per path, whose speed need not follow the single-mesh ranking)
and keeps, class by class, the candidate with the fastest whole-batch
replay.
"""
from __future__ import annotations

import json
import math
from dataclasses import asdict, dataclass

import torch

from . import (FMT_CSR, SCATTER_ATOMIC, SCATTER_COLOURED, SCATTER_OWNER,
               TUNE_OWNER_BATCH, TUNE_OWNER_ROWS, TUNE_STRATEGY, TUNE_THREADS_PER_ELEM,
               BUILD_COLOUR, FeasmError, assemble_crac, assemble_csr)


@dataclass
class Choice:
    strategy: int
    tpe: int = 0
    rows: int = 0
    batch: int = 0
    ms: float = float("nan")

    def label(self):
        name = {SCATTER_OWNER: "owner", SCATTER_ATOMIC: "atomic", SCATTER_COLOURED: "coloured"}
        s = name[self.strategy]
        if self.strategy == SCATTER_OWNER:
            return f"{s}(rows={self.rows or 'auto'},batch={self.batch or 8})"
        return f"{s}(tpe={self.tpe or 'auto'})"


def size_class(p):
    return (p.nodes_per_elem, p.dofs_per_node, int(math.log2(max(p.n_elem, 1)) // 2))


def candidates(p, max_tpe=64):
    n2 = p.n * p.n
    out = []
    dn = p.dofs_per_node * p.n
    rows_opts = (1, 2) if dn > 64 else (0,)
    for rows in rows_opts:
        for batch in (8, 16):
            out.append(Choice(SCATTER_OWNER, rows=rows, batch=batch))
    for tpe in (16, 32, 64, 128, 256):
        if tpe > max_tpe or n2 > 16 * tpe:
            continue
        out.append(Choice(SCATTER_ATOMIC, tpe=tpe))
        if p.flags & BUILD_COLOUR:
            out.append(Choice(SCATTER_COLOURED, tpe=tpe))
    return out


def apply(p, c: Choice):
    p.tune(TUNE_STRATEGY, c.strategy)
    p.tune(TUNE_THREADS_PER_ELEM, c.tpe)
    p.tune(TUNE_OWNER_ROWS, c.rows)
    p.tune(TUNE_OWNER_BATCH, c.batch)


def _time(fn, reps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune_one(p, ke, values, fmt, reps=5, warmup=2, max_tpe=64):
    """Time every candidate on one mesh; returns choices sorted fastest first."""
    fn = assemble_csr if fmt == FMT_CSR else assemble_crac
    res = []
    for c in candidates(p, max_tpe):
        try:
            apply(p, c)
        except FeasmError:
            continue
        # a full assembly: the row-owned strategy writes values once, the
        # others reset them first
        c.ms = _time(lambda: fn(p, ke, values, c.strategy), reps, warmup)
        res.append(c)
    res.sort(key=lambda c: c.ms)
    return res


def autotune(patterns, kes, values, fmt, reps=5, warmup=2, max_tpe=64, log=None):
    """Tune each size class on its largest mesh and apply the winner to the class.

    Returns {class: [Choice, ...] sorted}.  ``max_tpe`` caps lanes per element
    (64 for the batched launch)."""
    classes = {}
    for i, p in enumerate(patterns):
        classes.setdefault(size_class(p), []).append(i)
    out = {}
    for cls, members in sorted(classes.items()):
        rep = max(members, key=lambda i: patterns[i].n_elem)
        ranked = tune_one(patterns[rep], kes[rep], values[rep], fmt, reps, warmup, max_tpe)
        out[cls] = ranked
        for i in members:
            apply(patterns[i], ranked[0])
        if log:
            log(f"[autotune] class k={cls[0]} d={cls[1]} bucket={cls[2]} ({len(members)} meshes, "
                f"rep {patterns[rep].n_elem} elements): "
                + ", ".join(f"{c.label()} {c.ms:.3f} ms" for c in ranked[:4]))
    return out


def autotune_batch(patterns, kes, values, fmt, make_batch, reps=3, warmup=1, top=3, rounds=3,
                   log=None):
    """Tune for the batched launch: single-mesh ranking per class first, then,
    class by class (largest work first), each of the class's ``top`` leading
    candidates (and the row-owned one with one row per wavefront) applied to
    the whole class, one ``make_batch(patterns)`` each; the batches are
    replayed in turn for ``rounds`` rounds (so that clock drift hits every
    candidate alike) and each keeps its fastest round; the fastest candidate
    stays.  Returns ({class: [Choice ranked by batch time]}, batch time in ms
    of the final choice)."""
    single = autotune(patterns, kes, values, fmt, reps=reps, warmup=warmup, max_tpe=64, log=log)
    classes = {}
    for i, p in enumerate(patterns):
        classes.setdefault(size_class(p), []).append(i)
    work = {c: sum(patterns[i].n_elem * patterns[i].n ** 2 for i in m) for c, m in classes.items()}

    out = {}
    current = None
    for cls in sorted(classes, key=lambda c: -work[c]):
        members = classes[cls]
        tried = list(single[cls][:top])
        if not any(c.strategy == SCATTER_OWNER and c.rows in (0, 1) for c in tried):
            tried += [c for c in single[cls] if c.strategy == SCATTER_OWNER and c.rows in (0, 1)][:1]
        batches = []
        try:
            for c in tried:
                for i in members:
                    apply(patterns[i], c)
                batches.append(make_batch(patterns))  # the batch keeps the tuning it was built with
            best = [float("inf")] * len(tried)
            for _ in range(rounds):
                for j, b in enumerate(batches):
                    best[j] = min(best[j], _time(lambda: b.assemble(kes, values), reps, warmup))
        finally:
            for b in batches:
                b.free()
        timed = sorted((Choice(c.strategy, c.tpe, c.rows, c.batch, t) for c, t in zip(tried, best)),
                       key=lambda c: c.ms)
        for i in members:
            apply(patterns[i], timed[0])
        current = timed[0].ms
        out[cls] = timed
        if log:
            log(f"[autotune] batch, class k={cls[0]} d={cls[1]} bucket={cls[2]}: "
                + ", ".join(f"{c.label()} {c.ms:.3f} ms" for c in timed))
    return out, current


def save(choices, path):
    with open(path, "w") as f:
        json.dump({json.dumps(list(k)): [asdict(c) for c in v] for k, v in choices.items()}, f,
                  indent=1)


def load(path):
    with open(path) as f:
        raw = json.load(f)
    return {tuple(json.loads(k)): [Choice(**c) for c in v] for k, v in raw.items()}


def apply_choices(patterns, choices):
    for p in patterns:
        ranked = choices.get(size_class(p))
        if ranked:
            apply(p, ranked[0])

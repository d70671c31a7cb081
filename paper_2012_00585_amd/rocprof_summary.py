"""Summaries of rocprofv3 runs of the library's kernels.

rocprofv3 writes a SQLite ("rocpd") database per run.  This module reads

* a ``--kernel-trace`` database: per-kernel dispatch count and duration;
* ``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE`` databases: per-dispatch HBM
  read and write counters (KiB).  Each counter is scaled by what it reads for
  a plain device copy of known size found in the same run (bench.py's
  ``--copy-mib``), so the bytes are real bytes.

and writes a short markdown summary with the numbers and the commands that
produced them.  With ``--shares`` it writes instead each kernel's share of the
summed kernel time of a trace (optionally of its busiest window,
``--window-s``), e.g. for a serving run.  ``source_hash()`` fingerprints the HIP sources, so a reader
can tell whether a summary still describes the current kernels.

    python -m paper_2012_00585_amd.rocprof_summary --trace T.db --fetch F.db \
        --write W.db --kernel k_owner_rows --copy-mib 1024 --workload hex64 \
        --command "..." --out profiles/k_owner_rows_hex64.md
"""
from __future__ import annotations

import argparse
import bisect
import collections
import glob
import hashlib
import os
import re
import sqlite3

PKG = os.path.dirname(os.path.abspath(__file__))


def _code_only(text: str) -> str:
    """C/C++ source without comments and blank space: what the compiler sees."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":  # string or character literal, kept whole
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_hash() -> str:
    """Fingerprint of the HIP sources' code (comments and blank space do not
    count), so a summary can be matched to the kernels it measured."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(PKG, "csrc", "*"))):
        with open(f, encoding="utf-8") as fh:
            h.update(os.path.basename(f).encode())
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def kernel_durations(db):
    """{kernel name: [durations in us]} from a kernel-trace database."""
    c = sqlite3.connect(db)
    out = collections.defaultdict(list)
    for name, start, end in c.execute("select name, start, end from kernels order by start"):
        out[name].append((end - start) / 1e3)
    return dict(out)


def counter_values(db, counter):
    """{kernel name: [per-dispatch values]} of one counter."""
    c = sqlite3.connect(db)
    out = collections.defaultdict(list)
    for name, cn, val in c.execute(
            "select kernel_name, counter_name, value from counters_collection"):
        if cn == counter:
            out[name].append(float(val))
    return dict(out)


def _match(d, pattern):
    keys = [k for k in d if re.search(pattern, k)]
    return keys


def copy_factor(values, copy_mib):
    """Bytes per counter unit, from the largest copyBuffer dispatch of copy_mib MiB."""
    keys = _match(values, r"copyBuffer|copy")
    best = 0.0
    for k in keys:
        best = max(best, max(values[k]))
    if best <= 0:
        return None
    return copy_mib * (1 << 20) / best


def summarize(trace, fetch, write, kernel, copy_mib, workload, command, algorithmic_bytes=None,
              title=None):
    durs = kernel_durations(trace)
    names = _match(durs, kernel)
    if not names:
        raise SystemExit(f"kernel {kernel!r} not in trace; have {sorted(durs)[:8]}")
    lines = [f"# {title or kernel} on {workload}", ""]
    lines.append(f"source hash: {source_hash()}")
    lines.append("")
    lines.append("Commands (run from the repository root on the GPU host):")
    lines.append("")
    for c in command:
        lines.append(f"    {c}")
    lines.append("")
    # "warm" leaves out each kernel's first dispatch, which also pays for
    # first-touch page mapping of its buffers
    lines.append("| kernel | dispatches | mean us | warm mean us | median us | min us |")
    lines.append("|---|---|---|---|---|---|")
    for nme in sorted(names, key=lambda x: -len(durs[x])):
        v = durs[nme]
        warm = v[1:] if len(v) > 1 else v
        med = sorted(v)[len(v) // 2]
        lines.append(f"| {nme[:100]} | {len(v)} | {sum(v) / len(v):.2f} | "
                     f"{sum(warm) / len(warm):.2f} | {med:.2f} | {min(v):.2f} |")
    lines.append("")
    copies = [d for k in _match(durs, r"copyBuffer|copy") for d in durs[k]]
    if copies and copy_mib:
        # the copy kernel of the same run reads and writes copy_mib MiB: a
        # practical ceiling for streaming kernels on this device
        big = max(copies)
        best = min(d for d in copies if d > 0.5 * big)  # fastest of the large copies
        lines.append(f"Device copy of {copy_mib} MiB in the same run: {best:.1f} us, "
                     f"{2 * copy_mib * (1 << 20) / (best * 1e-6) / 1e9:.0f} GB/s read+write")
        lines.append("")
    if algorithmic_bytes:
        # one step launches every matched kernel once
        mean = sum(sum(durs[n]) / len(durs[n]) for n in names)
        lines.append(f"algorithmic bytes / summed mean duration: "
                     f"{algorithmic_bytes / (mean * 1e-6) / 1e9:.0f} GB/s")
        lines.append("")
    fv = counter_values(fetch, "FETCH_SIZE") if fetch else {}
    wv = counter_values(write, "WRITE_SIZE") if write else {}
    ff = copy_factor(fv, copy_mib) if fv else None
    wf = copy_factor(wv, copy_mib) if wv else None
    if fv and wv and ff and wf:
        lines.append(f"Counter scale from a {copy_mib} MiB device copy: FETCH_SIZE x {ff:.1f} "
                     f"bytes/unit, WRITE_SIZE x {wf:.1f} bytes/unit")
        lines.append("")
        lines.append("| kernel | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | HBM bytes/dispatch |")
        lines.append("|---|---|---|---|")
        total = 0.0
        for nme in names:
            f = fv.get(nme, [])
            w = wv.get(nme, [])
            if not f or not w:
                continue
            fa, wa = sum(f) / len(f), sum(w) / len(w)
            tb = fa * ff + wa * wf
            total += tb
            lines.append(f"| {nme[:100]} | {fa:.1f} | {wa:.1f} | {tb:.0f} |")
        lines.append("")
        # one step launches every matched kernel once
        lines.append(f"traffic_bytes_per_launch: {total:.0f}")
        if algorithmic_bytes:
            lines.append(f"algorithmic_bytes_per_launch: {algorithmic_bytes}")
            lines.append(f"traffic_over_algorithmic: {total / algorithmic_bytes:.3f}")
    lines.append("")
    return "\n".join(lines)


def _short_name(name):
    """Kernel identifier with its template arguments, without the namespace
    and parameter list."""
    m = re.search(r"(k_\w+)(<[^()]*>)?", name)
    return m.group(1) + (m.group(2) or "") if m else name.split("(")[0][-60:]


def shares(trace, window_s, command, workload, title=None):
    """Each kernel's share of the summed kernel time, over the whole trace or
    over the window of window_s seconds with the most dispatches (the
    saturated part of a serving run), and how busy the device was there."""
    c = sqlite3.connect(trace)
    rows = list(c.execute("select name, start, end from kernels order by start"))
    if not rows:
        raise SystemExit("no kernels in trace")
    lo, hi = 0, len(rows)
    if window_s:
        starts = [r[1] for r in rows]
        w, step = int(window_s * 1e9), int(0.25e9)
        best, t = (-1, 0, 0), rows[0][1]
        while t <= rows[-1][2]:
            a, b = bisect.bisect_left(starts, t), bisect.bisect_left(starts, t + w)
            if b - a > best[0]:
                best = (b - a, a, b)
            t += step
        _, lo, hi = best
    sel = rows[lo:hi]
    tot, cnt = collections.defaultdict(float), collections.Counter()
    for name, s0, e0 in sel:
        k = _short_name(name)
        tot[k] += (e0 - s0) / 1e6
        cnt[k] += 1
    summed = sum(tot.values())
    ivs = sorted((s0, e0) for _, s0, e0 in sel)
    busy, cs, ce = 0, ivs[0][0], ivs[0][1]
    for s0, e0 in ivs[1:]:
        if s0 > ce:
            busy, cs, ce = busy + ce - cs, s0, e0
        else:
            ce = max(ce, e0)
    busy += ce - cs
    span = ivs[-1][1] - ivs[0][0]
    lines = [f"# {title or 'kernel time shares'} on {workload}", "",
             f"source hash: {source_hash()}", "",
             "Commands (run from the repository root on the GPU host):", ""]
    lines += [f"    {x}" for x in command] + [""]
    where = (f"the {window_s:g} s window with the most dispatches" if window_s
             else "the whole trace")
    lines.append(f"Over {where}: {len(sel)} dispatches, device busy (union of kernel "
                 f"intervals) for {100 * busy / span:.1f}% of its {span / 1e6:.1f} ms; kernels of "
                 f"concurrent streams overlap, so the summed time ({summed:.1f} ms) exceeds it.")
    lines.append("")
    lines.append("| kernel | summed ms | share | dispatches | mean us |")
    lines.append("|---|---|---|---|---|")
    for k, v in sorted(tot.items(), key=lambda x: -x[1]):
        if v < 0.001 * summed:
            continue
        lines.append(f"| {k[:100]} | {v:.1f} | {100 * v / summed:.1f}% | {cnt[k]} | "
                     f"{1e3 * v / cnt[k]:.1f} |")
    lines.append("")
    return "\n".join(lines)


def read_traffic(path):
    """(traffic bytes per launch, source hash) from a summary, or (None, None)."""
    if not os.path.exists(path):
        return None, None
    text = open(path).read()
    m = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    h = re.search(r"source hash: (\w+)", text)
    return (int(m.group(1)) if m else None), (h.group(1) if h else None)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--kernel", help="regular expression of the kernel name")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--workload", default="hex64")
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--algorithmic-bytes", type=int)
    ap.add_argument("--title")
    ap.add_argument("--out")
    ap.add_argument("--shares", action="store_true",
                    help="kernel time shares of the trace instead of one kernel's summary")
    ap.add_argument("--window-s", type=float, default=0.0,
                    help="with --shares: the window of this many seconds with most dispatches")
    a = ap.parse_args()
    if a.shares:
        text = shares(a.trace, a.window_s, a.command, a.workload, a.title)
    else:
        if not a.kernel:
            ap.error("--kernel is required without --shares")
        text = summarize(a.trace, a.fetch, a.write, a.kernel, a.copy_mib, a.workload, a.command,
                         a.algorithmic_bytes, a.title)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    print(text)


if __name__ == "__main__":
    main()

"""Benchmark of FE sparse-matrix assembly on one MI355X.

Workload (default): the 64^3 trilinear hex mesh, 3 DOFs per node (823 875
DOFs, 262 144 elements), 24 x 24 FP64 SPD element matrices (B B^T/24 + I,
seed 0); CSR and CRAC patterns built once on the device.

A step is one numeric assembly of all 262 144 element matrices into the
global values array (reset + scatter-add), with inputs resident in HBM.
`value` is element matrices assembled per second for the fastest full
assembly variant; every variant is reported under "variants", value-only
re-assembly latency under "reassembly_ms", the symbolic phase under
"pattern_build_ms".  Progress goes to stderr; stdout gets one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload hex64|quad64|tet40]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("element matrices assembled/s + effective HBM GB/s (64³ hex); "
          "p50/p99 reassembly")
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def stats(ms):
    a = np.asarray(ms, dtype=np.float64)
    return {"mean": float(a.mean()), "min": float(a.min()), "p50": float(np.percentile(a, 50)),
            "p99": float(np.percentile(a, 99)), "n": int(a.size)}


def time_calls(fn, reps, warmup):
    """Per-call device time (ms) from HIP events on torch's current stream,
    which is the stream the library launches on."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    for i in range(reps):
        starts[i].record()
        fn()
        ends[i].record()
    torch.cuda.synchronize()
    return [s.elapsed_time(e) for s, e in zip(starts, ends)]


def workload(name):
    from fe_inputs import configs

    if name == "hex64":
        return configs.hex64(), "hex64: 64^3 Q1 hex, 3 DOF/node, 24x24 SPD FP64 Ke, seed 0"
    if name == "quad64":
        return configs.quad64(), "quad64: 64^2 Q1 quad, 1 DOF/node, 4x4 zero-row-sum FP64 Ke, seed 0"
    if name == "tet40":
        return configs.tet40(), ("tet40: 40^3 cubes x 6 tet10, permuted nodes (seed 0), "
                                 "3 DOF/node, 30x30 SPD FP64 Ke, seed 0")
    raise ValueError(name)


def algorithmic_bytes(w, p, fmt, strategy="atomic"):
    """Bytes a scatter method must move per assembly: Ke once, conn once, the
    format's index arrays once, values read and written once (the reset is
    counted separately).

    The row-owned method needs less: Ke once, values written once (never
    read), the node->element incidence once, and the index data of the first
    DOF row of every node (the other d-1 rows of a node share it)."""
    E, k, n, d = w.n_elem, w.nodes_per_elem, w.n, w.dofs_per_node
    if strategy == "record":
        # row-owned re-assembly from the recorded lookup map: Ke, values
        # written once, the incidence, the map (k offsets per entry) and the
        # row extents
        return E * n * n * 8 + p.nnz * 8 + E * k * 4 + E * k * k * 4 + 2 * (w.n_nodes + 1) * 8
    if strategy == "owner":
        b = E * n * n * 8 + p.nnz * 8 + E * k * 4 + E * k * 4 + (w.n_nodes + 1) * 8
        if fmt == "csr":
            b += (w.n_nodes + 1) * 4 * 2 + (p.nnz // d) * 4
        else:
            b += (w.n_nodes + 1) * 4 * 2 + ((p.n_ca - 2) // d + 2 * w.n_nodes) * 4
        return b
    b = E * n * n * 8 + E * k * 4 + 2 * p.nnz * 8
    if fmt == "csr":
        b += (p.n_rows + 1) * 4 + p.nnz * 4
    else:
        b += (p.n_rows + 1) * 4 + p.n_ca * 4
    return b


def cpu_baseline(w, ke, reps):
    """The serial oracle's numeric phase on one pinned core."""
    from oracle import oracle

    old = os.sched_getaffinity(0)
    core = min(old)
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        rp, ci = oracle.pattern(w.conn, w.dofs_per_node, w.n_nodes)
        pattern_s = time.perf_counter() - t0
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.assemble(w.conn, w.dofs_per_node, ke, rp, ci, with_abs=False)
            ts.append(time.perf_counter() - t0)
    finally:
        os.sched_setaffinity(0, old)
    mean = float(np.mean(ts))
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": w.n_elem / mean, "unit": "element matrices/s", "cores": 1, "kind": "oracle",
            "sample": (f"whole {w.name} numeric phase (values reset + sequential scatter with "
                       f"binary search), {reps} reps, pinned to core {core}; mean "
                       f"{mean * 1e3:.1f} ms, min {min(ts) * 1e3:.1f} ms; the oracle's pattern "
                       f"build (timed apart) {pattern_s * 1e3:.0f} ms; host: {model}, "
                       f"{os.cpu_count()} logical CPUs")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="hex64",
                    choices=["hex64", "quad64", "tet40", "batch512", "serve", "refine", "hex8"])
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="mean arrivals per second")
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--batch-count", type=int, default=512,
                    help="batch512: number of meshes (the mix is the first N of the 512)")
    ap.add_argument("--cpu-reps", type=int, default=3, help="0 skips the oracle baseline")
    ap.add_argument("--only", default="", help="comma-separated variants to time (default: all)")
    ap.add_argument("--sections", default="reassembly,spmv,tet40,batch512,serve",
                    help="single-mesh workloads: the sections reported after the variants, "
                         "comma-separated from reassembly, spmv, and (hex64 only) tet40, "
                         "batch512, serve (empty: none, e.g. for a profile of the assembly "
                         "kernels alone)")
    ap.add_argument("--section-serve-seconds", type=float, default=2.0,
                    help="length of each serving scenario in the serve section")
    ap.add_argument("--hex8-pipe", type=int, default=0,
                    help="hex8 workload: fused-kernel setting (0 auto, n blocks per CU, -1 off)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run 3 plain device copies of this many MiB (a known-size "
                         "reference for hardware byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(rows would be sharded in contiguous blocks per GPU); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2012_00585_amd as feasm

    feasm.load()
    dev = torch.device("cuda:0")
    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.copy_mib} MiB three times (counter reference)")
        del src, dst
    if args.workload == "batch512":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "refine":
        return bench_refine(args)
    if args.workload == "hex8":
        return bench_hex8(args)
    w, wdesc = workload(args.workload)
    log(f"[bench] {wdesc}: generating element matrices")
    ke = w.ke()
    conn_d = torch.from_numpy(w.conn).to(dev)
    ke_d = torch.from_numpy(ke).to(dev)
    torch.cuda.synchronize()

    log("[bench] pattern_build")
    flags = feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_COLOUR
    pb_ms = []
    for _ in range(3):
        t0 = time.perf_counter()
        p = feasm.pattern_build(conn_d, w.dofs_per_node, w.n_nodes, flags)
        pb_ms.append((time.perf_counter() - t0) * 1e3)
        if _ < 2:
            p.free()
    # the same pattern with element tiles: the atomic scatter with per-tile
    # LDS sums (one write per distinct entry of a tile)
    p_t = feasm.pattern_build(conn_d, w.dofs_per_node, w.n_nodes,
                              feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_TILES)
    values = torch.zeros(p.nnz, dtype=torch.float64, device=dev)

    A, C, O, S, ACC = (feasm.SCATTER_ATOMIC, feasm.SCATTER_COLOURED, feasm.SCATTER_OWNER,
                       feasm.SCATTER_SPIN, feasm.ACCUMULATE)
    full = {
        "csr_owner": lambda: feasm.assemble_csr(p, ke_d, values, O),
        "crac_owner": lambda: feasm.assemble_crac(p, ke_d, values, O),
        "csr_atomic": lambda: feasm.assemble_csr(p, ke_d, values, A),
        "crac_atomic": lambda: feasm.assemble_crac(p, ke_d, values, A),
        "csr_atomic_tiled": lambda: feasm.assemble_csr(p_t, ke_d, values, A),
        "crac_atomic_tiled": lambda: feasm.assemble_crac(p_t, ke_d, values, A),
        "csr_coloured": lambda: feasm.assemble_csr(p, ke_d, values, C),
        "crac_coloured": lambda: feasm.assemble_crac(p, ke_d, values, C),
        "csr_spin": lambda: feasm.assemble_csr(p, ke_d, values, S),
        "crac_spin": lambda: feasm.assemble_crac(p, ke_d, values, S),
    }
    scatter_only = {
        "csr_owner": lambda: feasm.assemble_csr(p, ke_d, values, O),
        "crac_owner": lambda: feasm.assemble_crac(p, ke_d, values, O),
        "csr_atomic": lambda: feasm.assemble_csr(p, ke_d, values, A | ACC),
        "crac_atomic": lambda: feasm.assemble_crac(p, ke_d, values, A | ACC),
        "csr_atomic_tiled": lambda: feasm.assemble_csr(p_t, ke_d, values, A | ACC),
        "crac_atomic_tiled": lambda: feasm.assemble_crac(p_t, ke_d, values, A | ACC),
        "csr_coloured": lambda: feasm.assemble_csr(p, ke_d, values, C | ACC),
        "crac_coloured": lambda: feasm.assemble_crac(p, ke_d, values, C | ACC),
        "csr_spin": lambda: feasm.assemble_csr(p, ke_d, values, S | ACC),
        "crac_spin": lambda: feasm.assemble_crac(p, ke_d, values, S | ACC),
    }
    p_r = None
    if args.workload == "tet40":
        # scattered node numbering: the row-owned lookup record built with the
        # pattern (on grid-numbered meshes it only adds reads; the hex64
        # re-assembly figures, which use the same record, show that)
        p_r = feasm.pattern_build(conn_d, w.dofs_per_node, w.n_nodes,
                                  feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_OWNER_MAP)
        for name, fn in (("csr_owner_record", feasm.assemble_csr),
                         ("crac_owner_record", feasm.assemble_crac)):
            full[name] = scatter_only[name] = (lambda f=fn: f(p_r, ke_d, values, O))
    reps = max(args.steps, 5)
    variants = {}
    if args.only:
        keep = set(args.only.split(","))
        full = {k: v for k, v in full.items() if k in keep}
    for name, fn in full.items():
        log(f"[bench] variant {name}")
        t_full = stats(time_calls(fn, reps, args.warmup))
        t_sc = stats(time_calls(scatter_only[name], reps, args.warmup))
        fmt, strategy = name.split("_", 1)
        nbytes = algorithmic_bytes(w, p, fmt, "record" if strategy == "owner_record" else strategy)
        variants[name] = {
            "assemble_ms": t_full,
            "scatter_only_ms": t_sc,
            "elements_per_s": w.n_elem / (t_full["mean"] * 1e-3),
            "algorithmic_bytes": nbytes,
            "effective_GBps": nbytes / (t_full["mean"] * 1e-3) / 1e9,
            "scatter_GBps": nbytes / (t_sc["mean"] * 1e-3) / 1e9,
            # the element matrices alone: the stream every strategy must read
            "Ke_only_GBps": w.n_elem * w.n * w.n * 8 / (t_sc["mean"] * 1e-3) / 1e9,
        }
        if strategy.startswith("atomic"):
            # one FP64 atomic add per element-matrix entry (the second ceiling
            # of this method besides HBM bandwidth)
            variants[name]["atomic_adds_per_launch"] = w.n_elem * w.n * w.n
            variants[name]["atomic_adds_per_s"] = w.n_elem * w.n * w.n / (t_sc["mean"] * 1e-3)
    sections = set(filter(None, args.sections.split(",")))
    unknown = sections - {"reassembly", "spmv", "tet40", "batch512", "serve"}
    if unknown:
        raise SystemExit(f"--sections: unknown {sorted(unknown)}")
    reasm = {}
    if "reassembly" in sections:
        log("[bench] value-only re-assembly latency")
        for name, fmt, sc in (("csr_atomic", feasm.FMT_CSR, A), ("crac_atomic", feasm.FMT_CRAC, A),
                              ("csr_owner", feasm.FMT_CSR, O), ("crac_owner", feasm.FMT_CRAC, O)):
            fn = (lambda f=fmt, c=sc: feasm.reassemble_values(p, f, ke_d, values, c))
            reasm[name] = stats(time_calls(fn, max(reps, 50), args.warmup))
            if sc == O:
                nb = algorithmic_bytes(w, p, name.split("_")[0], "record")
                reasm[name]["algorithmic_bytes"] = nb
                reasm[name]["GBps"] = nb / (reasm[name]["mean"] * 1e-3) / 1e9

    spmv = {}
    if "spmv" in sections:
        log("[bench] matrix-vector product y = G x")
        xv = torch.randn(p.n_rows, dtype=torch.float64, device=dev)
        yv = torch.empty_like(xv)
        # values, the format's index arrays and x read once, y written once
        for name, fn, index_bytes in (("csr", feasm.spmv_csr, (p.n_rows + 1) * 4 + p.nnz * 4),
                                      ("crac", feasm.spmv_crac, (p.n_rows + 1) * 4 + p.n_ca * 4)):
            st = stats(time_calls(lambda f=fn: f(p, values, xv, yv), max(reps, 50), args.warmup))
            nb = p.nnz * 8 + index_bytes + 2 * p.n_rows * 8
            st["algorithmic_bytes"] = nb
            st["GBps"] = nb / (st["mean"] * 1e-3) / 1e9
            spmv[name] = st

    best = min(variants, key=lambda k: variants[k]["assemble_ms"]["mean"])
    step = full[best]
    log(f"[bench] timed steps: {best} x {args.steps}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    ms_per_step = t0.elapsed_time(t1) / args.steps

    v = variants[best]
    fmt, strategy = best.split("_", 1)
    kernel_ms = v["scatter_only_ms"]["mean"]
    spec_bytes = algorithmic_bytes(w, p, fmt, "atomic")
    achieved = v["algorithmic_bytes"] / (kernel_ms * 1e-3) / 1e9
    # HBM traffic measured by rocprofv3 counters for this variant and workload,
    # valid only while the kernel sources are those the counters were taken on
    from paper_2012_00585_amd import rocprof_summary

    prof = os.path.join(ROOT, "profiles", f"{best}_{args.workload}.md")
    tbytes, thash = rocprof_summary.read_traffic(prof)
    traffic = None
    if tbytes is not None and thash == rocprof_summary.source_hash():
        traffic = tbytes
    line = {
        "metric": METRIC,
        "value": w.n_elem / (ms_per_step * 1e-3),
        "unit": "element matrices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wdesc, "n_elem": w.n_elem, "n_rows": p.n_rows, "nnz": p.nnz,
                   "n_ca": p.n_ca, "n_colours": p.n_colours, "step_variant": best,
                   "step": "values reset + scatter-add of every element matrix"},
        # the step's own algorithmic bytes (those its kernel must move) over
        # the step time
        "effective_GBps": v["algorithmic_bytes"] / (ms_per_step * 1e-3) / 1e9,
        "effective_GBps_note": (f"algorithmic bytes of the step's variant ({best}: "
                                f"{v['algorithmic_bytes']} B) over the step time"),
        # for comparison across strategies only: the bytes a scatter method
        # (atomic or coloured) moves, over the same step time; the row-owned
        # step does not move them
        "scatter_method_equivalent_GBps": spec_bytes / (ms_per_step * 1e-3) / 1e9,
        # rocprofv3-measured HBM bytes of the dominant kernel over its live
        # duration (null while the counters are stale)
        "traffic_GBps": traffic / (kernel_ms * 1e-3) / 1e9 if traffic else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_source": os.path.relpath(prof, ROOT) if traffic else None,
                     "kernel": (f"row-owned kernels of one call ({best}; one launch, or two "
                                f"where light and heavy rows are split)"
                                if strategy.startswith("owner") else
                                f"k_assemble ({best}, scatter only)"),
                     "bytes_per_launch": v["algorithmic_bytes"],
                     "kernel_ms": kernel_ms},
        "reassembly_ms": reasm,
        "spmv_ms": spmv,
        "pattern_build_ms": {"runs": pb_ms},
        "variants": variants,
    }
    if args.cpu_reps > 0:
        log("[bench] CPU baseline (serial oracle)")
        line["cpu_baseline"] = cpu_baseline(w, ke, args.cpu_reps)
    p.free()
    p_t.free()
    if p_r is not None:
        p_r.free()
    del ke_d, values, ke
    if args.workload == "hex64":
        # the other workloads, compact, in the same line
        if "tet40" in sections:
            line["tet40"] = tet40_section(args)
        if "batch512" in sections:
            out, (pats, _k, _v, b, _s) = batch_section(args, colour=False)
            b.free()
            for q in pats:
                q.free()
            del _k, _v
            line["batch512"] = out
        if "serve" in sections:
            line["serve"] = serve_section(args, args.serve_rate, args.section_serve_seconds)
    print(json.dumps(line), flush=True)


def tet40_section(args):
    """The permuted tet10 mesh (40^3 cubes x 6, 3 DOFs per node), element
    matrices from the device generator (30 x 30 SPD, key 0): step time and
    HBM roofline fraction of the row-owned assembly, and the atomic
    strategy beside it."""
    import torch

    import paper_2012_00585_amd as feasm

    w, wdesc = workload("tet40")
    dev = torch.device("cuda:0")
    log("[bench] tet40 section: pattern build")
    conn_d = torch.from_numpy(w.conn).to(dev)
    t0 = time.perf_counter()
    p = feasm.pattern_build(conn_d, w.dofs_per_node, w.n_nodes, feasm.BUILD_CSR | feasm.BUILD_CRAC)
    build_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    p_rec = feasm.pattern_build(conn_d, w.dofs_per_node, w.n_nodes,
                                feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_OWNER_MAP)
    build_rec_ms = (time.perf_counter() - t0) * 1e3
    ke_d = feasm.generate_ke(feasm.RECIPE_SPD, w.n_elem, w.n, 0)
    values = torch.zeros(p.nnz, dtype=torch.float64, device=dev)
    O, A, ACC = feasm.SCATTER_OWNER, feasm.SCATTER_ATOMIC, feasm.ACCUMULATE
    reps = max(args.steps, 5)
    out = {"workload": wdesc.replace("30x30 SPD FP64 Ke, seed 0",
                                     "30x30 SPD FP64 Ke from the device generator, key 0"),
           "n_elem": w.n_elem, "nnz": p.nnz, "n_ca": p.n_ca, "pattern_build_ms": build_ms,
           "pattern_build_with_record_ms": build_rec_ms}
    for name, q, fn, sc in (("crac_owner", p, feasm.assemble_crac, O),
                            ("csr_owner", p, feasm.assemble_csr, O),
                            ("crac_owner_record", p_rec, feasm.assemble_crac, O),
                            ("csr_owner_record", p_rec, feasm.assemble_csr, O),
                            ("crac_atomic", p, feasm.assemble_crac, A),
                            ("csr_atomic", p, feasm.assemble_csr, A)):
        full = stats(time_calls(lambda f=fn, c=sc, q=q: f(q, ke_d, values, c), reps, args.warmup))
        # the row-owned strategy writes every value once and has no reset
        # pass: its full assembly is its scatter
        sco = full if sc == O else stats(time_calls(lambda f=fn, c=sc: f(p, ke_d, values, c | ACC),
                                                    reps, args.warmup))
        fmt, strategy = name.split("_")[:2]
        if name.endswith("_record"):
            strategy = "record"  # the record replaces conn and the row index words
        nb = algorithmic_bytes(w, p, fmt, strategy)
        out[name] = {"assemble_ms": full["mean"], "scatter_only_ms": sco["mean"],
                     "algorithmic_bytes": nb,
                     "GBps": nb / (sco["mean"] * 1e-3) / 1e9,
                     "roofline_frac": nb / (sco["mean"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
        log(f"[bench]   tet40 {name}: {full['mean']:.3f} ms (scatter only {sco['mean']:.3f} ms, "
            f"{out[name]['roofline_frac']:.2f} of HBM peak)")
    best = min(("crac_owner", "csr_owner", "crac_owner_record", "csr_owner_record"),
               key=lambda k: out[k]["assemble_ms"])
    out["step_variant"] = best
    out["step_ms"] = out[best]["assemble_ms"]
    out["step_roofline_frac"] = out[best]["roofline_frac"]
    out["elements_per_s"] = w.n_elem / (out["step_ms"] * 1e-3)
    p.free()
    p_rec.free()
    return out


def _oracle_mesh(spec):
    """One mesh of the batch mix through the serial oracle (pattern, then
    assembly); returns (elements, seconds).  The oracle's work does not
    depend on the values, so the paper's all-ones dummy element stands in
    for the generated matrices."""
    from fe_inputs import matrices, meshes
    from oracle import oracle

    conn, nn = meshes.quad_mesh(spec.size) if spec.kind == "quad" else meshes.hex_mesh(spec.size)
    E, k = conn.shape
    d = spec.dofs_per_node
    ke = matrices.ke_ones(E, k * d)
    t0 = time.perf_counter()
    rp, ci = oracle.pattern(conn, d, nn)
    oracle.assemble(conn, d, ke, rp, ci, with_abs=False)
    return E, time.perf_counter() - t0


def batch_cpu_baseline(specs, count):
    """The serial oracle on the first `count` meshes of the mix, one mesh per
    process on every host core (independent meshes, no threading inside an
    assembly); pattern + numeric phase."""
    import multiprocessing as mp

    sample = list(specs[:count])
    cores = os.cpu_count() or 1
    # fork: the workers never touch the GPU
    with mp.get_context("fork").Pool(min(cores, len(sample))) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_mesh, sample, chunksize=1)
        wall = time.perf_counter() - t0
    E = sum(r[0] for r in res)
    busy = sum(r[1] for r in res)
    return {"value": E / wall, "unit": "element matrices/s", "cores": min(cores, len(sample)),
            "kind": "oracle",
            "sample": (f"first {len(sample)} meshes of the mix ({E} elements), one mesh per "
                       f"process on {min(cores, len(sample))} host cores, pattern + numeric "
                       f"phase; wall {wall:.1f} s, {busy:.1f} s of oracle work")}


def batch_section(args, colour=True, log_prefix="[bench]"):
    """Many meshes in one graph-captured launch (a workgroup per tile; also
    persistent, and every mesh's own kernels) vs one launch per mesh, on the
    512-mesh mix (quads n in [16,512], d=1; hexes m in [8,48],
    d=3; device-generated element matrices), CRAC, autotuned inside the batch."""
    import torch

    import paper_2012_00585_amd as feasm
    from fe_inputs import configs, meshes
    from paper_2012_00585_amd import autotune
    from paper_2012_00585_amd.batch import Batch

    dev = torch.device("cuda:0")
    specs = configs.batch_mix()[: args.batch_count]
    log(f"{log_prefix} batch of {len(specs)} meshes: building patterns")
    flags = feasm.BUILD_CSR | feasm.BUILD_CRAC | (feasm.BUILD_COLOUR if colour else 0)
    pats, kes, vals = [], [], []
    t0 = time.perf_counter()
    for i, sp in enumerate(specs):
        conn, nn = meshes.quad_mesh(sp.size) if sp.kind == "quad" else meshes.hex_mesh(sp.size)
        p = feasm.pattern_build(torch.from_numpy(conn).to(dev), sp.dofs_per_node, nn, flags)
        recipe = feasm.RECIPE_LAPLACIAN if sp.kind == "quad" else feasm.RECIPE_SPD
        kes.append(feasm.generate_ke(recipe, p.n_elem, p.n, sp.seed))
        vals.append(torch.empty(p.nnz, dtype=torch.float64, device=dev))
        pats.append(p)
        if (i + 1) % 128 == 0:
            log(f"{log_prefix}   {i + 1} meshes")
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    E = sum(p.n_elem for p in pats)
    nnz = sum(p.nnz for p in pats)
    ke_bytes = sum(p.n_elem * p.n * p.n * 8 for p in pats)
    log(f"{log_prefix} {E} elements, nnz {nnz}, Ke {ke_bytes / 1e9:.1f} GB; autotuning in the batch")
    fmt = feasm.FMT_CRAC
    # the tuner times its candidates inside the batch itself
    choices, _ = autotune.autotune_batch(pats, kes, vals, fmt, lambda ps: Batch(ps, fmt=fmt),
                                         reps=3, warmup=1, log=log)
    b = Batch(pats, fmt=fmt)
    info = b.info()
    log(f"{log_prefix} batch: {info['phases']} phase(s), {info['tiles']} tiles, largest launch "
        f"{info['grid']} workgroups")
    reps = max(args.steps, 5)
    tiles = stats(time_calls(lambda: b.assemble(kes, vals), reps, args.warmup))
    q = Batch(pats, fmt=fmt, persistent=True)
    pinfo = q.info()
    persistent = stats(time_calls(lambda: q.assemble(kes, vals), reps, args.warmup))
    q.free()
    g = Batch(pats, fmt=fmt, per_mesh_graph=True)
    graph = stats(time_calls(lambda: g.assemble(kes, vals), reps, args.warmup))
    g.free()

    def one_per_launch():
        for p, k, v in zip(pats, kes, vals):
            feasm.assemble_crac(p, k, v)

    single = stats(time_calls(one_per_launch, max(reps // 4, 3), 1))
    log(f"{log_prefix} tile grid {tiles['mean']:.3f} ms, persistent {persistent['mean']:.3f} ms, "
        f"per-mesh graph {graph['mean']:.3f} ms, one launch per mesh {single['mean']:.3f} ms")
    nbytes = sum(p.n_elem * p.n * p.n * 8 + p.nnz * 8 for p in pats)
    out = {
        "workload": f"batch mix: {len(specs)} meshes (quads n in [16,512], d=1, 4x4; hexes m in "
                    f"[8,48], d=3, 24x24), CRAC, device-generated Ke",
        "n_elem": E, "nnz": nnz, "ke_GB": ke_bytes / 1e9,
        "phases": info["phases"], "tiles": info["tiles"], "grid": info["grid"],
        "persistent_grid": pinfo["grid"],
        "paths": {k: info["paths"].count(k) for k in sorted(set(info["paths"]))},
        "tile_grid_ms": tiles,
        "persistent_ms": persistent,
        "per_mesh_graph_ms": graph,
        "one_mesh_per_launch_ms": single,
        "tile_grid_speedup_vs_one_per_launch": single["mean"] / tiles["mean"],
        "tile_grid_Ke_plus_values_GBps": nbytes / (tiles["mean"] * 1e-3) / 1e9,
        "autotune_in_batch": {f"k{c[0]}_d{c[1]}_b{c[2]}": [x.label() + f" {x.ms:.3f}ms"
                                                           for x in v[:3]]
                              for c, v in choices.items()},
        "build_s": build_s,
    }
    return out, (pats, kes, vals, b, specs)


def bench_batch(args):
    """Many meshes in one graph-captured launch vs one launch per mesh."""
    import torch

    out, (pats, kes, vals, b, specs) = batch_section(args)
    # timed steps: the batched replay (a workgroup per tile)
    for _ in range(args.warmup):
        b.assemble(kes, vals)
    torch.cuda.synchronize()
    a0 = torch.cuda.Event(enable_timing=True)
    a1 = torch.cuda.Event(enable_timing=True)
    a0.record()
    for _ in range(args.steps):
        b.assemble(kes, vals)
    a1.record()
    torch.cuda.synchronize()
    ms = a0.elapsed_time(a1) / args.steps
    line = {
        "metric": "element matrices assembled/s (batched, 512 meshes)",
        "value": out["n_elem"] / (ms * 1e-3), "unit": "element matrices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": out["workload"], "n_elem": out["n_elem"], "nnz": out["nnz"],
                   "ke_GB": out["ke_GB"], "phases": out["phases"], "tiles": out["tiles"],
                   "grid": out["grid"]},
        "batch": out,
    }
    b.free()
    for p in pats:
        p.free()
    if args.cpu_reps > 0:
        log("[bench] CPU baseline (serial oracle, one mesh per process)")
        line["cpu_baseline"] = batch_cpu_baseline(specs, 32)
    print(json.dumps(line), flush=True)


def bench_refine(args):
    """p- and d-refinement on structured quad meshes (the paper's p- and
    d-benchmarks, Section 4): Q_p quads p = 1..8 on 48 x 48 elements (d = 1,
    and d = 4 for p <= 4), and Q1 quads with d = 1..8 and 20 DOFs per node on
    192 x 192 elements.  For each: pattern build, CSR and CRAC assembly with
    the row-owned and the atomic strategy, the CRAC storage factor
    gamma = n_ca / nnz, and the matrix-vector product."""
    import torch

    import paper_2012_00585_amd as feasm
    from fe_inputs import matrices, meshes

    dev = torch.device("cuda:0")
    cases = ([("p", 48, p, 1) for p in range(1, 9)] + [("p", 48, p, 4) for p in range(1, 5)] +
             [("d", 192, 1, d) for d in (1, 2, 3, 4, 5, 6, 7, 8, 20)])
    rows = []
    O, A = feasm.SCATTER_OWNER, feasm.SCATTER_ATOMIC
    reps = max(args.steps, 5)
    for bench_kind, m, pdeg, d in cases:
        conn, nn = meshes.qp_quad_mesh(m, pdeg)
        E, k = conn.shape
        n = k * d
        t0 = time.perf_counter()
        pat = feasm.pattern_build(torch.from_numpy(conn).to(dev), d, nn,
                                  feasm.BUILD_CSR | feasm.BUILD_CRAC)
        build_ms = (time.perf_counter() - t0) * 1e3
        if n * n * 8 <= 64 * 1024:
            ke = feasm.generate_ke(feasm.RECIPE_SPD, E, n, seed=pdeg * 100 + d)
        else:
            ke = torch.from_numpy(matrices.ke_spd(E, n, seed=pdeg * 100 + d)).to(dev)
        vals = torch.empty(pat.nnz, dtype=torch.float64, device=dev)
        r = {"benchmark": bench_kind, "elements_per_side": m, "p": pdeg, "d": d, "n_elem": E,
             "n": n, "n_rows": pat.n_rows, "nnz": pat.nnz, "n_ca": pat.n_ca,
             "gamma": pat.n_ca / pat.nnz, "pattern_build_ms": build_ms}
        for name, fn, sc in (("csr_owner", feasm.assemble_csr, O),
                             ("crac_owner", feasm.assemble_crac, O),
                             ("csr_atomic", feasm.assemble_csr, A),
                             ("crac_atomic", feasm.assemble_crac, A)):
            r[name + "_ms"] = stats(time_calls(lambda f=fn, c=sc: f(pat, ke, vals, c), reps,
                                               args.warmup))["mean"]
        # row-owned bytes: Ke, values written once, incidence, row index data
        own_bytes = E * n * n * 8 + pat.nnz * 8 + 2 * E * k * 4
        r["owner_GBps"] = own_bytes / (min(r["csr_owner_ms"], r["crac_owner_ms"]) * 1e-3) / 1e9
        r["elements_per_s"] = E / (min(r["csr_owner_ms"], r["crac_owner_ms"]) * 1e-3)
        x = torch.randn(pat.n_rows, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        r["spmv_csr_ms"] = stats(time_calls(lambda: feasm.spmv_csr(pat, vals, x, y), reps,
                                            args.warmup))["mean"]
        r["spmv_crac_ms"] = stats(time_calls(lambda: feasm.spmv_crac(pat, vals, x, y), reps,
                                             args.warmup))["mean"]
        log(f"[bench] {bench_kind}-benchmark m={m} p={pdeg} d={d}: nnz {pat.nnz} "
            f"gamma {r['gamma']:.3f} owner csr {r['csr_owner_ms']:.3f} crac "
            f"{r['crac_owner_ms']:.3f} ms, atomic csr {r['csr_atomic_ms']:.3f} crac "
            f"{r['crac_atomic_ms']:.3f} ms, spmv csr {r['spmv_csr_ms']:.3f} crac "
            f"{r['spmv_crac_ms']:.3f} ms")
        rows.append(r)
        pat.free()
        del ke, vals, x, y
    total_e = sum(r["n_elem"] for r in rows)
    total_ms = sum(min(r["csr_owner_ms"], r["crac_owner_ms"]) for r in rows)
    line = {
        "metric": "element matrices assembled/s (p- and d-refinement sweep)",
        "value": total_e / (total_ms * 1e-3), "unit": "element matrices/s", "n_gpus": 1,
        "steps": reps, "warmup": args.warmup, "ms_per_step": total_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "p-benchmark: Q_p quads p=1..8 on 48x48 (d=1; d=4 for p<=4); "
                               "d-benchmark: Q1 quads on 192x192, d=1..8 and 20; SPD FP64 Ke",
                   "step": "one row-owned assembly of every case, faster format each"},
        "cases": rows,
    }
    print(json.dumps(line), flush=True)


def bench_hex8(args):
    """Element stiffness computed on the device (8-node hexahedra, 64^3,
    jittered nodes, per-element materials): the fused element-matrix +
    row-owned assembly against the two-pass path (element matrices to HBM,
    then assembly), for elasticity (d = 3) and Laplace (d = 1)."""
    import torch

    import paper_2012_00585_amd as feasm
    from fe_inputs import matrices, meshes

    dev = torch.device("cuda:0")
    m = 64
    conn, nn = meshes.hex_mesh(m)
    x = torch.from_numpy(meshes.hex_coords(m, jitter=0.2, seed=11)).to(dev)
    reps = max(args.steps, 5)
    out = {}
    for d in (3, 1):
        E = conn.shape[0]
        mat = torch.from_numpy(np.ascontiguousarray(matrices.hex_materials(E, d, seed=12))).to(dev)
        p = feasm.pattern_build(torch.from_numpy(conn).to(dev), d, nn,
                                feasm.BUILD_CSR | feasm.BUILD_CRAC)
        vals = torch.empty(p.nnz, dtype=torch.float64, device=dev)
        ke = torch.empty((E, p.n, p.n), dtype=torch.float64, device=dev)
        r = {}
        p.tune(feasm.TUNE_HEX8_PIPE, -1)
        r["fused_one_node_per_wave_crac_ms"] = stats(time_calls(
            lambda: feasm.assemble_hex8(p, feasm.FMT_CRAC, x, mat, vals), reps, args.warmup))
        p.tune(feasm.TUNE_HEX8_PIPE, args.hex8_pipe)
        for name, fmt in (("csr", feasm.FMT_CSR), ("crac", feasm.FMT_CRAC)):
            r[f"fused_{name}_ms"] = stats(time_calls(
                lambda f=fmt: feasm.assemble_hex8(p, f, x, mat, vals), reps, args.warmup))
        r["element_matrices_ms"] = stats(time_calls(
            lambda: feasm.hex8_element_matrices(p, x, mat, ke), reps, args.warmup))
        r["assembly_from_matrices_ms"] = stats(time_calls(
            lambda: feasm.assemble_crac(p, ke, vals, feasm.SCATTER_OWNER), reps, args.warmup))
        r["two_pass_ms"] = stats(time_calls(
            lambda: (feasm.hex8_element_matrices(p, x, mat, ke),
                     feasm.assemble_crac(p, ke, vals, feasm.SCATTER_OWNER)), reps, args.warmup))
        best = min(r["fused_csr_ms"]["mean"], r["fused_crac_ms"]["mean"])
        # fused bytes: coordinates and materials read once, incidence and the
        # row index data, values written once
        fused_bytes = (3 * nn * 8 + mat.numel() * 8 + 2 * E * 8 * 4 + p.nnz * 8 +
                       (p.n_ca // d) * 4)
        r["fused_elements_per_s"] = E / (best * 1e-3)
        r["fused_algorithmic_GBps"] = fused_bytes / (best * 1e-3) / 1e9
        r["two_pass_elements_per_s"] = E / (r["two_pass_ms"]["mean"] * 1e-3)
        r["speedup_fused_vs_two_pass"] = r["two_pass_ms"]["mean"] / best
        r["nnz"] = p.nnz
        log(f"[bench] hex8 d={d}: fused csr {r['fused_csr_ms']['mean']:.3f} crac "
            f"{r['fused_crac_ms']['mean']:.3f} ms (one node per wavefront "
            f"{r['fused_one_node_per_wave_crac_ms']['mean']:.3f}); element matrices "
            f"{r['element_matrices_ms']['mean']:.3f} + assembly "
            f"{r['assembly_from_matrices_ms']['mean']:.3f} = two-pass "
            f"{r['two_pass_ms']['mean']:.3f} ms")
        out[f"d{d}"] = r
        p.free()
        del ke, vals
    r3 = out["d3"]
    best3 = min(r3["fused_csr_ms"]["mean"], r3["fused_crac_ms"]["mean"])
    line = {
        "metric": "element matrices computed and assembled/s (64^3 hex elasticity, fused)",
        "value": conn.shape[0] / (best3 * 1e-3), "unit": "element matrices/s", "n_gpus": 1,
        "steps": reps, "warmup": args.warmup, "ms_per_step": best3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "64^3 trilinear hexahedra, nodes jittered 0.2 h (seed 11), "
                               "per-element Lame parameters (seed 12); d=3 elasticity and d=1 "
                               "Laplace, 2x2x2 Gauss",
                   "step": "element stiffness of every element computed and assembled, fused"},
        "results": out,
    }
    print(json.dumps(line), flush=True)


def serve_section(args, rate, seconds, log_prefix="[bench]"):
    """Serving on the 512-mesh batch mix: Poisson arrivals, assembly + 10
    re-assemblies per request.  Scenarios: continuous batching with fresh
    element matrices generated on the device per iteration (generator time
    reported apart), the same at 500 req/s (unsaturated), continuous batching
    on pre-generated per-mesh element-matrix pools (no generator in the
    loop) at the offered rate and at twice it (assembly-side capacity),
    patterns built on demand in a byte-bounded cache and in a 1-byte one
    (nearly every request builds its own), and one request at a time
    on one stream (FIFO, the one-mesh-per-launch baseline)."""
    import torch

    import paper_2012_00585_amd as feasm
    from fe_inputs import configs, meshes
    from paper_2012_00585_amd import autotune
    from paper_2012_00585_amd.serve import Request, Server

    dev = torch.device("cuda:0")
    specs = configs.batch_mix()[: args.batch_count]
    log(f"{log_prefix} serve: building {len(specs)} resident patterns")
    pats, recipes, conns = [], [], []
    for sp in specs:
        conn, nn = meshes.quad_mesh(sp.size) if sp.kind == "quad" else meshes.hex_mesh(sp.size)
        conn_d = torch.from_numpy(conn).to(dev)
        conns.append((conn_d, sp.dofs_per_node, nn))
        pats.append(feasm.pattern_build(conn_d, sp.dofs_per_node, nn,
                                        feasm.BUILD_CSR | feasm.BUILD_CRAC))
        recipes.append(feasm.RECIPE_LAPLACIAN if sp.kind == "quad" else feasm.RECIPE_SPD)
    # one tuning pass per size class on generated matrices
    classes = {}
    for i, p in enumerate(pats):
        classes.setdefault(autotune.size_class(p), []).append(i)
    for cls, members in classes.items():
        rep = max(members, key=lambda i: pats[i].n_elem)
        ke = feasm.generate_ke(recipes[rep], pats[rep].n_elem, pats[rep].n, 1)
        vals = torch.empty(pats[rep].nnz, dtype=torch.float64, device=dev)
        ranked = autotune.tune_one(pats[rep], ke, vals, feasm.FMT_CRAC, reps=3, warmup=1)
        for i in members:
            autotune.apply(pats[i], ranked[0])
        del ke, vals
    # per-mesh pools of two pre-generated blocks (about 85 GB for the mix)
    pools = [torch.stack([feasm.generate_ke(recipes[i], p.n_elem, p.n, 7000 + 2 * i + b)
                          for b in range(2)]) for i, p in enumerate(pats)]
    torch.cuda.synchronize()

    def stream(rate_, seconds_, seed):
        n = int(rate_ * seconds_)
        t = configs.arrival_times(n, 1.0 / rate_, seed=seed)
        rng = np.random.default_rng(seed + 1)
        mesh = rng.integers(len(specs), size=n)
        rs = rng.integers(1 << 40, size=n)
        return [Request(i, float(t[i]), int(mesh[i]), int(rs[i]), 10) for i in range(n)]

    def server(slots, pool=False, cache=None):
        srv = Server(fmt=feasm.FMT_CRAC, slots=slots, hbm_budget=96 << 30,
                     pattern_cache_bytes=cache)
        for i, p in enumerate(pats):
            if cache is not None:
                srv.register_mesh(i, conns[i][0], conns[i][1], conns[i][2], recipes[i])
            else:
                srv.register(i, p, recipes[i], ke_pool=pools[i] if pool else None)
        return srv

    out = {}
    for name, rate_, secs, slots, pool, cache in (
            ("continuous", rate, seconds, args.serve_slots, False, None),
            ("continuous_500", 500.0, seconds / 2, args.serve_slots, False, None),
            ("continuous_pooled_K", rate, seconds, args.serve_slots, True, None),
            # twice the offered rate: where the assembly side alone saturates
            ("continuous_pooled_K_2x_rate", 2 * rate, seconds / 2, args.serve_slots, True, None),
            ("continuous_pattern_cache_16GB", rate, seconds / 2, args.serve_slots, False, 16 << 30),
            # a 1-byte cache: an idle pattern stays only until the next miss, so
            # nearly every request builds its pattern (pattern_build + assembly
            # + 10 re-assemblies, the request recipe taken literally; the
            # engine reports the hits)
            ("pattern_build_per_request", rate, seconds / 10, args.serve_slots, False, 1),
            ("fifo_one_per_launch", rate, seconds / 5, 1, False, None)):
        log(f"{log_prefix} serve {name}: {rate_:.0f} req/s for {secs:.1f} s, {slots} slot(s); "
            "warm-up")
        server(slots, pool, cache).run(stream(rate_, min(1.0, secs), seed=99))
        res = server(slots, pool, cache).run(stream(rate_, secs, seed=0))
        eng = res["engine"]
        if eng["assemble_ms"] > 0:
            res["generator_share_of_device_time"] = eng["generate_ms"] / (eng["generate_ms"] +
                                                                          eng["assemble_ms"])
        log(f"{log_prefix}   {name}: {res['achieved_req_per_s']:.0f} req/s, re-assembly p50 "
            f"{res['reassembly_ms']['p50']:.3f} p99 {res['reassembly_ms']['p99']:.3f} ms, "
            f"generator {eng['generate_ms']:.0f} ms vs assembly {eng['assemble_ms']:.0f} ms")
        out[name] = res
    for p in pats:
        p.free()
    del pools
    return out


def bench_serve(args):
    """Poisson request stream over the batch mix: assembly + 10 re-assemblies each."""
    out = serve_section(args, args.serve_rate, args.serve_seconds)
    c = out["continuous"]
    line = {
        "metric": "served element matrices/s; p50/p99 re-assembly latency",
        "value": c["element_matrices_per_s"], "unit": "element matrices/s", "n_gpus": 1,
        "steps": c["requests"], "warmup": 1, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"serving: Poisson arrivals at {args.serve_rate:.0f} req/s over "
                               f"the {args.batch_count}-mesh batch mix, assembly + 10 "
                               f"re-assemblies with device-generated Ke, resident CRAC patterns",
                   "slots": args.serve_slots, "seconds": args.serve_seconds},
        "scenarios": out,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

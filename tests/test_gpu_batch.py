"""Batched persistent assembly, the autotuner and the device generator (GPU)."""
import sys

import numpy as np
import pytest
import torch

from fe_inputs import matrices, meshes, philox
from tests._checks import assert_values_close

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def feasm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_00585_amd as f

    f.load()
    return f


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("recipe,n", [(0, 1), (0, 2), (0, 3), (0, 4), (0, 8), (0, 9),
                                      (1, 3), (1, 8), (1, 16), (1, 24), (1, 30), (1, 40)])
def test_device_generator_matches_host_twin(feasm, recipe, n):
    seed, e0, E = 2 ** 33 + 17, 1000, 77
    say(f"[gen] recipe={recipe} n={n}")
    dev = feasm.generate_ke(recipe, E, n, seed, e0)
    host = (philox.ke_laplacian if recipe == 0 else philox.ke_spd)(E, n, seed, e0)
    assert (_np(dev) == host).all()


def _tris(nx, ny, perm_seed):
    conn, nn = meshes.quad_mesh(nx, ny)
    tri = np.concatenate([conn[:, [0, 1, 2]], conn[:, [0, 2, 3]]]).astype(np.int32)
    return np.ascontiguousarray(meshes.permute_nodes(tri, nn, perm_seed)), nn


def _mix():
    """A small batch of uneven meshes of several element types."""
    rep_conn, rep_nn = meshes.quad_mesh(5)
    rep_conn = rep_conn.copy()
    rep_conn[7, 3] = rep_conn[7, 1]
    return [
        ("quad7", *meshes.quad_mesh(7), 1),
        ("quad20", *meshes.quad_mesh(20), 1),
        ("hex3", *meshes.hex_mesh(3), 3),
        ("hex6", *meshes.hex_mesh(6), 3),
        ("tet2", *meshes.tet10_mesh(2, perm_seed=4), 3),
        ("q3quad3_d2", *meshes.qp_quad_mesh(3, 3), 2),
        ("repeated", rep_conn, rep_nn, 2),
        ("hex5_d1", *meshes.hex_mesh(5), 1),
        # one DOF per node, 3- and 4-node elements: the row-per-lane path
        ("tri_perm_d1", *_tris(11, 9, perm_seed=3), 1),
        ("repeated_d1", rep_conn, rep_nn, 1),
    ]


# batch modes: one launch per path with a workgroup per tile (default),
# persistent launches, every mesh's own kernels
MODES = {"grid": {}, "persistent": {"persistent": True}, "per_mesh_graph": {"per_mesh_graph": True}}

STRATS = {
    "owner": (3, 0),
    "atomic16": (1, 16),
    "atomic64": (1, 64),
    "coloured32": (2, 32),
    "coloured64": (2, 64),
}


@pytest.mark.parametrize("fmt", [0, 1])
@pytest.mark.parametrize("assign", ["owner", "mixed"])
@pytest.mark.parametrize("mode", MODES)
def test_batch_matches_oracle(feasm, orc, fmt, assign, mode):
    from paper_2012_00585_amd.batch import Batch

    dev = torch.device("cuda:0")
    mix = _mix()
    pats, kes, vals, refs = [], [], [], []
    for i, (name, conn, nn, d) in enumerate(mix):
        E, k = conn.shape
        p = feasm.pattern_build(torch.from_numpy(conn).to(dev), d, nn,
                                feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_COLOUR)
        strat = "owner" if assign == "owner" else list(STRATS)[i % len(STRATS)]
        sc, tpe = STRATS[strat]
        if tpe and k * d * k * d > 16 * tpe:
            tpe = 64
        p.tune(feasm.TUNE_STRATEGY, sc)
        p.tune(feasm.TUNE_THREADS_PER_ELEM, tpe)
        ke = matrices.ke_spd(E, k * d, seed=i)
        rp, ci = orc.pattern(conn, d, nn)
        ov, oa = orc.assemble(conn, d, ke, rp, ci)
        pats.append(p)
        kes.append(torch.from_numpy(ke).to(dev))
        vals.append(torch.full((p.nnz,), np.nan, dtype=torch.float64, device=dev))
        refs.append((name, strat, ov, oa))
    b = Batch(pats, fmt=fmt, **MODES[mode])
    info = b.info()
    say(f"[batch] fmt={fmt} assign={assign} mode={mode} {info}")
    for rep in range(3):
        if rep == 2:  # new buffers: the pointer table is refreshed
            kes = [k.clone() for k in kes]
            vals = [torch.full_like(v, np.nan) for v in vals]
        b.assemble(kes, vals)
        torch.cuda.synchronize()
        for (name, strat, ov, oa), v in zip(refs, vals):
            got = _np(v)
            if strat == "owner" and not name.startswith("repeated"):  # element order: exact
                assert (got == ov).all(), (name, rep)
            else:
                assert_values_close(got, ov, oa, what=f"{name} {strat} rep{rep}")
    # same values as the single-mesh calls
    fn = feasm.assemble_csr if fmt == 0 else feasm.assemble_crac
    for p, k, v, (name, strat, ov, oa) in zip(pats, kes, vals, refs):
        single = _np(fn(p, k))
        if strat == "owner" and not name.startswith("repeated"):
            assert (single == _np(v)).all(), name
    b.free()
    for p in pats:
        p.free()


def test_batch_accumulate_and_integer_exact(feasm, orc):
    from paper_2012_00585_amd.batch import Batch

    dev = torch.device("cuda:0")
    mix = _mix()[:5]
    pats, kes, vals, refs = [], [], [], []
    for i, (name, conn, nn, d) in enumerate(mix):
        E, k = conn.shape
        p = feasm.pattern_build(torch.from_numpy(conn).to(dev), d, nn,
                                feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_COLOUR)
        p.tune(feasm.TUNE_STRATEGY, [3, 1, 2, 3, 1][i])
        ke = matrices.ke_small_int(E, k * d, seed=i)
        rp, ci = orc.pattern(conn, d, nn)
        ov, _ = orc.assemble(conn, d, ke, rp, ci)
        pats.append(p)
        kes.append(torch.from_numpy(ke).to(dev))
        vals.append(torch.full((p.nnz,), 5.0, dtype=torch.float64, device=dev))
        refs.append(ov)
    for mode in MODES:
        for v in vals:
            v.fill_(5.0)
        b = Batch(pats, fmt=1, accumulate=True, **MODES[mode])
        b.assemble(kes, vals)
        for v, ov in zip(vals, refs):
            assert (_np(v) == ov + 5.0).all()
        b.free()
    for p in pats:
        p.free()


def test_autotune_keeps_results(feasm, orc):
    from paper_2012_00585_amd import autotune
    from paper_2012_00585_amd.batch import Batch

    dev = torch.device("cuda:0")
    mix = [("quad30", *meshes.quad_mesh(30), 1), ("quad40", *meshes.quad_mesh(40), 1),
           ("hex8", *meshes.hex_mesh(8), 3), ("hex10", *meshes.hex_mesh(10), 3)]
    pats, kes, vals, refs = [], [], [], []
    for i, (name, conn, nn, d) in enumerate(mix):
        E, k = conn.shape
        p = feasm.pattern_build(torch.from_numpy(conn).to(dev), d, nn,
                                feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_COLOUR)
        ke = matrices.ke_small_int(E, k * d, seed=i)
        rp, ci = orc.pattern(conn, d, nn)
        refs.append(orc.assemble(conn, d, ke, rp, ci)[0])
        pats.append(p)
        kes.append(torch.from_numpy(ke).to(dev))
        vals.append(torch.zeros(p.nnz, dtype=torch.float64, device=dev))
    choices = autotune.autotune(pats, kes, vals, fmt=1, reps=2, warmup=1, log=say)
    assert len(choices) >= 2 and all(len(v) >= 3 for v in choices.values())
    b = Batch(pats, fmt=1)
    b.assemble(kes, vals)
    for v, ov in zip(vals, refs):
        assert (_np(v) == ov).all()
    b.free()
    for p in pats:
        p.free()


def _closed_form_nnz(sp):
    """Structured Q1 meshes: (3N - 2)^2 for quads with N nodes per side and
    d = 1, 9 (3N - 2)^3 for hexes with d = 3."""
    N = sp.size + 1
    return (3 * N - 2) ** 2 if sp.kind == "quad" else 9 * (3 * N - 2) ** 3


def _row_sum_invariant(p, conn, ke, v, laplacian):
    """On the device, with torch only: no value left unwritten, and the row
    sums of G equal sum_e P_e^T (K_e 1) within 1e-12 of the same sum of
    |K_e| row sums; zero for the zero-row-sum (Laplacian) matrices.  The
    total of G equals the total of every element entry."""
    assert not torch.isnan(v).any()
    dev = v.device
    E, k = conn.shape
    d, n = p.dofs_per_node, p.n
    rp, _ = p.csr()
    counts = (rp[1:] - rp[:-1]).long()
    rows = torch.repeat_interleave(torch.arange(p.n_rows, device=dev), counts)
    g = torch.zeros(p.n_rows, dtype=torch.float64, device=dev).index_add_(0, rows, v[:p.nnz])
    c = torch.from_numpy(conn).to(dev).long()
    D = (d * c[:, :, None] + torch.arange(d, device=dev)).reshape(-1)
    K = ke.view(E, n, n)
    ref = torch.zeros_like(g).index_add_(0, D, K.sum(2).reshape(-1))
    bound = 1e-12 * torch.zeros_like(g).index_add_(0, D, K.abs().sum(2).reshape(-1))
    assert bool(((g - ref).abs() <= bound).all())
    if laplacian:
        assert bool((g.abs() <= bound).all())
    tot, kt, ka = v[:p.nnz].sum().item(), ke.sum().item(), ke.abs().sum().item()
    assert abs(tot - kt) <= 1e-12 * ka


# oracle results of sampled meshes of the mix, shared by both formats
_MIX_REFS = {}


@pytest.mark.parametrize("fmt", [1, 0], ids=["crac", "csr"])
def test_batch512_full_mix(feasm, orc, fmt):
    """The full 512-mesh mix in the launch configurations the benchmark
    times (autotuned handles; tile-grid, persistent and per-mesh-graph
    batches), with
    element matrices from the device generator.
    * every mesh: nnz equals the structured closed form, no value is left
      unwritten, and the row-sum and total invariants hold;
    * one mesh per (kind, autotuner size class, kernel path), the smallest of
      each, plus the largest of each kind: every value against the oracle
      fed with the generator's host twin -- row-owned meshes bit for bit,
      the others within the value tolerance."""
    from fe_inputs import configs
    from paper_2012_00585_amd import autotune
    from paper_2012_00585_amd.batch import Batch

    dev = torch.device("cuda:0")
    specs = configs.batch_mix()
    say(f"[batch512] fmt={fmt}: building {len(specs)} meshes")
    flags = feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_COLOUR
    pats, kes, vals, meta = [], [], [], []
    for sp in specs:
        conn, nn = meshes.quad_mesh(sp.size) if sp.kind == "quad" else meshes.hex_mesh(sp.size)
        p = feasm.pattern_build(torch.from_numpy(conn).to(dev), sp.dofs_per_node, nn, flags)
        assert p.nnz == _closed_form_nnz(sp), sp
        recipe = feasm.RECIPE_LAPLACIAN if sp.kind == "quad" else feasm.RECIPE_SPD
        kes.append(feasm.generate_ke(recipe, p.n_elem, p.n, sp.seed))
        vals.append(torch.empty(p.nnz, dtype=torch.float64, device=dev))
        pats.append(p)
        meta.append((sp, conn, nn))
    torch.cuda.synchronize()
    autotune.autotune(pats, kes, vals, fmt, reps=2, warmup=1, log=say)
    paths = None
    refs = _MIX_REFS
    for mode in MODES:
        say(f"[batch512] fmt={fmt} mode={mode}")
        for v in vals:
            v.fill_(np.nan)
        b = Batch(pats, fmt=fmt, **MODES[mode])
        if paths is None:
            paths = b.info()["paths"]
            groups = {}
            for i, sp in enumerate(specs):
                groups.setdefault((sp.kind, autotune.size_class(pats[i]), paths[i]), []).append(i)
            sample = {min(m, key=lambda i: pats[i].n_elem) for m in groups.values()}
            for kind in ("quad", "hex"):
                sample.add(max((i for i in range(len(specs)) if specs[i].kind == kind),
                               key=lambda i: pats[i].n_elem))
            say(f"[batch512] {len(groups)} (kind, class, path) groups; oracle on "
                f"{len(sample)} meshes")
            for i in sorted(sample - set(refs)):
                sp, conn, nn = meta[i]
                E, k = conn.shape
                twin = philox.ke_laplacian if sp.kind == "quad" else philox.ke_spd
                ke = twin(E, k * sp.dofs_per_node, sp.seed)
                rp, ci = orc.pattern(conn, sp.dofs_per_node, nn)
                refs[i] = orc.assemble(conn, sp.dofs_per_node, ke, rp, ci)
        b.assemble(kes, vals)
        torch.cuda.synchronize()
        for i, (sp, conn, nn) in enumerate(meta):
            _row_sum_invariant(pats[i], conn, kes[i], vals[i], sp.kind == "quad")
        for i in sorted(sample):
            got = _np(vals[i])
            ov, oa = refs[i]
            if paths[i].startswith(("own", "rows")):  # row-owned: element order
                assert (got == ov).all(), (i, specs[i], paths[i], mode)
            else:
                assert_values_close(got, ov, oa, what=f"mesh {i} {specs[i]} {paths[i]}")
        b.free()
    for p in pats:
        p.free()

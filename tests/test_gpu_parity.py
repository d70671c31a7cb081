"""Parity of the HIP path with the serial oracle (GPU).

Patterns (row_ptr, col_idx, CRAC pairs) must be bit-exact.  Values must meet
|g - o| <= 1e-12 * A per entry (A = sum of |contributions|, from the oracle);
small-integer element matrices, whose sums are exact in any order, must match
bit for bit.  Every case runs CSR and CRAC, atomic and coloured, assembly and
value-only re-assembly (first call records lookups, second reuses them).
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest
import torch

from fe_inputs import configs, matrices, meshes
from tests._checks import assert_values_close

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


def run_device(feasm, conn, d, nn, ke, flags=None, strategies=None):
    """Pattern + every numeric variant on the device; returns numpy results."""
    flags = flags or (feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_COLOUR)
    dev = torch.device("cuda:0")
    conn_d = torch.from_numpy(np.ascontiguousarray(conn, dtype=np.int32)).to(dev)
    p = feasm.pattern_build(conn_d, d, nn, flags)
    out = {"p": p, "nnz": p.nnz, "n_ca": p.n_ca, "n_colours": p.n_colours}
    out["row_ptr"], out["col_idx"] = (_np(t) for t in p.csr())
    out["crac_row_ptr"], out["ca"] = (_np(t) for t in p.crac())
    cptr, celems, ecol = p.colouring()
    out["colour_ptr"], out["colour_elems"], out["elem_colour"] = cptr, _np(celems), _np(ecol)
    ke_d = torch.from_numpy(np.ascontiguousarray(ke)).to(dev)
    strategies = strategies or [(fmt, sc) for fmt in ("csr", "crac")
                                for sc in (feasm.SCATTER_ATOMIC, feasm.SCATTER_COLOURED,
                                           feasm.SCATTER_OWNER)]
    vals = {}
    for fmt, sc in strategies:
        fn = feasm.assemble_csr if fmt == "csr" else feasm.assemble_crac
        fcode = feasm.FMT_CSR if fmt == "csr" else feasm.FMT_CRAC
        vals[(fmt, sc, "assemble")] = _np(fn(p, ke_d, scatter=sc))
        vals[(fmt, sc, "reassemble1")] = _np(feasm.reassemble_values(p, fcode, ke_d, scatter=sc))
        vals[(fmt, sc, "reassemble2")] = _np(feasm.reassemble_values(p, fcode, ke_d, scatter=sc))
    torch.cuda.synchronize()
    out["values"] = vals
    return out


OWNER = 3  # FEASM_SCATTER_OWNER


def check_against_oracle(orc, conn, d, nn, ke, res, exact=False, owner_exact=True):
    """owner_exact: the row-owned strategy sums every entry in increasing
    element order, the sequential listing's order, so without repeated nodes
    its values equal the oracle's bit for bit."""
    rp, ci = orc.pattern(conn, d, nn)
    crp, ca = orc.crac(rp, ci, d * nn)
    assert res["nnz"] == rp[-1]
    assert (res["row_ptr"] == rp).all()
    assert (res["col_idx"] == ci).all()
    assert res["n_ca"] == ca.size
    assert (res["crac_row_ptr"] == crp).all()
    assert (res["ca"] == ca).all()
    # colouring: valid, the sequential greedy colouring in element order, and
    # the grouped list is a permutation sorted within colours
    nc = res["n_colours"]
    assert orc.colouring_valid(conn, nn, res["elem_colour"], nc)
    gcol, gnc = orc.greedy_colour(conn, nn)
    assert nc == gnc and (res["elem_colour"] == gcol).all()
    ptr = res["colour_ptr"]
    assert ptr[0] == 0 and ptr[-1] == conn.shape[0]
    ce = res["colour_elems"]
    assert (np.sort(ce) == np.arange(conn.shape[0])).all()
    for c in range(nc):
        seg = ce[ptr[c]:ptr[c + 1]]
        assert (res["elem_colour"][seg] == c).all()
        assert (np.diff(seg) > 0).all()
    ov, oa = orc.assemble(conn, d, ke, rp, ci)
    for key, v in res["values"].items():
        if exact or (owner_exact and key[1] == OWNER):
            assert (v == ov).all(), key
        else:
            assert_values_close(v, ov, oa, what=str(key))


def _fan(n_tri):
    """Triangles (centre, i, i+1) around node 0: node 0 has n_tri elements."""
    i = np.arange(n_tri)
    conn = np.stack([np.zeros_like(i), 1 + i, 1 + (i + 1) % n_tri], axis=1)
    return conn.astype(np.int32), n_tri + 1


def _repeated():
    conn, nn = meshes.quad_mesh(3)
    conn = conn.copy()
    conn[4, 2] = conn[4, 0]  # element 4 lists a node twice (degenerate quad)
    return conn, nn


def _tris(nx, ny, perm_seed=None):
    """Each quad of an nx x ny grid cut into two triangles (3 nodes, d = 1
    cases take the one-row-per-lane kernel)."""
    conn, nn = meshes.quad_mesh(nx, ny)
    tri = np.concatenate([conn[:, [0, 1, 2]], conn[:, [0, 2, 3]]]).astype(np.int32)
    if perm_seed is not None:
        tri = meshes.permute_nodes(tri, nn, perm_seed)
    return np.ascontiguousarray(tri), nn


def _tet4(m, perm_seed):
    """Linear tets: the vertex nodes of the tet10 mesh (its edge nodes stay
    unused, so many rows are empty)."""
    conn, nn = meshes.tet10_mesh(m, perm_seed=perm_seed)
    return np.ascontiguousarray(conn[:, :4]), nn


CASES = [
    ("one_quad", lambda: meshes.quad_mesh(1), 1),
    ("quad3x5_d2", lambda: meshes.quad_mesh(3, 5), 2),
    ("hex2_d3", lambda: meshes.hex_mesh(2), 3),
    ("hex5x3x2_d1", lambda: meshes.hex_mesh(5, 3, 2), 1),
    ("hex7_d3", lambda: meshes.hex_mesh(7), 3),
    ("tet2perm_d3", lambda: meshes.tet10_mesh(2, perm_seed=0), 3),
    ("tet3perm_d2", lambda: meshes.tet10_mesh(3, perm_seed=5), 2),
    ("q3quad3_d2", lambda: meshes.qp_quad_mesh(3, 3), 2),
    ("q8quad2_d1", lambda: meshes.qp_quad_mesh(2, 8), 1),
    ("q4quad2_d4", lambda: meshes.qp_quad_mesh(2, 4), 4),
    ("fan400_bignode", lambda: _fan(400), 1),
    ("repeated_node", _repeated, 2),
    ("unused_nodes", lambda: (meshes.quad_mesh(4)[0], 40), 1),
    # p- and d-refinement shapes: Q6 quads with 3 DOFs (d*n = 441), Q1 quads
    # with 8 and 20 DOFs per node (d*n = 256 and 1600)
    ("q6quad2_d3", lambda: meshes.qp_quad_mesh(2, 6), 3),
    ("quad4_d8", lambda: meshes.quad_mesh(4), 8),
    ("quad3_d20", lambda: meshes.quad_mesh(3), 20),
    # one DOF per node, 3- and 4-node elements: the one-row-per-lane kernel
    # (rows of several wavefronts, permuted numbering, empty rows, a node
    # listed twice by one element)
    ("tri9x7_d1", lambda: _tris(9, 7), 1),
    ("tri13x11perm_d1", lambda: _tris(13, 11, perm_seed=2), 1),
    ("tet4perm_d1", lambda: _tet4(3, perm_seed=1), 1),
    ("repeated_node_d1", _repeated, 1),
]


@pytest.mark.parametrize("name,make,d", CASES, ids=[c[0] for c in CASES])
def test_small_cases_spd(feasm, orc, name, make, d):
    conn, nn = make()
    E, k = conn.shape
    say(f"[parity] {name}: E={E} k={k} d={d} nodes={nn}")
    ke = matrices.ke_spd(E, k * d, seed=3)
    res = run_device(feasm, conn, d, nn, ke)
    check_against_oracle(orc, conn, d, nn, ke, res,
                         owner_exact=not name.startswith("repeated_node"))
    res["p"].free()


@pytest.mark.parametrize("name,make,d", CASES[:8] + CASES[10:], ids=[c[0] for c in CASES[:8] + CASES[10:]])
def test_small_cases_integer_exact(feasm, orc, name, make, d):
    conn, nn = make()
    E, k = conn.shape
    say(f"[exact] {name}: E={E} k={k} d={d}")
    ke = matrices.ke_small_int(E, k * d, seed=9)
    res = run_device(feasm, conn, d, nn, ke)
    check_against_oracle(orc, conn, d, nn, ke, res, exact=True)
    res["p"].free()


def test_quad64_workload(feasm, orc):
    w = configs.quad64()
    say("[parity] quad64 (64x64 Q1, d=1, zero-row-sum Ke)")
    ke = w.ke()
    res = run_device(feasm, w.conn, w.dofs_per_node, w.n_nodes, ke)
    assert res["nnz"] == 37249 and res["n_ca"] == 25092
    # structured quads: the paper's four even colours
    assert res["n_colours"] == 4
    assert np.diff(res["colour_ptr"]).tolist() == [1024] * 4
    check_against_oracle(orc, w.conn, w.dofs_per_node, w.n_nodes, ke, res)
    res["p"].free()


def test_all_ones_dummy_element_bit_exact(feasm, orc):
    # The paper's dummy element (all ones): sums are exact small integers.
    conn, nn = meshes.hex_mesh(16)
    d = 3
    E, k = conn.shape
    say("[exact] hex16 all-ones")
    ke = matrices.ke_ones(E, k * d)
    res = run_device(feasm, conn, d, nn, ke)
    check_against_oracle(orc, conn, d, nn, ke, res, exact=True)
    for v in res["values"].values():
        assert v.sum() == E * (k * d) ** 2
    res["p"].free()


@pytest.fixture(scope="module")
def hex64(feasm):
    w = configs.hex64()
    say("[hex64] generating Ke (262144 x 24 x 24)")
    return w, w.ke()


def test_hex64_pattern_and_values(feasm, orc, hex64):
    w, ke = hex64
    say("[parity] hex64 full size: pattern, CSR/CRAC atomic/coloured")
    res = run_device(feasm, w.conn, 3, w.n_nodes, ke, strategies=[
        ("csr", feasm.SCATTER_ATOMIC), ("crac", feasm.SCATTER_ATOMIC),
        ("crac", feasm.SCATTER_COLOURED), ("csr", feasm.SCATTER_OWNER),
        ("crac", feasm.SCATTER_OWNER)])
    assert res["nnz"] == 64701513 and res["n_ca"] == 14527112
    # structured hexahedra: eight even colours
    assert res["n_colours"] == 8
    assert np.diff(res["colour_ptr"]).tolist() == [32768] * 8
    check_against_oracle(orc, w.conn, 3, w.n_nodes, ke, res)
    res["p"].free()


def _sha(a):
    return hashlib.sha256(np.asarray(a, dtype=np.int64).tobytes()).hexdigest()


def test_tet40_full(feasm, orc, tet40_ref):
    """The permuted tet10 workload in full: pattern and CRAC arrays equal to
    the oracle's, the colouring equal to the oracle's greedy colouring, and
    every value of every strategy compared with the oracle's assembly."""
    g = json.load(open(os.path.join(GOLDEN, "tet40_counts.json")))
    r = tet40_ref
    w, ke = r.w, r.ke
    dev = torch.device("cuda:0")
    say("[parity] tet40 (permuted tet10) full size: pattern, colouring")
    p = feasm.pattern_build(torch.from_numpy(w.conn).to(dev), 3, w.n_nodes,
                            feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_COLOUR)
    assert (p.nnz, p.n_ca) == (g["nnz"], g["n_ca"])
    rp, ci = (_np(t) for t in p.csr())
    crp, ca = (_np(t) for t in p.crac())
    assert (rp == r.rp).all() and (ci == r.ci).all()
    assert (crp == r.crp).all() and (ca == r.ca).all()
    assert _sha(crp) == g["crac_row_ptr_sha_int64"]
    gcol, gnc = orc.greedy_colour(w.conn, w.n_nodes)
    _, _, ecol = p.colouring()
    assert p.n_colours == gnc == 31
    assert (_np(ecol) == gcol).all()
    ke_d = torch.from_numpy(ke).to(dev)
    total = abs(ke.sum())
    for fmt, sc in (("csr", feasm.SCATTER_ATOMIC), ("crac", feasm.SCATTER_ATOMIC),
                    ("csr", feasm.SCATTER_COLOURED), ("crac", feasm.SCATTER_COLOURED),
                    ("csr", feasm.SCATTER_OWNER), ("crac", feasm.SCATTER_OWNER),
                    ("csr", feasm.SCATTER_SPIN), ("crac", feasm.SCATTER_SPIN)):
        fn = feasm.assemble_csr if fmt == "csr" else feasm.assemble_crac
        say(f"[parity] tet40 {fmt} strategy {sc}: every value")
        v = _np(fn(p, ke_d, scatter=sc))
        if sc == feasm.SCATTER_SPIN:
            assert p.spin_aborts() == 0
        if sc == feasm.SCATTER_OWNER:
            assert (v == r.ov).all()
        else:
            assert_values_close(v, r.ov, r.oa, what=f"tet40 {fmt} {sc}")
        assert abs(v.sum() - ke.sum()) <= 1e-12 * np.abs(ke).sum() + 1e-12 * total
        del v
    p.free()
    say("[parity] tet40 with the lookup record built with the pattern: every value")
    p = feasm.pattern_build(torch.from_numpy(w.conn).to(dev), 3, w.n_nodes,
                            feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_OWNER_MAP)
    for fn in (feasm.assemble_csr, feasm.assemble_crac):
        assert (_np(fn(p, ke_d)) == r.ov).all(), fn.__name__
    p.free()


@pytest.mark.parametrize("name,make,d", CASES, ids=[c[0] for c in CASES])
def test_owner_record_built_with_pattern(feasm, orc, name, make, d):
    """FEASM_BUILD_OWNER_MAP: the row-owned calls read the lookup record from
    the first assembly on; the same sums in the same element order, so the
    values equal the oracle's bit for bit (a repeated node: within the
    tolerance), for assembly, accumulation and re-assembly."""
    conn, nn = make()
    E, k = conn.shape
    dev = torch.device("cuda:0")
    p = feasm.pattern_build(torch.from_numpy(np.ascontiguousarray(conn, dtype=np.int32)).to(dev), d,
                            nn, feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_OWNER_MAP)
    ke = matrices.ke_spd(E, k * d, seed=11)
    rp, ci = orc.pattern(conn, d, nn)
    ov, oa = orc.assemble(conn, d, ke, rp, ci)
    ke_d = torch.from_numpy(ke).to(dev)
    exact = not name.startswith("repeated_node")
    say(f"[parity] lookup record built with the pattern: {name}")
    for fmt, fn in ((feasm.FMT_CSR, feasm.assemble_csr), (feasm.FMT_CRAC, feasm.assemble_crac)):
        try:
            v = fn(p, ke_d, scatter=feasm.SCATTER_OWNER)
        except feasm.FeasmError as e:  # rows longer than the LDS accumulator
            assert "ELIMIT" in str(e)
            continue
        got = [("assemble", _np(v))]
        fn(p, ke_d, values=v, scatter=feasm.SCATTER_OWNER | feasm.ACCUMULATE)
        got.append(("accumulate", _np(v) / 2))
        got.append(("reassemble", _np(feasm.reassemble_values(p, fmt, ke_d,
                                                              scatter=feasm.SCATTER_OWNER))))
        for what, g in got:
            if exact:
                assert (g == ov).all(), (name, fmt, what)
            else:
                assert_values_close(g, ov, oa, what=f"{name} {fmt} {what}")
    p.free()


def test_colour_blocks(feasm, orc):
    """The coloured scatter run element block by element block: every block
    count gives the oracle's values (integer element matrices: exact in any
    order), on a grid-numbered hex mesh and a permuted tet10 mesh; the knob
    needs a coloured handle and a count in [0, 256]."""
    dev = torch.device("cuda:0")
    for name, (conn, nn), d in (("hex 9x7x5", meshes.hex_mesh(9, 7, 5), 3),
                                ("tet10 3^3 permuted", meshes.tet10_mesh(3, perm_seed=6), 3)):
        E, k = conn.shape
        p = feasm.pattern_build(torch.from_numpy(conn).to(dev), d, nn,
                                feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_COLOUR)
        rp, ci = orc.pattern(conn, d, nn)
        kei = matrices.ke_small_int(E, k * d, seed=13)
        ov, _ = orc.assemble(conn, d, kei, rp, ci)
        ke_d = torch.from_numpy(kei).to(dev)
        for nb in (2, 3, 7, min(E, 256), 256, 1, 0):
            say(f"[parity] {name}: coloured scatter in {nb} element blocks")
            p.tune(feasm.TUNE_COLOUR_BLOCKS, nb)
            for fn in (feasm.assemble_csr, feasm.assemble_crac):
                v = fn(p, ke_d, scatter=feasm.SCATTER_COLOURED)
                assert (_np(v) == ov).all(), (name, nb, fn.__name__)
                fn(p, ke_d, values=v, scatter=feasm.SCATTER_COLOURED | feasm.ACCUMULATE)
                assert (_np(v) == 2 * ov).all(), (name, nb, fn.__name__, "accumulate")
        with pytest.raises(feasm.FeasmError):
            p.tune(feasm.TUNE_COLOUR_BLOCKS, 257)
        p.free()
    conn, nn = meshes.quad_mesh(4)
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), 1, nn)
    with pytest.raises(feasm.FeasmError):
        p.tune(feasm.TUNE_COLOUR_BLOCKS, 2)
    p.free()


def test_error_paths_on_device(feasm):
    dev = torch.device("cuda:0")
    conn, nn = meshes.quad_mesh(3)
    bad = conn.copy()
    bad[5, 1] = nn + 7
    with pytest.raises(feasm.FeasmError, match="ERANGE"):
        feasm.pattern_build(torch.from_numpy(bad).to(dev), 1, nn)
    bad[5, 1] = -1
    with pytest.raises(feasm.FeasmError, match="element 5, local node 1"):
        feasm.pattern_build(torch.from_numpy(bad).to(dev), 1, nn)
    conn_f, nn_f = _fan(3000)  # node 0: 9000 candidate entries > 8192
    with pytest.raises(feasm.FeasmError, match="ELIMIT"):
        feasm.pattern_build(torch.from_numpy(conn_f).to(dev), 1, nn_f)
    # a handle without colouring rejects the coloured strategy
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), 1, nn, feasm.BUILD_CSR)
    ke = torch.zeros(conn.shape[0] * 16, dtype=torch.float64, device=dev)
    with pytest.raises(feasm.FeasmError, match="colour"):
        feasm.assemble_csr(p, ke, scatter=feasm.SCATTER_COLOURED)
    with pytest.raises(feasm.FeasmError, match="without CRAC"):
        feasm.assemble_crac(p, ke)
    with pytest.raises(ValueError):
        feasm.assemble_csr(p, ke[:-1])
    p.free()


def test_accumulate_adds_without_reset(feasm, orc):
    conn, nn = meshes.hex_mesh(3)
    d = 2
    E, k = conn.shape
    ke = matrices.ke_small_int(E, k * d, seed=2)
    dev = torch.device("cuda:0")
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), d, nn,
                            feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_COLOUR)
    rp, ci = orc.pattern(conn, d, nn)
    ov, _ = orc.assemble(conn, d, ke, rp, ci)
    ke_d = torch.from_numpy(ke).to(dev)
    for sc in (feasm.SCATTER_ATOMIC, feasm.SCATTER_COLOURED, feasm.SCATTER_OWNER):
        for fn in (feasm.assemble_csr, feasm.assemble_crac):
            base = torch.full((p.nnz,), 3.0, dtype=torch.float64, device=dev)
            v = _np(fn(p, ke_d, base, sc | feasm.ACCUMULATE))
            assert (v == ov + 3.0).all(), (fn.__name__, sc)
    p.free()


def test_owner_is_deterministic(feasm):
    w = configs.tet40(m=12)
    dev = torch.device("cuda:0")
    ke = torch.from_numpy(w.ke()).to(dev)
    p = feasm.pattern_build(torch.from_numpy(w.conn).to(dev), 3, w.n_nodes)
    a = feasm.assemble_crac(p, ke, scatter=feasm.SCATTER_OWNER).clone()
    b = feasm.assemble_csr(p, ke, scatter=feasm.SCATTER_OWNER)
    c = feasm.reassemble_values(p, feasm.FMT_CRAC, ke)
    assert torch.equal(a, b) and torch.equal(a, c)
    p.free()


@pytest.mark.parametrize("rows,batch", [(1, 8), (2, 8), (2, 16), (4, 8), (4, 16)])
@pytest.mark.parametrize("mesh", ["hex7_d3", "tet3perm_d3", "q8quad2_d1"])
def test_owner_launch_shapes_bit_exact(feasm, orc, mesh, rows, batch):
    make = {"hex7_d3": (lambda: meshes.hex_mesh(7), 3),
            "tet3perm_d3": (lambda: meshes.tet10_mesh(3, perm_seed=1), 3),
            "q8quad2_d1": (lambda: meshes.qp_quad_mesh(2, 8), 1)}[mesh]
    (conn, nn), d = make[0](), make[1]
    E, k = conn.shape
    say(f"[owner shapes] {mesh} rows={rows} batch={batch}")
    ke = matrices.ke_spd(E, k * d, seed=6)
    dev = torch.device("cuda:0")
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), d, nn)
    rp, ci = orc.pattern(conn, d, nn)
    ov, _ = orc.assemble(conn, d, ke, rp, ci)
    ke_d = torch.from_numpy(ke).to(dev)
    p.tune(feasm.TUNE_OWNER_FLAT, -1)  # the row-batched kernels, not the flat ones
    for bpc in (0, 3):
        p.tune(feasm.TUNE_OWNER_ROWS, rows)
        p.tune(feasm.TUNE_OWNER_BATCH, batch)
        p.tune(feasm.TUNE_OWNER_BLOCKS_PER_CU, bpc)
        for fn in (feasm.assemble_csr, feasm.assemble_crac):
            v = _np(fn(p, ke_d, scatter=feasm.SCATTER_OWNER))
            assert (v == ov).all(), (fn.__name__, bpc)
    p.free()


@pytest.mark.parametrize("mesh", ["hex7_d3", "tet3perm_d3", "q8quad2_d1", "hex4_d2"])
def test_owner_flat_batches_bit_exact(feasm, orc, mesh):
    """Flat batches keep element order in every value, so all launch shapes
    give the oracle's values bit for bit, for assembly and re-assembly.
    The flat kernels are compiled for 8-node hexes and 10-node tets with 3
    DOFs per node; on the other meshes the setting must fall back."""
    make = {"hex7_d3": (lambda: meshes.hex_mesh(7), 3),
            "tet3perm_d3": (lambda: meshes.tet10_mesh(3, perm_seed=1), 3),
            "q8quad2_d1": (lambda: meshes.qp_quad_mesh(2, 8), 1),
            "hex4_d2": (lambda: meshes.hex_mesh(4), 2)}[mesh]
    (conn, nn), d = make[0](), make[1]
    E, k = conn.shape
    ke = matrices.ke_spd(E, k * d, seed=9)
    dev = torch.device("cuda:0")
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), d, nn)
    rp, ci = orc.pattern(conn, d, nn)
    ov, _ = orc.assemble(conn, d, ke, rp, ci)
    ke_d = torch.from_numpy(ke).to(dev)
    for rows, prefetch in ((1, 0), (2, 1), (4, 0)):
        for flat in (0, 8, 16):
            say(f"[owner flat] {mesh} rows={rows} flat={flat} prefetch={prefetch}")
            p.tune(feasm.TUNE_OWNER_ROWS, rows)
            p.tune(feasm.TUNE_OWNER_FLAT, flat)
            p.tune(feasm.TUNE_OWNER_PREFETCH, prefetch)
            for fn in (feasm.assemble_csr, feasm.assemble_crac):
                v = _np(fn(p, ke_d, scatter=feasm.SCATTER_OWNER))
                assert (v == ov).all(), (fn.__name__, rows, flat)
            v = _np(feasm.reassemble_values(p, feasm.FMT_CRAC, ke_d, scatter=feasm.SCATTER_OWNER))
            assert (v == ov).all(), ("reassemble", rows, flat, prefetch)
    with pytest.raises(feasm.FeasmError):
        p.tune(feasm.TUNE_OWNER_FLAT, 10)
    p.free()


def test_atomic_threads_per_element_tuning(feasm, orc):
    conn, nn = meshes.hex_mesh(5)
    d = 3
    E, k = conn.shape
    ke = matrices.ke_small_int(E, k * d, seed=1)
    dev = torch.device("cuda:0")
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), d, nn,
                            feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_COLOUR)
    rp, ci = orc.pattern(conn, d, nn)
    ov, _ = orc.assemble(conn, d, ke, rp, ci)
    ke_d = torch.from_numpy(ke).to(dev)
    for tpe in (64, 128, 256):
        p.tune(feasm.TUNE_THREADS_PER_ELEM, tpe)
        for sc in (feasm.SCATTER_ATOMIC, feasm.SCATTER_COLOURED):
            for fn in (feasm.assemble_csr, feasm.assemble_crac):
                assert (_np(fn(p, ke_d, scatter=sc)) == ov).all(), (tpe, sc)
    with pytest.raises(feasm.FeasmError):
        p.tune(feasm.TUNE_THREADS_PER_ELEM, 16)  # 576 entries need >= 36 lanes
    with pytest.raises(feasm.FeasmError):
        p.tune(99, 1)
    p.free()


def test_reassembly_record_after_row_owned_calls(feasm, orc):
    # the row-owned strategy records no lookups; a later atomic or coloured
    # re-assembly on the same handle must record its own before reading them
    conn, nn = meshes.tet10_mesh(3, perm_seed=8)
    d = 3
    E, k = conn.shape
    ke = matrices.ke_small_int(E, k * d, seed=4)
    dev = torch.device("cuda:0")
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), d, nn,
                            feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_COLOUR)
    rp, ci = orc.pattern(conn, d, nn)
    ov, _ = orc.assemble(conn, d, ke, rp, ci)
    ke_d = torch.from_numpy(ke).to(dev)
    for fmt in (feasm.FMT_CRAC, feasm.FMT_CSR):
        for sc in (feasm.SCATTER_OWNER, feasm.SCATTER_OWNER, feasm.SCATTER_ATOMIC,
                   feasm.SCATTER_ATOMIC, feasm.SCATTER_COLOURED, feasm.SCATTER_OWNER):
            v = _np(feasm.reassemble_values(p, fmt, ke_d, scatter=sc))
            assert (v == ov).all(), (fmt, sc)
    p.free()

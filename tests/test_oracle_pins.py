"""Pins of the serial oracle against what the paper and mathematics fix.

None of these checks re-types an oracle formula: they compare against the
paper's printed arrays and counts (tests/golden), closed forms, brute-force
dense assembly with ``numpy.add.at`` and invariants of the assembled matrix.
"""
import json
import os

import numpy as np
import pytest

from fe_inputs import matrices, meshes
from tests._checks import assert_values_close, dof_indices

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# Figure 1 (Section 2.2): CSR and CRAC arrays of a 6x6 matrix and the lookup
# of coefficient (3,6).


def _fig1_contributions(g):
    """Nonzeros of Fig. 1(a) as coordinate contributions, in a scrambled
    order and with each value split in two parts, so that the pattern build
    must sort, merge duplicates and sum."""
    dense = np.array(g["dense"])
    r, c = np.nonzero(dense)
    v = dense[r, c]
    rng = np.random.default_rng(7)
    order = rng.permutation(r.size)
    r, c, v = r[order], c[order], v[order]
    # v = v/2 + v/2 exactly (halving is exact in binary floating point)
    return (np.concatenate([r, r[::-1]]), np.concatenate([c, c[::-1]]),
            np.concatenate([v / 2, (v / 2)[::-1]]))


def test_fig1_csr_pattern_and_values(orc):
    g = _golden("fig1_csr_crac.json")
    rows, cols, vals = _fig1_contributions(g)
    row_ptr, col_idx = orc.pattern_pairs(rows, cols, 6, 6)
    assert list(row_ptr + 1) == g["csr_row_ptr"]
    assert list(col_idx + 1) == g["csr_col_idx"]
    values = orc.assemble_pairs(rows, cols, vals, row_ptr, col_idx)
    assert list(values) == g["values"]


def test_fig1_crac_arrays(orc):
    g = _golden("fig1_csr_crac.json")
    row_ptr = np.array(g["csr_row_ptr"]) - 1
    col_idx = np.array(g["csr_col_idx"]) - 1
    crp, ca = orc.crac(row_ptr, col_idx, n_cols=6)
    assert list(crp + 1) == g["crac_row_ptr"]
    printed = g["crac_ca"]
    assert len(ca) == len(printed)
    # every printed entry (1-based) except the final pair's column, printed '-'
    for got, want in zip(ca, printed):
        if want is not None:
            assert got + 1 == want
    assert ca[-2] == 6  # final-pair column: the sentinel n_cols


def test_fig1_lookup_3_6(orc):
    g = _golden("fig1_csr_crac.json")
    lk = g["lookup"]
    row_ptr = np.array(g["csr_row_ptr"]) - 1
    col_idx = np.array(g["csr_col_idx"]) - 1
    crp, ca = orc.crac(row_ptr, col_idx, n_cols=6)
    p_csr = orc.csr_find(row_ptr, col_idx, lk["row"] - 1, lk["col"] - 1)
    p_crac = orc.crac_find(crp, ca, lk["row"] - 1, lk["col"] - 1)
    assert p_csr + 1 == lk["position"] and p_crac + 1 == lk["position"]
    assert g["values"][p_csr] == lk["value"]


def test_fig1_every_lookup(orc):
    g = _golden("fig1_csr_crac.json")
    dense = np.array(g["dense"])
    row_ptr = np.array(g["csr_row_ptr"]) - 1
    col_idx = np.array(g["csr_col_idx"]) - 1
    crp, ca = orc.crac(row_ptr, col_idx, n_cols=6)
    for i in range(6):
        for j in range(6):
            p = orc.csr_find(row_ptr, col_idx, i, j)
            q = orc.crac_find(crp, ca, i, j)
            assert p == q
            if dense[i, j] != 0:
                assert g["values"][p] == dense[i, j]
            else:
                assert p == -1


# --------------------------------------------------------------------------
# Section 2.1: the element DOF array and its run-length form.


def test_dof_map_and_runs_example(orc):
    # A 4-node quad with 4 DOFs per node on nodes 13, 24, 25, 12 gives the
    # paper's example array 52..55, 96..103, 48..51 and runs [52,4,96,8,48,4].
    D = orc.dof_map([13, 24, 25, 12], 4)
    assert list(D) == list(range(52, 56)) + list(range(96, 104)) + list(range(48, 52))
    assert list(orc.dof_runs(D)) == [52, 4, 96, 8, 48, 4]


def test_runs_follow_local_order(orc):
    assert list(orc.dof_runs([5, 6, 7, 3, 4, 9])) == [5, 3, 3, 2, 9, 1]
    assert list(orc.dof_runs([4, 3, 2])) == [4, 1, 3, 1, 2, 1]
    assert list(orc.dof_runs([8])) == [8, 1]


# --------------------------------------------------------------------------
# Printed nnz counts (Section 4) and closed forms.


def test_h_benchmark_nnz_matches_paper(orc):
    g = _golden("paper_counts.json")["h_benchmark_structured_d1"]
    for m, want in zip(g["elements_per_side"], g["nnz"]):
        conn, nn = meshes.quad_mesh(m)
        row_ptr, _ = orc.pattern(conn, 1, nn)
        assert row_ptr[-1] == want
        N = m + 1
        assert want == (3 * N - 2) ** 2  # closed form for structured Q1 quads


def test_h_benchmark_d4_nnz_matches_paper(orc):
    g = _golden("paper_counts.json")["h_benchmark_structured_d4"]
    for m, want in list(zip(g["elements_per_side"], g["nnz"]))[:5]:
        conn, nn = meshes.quad_mesh(m)
        row_ptr, _ = orc.pattern(conn, 4, nn)
        assert row_ptr[-1] == want


@pytest.mark.slow
def test_p_benchmark_nnz_matches_paper(orc):
    g = _golden("paper_counts.json")["p_benchmark_structured_d1"]
    m = g["elements_per_side"]
    for p, want in zip(g["p"], g["nnz"]):
        conn, nn = meshes.qp_quad_mesh(m, p)
        row_ptr, _ = orc.pattern(conn, 1, nn)
        assert row_ptr[-1] == want, p


@pytest.mark.slow
def test_p4_d4_nnz_matches_paper(orc):
    g = _golden("paper_counts.json")["p_benchmark_structured_d4_p4_nnz"]
    conn, nn = meshes.qp_quad_mesh(g["elements_per_side"], g["p"])
    row_ptr, _ = orc.pattern(conn, 4, nn)
    assert row_ptr[-1] == g["nnz"]


def test_d_benchmark_nnz_and_crac_law(orc):
    g = _golden("paper_counts.json")["d_benchmark_structured"]
    # The paper's own n_ca values obey n_ca(d) = d (n_ca(1) - 2) + 2, i.e. its
    # n_ca counts the final pair and every run of a node row repeats d times.
    pc = g["n_ca_gmsh_numbering"]
    for d, nca in zip(g["d"], pc):
        assert nca == d * (pc[0] - 2) + 2
    # Our numbering on a smaller mesh: nnz(d) = d^2 nnz(1), same n_ca law.
    conn, nn = meshes.quad_mesh(48)
    base_nnz = base_nca = None
    for d in range(1, 9):
        row_ptr, col_idx = orc.pattern(conn, d, nn)
        _, ca = orc.crac(row_ptr, col_idx, d * nn)
        if d == 1:
            base_nnz, base_nca = row_ptr[-1], ca.size
            assert base_nnz == 21025  # the paper's 48x48 mesh (h-benchmark mesh 4)
        assert row_ptr[-1] == d * d * base_nnz
        assert ca.size == d * (base_nca - 2) + 2


@pytest.mark.slow
def test_d_benchmark_nnz_matches_paper(orc):
    g = _golden("paper_counts.json")["d_benchmark_structured"]
    conn, nn = meshes.quad_mesh(g["elements_per_side"])
    for d, want in zip(g["d"], g["nnz"]):
        row_ptr, _ = orc.pattern(conn, d, nn)
        assert row_ptr[-1] == want


def test_structured_closed_forms(orc):
    # Lexicographic structured meshes: every node row splits into runs by
    # neighbouring grid line (quads) or grid line x plane (hexes).  With at
    # least 4 nodes per side no node row's neighbourhood spans a whole grid
    # line, so runs of neighbouring lines never merge.
    for m in (3, 5, 9):
        N = m + 1
        conn, nn = meshes.quad_mesh(m)
        rp, ci = orc.pattern(conn, 1, nn)
        _, ca = orc.crac(rp, ci, nn)
        assert rp[-1] == (3 * N - 2) ** 2
        assert ca.size == 2 * N * (3 * N - 2) + 2
    for m in (3, 4):
        N = m + 1
        conn, nn = meshes.hex_mesh(m)
        rp, ci = orc.pattern(conn, 3, nn)
        _, ca = orc.crac(rp, ci, 3 * nn)
        assert rp[-1] == 9 * (3 * N - 2) ** 3
        assert ca.size == 2 * 3 * N * (3 * N - 2) ** 2 + 2


def test_tiny_mesh_counts(orc):
    conn, nn = meshes.quad_mesh(3)
    rp, ci = orc.pattern(conn, 1, nn)
    _, ca = orc.crac(rp, ci, nn)
    assert (rp[-1], (ca.size - 2) // 2, ca.size) == (100, 40, 82)
    conn, nn = meshes.hex_mesh(2)
    rp, ci = orc.pattern(conn, 3, nn)
    _, ca = orc.crac(rp, ci, 3 * nn)
    assert (rp[-1], (ca.size - 2) // 2, ca.size) == (3087, 345, 692)


# --------------------------------------------------------------------------
# Brute-force dense assembly (numpy.add.at) on tiny meshes.

TINY = [
    ("quad3_d1", lambda: meshes.quad_mesh(3), 1),
    ("quad2x3_d2", lambda: meshes.quad_mesh(2, 3), 2),
    ("hex2_d3", lambda: meshes.hex_mesh(2), 3),
    ("hex1x2x3_d1", lambda: meshes.hex_mesh(1, 2, 3), 1),
    ("tet1_d3", lambda: meshes.tet10_mesh(1), 3),
    ("tet2perm_d2", lambda: meshes.tet10_mesh(2, perm_seed=3), 2),
    ("q3quad2_d1", lambda: meshes.qp_quad_mesh(2, 3), 1),
]


def _dense_reference(conn, d, nn, ke):
    DI = dof_indices(conn, d)
    N = d * nn
    E, n = DI.shape
    rr = np.repeat(DI, n, axis=1).ravel()  # (e, r, s) order, r-major
    cc = np.tile(DI, (1, n)).ravel()
    G = np.zeros((N, N))
    np.add.at(G, (rr, cc), ke.reshape(-1))
    P = np.zeros((N, N), dtype=bool)
    P[rr, cc] = True
    A = np.zeros((N, N))
    np.add.at(A, (rr, cc), np.abs(ke.reshape(-1)))
    return G, P, A


@pytest.mark.parametrize("name,make,d", TINY, ids=[t[0] for t in TINY])
def test_bruteforce_dense(orc, name, make, d):
    conn, nn = make()
    E, k = conn.shape
    n = k * d
    N = d * nn
    ke = matrices.ke_spd(E, n, seed=11)
    G, P, A = _dense_reference(conn, d, nn, ke)
    rp, ci = orc.pattern(conn, d, nn)
    # pattern == set of touched (i, j), rows sorted ascending
    rows = np.repeat(np.arange(N), np.diff(rp))
    Pc = np.zeros((N, N), dtype=bool)
    Pc[rows, ci] = True
    assert (Pc == P).all()
    assert rp[-1] == P.sum()
    for i in range(N):
        seg = ci[rp[i]:rp[i + 1]]
        assert (np.diff(seg) > 0).all()
    # values: numpy.add.at sums in the same (e, r, s) order, so bit-exact
    vals, absv = orc.assemble(conn, d, ke, rp, ci)
    assert (vals == G[rows, ci]).all()
    assert (absv == A[rows, ci]).all()
    # CRAC lookups agree with CSR for every stored and every absent entry
    crp, ca = orc.crac(rp, ci, N)
    for i in range(N):
        for j in range(N):
            p = orc.csr_find(rp, ci, i, j)
            assert orc.crac_find(crp, ca, i, j) == p
            assert (p >= 0) == P[i, j]
    # CRAC runs are maximal: neighbouring runs of a row are not adjacent
    for i in range(N):
        pairs = ca[crp[i]:crp[i + 1]].reshape(-1, 2)
        for (c0, v0), (c1, v1) in zip(pairs[:-1], pairs[1:]):
            assert c1 > c0 + (v1 - v0)


def test_small_integer_values_exact(orc):
    conn, nn = meshes.hex_mesh(3)
    d = 2
    E, k = conn.shape
    ke = matrices.ke_small_int(E, k * d, seed=5)
    G, P, _ = _dense_reference(conn, d, nn, ke)
    rp, ci = orc.pattern(conn, d, nn)
    vals, _ = orc.assemble(conn, d, ke, rp, ci)
    rows = np.repeat(np.arange(d * nn), np.diff(rp))
    assert (vals == G[rows, ci]).all()


def test_all_ones_multiplicity(orc):
    # The paper's dummy element (all ones): every value is the number of
    # (element, r, s) triples that hit it -- exact in any order.
    conn, nn = meshes.hex_mesh(4)
    d = 3
    E, k = conn.shape
    n = k * d
    rp, ci = orc.pattern(conn, d, nn)
    vals, _ = orc.assemble(conn, d, matrices.ke_ones(E, n), rp, ci)
    assert vals.sum() == E * n * n
    DI = dof_indices(conn, d)
    cnt = np.zeros((d * nn, d * nn))
    np.add.at(cnt, (np.repeat(DI, n, axis=1).ravel(), np.tile(DI, (1, n)).ravel()), 1.0)
    rows = np.repeat(np.arange(d * nn), np.diff(rp))
    assert (vals == cnt[rows, ci]).all()
    # interior node of a structured hex mesh: 8 elements share it
    centre = 2 + 5 * 2 + 25 * 2
    p = orc.csr_find(rp, ci, 3 * centre, 3 * centre)
    assert vals[p] == 8.0


# --------------------------------------------------------------------------
# Invariants on the quad64 workload and a small SPD hex mesh.


def _matfree(conn, d, ke, x):
    """y = sum_e P_e^T (K_e x_e), an assembly-free product."""
    DI = dof_indices(conn, d)
    ye = np.einsum("ers,es->er", ke, x[DI])
    y = np.zeros_like(x)
    np.add.at(y, DI.ravel(), ye.ravel())
    return y


def _csr_matvec(rp, ci, vals, x):
    rows = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    y = np.zeros(rp.size - 1)
    np.add.at(y, rows, vals * x[ci])
    return y


def test_invariants_quad64(orc):
    conn, nn = meshes.quad_mesh(64)
    E = conn.shape[0]
    ke = matrices.ke_laplacian(E, 4, seed=0)
    # the generator's promise: bit-symmetric, zero row sums
    assert (ke == ke.transpose(0, 2, 1)).all()
    rp, ci = orc.pattern(conn, 1, nn)
    vals, absv = orc.assemble(conn, 1, ke, rp, ci)
    assert rp[-1] == 37249
    # sum of all entries == sum of all element entries (to rounding)
    assert abs(vals.sum() - ke.sum()) <= 1e-12 * np.abs(ke).sum()
    # bit symmetry: G_ij and G_ji sum mirrored terms in the same order
    rows = np.repeat(np.arange(nn), np.diff(rp))
    tpos = np.array([orc.csr_find(rp, ci, j, i) for i, j in zip(rows[:5000], ci[:5000])])
    assert (vals[:5000] == vals[tpos]).all()
    # zero row sums within the rounding bound of the row
    rs = np.zeros(nn)
    np.add.at(rs, rows, vals)
    ra = np.zeros(nn)
    np.add.at(ra, rows, absv)
    assert (np.abs(rs) <= 64 * 2.0 ** -52 * ra).all()
    # G x == sum_e P_e^T K_e x_e
    x = np.random.default_rng(1).standard_normal(nn)
    y1 = _csr_matvec(rp, ci, vals, x)
    y2 = _matfree(conn, 1, ke, x)
    assert np.abs(y1 - y2).max() <= 1e-12 * np.abs(ke).sum(axis=(1, 2)).max() * 10


def test_invariants_spd_hex(orc):
    conn, nn = meshes.hex_mesh(6)
    d = 3
    E, k = conn.shape
    ke = matrices.ke_spd(E, k * d, seed=0)
    rp, ci = orc.pattern(conn, d, nn)
    vals, absv = orc.assemble(conn, d, ke, rp, ci)
    x = np.random.default_rng(2).standard_normal(d * nn)
    y1 = _csr_matvec(rp, ci, vals, x)
    y2 = _matfree(conn, d, ke, x)
    assert np.allclose(y1, y2, rtol=1e-12, atol=1e-10)
    assert float(x @ y1) > 0.0  # energy of an SPD sum


def test_rows_match_full_assembly(orc):
    from fe_inputs import meshes as M
    conn, nn = M.tet10_mesh(3, perm_seed=0)
    d = 3
    E, k = conn.shape
    ke = matrices.ke_spd(E, k * d, seed=4)
    rp, ci = orc.pattern(conn, d, nn)
    vals, absv = orc.assemble(conn, d, ke, rp, ci)
    req = np.random.default_rng(0).choice(d * nn, size=60, replace=False)
    for i, (cols, v, a) in zip(req, orc.rows(conn, d, nn, ke, req)):
        s, e = rp[i], rp[i + 1]
        assert (cols == ci[s:e]).all()
        assert (v == vals[s:e]).all()
        assert (a == absv[s:e]).all()


# --------------------------------------------------------------------------
# Colouring (Section 3.3; colour distribution figure in Section 4).


def test_structured_quad_colouring_is_four_even(orc):
    g = _golden("paper_counts.json")["structured_colouring"]
    for m in (6, 12, 48, 64):
        conn, nn = meshes.quad_mesh(m)
        col, nc = orc.greedy_colour(conn, nn)
        assert nc == g["colours"]
        share = 100.0 * np.bincount(col) / col.size
        assert np.allclose(share, g["share_percent"])
        assert orc.colouring_valid(conn, nn, col, nc)


def test_hex_and_tet_colouring_valid(orc):
    conn, nn = meshes.hex_mesh(6)
    col, nc = orc.greedy_colour(conn, nn)
    assert nc == 8 and orc.colouring_valid(conn, nn, col, nc)
    conn, nn = meshes.tet10_mesh(4, perm_seed=0)
    col, nc = orc.greedy_colour(conn, nn)
    assert orc.colouring_valid(conn, nn, col, nc)


def test_colouring_validator_rejects_conflict(orc):
    conn, nn = meshes.quad_mesh(4)
    col, nc = orc.greedy_colour(conn, nn)
    bad = col.copy()
    bad[1] = bad[0]  # elements 0 and 1 share an edge
    assert not orc.colouring_valid(conn, nn, bad, nc)
    bad = col.copy()
    bad[5] = nc  # colour out of range
    assert not orc.colouring_valid(conn, nn, bad, nc)

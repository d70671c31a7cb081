"""Device hexahedron stiffness and the fused element-matrix + assembly path
against the oracle (GPU).

The oracle evaluates the textbook element formulas as written; the device
uses its own fixed sequence of fused multiply-adds, so the two differ by
rounding only.  Element matrices pass when |g - o| <= 1e-12 * kabs per entry
(kabs = the sum of the absolute values of the terms, from the oracle), and
assembled values against the oracle's assembly of K with the bound
assembled from kabs.  Inside the device, the fused path and the two-pass
path (element matrices, then the row-owned assembly) evaluate the same
sequence and add in element order, so they must agree bit for bit.
"""
import sys

import numpy as np
import pytest
import torch

from tests._checks import assert_values_close
from fe_inputs import matrices, meshes

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


def _case(feasm, conn, nn, x, d, seed):
    dev = torch.device("cuda:0")
    E = conn.shape[0]
    mat = matrices.hex_materials(E, d, seed=seed)
    p = feasm.pattern_build(torch.from_numpy(np.ascontiguousarray(conn)).to(dev), d, nn,
                            feasm.BUILD_CSR | feasm.BUILD_CRAC)
    return p, torch.from_numpy(x).to(dev), torch.from_numpy(np.ascontiguousarray(mat)).to(dev), mat


MESHES = [
    ("hex4_jitter", lambda: (*meshes.hex_mesh(4), meshes.hex_coords(4, jitter=0.25, seed=1))),
    ("hex3x2x5_jitter", lambda: (*meshes.hex_mesh(3, 2, 5),
                                 meshes.hex_coords(3, 2, 5, jitter=0.2, seed=2))),
    ("hex3_doubled", lambda: _doubled()),
    ("hex6x5x4_permuted_isolated", lambda: _permuted_isolated()),
    ("hex12x10x9_jitter", lambda: (*meshes.hex_mesh(12, 10, 9),
                                   meshes.hex_coords(12, 10, 9, jitter=0.25, seed=4))),
]


def _doubled():
    """Every element listed twice: nodes with up to 16 incident entries, so
    the fused kernel walks more than one batch per row."""
    conn, nn = meshes.hex_mesh(3)
    return np.concatenate([conn, conn[::-1]]), nn, meshes.hex_coords(3, jitter=0.2, seed=3)


def _permuted_isolated():
    """Relabelled nodes (the node order is no longer the geometric order)
    plus two nodes no element uses (rows without entries)."""
    conn, nn = meshes.hex_mesh(6, 5, 4)
    x = meshes.hex_coords(6, 5, 4, jitter=0.2, seed=6)
    perm = np.random.default_rng(7).permutation(nn + 2)
    xp = np.zeros((nn + 2, 3))
    xp[perm[:nn]] = x
    return perm[conn].astype(np.int32), nn + 2, xp


# fused kernel settings: 0 = pipelined light nodes (grid from occupancy),
# 1 = pipelined with one block per compute unit (several nodes per wavefront
# on the larger meshes), -1 = one node per wavefront everywhere
PIPE = [0, 1, -1]


@pytest.mark.parametrize("d", [1, 3])
@pytest.mark.parametrize("name,make", MESHES, ids=[m[0] for m in MESHES])
def test_element_matrices_and_fused_assembly(feasm, orc, name, make, d):
    conn, nn, x = make()
    say(f"[hex8] {name} d={d}")
    p, xd, md, mat = _case(feasm, conn, nn, x, d, seed=5)
    K, KA = orc.hex8_matrices(conn, x, d, mat)
    kd_t = feasm.hex8_element_matrices(p, xd, md)
    kd = _np(kd_t)
    assert_values_close(kd.ravel(), K.ravel(), KA.ravel(), what="element matrices")
    rp, ci = orc.pattern(conn, d, nn)
    ov, _ = orc.assemble(conn, d, K, rp, ci, with_abs=False)
    oa, _ = orc.assemble(conn, d, KA, rp, ci, with_abs=False)  # terms of every entry: >= 0
    # the device's two-pass result: its element matrices, assembled in element order
    two_pass = _np(feasm.assemble_crac(p, kd_t, scatter=feasm.SCATTER_OWNER))
    assert_values_close(two_pass, ov, oa, what="two-pass values")
    for pipe in PIPE:
        p.tune(feasm.TUNE_HEX8_PIPE, pipe)
        for fmt in (feasm.FMT_CSR, feasm.FMT_CRAC):
            say(f"[hex8] {name} d={d} pipe={pipe} fmt={fmt}")
            v = _np(feasm.assemble_hex8(p, fmt, xd, md))
            assert_values_close(v, ov, oa, what=f"fused values pipe={pipe} fmt={fmt}")
            assert (v == two_pass).all(), ("fused != two-pass", pipe, fmt)
            acc = torch.full((p.nnz,), 2.0, dtype=torch.float64, device="cuda")
            feasm.assemble_hex8(p, fmt, xd, md, acc, accumulate=True)
            assert_values_close(_np(acc), ov + 2.0, oa + 2.0, what="accumulated fused values")
            assert (_np(acc) == two_pass + 2.0).all(), (pipe, fmt)
    p.free()


def test_hex64_elasticity_full_size(feasm, orc):
    m = 64
    conn, nn = meshes.hex_mesh(m)
    x = meshes.hex_coords(m, jitter=0.2, seed=11)
    say("[hex8] 64^3 elasticity, full size")
    p, xd, md, mat = _case(feasm, conn, nn, x, 3, seed=12)
    K, KA = orc.hex8_matrices(conn, x, 3, mat)
    kd_t = feasm.hex8_element_matrices(p, xd, md)
    assert_values_close(_np(kd_t).ravel(), K.ravel(), KA.ravel(), what="element matrices")
    rp, ci = orc.pattern(conn, 3, nn)
    ov, _ = orc.assemble(conn, 3, K, rp, ci, with_abs=False)
    oa, _ = orc.assemble(conn, 3, KA, rp, ci, with_abs=False)
    del K, KA
    two_pass = _np(feasm.assemble_crac(p, kd_t, scatter=feasm.SCATTER_OWNER))
    del kd_t
    assert_values_close(two_pass, ov, oa, what="two-pass values")
    for pipe in PIPE:
        say(f"[hex8] 64^3 elasticity pipe={pipe}")
        p.tune(feasm.TUNE_HEX8_PIPE, pipe)
        v = _np(feasm.assemble_hex8(p, feasm.FMT_CRAC, xd, md))
        assert_values_close(v, ov, oa, what=f"fused values pipe={pipe}")
        assert (v == two_pass).all(), pipe
    p.tune(feasm.TUNE_HEX8_PIPE, 0)
    v = _np(feasm.assemble_hex8(p, feasm.FMT_CSR, xd, md))
    assert_values_close(v, ov, oa, what="fused CSR values")
    assert (v == two_pass).all()
    p.free()


def test_pipeline_setting_range(feasm):
    dev = torch.device("cuda:0")
    conn, nn = meshes.hex_mesh(2)
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), 1, nn)
    for bad in (-2, 17):
        with pytest.raises(feasm.FeasmError):
            p.tune(feasm.TUNE_HEX8_PIPE, bad)
    p.free()


def test_rejects_other_elements(feasm):
    dev = torch.device("cuda:0")
    conn, nn = meshes.quad_mesh(3)
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), 1, nn)
    x = torch.zeros(3 * nn, dtype=torch.float64, device=dev)
    m = torch.ones(p.n_elem, dtype=torch.float64, device=dev)
    with pytest.raises(feasm.FeasmError):
        feasm.assemble_hex8(p, feasm.FMT_CRAC, x, m)  # 4-node elements
    p.free()
    conn, nn = meshes.hex_mesh(2)
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), 2, nn)
    x = torch.zeros(3 * nn, dtype=torch.float64, device=dev)
    m = torch.ones(2 * p.n_elem, dtype=torch.float64, device=dev)
    with pytest.raises(feasm.FeasmError):
        feasm.assemble_hex8(p, feasm.FMT_CRAC, x, m)  # d = 2
    p.free()

"""Parity of the device matrix-vector product with the oracle (GPU).

spmv_csr and spmv_crac sum each row in increasing column order with every
product and sum rounded, as the oracle's sequential loop does, so y must
equal the oracle's bit for bit.  Values and x are seeded inputs that do not
come from the device.
"""
import sys

import numpy as np
import pytest
import torch

from fe_inputs import configs, matrices
from tests.test_gpu_parity import CASES, _fan

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


def _device_case(feasm, orc, conn, d, nn, ke, seed):
    dev = torch.device("cuda:0")
    p = feasm.pattern_build(torch.from_numpy(np.ascontiguousarray(conn, dtype=np.int32)).to(dev),
                            d, nn, feasm.BUILD_CSR | feasm.BUILD_CRAC)
    rp, ci = orc.pattern(conn, d, nn)
    vals, _ = orc.assemble(conn, d, ke, rp, ci)
    x = np.random.default_rng(seed).standard_normal(d * nn)
    y, _ = orc.spmv_csr(rp, ci, vals, x)
    vd = torch.from_numpy(vals).to(dev)
    xd = torch.from_numpy(x).to(dev)
    return p, vd, xd, y


@pytest.mark.parametrize("name,make,d", CASES, ids=[c[0] for c in CASES])
def test_small_cases_bit_exact(feasm, orc, name, make, d):
    conn, nn = make()
    E, k = conn.shape
    say(f"[spmv] {name}: E={E} k={k} d={d} nodes={nn}")
    ke = matrices.ke_spd(E, k * d, seed=12)
    p, vd, xd, y = _device_case(feasm, orc, conn, d, nn, ke, seed=2)
    for fn in (feasm.spmv_csr, feasm.spmv_crac):
        yd = torch.full_like(xd, np.nan)
        got = _np(fn(p, vd, xd, yd))
        assert (got == y).all(), fn.__name__
    p.free()


@pytest.mark.parametrize("n_tri,d", [(1200, 1), (700, 2)])
def test_rows_longer_than_a_chunk(feasm, orc, n_tri, d):
    """The centre row holds n_tri*d + d values, several LDS chunks."""
    conn, nn = _fan(n_tri)
    ke = matrices.ke_spd(conn.shape[0], 3 * d, seed=4)
    p, vd, xd, y = _device_case(feasm, orc, conn, d, nn, ke, seed=6)
    for fn in (feasm.spmv_csr, feasm.spmv_crac):
        assert (_np(fn(p, vd, xd)) == y).all(), fn.__name__
    p.free()


def test_hex64_full_bit_exact(feasm, orc):
    w = configs.hex64()
    say("[spmv] hex64 full size")
    ke = w.ke()
    p, vd, xd, y = _device_case(feasm, orc, w.conn, 3, w.n_nodes, ke, seed=5)
    for fn in (feasm.spmv_csr, feasm.spmv_crac):
        got = _np(fn(p, vd, xd))
        assert (got == y).all(), fn.__name__
    p.free()


def test_tet40_full_bit_exact(feasm, orc, tet40_ref):
    """Full-size permuted tet10 mesh: the oracle's assembled values, every
    row of y through CSR and CRAC against the oracle's product."""
    r = tet40_ref
    say("[spmv] tet40 full size")
    dev = torch.device("cuda:0")
    p = feasm.pattern_build(torch.from_numpy(r.w.conn).to(dev), 3, r.w.n_nodes,
                            feasm.BUILD_CSR | feasm.BUILD_CRAC)
    x = np.random.default_rng(8).standard_normal(p.n_rows)
    y, _ = orc.spmv_csr(r.rp, r.ci, r.ov, x, with_abs=False)
    vd, xd = torch.from_numpy(r.ov).to(dev), torch.from_numpy(x).to(dev)
    for fn in (feasm.spmv_csr, feasm.spmv_crac):
        got = _np(fn(p, vd, xd))
        assert (got == y).all(), fn.__name__
    p.free()


def test_rejects_bad_arguments(feasm):
    from fe_inputs import meshes

    dev = torch.device("cuda:0")
    conn, nn = meshes.quad_mesh(3)
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), 1, nn, feasm.BUILD_CSR)
    v = torch.zeros(p.nnz, dtype=torch.float64, device=dev)
    x = torch.zeros(p.n_rows, dtype=torch.float64, device=dev)
    with pytest.raises(feasm.FeasmError):
        feasm.spmv_crac(p, v, x)  # handle built without CRAC
    with pytest.raises(feasm.FeasmError):
        feasm.spmv_csr(p, v, x, x)  # y overlaps x
    p.free()

"""Random small meshes through every device path (GPU).

Random connectivity with repeated and unused nodes and small-integer
element matrices, whose sums are exact in any order: the pattern, the
values of every strategy and format, re-assembly and the matrix-vector
product must equal the oracle bit for bit.
"""
import sys

import numpy as np
import pytest
import torch

from fe_inputs import matrices
from tests.test_oracle_random import _random_mesh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def feasm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_00585_amd as f

    f.load()
    return f


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("seed", range(24))
def test_random_mesh_every_path(feasm, orc, seed):
    rng = np.random.default_rng(5000 + seed)
    conn, nn, d = _random_mesh(rng)
    E, k = conn.shape
    print(f"[random] seed={seed} E={E} k={k} d={d} nodes={nn}", flush=True)
    sys.stdout.flush()
    ke = matrices.ke_small_int(E, k * d, seed=seed)
    dev = torch.device("cuda:0")
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), d, nn,
                            feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_COLOUR)
    rp, ci = orc.pattern(conn, d, nn)
    crp, ca = orc.crac(rp, ci, d * nn)
    grp, gci = (_np(t) for t in p.csr())
    gcrp, gca = (_np(t) for t in p.crac())
    assert (grp == rp).all() and (gci == ci).all()
    assert (gcrp == crp).all() and (gca == ca).all()
    ov, _ = orc.assemble(conn, d, ke, rp, ci)
    ke_d = torch.from_numpy(ke).to(dev)
    for sc in (feasm.SCATTER_AUTO, feasm.SCATTER_ATOMIC, feasm.SCATTER_COLOURED,
               feasm.SCATTER_OWNER):
        for fn, fmt in ((feasm.assemble_csr, feasm.FMT_CSR), (feasm.assemble_crac, feasm.FMT_CRAC)):
            assert (_np(fn(p, ke_d, scatter=sc)) == ov).all(), (sc, fmt)
            for _ in range(2):  # recording call, then the recorded path
                assert (_np(feasm.reassemble_values(p, fmt, ke_d, scatter=sc)) == ov).all()
    x = rng.integers(-5, 6, size=d * nn).astype(np.float64)
    y, _ = orc.spmv_csr(rp, ci, ov, x)
    vd, xd = torch.from_numpy(ov).to(dev), torch.from_numpy(x).to(dev)
    assert (_np(feasm.spmv_csr(p, vd, xd)) == y).all()
    assert (_np(feasm.spmv_crac(p, vd, xd)) == y).all()
    p.free()

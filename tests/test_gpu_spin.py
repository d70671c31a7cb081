"""Row-lock scatter (FEASM_SCATTER_SPIN, the GPU form of the paper's
spin-lock methods) against the oracle (GPU).

Rows are summed in lock order, so values agree with the oracle within the
per-entry reorder bound for real matrices and exactly for small-integer
matrices; no lane may reach the spin limit.  The give-up path is exercised
from the host with a spin limit of zero attempts."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from fe_inputs import configs, matrices, meshes
from tests.test_gpu_parity import CASES, check_against_oracle, run_device

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


def _strategies(feasm):
    return [("csr", feasm.SCATTER_SPIN), ("crac", feasm.SCATTER_SPIN)]


@pytest.mark.parametrize("name,make,d", CASES, ids=[c[0] for c in CASES])
def test_small_cases(feasm, orc, name, make, d):
    conn, nn = make()
    E, k = conn.shape
    if k * d > 32:
        # element rows longer than the lanes hold: a documented limit
        p = feasm.pattern_build(torch.from_numpy(np.ascontiguousarray(conn)).cuda(), d, nn)
        ke = torch.zeros((E, k * d, k * d), dtype=torch.float64, device="cuda")
        with pytest.raises(feasm.FeasmError, match="ELIMIT"):
            feasm.assemble_csr(p, ke, scatter=feasm.SCATTER_SPIN)
        p.free()
        return
    for exact, ke in ((False, matrices.ke_spd(E, k * d, seed=3)),
                      (True, matrices.ke_small_int(E, k * d, seed=9))):
        say(f"[spin] {name}: E={E} k={k} d={d} exact={exact}")
        res = run_device(feasm, conn, d, nn, ke, strategies=_strategies(feasm))
        check_against_oracle(orc, conn, d, nn, ke, res, exact=exact)
        assert res["p"].spin_aborts() == 0
        res["p"].free()


def test_hex16_all_ones_exact(feasm, orc):
    conn, nn = meshes.hex_mesh(16)
    E, k = conn.shape
    ke = matrices.ke_ones(E, k * 3)
    say("[spin] hex16 all-ones")
    res = run_device(feasm, conn, 3, nn, ke, strategies=_strategies(feasm))
    check_against_oracle(orc, conn, 3, nn, ke, res, exact=True)
    assert res["p"].spin_aborts() == 0
    res["p"].free()


def test_hex64_full_within_tolerance(feasm, orc):
    w = configs.hex64()
    say("[spin] hex64 full size")
    ke = w.ke()
    dev = torch.device("cuda:0")
    p = feasm.pattern_build(torch.from_numpy(w.conn).to(dev), 3, w.n_nodes,
                            feasm.BUILD_CSR | feasm.BUILD_CRAC)
    rp, ci = orc.pattern(w.conn, 3, w.n_nodes)
    ov, oa = orc.assemble(w.conn, 3, ke, rp, ci)
    ke_d = torch.from_numpy(ke).to(dev)
    for fn in (feasm.assemble_csr, feasm.assemble_crac):
        v = _np(fn(p, ke_d, scatter=feasm.SCATTER_SPIN))
        assert (np.abs(v - ov) <= 1e-12 * oa).all(), fn.__name__
    assert p.spin_aborts() == 0
    p.free()


def test_give_up_path(feasm):
    """A spin limit of zero attempts makes every lane give up: nothing is
    added and every element row is counted; the default limit again adds
    everything."""
    conn, nn = meshes.hex_mesh(3)
    E, k = conn.shape
    dev = torch.device("cuda:0")
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), 3, nn)
    ke = torch.ones((E, 24, 24), dtype=torch.float64, device=dev)
    p.tune(feasm.TUNE_SPIN_LIMIT, -1)
    v = _np(feasm.assemble_crac(p, ke, scatter=feasm.SCATTER_SPIN))
    assert (v == 0).all()
    c = ctypes.c_int64()
    assert feasm._lib.load().spin_aborts(p.handle, ctypes.byref(c)) == feasm._lib.FEASM_EINCOMPLETE
    assert c.value == E * 24
    assert feasm._lib.load().spin_aborts(p.handle, ctypes.byref(c)) == 0  # cleared by the read
    assert c.value == 0
    v = _np(feasm.assemble_crac(p, ke, scatter=feasm.SCATTER_SPIN))
    assert p.spin_aborts() == E * 24
    assert p.spin_aborts() == 0
    p.tune(feasm.TUNE_SPIN_LIMIT, 0)
    v = _np(feasm.assemble_crac(p, ke, scatter=feasm.SCATTER_SPIN))
    assert v.sum() == E * 24 * 24
    assert p.spin_aborts() == 0
    with pytest.raises(feasm.FeasmError):
        p.tune(feasm.TUNE_SPIN_LIMIT, -2)
    p.free()

"""assemble_spin_noalloc, the row-lock scatter that allocates nothing
(GPU), against the allocating row-lock scatter (assemble_csr /
assemble_crac with FEASM_SCATTER_SPIN) through the C ABI.

Both sum each value's contributions in lock order, so they agree exactly
on small-integer element matrices and within the per-entry reorder bound
of the oracle (|g - o| <= 1e-12 * sum |contributions|) on real ones.  Two
calls in a row on the shared static lock array, the second on a smaller
mesh, must both be right; a mesh beyond the array is rejected."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from fe_inputs import matrices, meshes

pytestmark = pytest.mark.gpu

MAX_ROWS = 1 << 21


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def feasm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_00585_amd as feasm

    feasm.load()
    return feasm


def _noalloc(feasm, p, fmt, ke_d, values, aborts, flags=0):
    lib = feasm._lib.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.assemble_spin_noalloc(p.handle, fmt, ctypes.c_void_p(ke_d.data_ptr()),
                                   ctypes.c_void_p(values.data_ptr()),
                                   ctypes.c_void_p(aborts.data_ptr()), flags, stream)
    return rc


def _case(feasm, orc, conn, nn, d, ke, label):
    """Both row-lock entry points on one mesh, both formats; returns the
    no-alloc values of the last call."""
    dev = torch.device("cuda:0")
    E, k = conn.shape
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), d, nn)
    rp, ci = orc.pattern(conn, d, nn)
    ov, oa = orc.assemble(conn, d, ke, rp, ci)
    exact = bool((np.round(ke) == ke).all())
    ke_d = torch.from_numpy(ke).to(dev)
    for fmt, fn in ((feasm.FMT_CSR, feasm.assemble_csr), (feasm.FMT_CRAC, feasm.assemble_crac)):
        say(f"[no-alloc] {label}: fmt {fmt}, E={E}, n_rows={p.n_rows}")
        ref = fn(p, ke_d, scatter=feasm.SCATTER_SPIN).cpu().numpy()
        assert p.spin_aborts() == 0
        # stale values and lock words from elsewhere must not matter
        values = torch.full((p.nnz,), float("nan"), dtype=torch.float64, device=dev)
        aborts = torch.zeros(1, dtype=torch.int32, device=dev)
        assert _noalloc(feasm, p, fmt, ke_d, values, aborts) == 0
        torch.cuda.synchronize()
        got = values.cpu().numpy()
        assert int(aborts.item()) == 0
        if exact:
            assert (got == ref).all() and (got == ov).all()
        else:
            assert (np.abs(got - ov) <= 1e-12 * oa).all()
            assert (np.abs(ref - ov) <= 1e-12 * oa).all()
            assert (np.abs(got - ref) <= 2e-12 * oa).all()
        # accumulate: a second pass doubles every sum
        assert _noalloc(feasm, p, fmt, ke_d, values, aborts, feasm.ACCUMULATE) == 0
        torch.cuda.synchronize()
        twice = values.cpu().numpy()
        if exact:
            assert (twice == 2 * ov).all()
        else:
            assert (np.abs(twice - 2 * ov) <= 2e-12 * oa).all()
    p.free()
    return got


def test_two_calls_second_smaller(feasm, orc):
    conn, nn = meshes.hex_mesh(8)
    E, k = conn.shape
    rng = np.random.default_rng(5)
    ke_int = rng.integers(-3, 4, size=(E, k * 3, k * 3)).astype(np.float64)
    _case(feasm, orc, conn, nn, 3, ke_int, "hex 8^3 integer")
    qconn, qnn = meshes.quad_mesh(5)
    _case(feasm, orc, qconn, qnn, 1, matrices.ke_laplacian(qconn.shape[0], 4, seed=1),
          "quad 5^2 real (smaller)")


def test_real_matrices_then_smaller(feasm, orc):
    conn, nn = meshes.hex_mesh(6)
    _case(feasm, orc, conn, nn, 3, matrices.ke_spd(conn.shape[0], 24, seed=2), "hex 6^3 SPD")
    conn, nn = meshes.hex_mesh(3)
    _case(feasm, orc, conn, nn, 2, matrices.ke_spd(conn.shape[0], 16, seed=4), "hex 3^3 d=2")


def test_give_up_count_goes_to_the_caller(feasm):
    conn, nn = meshes.hex_mesh(3)
    E, k = conn.shape
    dev = torch.device("cuda:0")
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), 3, nn)
    ke = torch.ones((E, 24, 24), dtype=torch.float64, device=dev)
    values = torch.empty(p.nnz, dtype=torch.float64, device=dev)
    aborts = torch.zeros(1, dtype=torch.int32, device=dev)
    say("[no-alloc] give-up path (spin limit -1)")
    p.tune(feasm.TUNE_SPIN_LIMIT, -1)
    assert _noalloc(feasm, p, feasm.FMT_CRAC, ke, values, aborts) == 0
    torch.cuda.synchronize()
    assert int(aborts.item()) == E * 24
    assert (values.cpu().numpy() == 0).all()
    p.tune(feasm.TUNE_SPIN_LIMIT, 0)
    aborts.zero_()
    assert _noalloc(feasm, p, feasm.FMT_CRAC, ke, values, aborts) == 0
    torch.cuda.synchronize()
    assert int(aborts.item()) == 0
    assert values.sum().item() == E * 24 * 24
    p.free()


def test_rejects_what_it_cannot_hold(feasm):
    lib = feasm._lib.load()
    dev = torch.device("cuda:0")
    conn, nn = meshes.quad_mesh(1450)  # 1451^2 nodes, d = 1: above 2^21 rows
    assert nn > MAX_ROWS
    say(f"[no-alloc] rejection: {nn} rows")
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), 1, nn, feasm.BUILD_CSR)
    small = torch.zeros(16, dtype=torch.float64, device=dev)
    aborts = torch.zeros(1, dtype=torch.int32, device=dev)
    assert _noalloc(feasm, p, feasm.FMT_CSR, small, small, aborts) == -6  # ELIMIT
    assert b"2^21" in lib.last_error()
    assert _noalloc(feasm, p, feasm.FMT_CRAC, small, small, aborts) == -1  # no CRAC built
    assert _noalloc(feasm, p, feasm.FMT_CSR, small, small, aborts, flags=7) == -1
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.assemble_spin_noalloc(p.handle, 0, ctypes.c_void_p(small.data_ptr()),
                                     ctypes.c_void_p(small.data_ptr()), None, 0, stream) == -1
    p.free()

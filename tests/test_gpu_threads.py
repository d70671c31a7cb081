"""Several host threads sharing one handle (GPU).

The first value-only re-assembly of a strategy family creates the handle's
lookup record; when four threads make that first call at once, on their own
streams, the record must be made once and every thread must get the values
a single-threaded call gives (bit-exact for the row-owned strategy, within
the per-entry reorder bound of the oracle for the atomic one)."""
import sys
import threading

import numpy as np
import pytest
import torch

from fe_inputs import matrices, meshes

pytestmark = pytest.mark.gpu

N_THREADS = 4


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


def _run_threads(feasm, p, ke_d, fmt, scatter):
    dev = ke_d.device
    streams = [torch.cuda.Stream(device=dev) for _ in range(N_THREADS)]
    outs = [torch.full((p.nnz,), float("nan"), dtype=torch.float64, device=dev)
            for _ in range(N_THREADS)]
    torch.cuda.synchronize()
    errors = []
    start = threading.Barrier(N_THREADS)

    def work(i):
        try:
            start.wait()
            feasm.reassemble_values(p, fmt, ke_d, values=outs[i], scatter=scatter,
                                    stream=streams[i])
            streams[i].synchronize()
        except Exception as ex:  # reported in the main thread
            errors.append(ex)

    threads = [threading.Thread(target=work, args=(i,)) for i in range(N_THREADS)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    return [o.cpu().numpy() for o in outs]


@pytest.mark.parametrize("fmt_name", ["CSR", "CRAC"])
def test_first_reassembly_from_four_threads(feasm, orc, fmt_name):
    conn, nn = meshes.hex_mesh(10)
    d = 3
    E, k = conn.shape
    ke = matrices.ke_spd(E, k * d, seed=3)
    say(f"[threads] hex 10^3, {fmt_name}, {N_THREADS} threads, first re-assembly")
    dev = torch.device("cuda:0")
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), d, nn)
    rp, ci = orc.pattern(conn, d, nn)
    ov, oa = orc.assemble(conn, d, ke, rp, ci)
    ke_d = torch.from_numpy(ke).to(dev)
    fmt = feasm.FMT_CSR if fmt_name == "CSR" else feasm.FMT_CRAC
    for v in _run_threads(feasm, p, ke_d, fmt, feasm.SCATTER_OWNER):
        assert (v == ov).all()
    for v in _run_threads(feasm, p, ke_d, fmt, feasm.SCATTER_ATOMIC):
        assert (np.abs(v - ov) <= 1e-12 * oa).all()
    p.free()

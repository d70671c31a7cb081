"""Tiled hardware-atomic scatter (handles built with FEASM_BUILD_TILES)
against the oracle (GPU).

A tile's workgroup sums its elements' contributions per distinct (row,
column) in LDS and writes each sum once: a plain store where the tile holds
every element coupling the two nodes, an atomic add otherwise.  The values
are sums of the same contributions in another order, so they agree with the
oracle within the per-entry reorder bound, and exactly for small-integer
element matrices.  A wrongly "complete" pair would overwrite another tile's
sum and fail these checks.  Covered: the small and ragged meshes of the
parity test (tiles of any shape, elements too large for tiles, a node shared
by 400 elements, a repeated node), accumulate mode, every tile size from one
element to the largest, tiles whose pairs exceed the accumulator (those
elements take the one-atomic-per-entry kernel), and the 64^3 hexahedra and
the permuted tet10 mesh in full."""
import sys

import numpy as np
import pytest
import torch

from fe_inputs import configs, matrices
from tests._checks import assert_values_close
from tests.test_gpu_parity import CASES

pytestmark = pytest.mark.gpu


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


def _np(t):
    return t.detach().cpu().numpy()


def _build(feasm, conn, d, nn):
    dev = torch.device("cuda:0")
    return feasm.pattern_build(torch.from_numpy(np.ascontiguousarray(conn, dtype=np.int32)).to(dev),
                               d, nn, feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_TILES)


def _check_all(feasm, p, ke_d, ov, oa, exact, what):
    for fmt, fn in (("csr", feasm.assemble_csr), ("crac", feasm.assemble_crac)):
        v = _np(fn(p, ke_d, scatter=feasm.SCATTER_ATOMIC))
        if exact:
            assert (v == ov).all(), f"{what} {fmt}"
        else:
            assert_values_close(v, ov, oa, what=f"{what} {fmt}")
        fcode = feasm.FMT_CSR if fmt == "csr" else feasm.FMT_CRAC
        r = _np(feasm.reassemble_values(p, fcode, ke_d, scatter=feasm.SCATTER_ATOMIC))
        if exact:
            assert (r == ov).all(), f"{what} {fmt} re-assembly"
        else:
            assert_values_close(r, ov, oa, what=f"{what} {fmt} re-assembly")


@pytest.mark.parametrize("name,make,d", CASES, ids=[c[0] for c in CASES])
def test_small_cases(feasm, orc, name, make, d):
    conn, nn = make()
    E, k = conn.shape
    say(f"[tiles] {name}: E={E} k={k} d={d}")
    p = _build(feasm, conn, d, nn)
    rp, ci = orc.pattern(conn, d, nn)
    dev = torch.device("cuda:0")
    ke = matrices.ke_spd(E, k * d, seed=7)
    ov, oa = orc.assemble(conn, d, ke, rp, ci)
    _check_all(feasm, p, torch.from_numpy(ke).to(dev), ov, oa, False, name)
    kei = matrices.ke_small_int(E, k * d, seed=8)
    ovi, _ = orc.assemble(conn, d, kei, rp, ci)
    _check_all(feasm, p, torch.from_numpy(kei).to(dev), ovi, None, True, name + " integer")
    p.free()


def test_accumulate_and_every_tile_size(feasm, orc):
    from fe_inputs import meshes

    conn, nn = meshes.hex_mesh(9, 7, 5)
    d = 3
    E, k = conn.shape
    dev = torch.device("cuda:0")
    p = _build(feasm, conn, d, nn)
    rp, ci = orc.pattern(conn, d, nn)
    kei = matrices.ke_small_int(E, k * d, seed=9)
    ov, _ = orc.assemble(conn, d, kei, rp, ci)
    ke_d = torch.from_numpy(kei).to(dev)
    for cap in (1, 2, 3, 7, 16, 33, 64, 0):
        say(f"[tiles] hex 9x7x5 integer, tile cap {cap}")
        p.tune(feasm.TUNE_TILE_CAP, cap)
        for fn in (feasm.assemble_csr, feasm.assemble_crac):
            v = fn(p, ke_d, scatter=feasm.SCATTER_ATOMIC)
            assert (_np(v) == ov).all(), (cap, fn.__name__)
            fn(p, ke_d, values=v, scatter=feasm.SCATTER_ATOMIC | feasm.ACCUMULATE)
            assert (_np(v) == 2 * ov).all(), (cap, fn.__name__, "accumulate")
    p.free()


def test_tiles_beyond_the_accumulator(feasm, orc):
    """Tet10 tiles of up to 40 elements hold far more distinct node pairs
    than the accumulator: their elements take the per-entry atomic kernel,
    the rest the tiles."""
    from fe_inputs import meshes

    conn, nn = meshes.tet10_mesh(4, perm_seed=3)
    d = 3
    E, k = conn.shape
    dev = torch.device("cuda:0")
    p = _build(feasm, conn, d, nn)
    rp, ci = orc.pattern(conn, d, nn)
    kei = matrices.ke_small_int(E, k * d, seed=10)
    ov, _ = orc.assemble(conn, d, kei, rp, ci)
    ke_d = torch.from_numpy(kei).to(dev)
    for cap in (64, 12, 0):
        say(f"[tiles] tet10 4^3 integer, tile cap {cap}")
        p.tune(feasm.TUNE_TILE_CAP, cap)
        for fn in (feasm.assemble_csr, feasm.assemble_crac):
            assert (_np(fn(p, ke_d, scatter=feasm.SCATTER_ATOMIC)) == ov).all(), (cap, fn.__name__)
    p.free()


def test_tile_cap_rejected_without_tiles(feasm):
    from fe_inputs import meshes

    conn, nn = meshes.quad_mesh(3)
    dev = torch.device("cuda:0")
    p = feasm.pattern_build(torch.from_numpy(conn).to(dev), 1, nn)
    with pytest.raises(feasm.FeasmError):
        p.tune(feasm.TUNE_TILE_CAP, 8)
    p.free()
    p = _build(feasm, conn, 1, nn)
    with pytest.raises(feasm.FeasmError):
        p.tune(feasm.TUNE_TILE_CAP, 65)
    p.free()


def test_hex64_full(feasm, orc):
    w = configs.hex64()
    say("[tiles] hex64 full size")
    ke = w.ke()
    p = _build(feasm, w.conn, 3, w.n_nodes)
    rp, ci = orc.pattern(w.conn, 3, w.n_nodes)
    ov, oa = orc.assemble(w.conn, 3, ke, rp, ci)
    _check_all(feasm, p, torch.from_numpy(ke).to(torch.device("cuda:0")), ov, oa, False, "hex64")
    p.free()


def test_tet40_full(feasm, orc, tet40_ref):
    r = tet40_ref
    say("[tiles] tet40 full size")
    p = _build(feasm, r.w.conn, 3, r.w.n_nodes)
    _check_all(feasm, p, torch.from_numpy(r.ke).to(torch.device("cuda:0")), r.ov, r.oa, False,
               "tet40")
    p.free()

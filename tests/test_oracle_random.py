"""Randomised pins of the oracle on small random meshes (CPU).

Random connectivity -- arbitrary node ids, repeated nodes inside an element,
nodes no element uses -- is checked against dense brute force computed with
numpy alone: the pattern is the set of touched (row, column) pairs, values
are the element contributions summed in (element, row, column) order, every
CSR and CRAC lookup agrees with the dense pattern, and the matrix-vector
product satisfies G x = sum_e P_e^T K_e x_e exactly with small integers.
"""
import numpy as np
import pytest

from fe_inputs import matrices
from tests._checks import dof_indices


def _random_mesh(rng):
    k = int(rng.integers(2, 7))
    E = int(rng.integers(1, 12))
    n_nodes = int(rng.integers(k, 3 * k + 8))
    conn = rng.integers(0, n_nodes, size=(E, k)).astype(np.int32)
    d = int(rng.integers(1, 4))
    return conn, n_nodes, d


@pytest.mark.parametrize("seed", range(40))
def test_random_mesh_against_brute_force(orc, seed):
    rng = np.random.default_rng(1000 + seed)
    conn, nn, d = _random_mesh(rng)
    E, k = conn.shape
    n = k * d
    N = d * nn
    ke = matrices.ke_small_int(E, n, seed=seed)
    DI = dof_indices(conn, d)
    rr = np.repeat(DI, n, axis=1).ravel()
    cc = np.tile(DI, (1, n)).ravel()
    G = np.zeros((N, N))
    np.add.at(G, (rr, cc), ke.reshape(-1))
    P = np.zeros((N, N), dtype=bool)
    P[rr, cc] = True
    rp, ci = orc.pattern(conn, d, nn)
    rows = np.repeat(np.arange(N), np.diff(rp))
    Pc = np.zeros((N, N), dtype=bool)
    Pc[rows, ci] = True
    assert (Pc == P).all() and rp[-1] == P.sum()
    vals, _ = orc.assemble(conn, d, ke, rp, ci)
    assert (vals == G[rows, ci]).all()
    crp, ca = orc.crac(rp, ci, N)
    assert ca.size == 2 * orc.lib().orc_crac_count(orc._p(rp), orc._p(ci), N) + 2
    for i in range(N):
        for j in range(N):
            p = orc.csr_find(rp, ci, i, j)
            assert (p >= 0) == P[i, j]
            assert orc.crac_find(crp, ca, i, j) == p
    x = rng.integers(-5, 6, size=N).astype(np.float64)
    y, _ = orc.spmv_csr(rp, ci, vals, x)
    ref = np.zeros(N)
    np.add.at(ref, DI.ravel(), np.einsum("ers,es->er", ke, x[DI]).ravel())
    assert (y == ref).all()
    assert (orc.spmv_crac(crp, ca, vals, x) == y).all()

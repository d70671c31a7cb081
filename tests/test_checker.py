"""The value checker against planted mistakes (CPU).

The parity tests accept a device result when every entry is within
``1e-12 * A`` of the oracle (``A`` = sum of the absolute values of the
entry's contributions).  These tests plant the mistakes a broken scatter
makes -- one contribution dropped, one added twice, one added at the
transposed position -- into the oracle's own result, and require the
checker to reject every one of them on small meshes of each workload kind,
while it accepts the same result summed in other orders.
"""
import numpy as np
import pytest

from fe_inputs import matrices, meshes
from tests._checks import assert_values_close, dof_indices


def _cases():
    qc, qn = meshes.quad_mesh(3)
    hc, hn = meshes.hex_mesh(2)
    tc, tn = meshes.tet10_mesh(1, perm_seed=0)
    return [
        ("quad3 laplacian", qc, qn, 1, matrices.ke_laplacian(qc.shape[0], 4, 3)),
        ("hex2 spd", hc, hn, 3, matrices.ke_spd(hc.shape[0], 24, 4)),
        ("tet10 cube spd", tc, tn, 3, matrices.ke_spd(tc.shape[0], 30, 5)),
    ]


def _positions(orc, rp, ci, D):
    """CSR position of every contribution (e, r, s), by the oracle's search."""
    E, n = D.shape
    pos = np.empty((E, n, n), dtype=np.int64)
    for e in range(E):
        for r in range(n):
            for s in range(n):
                pos[e, r, s] = orc.csr_find(rp, ci, D[e, r], D[e, s])
    assert (pos >= 0).all()
    return pos


def _rejects(g, o, a):
    try:
        assert_values_close(g, o, a)
    except AssertionError:
        return True
    return False


@pytest.mark.parametrize("case", range(3), ids=["quad3", "hex2", "tet10_cube"])
def test_checker_rejects_every_dropped_doubled_or_misplaced_contribution(orc, case):
    name, conn, nn, d, ke = _cases()[case]
    rp, ci = orc.pattern(conn, d, nn)
    ov, oa = orc.assemble(conn, d, ke, rp, ci)
    assert_values_close(ov, ov, oa)
    D = dof_indices(conn, d)
    pos = _positions(orc, rp, ci, D)
    E, n, _ = ke.shape
    # a reordered sum must pass: elements in reverse order, rows reversed
    rev = np.zeros_like(ov)
    for e in reversed(range(E)):
        for r in reversed(range(n)):
            for s in range(n):
                rev[pos[e, r, s]] += ke[e, r, s]
    assert_values_close(rev, ov, oa)
    missed = []
    for e in range(E):
        for r in range(n):
            for s in range(n):
                p, v = pos[e, r, s], ke[e, r, s]
                if v == 0.0:
                    continue  # nothing to lose
                dropped = ov.copy()
                dropped[p] -= v
                doubled = ov.copy()
                doubled[p] += v
                if not (_rejects(dropped, ov, oa) and _rejects(doubled, ov, oa)):
                    missed.append((e, r, s))
                if r != s and D[e, r] != D[e, s]:
                    # added at the transposed global position instead
                    q = pos[e, s, r]
                    moved = ov.copy()
                    moved[p] -= v
                    moved[q] += v
                    if abs(ke[e, s, r] - v) > 0 and not _rejects(moved, ov, oa):
                        # only a symmetric matrix may hide a transposition
                        missed.append(("T", e, r, s))
    symmetric = np.array_equal(ke, ke.transpose(0, 2, 1))
    assert not [m for m in missed if m[0] != "T"], (name, missed[:5])
    if not symmetric:
        assert not missed, (name, missed[:5])


def test_checker_bound_sits_between_rounding_and_mistakes(orc):
    """The bound sits between reordering error and a real mistake: noise of
    1e-14 * A passes, an error of 1e-11 * A fails."""
    conn, nn = meshes.hex_mesh(2)
    ke = matrices.ke_spd(conn.shape[0], 24, 9)
    rp, ci = orc.pattern(conn, 3, nn)
    ov, oa = orc.assemble(conn, 3, ke, rp, ci)
    rng = np.random.default_rng(0)
    noise = rng.uniform(-1, 1, ov.size) * 1e-14 * oa
    assert_values_close(ov + noise, ov, oa)
    bad = ov.copy()
    bad[rng.integers(ov.size)] += 1e-11 * oa.max()
    assert _rejects(bad, ov, oa)

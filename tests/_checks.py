"""Shared test helpers: the value tolerance and small reference computations.

Tolerance (FP64 values): a computed entry ``g`` passes against the oracle's
``o`` when ``|g - o| <= rtol * A`` with ``A`` the sum of the absolute values
of the contributions to that entry and ``rtol = 1e-12``.  Any summation
order of ``m`` terms is within ``(m - 1) * 2^-53 * A`` of the exact sum, so
a correct kernel lands far inside the bound while a dropped or duplicated
contribution (an error of the size of a whole term) does not.
"""
from __future__ import annotations

import numpy as np

RTOL = 1e-12


def assert_values_close(g, o, abssum, rtol=RTOL, what="values"):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    a = np.asarray(abssum, dtype=np.float64)
    assert g.shape == o.shape == a.shape, (g.shape, o.shape, a.shape)
    err = np.abs(g - o)
    bad = np.nonzero(err > rtol * a)[0]
    if bad.size:
        i = bad[0]
        raise AssertionError(
            f"{what}: {bad.size} of {g.size} entries outside |g-o| <= {rtol}*A; "
            f"first at {i}: g={g[i]!r} o={o[i]!r} A={a[i]!r}")


def dense_from_csr(row_ptr, col_idx, values, n_rows, n_cols):
    M = np.zeros((n_rows, n_cols), dtype=np.float64)
    for i in range(n_rows):
        for p in range(row_ptr[i], row_ptr[i + 1]):
            M[i, col_idx[p]] = values[p]
    return M


def dof_indices(conn, d):
    """Node-major DOF indices of every element, [E, k*d] (test-side, numpy)."""
    conn = np.asarray(conn, dtype=np.int64)
    E, k = conn.shape
    return (d * conn[:, :, None] + np.arange(d)[None, None, :]).reshape(E, k * d)

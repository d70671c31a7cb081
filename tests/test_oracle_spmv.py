"""Pins of the oracle's matrix-vector product y = G x (CSR and CRAC runs).

The product is the use of the CRAC runs the paper names in its conclusions
and outlook; its definition is the textbook one.  The oracle computes it
twice, through CSR and through the CRAC pairs, with separate code; the pins
tie both to things fixed independently of that code: exact rational
arithmetic on Fig. 1, dense brute force, the element-wise identity
G x = sum_e P_e^T K_e x_e (exact with small integers), zero row sums of
Laplacian-type element matrices, and symmetry.
"""
from fractions import Fraction

import numpy as np
import pytest

from fe_inputs import matrices, meshes
from tests._checks import dof_indices
from tests.test_oracle_pins import TINY, _dense_reference, _golden

EPS = 2.0 ** -53


def test_fig1_product_exact_rational(orc):
    g = _golden("fig1_csr_crac.json")
    rp = np.array(g["csr_row_ptr"]) - 1
    ci = np.array(g["csr_col_idx"]) - 1
    vals = np.array(g["values"])
    ca = np.array([6 if c is None else c for c in g["crac_ca"]]) - 1
    ca[-2] = 6  # the final pair's column is n_cols
    crp = np.array(g["crac_row_ptr"]) - 1
    x = np.array([3.0, -1.0, 0.5, 2.0, -4.0, 1.25])
    y, ya = orc.spmv_csr(rp, ci, vals, x)
    yc = orc.spmv_crac(crp, ca, vals, x)
    dense = [[Fraction(str(v)) for v in row] for row in g["dense"]]
    for i in range(6):
        exact = sum(dense[i][j] * Fraction(x[j]) for j in range(6))
        bound = sum(abs(float(dense[i][j]) * x[j]) for j in range(6))
        # printed decimals are rounded to binary once; 6 terms of rounding
        assert abs(Fraction(y[i]) - exact) <= Fraction(12 * EPS * bound)
    assert (y == yc).all()
    assert ya[0] == abs(1.21 * 3.0) + abs(83.2 * -1.0)


@pytest.mark.parametrize("name,make,d", TINY, ids=[t[0] for t in TINY])
def test_bruteforce_dense_product(orc, name, make, d):
    conn, nn = make()
    E, k = conn.shape
    ke = matrices.ke_spd(E, k * d, seed=21)
    G, _, _ = _dense_reference(conn, d, nn, ke)
    rp, ci = orc.pattern(conn, d, nn)
    vals, _ = orc.assemble(conn, d, ke, rp, ci)
    crp, ca = orc.crac(rp, ci, d * nn)
    x = np.random.default_rng(3).standard_normal(d * nn)
    y, ya = orc.spmv_csr(rp, ci, vals, x)
    ref = G @ x
    bound = np.abs(G) @ np.abs(x)
    assert (np.abs(y - ref) <= 1e-12 * bound).all()
    assert (ya >= np.abs(y)).all()
    assert (orc.spmv_crac(crp, ca, vals, x) == y).all()


@pytest.mark.parametrize("make,d", [(lambda: meshes.hex_mesh(4), 3),
                                    (lambda: meshes.tet10_mesh(2, perm_seed=5), 3),
                                    (lambda: meshes.qp_quad_mesh(3, 4), 2)])
def test_elementwise_identity_exact(orc, make, d):
    """G x = sum_e P_e^T (K_e x_e): with small integers every step is exact,
    so the two sides agree bit for bit and any dropped, doubled or misplaced
    term shows."""
    conn, nn = make()
    E, k = conn.shape
    n = k * d
    ke = matrices.ke_small_int(E, n, seed=8)
    rp, ci = orc.pattern(conn, d, nn)
    vals, _ = orc.assemble(conn, d, ke, rp, ci)
    crp, ca = orc.crac(rp, ci, d * nn)
    x = np.random.default_rng(4).integers(-8, 9, size=d * nn).astype(np.float64)
    DI = dof_indices(conn, d)
    ref = np.zeros(d * nn)
    np.add.at(ref, DI.ravel(), np.einsum("ers,es->er", ke, x[DI]).ravel())
    y, _ = orc.spmv_csr(rp, ci, vals, x)
    assert (y == ref).all()
    assert (orc.spmv_crac(crp, ca, vals, x) == ref).all()


def test_laplacian_row_sums_vanish(orc):
    conn, nn = meshes.quad_mesh(12)
    E, k = conn.shape
    ke = matrices.ke_laplacian(E, k, seed=2)
    rp, ci = orc.pattern(conn, 1, nn)
    vals, _ = orc.assemble(conn, 1, ke, rp, ci)
    y, ya = orc.spmv_csr(rp, ci, vals, np.ones(nn))
    assert (np.abs(y) <= 1e-12 * ya).all()
    assert ya.min() > 0


def test_symmetry_of_the_product(orc):
    conn, nn = meshes.hex_mesh(3)
    d = 3
    E, k = conn.shape
    ke = matrices.ke_spd(E, k * d, seed=6)
    rp, ci = orc.pattern(conn, d, nn)
    vals, _ = orc.assemble(conn, d, ke, rp, ci)
    crp, ca = orc.crac(rp, ci, d * nn)
    rng = np.random.default_rng(9)
    x, z = rng.standard_normal(d * nn), rng.standard_normal(d * nn)
    gx = orc.spmv_crac(crp, ca, vals, x)
    gz = orc.spmv_crac(crp, ca, vals, z)
    a, b = z @ gx, x @ gz
    assert abs(a - b) <= 1e-12 * (np.abs(z) @ np.abs(gx) + np.abs(x) @ np.abs(gz))
    assert x @ gx > 0  # SPD element matrices give a positive definite G


def test_empty_rows_give_zero(orc):
    conn, nn = meshes.quad_mesh(3)
    nn_total = nn + 5  # five nodes no element uses
    rp, ci = orc.pattern(conn, 1, nn_total)
    ke = matrices.ke_spd(conn.shape[0], 4, seed=1)
    vals, _ = orc.assemble(conn, 1, ke, rp, ci)
    crp, ca = orc.crac(rp, ci, nn_total)
    x = np.arange(nn_total, dtype=np.float64)
    y, _ = orc.spmv_csr(rp, ci, vals, x)
    assert (y[nn:] == 0).all()
    assert (orc.spmv_crac(crp, ca, vals, x) == y).all()

"""Pins of the oracle's 8-node hexahedron stiffness (the element matrix the
paper replaces by a dummy, Remark 1), against closed forms and invariants
that do not depend on how the oracle evaluates it:

* unit cube, Laplace: diagonal 1/3, edge neighbours 0, face and body
  diagonals -1/12 (the classical trilinear brick matrix);
* K scales with the edge length h in 3D;
* Laplace: constants lie in the kernel; elasticity: the six rigid-body
  modes do, and no other mode (rank 7 and 18);
* for an affine element and a linear field u = A x the energy u^T K u is
  volume times the constant energy density;
* the assembled patch test: on a mesh of distorted elements, a linear
  displacement field leaves every interior node in equilibrium.
"""
import numpy as np
import pytest

from fe_inputs import matrices, meshes

REF = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)
UNIT = (REF + 1) / 2


def test_unit_cube_laplace_closed_form(orc):
    K, _ = orc.hex8_stiffness(UNIT, 1, [1.0])
    expect = np.zeros((8, 8))
    for a in range(8):
        for b in range(8):
            diff = int(np.abs(REF[a] - REF[b]).sum() / 2)  # 0 same, 1 edge, 2 face, 3 body
            expect[a, b] = {0: 4.0, 1: 0.0, 2: -1.0, 3: -1.0}[diff] / 12.0
    assert np.abs(K - expect).max() < 1e-15


@pytest.mark.parametrize("d,mat", [(1, [1.7]), (3, [1.3, 0.6])])
def test_scaling_with_edge_length(orc, d, mat):
    K1, _ = orc.hex8_stiffness(UNIT, d, mat)
    K3, _ = orc.hex8_stiffness(3.0 * UNIT + 0.25, d, mat)
    assert np.abs(K3 - 3.0 * K1).max() <= 1e-13 * np.abs(K1).max()


def _distorted(seed, amount=0.25):
    rng = np.random.default_rng(seed)
    return UNIT + amount * (rng.random((8, 3)) - 0.5)


def _rigid_modes(x):
    modes = []
    for i in range(3):
        t = np.zeros((8, 3))
        t[:, i] = 1.0
        modes.append(t.ravel())
    for axis in range(3):
        w = np.zeros(3)
        w[axis] = 1.0
        modes.append(np.cross(w, x).ravel())
    return np.array(modes)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_kernels_and_rank(orc, seed):
    x = _distorted(seed)
    KL, AL = orc.hex8_stiffness(x, 1, [1.0])
    assert np.abs(KL @ np.ones(8)).max() <= 1e-14 * AL.sum()
    assert np.linalg.matrix_rank(KL, tol=1e-10 * np.abs(KL).max()) == 7
    KE, AE = orc.hex8_stiffness(x, 3, [1.2, 0.7])
    R = _rigid_modes(x)
    assert np.abs(KE @ R.T).max() <= 1e-14 * AE.sum()
    assert np.linalg.matrix_rank(KE, tol=1e-10 * np.abs(KE).max()) == 18
    assert np.abs(KE - KE.T).max() <= 1e-15 * AE.max() * 8
    assert (np.linalg.eigvalsh((KE + KE.T) / 2) > -1e-12 * np.abs(KE).max()).all()


@pytest.mark.parametrize("seed", [3, 4])
def test_linear_field_energy_on_affine_element(orc, seed):
    rng = np.random.default_rng(seed)
    M = np.eye(3) + 0.3 * (rng.random((3, 3)) - 0.5)
    x = UNIT @ M.T + rng.random(3)
    vol = abs(np.linalg.det(M))
    lam, mu, kappa = 1.4, 0.8, 0.9
    c = rng.standard_normal(3)
    KL, _ = orc.hex8_stiffness(x, 1, [kappa])
    u = x @ c
    assert abs(u @ KL @ u - kappa * (c @ c) * vol) <= 1e-13 * kappa * (c @ c) * vol
    A = rng.standard_normal((3, 3))
    KE, _ = orc.hex8_stiffness(x, 3, [lam, mu])
    U = (x @ A.T).ravel()
    eps = (A + A.T) / 2
    energy = vol * (lam * np.trace(eps) ** 2 + 2 * mu * (eps * eps).sum())
    assert abs(U @ KE @ U - energy) <= 1e-12 * energy


@pytest.mark.parametrize("d", [1, 3])
def test_assembled_patch_test(orc, d):
    m = 4
    conn, nn = meshes.hex_mesh(m)
    x = meshes.hex_coords(m, jitter=0.25, seed=7)
    mat = np.ones(conn.shape[0]) if d == 1 else np.tile([1.1, 0.6], (conn.shape[0], 1))
    K, _ = orc.hex8_matrices(conn, x, d, mat)
    rp, ci = orc.pattern(conn, d, nn)
    vals, _ = orc.assemble(conn, d, K, rp, ci)
    rng = np.random.default_rng(1)
    if d == 1:
        u = x @ rng.standard_normal(3) + 0.3
    else:
        u = (x @ rng.standard_normal((3, 3)).T + rng.standard_normal(3)).ravel()
    r, ra = orc.spmv_csr(rp, ci, vals, u)
    idx = np.arange(m + 1)
    inner = [i + (m + 1) * j + (m + 1) ** 2 * k for k in idx[1:-1] for j in idx[1:-1]
             for i in idx[1:-1]]
    dofs = (d * np.array(inner)[:, None] + np.arange(d)[None, :]).ravel()
    assert np.abs(r[dofs]).max() <= 1e-12 * ra[dofs].max()
    boundary = np.setdiff1d(np.arange(d * nn), dofs)
    assert np.abs(r[boundary]).max() > 1e-3 * ra[boundary].max()  # not trivially zero


def test_inverted_element_is_rejected(orc):
    with pytest.raises(ValueError):
        orc.hex8_stiffness(UNIT[[1, 0, 3, 2, 5, 4, 7, 6]], 1, [1.0])


def test_materials_generator_ranges():
    m1 = matrices.hex_materials(1000, 1, seed=2)
    m3 = matrices.hex_materials(1000, 3, seed=2)
    assert m1.shape == (1000,) and (0.5 <= m1).all() and (m1 < 2).all()
    assert m3.shape == (1000, 2) and (m3[:, 1] >= 0.25).all() and (m3[:, 1] < 1).all()

"""Checks of the synthetic input generators themselves."""
import itertools

import numpy as np

from fe_inputs import configs, matrices, meshes


def test_quad_and_hex_shapes():
    conn, nn = meshes.quad_mesh(64)
    assert conn.shape == (4096, 4) and nn == 65 * 65
    assert list(conn[0]) == [0, 1, 66, 65]
    conn, nn = meshes.hex_mesh(3)
    assert conn.shape == (27, 8) and nn == 64
    assert list(conn[0]) == [0, 1, 5, 4, 16, 17, 21, 20]


def _tet_volumes6(m):
    conn, nn = meshes.tet10_mesh(m)
    W = 2 * m + 1
    X = conn % W
    Y = (conn // W) % W
    Z = conn // (W * W)
    P = np.stack([X, Y, Z], axis=-1).astype(np.int64)  # half-step coords
    v = P[:, 1:4] - P[:, [0]]
    return conn, nn, np.linalg.det(v.astype(float)), P


def test_tet10_mesh_is_conforming_and_complete():
    m = 3
    conn, nn, vol, P = _tet_volumes6(m)
    assert conn.shape == (6 * m ** 3, 10) and nn == (2 * m + 1) ** 3
    # every lattice point is a vertex or an edge midpoint of some tet
    assert np.unique(conn).size == nn
    # no degenerate tet; the 6 tets of a cube fill it (volume 6 x 1/6 per cube)
    assert (np.abs(vol) > 0).all()
    assert np.isclose(np.abs(vol).sum() / 8 / 6, m ** 3)
    # edge nodes are midpoints of their edges
    for q, (a, b) in enumerate(meshes.TET10_EDGES):
        assert (2 * P[:, 4 + q] == P[:, a] + P[:, b]).all()
    # conformity: each face is shared by at most two tets; boundary faces
    # number 2 per unit square of the cube surface
    faces = {}
    for t in conn[:, :4]:
        for f in itertools.combinations(sorted(t), 3):
            faces[f] = faces.get(f, 0) + 1
    counts = np.array(list(faces.values()))
    assert counts.max() == 2
    assert (counts == 1).sum() == 12 * m * m


def test_tet10_permutation():
    a, nn = meshes.tet10_mesh(2)
    b, _ = meshes.tet10_mesh(2, perm_seed=0)
    perm = np.random.default_rng(0).permutation(nn)
    assert (perm[a] == b).all()


def test_ke_recipes():
    K = matrices.ke_laplacian(50, 4, seed=0)
    assert (K == K.transpose(0, 2, 1)).all()
    assert np.abs(K.sum(axis=2)).max() < 1e-14
    assert np.abs(K[:, 0, 1:]).max() <= 1.0
    S = matrices.ke_spd(40, 24, seed=0, chunk=7)
    assert (S == S.transpose(0, 2, 1)).all()
    assert np.linalg.eigvalsh(S).min() > 0
    # chunking does not change the stream
    S2 = matrices.ke_spd(40, 24, seed=0, chunk=40)
    assert (S == S2).all()


def test_batch_mix_is_deterministic():
    a = configs.batch_mix()
    b = configs.batch_mix()
    assert [(x.kind, x.size, x.seed) for x in a] == [(x.kind, x.size, x.seed) for x in b]
    assert sum(x.kind == "quad" for x in a) == 256
    assert all(16 <= x.size <= 512 for x in a if x.kind == "quad")
    assert all(8 <= x.size <= 48 for x in a if x.kind == "hex")

"""Seeded synthetic meshes (connectivity only).

These generators produce the element-to-node connectivity that both the
oracle and the device library consume.  They hold none of the assembly
arithmetic: no DOF maps, no sparsity patterns, no sums.

The paper benchmarks Gmsh square meshes (Section 4, mesh figure); those
files are not available, so structured meshes with a stated, lexicographic
node numbering stand in for them, and a permuted tetrahedral mesh stands in
for an unstructured one.

All arrays are ``int32`` of shape ``[n_elements, nodes_per_element]``.
"""
from __future__ import annotations

import itertools

import numpy as np


def quad_mesh(nx: int, ny: int | None = None):
    """Bilinear (Q1) quads on an ``nx`` x ``ny`` structured grid.

    Node ``(i, j)`` has id ``i + (nx+1) * j``.  Elements are lexicographic
    (``i`` fastest).  Local order is counter-clockwise:
    ``(i,j), (i+1,j), (i+1,j+1), (i,j+1)``.
    Returns ``(conn, n_nodes)``.
    """
    ny = nx if ny is None else ny
    W = nx + 1
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    i = i.ravel().astype(np.int64)
    j = j.ravel().astype(np.int64)
    n0 = i + W * j
    conn = np.stack([n0, n0 + 1, n0 + 1 + W, n0 + W], axis=1)
    return conn.astype(np.int32), W * (ny + 1)


def hex_mesh(m: int, my: int | None = None, mz: int | None = None):
    """Trilinear (Q1) hexahedra on an ``m`` x ``my`` x ``mz`` grid.

    Node ``(i, j, k)`` has id ``i + (m+1) j + (m+1)(my+1) k``.  Elements are
    lexicographic (``i`` fastest, then ``j``, then ``k``).  Local order is
    the bottom face ``(i,j,k),(i+1,j,k),(i+1,j+1,k),(i,j+1,k)`` followed by
    the same four corners at ``k+1``.  Returns ``(conn, n_nodes)``.
    """
    my = m if my is None else my
    mz = m if mz is None else mz
    W = m + 1
    A = W * (my + 1)
    k, j, i = np.meshgrid(np.arange(mz), np.arange(my), np.arange(m), indexing="ij")
    n0 = (i + W * j + A * k).ravel().astype(np.int64)
    bottom = [n0, n0 + 1, n0 + 1 + W, n0 + W]
    top = [b + A for b in bottom]
    conn = np.stack(bottom + top, axis=1)
    return conn.astype(np.int32), A * (mz + 1)


def qp_quad_mesh(m: int, p: int):
    """Tensor-product Lagrange quads of degree ``p`` on an ``m`` x ``m`` grid.

    Nodes sit on the ``(p m + 1)^2`` lattice, id ``X + (p m + 1) Y``.  The
    ``(p+1)^2`` local nodes of element ``(i, j)`` are ``X = p i + a``,
    ``Y = p j + b`` in lexicographic local order (``a`` fastest).  This is
    the structured analogue of the paper's p-refinement benchmark meshes
    (Section 4); its node numbering is lexicographic rather than Gmsh's.
    Returns ``(conn, n_nodes)``.
    """
    W = p * m + 1
    j, i = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    i = i.ravel().astype(np.int64)
    j = j.ravel().astype(np.int64)
    b, a = np.meshgrid(np.arange(p + 1), np.arange(p + 1), indexing="ij")
    a = a.ravel()
    b = b.ravel()
    X = p * i[:, None] + a[None, :]
    Y = p * j[:, None] + b[None, :]
    conn = X + W * Y
    return conn.astype(np.int32), W * W


# Edge order of the 10-node tetrahedron after its 4 vertices.
TET10_EDGES = ((0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3))


def tet10_mesh(m: int, perm_seed: int | None = None):
    """Quadratic 10-node tetrahedra from an ``m^3`` cube grid.

    Each cube is split into 6 tetrahedra along its main diagonal (the
    Kuhn/Freudenthal split, which is conforming across cubes): for each
    permutation ``pi`` of the axes, in ``itertools.permutations`` order,
    the vertices are ``v0`` = the cube's low corner,
    ``v1 = v0 + e_pi0``, ``v2 = v1 + e_pi1``, ``v3 = v2 + e_pi2``.
    Nodes live on the half-step lattice ``(2m+1)^3`` (every lattice point is
    a vertex or an edge midpoint), id ``X + (2m+1) Y + (2m+1)^2 Z`` in
    half-step coordinates.  Local order: 4 vertices, then the midpoints of
    edges 01, 12, 02, 03, 13, 23.  Cubes are lexicographic, then the 6 tets.

    With ``perm_seed`` set, node ids are relabelled by
    ``new = numpy.random.default_rng(perm_seed).permutation(n_nodes)[old]``
    to scatter memory access.  Returns ``(conn, n_nodes)``.
    """
    W = 2 * m + 1
    n_nodes = W ** 3
    k, j, i = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    corner = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.int64)  # [C,3]
    eye = np.eye(3, dtype=np.int64)
    tets = []
    for perm in itertools.permutations(range(3)):
        v = [corner]
        for ax in perm:
            v.append(v[-1] + eye[ax])
        verts2 = [2 * x for x in v]  # half-step coordinates
        mids = [(verts2[a] + verts2[b]) // 2 for a, b in TET10_EDGES]
        pts = verts2 + mids  # 10 x [C,3]
        ids = [p[:, 0] + W * p[:, 1] + W * W * p[:, 2] for p in pts]
        tets.append(np.stack(ids, axis=1))  # [C,10]
    conn = np.stack(tets, axis=1).reshape(-1, 10)  # cube-major, 6 tets per cube
    if perm_seed is not None:
        conn = permute_nodes(conn, n_nodes, perm_seed)
    return conn.astype(np.int32), n_nodes


def permute_nodes(conn, n_nodes: int, seed: int):
    """Relabel node ids with ``default_rng(seed).permutation(n_nodes)``."""
    perm = np.random.default_rng(seed).permutation(n_nodes)
    return perm[np.asarray(conn, dtype=np.int64)].astype(np.int32)


def hex_coords(m: int, my: int | None = None, mz: int | None = None, jitter: float = 0.0,
               seed: int = 0, size: float = 1.0):
    """Node coordinates ``[n_nodes, 3]`` for :func:`hex_mesh`'s numbering.

    Node ``(i, j, k)`` sits at ``h (i, j, k)`` with ``h = size / m``, moved by
    ``jitter * h`` times a seeded uniform offset in ``[-1/2, 1/2)^3`` (elements
    stay valid for ``jitter`` below about 0.3)."""
    my = m if my is None else my
    mz = m if mz is None else mz
    h = size / m
    k, j, i = np.meshgrid(np.arange(mz + 1), np.arange(my + 1), np.arange(m + 1), indexing="ij")
    x = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64) * h
    if jitter:
        rng = np.random.default_rng(seed)
        x = x + jitter * h * (rng.random(x.shape) - 0.5)
    return x

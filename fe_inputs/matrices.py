"""Seeded synthetic element matrices ``Ke[E][n][n]`` (FP64, row-major).

The paper deliberately replaces element-matrix computation by a dummy
matrix filled with ones (Section 2.1); that recipe is ``ke_ones``.  The
other recipes give non-trivial values with a known structure:

* ``ke_laplacian``: symmetric, off-diagonals uniform in [-1, 1), diagonal
  equal to minus the off-diagonal row sum (zero row sums).
* ``ke_spd``: ``B B^T / n + I`` with ``B`` standard normal (SPD).

Every recipe mirrors the upper triangle into the lower one, so each
``Ke`` is bit-symmetric.  Draw order is element-major, then row-major over
the upper triangle.  Large batches are produced in chunks; the random
stream does not depend on the chunk size.
"""
from __future__ import annotations

import numpy as np


def _mirror_upper(K):
    """Copy the strict upper triangle of each ``K[e]`` into its lower one."""
    n = K.shape[-1]
    iu = np.triu_indices(n, 1)
    K[:, iu[1], iu[0]] = K[:, iu[0], iu[1]]
    return K


def ke_ones(E: int, n: int):
    """The paper's dummy element: every entry is 1.0."""
    return np.ones((E, n, n), dtype=np.float64)


def ke_laplacian(E: int, n: int, seed: int = 0):
    """Zero-row-sum symmetric element matrices.

    Upper off-diagonals ``U[-1, 1)`` (``default_rng(seed).uniform``), drawn
    element-major and row-major over the strict upper triangle, mirrored;
    ``K_rr = -sum_{s != r} K_rs`` accumulated in increasing ``s`` in FP64.
    """
    rng = np.random.default_rng(seed)
    iu = np.triu_indices(n, 1)
    K = np.zeros((E, n, n), dtype=np.float64)
    K[:, iu[0], iu[1]] = rng.uniform(-1.0, 1.0, size=(E, len(iu[0])))
    _mirror_upper(K)
    for r in range(n):
        acc = np.zeros(E, dtype=np.float64)
        for s in range(n):
            if s != r:
                acc = acc + K[:, r, s]
        K[:, r, r] = -acc
    return K


def ke_spd(E: int, n: int, seed: int = 0, chunk: int = 32768, out=None):
    """SPD element matrices ``B B^T / n + I`` with ``B ~ N(0,1)`` of size n x n.

    ``B`` is drawn with ``default_rng(seed).standard_normal`` element by
    element; the product's upper triangle is mirrored so every matrix is
    bit-symmetric.  ``out`` may be a preallocated ``[E, n, n]`` float64 array.
    """
    rng = np.random.default_rng(seed)
    K = np.empty((E, n, n), dtype=np.float64) if out is None else out
    eye = np.eye(n)
    for e0 in range(0, E, chunk):
        e1 = min(E, e0 + chunk)
        B = rng.standard_normal((e1 - e0, n, n))
        Kc = np.matmul(B, B.transpose(0, 2, 1)) / n + eye
        K[e0:e1] = _mirror_upper(Kc)
    return K


def ke_small_int(E: int, n: int, seed: int = 0, lo: int = -8, hi: int = 8):
    """Symmetric matrices of small integers in ``[lo, hi]``.

    Sums of such entries are exact in FP64 in any order, so any correct
    assembly reproduces them bit for bit.
    """
    rng = np.random.default_rng(seed)
    K = rng.integers(lo, hi, size=(E, n, n), endpoint=True).astype(np.float64)
    return _mirror_upper(K)


def hex_materials(E: int, d: int, seed: int = 0):
    """Per-element material parameters: ``[E]`` conductivities in [0.5, 2)
    for d = 1, ``[E, 2]`` Lame parameters (lambda in [0.5, 2), mu in
    [0.25, 1)) for d = 3."""
    rng = np.random.default_rng(seed)
    if d == 1:
        return 0.5 + 1.5 * rng.random(E)
    lam = 0.5 + 1.5 * rng.random(E)
    mu = 0.25 + 0.75 * rng.random(E)
    return np.stack([lam, mu], axis=1)

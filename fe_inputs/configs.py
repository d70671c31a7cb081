"""The five synthetic workloads, with their recipes.

* ``quad64``   64 x 64 Q1 quads, 1 DOF/node, 4 x 4 zero-row-sum ``Ke``, seed 0.
* ``hex64``    64^3 Q1 hexes, 3 DOFs/node, 24 x 24 SPD ``Ke``, seed 0.
* ``tet40``    40^3 cubes x 6 tet10, node ids permuted (seed 0), 3 DOFs/node,
  30 x 30 SPD ``Ke``, seed 0.
* ``batch512`` 256 quad meshes n x n (n uniform in [16, 512]) and 256 hex
  meshes m^3 (m uniform in [8, 48]), drawn from ``default_rng(0)`` and
  shuffled by it; per-mesh ``Ke`` seeds from ``SeedSequence(0).spawn(512)``.
* ``serve``    Poisson arrivals (mean gap 0.5 ms) drawn from ``default_rng(0)``,
  sizes from the batch mix, 10 value-only re-assemblies per request.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import matrices, meshes


@dataclass
class Workload:
    name: str
    conn: np.ndarray  # int32 [E, k]
    n_nodes: int
    dofs_per_node: int
    ke_recipe: str  # "laplacian" | "spd" | "ones"
    seed: int = 0

    @property
    def n_elem(self):
        return int(self.conn.shape[0])

    @property
    def nodes_per_elem(self):
        return int(self.conn.shape[1])

    @property
    def n(self):
        return self.nodes_per_elem * self.dofs_per_node

    def ke(self, out=None):
        if self.ke_recipe == "laplacian":
            return matrices.ke_laplacian(self.n_elem, self.n, self.seed)
        if self.ke_recipe == "spd":
            return matrices.ke_spd(self.n_elem, self.n, self.seed, out=out)
        if self.ke_recipe == "ones":
            return matrices.ke_ones(self.n_elem, self.n)
        raise ValueError(self.ke_recipe)


def quad64(m: int = 64):
    conn, nn = meshes.quad_mesh(m)
    return Workload(f"quad{m}", conn, nn, 1, "laplacian", 0)


def hex64(m: int = 64):
    conn, nn = meshes.hex_mesh(m)
    return Workload(f"hex{m}", conn, nn, 3, "spd", 0)


def tet40(m: int = 40, perm_seed: int = 0):
    conn, nn = meshes.tet10_mesh(m, perm_seed=perm_seed)
    return Workload(f"tet10_{m}", conn, nn, 3, "spd", 0)


@dataclass
class MeshSpec:
    kind: str  # "quad" | "hex"
    size: int  # n for quads (n x n), m for hexes (m^3)
    seed: int  # Ke seed

    @property
    def n_elem(self):
        return self.size ** 2 if self.kind == "quad" else self.size ** 3

    @property
    def nodes_per_elem(self):
        return 4 if self.kind == "quad" else 8

    @property
    def dofs_per_node(self):
        return 1 if self.kind == "quad" else 3

    @property
    def n(self):
        return self.nodes_per_elem * self.dofs_per_node

    def workload(self):
        if self.kind == "quad":
            conn, nn = meshes.quad_mesh(self.size)
            return Workload(f"quad{self.size}", conn, nn, 1, "laplacian", self.seed)
        conn, nn = meshes.hex_mesh(self.size)
        return Workload(f"hex{self.size}", conn, nn, 3, "spd", self.seed)


def batch_mix(count: int = 512, seed: int = 0):
    """The batch size mix: half quads n in [16,512], half hexes m in [8,48].

    Sizes are drawn from ``default_rng(seed)`` (quads first, then hexes) and
    the combined list is shuffled by the same generator.  Each mesh gets the
    ``Ke`` seed ``SeedSequence(seed).spawn(count)[i]`` (as a 32-bit integer
    drawn from that child sequence).
    """
    rng = np.random.default_rng(seed)
    half = count // 2
    q = rng.integers(16, 512, size=half, endpoint=True)
    h = rng.integers(8, 48, size=count - half, endpoint=True)
    specs = [("quad", int(x)) for x in q] + [("hex", int(x)) for x in h]
    order = rng.permutation(len(specs))
    children = np.random.SeedSequence(seed).spawn(count)
    out = []
    for i, idx in enumerate(order):
        kind, size = specs[idx]
        out.append(MeshSpec(kind, size, int(children[i].generate_state(1)[0])))
    return out


def arrival_times(n_requests: int, mean_gap_s: float = 0.5e-3, seed: int = 0):
    """Poisson arrival times (exponential gaps) in seconds from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(mean_gap_s, size=n_requests))

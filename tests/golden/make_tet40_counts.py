"""Writes tet40_counts.json: pattern sizes of the 40^3 x 6 tet10 mesh (node
ids permuted with seed 0, 3 DOFs per node), computed by the serial oracle.

Run from the repository root: python tests/golden/make_tet40_counts.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from fe_inputs import meshes  # noqa: E402
from oracle import oracle  # noqa: E402


def main():
    t0 = time.time()
    conn, nn = meshes.tet10_mesh(40, perm_seed=0)
    d = 3
    rp, ci = oracle.pattern(conn, d, nn)
    crp, ca = oracle.crac(rp, ci, d * nn)
    col, nc = oracle.greedy_colour(conn, nn)
    lens = np.diff(rp)
    out = {
        "what": "tet10 mesh, 40^3 cubes x 6 (Kuhn split), node ids permuted by "
                "default_rng(0).permutation, 3 DOFs per node; sizes from the serial oracle",
        "n_elem": int(conn.shape[0]),
        "n_nodes": int(nn),
        "n_rows": int(d * nn),
        "nnz": int(rp[-1]),
        "n_ca": int(ca.size),
        "runs": int((ca.size - 2) // 2),
        "row_len_min": int(lens.min()),
        "row_len_max": int(lens.max()),
        "greedy_colours": int(nc),
        "row_ptr_sha_int64": __import__("hashlib").sha256(rp.astype(np.int64).tobytes()).hexdigest(),
        "col_idx_sha_int64": __import__("hashlib").sha256(ci.astype(np.int64).tobytes()).hexdigest(),
        "crac_row_ptr_sha_int64": __import__("hashlib").sha256(
            crp.astype(np.int64).tobytes()).hexdigest(),
        "ca_sha_int64": __import__("hashlib").sha256(ca.astype(np.int64).tobytes()).hexdigest(),
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tet40_counts.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1), f"{time.time() - t0:.1f}s")


if __name__ == "__main__":
    main()

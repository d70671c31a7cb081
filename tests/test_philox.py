"""The counter-based element-matrix generator's host implementation."""
import json
import os

import numpy as np

from fe_inputs import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    kat = json.load(open(os.path.join(GOLDEN, "philox_kat.json")))
    for v in kat["vectors"]:
        c = [np.array([int(x, 16)], dtype=np.uint32) for x in v["ctr"]]
        k = [int(x, 16) for x in v["key"]]
        out = philox.philox4x32_10(*c, *k)
        assert [format(int(o[0]), "08x") for o in out] == v["out"]


def test_recipes():
    L = philox.ke_laplacian(20, 4, seed=3)
    assert (L == L.transpose(0, 2, 1)).all()
    assert np.abs(L.sum(axis=2)).max() < 1e-14
    assert np.abs(L[:, 0, 1:]).max() <= 1.0
    S = philox.ke_spd(20, 24, seed=2 ** 40 + 5, e0=7)
    assert (S == S.transpose(0, 2, 1)).all()
    assert np.linalg.eigvalsh(S).min() > 0.9  # B B^T / n + I >= I
    # element offsets address the same stream
    a = philox.ke_spd(10, 6, seed=9, e0=0)
    b = philox.ke_spd(4, 6, seed=9, e0=3)
    assert (a[3:7] == b).all()

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle

    oracle.build()
    return oracle


class _Tet40Reference:
    """The permuted tet10 workload (40^3 cubes x 6, 3 DOFs per node, SPD
    30x30 element matrices, seed 0) with the serial oracle's full pattern,
    CRAC arrays, values and per-entry bounds; built once per session (about
    40 s of oracle work and 7 GB of host memory)."""

    def __init__(self, orc):
        from fe_inputs import configs

        self.w = configs.tet40()
        self.ke = self.w.ke()
        d, nn = self.w.dofs_per_node, self.w.n_nodes
        self.rp, self.ci = orc.pattern(self.w.conn, d, nn)
        self.crp, self.ca = orc.crac(self.rp, self.ci, d * nn)
        self.ov, self.oa = orc.assemble(self.w.conn, d, self.ke, self.rp, self.ci)


@pytest.fixture(scope="session")
def tet40_ref(orc):
    return _Tet40Reference(orc)

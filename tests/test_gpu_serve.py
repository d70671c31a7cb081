"""The serving loop: results alone vs in the mix, oracle parity, admission (GPU)."""
import sys

import numpy as np
import pytest
import torch

from fe_inputs import meshes, philox
from tests._checks import assert_values_close

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def feasm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_00585_amd as f

    f.load()
    return f


MESHES = {
    "quad24": (lambda: meshes.quad_mesh(24), 1, 0),
    "quad60": (lambda: meshes.quad_mesh(60), 1, 0),
    "hex6": (lambda: meshes.hex_mesh(6), 3, 1),
    "hex11": (lambda: meshes.hex_mesh(11), 3, 1),
    "tet3": (lambda: meshes.tet10_mesh(3, perm_seed=2), 3, 1),
}


@pytest.fixture(scope="module")
def registry(feasm):
    dev = torch.device("cuda:0")
    out = {}
    for key, (make, d, recipe) in MESHES.items():
        conn, nn = make()
        p = feasm.pattern_build(torch.from_numpy(conn).to(dev), d, nn,
                                feasm.BUILD_CSR | feasm.BUILD_CRAC | feasm.BUILD_COLOUR)
        out[key] = (p, recipe, conn, nn, d)
    yield out
    for p, *_ in out.values():
        p.free()


def _server(registry, **kw):
    from paper_2012_00585_amd.serve import Server

    srv = Server(**kw)
    for key, (p, recipe, *_rest) in registry.items():
        srv.register(key, p, recipe)
    return srv


def _requests(n, seed=0, gap=2e-4, n_re=3):
    from paper_2012_00585_amd.serve import Request

    rng = np.random.default_rng(seed)
    keys = list(MESHES)
    t = np.cumsum(rng.exponential(gap, size=n))
    return [Request(i, float(t[i]), keys[rng.integers(len(keys))], int(rng.integers(1 << 40)), n_re)
            for i in range(n)]


@pytest.mark.parametrize("fmt", [0, 1])
def test_alone_equals_in_mix_and_oracle(feasm, orc, registry, fmt):
    from paper_2012_00585_amd.serve import iteration_seed

    reqs = _requests(40, seed=fmt)
    watch = [r.rid for r in reqs[::7]]
    mix = _server(registry, fmt=fmt, slots=6, keep=watch)
    stats = mix.run(reqs)
    say(f"[serve] mix: {stats}")
    assert stats["requests"] == len(reqs)
    for r in reqs:
        if r.rid not in watch:
            continue
        alone = _server(registry, fmt=fmt, slots=1, keep=[r.rid])
        alone.run([type(r)(r.rid, 0.0, r.mesh, r.seed, r.n_reassembly)])
        a, b = alone.kept[r.rid], mix.kept[r.rid]
        assert (a == b).all(), r  # row-owned AUTO: deterministic, bit-identical
        # the last iteration's element matrices, regenerated on the host
        p, recipe, conn, nn, d = registry[r.mesh]
        gen = philox.ke_laplacian if recipe == 0 else philox.ke_spd
        ke = gen(p.n_elem, p.n, iteration_seed(r.seed, r.n_reassembly))
        rp, ci = orc.pattern(conn, d, nn)
        ov, oa = orc.assemble(conn, d, ke, rp, ci)
        assert (b == ov).all(), r


def test_mixed_strategies_in_mix_within_tolerance(feasm, orc, registry):
    # atomic handles: order of additions varies, results within tolerance
    for key, (p, *_r) in registry.items():
        p.tune(feasm.TUNE_STRATEGY, feasm.SCATTER_ATOMIC)
    try:
        reqs = _requests(24, seed=5)
        watch = [r.rid for r in reqs[::5]]
        mix = _server(registry, fmt=1, slots=8, keep=watch)
        mix.run(reqs)
        from paper_2012_00585_amd.serve import iteration_seed

        for r in reqs:
            if r.rid not in watch:
                continue
            p, recipe, conn, nn, d = registry[r.mesh]
            gen = philox.ke_laplacian if recipe == 0 else philox.ke_spd
            ke = gen(p.n_elem, p.n, iteration_seed(r.seed, r.n_reassembly))
            rp, ci = orc.pattern(conn, d, nn)
            ov, oa = orc.assemble(conn, d, ke, rp, ci)
            assert_values_close(mix.kept[r.rid], ov, oa, what=f"request {r.rid}")
    finally:
        for key, (p, *_r) in registry.items():
            p.tune(feasm.TUNE_STRATEGY, 0)


def test_small_budget_queues_requests(feasm, registry):
    reqs = _requests(12, seed=3, gap=1e-5, n_re=2)
    srv = _server(registry, fmt=1, slots=8)
    biggest = max(srv.footprint(r) for r in reqs)
    srv.budget = biggest  # at most about one request in flight
    stats = srv.run(reqs)
    assert stats["requests"] == len(reqs)
    assert stats["max_pending"] >= 2
    assert stats["queue_wait_ms"]["p99"] > 0


def _conn_tensor(conn):
    return torch.from_numpy(np.ascontiguousarray(conn, dtype=np.int32)).to(torch.device("cuda:0"))


def test_pattern_cache_builds_on_miss_and_evicts(feasm, orc, registry):
    """Meshes known by connectivity only: the engine builds each pattern on
    the first request for it and keeps at most about one pattern's bytes, so
    later requests evict and rebuild; every kept result equals the oracle
    (row-owned: bit for bit)."""
    from paper_2012_00585_amd.serve import Server, iteration_seed

    reqs = _requests(30, seed=11, n_re=2)
    watch = [r.rid for r in reqs[::3]]
    srv = Server(fmt=1, slots=4, keep=watch, pattern_cache_bytes=1)
    for key, (make, d, recipe) in MESHES.items():
        conn, nn = make()
        srv.register_mesh(key, _conn_tensor(conn), d, nn, recipe)
    stats = srv.run(reqs)
    eng = stats["engine"]
    say(f"[serve] cache: {eng}")
    assert stats["requests"] == len(reqs)
    used = {r.mesh for r in reqs}
    assert eng["pattern_misses"] >= len(used)
    assert eng["pattern_evictions"] >= 1
    assert eng["pattern_misses"] + eng["pattern_hits"] == len(reqs)
    for r in reqs:
        if r.rid not in watch:
            continue
        make, d, recipe = MESHES[r.mesh]
        conn, nn = make()
        E, k = conn.shape
        gen = philox.ke_laplacian if recipe == 0 else philox.ke_spd
        ke = gen(E, k * d, iteration_seed(r.seed, r.n_reassembly))
        rp, ci = orc.pattern(conn, d, nn)
        ov, _ = orc.assemble(conn, d, ke, rp, ci)
        got = srv.kept[r.rid][:ov.size]  # an engine-built pattern's values come first
        assert (got == ov).all(), r


def test_unbounded_cache_builds_each_mesh_once(feasm, registry):
    from paper_2012_00585_amd.serve import Server

    reqs = _requests(25, seed=12, n_re=1)
    srv = Server(fmt=0, slots=4)
    for key, (make, d, recipe) in MESHES.items():
        conn, nn = make()
        srv.register_mesh(key, _conn_tensor(conn), d, nn, recipe)
    eng = srv.run(reqs)["engine"]
    assert eng["pattern_misses"] == len({r.mesh for r in reqs})
    assert eng["pattern_evictions"] == 0
    assert eng["patterns_resident_at_end"] == eng["pattern_misses"]


def test_element_matrix_pools(feasm, orc, registry):
    """Requests read pre-generated element matrices from per-mesh pools (no
    generator in the loop): iteration i of a request with key s reads block
    (s + i) mod pool size."""
    from paper_2012_00585_amd.serve import Server, pool_block

    dev = torch.device("cuda:0")
    pool_n = 3
    srv = Server(fmt=1, slots=5)
    pools = {}
    for key, (p, recipe, conn, nn, d) in registry.items():
        blocks = [feasm.generate_ke(recipe, p.n_elem, p.n, 900 + b) for b in range(pool_n)]
        pools[key] = torch.stack(blocks).contiguous()
        srv.register(key, p, recipe, ke_pool=pools[key])
    reqs = _requests(20, seed=13, n_re=4)
    srv.keep = {r.rid for r in reqs[::4]}
    stats = srv.run(reqs)
    eng = stats["engine"]
    assert eng["generated_bytes"] == 0 and eng["generate_ms"] == 0.0
    assert eng["assemble_ms"] > 0
    for r in reqs:
        if r.rid not in srv.keep:
            continue
        p, recipe, conn, nn, d = registry[r.mesh]
        ke = pools[r.mesh][pool_block(r.seed, r.n_reassembly, pool_n)].cpu().numpy()
        rp, ci = orc.pattern(conn, d, nn)
        ov, _ = orc.assemble(conn, d, ke, rp, ci)
        assert (srv.kept[r.rid] == ov).all(), r


def test_batch_mix_stream_at_2000_per_s(feasm, orc):
    """A short stream shaped like the serving workload: Poisson arrivals at
    2000 requests/s over the 512-mesh size mix, 10 re-assemblies each, the
    patterns built by the engine on demand; requests of both kinds and of
    small and large sizes kept and compared with the oracle bit for bit."""
    from fe_inputs import configs
    from paper_2012_00585_amd.serve import Request, Server, iteration_seed

    specs = configs.batch_mix()
    n = 40
    t = configs.arrival_times(n, 0.5e-3, seed=0)
    rng = np.random.default_rng(1)
    pick = rng.integers(len(specs), size=n)
    reqs = [Request(i, float(t[i]), int(pick[i]), int(rng.integers(1 << 40)), 10) for i in range(n)]
    by_kind = {}
    for r in reqs:
        by_kind.setdefault(specs[r.mesh].kind, []).append(r)
    watch = []
    for kind, rs in by_kind.items():
        rs = sorted(rs, key=lambda r: specs[r.mesh].n_elem)
        watch += [rs[0].rid, rs[len(rs) // 2].rid, rs[-1].rid]
    srv = Server(fmt=1, slots=16, keep=watch, hbm_budget=96 << 30)
    conns = {}
    for i in sorted({r.mesh for r in reqs}):
        sp = specs[i]
        conn, nn = meshes.quad_mesh(sp.size) if sp.kind == "quad" else meshes.hex_mesh(sp.size)
        conns[i] = (conn, nn)
        srv.register_mesh(i, _conn_tensor(conn), sp.dofs_per_node, nn,
                          feasm.RECIPE_LAPLACIAN if sp.kind == "quad" else feasm.RECIPE_SPD)
    say(f"[serve] batch-mix stream: {n} requests over {len(conns)} meshes")
    stats = srv.run(reqs)
    say(f"[serve] batch-mix stream: {stats}")
    assert stats["requests"] == n
    for r in reqs:
        if r.rid not in watch:
            continue
        sp = specs[r.mesh]
        conn, nn = conns[r.mesh]
        E, k = conn.shape
        d = sp.dofs_per_node
        gen = philox.ke_laplacian if sp.kind == "quad" else philox.ke_spd
        ke = gen(E, k * d, iteration_seed(r.seed, r.n_reassembly))
        rp, ci = orc.pattern(conn, d, nn)
        ov, _ = orc.assemble(conn, d, ke, rp, ci, with_abs=False)
        say(f"[serve]   request {r.rid}: {sp.kind} {sp.size}, {E} elements")
        assert (srv.kept[r.rid][:ov.size] == ov).all(), (r, sp)

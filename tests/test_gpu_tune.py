"""Autotuners and the node-kernel path (needs an MI355X).

The tuners must return a candidate of their documented sets, record it in
the cache file and return it again from there, and a batch built with the
tuned shape must still give each mesh's single-solve result bit for bit.
A mesh with a node of more elements than a tile record can name runs on the
node kernel and must match the oracle like every other mesh.
"""

import numpy as np
import pytest

import oracle
import paper_2301_08357_amd as pm
from synth import fields, mesh as smesh, workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_batch_tuner_and_cache(tmp_path):
    probs = [workloads.cube(6, w=1e-2, jitter=0.2, rho="uniform"), workloads.tgv2d(12),
             workloads.cube(9, w=1.0, jitter=0.2, rho="lognormal")]
    print("case tune_batch", [p.mesh.n_nodes for p in probs], flush=True)
    systems = [pm.PressureSystem.from_problem(p) for p in probs]
    cache = tmp_path / "tune.txt"
    tps, npl, ms = pm.tune_batch(systems, iters=32, cache=cache)
    assert tps in (1, 2, 4, 8) and npl in (2, 4, 8, 16) and ms > 0
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and len(lines[0].split()) == 4
    # a cache hit returns the recorded choice and adds no line
    assert pm.tune_batch(systems, iters=32, cache=cache)[:2] == (tps, npl)
    assert len(cache.read_text().splitlines()) == 1
    # the tuned batch reproduces single solves bit for bit
    As = [oracle.assemble_problem(p) for p in probs]
    bs = [_dev(A.matvec(fields.sine_product(p.mesh.coords))) for p, A in zip(probs, As)]
    batch = pm.PressureBatch(systems, tps, npl)
    code, res = batch.solve(bs, rtol=1e-10)
    assert code == 0
    for s, b, r, A, p in zip(systems, bs, res, As, probs):
        x = _host(r.p).copy()
        single = s.solve(b, rtol=1e-10)
        assert single.iters == r.iters
        assert np.array_equal(_host(single.p).view(np.uint64), x.view(np.uint64))
        bh = _host(b)
        assert np.linalg.norm(bh - A.matvec(x)) / np.linalg.norm(bh) <= 1.05e-10
    batch.close()
    for s in systems:
        s.close()


def test_tile_tuner_and_cache(tmp_path):
    prob = workloads.cube(12, w=1e-3, jitter=0.2, rho="uniform")
    print("case tune_tile", prob.mesh.n_nodes, flush=True)
    cache = tmp_path / "tune.txt"
    flags, ms = pm.tune_tile(prob, flags=pm.PM_FP64, iters=16, cache=cache)
    assert flags & ~0xF0 == pm.PM_FP64
    assert flags & 0xF0 in (pm.PM_TILE_128, pm.PM_TILE_256, pm.PM_TILE_512) and ms > 0
    assert pm.tune_tile(prob, flags=pm.PM_FP64, iters=16, cache=cache)[0] == flags
    assert len(cache.read_text().splitlines()) == 1
    # another precision is another key
    flags32, _ = pm.tune_tile(prob, flags=pm.PM_FP64 | pm.PM_FP32_INNER, iters=16, cache=cache)
    assert flags32 & ~0xF0 == pm.PM_FP64 | pm.PM_FP32_INNER
    assert len(cache.read_text().splitlines()) == 2
    s = pm.PressureSystem.from_problem(prob, flags=flags)
    A = oracle.assemble_problem(prob)
    x = np.random.default_rng(3).normal(size=prob.mesh.n_nodes)
    y = _host(s.apply(_dev(x)))
    S = A.to_scipy()
    assert np.all(np.abs(y - A.matvec(x)) <= 1e-12 * (abs(S) @ np.abs(x)))
    s.close()


def test_high_degree_mesh_runs_on_node_kernel():
    m = smesh.fan_mesh(80)
    prob = workloads.Problem("fan80", m, 1.0 / fields.rho_uniform(5, m.n_elems), 1e-3, 1.0, 1e-10, 5)
    print("case fan80", m.n_nodes, m.n_elems, flush=True)
    A = oracle.assemble_problem(prob)
    s = pm.PressureSystem.from_problem(prob)
    assert s.info()["n_instances"] == 0
    with pytest.raises(pm.PressureError):
        s.set_variant(pm.PM_VARIANT_TILED)
    s.set_variant(pm.PM_VARIANT_AUTO)
    x = np.random.default_rng(1).normal(size=m.n_nodes)
    y = _host(s.apply(_dev(x)))
    S = A.to_scipy()
    assert np.all(np.abs(y - A.matvec(x)) <= 1e-12 * (abs(S) @ np.abs(x)))
    b = A.matvec(fields.sine_product(m.coords / 2.0))
    res = s.solve(_dev(b), rtol=1e-10)
    assert res.status == 0
    xs = _host(res.p)
    assert np.linalg.norm(b - A.matvec(xs)) / np.linalg.norm(b) <= 1.05e-10
    x_ref = oracle.cg(A, b, rtol=1e-10, max_iter=20000, dirichlet=m.dirichlet)[0]
    assert np.linalg.norm(xs - x_ref) / np.linalg.norm(x_ref) <= 1e-9
    s.close()
    # explicit tile sizes and the FP32 inner solve need the tiled kernel
    for flags in (pm.PM_FP64 | pm.PM_TILE_128, pm.PM_FP64 | pm.PM_FP32_INNER):
        with pytest.raises(pm.PressureError):
            pm.PressureSystem.from_problem(prob, flags=flags)

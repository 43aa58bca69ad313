"""Batched solves of many meshes (needs an MI355X).

Every mesh of a batch must give exactly (bit for bit) what a single-mesh
solve on the same handle gives, whether the iterations run from a replayed
HIP graph or from direct launches, and the oracle's operator must accept
each result at the requested tolerance.
"""

import numpy as np
import pytest

import oracle
import paper_2301_08357_amd as pm
from synth import fields, workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _small_mix():
    """Meshes of the batched workload's distribution (2D and 3D, w spread
    over [1e-6, 1]), limited to sizes the oracle assembles in a second."""
    params = workloads.batch_params()
    picked = [i for i, (d, n, w) in enumerate(params) if (n + 1) ** d <= 12000][:6]
    probs = [workloads.batch_problem(i, params) for i in picked]
    probs.append(workloads.cube(5, w=1.0, jitter=0.2, rho="uniform"))
    probs.append(workloads.tgv2d(9))
    return probs


def _rhs(prob, A):
    if "source" in prob.extra:
        return oracle.mass_rhs(prob, prob.extra["source"])
    return A.matvec(fields.sine_product(prob.mesh.coords))


def test_batch_matches_single_and_oracle():
    probs = _small_mix()
    print("case meshes", [(p.mesh.dim, p.mesh.n_nodes) for p in probs], flush=True)
    As = [oracle.assemble_problem(p) for p in probs]
    bs = [_rhs(p, A) for p, A in zip(probs, As)]
    systems = [pm.PressureSystem.from_problem(p) for p in probs]
    batch = pm.PressureBatch(systems, tiles_per_slot=2, nodes_per_lane=4)
    rhs = [_dev(b) for b in bs]
    code, res = batch.solve(rhs, rtol=1e-10)
    assert code == 0
    xb = [_host(r.p).copy() for r in res]
    for p, A, b, r, x in zip(probs, As, bs, res, xb):
        assert r.status == 0
        accept = np.linalg.norm(b - A.matvec(x)) / np.linalg.norm(b)
        assert accept <= 1.05e-10, (p.name, accept)
    # eager single solves in between, then bitwise equality with them
    for s, b, r, x in zip(systems, rhs, res, xb):
        single = s.solve(b, rtol=1e-10)
        assert single.iters == r.iters
        assert np.array_equal(_host(single.p).view(np.uint64), x.view(np.uint64))
    # a second replay of the same graphs gives the same bits
    code2, res2 = batch.solve(rhs, rtol=1e-10)
    assert code2 == 0
    for r, x in zip(res2, xb):
        assert np.array_equal(_host(r.p).view(np.uint64), x.view(np.uint64))
    # direct launches (no graph) and another chunk length: same bits
    for g in (0, 6):
        batch.set_graph(g)
        code3, res3 = batch.solve(rhs, rtol=1e-10)
        assert code3 == 0
        for r, x in zip(res3, xb):
            assert np.array_equal(_host(r.p).view(np.uint64), x.view(np.uint64))
    batch.close()
    for s in systems:
        s.close()


def test_batch_edge_cases():
    probs = [workloads.cube(4, w=1e-2, jitter=0.2, rho="uniform"), workloads.tgv2d(6)]
    systems = [pm.PressureSystem.from_problem(p) for p in probs]
    batch = pm.PressureBatch(systems)
    As = [oracle.assemble_problem(p) for p in probs]
    b0 = _dev(_rhs(probs[0], As[0]))
    zero = _dev(np.zeros(probs[1].mesh.n_nodes))
    code, res = batch.solve([b0, zero], rtol=1e-10)
    assert code == 0 and res[1].iters == 0 and np.all(_host(res[1].p) == 0)
    iters_ref, p_ref = res[0].iters, _host(res[0].p).copy()
    code, res = batch.solve([b0, _dev(_rhs(probs[1], As[1]))], rtol=1e-12, max_iter=3)
    assert code == pm.PM_NOT_CONVERGED
    assert all(r.status == pm.PM_NOT_CONVERGED and r.iters == 3 for r in res)
    # warm start from the solution: no iterations
    code, res = batch.solve([b0, zero], rtol=1e-11)
    code, res2 = batch.solve([b0, zero], x0=[res[0].p.clone(), None], rtol=1e-10)
    assert code == 0 and res2[0].iters == 0
    with pytest.raises(pm.PressureError):
        batch.set_graph(3)
    # a step split in two: nothing else may run on the batch in between
    batch.begin(0, b0, rtol=1e-10)
    batch.step_launch()
    with pytest.raises(pm.PressureError):
        batch.begin(1, zero, rtol=1e-10)
    with pytest.raises(pm.PressureError):
        batch.step_launch()
    done = batch.step_wait()
    with pytest.raises(pm.PressureError):
        batch.step_wait()
    for _ in range(1000):
        if done[0]:
            break
        batch.step_launch()
        # the non-blocking form ends the step as step_wait does
        done = None
        for _ in range(10 ** 6):
            done = batch.step_poll()
            if done is not None:
                break
        assert done is not None
    res3 = batch.finish(0, b0, rtol=1e-10)
    assert res3.status == 0 and res3.iters == iters_ref
    assert np.array_equal(_host(res3.p).view(np.uint64), p_ref.view(np.uint64))
    batch.close()
    for s in systems:
        s.close()


def test_mixed_batch_matches_single_mixed():
    """Batched mixed-precision solves (FP32 inner CG of every mesh in the
    batched launches, FP64 corrections per mesh) give each mesh's
    pressure_solve_mixed result bit for bit, in both inner modes, and solves
    may start at different steps."""
    probs = _small_mix()[:5]
    print("case mixed batch", [(p.mesh.dim, p.mesh.n_nodes) for p in probs], flush=True)
    As = [oracle.assemble_problem(p) for p in probs]
    bs = [_rhs(p, A) for p, A in zip(probs, As)]
    systems = [pm.PressureSystem.from_problem(p, flags=pm.PM_FP64 | pm.PM_FP32_INNER) for p in probs]
    systems[1].set_mixed_mode(pm.PM_MIXED_RESTART)
    batch = pm.PressureBatch(systems, tiles_per_slot=2, nodes_per_lane=4, mixed=True, inner_rtol=1e-2)
    rhs = [_dev(b) for b in bs]
    code, res = batch.solve(rhs, rtol=1e-10)
    assert code == 0
    xb = [_host(r.p).copy() for r in res]
    for p, A, b, r, x in zip(probs, As, bs, res, xb):
        assert r.status == 0 and r.true_relres <= 1e-10
        accept = np.linalg.norm(b - A.matvec(x)) / np.linalg.norm(b)
        assert accept <= 1.05e-10, (p.name, accept)
    for s, b, r, x in zip(systems, rhs, res, xb):
        single = s.solve_mixed(b, rtol=1e-10, inner_rtol=1e-2)
        assert single.iters == r.iters
        assert np.array_equal(_host(single.p).view(np.uint64), x.view(np.uint64))
    # continuous batching: mesh 2 joins two steps after mesh 0
    outs = {}
    batch.begin(0, rhs[0], rtol=1e-10)
    started, steps = {0}, 0
    while True:
        done = batch.step()
        steps += 1
        for m in sorted(started):
            if done[m] and m not in outs:
                outs[m] = batch.finish(m, rhs[m], rtol=1e-10)
        if steps == 2:
            batch.begin(2, rhs[2], rtol=1e-10)
            started.add(2)
        if len(outs) == 2:
            break
        assert steps < 10000
    for m in (0, 2):
        assert outs[m].iters == res[m].iters
        assert np.array_equal(_host(outs[m].p).view(np.uint64), xb[m].view(np.uint64))
    batch.close()
    for s in systems:
        s.close()


def _real_mix_sample(k=16):
    """k meshes of the 256-mesh batched workload itself (its largest 2D and
    3D meshes, its smallest one, its extreme mass weights, the rest spread
    over the list)."""
    params = workloads.batch_params()
    return [workloads.batch_problem(i, params) for i in workloads.batch_sample(k, params)]


@pytest.mark.parametrize("mixed", [False, True])
def test_batch_real_mix_at_tuned_shape(mixed):
    """16 meshes of the real 256-mesh mix (up to 2e5 nodes, both its
    largest 2D and 3D meshes) in the launch shape the autotuner picks for
    that mix on the MI355X (8 Morton tiles per apply slot, 4 nodes per lane
    of an update slot): every result accepted by the oracle's operator at
    1.05 x rtol, and equal to the single solve on the same grids."""
    probs = _real_mix_sample()
    assert max(p.mesh.n_nodes for p in probs if p.mesh.dim == 2) > 1.5e5
    assert max(p.mesh.n_nodes for p in probs if p.mesh.dim == 3) > 1.5e5
    print("case real mix mixed=%s" % mixed, [(p.mesh.dim, p.mesh.n_nodes) for p in probs], flush=True)
    As = [oracle.assemble_problem(p) for p in probs]
    bs = [A.matvec(p.extra["xstar"]) for p, A in zip(probs, As)]
    flags = pm.PM_FP64 | (pm.PM_FP32_INNER if mixed else 0)
    systems = [pm.PressureSystem.from_problem(p, flags=flags) for p in probs]
    batch = pm.PressureBatch(systems, tiles_per_slot=8, nodes_per_lane=4, mixed=mixed, inner_rtol=1e-2)
    rhs = [_dev(b) for b in bs]
    code, res = batch.solve(rhs, rtol=1e-10)
    assert code == 0
    xb = [_host(r.p).copy() for r in res]
    batch.close()
    for p, A, b, r, x in zip(probs, As, bs, res, xb):
        assert r.status == 0 and r.true_relres <= 1e-10
        accept = np.linalg.norm(b - A.matvec(x)) / np.linalg.norm(b)
        assert accept <= 1.05e-10, (p.name, accept)
        err = np.linalg.norm(x - p.extra["xstar"]) / np.linalg.norm(p.extra["xstar"])
        print(p.name, p.mesh.dim, p.mesh.n_nodes, "iters", r.iters, "accept %.2e err %.2e" % (accept, err),
              flush=True)
    for s, b, r, x in zip(systems, rhs, res, xb):
        single = s.solve_mixed(b, rtol=1e-10, inner_rtol=1e-2) if mixed else s.solve(b, rtol=1e-10)
        assert single.iters == r.iters
        assert np.array_equal(_host(single.p).view(np.uint64), x.view(np.uint64))
        s.close()


def test_persistent_batch_equals_two_launch_form():
    """One cooperative launch per step (grid barriers between the CG phases)
    gives the two-launch form's results bit for bit: whole batched solves
    (FP64 and mixed, two chunk lengths), continuous batching with a late
    join, and the real mix at its tuned shape."""
    probs = _small_mix()
    print("case persistent small mix", [(p.mesh.dim, p.mesh.n_nodes) for p in probs], flush=True)
    As = [oracle.assemble_problem(p) for p in probs]
    rhs = [_dev(_rhs(p, A)) for p, A in zip(probs, As)]
    for mixed in (False, True):
        flags = pm.PM_FP64 | (pm.PM_FP32_INNER if mixed else 0)
        systems = [pm.PressureSystem.from_problem(p, flags=flags) for p in probs]
        batch = pm.PressureBatch(systems, tiles_per_slot=2, nodes_per_lane=4, mixed=mixed, inner_rtol=1e-2)
        code, res = batch.solve(rhs, rtol=1e-10)
        assert code == 0
        xb = [_host(r.p).copy() for r in res]
        batch.set_persistent(True)
        for g in (16, 6):
            batch.set_graph(g)
            print("case persistent mixed=%s chunk %d" % (mixed, g), flush=True)
            code2, res2 = batch.solve(rhs, rtol=1e-10)
            assert code2 == 0
            for r, r2, x in zip(res, res2, xb):
                assert r2.iters == r.iters
                assert np.array_equal(_host(r2.p).view(np.uint64), x.view(np.uint64))
        # continuous batching: mesh 3 joins two steps after mesh 0
        print("case persistent continuous mixed=%s" % mixed, flush=True)
        outs = {}
        batch.begin(0, rhs[0], rtol=1e-10)
        started, steps = {0}, 0
        while len(outs) < 2:
            done = batch.step()
            steps += 1
            for m in sorted(started):
                if done[m] and m not in outs:
                    outs[m] = batch.finish(m, rhs[m], rtol=1e-10)
            if steps == 2:
                batch.begin(3, rhs[3], rtol=1e-10)
                started.add(3)
            assert steps < 10000
        for m in (0, 3):
            assert outs[m].iters == res[m].iters
            assert np.array_equal(_host(outs[m].p).view(np.uint64), xb[m].view(np.uint64))
        batch.close()
        for s in systems:
            s.close()
    # the real mix at the tuned shape (its 3D FP64 size class)
    probs = _real_mix_sample()
    print("case persistent real mix", [(p.mesh.dim, p.mesh.n_nodes) for p in probs], flush=True)
    rhs = [_dev(fields.sine_product(p.mesh.coords)) for p in probs]
    systems = [pm.PressureSystem.from_problem(p) for p in probs]
    batch = pm.PressureBatch(systems, tiles_per_slot=8, nodes_per_lane=4)
    code, res = batch.solve(rhs, rtol=1e-10)
    assert code == 0
    xb = [_host(r.p).copy() for r in res]
    batch.set_persistent(True)
    code2, res2 = batch.solve(rhs, rtol=1e-10)
    assert code2 == 0
    for r, r2, x in zip(res, res2, xb):
        assert r2.iters == r.iters
        assert np.array_equal(_host(r2.p).view(np.uint64), x.view(np.uint64))
    batch.close()
    for s in systems:
        s.close()


def test_persistent_barrier_time_out_is_reported():
    """A grid-barrier wait bound far below what the launch needs (1 us) ends
    the step with PM_ETIMEOUT instead of waiting: every wait of the kernel
    is bounded, so the launch ends on its own.  The batch then clears its
    barrier; destroyed, it leaves handles that solve correctly again.  (If
    every barrier happened to complete within the bound, the results must
    be the two-launch form's.)"""
    probs = _small_mix()[:4]
    print("case persistent barrier limit", [(p.mesh.dim, p.mesh.n_nodes) for p in probs], flush=True)
    As = [oracle.assemble_problem(p) for p in probs]
    rhs = [_dev(_rhs(p, A)) for p, A in zip(probs, As)]
    systems = [pm.PressureSystem.from_problem(p) for p in probs]
    batch = pm.PressureBatch(systems, tiles_per_slot=2, nodes_per_lane=4)
    code, ref = batch.solve(rhs, rtol=1e-10)
    assert code == 0
    xr = [_host(r.p).copy() for r in ref]
    batch.set_persistent(True)
    with pytest.raises(pm.PressureError):
        batch.set_barrier_limit(-1)
    batch.set_barrier_limit(1)
    try:
        code2, res2 = batch.solve(rhs, rtol=1e-10)
        timed_out = False
    except pm.PressureError as e:
        assert e.status == pm.PM_ETIMEOUT, e
        timed_out = True
    print("timed out:", timed_out, flush=True)
    if not timed_out:
        for r, x in zip(res2, xr):
            assert np.array_equal(_host(r.p).view(np.uint64), x.view(np.uint64))
    batch.close()
    # the handles are usable again: single solves give the batched results
    for s, b, r, x in zip(systems, rhs, ref, xr):
        single = s.solve(b, rtol=1e-10)
        assert single.iters == r.iters
        assert np.array_equal(_host(single.p).view(np.uint64), x.view(np.uint64))
        s.close()

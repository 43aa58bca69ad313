"""pressure_solve_noalloc (needs an MI355X): the solve whose CG state lives in
the library's static scratch gives what pressure_solve gives on the same
handle, bit for bit, on two calls in a row (the second on a smaller mesh,
so the scratch holds the first call's contents), and the handle's own
solves are unchanged around it."""

import numpy as np
import pytest

import oracle
import paper_2301_08357_amd as pm
from synth import workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _bits(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def _case(prob, mixed_flags=False):
    m = prob.mesh
    A = oracle.assemble_problem(prob)
    if "source" in prob.extra:
        b = oracle.mass_rhs(prob, prob.extra["source"])
    else:
        b = A.matvec(prob.extra["xstar"])
    return A, b


def test_noalloc_solve_equals_solve_twice_second_smaller():
    probs = [workloads.cube(22, w=1e-3, jitter=0.2, rho="lognormal"), workloads.tgv2d(20)]
    assert probs[1].mesh.n_nodes < probs[0].mesh.n_nodes <= pm.PM_NOALLOC_MAX_NODES
    for prob in probs:
        m = prob.mesh
        print("case noalloc", prob.name, m.n_nodes, flush=True)
        A, b = _case(prob)
        s = pm.PressureSystem.from_problem(prob)
        bd = torch.tensor(b, device="cuda")
        x0 = torch.tensor(np.random.default_rng(1).normal(size=m.n_nodes), device="cuda")
        for guess in (None, x0):
            out = torch.empty_like(bd)
            dev_bytes = s.info()["device_bytes"]
            na = s.solve_noalloc(bd, out, x0=guess, rtol=prob.rtol, max_iter=5000)
            # the handle allocated nothing (pressure_solve may grow its history)
            assert s.info()["device_bytes"] == dev_bytes
            ref = s.solve(bd, x0=guess, rtol=prob.rtol, max_iter=5000)
            assert na.status == ref.status == 0
            assert na.iters == ref.iters
            assert np.array_equal(_bits(na.p), _bits(ref.p))
            assert np.array_equal(na.hist.view(np.uint64), ref.hist.view(np.uint64))
            assert na.true_relres == ref.true_relres
            acc = np.linalg.norm(b - A.matvec(na.p.cpu().numpy())) / np.linalg.norm(b)
            assert acc <= 1.05 * prob.rtol, acc
        s.close()


def test_noalloc_limits():
    prob = workloads.cube(6, w=1e-2, jitter=0.2, rho="uniform")
    s = pm.PressureSystem.from_problem(prob)
    b = torch.ones(prob.mesh.n_nodes, dtype=torch.float64, device="cuda")
    out = torch.empty_like(b)
    with pytest.raises(pm.PressureError) as ei:
        s.solve_noalloc(b, out, max_iter=pm.PM_NOALLOC_MAX_ITER + 1)
    assert ei.value.status == pm.PM_ETOOLARGE
    s.close()
    big = workloads.cube(80, w=1e-2, jitter=0.0, rho="uniform")        # 531,441 nodes
    assert big.mesh.n_nodes > pm.PM_NOALLOC_MAX_NODES
    s = pm.PressureSystem.from_problem(big)
    b = torch.ones(big.mesh.n_nodes, dtype=torch.float64, device="cuda")
    with pytest.raises(pm.PressureError) as ei:
        s.solve_noalloc(b, torch.empty_like(b), max_iter=10)
    assert ei.value.status == pm.PM_ETOOLARGE
    s.close()

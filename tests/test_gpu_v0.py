"""The pressure system with no mass term and no Dirichlet node (the zero-Mach
limit; needs an MI355X).  The operator is singular and the weak problem is
posed in V_0 = {z : int z = 0} (paper Sec. 3.4): the library projects the
right-hand side to b - (sum b / |Omega|) m, runs CG, and returns the solution
with int p_h = 0.  Checked against the oracle's dense bordered solve
[A m; m^T 0][p; lam] = [b; 0] at rtol 1e-12 (solutions agree to 1e-9, the
constraint holds to rounding), in FP64, mixed precision and batched form.
"""

import numpy as np
import pytest

import oracle
import paper_2301_08357_amd as pm
from synth import workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _case(prob):
    m = prob.mesh
    A = oracle.assemble_problem(prob)
    mw = oracle.lumped_mass(m.dim, m.coords, m.elems)
    if "source" in prob.extra:
        b = oracle.mass_rhs(prob, prob.extra["source"])
    else:
        b = A.matvec(prob.extra["xstar"])
    return A, mw, b, oracle.solve_v0(A, b, mw)


def _check(prob, A, mw, b, p_ref, x, rtol, tol):
    lam = b.sum() / mw.sum()
    bt = b - lam * mw
    accept = np.linalg.norm(bt - A.matvec(x)) / np.linalg.norm(bt)
    assert accept <= 1.05 * rtol, accept
    assert abs(mw @ x) <= 1e-12 * (np.abs(mw) @ np.abs(x))
    rel = np.linalg.norm(x - p_ref) / np.linalg.norm(p_ref)
    assert rel <= tol, (prob.name, rel)


PROBLEMS = [("square32", lambda: workloads.neumann_square(32)),
            ("cube10_lognormal", lambda: workloads.neumann_cube(10))]


@pytest.mark.parametrize("name,make", PROBLEMS)
def test_v0_apply_and_solve_match_oracle(name, make):
    prob = make()
    print("case", name, prob.mesh.n_nodes, flush=True)
    A, mw, b, p_ref = _case(prob)
    s = pm.PressureSystem.from_problem(prob)
    x = np.random.default_rng(2).normal(size=prob.mesh.n_nodes)
    y = _host(s.apply(_dev(x)))
    S = A.to_scipy()
    assert np.all(np.abs(y - A.matvec(x)) <= 1e-12 * (abs(S) @ np.abs(x)))
    res = s.solve(_dev(b), rtol=1e-12, max_iter=20000)
    assert res.status == 0
    _check(prob, A, mw, b, p_ref, _host(res.p), 1e-12, 1e-9)
    # a warm start from the answer (shifted by a constant) takes no iteration
    res2 = s.solve(_dev(b), x0=res.p + 3.0, rtol=1e-10)
    assert res2.status == 0 and res2.iters <= 1
    _check(prob, A, mw, b, p_ref, _host(res2.p), 1e-10, 1e-9)
    s.close()


def test_v0_mixed_batched_and_coefficient_update():
    prob = workloads.neumann_square(24)
    print("case v0 mixed/batch", prob.mesh.n_nodes, flush=True)
    A, mw, b, p_ref = _case(prob)
    s = pm.PressureSystem.from_problem(prob, flags=pm.PM_FP64 | pm.PM_FP32_INNER)
    r = s.solve_mixed(_dev(b), rtol=1e-10, inner_rtol=1e-2)
    assert r.status == 0
    _check(prob, A, mw, b, p_ref, _host(r.p), 1e-10, 1e-7)
    # batched with a Dirichlet mesh: each result equals its single solve
    other = workloads.tgv2d(12)
    o = pm.PressureSystem.from_problem(other)
    bo = _dev(oracle.mass_rhs(other, other.extra["source"]))
    batch = pm.PressureBatch([s, o], tiles_per_slot=2, nodes_per_lane=4)
    code, res = batch.solve([_dev(b), bo], rtol=1e-12)
    assert code == 0
    _check(prob, A, mw, b, p_ref, _host(res[0].p), 1e-12, 1e-9)
    for sys_, rhs, rb in ((s, _dev(b), res[0]), (o, bo, res[1])):
        single = sys_.solve(rhs, rtol=1e-12)
        assert single.iters == rb.iters
        assert np.array_equal(_host(single.p).view(np.uint64), _host(rb.p).view(np.uint64))
    batch.close()
    o.close()
    # a mass term makes the operator regular again; setting it back to 0
    # returns to V_0
    s.update_coef(prob.coef, mass_coef=1e-3, dt=1.0)
    reg = oracle.assemble(2, prob.mesh.coords, prob.mesh.elems, prob.coef, 1e-3, 1.0, None)
    r = s.solve(_dev(b), rtol=1e-12)
    x_reg = oracle.cg(reg, b, rtol=1e-13, max_iter=20000)[0]
    assert np.linalg.norm(_host(r.p) - x_reg) / np.linalg.norm(x_reg) < 1e-9
    s.update_coef(prob.coef, mass_coef=0.0, dt=1.0)
    r = s.solve(_dev(b), rtol=1e-12)
    _check(prob, A, mw, b, p_ref, _host(r.p), 1e-12, 1e-9)
    s.close()

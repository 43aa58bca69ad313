"""The lumped-mass operator (PM_MASS_LUMPED; needs an MI355X).

alpha diag(m) + beta K_c, m the row sums of the consistent mass, against the
oracle's ``assemble_lumped`` (its own weights from NumPy determinants plus
the assembled stiffness): applies within the rounding bound 1e-12 (|A||x|)_i,
the two apply kernels bit for bit, FP64 solves to the oracle's CG (solution
1e-10, iterations within 2 %), mixed precision, a batch that mixes lumped
and consistent meshes (each equal to its single solve bit for bit), and a
coefficient update.
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


def _rhs(prob, A):
    if "source" in prob.extra:
        return oracle.mass_rhs(prob, prob.extra["source"])
    return A.matvec(prob.extra["xstar"])


PROBS = [("tgv2d_24", lambda: workloads.lumped(workloads.tgv2d(24, w=1.0))),
         ("cube10_lognormal", lambda: workloads.lumped(workloads.cube(10, w=1e-1, jitter=0.2, rho="lognormal"))),
         ("periodic_cube8", lambda: workloads.lumped(workloads.periodic_cube(8, w=1e-2))),
         ("channel12", lambda: workloads.lumped(workloads.periodic_channel(12)))]


@pytest.mark.parametrize("name,make", PROBS)
def test_lumped_apply_and_solve_match_oracle(name, make):
    prob = make()
    m = prob.mesh
    print("case", name, flush=True)
    A = oracle.assemble_problem(prob)
    S = abs(A.to_scipy())
    s = pm.PressureSystem.from_problem(prob)
    x = np.random.default_rng(6).normal(size=m.n_nodes)
    xd = _dev(x)
    s.set_variant(pm.PM_VARIANT_TILED)
    yt = _host(s.apply(xd)).copy()
    s.set_variant(pm.PM_VARIANT_NODE)
    yn = _host(s.apply(xd)).copy()
    s.set_variant(pm.PM_VARIANT_AUTO)
    assert np.array_equal(yt.view(np.uint64), yn.view(np.uint64))
    assert np.all(np.abs(yt - A.matvec(x)) <= 1e-12 * (S @ np.abs(x)))
    # the consistent operator of the same mesh differs (the flag is honoured)
    c = pm.PressureSystem(m.dim, m.coords, m.elems, prob.coef, prob.alpha, 1.0, m.dirichlet, m.lattice,
                          period=m.period)
    assert np.max(np.abs(_host(c.apply(xd)) - yt)) > 1e-6 * np.max(np.abs(yt))
    c.close()
    b = _rhs(prob, A)
    rtol = 1e-12
    x_ref, st_ref, it_ref, _, _ = oracle.cg(A, b, rtol=rtol, max_iter=20000, dirichlet=m.dirichlet)
    res = s.solve(_dev(b), rtol=rtol, max_iter=20000)
    xg = _host(res.p)
    assert res.status == 0 and st_ref == 0
    assert np.linalg.norm(b - A.matvec(xg)) / np.linalg.norm(b) <= 1.05 * rtol
    assert np.linalg.norm(xg - x_ref) / np.linalg.norm(x_ref) <= 1e-10
    assert abs(res.iters - it_ref) <= max(1, 0.02 * it_ref), (res.iters, it_ref)
    s.close()


def test_lumped_mixed_batched_and_update():
    prob = workloads.lumped(workloads.cube(9, w=1e-2, jitter=0.2, rho="lognormal"))
    m = prob.mesh
    print("case lumped mixed/batch", flush=True)
    A = oracle.assemble_problem(prob)
    b = _rhs(prob, A)
    x_ref = oracle.cg(A, b, rtol=1e-13, max_iter=20000, dirichlet=m.dirichlet)[0]
    s = pm.PressureSystem.from_problem(prob, flags=pm.PM_FP64 | pm.PM_FP32_INNER)
    r = s.solve_mixed(_dev(b), rtol=1e-10, inner_rtol=1e-2)
    assert r.status == 0
    assert np.linalg.norm(_host(r.p) - x_ref) / np.linalg.norm(x_ref) < 1e-8
    # a batch with a lumped and a consistent mesh
    other = workloads.cube(7, w=1e-2, jitter=0.2, rho="uniform")
    o = pm.PressureSystem.from_problem(other, flags=pm.PM_FP64 | pm.PM_FP32_INNER)
    bo = _dev(oracle.assemble_problem(other).matvec(other.extra["xstar"]))
    for mixed in (False, True):
        batch = pm.PressureBatch([s, o], tiles_per_slot=2, nodes_per_lane=4, mixed=mixed, inner_rtol=1e-2)
        code, res = batch.solve([_dev(b), bo], rtol=1e-10)
        assert code == 0
        for sys_, rb, rr in ((s, _dev(b), res[0]), (o, bo, res[1])):
            single = (sys_.solve_mixed(rb, rtol=1e-10, inner_rtol=1e-2) if mixed else sys_.solve(rb, rtol=1e-10))
            assert single.iters == rr.iters
            assert np.array_equal(_host(single.p).view(np.uint64), _host(rr.p).view(np.uint64))
        batch.close()
    o.close()
    # a new mass coefficient keeps the lumping
    s.update_coef(None, mass_coef=0.5, dt=0.7)
    A2 = oracle.assemble_lumped(m, prob.coef, 0.5, 0.49)
    x = np.random.default_rng(8).normal(size=m.n_nodes)
    y = _host(s.apply(_dev(x)))
    assert np.all(np.abs(y - A2.matvec(x)) <= 1e-12 * (abs(A2.to_scipy()) @ np.abs(x)))
    s.close()


def test_unknown_flag_bits_rejected():
    prob = workloads.cube(3)
    m = prob.mesh
    with pytest.raises(pm.PressureError) as ei:
        pm.PressureSystem(3, m.coords, m.elems, prob.coef, 1.0, 1.0, m.dirichlet, flags=pm.PM_FP64 | 0x200)
    assert ei.value.status == pm.PM_EINVAL

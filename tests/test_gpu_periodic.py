"""Periodic meshes with merged images (Sec. 3.6; needs an MI355X).

The library takes the merged mesh and the period of each axis and computes
every element from the minimum image of its edge vectors; the oracle
assembles the unmerged mesh, whose images carry their own coordinates, and
forms P^T A P with the 0/1 merge matrix P.  Apply parity within the
rounding bound 1e-12 (|A||x|)_i of the other parity tests; FP64 solves to
the oracle's CG (solution 1e-10, iterations within 2 %, the oracle's
operator accepts the GPU solution at 1.05 rtol); V_0 (alpha = 0, fully
periodic) against the dense bordered solve; mixed precision; a batch that
holds periodic and open meshes, each bit for bit equal to its single
solve; and sampled rows of the 160^3 periodic cube.
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


SMALL = [("square12", lambda: workloads.periodic_square(12)),
         ("channel10", lambda: workloads.periodic_channel(10)),
         ("cube8", lambda: workloads.periodic_cube(8)),
         ("cube7_x_only", lambda: _cube_axes(7, (0,))),
         ("cube9_alpha0", lambda: workloads.periodic_cube(9, w=0.0))]


def _cube_axes(n, axes):
    from synth import fields, mesh as smesh
    m = smesh.periodic_mesh(3, n, axes, jitter=0.2, seed=17)
    c = 1.0 / fields.rho_uniform(17, m.n_elems)
    xs = np.prod(np.sin(2.0 * np.pi * m.coords), axis=1)
    return workloads.Problem("cube%d_axes" % n, m, c, 1e-2, 1.0, 1e-10, 17, extra={"xstar": xs})


@pytest.mark.parametrize("name,make", SMALL)
def test_periodic_apply_matches_oracle_and_kernels_agree(name, make):
    prob = make()
    m = prob.mesh
    print("case", name, m.n_nodes, flush=True)
    A = oracle.assemble_problem(prob)
    S = abs(A.to_scipy())
    x = np.random.default_rng(4).normal(size=m.n_nodes)
    for tile in (pm.PM_TILE_128, pm.PM_TILE_256):
        s = pm.PressureSystem.from_problem(prob, flags=pm.PM_FP64 | tile)
        xd = _dev(x)
        s.set_variant(pm.PM_VARIANT_TILED)
        yt = _host(s.apply(xd)).copy()
        s.set_variant(pm.PM_VARIANT_NODE)
        yn = _host(s.apply(xd)).copy()
        assert np.array_equal(yt.view(np.uint64), yn.view(np.uint64))
        assert np.all(np.abs(yt - A.matvec(x)) <= 1e-12 * (S @ np.abs(x)))
        s.close()


@pytest.mark.parametrize("name,make", SMALL[:4])
def test_periodic_solve_matches_oracle(name, make):
    prob = make()
    m = prob.mesh
    print("case", name, flush=True)
    A = oracle.assemble_problem(prob)
    b = _rhs(prob, A)
    x_ref, st_ref, it_ref, _, _ = oracle.cg(A, b, rtol=prob.rtol, max_iter=20000, dirichlet=m.dirichlet)
    assert st_ref == 0
    s = pm.PressureSystem.from_problem(prob)
    res = s.solve(_dev(b), rtol=prob.rtol, max_iter=20000)
    x = _host(res.p)
    assert res.status == 0
    assert abs(res.iters - it_ref) <= max(1, 0.02 * it_ref), (res.iters, it_ref)
    assert np.linalg.norm(b - A.matvec(x)) / np.linalg.norm(b) <= 1.05 * prob.rtol
    rel = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)
    assert rel <= 1e-10, rel
    assert res.true_relres <= prob.rtol
    if "xstar" in prob.extra:
        xs = prob.extra["xstar"]
        assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-6
    s.close()


def test_periodic_v0_mixed_and_batched():
    prob = workloads.periodic_cube(10, w=0.0)
    m = prob.mesh
    print("case periodic V_0", m.n_nodes, flush=True)
    A = oracle.assemble_problem(prob)
    mw = oracle.lumped_mass_mesh(m)
    b = A.matvec(prob.extra["xstar"])
    p_ref = oracle.solve_v0(A, b, mw)
    s = pm.PressureSystem.from_problem(prob, flags=pm.PM_FP64 | pm.PM_FP32_INNER)
    res = s.solve(_dev(b), rtol=1e-12)
    x = _host(res.p)
    assert res.status == 0
    assert abs(mw @ x) <= 1e-12 * (mw @ np.abs(x))
    assert np.linalg.norm(x - p_ref) / np.linalg.norm(p_ref) < 1e-9
    r = s.solve_mixed(_dev(b), rtol=1e-10, inner_rtol=1e-2)
    assert r.status == 0
    assert np.linalg.norm(_host(r.p) - p_ref) / np.linalg.norm(p_ref) < 1e-7
    # a batch with a periodic and an open mesh: each equals its single solve
    other = workloads.tgv2d(12)
    o = pm.PressureSystem.from_problem(other)
    bo = _dev(oracle.mass_rhs(other, other.extra["source"]))
    sq = workloads.periodic_square(16)
    q = pm.PressureSystem.from_problem(sq)
    bq = _dev(oracle.mass_rhs(sq, sq.extra["source"]))
    systems, rhs = [s, o, q], [_dev(b), bo, bq]
    batch = pm.PressureBatch(systems, tiles_per_slot=2, nodes_per_lane=4)
    code, res_b = batch.solve(rhs, rtol=1e-11)
    assert code == 0
    for sys_, rb, rr in zip(systems, rhs, res_b):
        single = sys_.solve(rb, rtol=1e-11)
        assert single.iters == rr.iters
        assert np.array_equal(_host(single.p).view(np.uint64), _host(rr.p).view(np.uint64))
    batch.close()
    for t in (s, o, q):
        t.close()


def test_cube160_periodic_sampled_rows():
    """The fully periodic 160^3 cube (the bench's periodic workload): sampled
    rows of y = A x against the oracle's element sums on the unmerged mesh,
    added over the images of each sampled node."""
    prob = workloads.cube160p()
    m = prob.mesh
    u = m.unmerged
    print("case cube160p", m.n_nodes, flush=True)
    x = np.random.default_rng(21).normal(size=m.n_nodes)
    s = pm.PressureSystem.from_problem(prob)
    y = _host(s.apply(_dev(x)))
    s.close()
    rows = np.random.default_rng(22).choice(m.n_nodes, 1500, replace=False)
    rows = np.concatenate([rows, [0, m.n_nodes - 1]])      # node 0 has 8 images
    want = np.zeros(m.n_nodes, dtype=bool)
    want[rows] = True
    images = np.nonzero(want[m.rep])[0]
    yu = oracle.apply_elements(3, u.coords, u.elems, prob.coef, prob.alpha, prob.beta, None, x[m.rep], rows=images)
    yr = np.bincount(m.rep[images], weights=yu, minlength=m.n_nodes)[rows]
    scale = np.abs(yr).max()
    np.testing.assert_allclose(y[rows], yr, rtol=1e-11, atol=1e-12 * scale)

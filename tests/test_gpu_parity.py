"""Parity of the HIP path with the CPU oracle (needs an MI355X).

Apply: element by element against the oracle's assembled operator, within
a rounding bound derived from the arithmetic: each output is a sum of at
most ~100 FP64 products, so |y_gpu - y_oracle| <= 1e-12 * (|A| |x|)_i
(two orders of magnitude above gamma_100 * (|A||x|)_i).
Solve (FP64 CG): the oracle's operator accepts the GPU solution at the
requested tolerance (1.05 x rtol), the solutions agree to 1e-10 relative on
the smooth manufactured problems, iteration counts agree within 2 %, and the
residual histories agree to 1e-8 relative over their first 50 entries or,
if shorter, over the prefix where the oracle's own history is insensitive
to 1e-15 perturbations of the right-hand side.
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


def _abs_bound(A, x):
    import scipy.sparse as sp
    S = A.to_scipy()
    return abs(S) @ np.abs(x)


PROBLEMS = [
    ("tgv2d_32", lambda: workloads.tgv2d(32)),
    ("cube12_lognormal_jit", lambda: workloads.cube(12, w=1e-4, jitter=0.2, rho="lognormal")),
    ("cube9_uniform", lambda: workloads.cube(9, w=1.0, jitter=0.0, rho="uniform")),
    ("square37_w1e-6", lambda: workloads.Problem("sq37", smesh.structured_mesh(2, 37, jitter=0.2, seed=4),
                                                  1.0 / fields.rho_uniform(4, 2 * 37 * 37), 1e-6, 1.0,
                                                  1e-10, 4)),
]


@pytest.mark.parametrize("name,make", PROBLEMS)
def test_apply_matches_oracle(name, make):
    prob = make()
    m = prob.mesh
    print("case", name, m.n_nodes, m.n_elems, flush=True)
    A = oracle.assemble_problem(prob)
    rng = np.random.default_rng(7)
    x = rng.normal(size=m.n_nodes)
    y_ref = A.matvec(x)
    s = pm.PressureSystem.from_problem(prob)
    y = _host(s.apply(_dev(x)))
    bound = 1e-12 * _abs_bound(A, x)
    assert np.all(np.abs(y - y_ref) <= bound), np.max(np.abs(y - y_ref) / bound)
    # Dirichlet rows are the identity
    d = m.dirichlet == 1
    assert np.array_equal(y[d], x[d])
    s.close()


def _stable_prefix(A, b, rtol, dirichlet, h_ref, cap):
    """Length of the leading part of the oracle's residual history that is
    insensitive to rounding: the oracle rerun with b perturbed by 1e-15
    relative noise must agree there to 1e-10.  Past that point CG's
    finite-precision trajectory amplifies last-bit differences (by up to
    ~1e14 on the w = 1e-6 square), so no implementation with another
    summation order can be held to the oracle's history there."""
    rng = np.random.default_rng(0)
    b2 = b * (1 + 1e-15 * rng.normal(size=b.size))
    _, _, _, h2, _ = oracle.cg(A, b2, rtol=rtol, max_iter=20000, dirichlet=dirichlet)
    k = min(cap, len(h_ref), len(h2))
    bad = np.nonzero(np.abs(h2[:k] - h_ref[:k]) > 1e-10 * h_ref[:k])[0]
    return int(bad[0]) if bad.size else k


def _rhs_for(prob, A):
    if "source" in prob.extra:
        return oracle.mass_rhs(prob, prob.extra["source"])
    return A.matvec(fields.sine_product(prob.mesh.coords))


@pytest.mark.parametrize("name,make", PROBLEMS)
def test_solve_matches_oracle(name, make):
    prob = make()
    m = prob.mesh
    print("case", name, flush=True)
    A = oracle.assemble_problem(prob)
    b = _rhs_for(prob, A)
    x_ref, st_ref, it_ref, h_ref, tr_ref = oracle.cg(A, b, rtol=prob.rtol, max_iter=20000, dirichlet=m.dirichlet)
    assert st_ref == 0
    s = pm.PressureSystem.from_problem(prob)
    res = s.solve(_dev(b), rtol=prob.rtol, max_iter=20000)
    x = _host(res.p)
    assert res.status == 0
    accept = np.linalg.norm(b - A.matvec(x)) / np.linalg.norm(b)
    assert accept <= 1.05 * prob.rtol, accept
    rel = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)
    assert rel <= 1e-10 if prob.rtol <= 1e-10 else rel <= 100 * prob.rtol, rel
    assert abs(res.iters - it_ref) <= max(1, 0.02 * it_ref), (res.iters, it_ref)
    k = _stable_prefix(A, b, prob.rtol, m.dirichlet, h_ref, 50)
    assert k >= 10
    np.testing.assert_allclose(res.hist[:k], h_ref[:k], rtol=1e-8)
    assert res.true_relres <= prob.rtol
    s.close()


def test_solve_is_bitwise_deterministic():
    prob = workloads.cube(10, w=1e-3, jitter=0.2, rho="lognormal")
    A = oracle.assemble_problem(prob)
    b = _dev(_rhs_for(prob, A))
    s = pm.PressureSystem.from_problem(prob)
    r1 = s.solve(b, rtol=1e-10)
    x1 = _host(r1.p).copy()
    r2 = s.solve(b, rtol=1e-10)
    x2 = _host(r2.p)
    assert r1.iters == r2.iters
    assert np.array_equal(x1.view(np.uint64), x2.view(np.uint64))
    assert np.array_equal(r1.hist.view(np.uint64), r2.hist.view(np.uint64))
    y1 = _host(s.apply(b)).copy()
    y2 = _host(s.apply(b))
    assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))
    s.close()


def test_solve_edge_cases():
    prob = workloads.cube(6, w=1e-2, jitter=0.2, rho="uniform")
    m = prob.mesh
    A = oracle.assemble_problem(prob)
    b = _rhs_for(prob, A)
    s = pm.PressureSystem.from_problem(prob)
    # zero right-hand side: p = 0, no iterations, even from a nonzero guess
    r = s.solve(_dev(np.zeros(m.n_nodes)), x0=_dev(np.ones(m.n_nodes)), rtol=1e-10)
    assert r.status == 0 and r.iters == 0 and np.all(_host(r.p) == 0)
    # iteration cap: not converged, history of max_iter + 1 entries
    r = s.solve(_dev(b), rtol=1e-12, max_iter=3)
    assert r.status == pm.PM_NOT_CONVERGED and r.iters == 3 and r.hist.shape[0] == 4
    x3, st3, it3, h3, _ = oracle.cg(A, b, rtol=1e-12, max_iter=3, dirichlet=m.dirichlet)
    np.testing.assert_allclose(_host(r.p), x3, rtol=1e-11, atol=1e-14)
    # max_iter = 0
    r = s.solve(_dev(b), rtol=1e-12, max_iter=0)
    assert r.status == pm.PM_NOT_CONVERGED and r.iters == 0
    # warm start from the solution: converged without iterations
    r = s.solve(_dev(b), rtol=1e-11)
    r2 = s.solve(_dev(b), x0=r.p.clone(), rtol=1e-10)
    assert r2.status == 0 and r2.iters == 0
    # warm start from an arbitrary guess equals the oracle's warm start
    x0 = np.random.default_rng(3).normal(size=m.n_nodes)
    r3 = s.solve(_dev(b), x0=_dev(x0), rtol=1e-10)
    xo, sto, ito, _, _ = oracle.cg(A, b, x0=x0, rtol=1e-10, dirichlet=m.dirichlet)
    assert abs(r3.iters - ito) <= 1
    # Dirichlet values are imposed exactly
    bd = b.copy()
    bd[m.dirichlet == 1] = 0.25
    r4 = s.solve(_dev(bd), rtol=1e-10)
    assert np.all(_host(r4.p)[m.dirichlet == 1] == 0.25)
    # NaN in the rhs is an invalid argument
    bn = b.copy()
    bn[5] = np.nan
    with pytest.raises(pm.PressureError) as ei:
        s.solve(_dev(bn), rtol=1e-10)
    assert ei.value.status == pm.PM_EINVAL
    with pytest.raises(pm.PressureError):
        s.solve(_dev(b), rtol=0.0)
    s.close()


def test_setup_errors():
    m = smesh.structured_mesh(3, 3, jitter=0.2, seed=1)
    with pytest.raises(pm.PressureError) as ei:
        pm.PressureSystem(3, m.coords, m.elems, -np.ones(m.n_elems), 1.0, 1.0, m.dirichlet, m.lattice)
    assert ei.value.status == pm.PM_EINVAL
    bad = m.elems.copy()
    bad[0, 1] = bad[0, 0]
    with pytest.raises(pm.PressureError) as ei:
        pm.PressureSystem(3, m.coords, bad, np.ones(m.n_elems), 1.0, 1.0, m.dirichlet)
    assert ei.value.status == pm.PM_EDEGENERATE


def test_update_coef_matches_new_setup():
    prob = workloads.cube(8, w=1e-3, jitter=0.2, rho="uniform")
    m = prob.mesh
    s = pm.PressureSystem.from_problem(prob)
    c2 = 1.0 / fields.rho_lognormal(99, m.n_elems)
    s.update_coef(c2, mass_coef=0.5, dt=0.3)
    A2 = oracle.assemble(3, m.coords, m.elems, c2, 0.5, 0.09, m.dirichlet)
    x = np.random.default_rng(2).normal(size=m.n_nodes)
    y = _host(s.apply(_dev(x)))
    bound = 1e-12 * _abs_bound(A2, x)
    assert np.all(np.abs(y - A2.matvec(x)) <= bound)
    s.close()


# ------------------------------------------------------------ full sizes
def test_cube64_full_size_solve():
    """The 64^3 benchmark mesh, w = 1e-3: the oracle's matrix-free operator
    accepts the GPU solution, which agrees with the oracle's own CG solution
    to 1e-10 relative, and the discrete manufactured solution is
    recovered."""
    prob = workloads.cube64(1e-3)
    m = prob.mesh
    print("case cube64", flush=True)
    xs = prob.extra["xstar"]
    s = pm.PressureSystem.from_problem(prob)
    b = _host(s.apply(_dev(xs)))
    b_ref = oracle.apply_elements(3, m.coords, m.elems, prob.coef, prob.alpha, prob.beta, m.dirichlet, xs)
    assert np.linalg.norm(b - b_ref) <= 1e-13 * np.linalg.norm(b_ref)
    res = s.solve(_dev(b_ref), rtol=1e-10)
    x = _host(res.p)
    assert res.status == 0
    r = b_ref - oracle.apply_elements(3, m.coords, m.elems, prob.coef, prob.alpha, prob.beta, m.dirichlet, x)
    assert np.linalg.norm(r) / np.linalg.norm(b_ref) <= 1.05e-10
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-10
    A = oracle.assemble_problem(prob)
    x_o, st_o, it_o, _, _ = oracle.cg(A, b_ref, rtol=1e-10, max_iter=20000, dirichlet=m.dirichlet)
    assert st_o == 0 and abs(res.iters - it_o) <= max(1, 0.02 * it_o), (res.iters, it_o)
    assert np.linalg.norm(x - x_o) / np.linalg.norm(x_o) <= 1e-10
    s.close()


@pytest.mark.parametrize("tile", [pm.PM_TILE_128, pm.PM_TILE_256])
def test_cube160_full_size_solves(tile):
    """The 160^3 benchmark system (jittered, lognormal rho, w = 1e-4), in the
    bench's launch configurations (the default 128-node tiles and the
    256-node tiles the autotuner picks for it): the FP64 CG solve and the mixed solve
    (FP32 inner CG, FP64 corrections, inner residual drop 1e-2) of the
    oracle's right-hand side b = A x*, each accepted by one full residual of
    the oracle's element-by-element operator at 1.05 x rtol, and each within
    1e-10 relative of x*, the exact solution of that system."""
    prob = workloads.cube160()
    m = prob.mesh
    print("case cube160 solves, tile flag", tile, flush=True)
    xs = prob.extra["xstar"]
    args = (3, m.coords, m.elems, prob.coef, prob.alpha, prob.beta, m.dirichlet)
    b = oracle.apply_elements(*args, xs)
    bn = np.linalg.norm(b)
    s = pm.PressureSystem.from_problem(prob, flags=pm.PM_FP64 | pm.PM_FP32_INNER | tile)
    bd = _dev(b)
    r64 = s.solve(bd, rtol=1e-10)
    x64 = _host(r64.p).copy()
    rmx = s.solve_mixed(bd, rtol=1e-10, inner_rtol=1e-2)
    xmx = _host(rmx.p).copy()
    s.close()
    print("iterations fp64 %d mixed %d (%d corrections)" % (r64.iters, rmx.iters, rmx.outer), flush=True)
    assert r64.status == 0 and rmx.status == 0
    for name, x in (("fp64", x64), ("mixed", xmx)):
        acc = np.linalg.norm(b - oracle.apply_elements(*args, x)) / bn
        err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
        print(name, "oracle residual %.3e error vs x* %.3e" % (acc, err), flush=True)
        assert acc <= 1.05e-10, (name, acc)
        assert err <= 1e-10, (name, err)


@pytest.mark.parametrize("tile", [pm.PM_TILE_128, pm.PM_TILE_256])
def test_cube160_sampled_rows(tile):
    """The 160^3 mesh: sampled rows of y = A x against the oracle row by row."""
    prob = workloads.cube160()
    m = prob.mesh
    print("case cube160, tile flag", tile, flush=True)
    x = np.random.default_rng(11).normal(size=m.n_nodes)
    s = pm.PressureSystem.from_problem(prob, flags=pm.PM_FP64 | tile)
    y = _host(s.apply(_dev(x)))
    rows = np.random.default_rng(12).choice(m.n_nodes, 2000, replace=False)
    rows = np.concatenate([rows, [0, m.n_nodes - 1]])
    yr = oracle.apply_elements(3, m.coords, m.elems, prob.coef, prob.alpha, prob.beta, m.dirichlet, x, rows=rows)
    scale = np.abs(yr).max()
    np.testing.assert_allclose(y[rows], yr, rtol=1e-11, atol=1e-12 * scale)
    s.close()


# ------------------------------------------------------ kernel variants
@pytest.mark.parametrize("tile", [pm.PM_TILE_128, pm.PM_TILE_256, pm.PM_TILE_512])
def test_tiled_and_node_kernels_agree_bitwise(tile):
    """Both apply kernels sum each node's element contributions in ascending
    element order with the same arithmetic, so they agree bit for bit, for
    every tile size (ragged last tile included)."""
    for prob in (workloads.cube(13, w=1e-4, jitter=0.2, rho="lognormal"), workloads.tgv2d(45)):
        m = prob.mesh
        print("case", prob.name, tile, flush=True)
        s = pm.PressureSystem.from_problem(prob, flags=pm.PM_FP64 | tile)
        x = _dev(np.random.default_rng(5).normal(size=m.n_nodes))
        s.set_variant(pm.PM_VARIANT_TILED)
        yt = _host(s.apply(x)).copy()
        s.set_variant(pm.PM_VARIANT_NODE)
        yn = _host(s.apply(x)).copy()
        assert np.array_equal(yt.view(np.uint64), yn.view(np.uint64))
        A = oracle.assemble_problem(prob)
        b = _dev(_rhs_for(prob, A))
        rn = s.solve(b, rtol=1e-10)
        xn = _host(rn.p).copy()
        s.set_variant(pm.PM_VARIANT_TILED)
        rt = s.solve(b, rtol=1e-10)
        assert rt.iters == rn.iters
        assert np.array_equal(_host(rt.p).view(np.uint64), xn.view(np.uint64))
        s.close()


# ------------------------------------------------------ one-launch small-mesh solve
ONE_LAUNCH = [
    ("tgv2d_32", lambda: workloads.tgv2d(32)),
    ("cube7_lognormal_jit", lambda: workloads.cube(7, w=1e-4, jitter=0.2, rho="lognormal")),
    ("periodic_square_24", lambda: workloads.periodic_square(24)),
    ("periodic_cube6_alpha0", lambda: workloads.periodic_cube(6, w=0.0)),
]


@pytest.mark.parametrize("name,make", ONE_LAUNCH)
def test_one_launch_solve_equals_two_launch_loop(name, make):
    """A mesh that fits one workgroup's LDS runs all its CG iterations in one
    launch; kernel timing keeps the two-launch loop.  The two give the same
    bits (solution, status, iteration count, residual history, true
    residual) on a cold start, a warm start, an iteration cap, an rtol
    below what FP64 reaches (residual replacement and its restart) and a
    zero right-hand side."""
    prob = make()
    m = prob.mesh
    print("case", name, m.n_nodes, m.n_elems, flush=True)
    A = oracle.assemble_problem(prob)
    b = _dev(_rhs_for(prob, A))
    s = pm.PressureSystem.from_problem(prob)
    assert s.info()["one_launch_solve"] == 1
    x0 = _dev(np.random.default_rng(3).normal(size=m.n_nodes))
    cases = [("cold", b, dict(rtol=1e-10)), ("warm", b, dict(x0=x0, rtol=1e-10)),
             ("cap7", b, dict(rtol=1e-10, max_iter=7)), ("tight", b, dict(rtol=1e-17, max_iter=3000)),
             ("zero", torch.zeros_like(b), dict(rtol=1e-10))]
    for label, rhs, kw in cases:
        print("  ", label, flush=True)
        out = []
        for timing in (False, True):
            s.timing_enable(timing)
            assert s.info()["one_launch_solve"] == (0 if timing else 1)
            r = s.solve(rhs, **kw)
            out.append((_host(r.p).copy(), r.status, r.iters, r.hist, r.true_relres))
        (p1, st1, it1, h1, t1), (p2, st2, it2, h2, t2) = out
        assert (st1, it1) == (st2, it2), (label, st1, it1, st2, it2)
        assert np.array_equal(p1.view(np.uint64), p2.view(np.uint64)), label
        assert np.array_equal(h1.view(np.uint64), h2.view(np.uint64)), label
        assert t1 == t2 or (np.isnan(t1) and np.isnan(t2)), label
        if label == "cold":
            assert st1 == 0 and t1 <= 1e-10
        if label == "cap7":
            assert st1 == pm.PM_NOT_CONVERGED and it1 == 7
        if label == "zero":
            assert it1 == 0 and not np.any(p1)
    s.timing_enable(False)
    s.close()
    # a mesh too large for one workgroup's LDS keeps the two-launch form
    big = pm.PressureSystem.from_problem(workloads.tgv2d(45))
    assert big.info()["one_launch_solve"] == 0
    big.close()


# ------------------------------------------------------ mixed precision
@pytest.mark.parametrize("mode", [pm.PM_MIXED_KEEP_DIRECTION, pm.PM_MIXED_RESTART])
@pytest.mark.parametrize("name,make", [PROBLEMS[0], PROBLEMS[1], PROBLEMS[3]])
def test_mixed_precision_reaches_fp64_residual(name, make, mode):
    """FP32 inner CG inside FP64 defect correction: the oracle's FP64
    operator accepts the result at the requested tolerance, and the result
    agrees with the oracle's FP64 CG solution.  Keeping the inner search
    direction across corrections keeps the inner iteration count close to
    the FP64 CG's."""
    prob = make()
    m = prob.mesh
    print("case", name, "mode", mode, flush=True)
    A = oracle.assemble_problem(prob)
    b = _rhs_for(prob, A)
    x_ref, st_ref, it_ref, _, _ = oracle.cg(A, b, rtol=prob.rtol, max_iter=20000, dirichlet=m.dirichlet)
    s = pm.PressureSystem.from_problem(prob, flags=pm.PM_FP64 | pm.PM_FP32_INNER)
    s.set_mixed_mode(mode)
    eta = 1e-2 if mode == pm.PM_MIXED_KEEP_DIRECTION else 1e-4
    res = s.solve_mixed(_dev(b), rtol=prob.rtol, inner_rtol=eta, max_iter=20000)
    x = _host(res.p)
    assert res.status == 0 and res.outer >= 1
    accept = np.linalg.norm(b - A.matvec(x)) / np.linalg.norm(b)
    assert accept <= 1.05 * prob.rtol, accept
    assert res.true_relres <= prob.rtol
    assert np.all(np.diff(res.hist) < 0) and res.hist[-1] <= prob.rtol
    rel = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)
    assert rel <= 1e-10 if prob.rtol <= 1e-10 else rel <= 100 * prob.rtol, rel
    if mode == pm.PM_MIXED_KEEP_DIRECTION:
        assert res.iters <= 1.5 * it_ref + 20, (res.iters, it_ref)
    # bitwise reproducible
    res2 = s.solve_mixed(_dev(b), rtol=prob.rtol, inner_rtol=eta, max_iter=20000)
    assert res2.iters == res.iters
    assert np.array_equal(_host(res2.p).view(np.uint64), x.view(np.uint64))
    s.close()


def test_mixed_precision_edge_cases():
    prob = workloads.cube(6, w=1e-2, jitter=0.2, rho="uniform")
    m = prob.mesh
    s64 = pm.PressureSystem.from_problem(prob)
    with pytest.raises(pm.PressureError):
        s64.solve_mixed(_dev(np.ones(m.n_nodes)), rtol=1e-10)
    s64.close()
    s = pm.PressureSystem.from_problem(prob, flags=pm.PM_FP64 | pm.PM_FP32_INNER)
    r = s.solve_mixed(_dev(np.zeros(m.n_nodes)), rtol=1e-10)
    assert r.status == 0 and r.iters == 0 and np.all(_host(r.p) == 0)
    A = oracle.assemble_problem(prob)
    b = _rhs_for(prob, A)
    r = s.solve_mixed(_dev(b), rtol=1e-10, max_iter=5)
    assert r.status == pm.PM_NOT_CONVERGED and r.iters <= 5
    with pytest.raises(pm.PressureError):
        s.solve_mixed(_dev(b), rtol=1e-10, inner_rtol=1.5)
    s.close()

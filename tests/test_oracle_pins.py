"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: counts
printed in the paper, closed-form element matrices, finite-difference
stencils that the P1 operator reduces to on uniform meshes, a closed-form
eigenpair, a library Cholesky factorisation, symmetry/positivity, and the
textbook O(h^2) L2 convergence to a manufactured solution.
"""

import math
import os

import numpy as np
import pytest

import oracle
from synth import mesh as smesh
from synth import workloads, fields


# ---------------------------------------------------------------- meshes
def _edges(elems):
    nv = elems.shape[1]
    pairs = []
    for a in range(nv):
        for b in range(a + 1, nv):
            pairs.append(np.sort(elems[:, [a, b]], axis=1))
    p = np.concatenate(pairs).astype(np.int64)
    return np.unique(p[:, 0] * (1 << 32) + p[:, 1]).size


def test_table1_counts(golden_dir):
    """Paper Table 1: elements / vertices / dual elements (= edges) of M1..M6."""
    rows = [l.split() for l in open(os.path.join(golden_dir, "table1_meshes.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 6
    for name, N, ne, nv, nd in rows:
        N, ne, nv, nd = int(N), int(ne), int(nv), int(nd)
        assert smesh.table1_counts(N) == (nv, ne, nd), name
        if N <= 128:  # build the actual meshes for the smaller ones
            m = smesh.structured_mesh(2, N)
            assert m.n_elems == ne and m.n_nodes == nv, name
            assert _edges(m.elems) == nd, name


def test_3d_counts_and_degrees():
    for n in (2, 3, 5):
        m = smesh.structured_mesh(3, n, jitter=0.2, seed=7)
        assert m.n_nodes == (n + 1) ** 3 and m.n_elems == 6 * n ** 3
        deg = np.bincount(m.elems.ravel(), minlength=m.n_nodes)
        assert deg.sum() == 4 * m.n_elems
        interior = m.dirichlet == 0
        assert np.all(deg[interior] == 24)
    m = smesh.structured_mesh(2, 6, jitter=0.2, seed=7)
    deg = np.bincount(m.elems.ravel(), minlength=m.n_nodes)
    assert np.all(deg[m.dirichlet == 0] == 6)


def test_generated_orientation_positive():
    for dim, n in ((2, 9), (3, 4)):
        m = smesh.structured_mesh(dim, n, jitter=0.2, seed=11)
        dets = np.array([oracle.lib().orc_element_det(dim, oracle._p(np.ascontiguousarray(m.coords[m.elems[e]])))
                         for e in range(m.n_elems)])
        h = 1.0 / n
        nominal = h ** dim
        assert np.all(dets > 0.1 * nominal)


# ------------------------------------------------------- element matrices
def test_reference_triangle():
    xv = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    K, det = oracle.element_matrix(2, xv, c=1.0, alpha=0.0, beta=1.0)
    assert det == 1.0
    np.testing.assert_allclose(K, 0.5 * np.array([[2, -1, -1], [-1, 1, 0], [-1, 0, 1]]), atol=1e-15)
    M, _ = oracle.element_matrix(2, xv, c=1.0, alpha=1.0, beta=0.0)
    np.testing.assert_allclose(M, (1.0 / 24.0) * (np.ones((3, 3)) + np.eye(3)), atol=1e-16)


def test_reference_tetrahedron():
    xv = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    K, det = oracle.element_matrix(3, xv, c=1.0, alpha=0.0, beta=1.0)
    assert det == 1.0
    ref = np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]]) / 6.0
    np.testing.assert_allclose(K, ref, atol=1e-15)
    M, _ = oracle.element_matrix(3, xv, c=1.0, alpha=1.0, beta=0.0)
    np.testing.assert_allclose(M, (np.ones((4, 4)) + np.eye(4)) / 120.0, atol=1e-16)


@pytest.mark.parametrize("dim", [2, 3])
def test_element_invariants(dim):
    rng = np.random.default_rng(3)
    for _ in range(50):
        xv = rng.normal(size=(dim + 1, dim))
        c, alpha, beta = rng.uniform(0.5, 2), rng.uniform(0, 3), rng.uniform(0.1, 2)
        A, det = oracle.element_matrix(dim, xv, c, alpha, beta)
        vol = abs(det) / math.factorial(dim)
        K, _ = oracle.element_matrix(dim, xv, 1.0, 0.0, 1.0)
        M, _ = oracle.element_matrix(dim, xv, 1.0, 1.0, 0.0)
        np.testing.assert_allclose(A, beta * c * K + alpha * M, rtol=1e-12, atol=1e-12)
        # constants are in the kernel of K; M integrates to |T|
        np.testing.assert_allclose(K @ np.ones(dim + 1), 0.0, atol=1e-10 * np.abs(K).max())
        assert abs(M.sum() - vol) <= 1e-13 * vol
        # a linear field l(x) = g.x: (K l)_a = |T| grad(phi_a).g and sum_a = 0
        g = rng.normal(size=dim)
        Kl = K @ (xv @ g)
        assert abs(Kl.sum()) <= 1e-10 * np.abs(Kl).max()
        # energy of a linear field = |T| |g|^2
        np.testing.assert_allclose((xv @ g) @ Kl, vol * g @ g, rtol=1e-10)
        # symmetric, invariant under translation and relabelling of vertices
        assert np.array_equal(A, A.T)
        A2, _ = oracle.element_matrix(dim, xv + 3.25, c, alpha, beta)
        np.testing.assert_allclose(A2, A, rtol=1e-9, atol=1e-12 * np.abs(A).max())
        perm = rng.permutation(dim + 1)
        A3, _ = oracle.element_matrix(dim, xv[perm], c, alpha, beta)
        np.testing.assert_allclose(A3, A[np.ix_(perm, perm)], rtol=1e-9, atol=1e-12 * np.abs(A).max())
        # scaling by s: K scales with s^(d-2), M with s^d
        Ks, _ = oracle.element_matrix(dim, 2.0 * xv, 1.0, 0.0, 1.0)
        np.testing.assert_allclose(Ks, 2.0 ** (dim - 2) * K, rtol=1e-10, atol=1e-12 * np.abs(K).max())


# ------------------------------------------------------- assembled operator
def test_stencil_2d_five_point():
    """Unjittered two-triangle split: the P1 stiffness row of an interior node
    is the 5-point Laplacian [-1 -1 4 -1 -1]; the consistent mass row is
    h^2/2 on the diagonal and h^2/12 on the six edge neighbours."""
    n = 8
    m = smesh.structured_mesh(2, n)
    K = oracle.assemble(2, m.coords, m.elems, np.ones(m.n_elems), 0.0, 1.0).dense()
    M = oracle.assemble(2, m.coords, m.elems, np.ones(m.n_elems), 1.0, 0.0).dense()
    h = 1.0 / n
    idx = lambda i, j: i + (n + 1) * j
    for i in range(1, n):
        for j in range(1, n):
            r = idx(i, j)
            kr = np.zeros(m.n_nodes)
            kr[r] = 4
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                kr[idx(i + di, j + dj)] = -1
            np.testing.assert_allclose(K[r], kr, atol=1e-12)
            mr = np.zeros(m.n_nodes)
            mr[r] = h * h / 2
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1)):
                mr[idx(i + di, j + dj)] = h * h / 12
            np.testing.assert_allclose(M[r], mr, atol=1e-15)


def test_stencil_3d_seven_point():
    """Unjittered Kuhn split: interior stiffness row = h * 7-point stencil."""
    n = 6
    m = smesh.structured_mesh(3, n)
    K = oracle.assemble(3, m.coords, m.elems, np.ones(m.n_elems), 0.0, 1.0).dense()
    h = 1.0 / n
    m1 = n + 1
    idx = lambda i, j, k: i + m1 * (j + m1 * k)
    for i in range(1, n):
        for j in range(1, n):
            for k in range(1, n):
                r = idx(i, j, k)
                kr = np.zeros(m.n_nodes)
                kr[r] = 6 * h
                for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    kr[idx(i + d[0], j + d[1], k + d[2])] = -h
                np.testing.assert_allclose(K[r], kr, atol=1e-13)


@pytest.mark.parametrize("dim,n", [(2, 12), (3, 7)])
def test_sine_eigenpair(dim, n):
    """K_II s = lambda s for s = prod sin(pi x_i) with the closed-form
    eigenvalue of the 5-/7-point stencil."""
    m = smesh.structured_mesh(dim, n)
    A = oracle.assemble(dim, m.coords, m.elems, np.ones(m.n_elems), 0.0, 1.0, m.dirichlet)
    s = fields.sine_product(m.coords)
    h = 1.0 / n
    lam = 4 - 4 * math.cos(math.pi * h) if dim == 2 else h * (6 - 6 * math.cos(math.pi * h))
    As = A.matvec(s)
    free = m.dirichlet == 0
    np.testing.assert_allclose(As[free], lam * s[free], atol=1e-13)


def test_mass_integrates_domain_and_patch_test():
    for dim, n in ((2, 7), (3, 4)):
        m = smesh.structured_mesh(dim, n, jitter=0.2, seed=5)
        M = oracle.assemble(dim, m.coords, m.elems, np.ones(m.n_elems), 1.0, 0.0).to_scipy()
        assert abs(M.sum() - 1.0) < 1e-13
        # patch test with a variable coefficient: linear fields are
        # K-harmonic at interior nodes (P1 reproduces linears exactly)
        c = 1.0 / fields.rho_uniform(5, m.n_elems)
        K = oracle.assemble(dim, m.coords, m.elems, np.ones(m.n_elems), 0.0, 1.0).to_scipy()
        g = np.arange(1, dim + 1) * 0.7
        lin = m.coords @ g
        free = m.dirichlet == 0
        assert np.abs((K @ lin)[free]).max() < 1e-12
        # with a variable coefficient only the constant is in the kernel
        Kc = oracle.assemble(dim, m.coords, m.elems, c, 0.0, 1.0).to_scipy()
        assert np.abs(Kc @ np.ones(m.n_nodes)).max() < 1e-12


def _numpy_element_sum(dim, coords, elems, coef, alpha, beta, dirichlet, x):
    """Brute force: y = A_D x from element matrices written out with NumPy
    (gradients of the barycentric coordinates from numpy.linalg.inv of the
    edge matrix, |T| from numpy.linalg.det), scattered with numpy.add.at,
    then the Dirichlet rows and columns eliminated.  No oracle code."""
    X = coords[elems]                                    # [E, d+1, d]
    J = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))   # columns e_k
    vol = np.abs(np.linalg.det(J)) / math.factorial(dim)
    Gi = np.linalg.inv(J)                                # rows: grad(phi_k), k = 1..d
    G = np.concatenate([-Gi.sum(axis=1, keepdims=True), Gi], axis=1)   # [E, d+1, d]
    K = np.einsum("eak,ebk->eab", G, G) * (beta * coef * vol)[:, None, None]
    Mm = (np.ones((dim + 1, dim + 1)) + np.eye(dim + 1)) / ((dim + 1) * (dim + 2))
    Ae = K + alpha * vol[:, None, None] * Mm[None]
    free = dirichlet == 0
    xf = np.where(free, x, 0.0)
    contrib = np.einsum("eab,eb->ea", Ae, xf[elems])
    y = np.zeros(coords.shape[0])
    np.add.at(y, elems.ravel(), contrib.ravel())
    return np.where(free, y, x)


@pytest.mark.parametrize("dim,n,seed", [(2, 11, 3), (3, 5, 4)])
def test_apply_elements_pinned(dim, n, seed):
    """oracle.apply_elements, both the whole-vector and the rows= branch,
    against (1) the oracle's assembled operator and (2) a NumPy element sum
    written out here: jittered mesh, lognormal coefficient, alpha and beta
    both nonzero, Dirichlet nodes on the boundary and inside, elements in a
    shuffled order with some of them negatively oriented, and a random x
    (so a wrong local index, a kept Dirichlet column or a dropped mass or
    stiffness term changes the result)."""
    m = smesh.structured_mesh(dim, n, jitter=0.2, seed=seed)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(m.n_elems)
    elems = m.elems[perm].copy()
    flip = rng.random(m.n_elems) < 0.3
    elems[flip, 1], elems[flip, 2] = m.elems[perm][flip, 2], m.elems[perm][flip, 1]
    coef = 1.0 / fields.rho_lognormal(seed, m.n_elems)
    alpha, beta = 0.37, 1.9
    dirichlet = m.dirichlet.copy()
    inner = np.nonzero(dirichlet == 0)[0]
    dirichlet[rng.choice(inner, 3, replace=False)] = 1
    x = rng.normal(size=m.n_nodes)
    y = oracle.apply_elements(dim, m.coords, elems, coef, alpha, beta, dirichlet, x)
    A = oracle.assemble(dim, m.coords, m.elems[perm], coef, alpha, beta, dirichlet)
    bound = np.abs(A.to_scipy()) @ np.abs(x)
    assert np.all(np.abs(y - A.matvec(x)) <= 1e-14 * bound)
    yn = _numpy_element_sum(dim, m.coords, elems, coef, alpha, beta, dirichlet, x)
    assert np.all(np.abs(y - yn) <= 1e-13 * bound)
    # Dirichlet rows are the identity; free rows see no Dirichlet column
    d = dirichlet == 1
    assert np.array_equal(y[d], x[d])
    x2 = x.copy()
    x2[d] += 5.0
    y2 = oracle.apply_elements(dim, m.coords, elems, coef, alpha, beta, dirichlet, x2)
    assert np.array_equal(y2[~d], y[~d])
    # the rows= branch: random free and Dirichlet rows, repeats and the ends
    rows = np.concatenate([rng.choice(m.n_nodes, 40), np.nonzero(d)[0][:4], [0, m.n_nodes - 1, 5, 5]])
    yr = oracle.apply_elements(dim, m.coords, elems, coef, alpha, beta, dirichlet, x, rows=rows)
    assert np.all(np.abs(yr - yn[rows]) <= 1e-13 * bound[rows])
    yall = oracle.apply_elements(dim, m.coords, elems, coef, alpha, beta, dirichlet, x,
                                 rows=np.arange(m.n_nodes))
    assert np.all(np.abs(yall - y) <= 1e-14 * bound)
    # without Dirichlet nodes (the unmerged periodic use): the plain A x
    yo = oracle.apply_elements(dim, m.coords, elems, coef, alpha, beta, None, x)
    zero = np.zeros(m.n_nodes, dtype=np.uint8)
    yno = _numpy_element_sum(dim, m.coords, elems, coef, alpha, beta, zero, x)
    b0 = np.abs(oracle.assemble(dim, m.coords, m.elems[perm], coef, alpha, beta).to_scipy()) @ np.abs(x)
    assert np.all(np.abs(yo - yno) <= 1e-13 * b0)
    yor = oracle.apply_elements(dim, m.coords, elems, coef, alpha, beta, None, x, rows=rows)
    assert np.all(np.abs(yor - yno[rows]) <= 1e-13 * b0[rows])


@pytest.mark.parametrize("dim,n", [(2, 5), (3, 3)])
def test_spd_and_symmetric(dim, n):
    m = smesh.structured_mesh(dim, n, jitter=0.2, seed=9)
    c = 1.0 / fields.rho_lognormal(9, m.n_elems)
    for alpha in (0.0, 1e-3, 10.0):
        A = oracle.assemble(dim, m.coords, m.elems, c, alpha, 1.0, m.dirichlet).dense()
        assert np.array_equal(A, A.T)
        ev = np.linalg.eigvalsh(A)
        assert ev.min() > 0
        # Gershgorin: every eigenvalue within the union of the discs
        radius = np.abs(A).sum(1) - np.abs(np.diag(A))
        assert ev.max() <= (np.diag(A) + radius).max() * (1 + 1e-12)
    # without Dirichlet nodes and alpha = 0 the operator is singular
    A0 = oracle.assemble(dim, m.coords, m.elems, c, 0.0, 1.0).dense()
    assert abs(np.linalg.eigvalsh(A0).min()) < 1e-10


# ------------------------------------------------------------------ solve
@pytest.mark.parametrize("dim,n", [(2, 10), (3, 5)])
def test_cg_matches_dense_cholesky(dim, n):
    m = smesh.structured_mesh(dim, n, jitter=0.2, seed=13)
    c = 1.0 / fields.rho_uniform(13, m.n_elems)
    A = oracle.assemble(dim, m.coords, m.elems, c, 1e-2, 1.0, m.dirichlet)
    rng = np.random.default_rng(1)
    b = rng.normal(size=m.n_nodes)
    x, st, it, hist, tr = oracle.cg(A, b, rtol=1e-14, max_iter=5000, dirichlet=m.dirichlet)
    assert st == 0 and tr <= 1e-14
    Ad = A.dense()
    L = np.linalg.cholesky(Ad)
    xc = np.linalg.solve(L.T, np.linalg.solve(L, b))
    assert np.linalg.norm(x - xc) / np.linalg.norm(xc) <= 1e-12
    # history is the recursive residual, starting at ||b - A x0|| / ||b||
    assert hist.shape[0] == it + 1 and hist[-1] <= 1e-14
    # Dirichlet values imposed exactly
    np.testing.assert_array_equal(x[m.dirichlet == 1], b[m.dirichlet == 1])


def test_cg_finite_termination_tiny():
    """On a tiny well-conditioned system CG terminates in at most N_f steps."""
    m = smesh.structured_mesh(2, 4, jitter=0.2, seed=2)
    A = oracle.assemble(2, m.coords, m.elems, np.ones(m.n_elems), 10.0, 1.0, m.dirichlet)
    b = fields.sine_product(m.coords) + 0.1
    b[m.dirichlet == 1] = 0.0
    x, st, it, hist, tr = oracle.cg(A, b, rtol=1e-13, max_iter=1000, dirichlet=m.dirichlet)
    assert st == 0
    assert it <= int((m.dirichlet == 0).sum())


def test_cg_edge_cases():
    m = smesh.structured_mesh(2, 4)
    A = oracle.assemble(2, m.coords, m.elems, np.ones(m.n_elems), 1.0, 1.0, m.dirichlet)
    x, st, it, hist, tr = oracle.cg(A, np.zeros(m.n_nodes), rtol=1e-10)
    assert st == 0 and it == 0 and np.all(x == 0)
    b = np.ones(m.n_nodes)
    x, st, it, hist, tr = oracle.cg(A, b, rtol=1e-12, max_iter=2, dirichlet=m.dirichlet)
    assert st == 1 and it == 2 and hist.shape[0] == 3
    # warm start at the solution: no iterations
    xs, st, it, _, _ = oracle.cg(A, b, rtol=1e-12, dirichlet=m.dirichlet)
    _, st2, it2, _, _ = oracle.cg(A, b, x0=xs, rtol=1e-10, dirichlet=m.dirichlet)
    assert st2 == 0 and it2 == 0
    # an indefinite operator (negative coefficient) is reported as breakdown
    An = oracle.assemble(2, m.coords, m.elems, -np.ones(m.n_elems), 0.0, 1.0, m.dirichlet)
    _, st3, _, _, _ = oracle.cg(An, b, rtol=1e-10, dirichlet=m.dirichlet)
    assert st3 == oracle.EBREAKDOWN


def test_pure_mass_solve_returns_source():
    """beta = 0: the system is alpha M x = M f, so x = f / alpha."""
    prob = workloads.tgv2d(16)
    m = prob.mesh
    f = fields.sine_product(m.coords) * 3.0
    b = oracle.mass_rhs(prob, f)
    A = oracle.assemble(2, m.coords, m.elems, np.ones(m.n_elems), 1.0, 0.0, m.dirichlet)
    x, st, *_ = oracle.cg(A, b, rtol=1e-14, max_iter=2000, dirichlet=m.dirichlet)
    assert st == 0
    np.testing.assert_allclose(x, f, atol=1e-12)


def _l2_error(prob, x):
    m = prob.mesh
    M = oracle.assemble(m.dim, m.coords, m.elems, np.ones(m.n_elems), 1.0, 0.0).to_scipy()
    e = x - fields.sine_product(m.coords)
    return math.sqrt(e @ (M @ e))


def test_second_order_l2_convergence():
    """Manufactured p = sin(pi x) sin(pi y) of the 2D workload (w = 1e-2,
    jitter 0.2h): the P1 solution converges at the textbook O(h^2) rate."""
    errs = []
    ns = (8, 16, 32, 64)
    for n in ns:
        prob = workloads.tgv2d(n)
        m = prob.mesh
        b = oracle.mass_rhs(prob, prob.extra["source"])
        A = oracle.assemble_problem(prob)
        x, st, it, _, _ = oracle.cg(A, b, rtol=1e-12, max_iter=5000, dirichlet=m.dirichlet)
        assert st == 0
        errs.append(_l2_error(prob, x))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(r > 1.85 for r in rates[1:]), rates
    assert all(r < 2.3 for r in rates), rates


def test_mixed_reaches_fp64_residual():
    prob = workloads.cube(10, w=1e-4, jitter=0.2, rho="lognormal")
    m = prob.mesh
    A = oracle.assemble_problem(prob)
    b = A.matvec(prob.extra["xstar"])
    x, st, outer, inner, tr = oracle.cg_mixed(A, b, rtol=1e-10, dirichlet=m.dirichlet)
    assert st == 0 and tr <= 1e-10 and outer >= 2
    x64, st64, it64, _, _ = oracle.cg(A, b, rtol=1e-10, dirichlet=m.dirichlet)
    assert np.linalg.norm(x - x64) / np.linalg.norm(x64) < 1e-8


# ----------------------------------------------------------------- layout
def test_morton_small_lattice():
    m = smesh.structured_mesh(2, 1)   # 2 x 2 lattice
    lay = oracle.layout(2, m.coords, m.elems, m.lattice)
    order = [tuple(m.lattice[i]) for i in lay["node_new2old"]]
    assert order == [(0, 0), (1, 0), (0, 1), (1, 1)]
    m3 = smesh.structured_mesh(3, 1)
    lay3 = oracle.layout(3, m3.coords, m3.elems, m3.lattice)
    order3 = [tuple(m3.lattice[i]) for i in lay3["node_new2old"]]
    assert order3 == [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0),
                      (0, 0, 1), (1, 0, 1), (0, 1, 1), (1, 1, 1)]


@pytest.mark.parametrize("dim,n", [(2, 13), (3, 6)])
def test_layout_invariants(dim, n):
    m = smesh.structured_mesh(dim, n, jitter=0.2, seed=4)
    st, el = oracle.orient(dim, m.coords, m.elems)
    assert st == 0
    lay = oracle.layout(dim, m.coords, el, m.lattice)
    p = lay["node_new2old"]
    assert np.array_equal(np.sort(p), np.arange(m.n_nodes))
    assert np.array_equal(np.sort(lay["elem_new2old"]), np.arange(m.n_elems))
    # aligned 2^k blocks of the lattice are contiguous in the new order
    lat = m.lattice[p]
    blk = lat // 2
    key = np.zeros(m.n_nodes, dtype=np.int64)
    for ax in range(dim):
        key = key * 1000 + blk[:, ax]
    # nodes of one 2x2(x2) block appear consecutively
    changes = np.count_nonzero(key[1:] != key[:-1])
    assert changes == np.unique(key).size - 1
    # elements ordered by smallest new vertex
    mins = lay["elems_new"].min(axis=1)
    assert np.all(np.diff(mins) >= 0)
    # node-to-element lists: degrees and entries
    off, ent = lay["n2e_off"], lay["n2e_ent"]
    assert off[-1] == (dim + 1) * m.n_elems
    for i in range(0, m.n_nodes, 7):
        es = ent[off[i]:off[i + 1]]
        assert np.all(np.diff(es >> 2) > 0)
        for v in es:
            assert lay["elems_new"][v >> 2, v & 3] == i
    # the element map agrees with the old connectivity
    inv = np.empty_like(p)
    inv[p] = np.arange(m.n_nodes)
    np.testing.assert_array_equal(lay["elems_new"], inv[el[lay["elem_new2old"]]])


def test_orientation_repair_and_errors():
    m = smesh.structured_mesh(3, 3, jitter=0.2, seed=8)
    el = m.elems.copy()
    flip = np.arange(0, m.n_elems, 3)
    el[flip, 1], el[flip, 2] = m.elems[flip, 2], m.elems[flip, 1]
    st, fixed = oracle.orient(3, m.coords, el)
    assert st == 0 and np.array_equal(fixed, m.elems)
    bad = m.elems.copy()
    bad[5, 2] = bad[5, 1]                     # repeated vertex: zero volume
    assert oracle.orient(3, m.coords, bad)[0] == oracle.EDEGENERATE
    bad = m.elems.copy()
    bad[0, 0] = m.n_nodes
    assert oracle.orient(3, m.coords, bad)[0] == oracle.EINVAL


# ---------------------------------------------------------------- V_0 (Sec. 3.4)

def test_lumped_mass_weights_pins():
    """m_i = int phi_i: the weights sum to |Omega| = 1 on the unit square and
    cube, and equal the row sums of the consistent mass matrix."""
    for dim, n in ((2, 7), (3, 4)):
        m = smesh.structured_mesh(dim, n, jitter=0.2, seed=5)
        mw = oracle.lumped_mass(dim, m.coords, m.elems)
        assert abs(mw.sum() - 1.0) < 1e-13
        M = oracle.assemble(dim, m.coords, m.elems, np.ones(m.n_elems), 1.0, 0.0, None)
        assert np.max(np.abs(M.matvec(np.ones(m.n_nodes)) - mw)) < 1e-15


def test_v0_solution_pins():
    """The weak problem in V_0 with no mass term and no Dirichlet node: the
    bordered solution is mean-zero (int p_h = 0), solves A p = b - lam m with
    lam = sum b / |Omega|, and converges at second order in L2 to
    p = cos(pi x) cos(pi y), the Neumann solution of -Laplace p = 2 pi^2 p."""
    errs = []
    for n in (8, 16, 32):
        prob = workloads.neumann_square(n)
        m = prob.mesh
        mw = oracle.lumped_mass(2, m.coords, m.elems)
        K = oracle.assemble_problem(prob)
        b = oracle.mass_rhs(prob, prob.extra["source"])
        p = oracle.solve_v0(K, b, mw)
        assert abs(mw @ p) < 1e-14
        lam = b.sum() / mw.sum()
        assert np.max(np.abs(K.matvec(p) - (b - lam * mw))) < 1e-11 * np.max(np.abs(b))
        M = oracle.assemble(2, m.coords, m.elems, np.ones(m.n_elems), 1.0, 0.0, None)
        e = p - prob.extra["exact"]
        errs.append(np.sqrt(e @ M.matvec(e)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.85) and np.all(rates < 2.15), rates


# ---------------------------------------------------------------- periodic
def test_periodic_merge_fourier_eigenpairs():
    """Uniform fully periodic meshes (no jitter): the merged operator is
    circulant, so cos(2 pi (k.i)/n) over the lattice is an exact eigenvector.
    Closed-form symbols with theta = 2 pi k / n: the two-triangle stiffness
    is the 5-point stencil, 4 sin^2(theta_x/2) + 4 sin^2(theta_y/2), and its
    consistent mass h^2/12 (6 + 2 cos theta_x + 2 cos theta_y +
    2 cos(theta_x + theta_y)) (neighbours +-x, +-y, +-(1,1)); the Kuhn
    stiffness is h times the 7-point stencil.  A wrong merge or a missed
    image breaks the circulant structure at the seam."""
    n, alpha = 6, 0.7
    m = smesh.periodic_mesh(2, n, (0, 1))
    A = oracle.assemble_periodic(m, np.ones(m.n_elems), alpha, 1.0)
    h = 1.0 / n
    for k in ((1, 0), (1, 2), (3, 3), (2, 5)):
        th = 2.0 * np.pi * np.array(k) / n
        v = np.cos(m.lattice @ th)
        lam = (4 * np.sin(th[0] / 2) ** 2 + 4 * np.sin(th[1] / 2) ** 2
               + alpha * h * h / 12 * (6 + 2 * np.cos(th[0]) + 2 * np.cos(th[1]) + 2 * np.cos(th[0] + th[1])))
        assert np.max(np.abs(A.matvec(v) - lam * v)) < 1e-13, k
    n = 5
    m = smesh.periodic_mesh(3, n, (0, 1, 2))
    A = oracle.assemble_periodic(m, np.ones(m.n_elems), 0.0, 1.0)
    for k in ((1, 0, 0), (1, 2, 3), (4, 4, 1)):
        th = 2.0 * np.pi * np.array(k) / n
        v = np.cos(m.lattice @ th)
        lam = (1.0 / n) * np.sum(4 * np.sin(th / 2) ** 2)
        assert np.max(np.abs(A.matvec(v) - lam * v)) < 1e-13, k


def test_periodic_merge_counts_and_invariants():
    """Merging removes one node per image: n^d nodes when fully periodic,
    n (n+1) for the 2D channel; the elements are unchanged.  The stiffness
    part annihilates constants, the merged mass sums to |Omega| = 1 and the
    merged lumped weights equal the mass row sums."""
    for dim, n, axes, nodes in ((2, 5, (0, 1), 25), (2, 5, (0,), 30), (3, 4, (0, 1, 2), 64), (3, 4, (2,), 100)):
        m = smesh.periodic_mesh(dim, n, axes, jitter=0.2, seed=3)
        assert m.n_nodes == nodes and m.n_elems == (2 * n * n if dim == 2 else 6 * n ** 3)
        c = 1.0 / fields.rho_uniform(3, m.n_elems)
        K = oracle.assemble_periodic(m, c, 0.0, 1.0)
        free = m.dirichlet == 0
        one = free.astype(np.float64)
        if not m.dirichlet.any():
            assert np.max(np.abs(K.matvec(one))) < 1e-12
        M = oracle.assemble_periodic(m, np.ones(m.n_elems), 1.0, 0.0)
        if not m.dirichlet.any():
            assert abs(M.to_scipy().sum() - 1.0) < 1e-13
            mw = oracle.lumped_mass_mesh(m)
            assert np.max(np.abs(M.matvec(np.ones(m.n_nodes)) - mw)) < 1e-15
        S = K.to_scipy()
        assert abs(S - S.T).max() < 1e-15


def test_periodic_second_order_convergence():
    """Fully periodic square (w p - Laplace p = f) and the channel periodic in
    x with Dirichlet walls: second-order L2 convergence (from 16 cells per
    axis, 8 per wavelength; w = 1, since with a small w the fully periodic
    operator's constant mode, eigenvalue w, amplifies the O(h^4) discrete
    mean of the jittered source into the error) to
    sin(2 pi x) sin(2 pi y) and sin(2 pi x) sin(pi y) on jittered meshes."""
    for make in (workloads.periodic_square, workloads.periodic_channel):
        errs = []
        for n in (16, 32, 64):
            prob = make(n, w=1.0)
            m = prob.mesh
            A = oracle.assemble_problem(prob)
            b = oracle.mass_rhs(prob, prob.extra["source"])
            x = oracle.cg(A, b, rtol=1e-13, max_iter=20000, dirichlet=m.dirichlet)[0]
            M = oracle.assemble_periodic(m, np.ones(m.n_elems), 1.0, 0.0)
            e = x - prob.extra["exact"]
            errs.append(np.sqrt(e @ M.matvec(e)))
        rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        assert np.all(rates > 1.8) and np.all(rates < 2.2), (make.__name__, rates)


def test_periodic_v0_poisson():
    """alpha = 0 on the fully periodic square: the V_0 solution of
    -Laplace p = 8 pi^2 sin(2 pi x) sin(2 pi y) has zero mean and converges
    at second order to sin(2 pi x) sin(2 pi y)."""
    errs = []
    for n in (12, 24, 48):
        prob = workloads.periodic_square(n, w=0.0)
        m = prob.mesh
        A = oracle.assemble_problem(prob)
        mw = oracle.lumped_mass_mesh(m)
        b = oracle.mass_rhs(prob, prob.extra["source"])
        p = oracle.solve_v0(A, b, mw)
        assert abs(mw @ p) < 1e-14
        M = oracle.assemble_periodic(m, np.ones(m.n_elems), 1.0, 0.0)
        e = p - prob.extra["exact"]
        errs.append(np.sqrt(e @ M.matvec(e)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8) and np.all(rates < 2.2), rates


# ------------------------------------------------------------- lumped mass
def test_lumped_operator_fourier_and_row_sums():
    """The lumped operator alpha diag(m) + K: on uniform fully periodic
    meshes every node carries m_i = h^d (six triangles of h^2/2 over 3 nodes;
    24 Kuhn tetrahedra of h^3/6 over 4), so cos 2 pi (k.i)/n is an eigenvector
    with eigenvalue (5-point or h times 7-point symbol) + alpha h^d; the
    lumped matrix is diagonal with the consistent mass row sums."""
    alpha = 0.9
    for dim, n in ((2, 6), (3, 5)):
        m = smesh.periodic_mesh(dim, n, tuple(range(dim)))
        A = oracle.assemble_lumped(m, np.ones(m.n_elems), alpha, 1.0)
        h = 1.0 / n
        for k in ((1, 0, 2), (2, 3, 1), (3, 3, 3)):
            th = 2.0 * np.pi * np.array(k[:dim]) / n
            v = np.cos(m.lattice @ th)
            lam = h ** (dim - 2) * np.sum(4 * np.sin(th / 2) ** 2) + alpha * h ** dim
            assert np.max(np.abs(A.matvec(v) - lam * v)) < 1e-13, (dim, k)
    m = smesh.structured_mesh(3, 4, jitter=0.2, seed=9)
    ML = oracle.assemble_lumped(m, np.ones(m.n_elems), 1.0, 0.0).to_scipy()
    M = oracle.assemble(3, m.coords, m.elems, np.ones(m.n_elems), 1.0, 0.0, m.dirichlet).to_scipy()
    free = m.dirichlet == 0
    assert abs(ML - __import__("scipy.sparse").sparse.diags(ML.diagonal())).max() == 0.0
    full = oracle.assemble(3, m.coords, m.elems, np.ones(m.n_elems), 1.0, 0.0, None).to_scipy()
    np.testing.assert_allclose(ML.diagonal()[free], np.asarray(full.sum(axis=1)).ravel()[free], rtol=1e-14)
    assert np.all(ML.diagonal()[~free] == 1.0) and np.all(M.diagonal()[~free] == 1.0)


def test_lumped_second_order_convergence():
    """Mass lumping keeps P1 second order: w p - Laplace p = f on the
    jittered square with Dirichlet boundary (w = 1) and on the periodic
    square, to sin(pi x) sin(pi y) and sin(2 pi x) sin(2 pi y)."""
    cases = ((lambda n: workloads.tgv2d(n, w=1.0), (16, 32, 64), "exact_tgv"),
             (lambda n: workloads.periodic_square(n, w=1.0), (16, 32, 64), "exact"))
    for make, ns, key in cases:
        errs = []
        for n in ns:
            prob = workloads.lumped(make(n))
            m = prob.mesh
            A = oracle.assemble_problem(prob)
            b = oracle.mass_rhs(prob, prob.extra["source"])
            x = oracle.cg(A, b, rtol=1e-13, max_iter=20000, dirichlet=m.dirichlet)[0]
            exact = (prob.extra["exact"] if key == "exact"
                     else np.sin(np.pi * m.coords[:, 0]) * np.sin(np.pi * m.coords[:, 1]))
            M = (oracle.assemble_periodic(m, np.ones(m.n_elems), 1.0, 0.0) if m.period is not None
                 else oracle.assemble(2, m.coords, m.elems, np.ones(m.n_elems), 1.0, 0.0, None))
            e = x - exact
            errs.append(np.sqrt(e @ M.matvec(e)))
        rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        assert np.all(rates > 1.8) and np.all(rates < 2.2), (key, rates)


def test_threaded_cg_matches_sequential():
    """The all-core leg of the CPU baseline: the SpMV gives the same bits on
    4 threads, and the CG solution agrees with the sequential oracle's."""
    prob = workloads.cube(10, w=1e-3, jitter=0.2, rho="lognormal")
    m = prob.mesh
    A = oracle.assemble_problem(prob)
    b = A.matvec(fields.sine_product(m.coords))
    x1, st1, it1, _, tr1 = oracle.cg(A, b, rtol=1e-10, dirichlet=m.dirichlet)
    y1 = A.matvec(b)
    try:
        oracle.set_threads(4)
        y4 = A.matvec(b)
        x4, st4, it4, _, tr4 = oracle.cg(A, b, rtol=1e-10, dirichlet=m.dirichlet)
    finally:
        oracle.set_threads(1)
    assert np.array_equal(y1.view(np.uint64), y4.view(np.uint64))
    assert st1 == st4 == 0 and abs(it1 - it4) <= 1 and tr4 <= 1e-10
    assert np.linalg.norm(x4 - x1) <= 1e-10 * np.linalg.norm(x1)

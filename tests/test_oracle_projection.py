"""Pins of the projection-stage oracle (oracle/projection.py) against what
the paper and the mathematics fix, independent of the oracle's own
arithmetic:
  * dual-cell counts: Table 1's dual elements (3N^2 + 2N edges of the N x N
    two-triangle split), the Kuhn cube's 12 n^3 + 6 n^2 faces, and the
    periodic meshes (every face interior: 3 n^2 and 12 n^3);
  * the dual -> primal mean is exact at the element centroid for linear
    fields, and the basis gradients reproduce the gradient of a linear field;
  * a uniform state at rest, and a uniform flow on a periodic mesh, are
    steady (dP = 0, W unchanged);
  * global energy balance: the right-hand side sums to
    int(W_E - rho K) - alpha int P^n - dt sum_f bflux_f |f| on a mesh with no
    Dirichlet node (the advection term sums to zero by the partition of
    unity);
  * the discrete energy equation: after each Picard iteration the new
    element momenta satisfy, on every free row,
    alpha (M (P^n + dP))_i - sum_k (W_E - rho K)_k |T_k|/(d+1)
      - dt sum_k H_k W_k . grad(phi_i) |T_k| + boundary_i = 0,
    which ties the right-hand side, the solve and the momentum update
    together (a wrong sign or factor in any of them breaks it).
"""

import numpy as np
import pytest

import oracle
from oracle import projection as op
from synth import mesh as smesh
from synth import projection as sproj
from synth import workloads


def _golden_table1(golden_dir):
    rows = []
    import os
    for line in open(os.path.join(golden_dir, "table1_meshes.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([int(v) for v in line.split()[1:5]])
    return rows


def test_dual_cell_counts(golden_dir):
    for N, _tri, _ver, dual in _golden_table1(golden_dir)[:3]:
        m = smesh.structured_mesh(2, N)
        fv, fe, ef = op.dual_faces(2, m.elems)
        assert fv.shape[0] == dual == 3 * N * N + 2 * N
        assert (fe[:, 1] < 0).sum() == 4 * N
    for n in (2, 3, 5):
        m = smesh.structured_mesh(3, n)
        fv, fe, ef = op.dual_faces(3, m.elems)
        assert fv.shape[0] == 12 * n ** 3 + 6 * n * n and (fe[:, 1] < 0).sum() == 12 * n * n
        mp = smesh.periodic_mesh(3, n + 1, (0, 1, 2))
        fv, fe, ef = op.dual_faces(3, mp.elems)
        assert fv.shape[0] == 12 * (n + 1) ** 3 and (fe[:, 1] < 0).sum() == 0
    mp = smesh.periodic_mesh(2, 5, (0, 1))
    assert op.dual_faces(2, mp.elems)[0].shape[0] == 75
    # every element sees d+1 distinct faces, each face lists it
    m = smesh.structured_mesh(3, 3, jitter=0.2, seed=2)
    fv, fe, ef = op.dual_faces(3, m.elems)
    for k in range(m.n_elems):
        assert len(set(ef[k])) == 4
        for a, f in enumerate(ef[k]):
            assert k in fe[f]
            assert sorted(np.delete(m.elems[k], a)) == list(fv[f])


def test_linear_fields_are_exact():
    rng = np.random.default_rng(1)
    for dim, n in ((2, 6), (3, 4)):
        m = smesh.structured_mesh(dim, n, jitter=0.2, seed=4)
        fv, fe, ef = op.dual_faces(dim, m.elems)
        c = rng.normal(size=dim)
        cf = m.coords[fv].mean(axis=1) @ c                  # linear field at face centroids
        ck = m.coords[m.elems].mean(axis=1) @ c             # ... at element centroids
        assert np.max(np.abs(cf[ef].mean(axis=1) - ck)) < 1e-14
        vol, grad = op.element_geometry(m)
        gl = np.einsum("ka,kac->kc", (m.coords @ c)[m.elems], grad)
        assert np.max(np.abs(gl - c)) < 1e-12
        assert abs(vol.sum() - 1.0) < 1e-13


def _stage(m, inp, lumped=False, **kw):
    return op.projection_stage(m, inp["rho_f"], inp["we_f"], inp["wu_f"], inp["p"], kw.pop("gamma", 1.4),
                               kw.pop("dt", 0.02), lumped=lumped, **kw)


def test_rest_and_uniform_flow_are_steady():
    gamma = 1.4
    m = smesh.structured_mesh(2, 8, jitter=0.2, seed=3)
    fv, fe, ef = op.dual_faces(2, m.elems)
    F = fv.shape[0]
    rho = 1.0 + 0.2 * np.random.default_rng(0).random(F)
    inp = {"rho_f": rho, "wu_f": np.zeros((F, 2)), "p": np.full(m.n_nodes, 0.7)}
    inp["we_f"] = np.full(F, 0.7 / (gamma - 1.0))
    out = _stage(m, inp, rtol=1e-12)
    assert np.max(np.abs(out["p_new"] - 0.7)) < 1e-13 and np.max(np.abs(out["wu_new"])) < 1e-13
    mp = smesh.periodic_mesh(3, 5, (0, 1, 2), jitter=0.2, seed=3)
    fv, fe, ef = op.dual_faces(3, mp.elems)
    F = fv.shape[0]
    w0 = np.array([0.3, -0.1, 0.2])
    inp = {"rho_f": np.full(F, 1.3), "wu_f": np.tile(w0, (F, 1)), "p": np.full(mp.n_nodes, 0.7)}
    inp["we_f"] = np.full(F, 0.7 / (gamma - 1.0) + (w0 @ w0) / 2.6)
    for lumped in (False, True):
        out = _stage(mp, inp, lumped=lumped, rtol=1e-12)
        assert np.max(np.abs(out["p_new"] - 0.7)) < 1e-12
        assert np.max(np.abs(out["wu_new"] - w0)) < 1e-12


def test_global_energy_balance():
    prob = workloads.neumann_square(10)
    m = prob.mesh
    fv, fe, ef = op.dual_faces(2, m.elems)
    inp = sproj.fields(m, fv, fe, seed=5)
    gamma, dt = 1.4, 0.02
    out = _stage(m, inp, bflux=inp["bflux"], n_picard=1, rtol=1e-12, dt=dt)
    vol = out["vol"]
    area = op.face_areas(m, fe, ef)
    bnd = fe[:, 1] < 0
    assert abs(area[bnd].sum() - 4.0) < 1e-13
    mw = oracle.lumped_mass_mesh(m)
    want = (((out["we_k"] - out["rk_used"][0]) * vol).sum() - mw @ inp["p"] / (gamma - 1.0)
            - dt * (inp["bflux"][bnd] * area[bnd]).sum())
    assert abs(out["b"][0].sum() - want) < 1e-12 * np.abs(out["b"][0]).sum()


@pytest.mark.parametrize("case", ["square_dirichlet", "cube_lumped", "periodic_channel"])
def test_discrete_energy_equation_holds(case):
    gamma, dt = 1.4, 0.03
    if case == "square_dirichlet":
        m = workloads.tgv2d(10).mesh
        lumped = False
    elif case == "cube_lumped":
        m = smesh.structured_mesh(3, 4, jitter=0.2, seed=7)
        lumped = True
    else:
        m = smesh.periodic_mesh(2, 9, (0,), jitter=0.2, seed=7)
        lumped = False
    fv, fe, ef = op.dual_faces(m.dim, m.elems)
    inp = sproj.fields(m, fv, fe, seed=9)
    out = _stage(m, inp, lumped=lumped, pb=inp["pb"], bflux=inp["bflux"], n_picard=2, rtol=1e-13, dt=dt)
    alpha = 1.0 / (gamma - 1.0)
    M = op.operator_matrix(m, np.ones(m.n_elems), 1.0, 0.0, lumped=lumped, eliminate=False)
    vol, grad = out["vol"], out["grad"]
    el = np.asarray(m.elems, dtype=np.int64)
    area = op.face_areas(m, fe, ef)
    bnd = fe[:, 1] < 0
    free = m.dirichlet == 0
    for it in range(2):
        H, rk, dp, W = out["H_used"][it], out["rk_used"][it], out["dp"][it], out["w_elem"][it]
        r = alpha * (M @ (inp["p"] + dp))
        src = np.zeros(m.n_nodes)
        np.add.at(src, el, np.repeat(((out["we_k"] - rk) * vol / (m.dim + 1))[:, None], m.dim + 1, axis=1))
        flux = np.zeros(m.n_nodes)
        np.add.at(flux, el, dt * H[:, None] * np.einsum("kc,kac->ka", W, grad) * vol[:, None])
        bd = np.zeros(m.n_nodes)
        vals = dt * np.where(bnd, inp["bflux"], 0.0) * area / m.dim
        np.add.at(bd, fv[bnd].astype(np.int64), np.repeat(vals[bnd][:, None], m.dim, axis=1))
        res = (r - src - flux + bd)[free]
        scale = np.abs(r).max() + np.abs(src).max()
        assert np.max(np.abs(res)) < 1e-9 * scale, (case, it, np.max(np.abs(res)) / scale)
        # the Dirichlet values are imposed exactly
        assert np.max(np.abs((inp["p"] + dp - inp["pb"])[~free])) < 1e-15 if (~free).any() else True


def test_post_projection_conserves_and_keeps_uniform_states():
    """Sec. 3.5: on a periodic mesh every face's enthalpy flux cancels
    between its two elements, so sum |C_f| W_E^{n+1} = sum |C_f| tilde W_E;
    on a walled mesh the change is -dt times the flux through the primal
    boundary; a uniform state (uniform W_u, P and rho) is unchanged."""
    gamma, dt = 1.4, 0.02
    mp = smesh.periodic_mesh(3, 5, (0, 1, 2), jitter=0.2, seed=3)
    fv, fe, ef = faces = op.dual_faces(3, mp.elems)
    inp = sproj.fields(mp, fv, fe, seed=4)
    we_new, we_el, vol = op.post_projection(mp, inp["rho_f"], inp["we_f"], inp["wu_f"], inp["p"], gamma, dt, faces)
    cvol = np.zeros(fv.shape[0])
    np.add.at(cvol, ef, vol[:, None] * np.ones((1, 4)) / 4)
    assert abs(cvol @ we_new - cvol @ inp["we_f"]) < 1e-13 * (cvol @ inp["we_f"])
    assert abs(vol @ we_el - cvol @ inp["we_f"]) < 1e-13 * (cvol @ inp["we_f"])
    F = fv.shape[0]
    w0 = np.array([0.2, -0.1, 0.4])
    we_u, _, _ = op.post_projection(mp, np.full(F, 1.1), np.full(F, 3.0), np.tile(w0, (F, 1)),
                                    np.full(mp.n_nodes, 0.8), gamma, dt, faces)
    assert np.abs(we_u - 3.0).max() < 1e-13
    # walled square: the total changes by the boundary flux only
    m = smesh.structured_mesh(2, 6, jitter=0.2, seed=5)
    fv, fe, ef = faces = op.dual_faces(2, m.elems)
    inp = sproj.fields(m, fv, fe, seed=6)
    we_new, we_el, vol = op.post_projection(m, inp["rho_f"], inp["we_f"], inp["wu_f"], inp["p"], gamma, dt, faces)
    bnd = fe[:, 1] < 0
    area = op.face_areas(m, fe, ef)
    # outward unit normals of the boundary edges of the unit square
    c = m.coords[fv].mean(axis=1)
    nrm = np.zeros((fv.shape[0], 2))
    nrm[np.isclose(c[:, 0], 0.0), 0] = -1.0
    nrm[np.isclose(c[:, 0], 1.0), 0] = 1.0
    nrm[np.isclose(c[:, 1], 0.0), 1] = -1.0
    nrm[np.isclose(c[:, 1], 1.0), 1] = 1.0
    hf = gamma / (gamma - 1.0) * inp["p"][fv].mean(axis=1) / inp["rho_f"]
    bflux = (hf * (inp["wu_f"] * nrm).sum(axis=1) * area)[bnd].sum()
    cvol = np.zeros(fv.shape[0])
    np.add.at(cvol, ef, vol[:, None] * np.ones((1, 3)) / 3)
    assert abs((cvol @ we_new - cvol @ inp["we_f"]) + dt * bflux) < 1e-13 * (cvol @ inp["we_f"])


@pytest.mark.parametrize("dim,n", [(2, 7), (3, 4)])
def test_dual_face_count_and_checker(dim, n):
    """The oracle's dual cells of the structured meshes number 3n^2 + 2n (2D,
    Table 1's dual elements) and 12n^3 + 6n^2 (3D Kuhn cube: (4E + 12n^2)/2),
    and the definition checker used on the full-size mesh accepts the
    oracle's list and rejects it with two faces swapped, an element dropped
    or a wrong count."""
    from dualcheck import check_dual_faces
    m = smesh.structured_mesh(dim, n, jitter=0.2, seed=3)
    rank = op.morton_rank(m)
    fv, fe, _ = op.dual_faces(dim, m.elems, rank)
    want = 3 * n * n + 2 * n if dim == 2 else 12 * n ** 3 + 6 * n ** 2
    assert fv.shape[0] == want
    check_dual_faces(m.elems, fv, fe, rank, want)
    with pytest.raises(AssertionError):
        check_dual_faces(m.elems, fv, fe, rank, want + 1)
    sw = fv.copy(), fe.copy()
    for a in sw:
        a[[3, 4]] = a[[4, 3]]
    with pytest.raises(AssertionError):
        check_dual_faces(m.elems, sw[0], sw[1], rank, want)
    bad = fe.copy()
    k = np.nonzero(bad[:, 1] >= 0)[0][0]
    bad[k, 1] = -1
    with pytest.raises(AssertionError):
        check_dual_faces(m.elems, fv, bad, rank, want)

"""The first-order transport step on the GPU (pressure_transport; needs an
MI355X) against the CPU oracle (oracle/transport.py), and one whole time
step (transport, then the projection stage) against the oracle chain.

The oracle builds the dual faces from their geometric definition and the
pressure force from face means; the GPU uses the closed-form area vectors
and the element gradients.  Both are exact up to rounding, so the updates
agree to 1e-10 of the largest change (plus 1e-14 of the field), on walled
and periodic meshes, with gravity and artificial viscosity; mass is
conserved to rounding on a periodic mesh.
"""

import numpy as np
import pytest

from oracle import projection as op
from oracle import transport as ot
import paper_2301_08357_amd as pm
from synth import mesh as smesh
from synth import projection as sproj
from synth import workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _mesh(case):
    if case == "square_walls":
        return workloads.tgv2d(20).mesh
    if case == "cube_walls":
        return smesh.structured_mesh(3, 7, jitter=0.2, seed=3)
    if case == "channel":
        return smesh.periodic_mesh(2, 15, (0,), jitter=0.2, seed=5)
    if case == "one_square":                      # 2 triangles: every cell on the boundary but one
        return smesh.structured_mesh(2, 1, jitter=0.0, seed=1)
    if case == "one_cube":                        # 6 tets, every node a Dirichlet node
        return smesh.structured_mesh(3, 1, jitter=0.0, seed=1)
    return smesh.periodic_mesh(3, 7, (0, 1, 2), jitter=0.2, seed=6)


CASES = ["square_walls", "cube_walls", "channel", "periodic_cube", "one_square", "one_cube"]


def _system(m, gamma=1.4, dt=0.02):
    return pm.PressureSystem(m.dim, m.coords, m.elems, np.ones(m.n_elems), 1.0 / (gamma - 1.0), dt, m.dirichlet,
                             m.lattice, period=m.period)


def _close(a, b, a0):
    scale = np.abs(b - a0).max()
    return np.abs(a - b).max() <= 1e-10 * scale + 1e-14 * np.abs(a0).max()


@pytest.mark.parametrize("mu,lam", [(0.0, 0.0), (0.05, 0.0), (0.0, 0.08), (0.05, 0.08)])
@pytest.mark.parametrize("case", CASES)
def test_transport_matches_oracle(case, mu, lam):
    m = _mesh(case)
    print("case", case, "mu", mu, "lambda", lam, flush=True)
    fv, fe, ef = faces = op.dual_faces(m.dim, m.elems, op.morton_rank(m))
    inp = sproj.fields(m, fv, fe, seed=13)
    g = np.array([0.1, -0.8, 0.3])[: m.dim]
    dt = 0.2 / (m.n ** 1)
    ref = ot.transport_step(m, inp["rho_f"], inp["wu_f"], inp["we_f"], inp["p"], dt, gravity=g, c_alpha=0.4,
                           faces=faces, mu=mu, lam=lam, r_gas=0.4)
    s = _system(m)
    rho, wu, we = s.transport(_dev(inp["rho_f"]), _dev(inp["wu_f"]), _dev(inp["we_f"]), _dev(inp["p"]), dt,
                              gravity=g, c_alpha=0.4, mu=mu, lam=lam, r_gas=0.4)
    if mu > 0.0:
        assert np.abs(ref["visc"]).max() > 1e-3 * np.abs(ref["flux_sum"]).max()
    if lam > 0.0:
        assert np.abs(ref["heat"]).max() > 1e-3 * np.abs(ref["flux_sum"]).max()
    rho, wu, we = _host(rho), _host(wu).reshape(-1, m.dim), _host(we)
    assert _close(rho, ref["rho"], inp["rho_f"])
    assert _close(wu, ref["wu"], inp["wu_f"])
    assert _close(we, ref["we"], inp["we_f"])
    if m.period is not None and not m.dirichlet.any():
        vol = ref["vol"]
        assert abs(vol @ rho - vol @ inp["rho_f"]) < 1e-13 * (vol @ inp["rho_f"])
    s.close()


@pytest.mark.parametrize("visc", [False, True])
@pytest.mark.parametrize("case", CASES)
def test_lader_transport_matches_oracle(case, visc):
    """The second-order (LADER, Sec. 3.2.1) step against the oracle's: ENO
    choices, extrapolation, half-step evolution and the flux at the evolved
    states, with gravity, pressure and artificial viscosity (and, with
    visc, the first-order viscous and heat-flux terms)."""
    m = _mesh(case)
    mu, lam = (0.05, 0.08) if visc else (0.0, 0.0)
    print("case lader", case, "mu", mu, "lambda", lam, flush=True)
    fv, fe, ef = faces = op.dual_faces(m.dim, m.elems, op.morton_rank(m))
    inp = sproj.fields(m, fv, fe, seed=19)
    g = np.array([0.1, -0.8, 0.3])[: m.dim]
    dt = 0.2 / m.n
    ref = ot.transport_step(m, inp["rho_f"], inp["wu_f"], inp["we_f"], inp["p"], dt, gravity=g, c_alpha=0.4,
                           faces=faces, mu=mu, lam=lam, r_gas=0.4, lader=True)
    first = ot.transport_step(m, inp["rho_f"], inp["wu_f"], inp["we_f"], inp["p"], dt, gravity=g, c_alpha=0.4,
                             faces=faces, mu=mu, lam=lam, r_gas=0.4)
    s = _system(m)
    rho, wu, we = s.transport(_dev(inp["rho_f"]), _dev(inp["wu_f"]), _dev(inp["we_f"]), _dev(inp["p"]), dt,
                              gravity=g, c_alpha=0.4, mu=mu, lam=lam, r_gas=0.4, lader=True)
    rho, wu, we = _host(rho), _host(wu).reshape(-1, m.dim), _host(we)
    if m.n > 1:
        assert np.abs(ref["rho"] - first["rho"]).max() > 1e-3 * np.abs(first["rho"] - inp["rho_f"]).max()
    assert _close(rho, ref["rho"], inp["rho_f"])
    assert _close(wu, ref["wu"], inp["wu_f"])
    assert _close(we, ref["we"], inp["we_f"])
    if m.period is not None and not m.dirichlet.any():
        vol = ref["vol"]
        assert abs(vol @ rho - vol @ inp["rho_f"]) < 1e-13 * (vol @ inp["rho_f"])
    s.close()


def test_one_time_step_transport_then_projection():
    m = smesh.periodic_mesh(2, 16, (0,), jitter=0.2, seed=9)
    gamma, dt = 1.4, 0.01
    fv, fe, ef = faces = op.dual_faces(2, m.elems, op.morton_rank(m))
    inp = sproj.fields(m, fv, fe, seed=21)
    tr = ot.transport_step(m, inp["rho_f"], inp["wu_f"], inp["we_f"], inp["p"], dt, faces=faces)
    ref = op.projection_stage(m, tr["rho"], tr["we"], tr["wu"], inp["p"], gamma, dt, pb=inp["pb"],
                              n_picard=2, rtol=1e-12, faces=faces)
    s = _system(m, gamma, dt)
    rho, wu, we = s.transport(_dev(inp["rho_f"]), _dev(inp["wu_f"]), _dev(inp["we_f"]), _dev(inp["p"]), dt)
    p_new, wu_new, h_new, its, st = s.projection(rho, we, wu, _dev(inp["p"]), gamma, dt, pb=_dev(inp["pb"]),
                                                 n_picard=2, rtol=1e-12)
    assert st == 0
    dp = ref["p_new"] - inp["p"]
    assert np.linalg.norm(_host(p_new) - ref["p_new"]) <= 1e-9 * np.linalg.norm(dp)
    dw = ref["wu_new"] - inp["wu_f"]
    assert np.linalg.norm(_host(wu_new).reshape(-1, 2) - ref["wu_new"]) <= 1e-9 * np.linalg.norm(dw)
    s.close()


@pytest.mark.parametrize("case", ["square_walls", "periodic_cube", "one_cube"])
def test_post_projection_matches_oracle(case):
    m = _mesh(case)
    gamma, dt = 1.4, 0.02
    fv, fe, ef = faces = op.dual_faces(m.dim, m.elems, op.morton_rank(m))
    inp = sproj.fields(m, fv, fe, seed=17)
    ref, _, _ = op.post_projection(m, inp["rho_f"], inp["we_f"], inp["wu_f"], inp["p"], gamma, dt, faces)
    s = _system(m, gamma, dt)
    we = _host(s.post_projection(_dev(inp["rho_f"]), _dev(inp["we_f"]), _dev(inp["wu_f"]), _dev(inp["p"]), gamma, dt))
    assert _close(we, ref, inp["we_f"])
    s.close()


def _gpu_step(s, st, gamma, dt, pb=None, mu=0.0):
    rho, wu, we = s.transport(st["rho"], st["wu"], st["we"], st["p"], dt, mu=mu)
    p_new, wu_new, _, its, code = s.projection(rho, we, wu, st["p"], gamma, dt, pb=pb, n_picard=2, rtol=1e-12)
    assert code == 0
    we_new = s.post_projection(rho, we, wu_new, p_new, gamma, dt)
    return {"rho": rho, "wu": wu_new, "we": we_new, "p": p_new}


@pytest.mark.parametrize("mu", [0.0, 1e-3])
def test_three_time_steps_match_oracle_and_conserve(mu):
    """Three whole time steps (transport, projection with N_Pic = 2,
    post-projection) on a fully periodic square, inviscid and viscous: the
    GPU state matches the oracle chain, and mass, momentum and total energy
    are conserved (the periodic pressure gradient integrates to zero, the
    viscous exchanges cancel in pairs)."""
    gamma, dt = 1.4, 0.01
    m = smesh.periodic_mesh(2, 18, (0, 1), jitter=0.2, seed=23)
    fv, fe, ef = faces = op.dual_faces(2, m.elems, op.morton_rank(m))
    inp = sproj.fields(m, fv, fe, seed=29)
    ref = {"rho": inp["rho_f"], "wu": inp["wu_f"], "we": inp["we_f"], "p": inp["p"]}
    s = _system(m, gamma, dt)
    st = {k: _dev(v) for k, v in ref.items()}
    vol, _ = op.element_geometry(m)
    cvol = np.zeros(fv.shape[0])
    np.add.at(cvol, ef, vol[:, None] * np.ones((1, 3)) / 3)
    tot0 = (cvol @ inp["rho_f"], cvol @ inp["wu_f"], cvol @ inp["we_f"])
    for step in range(3):
        tr = ot.transport_step(m, ref["rho"], ref["wu"], ref["we"], ref["p"], dt, faces=faces, mu=mu)
        pr = op.projection_stage(m, tr["rho"], tr["we"], tr["wu"], ref["p"], gamma, dt, n_picard=2, rtol=1e-12,
                                 faces=faces)
        we_new, _, _ = op.post_projection(m, tr["rho"], tr["we"], pr["wu_new"], pr["p_new"], gamma, dt, faces)
        ref = {"rho": tr["rho"], "wu": pr["wu_new"], "we": we_new, "p": pr["p_new"]}
        st = _gpu_step(s, st, gamma, dt, mu=mu)
    got = {k: _host(v) for k, v in st.items()}
    got["wu"] = got["wu"].reshape(-1, 2)
    for k in ("rho", "we", "p"):
        assert np.linalg.norm(got[k] - ref[k]) <= 1e-9 * np.linalg.norm(ref[k] - (inp["p"] if k == "p" else
                                                                            inp[k + "_f"])), k
    assert np.linalg.norm(got["wu"] - ref["wu"]) <= 1e-9 * np.linalg.norm(ref["wu"] - inp["wu_f"])
    assert abs(cvol @ got["rho"] - tot0[0]) < 1e-13 * tot0[0]
    assert np.abs(cvol @ got["wu"] - tot0[1]).max() < 1e-13 * np.abs(cvol @ np.abs(inp["wu_f"])).max()
    assert abs(cvol @ got["we"] - tot0[2]) < 1e-13 * tot0[2]
    s.close()


@pytest.mark.parametrize("periodic", [True, False])
def test_full_size_uniform_states_are_kept(periodic):
    """160^3 (the bench meshes, 49M dual cells): a uniform flow on the fully
    periodic mesh, and a state at rest on the walled one, pass unchanged
    through transport, projection (N_Pic = 2) and post-projection: every
    flux difference, pressure gradient and enthalpy flux then vanishes."""
    n = 160
    if periodic:
        m = smesh.periodic_mesh(3, n, (0, 1, 2), jitter=0.2, seed=31)
        w0 = np.array([0.05, -0.03, 0.02])
    else:
        m = smesh.structured_mesh(3, n, jitter=0.2, seed=31)
        w0 = np.zeros(3)
    print("case full size uniform, periodic=%s" % periodic, flush=True)
    gamma, dt = 1.4, 2e-3
    s = _system(m, gamma, dt)
    F = s.dual_faces()[0].shape[0]
    rho0, p0 = 1.2, 0.7
    we0 = p0 / (gamma - 1.0) + (w0 @ w0) / (2.0 * rho0)
    st = {"rho": _dev(np.full(F, rho0)), "wu": _dev(np.tile(w0, F)), "we": _dev(np.full(F, we0)),
          "p": _dev(np.full(m.n_nodes, p0))}
    out = _gpu_step(s, st, gamma, dt)
    assert float((out["rho"] - rho0).abs().max()) < 1e-14
    assert float((out["wu"] - _dev(np.tile(w0, F))).abs().max()) < 1e-13
    assert float((out["we"] - we0).abs().max()) < 1e-12
    assert float((out["p"] - p0).abs().max()) < 1e-12
    s.close()


def test_transport_rejects_invalid_diffusion_parameters():
    """mu < 0, lambda < 0, or lambda > 0 without a positive gas constant are
    refused before any launch."""
    m = _mesh("square_walls")
    fv, fe, ef = op.dual_faces(m.dim, m.elems, op.morton_rank(m))
    inp = sproj.fields(m, fv, fe, seed=13)
    s = _system(m)
    args = (_dev(inp["rho_f"]), _dev(inp["wu_f"]), _dev(inp["we_f"]), _dev(inp["p"]), 0.01)
    for kw in ({"mu": -1.0}, {"lam": -0.1}, {"lam": 0.1, "r_gas": 0.0}, {"mu": float("nan")}):
        with pytest.raises(pm.PressureError):
            s.transport(*args, **kw)
    s.transport(*args, lam=0.0, r_gas=0.0)          # R is read only when lambda > 0
    s.close()


def _sub_faces(elems, fv, fe, cells, sub=None):
    """The elements of `cells` (face ids of the full mesh), or the element
    ids `sub`, as a sub-mesh for the oracle: (sub element ids, sub faces
    (fv, fe, ef) in a local numbering, full face id of each local face).  A
    first-order cell update depends only on its one or two elements, their
    faces' states and their vertex pressures, so on this sub-mesh the oracle
    gives the full mesh's update for every cell in `cells`; a LADER update
    also reads the gradients of the other elements of those faces, which
    the caller then adds to `sub`."""
    E = elems.shape[0]
    if sub is None:
        sub = np.unique(fe[cells].ravel())
        sub = sub[sub >= 0]
    pos = np.full(E + 1, -1, dtype=np.int64)           # pos[-1] stays -1 for "no element"
    pos[sub] = np.arange(sub.size)
    fe64 = fe.astype(np.int64)
    touch = (pos[fe64[:, 0]] >= 0) | (pos[fe64[:, 1]] >= 0)
    rows = np.nonzero(touch)[0]
    fe_sub = pos[fe64[rows]]
    ef_sub = np.full((sub.size, elems.shape[1]), -1, dtype=np.int64)
    for slot in (0, 1):
        r = np.nonzero(fe_sub[:, slot] >= 0)[0]
        kl = fe_sub[r, slot]
        verts = elems[sub[kl]]
        on = (verts[:, :, None] == fv[rows[r]][:, None, :]).any(axis=2)
        a = np.argmin(on, axis=1)                       # the vertex opposite the face
        ef_sub[kl, a] = r
    assert (ef_sub >= 0).all()
    return sub, (fv[rows], fe_sub, ef_sub), rows


def test_transport_and_post_projection_full_size_sampled_cells():
    """160^3 walled cube with the projection-stage input recipe (49M dual
    cells): one transport step with every term (Rusanov with c_alpha,
    pressure force, gravity, viscous stress, heat flux), then the
    post-projection of its output with a perturbed P^{n+1}; 4000 seeded
    random cells match the oracle, evaluated on the sub-mesh of their
    elements."""
    import types
    from synth.rng import MASTER_SEED
    n = 160
    m = smesh.structured_mesh(3, n, jitter=0.2, seed=MASTER_SEED)
    print("case full size sampled transport", flush=True)
    s = _system(m)
    fv, fe, _ = s.dual_faces()
    # the library's dual cells against the oracle's definition (every face
    # once, in the order of the sorted Morton-rank tuples, with its
    # elements), so the sampled cells below are the oracle's cells too
    from dualcheck import check_dual_faces
    check_dual_faces(m.elems, fv, fe, op.morton_rank(m), 12 * n ** 3 + 6 * n ** 2)
    inp = sproj.fields(m, fv, fe, gamma=1.4, mach=0.1)
    g = np.array([0.0, 0.0, -1.0])
    dt, mu, lam, R = 2e-4, 1e-3, 5e-3, 1.0
    rho, wu, we = s.transport(_dev(inp["rho_f"]), _dev(inp["wu_f"]), _dev(inp["we_f"]), _dev(inp["p"]), dt,
                              gravity=g, c_alpha=0.4, mu=mu, lam=lam, r_gas=R)
    p_new = inp["p"] * (1.0 + 1e-3 * np.cos(2.0 * np.pi * m.coords[:, 0]))
    we_post = _host(s.post_projection(rho, we, wu, _dev(p_new), 1.4, dt))
    rho, wu, we = _host(rho), _host(wu).reshape(-1, 3), _host(we)
    s.close()
    F = fv.shape[0]
    cells = np.sort(np.random.default_rng(MASTER_SEED).choice(F, 4000, replace=False))
    sub, faces, rows = _sub_faces(m.elems, fv, fe, cells)
    sm = types.SimpleNamespace(dim=3, coords=m.coords, elems=m.elems[sub], n_nodes=m.n_nodes, n_elems=sub.size,
                               period=None)
    ref = ot.transport_step(sm, inp["rho_f"][rows], inp["wu_f"][rows], inp["we_f"][rows], inp["p"], dt, gravity=g,
                            c_alpha=0.4, faces=faces, mu=mu, lam=lam, r_gas=R)
    loc = np.searchsorted(rows, cells)
    assert np.array_equal(rows[loc], cells)
    assert np.abs(ref["visc"][loc]).max() > 0 and np.abs(ref["heat"][loc]).max() > 0
    for got, want, a0 in ((rho, ref["rho"], inp["rho_f"]), (wu, ref["wu"], inp["wu_f"]), (we, ref["we"], inp["we_f"])):
        assert _close(got[cells], want[loc], a0[cells])
    # the post-projection of the GPU transport output on the same sub-mesh
    post, _, _ = op.post_projection(sm, rho[rows], we[rows], wu[rows], p_new, 1.4, dt, faces)
    assert _close(we_post[cells], post[loc], we[cells])


def test_handle_returns_its_device_memory():
    """Setup, the dual cells, a projection stage and a transport step (whose
    element records take 64 B per dual cell) and destroy, three times over:
    the device's free memory comes back each time."""
    m = smesh.structured_mesh(3, 40, jitter=0.2, seed=3)
    print("case handle memory, 40^3", flush=True)
    s = _system(m)
    fv, fe, _ = s.dual_faces()
    inp = sproj.fields(m, fv, fe, seed=13)
    args = [_dev(inp[k]) for k in ("rho_f", "wu_f", "we_f", "p")]
    outs = [torch.empty_like(args[0]), torch.empty_like(args[1]), torch.empty_like(args[2])]
    proj = [torch.empty_like(args[3]), torch.empty_like(args[1]), torch.empty(m.n_elems, dtype=torch.float64,
                                                                                device=DEV)]

    def cycle(system):
        system.transport(*args, 0.01, mu=1e-3, lam=1e-3, rho_out=outs[0], wu_out=outs[1], we_out=outs[2])
        system.projection(args[0], args[2], args[1], args[3], 1.4, 0.01, n_picard=1, rtol=1e-8, p_out=proj[0],
                          wu_out=proj[1], h_out=proj[2])
        torch.cuda.synchronize()
        system.close()

    cycle(s)
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        cycle(_system(m))
    free1 = torch.cuda.mem_get_info()[0]
    F = fv.shape[0]
    assert free0 - free1 < 16 * F, (free0 - free1, 64 * F)


def test_lader_full_size_sampled_cells():
    """160^3 walled cube with the projection-stage input recipe: one LADER
    step (c_alpha, gravity, P^n) on the GPU; 3000 sampled cells against the
    oracle on the sub-mesh of the elements that their updates read: their own
    elements and, for each face of those, the face's other element (the
    upwind element of the neighbour's ENO choice)."""
    import types
    from synth.rng import MASTER_SEED
    n = 160
    m = smesh.structured_mesh(3, n, jitter=0.2, seed=MASTER_SEED)
    print("case full size sampled LADER transport", flush=True)
    s = _system(m)
    fv, fe, _ = s.dual_faces()
    from dualcheck import check_dual_faces
    check_dual_faces(m.elems, fv, fe, op.morton_rank(m), 12 * n ** 3 + 6 * n ** 2)
    inp = sproj.fields(m, fv, fe, gamma=1.4, mach=0.1)
    g = np.array([0.0, 0.0, -1.0])
    dt = 2e-4
    rho, wu, we = s.transport(_dev(inp["rho_f"]), _dev(inp["wu_f"]), _dev(inp["we_f"]), _dev(inp["p"]), dt,
                              gravity=g, c_alpha=0.4, lader=True)
    rho, wu, we = _host(rho), _host(wu).reshape(-1, 3), _host(we)
    s.close()
    F = fv.shape[0]
    cells = np.sort(np.random.default_rng(MASTER_SEED + 1).choice(F, 3000, replace=False))
    # elements of the sampled cells, then the other element of each of their faces
    own = np.unique(fe[cells].ravel())
    own = own[own >= 0]
    E = m.n_elems
    # faces of the own elements: those whose element list holds one of them
    inown = np.zeros(E + 1, dtype=bool)
    inown[own] = True
    fe64 = fe.astype(np.int64)
    touch = inown[fe64[:, 0]] | inown[fe64[:, 1]]
    sub = np.unique(fe64[touch].ravel())
    sub = sub[sub >= 0]
    _, faces, rows = _sub_faces(m.elems, fv, fe, None, sub=sub)
    sm = types.SimpleNamespace(dim=3, coords=m.coords, elems=m.elems[sub], n_nodes=m.n_nodes, n_elems=sub.size,
                               period=None)
    ref = ot.transport_step(sm, inp["rho_f"][rows], inp["wu_f"][rows], inp["we_f"][rows], inp["p"], dt, gravity=g,
                            c_alpha=0.4, faces=faces, lader=True)
    loc = np.searchsorted(rows, cells)
    assert np.array_equal(rows[loc], cells)
    for got, want, a0 in ((rho, ref["rho"], inp["rho_f"]), (wu, ref["wu"], inp["wu_f"]), (we, ref["we"], inp["we_f"])):
        assert _close(got[cells], want[loc], a0[cells])

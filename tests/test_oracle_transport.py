"""Pins of the transport oracle (oracle/transport.py) against what the
mathematics fixes:
  * the dual cells are closed: the area vectors of a cell's dual faces plus
    its primal boundary faces sum to zero; the sub-cell (B_k, face) has
    volume |T_k|/(d+1) and the cells tile the domain;
  * a uniform state is preserved (free stream), on periodic and walled
    meshes with zero velocity;
  * mass, momentum and energy are conserved on a periodic mesh (the
    pressure force of a periodic P^n integrates to zero); gravity adds
    dt g sum |C| rho to the momentum;
  * with a uniform velocity the Rusanov mass flux is the upwind flux, so
    under the CFL condition the density keeps its bounds;
  * the pressure force of a linear pressure G.x is |C_i| G on every cell
    (the face-mean rule of eq. pressterm is exact for P1 pressures);
  * viscous terms: Crouzeix-Raviart gradients exact for linear velocities,
    the Galerkin form of the momentum term, conservation, and second-order
    weak convergence of the momentum and energy terms on a shear wave;
  * heat flux: the constant flux of a linear temperature and its closure
    on boundary cells, conservation, and second-order weak convergence on
    a sine temperature.
"""

import numpy as np
import pytest

from oracle import projection as op
from oracle import transport as ot
from synth import mesh as smesh
from synth import projection as sproj


def _state(m, seed=3):
    fv, fe, ef = op.dual_faces(m.dim, m.elems)
    inp = sproj.fields(m, fv, fe, seed=seed)
    return inp, fv, fe, ef


@pytest.mark.parametrize("dim,periodic", [(2, False), (2, True), (3, False), (3, True)])
def test_dual_cells_are_closed_and_tile_the_domain(dim, periodic):
    m = (smesh.periodic_mesh(dim, 5, tuple(range(dim)), jitter=0.2, seed=2) if periodic
         else smesh.structured_mesh(dim, 4, jitter=0.2, seed=2))
    fv, fe, ef = op.dual_faces(dim, m.elems)
    pairs, eta, subvol, bnd_eta = ot.dual_geometry(m)
    F = fv.shape[0]
    clo = np.zeros((F, dim))
    for q, (a, b) in enumerate(pairs):
        np.add.at(clo, ef[:, a], eta[:, q])
        np.add.at(clo, ef[:, b], -eta[:, q])
    bnd = fe[:, 1] < 0
    for a in range(dim + 1):
        on = bnd[ef[:, a]]
        np.add.at(clo, ef[on, a], bnd_eta[on, a])
    assert np.abs(clo).max() < 1e-15
    vol, _ = op.element_geometry(m)
    assert np.abs(subvol - vol[:, None] / (dim + 1)).max() < 1e-16
    assert abs(subvol.sum() - 1.0) < 1e-13


def test_free_stream_and_rest():
    for m in (smesh.periodic_mesh(3, 5, (0, 1, 2), jitter=0.2, seed=4), smesh.periodic_mesh(2, 7, (0, 1), jitter=0.2, seed=4)):
        fv, fe, ef = op.dual_faces(m.dim, m.elems)
        F = fv.shape[0]
        w0 = np.array([0.3, -0.2, 0.1])[: m.dim]
        out = ot.transport_step(m, np.full(F, 1.2), np.tile(w0, (F, 1)), np.full(F, 2.5), np.full(m.n_nodes, 0.7),
                                dt=0.01, c_alpha=0.5)
        assert np.abs(out["rho"] - 1.2).max() < 1e-14
        assert np.abs(out["wu"] - w0).max() < 1e-14
        assert np.abs(out["we"] - 2.5).max() < 1e-14
    m = smesh.structured_mesh(3, 4, jitter=0.2, seed=4)
    fv, fe, ef = op.dual_faces(3, m.elems)
    F = fv.shape[0]
    out = ot.transport_step(m, np.full(F, 1.2), np.zeros((F, 3)), np.full(F, 2.5), np.full(m.n_nodes, 0.7), dt=0.01)
    assert np.abs(out["wu"]).max() < 1e-14 and np.abs(out["rho"] - 1.2).max() < 1e-15


def test_conservation_on_a_periodic_mesh():
    m = smesh.periodic_mesh(3, 6, (0, 1, 2), jitter=0.2, seed=5)
    inp, fv, fe, ef = _state(m)
    g = np.array([0.0, 0.0, -0.5])
    out = ot.transport_step(m, inp["rho_f"], inp["wu_f"], inp["we_f"], inp["p"], dt=0.01, gravity=g, c_alpha=0.3)
    vol = out["vol"]
    assert abs(vol @ out["rho"] - vol @ inp["rho_f"]) < 1e-14 * (vol @ inp["rho_f"])
    dmom = vol @ out["wu"] - vol @ inp["wu_f"]
    assert np.abs(dmom - 0.01 * g * (vol @ inp["rho_f"])).max() < 1e-14
    dE = vol @ out["we"] - vol @ inp["we_f"]
    assert abs(dE - 0.01 * (vol @ (inp["wu_f"] @ g))) < 1e-14 * (vol @ inp["we_f"])


def test_upwind_flux_keeps_density_bounds():
    m = smesh.periodic_mesh(2, 16, (0, 1), jitter=0.2, seed=6)
    fv, fe, ef = op.dual_faces(2, m.elems)
    F = fv.shape[0]
    c = m.coords[fv].mean(axis=1)
    rho = 1.0 + 0.5 * (np.sin(2 * np.pi * c[:, 0]) > 0)                 # a density jump
    u0 = np.array([0.7, 0.4])
    h = 1.0 / 16
    dt = 0.1 * h / np.abs(u0).sum()
    out = ot.transport_step(m, rho, rho[:, None] * u0, np.ones(F), np.full(m.n_nodes, 0.7), dt=dt)
    assert out["rho"].min() >= 1.0 - 1e-14 and out["rho"].max() <= 1.5 + 1e-14
    # the flux is the upwind one: phi = (u.eta) rho_upwind
    pairs, eta, _, _ = ot.dual_geometry(m)
    e = eta[:, 0, :]
    fa, fb = ef[:, 0], ef[:, 1]
    phi = ot.rusanov_flux(rho[fa], rho[fa, None] * u0, rho[fb], rho[fb, None] * u0, e, 0.0)
    un = e @ u0
    up = np.where(un > 0, rho[fa], rho[fb])
    assert np.abs(phi[:, 0] - un * up).max() < 1e-15


def test_pressure_force_is_exact_for_linear_pressure():
    G = np.array([0.3, -1.1, 0.7])
    for dim in (2, 3):
        m = smesh.structured_mesh(dim, 5, jitter=0.2, seed=7)
        fv, fe, ef = op.dual_faces(dim, m.elems)
        F = fv.shape[0]
        out = ot.transport_step(m, np.ones(F), np.zeros((F, dim)), np.ones(F), m.coords @ G[:dim], dt=0.01)
        assert np.abs(out["pforce"] - out["vol"][:, None] * G[:dim]).max() < 1e-14


def _face_centroids(m, fe, ef):
    """Face centroids from the face's first element (unmerged coordinates on a
    periodic mesh, so that seam faces are placed correctly)."""
    g = m.unmerged if m.period is not None else m
    k = fe[:, 0].astype(np.int64)
    F = fe.shape[0]
    a = np.argmax(ef[k] == np.arange(F)[:, None], axis=1)
    x = g.coords[g.elems[k]]
    return (x.sum(axis=1) - x[np.arange(F), a]) / m.dim


def test_viscous_terms():
    """Viscous terms (Sec. 3.2, Galerkin/Crouzeix-Raviart gradients):
      * the CR gradient is exact for linear velocities;
      * a linear velocity gives a constant stress, whose integral over every
        interior cell's closed surface vanishes;
      * on a periodic mesh the viscous momentum and energy exchanges sum to
        zero;
      * the momentum term, integrated by the oracle over the geometric dual
        faces, equals the Galerkin form sum_k |T_k| tau_k grad psi_a with the
        Crouzeix-Raviart basis psi_a = 1 - d phi_a and
        tau_k = mu (G + G^T - 2/3 tr G I), G = sum_b u_b (x) grad psi_b;
      * tested against the shear wave itself, the term of u = (sin 2 pi y, 0)
        tends to -mu (2 pi)^2 at second order.  (Cell by cell it does not:
        with the lumped CR mass the cells of differently oriented edges see
        1.5, 0 and 1.5 times the Laplacian on the uniform mesh, the known
        weak-only consistency of the CR Laplacian.)
      * its energy term tends weakly to -div(tau u) = -mu 4 pi^2 cos 4 pi y
        (tau u = mu g g' e_y), tested against cos 4 pi y, also at second
        order."""
    G = np.array([[0.3, -0.7], [1.1, 0.2]])
    m = smesh.structured_mesh(2, 8, jitter=0.2, seed=3)
    fv, fe, ef = op.dual_faces(2, m.elems)
    c = m.coords[fv].mean(axis=1)
    assert np.abs(ot.cr_gradients(m, c @ G.T, ef) - G).max() < 1e-13
    F = fv.shape[0]
    out = ot.transport_step(m, np.ones(F), c @ G.T, np.ones(F), np.zeros(m.n_nodes), 0.01, mu=0.3)
    inner = fe[:, 1] >= 0
    assert np.abs(out["visc"][inner, :2]).max() < 1e-14
    mp = smesh.periodic_mesh(3, 5, (0, 1, 2), jitter=0.2, seed=4)
    inp, fv, fe, ef = _state(mp, seed=7)
    out = ot.transport_step(mp, inp["rho_f"], inp["wu_f"], inp["we_f"], inp["p"], 0.01, mu=0.05)
    assert np.abs(out["visc"].sum(axis=0)).max() < 1e-15
    assert np.abs(out["visc"]).max() > 1e-6
    ratios, ratios_e = [], []
    for n in (16, 32, 64):
        m = smesh.periodic_mesh(2, n, (0, 1), jitter=0.2, seed=5)
        fv, fe, ef = op.dual_faces(2, m.elems)
        F = fv.shape[0]
        c = _face_centroids(m, fe, ef)
        g = np.sin(2 * np.pi * c[:, 1])
        u = np.zeros((F, 2))
        u[:, 0] = g
        out = ot.transport_step(m, np.ones(F), u, np.ones(F), np.zeros(m.n_nodes), 0.01, mu=1.0)
        if n == 16:
            vol, grad = op.element_geometry(m)
            psi = -2.0 * grad                                           # grad psi_a = -d grad phi_a
            Gk = np.einsum("kac,kae->kce", u[ef], psi)
            tr = np.trace(Gk, axis1=1, axis2=2)
            tau = Gk + np.transpose(Gk, (0, 2, 1)) - (2.0 / 3.0) * tr[:, None, None] * np.eye(2)[None]
            want_m = np.zeros((F, 2))
            for a in range(3):
                np.add.at(want_m, ef[:, a], vol[:, None] * np.einsum("kce,ke->kc", tau, psi[:, a]))
            assert np.abs(out["visc"][:, :2] - want_m).max() < 1e-12 * np.abs(want_m).max()
        ratios.append((out["visc"][:, 0] @ g) / ((2 * np.pi) ** 2 * (out["vol"] * g) @ g))
        w = np.cos(4 * np.pi * c[:, 1])
        ratios_e.append((out["visc"][:, 2] @ w) / (-(4 * np.pi ** 2) * (out["vol"] * w) @ w))
    for rs in (ratios, ratios_e):
        err = np.abs(np.array(rs) - 1.0)
        r = np.log2(err[:-1] / err[1:])
        assert err[-1] < 1e-2 and np.all(r > 1.7), (rs, r)


def test_heat_flux():
    """Heat flux (eq. heatflux with Theta = P / (rho R), Sec. 3.2 heat flux
    term):
      * a linear temperature gives the constant Q = -lambda grad Theta: no
        exchange for interior cells, and a boundary cell's term is
        -Q . (its primal boundary area vector), by closure;
      * on a periodic mesh the exchanges sum to zero;
      * Theta = 2 + sin 2 pi x (rho = R = 1): the term tends weakly to
        |C| div Q = lambda (2 pi)^2 sin 2 pi x |C| at second order, with
        the sign that takes energy from hot cells to cold ones;
      * mass and momentum are untouched."""
    m = smesh.structured_mesh(3, 4, jitter=0.2, seed=9)
    fv, fe, ef = op.dual_faces(3, m.elems)
    F = fv.shape[0]
    G = np.array([0.4, -0.3, 0.9])
    rho, R, lam = 2.0, 0.7, 0.3
    P = 3.0 + m.coords @ G
    out = ot.transport_step(m, np.full(F, rho), np.zeros((F, 3)), np.ones(F), P, 0.01, lam=lam, r_gas=R)
    Q = -lam * G / (rho * R)
    assert np.abs(ot.heat_flux(m, np.full(F, rho), P, fv, ef, lam, R) - Q).max() < 1e-13
    inner = fe[:, 1] >= 0
    assert np.abs(out["heat"][inner]).max() < 1e-14
    _, _, _, bnd_eta = ot.dual_geometry(m)
    want = np.zeros(F)
    bnd = ~inner
    for a in range(4):
        on = bnd[ef[:, a]]
        np.add.at(want, ef[on, a], -(bnd_eta[on, a] @ Q))
    assert np.abs(out["heat"] - want).max() < 1e-14
    mp = smesh.periodic_mesh(3, 5, (0, 1, 2), jitter=0.2, seed=4)
    inp, fv, fe, ef = _state(mp, seed=8)
    base = ot.transport_step(mp, inp["rho_f"], inp["wu_f"], inp["we_f"], inp["p"], 0.01)
    out = ot.transport_step(mp, inp["rho_f"], inp["wu_f"], inp["we_f"], inp["p"], 0.01, lam=0.05, r_gas=1.0)
    assert abs(out["heat"].sum()) < 1e-15 * np.abs(out["heat"]).sum() + 1e-17
    assert np.abs(out["heat"]).max() > 1e-6
    assert np.array_equal(out["rho"], base["rho"]) and np.array_equal(out["wu"], base["wu"])
    ratios = []
    for n in (16, 32, 64):
        m = smesh.periodic_mesh(2, n, (0, 1), jitter=0.2, seed=5)
        fv, fe, ef = op.dual_faces(2, m.elems)
        F = fv.shape[0]
        c = _face_centroids(m, fe, ef)
        P = 2.0 + np.sin(2 * np.pi * m.coords[:, 0])
        out = ot.transport_step(m, np.ones(F), np.zeros((F, 2)), np.ones(F), P, 0.01, lam=0.7, r_gas=1.0)
        g = np.sin(2 * np.pi * c[:, 0])
        ratios.append((out["heat"] @ g) / (0.7 * (2 * np.pi) ** 2 * (out["vol"] * g) @ g))
    err = np.abs(np.array(ratios) - 1.0)
    r = np.log2(err[:-1] / err[1:])
    assert err[-1] < 1e-2 and np.all(r > 1.7), (ratios, r)

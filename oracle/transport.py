"""CPU oracle of the first-order transport step on the dual cells -- TEST
INFRASTRUCTURE (imported only by tests/, __graft_entry__.smoke() and the
CPU-baseline leg of bench.py).

Follows Sec. 3.2 of the paper (eq. discrf_mass, discrf_momentum,
discrf_energy with the modified Rusanov flux of eq. flux, the viscous
terms of eq. visc_mom / visc_toten and the heat flux), without the LADER
reconstruction:

  dual_geometry   the dual faces from their definition (Sec. 2): inside
                  element k the cells of primal faces a and b meet on the
                  simplex joining the barycenter B_k to the primal vertices
                  the two faces share; its area vector comes from that
                  simplex (segment normal in 2D, half cross product in 3D),
                  oriented from cell a (which holds vertex b) to cell b
                  (which holds vertex a); cell volumes are the volumes of
                  the sub-simplices (B_k, face).
  rusanov_flux    phi = (Z_i + Z_j)/2 - alpha_RS (Wr_j - Wr_i)/2 with
                  Z = (W_u.eta, W_u (U.eta), rho K (U.eta)),
                  Wr = (rho, W_u, rho K), alpha_RS = max|U.eta| + c_alpha|eta|.
  transport_step  the update; the pressure force is eq. pressterm, the sum
                  over the dual faces of the face-mean pressure times the
                  area vector, plus the primal boundary faces of boundary
                  cells (so that it is the integral of grad P over the cell);
                  boundary faces carry no convective flux; gravity sources.
  lader_states    the second-order (LADER) states of Sec. 3.2.1 at each dual
                  face: Step 1, the ENO choice per scalar conservative
                  variable between the Galerkin (Crouzeix-Raviart) gradient
                  of the centred element T_ij and that of the upwind element
                  (the other primal element of the cell; none for a boundary
                  cell), by the smaller |grad W . (N_ij - N_i)|; Step 2, the
                  extrapolation W_i + (N_ij - N_i) . grad W to the dual
                  face's barycentre N_ij (N_i the barycentre of the cell's
                  primal face); Step 3, the half-step evolution by the
                  Cauchy-Kovalevskaya form of the mass and momentum
                  equations written with those gradients (drho/dt =
                  -div W_u, dW_u/dt = -div(W_u (x) U) - grad P + rho g, grad P
                  the P1 gradient of P^n on T_ij); Step 4 is the Rusanov flux
                  of eq. flux_lmnt_lader at the evolved states (lader=True in
                  transport_step).  The printed Step 3 (a length L_ij that
                  is not defined, the two sides' fluxes added across one
                  eta_ij) is read as this predictor; the energy flux takes
                  rho K from the evolved density and momentum.
"""

import numpy as np

from oracle import projection as op


def _geometry_coords(mesh):
    g = mesh.unmerged if getattr(mesh, "period", None) is not None else mesh
    return np.asarray(g.coords, dtype=np.float64)[np.asarray(g.elems, dtype=np.int64)]   # [E, d+1, d]


def _area_vector(pts, toward):
    """Area vector of the segment / triangle pts [.., d, d], oriented so that
    its dot with `toward` is positive."""
    if pts.shape[-1] == 2:
        t = pts[..., 1, :] - pts[..., 0, :]
        eta = np.stack([t[..., 1], -t[..., 0]], axis=-1)
    else:
        eta = 0.5 * np.cross(pts[..., 1, :] - pts[..., 0, :], pts[..., 2, :] - pts[..., 0, :])
    sgn = np.sign((eta * toward).sum(axis=-1))
    return eta * sgn[..., None]


def _simplex_volume(pts):
    d = pts.shape[-1]
    J = pts[..., 1:, :] - pts[..., :1, :]
    return np.abs(np.linalg.det(J)) / (2.0 if d == 2 else 6.0)


def dual_geometry(mesh):
    """pairs [P, 2] local (a, b); eta [E, P, d] from cell a to cell b;
    subvol [E, d+1] |(B, face a)|; bnd_eta [E, d+1] outward area vectors of
    the primal faces."""
    x = _geometry_coords(mesh)
    E, nv, d = x.shape
    B = x.mean(axis=1)
    pairs = [(a, b) for a in range(nv) for b in range(a + 1, nv)]
    eta = np.zeros((E, len(pairs), d))
    for p, (a, b) in enumerate(pairs):
        shared = [c for c in range(nv) if c not in (a, b)]
        pts = np.concatenate([B[:, None, :], x[:, shared, :]], axis=1)
        eta[:, p, :] = _area_vector(pts, x[:, a, :] - B)
    subvol = np.zeros((E, nv))
    bnd_eta = np.zeros((E, nv, d))
    for a in range(nv):
        others = [c for c in range(nv) if c != a]
        subvol[:, a] = _simplex_volume(np.concatenate([B[:, None, :], x[:, others, :]], axis=1))
        # outward: away from vertex a
        bnd_eta[:, a, :] = _area_vector(x[:, others, :], x[:, others, :].mean(axis=1) - x[:, a, :])
    return pairs, eta, subvol, bnd_eta


def rusanov_flux(rho_i, wu_i, rho_j, wu_j, eta, c_alpha):
    """phi [.., 2 + d]: (mass, momentum, energy)."""
    un_i = (wu_i * eta).sum(axis=-1)
    un_j = (wu_j * eta).sum(axis=-1)
    v_i, v_j = un_i / rho_i, un_j / rho_j
    rk_i = (wu_i * wu_i).sum(axis=-1) / (2.0 * rho_i)
    rk_j = (wu_j * wu_j).sum(axis=-1) / (2.0 * rho_j)
    a = np.maximum(np.abs(v_i), np.abs(v_j)) + c_alpha * np.sqrt((eta * eta).sum(axis=-1))
    mass = 0.5 * (un_i + un_j) - 0.5 * a * (rho_j - rho_i)
    mom = 0.5 * (wu_i * v_i[..., None] + wu_j * v_j[..., None]) - 0.5 * a[..., None] * (wu_j - wu_i)
    en = 0.5 * (rk_i * v_i + rk_j * v_j) - 0.5 * a * (rk_j - rk_i)
    return np.concatenate([mass[..., None], mom, en[..., None]], axis=-1)


def cr_gradients(mesh, vel_f, ef):
    """Galerkin (Crouzeix-Raviart) gradient of a face field on each primal
    element: the face-based P1 basis function of face a is 1 - d phi_a, so
    grad u = -d sum_a u_{f_a} (x) grad phi_a; returns [E, d, d] with
    [k, c, e] = d u_c / d x_e."""
    _, grad = op.element_geometry(mesh)
    return -mesh.dim * np.einsum("kac,kae->kce", vel_f[ef], grad)


def heat_flux(mesh, rho, p, fv, ef, lam, r_gas):
    """Q = -lambda grad Theta per element (eq. heatflux), Theta = P / (rho R)
    on the cells (eq. stateequation) with P the mean of the face's vertex
    pressures, grad Theta the Galerkin gradient as for the velocity."""
    theta = p[fv].mean(axis=1) / (rho * r_gas)
    _, grad = op.element_geometry(mesh)
    return lam * mesh.dim * np.einsum("ka,kae->ke", theta[ef], grad)


def viscous_stress(mesh, vel_f, ef, mu):
    """tau = mu (grad u + grad u^T - 2/3 div u I) per element."""
    G = cr_gradients(mesh, vel_f, ef)
    dv = np.trace(G, axis1=1, axis2=2)
    return mu * (G + np.transpose(G, (0, 2, 1)) - (2.0 / 3.0) * dv[:, None, None] * np.eye(mesh.dim)[None])


def other_element(fe, k):
    """The other primal element of the cell of face f (rows of fe [F, 2]
    for the faces of elements k), -1 when the face has one element."""
    return np.where(fe[:, 0] == k, fe[:, 1], fe[:, 0])


def eno_extrapolate(w, g_c, g_u, delta):
    """Step 1 and 2 for one scalar: the gradient of the upwind element g_u
    when |g_u . delta| <= |g_c . delta| (g_c that of the centred element),
    else g_c; returns (the chosen gradient, w + delta . gradient)."""
    dc = (g_c * delta).sum(axis=-1)
    du = (g_u * delta).sum(axis=-1)
    pick_u = np.abs(du) <= np.abs(dc)
    g = np.where(pick_u[..., None], g_u, g_c)
    return g, w + np.where(pick_u, du, dc)


def lader_states(mesh, rho, wu, p, dt, faces, gravity=None):
    """Evolved states (Steps 1-3) of both sides of every dual face.
    Returns dict with, per element and local pair (a, b) of
    dual_geometry's order, the extrapolated ("ext_*") and the evolved
    ("rho_a", "wu_a", "rho_b", "wu_b") density and momentum of side a (the
    cell of face a) and side b, the barycentres N_ab and the gradients."""
    dim = mesh.dim
    fv, fe, ef = faces
    F = fv.shape[0]
    nv = dim + 1
    rho = np.asarray(rho, dtype=np.float64)
    wu = np.asarray(wu, dtype=np.float64).reshape(F, dim)
    fe = np.asarray(fe, dtype=np.int64)
    ef = np.asarray(ef, dtype=np.int64)
    x = _geometry_coords(mesh)                                   # [E, d+1, d]
    E = x.shape[0]
    B = x.mean(axis=1)
    _, gphi = op.element_geometry(mesh)                          # grad phi_a [E, d+1, d]
    # Galerkin (Crouzeix-Raviart) gradients per element: the face-based P1
    # basis function of face a is 1 - d phi_a
    g_rho = -dim * np.einsum("ka,kae->ke", rho[ef], gphi)       # [E, d]
    g_wu = -dim * np.einsum("kac,kae->kce", wu[ef], gphi)       # [E, d, d]: d W_u,c / d x_e
    P = np.asarray(p, dtype=np.float64)[np.asarray(mesh.elems, dtype=np.int64)]
    g_p = np.einsum("ka,kae->ke", P, gphi)                      # grad P^n on each element
    g = np.zeros(dim) if gravity is None else np.asarray(gravity, dtype=np.float64)
    k_ids = np.arange(E)
    pairs = [(a, b) for a in range(nv) for b in range(a + 1, nv)]
    out = {k: np.zeros((E, len(pairs))) for k in ("rho_a", "rho_b", "ext_rho_a", "ext_rho_b")}
    for k in ("wu_a", "wu_b", "ext_wu_a", "ext_wu_b", "nab"):
        out[k] = np.zeros((E, len(pairs), dim))

    def side(face_loc, other_loc, q):
        f = ef[:, face_loc]
        ko = other_element(fe[f], k_ids)
        ko_safe = np.where(ko >= 0, ko, k_ids)                    # no upwind element: the centred one
        shared = [c for c in range(nv) if c not in (face_loc, other_loc)]
        n_ab = (B + x[:, shared, :].sum(axis=1)) / dim            # barycentre of the dual face
        n_i = x[:, [c for c in range(nv) if c != face_loc], :].mean(axis=1)   # barycentre of the cell's face
        delta = n_ab - n_i
        gr, r = eno_extrapolate(rho[f], g_rho, g_rho[ko_safe], delta)
        gw = np.zeros((E, dim, dim))
        u = np.zeros((E, dim))
        for c in range(dim):
            gw[:, c, :], u[:, c] = eno_extrapolate(wu[f, c], g_wu[:, c, :], g_wu[ko_safe, c, :], delta)
        # half-step evolution (Cauchy-Kovalevskaya with the chosen gradients)
        vel = u / r[:, None]
        tr = np.trace(gw, axis1=1, axis2=2)
        div_u = (tr - (vel * gr).sum(axis=1)) / r
        dr = -tr
        dw = -(np.einsum("kce,ke->kc", gw, vel) + u * div_u[:, None]) - g_p + r[:, None] * g[None, :]
        return r, u, r + 0.5 * dt * dr, u + 0.5 * dt * dw, n_ab

    for q, (a, b) in enumerate(pairs):
        ra, ua, rae, uae, nab = side(a, b, q)
        rb, ub, rbe, ube, _ = side(b, a, q)
        out["ext_rho_a"][:, q], out["ext_wu_a"][:, q] = ra, ua
        out["ext_rho_b"][:, q], out["ext_wu_b"][:, q] = rb, ub
        out["rho_a"][:, q], out["wu_a"][:, q] = rae, uae
        out["rho_b"][:, q], out["wu_b"][:, q] = rbe, ube
        out["nab"][:, q] = nab
    out["pairs"] = pairs
    out["g_rho"], out["g_wu"] = g_rho, g_wu
    return out


def transport_step(mesh, rho, wu, we, p, dt, gravity=None, c_alpha=0.0, faces=None, mu=0.0, lam=0.0, r_gas=1.0,
                   lader=False):
    """Returns dict(rho, wu, we, vol, flux_sum, pforce, visc); faces as
    ``projection.dual_faces`` returns them (default: by node ids).  With
    mu > 0 the viscous terms of eq. discrf_momentum / discrf_energy are
    added: the element stress integrated over each dual face (in the energy
    term times the mean velocity of the two cells).  With lam > 0 the heat
    flux Q . eta over each dual face enters the energy ("heat")."""
    dim = mesh.dim
    fv, fe, ef = op.dual_faces(dim, mesh.elems) if faces is None else faces
    F = fv.shape[0]
    pairs, eta, subvol, bnd_eta = dual_geometry(mesh)
    rho = np.asarray(rho, dtype=np.float64)
    wu = np.asarray(wu, dtype=np.float64).reshape(F, dim)
    we = np.asarray(we, dtype=np.float64)
    el = np.asarray(mesh.elems, dtype=np.int64)
    acc = np.zeros((F, 2 + dim))
    vol = np.zeros(F)
    np.add.at(vol, ef, subvol)
    ls = lader_states(mesh, rho, wu, p, dt, (fv, fe, ef), gravity) if lader else None
    for q, (a, b) in enumerate(pairs):
        fa, fb = ef[:, a], ef[:, b]
        if lader:
            # Step 4: the flux at the evolved states of the two sides
            phi = rusanov_flux(ls["rho_a"][:, q], ls["wu_a"][:, q], ls["rho_b"][:, q], ls["wu_b"][:, q],
                               eta[:, q, :], c_alpha)
        else:
            phi = rusanov_flux(rho[fa], wu[fa], rho[fb], wu[fb], eta[:, q, :], c_alpha)
        np.add.at(acc, fa, phi)
        np.add.at(acc, fb, -phi)
    # pressure force: face-mean pressure times area vector over the cell's
    # boundary (dual faces, then the primal boundary faces)
    P = np.asarray(p, dtype=np.float64)[el]                   # [E, d+1]
    PB = P.mean(axis=1)
    pforce = np.zeros((F, dim))
    nv = dim + 1
    for q, (a, b) in enumerate(pairs):
        shared = [c for c in range(nv) if c not in (a, b)]
        pm = (PB + P[:, shared].sum(axis=1)) / (len(shared) + 1)
        np.add.at(pforce, ef[:, a], pm[:, None] * eta[:, q, :])
        np.add.at(pforce, ef[:, b], -pm[:, None] * eta[:, q, :])
    bnd = fe[:, 1] < 0
    for a in range(nv):
        f = ef[:, a]
        on = bnd[f]
        others = [c for c in range(nv) if c != a]
        pm = P[:, others].mean(axis=1)
        np.add.at(pforce, f[on], pm[on, None] * bnd_eta[on, a, :])
    acc[:, 1:1 + dim] += pforce
    visc = np.zeros((F, 1 + dim))
    if mu > 0.0:
        vel = wu / rho[:, None]
        tau = viscous_stress(mesh, vel, ef, mu)
        for q, (a, b) in enumerate(pairs):
            fa, fb = ef[:, a], ef[:, b]
            te = np.einsum("kce,ke->kc", tau, eta[:, q, :])             # tau eta_ab
            en = (te * 0.5 * (vel[fa] + vel[fb])).sum(axis=1)
            np.add.at(visc, fa, -np.concatenate([te, en[:, None]], axis=1))
            np.add.at(visc, fb, np.concatenate([te, en[:, None]], axis=1))
        acc[:, 1:] += visc
    heat = np.zeros(F)
    if lam > 0.0:
        Q = heat_flux(mesh, rho, p, fv, ef, lam, r_gas)
        for q, (a, b) in enumerate(pairs):
            qe = (Q * eta[:, q, :]).sum(axis=1)                         # Q . eta_ab
            np.add.at(heat, ef[:, a], qe)
            np.add.at(heat, ef[:, b], -qe)
        acc[:, 1 + dim] += heat
    g = np.zeros(dim) if gravity is None else np.asarray(gravity, dtype=np.float64)
    q = dt / vol
    out_rho = rho - q * acc[:, 0]
    out_wu = wu - q[:, None] * acc[:, 1:1 + dim] + dt * rho[:, None] * g[None, :]
    out_we = we - q * acc[:, 1 + dim] + dt * (wu @ g)
    return {"rho": out_rho, "wu": out_wu, "we": out_we, "vol": vol, "flux_sum": acc, "pforce": pforce,
            "visc": visc, "heat": heat, "faces": (fv, fe, ef)}

"""CPU oracle of the projection stage around the pressure solve -- TEST
INFRASTRUCTURE (imported only by tests/, __graft_entry__.smoke() and the
CPU-baseline leg of bench.py).

Follows the paper's Sec. 3.3 (pre-projection), Sec. 3.4 (the weak problem
and its Picard iteration) and eq. momentum_dt_p, in plain NumPy/SciPy with
the operator from ``oracle.assemble`` and the solve from ``oracle.cg``:

  dual_faces        the face-type dual cells (Sec. 2): one per face (3D) or
                    edge (2D) of the primal mesh, numbered by the sorted
                    tuples of their vertices' ranks (morton_rank: the
                    library's node order) in lexicographic order; the one or
                    two elements of each face; the face opposite each
                    element vertex.
  element_geometry  volumes |T_k| and basis gradients grad(phi_a) from the
                    inverse Jacobian (on the unmerged mesh for a periodic
                    one).
  projection_stage  dual -> primal means (|T_kf| = |T_k|/(d+1)), the first
                    guesses (rho K) and H, then for each Picard iteration
                    the operator with c = H_k, the right-hand side of the
                    weak problem, CG, and the updates of P, W_u, (rho K) and
                    H; finally the momentum on the dual cells.

Readings (the paper is silent on them): the first momentum guess is
double-tilde W_u (dP^{n+1,1} = 0 in eq. momentum_dt_p); the dual-cell
pressure P_f is the mean of the face's vertex pressures; H is formed on the
dual cells and averaged to the elements, both for the first guess and in
the Picard updates; the gradient of dP on a dual cell is the volume-weighted
mean of its elements' gradients.
"""

import numpy as np
import scipy.sparse as sp

import oracle


def morton_rank(mesh):
    """Rank of each node in the library's internal node order (the Morton
    order of ``oracle.layout``, from the mesh's lattice if it has one)."""
    lay = oracle.layout(mesh.dim, mesh.coords, mesh.elems, getattr(mesh, "lattice", None))
    rank = np.empty(mesh.n_nodes, dtype=np.int64)
    rank[lay["node_new2old"].astype(np.int64)] = np.arange(mesh.n_nodes)
    return rank


def dual_faces(dim, elems, rank=None):
    """(face_vertices [F, dim] ascending node ids, face_elems [F, 2]
    ascending with -1, elem_face [E, dim+1] face opposite local vertex a).
    Faces are numbered by the sorted tuples of their vertices' ranks
    (``rank``, default the node ids themselves) in lexicographic order."""
    elems = np.asarray(elems, dtype=np.int64)
    E, nv = elems.shape
    r = elems if rank is None else np.asarray(rank, dtype=np.int64)[elems]
    recs = []
    for a in range(nv):
        others = np.delete(r, a, axis=1)
        recs.append(np.sort(others, axis=1))
    tup = np.stack(recs, axis=1).reshape(E * nv, dim)          # record e*nv + a
    uniq, inv = np.unique(tup, axis=0, return_inverse=True)
    if rank is not None:
        old = np.empty(len(rank), dtype=np.int64)
        old[np.asarray(rank, dtype=np.int64)] = np.arange(len(rank))
        uniq = np.sort(old[uniq], axis=1)
    inv = inv.ravel()
    F = uniq.shape[0]
    count = np.bincount(inv, minlength=F)
    if count.max() > 2:
        raise ValueError("a face has more than two elements")
    face_elems = np.full((F, 2), -1, dtype=np.int64)
    eid = np.repeat(np.arange(E), nv)
    order = np.lexsort((eid, inv))           # by face, then element
    first = np.ones(order.shape[0], dtype=bool)
    first[1:] = inv[order[1:]] != inv[order[:-1]]
    face_elems[inv[order[first]], 0] = eid[order[first]]
    face_elems[inv[order[~first]], 1] = eid[order[~first]]
    return uniq.astype(np.int32), face_elems.astype(np.int32), inv.reshape(E, nv).astype(np.int64)


def _geometry_mesh(mesh):
    return mesh.unmerged if getattr(mesh, "period", None) is not None else mesh


def element_geometry(mesh):
    """|T_k| and grad(phi_a) [E, d+1, d] from inv(J), J rows x_k - x_0."""
    g = _geometry_mesh(mesh)
    x = np.asarray(g.coords, dtype=np.float64)[np.asarray(g.elems, dtype=np.int64)]
    J = x[:, 1:, :] - x[:, :1, :]
    det = np.linalg.det(J)
    vol = np.abs(det) / (2.0 if mesh.dim == 2 else 6.0)
    Jinv = np.linalg.inv(J)                                   # [E, d, d]
    grad = np.empty((x.shape[0], mesh.dim + 1, mesh.dim))
    grad[:, 1:, :] = np.transpose(Jinv, (0, 2, 1))            # grad phi_k = column k of inv(J)
    grad[:, 0, :] = -grad[:, 1:, :].sum(axis=1)
    return vol, grad


def face_areas(mesh, face_elems, elem_face):
    """|f| from the vertices of the face in its first element (unmerged
    coordinates on a periodic mesh)."""
    g = _geometry_mesh(mesh)
    el = np.asarray(g.elems, dtype=np.int64)
    F = face_elems.shape[0]
    area = np.zeros(F)
    k = face_elems[:, 0].astype(np.int64)
    a = np.argmax(elem_face[k] == np.arange(F)[:, None], axis=1)      # local vertex opposite f
    for f in range(F):
        vs = np.delete(el[k[f]], a[f])
        p = np.asarray(g.coords)[vs]
        if mesh.dim == 2:
            area[f] = np.linalg.norm(p[1] - p[0])
        else:
            area[f] = 0.5 * np.linalg.norm(np.cross(p[1] - p[0], p[2] - p[0]))
    return area


def operator_matrix(mesh, coef, alpha, beta, lumped=False, eliminate=True):
    """alpha M + beta K_c (consistent or lumped M) as a SciPy matrix, with or
    without the Dirichlet elimination."""
    if lumped:
        if getattr(mesh, "period", None) is not None:
            K = oracle.assemble_periodic(mesh, coef, 0.0, beta, eliminate=False).to_scipy()
        else:
            K = oracle.assemble(mesh.dim, mesh.coords, mesh.elems, coef, 0.0, beta, None).to_scipy()
        S = (K + sp.diags(alpha * oracle.lumped_mass_mesh(mesh))).tocsr()
    elif getattr(mesh, "period", None) is not None:
        S = oracle.assemble_periodic(mesh, coef, alpha, beta, eliminate=False).to_scipy()
    else:
        S = oracle.assemble(mesh.dim, mesh.coords, mesh.elems, coef, alpha, beta, None).to_scipy()
    if eliminate:
        d = np.asarray(mesh.dirichlet, dtype=bool)
        keep = sp.diags((~d).astype(np.float64))
        S = (keep @ S @ keep + sp.diags(d.astype(np.float64))).tocsr()
    return S


def _enthalpy(g1, p_nodes, rho_f, face_vertices, elem_face, dim):
    """H_f = g1 P_f / rho_f (P_f the mean of the face's vertex pressures) on
    the dual cells, then H_k = the mean over the faces of T_k."""
    pf = p_nodes[face_vertices].mean(axis=1)
    hf = g1 * pf / rho_f
    return hf[elem_face].mean(axis=1)


def projection_stage(mesh, rho_f, we_f, wu_f, p, gamma, dt, pb=None, bflux=None, dp0=None, n_picard=2,
                     rtol=1e-10, max_iter=20000, lumped=False, faces=None):
    """Returns a dict: p_new, wu_new [F, d], H (per element, after the last
    update), iters, and per Picard iteration the H, (rho K), b, dP and
    element momenta it used or produced (for the identity checks)."""
    dim = mesh.dim
    fv, fe, ef = dual_faces(dim, mesh.elems) if faces is None else faces
    vol, grad = element_geometry(mesh)
    el = np.asarray(mesh.elems, dtype=np.int64)
    N = mesh.n_nodes
    dirm = np.asarray(mesh.dirichlet, dtype=bool)
    alpha = 1.0 / (gamma - 1.0)
    g1 = gamma / (gamma - 1.0)
    rho_f = np.asarray(rho_f, dtype=np.float64)
    wu_f = np.asarray(wu_f, dtype=np.float64).reshape(-1, dim)
    # pre-projection (Sec. 3.3): means over the d+1 sub-elements of equal volume
    rho_k = rho_f[ef].mean(axis=1)
    we_k = np.asarray(we_f, dtype=np.float64)[ef].mean(axis=1)
    wu_k = wu_f[ef].mean(axis=1)
    rk = (wu_k * wu_k).sum(axis=1) / (2.0 * rho_k)
    H = _enthalpy(g1, p, rho_f, fv, ef, dim)
    g = np.zeros(N)
    if pb is not None:
        g[dirm] = pb[dirm] - p[dirm]
    M = operator_matrix(mesh, np.ones(mesh.n_elems), 1.0, 0.0, lumped=lumped, eliminate=False)
    bnd = fe[:, 1] < 0
    area = face_areas(mesh, fe, ef) if (bflux is not None and bnd.any()) else None
    dp = np.zeros(N) if dp0 is None else np.asarray(dp0, dtype=np.float64).copy()
    out = {"iters": [], "H_used": [], "rk_used": [], "b": [], "dp": [], "w_elem": []}
    for _ in range(n_picard):
        # the weak problem (Sec. 3.4) with H and (rho K) of the previous iterate
        b = np.zeros(N)
        src = (we_k - rk) * vol / (dim + 1)
        np.add.at(b, el, np.repeat(src[:, None], dim + 1, axis=1))
        adv = dt * H[:, None] * np.einsum("kc,kac->ka", wu_k, grad) * vol[:, None]
        np.add.at(b, el, adv)
        b -= alpha * (M @ p)
        Afull = operator_matrix(mesh, H, alpha, dt * dt, lumped=lumped, eliminate=False)
        b -= Afull @ g
        if area is not None:
            fvals = -dt * np.where(bnd, bflux, 0.0) * area / dim
            np.add.at(b, fv[bnd].astype(np.int64), np.repeat(fvals[bnd][:, None], dim, axis=1))
        b[dirm] = g[dirm]
        A = oracle.CSR.from_scipy(operator_matrix(mesh, H, alpha, dt * dt, lumped=lumped, eliminate=True))
        dp, st, it, _, _ = oracle.cg(A, b, x0=dp, rtol=rtol, max_iter=max_iter, dirichlet=mesh.dirichlet)
        if st != 0:
            raise RuntimeError("oracle CG status %d" % st)
        out["iters"].append(it)
        out["H_used"].append(H.copy())
        out["rk_used"].append(rk.copy())
        out["b"].append(b)
        out["dp"].append(dp.copy())
        # updates (eq. momentum_dt_p and the Picard update of Sec. 3.4)
        gdp = np.einsum("ka,kac->kc", dp[el], grad)
        w_el = wu_k - dt * gdp
        out["w_elem"].append(w_el)
        rk = (w_el * w_el).sum(axis=1) / (2.0 * rho_k)
        H = _enthalpy(g1, p + dp, rho_f, fv, ef, dim)
    # momentum on the dual cells: volume-weighted gradient of the last dP
    v0 = vol[fe[:, 0]]
    gs = v0[:, None] * gdp[fe[:, 0]]
    vs = v0.copy()
    two = fe[:, 1] >= 0
    v1 = vol[fe[two, 1]]
    gs[two] += v1[:, None] * gdp[fe[two, 1]]
    vs[two] += v1
    out["wu_new"] = wu_f - dt * gs / vs[:, None]
    out["p_new"] = p + dp
    out["H"] = H
    out["faces"] = (fv, fe, ef)
    out["vol"] = vol
    out["grad"] = grad
    out["wu_k"] = wu_k
    out["we_k"] = we_k
    out["rho_k"] = rho_k
    return out


def post_projection(mesh, rho_f, we_f, wu_new, p_new, gamma, dt, faces=None):
    """Sec. 3.5: W_E per primal element from the intermediate energy (mean
    over the element's faces) minus dt/|T_k| times the enthalpy flux through
    its faces, each face l carrying the momentum of its dual cell and
    H_l = gamma/(gamma-1) P_l / rho_l (P_l the mean of the face's vertex
    pressures); the outward area vectors come from the face vertices (on the
    unmerged mesh for a periodic one); then the |T_kf|-weighted mean back to
    the dual cells.  Returns (we_new [F], we_elem [E], vol [E])."""
    dim = mesh.dim
    fv, fe, ef = dual_faces(dim, mesh.elems) if faces is None else faces
    g = _geometry_mesh(mesh)
    x = np.asarray(g.coords, dtype=np.float64)[np.asarray(g.elems, dtype=np.int64)]
    vol, _ = element_geometry(mesh)
    g1 = gamma / (gamma - 1.0)
    rho_f = np.asarray(rho_f, dtype=np.float64)
    wu = np.asarray(wu_new, dtype=np.float64).reshape(-1, dim)
    pf = np.asarray(p_new, dtype=np.float64)[fv].mean(axis=1)
    hf = g1 * pf / rho_f
    we_k = np.asarray(we_f, dtype=np.float64)[ef].mean(axis=1)
    flux = np.zeros(mesh.n_elems)
    nv = dim + 1
    for l in range(nv):
        others = [c for c in range(nv) if c != l]
        pts = x[:, others, :]
        if dim == 2:
            t = pts[:, 1] - pts[:, 0]
            A = np.stack([t[:, 1], -t[:, 0]], axis=1)
        else:
            A = 0.5 * np.cross(pts[:, 1] - pts[:, 0], pts[:, 2] - pts[:, 0])
        out = pts.mean(axis=1) - x[:, l, :]
        A = A * np.sign((A * out).sum(axis=1))[:, None]
        f = ef[:, l]
        flux += hf[f] * (wu[f] * A).sum(axis=1)
    we_el = we_k - dt * flux / vol
    num = np.zeros(fv.shape[0])
    den = np.zeros(fv.shape[0])
    np.add.at(num, ef, (vol * we_el)[:, None] * np.ones((1, nv)))
    np.add.at(den, ef, vol[:, None] * np.ones((1, nv)))
    return num / den, we_el, vol

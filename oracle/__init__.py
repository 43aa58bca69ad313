"""CPU oracle for the P1 pressure solve -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library
and its Python binding) never imports it, and it imports nothing from the
product.  Its numbers come from ``pm_oracle.c`` (plain sequential C, FP64)
plus NumPy/SciPy library routines for the independent cross-checks.

What each function follows in the paper:
  element_matrix  P1 element mass + stiffness of the weak problem of the
                  projection stage (Sec. 3.4); consistent mass, no lumping.
  assemble        the global matrix of that weak problem with Dirichlet
                  pressure nodes (Sec. 3.6) eliminated symmetrically.
  cg              the classical conjugate gradient method the paper names
                  for the resulting symmetric positive definite system
                  (abstract; Sec. 3.4).
  cg_mixed        FP64 defect correction around an FP32 inner CG (not in
                  the paper; pinned only through the FP64 oracle's residual).
  layout          Morton renumbering and node-to-element lists (not in the
                  paper; integer definitions compared bit for bit).
  lumped_mass     m_i = integral of the P1 basis function of node i (sum of
                  |T|/(d+1) over its elements): the weights of the
                  constraint of the space V_0 (Sec. 3.4).
  assemble_periodic  the operator of a periodic mesh whose matching
                  boundary vertices are merged (Sec. 3.6): P^T A P with A
                  assembled on the unmerged mesh and P the 0/1 merge matrix,
                  then Dirichlet elimination.
  assemble_lumped the operator with the lumped (row-sum, diagonal) mass
                  that the paper names for general equations of state
                  (Sec. 3): alpha diag(m) + beta K_c, lumped before the
                  Dirichlet elimination.
  solve_v0        the weak problem posed in V_0 = {z : int z = 0}
                  (Sec. 3.4) when the operator is singular (no mass term,
                  no Dirichlet node): the bordered system
                  [A m; m^T 0][p; lam] = [b; 0], solved densely (NumPy).
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pm_oracle.c")
_LIBDIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIBDIR, "libpm_oracle.so")

OK, NOT_CONVERGED, EINVAL, EDEGENERATE, ENOMEM, EBREAKDOWN = 0, 1, -1, -2, -3, -4

_lib = None


def build():
    """Compile the oracle with gcc (no FMA contraction)."""
    os.makedirs(_LIBDIR, exist_ok=True)
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                           _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    L = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.orc_element_det.restype = dbl
    L.orc_element_det.argtypes = [ctypes.c_int, P]
    L.orc_element_matrix.restype = dbl
    L.orc_element_matrix.argtypes = [ctypes.c_int, P, dbl, dbl, dbl, P]
    L.orc_orient.restype = ctypes.c_int
    L.orc_orient.argtypes = [ctypes.c_int, i64, i64, P, P]
    L.orc_assemble.restype = P
    L.orc_assemble.argtypes = [ctypes.c_int, i64, i64, P, P, P, dbl, dbl, P]
    L.orc_csr_nnz.restype = i64
    L.orc_csr_nnz.argtypes = [P]
    L.orc_csr_export.restype = None
    L.orc_csr_export.argtypes = [P, P, P, P]
    L.orc_csr_free.restype = None
    L.orc_csr_free.argtypes = [P]
    L.orc_csr_from.restype = P
    L.orc_csr_from.argtypes = [i64, P, P, P]
    L.orc_spmv.restype = None
    L.orc_spmv.argtypes = [P, P, P]
    L.orc_cg.restype = ctypes.c_int
    L.orc_cg.argtypes = [P, P, P, P, dbl, i32, P, P, P]
    L.orc_cg_mixed.restype = ctypes.c_int
    L.orc_cg_mixed.argtypes = [P, P, P, P, dbl, dbl, i32, i32, P, P, P]
    L.orc_apply_elements.restype = ctypes.c_int
    L.orc_apply_elements.argtypes = [ctypes.c_int, i64, i64, P, P, P, dbl, dbl, P, P, P, P, i64, P]
    L.orc_set_threads.restype = None
    L.orc_set_threads.argtypes = [ctypes.c_int]
    L.orc_layout.restype = ctypes.c_int
    L.orc_layout.argtypes = [ctypes.c_int, i64, i64, P, P, P, P, P, P, P, P]
    _lib = L
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _u8(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint8)


def element_matrix(dim, xv, c=1.0, alpha=0.0, beta=1.0):
    """Element matrix of one simplex, vertices xv[(dim+1), dim].
    Returns (A[(dim+1),(dim+1)], signed det J)."""
    xv = _f64(xv)
    A = np.zeros((dim + 1, dim + 1))
    det = lib().orc_element_matrix(dim, _p(xv), float(c), float(alpha), float(beta), _p(A))
    return A, det


def orient(dim, coords, elems):
    """Oriented copy of elems (vertices 1 and 2 swapped where det < 0)."""
    coords = _f64(coords)
    el = _i32(elems).copy()
    st = lib().orc_orient(dim, coords.shape[0], el.shape[0], _p(coords), _p(el))
    return st, el


class CSR:
    """The assembled operator A_D of the oracle (owning a C handle)."""

    def __init__(self, handle, n):
        self._h = handle
        self.n = n

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_csr_free(self._h)
            self._h = None

    @property
    def nnz(self):
        return lib().orc_csr_nnz(self._h)

    def export(self):
        nnz = self.nnz
        rp = np.zeros(self.n + 1, dtype=np.int64)
        ci = np.zeros(nnz, dtype=np.int32)
        va = np.zeros(nnz, dtype=np.float64)
        lib().orc_csr_export(self._h, _p(rp), _p(ci), _p(va))
        return rp, ci, va

    @classmethod
    def from_scipy(cls, S):
        """A handle holding a copy of the SciPy matrix S (rows sorted)."""
        S = S.tocsr()
        S.sort_indices()
        n = S.shape[0]
        rp = np.ascontiguousarray(S.indptr, dtype=np.int64)
        ci = _i32(S.indices)
        va = _f64(S.data)
        h = lib().orc_csr_from(n, _p(rp), _p(ci), _p(va))
        if not h:
            raise MemoryError("oracle CSR copy failed")
        return cls(h, n)

    def to_scipy(self):
        import scipy.sparse as sp
        rp, ci, va = self.export()
        return sp.csr_matrix((va, ci, rp), shape=(self.n, self.n))

    def dense(self):
        return self.to_scipy().toarray()

    def matvec(self, x):
        x = _f64(x)
        y = np.zeros(self.n)
        lib().orc_spmv(self._h, _p(x), _p(y))
        return y


def assemble(dim, coords, elems, coef, alpha, beta, dirichlet=None):
    coords, elems, coef = _f64(coords), _i32(elems), _f64(coef)
    d = _u8(dirichlet)
    h = lib().orc_assemble(dim, coords.shape[0], elems.shape[0], _p(coords), _p(elems), _p(coef),
                           float(alpha), float(beta), _p(d))
    if not h:
        raise ValueError("oracle assembly failed (bad index, degenerate element or no memory)")
    return CSR(h, coords.shape[0])


def merge_matrix(rep, n_merged):
    """P with P[i, rep[i]] = 1: the merged P1 basis function of node j is
    the sum of the unmerged basis functions of its images (Sec. 3.6,
    periodic vertices merged), so merged nodal values v give the unmerged
    ones P v."""
    import scipy.sparse as sp
    rep = np.asarray(rep, dtype=np.int64)
    return sp.csr_matrix((np.ones(rep.shape[0]), (np.arange(rep.shape[0]), rep)), shape=(rep.shape[0], n_merged))


def assemble_periodic(mesh, coef, alpha, beta, eliminate=True):
    """The operator of a periodic mesh with merged vertices (Sec. 3.6): the
    Galerkin matrix of the merged P1 space, P^T A P, where A is the matrix
    of the same weak problem (Sec. 3.4) on the unmerged mesh, whose images
    carry their own coordinates; then the Dirichlet nodes of the merged mesh
    are eliminated symmetrically as in ``assemble``."""
    u = mesh.unmerged
    full = assemble(u.dim, u.coords, u.elems, coef, alpha, beta, None).to_scipy()
    P = merge_matrix(mesh.rep, mesh.n_nodes)
    S = (P.T @ full @ P).tocsr()
    return CSR.from_scipy(_eliminate(S, mesh.dirichlet if eliminate else None))


def _eliminate(S, dirichlet):
    """P_I S P_I + P_B for the 0/1 Dirichlet flags (SciPy)."""
    import scipy.sparse as sp
    d = np.zeros(S.shape[0], dtype=bool) if dirichlet is None else np.asarray(dirichlet, dtype=bool)
    if d.any():
        keep = sp.diags((~d).astype(np.float64))
        S = keep @ S @ keep + sp.diags(d.astype(np.float64))
    S = S.tocsr()
    S.eliminate_zeros()
    return S


def assemble_lumped(mesh, coef, alpha, beta):
    """The operator with the lumped mass: alpha diag(m) + beta K_c, m the
    lumped weights (row sums of the consistent mass, ``lumped_mass_mesh``),
    K_c from ``assemble`` (or ``assemble_periodic``) with alpha = 0; the
    Dirichlet nodes are eliminated after lumping."""
    import scipy.sparse as sp
    if getattr(mesh, "period", None) is not None:
        K = assemble_periodic(mesh, coef, 0.0, beta, eliminate=False).to_scipy()
    else:
        K = assemble(mesh.dim, mesh.coords, mesh.elems, coef, 0.0, beta, None).to_scipy()
    S = K + sp.diags(alpha * lumped_mass_mesh(mesh))
    return CSR.from_scipy(_eliminate(S, mesh.dirichlet))


def assemble_problem(prob):
    m = prob.mesh
    if prob.extra.get("lumped"):
        return assemble_lumped(m, prob.coef, prob.alpha, prob.beta)
    if getattr(m, "period", None) is not None:
        return assemble_periodic(m, prob.coef, prob.alpha, prob.beta)
    return assemble(m.dim, m.coords, m.elems, prob.coef, prob.alpha, prob.beta, m.dirichlet)


def cg(A, b, x0=None, rtol=1e-10, max_iter=10000, dirichlet=None):
    """Returns (x, status, iterations, history, true relative residual)."""
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    hist = np.zeros(max_iter + 1)
    it = ctypes.c_int32(0)
    tr = ctypes.c_double(0.0)
    st = lib().orc_cg(A._h, _p(_u8(dirichlet)), _p(b), _p(x), float(rtol), int(max_iter), _p(hist),
                      ctypes.byref(it), ctypes.byref(tr))
    return x, st, it.value, hist[: it.value + 1].copy(), tr.value


def cg_mixed(A, b, x0=None, rtol=1e-10, inner_rtol=1e-5, max_outer=50, max_inner=100000,
             dirichlet=None):
    """Returns (x, status, outer steps, inner iterations, true relative residual)."""
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    o = ctypes.c_int32(0)
    i = ctypes.c_int32(0)
    tr = ctypes.c_double(0.0)
    st = lib().orc_cg_mixed(A._h, _p(_u8(dirichlet)), _p(b), _p(x), float(rtol), float(inner_rtol),
                            int(max_outer), int(max_inner), ctypes.byref(o), ctypes.byref(i),
                            ctypes.byref(tr))
    return x, st, o.value, i.value, tr.value


def set_threads(n):
    """Host threads of cg (1 = the plain sequential oracle).  More threads
    split the SpMV rows (same bits) and sum each dot product over n
    contiguous chunks in chunk order (a fixed order for a given n)."""
    lib().orc_set_threads(int(n))


def apply_elements(dim, coords, elems, coef, alpha, beta, dirichlet, x, rows=None):
    """y = A_D x element by element (no assembly); with rows given, only
    those rows are returned."""
    coords, elems, coef, x = _f64(coords), _i32(elems), _f64(coef), _f64(x)
    d = _u8(dirichlet)
    n = coords.shape[0]
    if rows is None:
        y = np.zeros(n)
        st = lib().orc_apply_elements(dim, n, elems.shape[0], _p(coords), _p(elems), _p(coef),
                                      float(alpha), float(beta), _p(d), _p(x), _p(y), None, 0, None)
        if st != OK:
            raise ValueError("oracle apply failed: %d" % st)
        return y
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(rows.shape[0])
    st = lib().orc_apply_elements(dim, n, elems.shape[0], _p(coords), _p(elems), _p(coef),
                                  float(alpha), float(beta), _p(d), _p(x), None, _p(rows),
                                  rows.shape[0], _p(out))
    if st != OK:
        raise ValueError("oracle apply failed: %d" % st)
    return out


def layout(dim, coords, elems_oriented, lattice=None):
    """Morton node order, element order and node-to-element lists.
    Returns dict of int32 arrays."""
    coords, el = _f64(coords), _i32(elems_oriented)
    lat = None if lattice is None else _i32(lattice)
    n, e = coords.shape[0], el.shape[0]
    out = {
        "node_new2old": np.zeros(n, dtype=np.int32),
        "elem_new2old": np.zeros(e, dtype=np.int32),
        "elems_new": np.zeros_like(el),
        "n2e_off": np.zeros(n + 1, dtype=np.int32),
        "n2e_ent": np.zeros(e * (dim + 1), dtype=np.int32),
    }
    st = lib().orc_layout(dim, n, e, _p(coords), _p(lat), _p(el), _p(out["node_new2old"]),
                          _p(out["elem_new2old"]), _p(out["elems_new"]), _p(out["n2e_off"]),
                          _p(out["n2e_ent"]))
    if st != OK:
        raise ValueError("oracle layout failed: %d" % st)
    return out


def mass_rhs(prob, f):
    """b = M f on free nodes, b_B = f_B on Dirichlet nodes (the interpolated
    source of the manufactured 2D problem)."""
    m = prob.mesh
    fi = np.where(m.dirichlet.astype(bool), 0.0, f)
    if getattr(m, "period", None) is not None:
        y = assemble_periodic(m, np.ones(m.n_elems), 1.0, 0.0).matvec(fi)
    else:
        y = apply_elements(m.dim, m.coords, m.elems, np.ones(m.n_elems), 1.0, 0.0, m.dirichlet, fi)
    return np.where(m.dirichlet.astype(bool), f, y)


def lumped_mass_mesh(mesh):
    """lumped_mass of a mesh; for a periodic mesh the weights of the
    unmerged mesh summed over the images of each merged node (P^T m)."""
    if getattr(mesh, "period", None) is not None:
        u = mesh.unmerged
        mu = lumped_mass(u.dim, u.coords, u.elems)
        return np.bincount(np.asarray(mesh.rep, dtype=np.int64), weights=mu, minlength=mesh.n_nodes)
    return lumped_mass(mesh.dim, mesh.coords, mesh.elems)


def lumped_mass(dim, coords, elems):
    """m_i = sum over the elements containing node i of |T| / (d+1), with
    |T| = |det J| / d! from NumPy's determinant of the edge matrix."""
    coords = _f64(coords)
    elems = np.asarray(elems, dtype=np.int64)
    x = coords[elems]                                   # [E, d+1, d]
    J = x[:, 1:, :] - x[:, :1, :]                       # rows e_k = x_k - x_0
    vol = np.abs(np.linalg.det(J)) / (2.0 if dim == 2 else 6.0)
    return np.bincount(elems.ravel(), weights=np.repeat(vol / (dim + 1), dim + 1), minlength=coords.shape[0])


def solve_v0(A, b, m):
    """The solution in V_0 (Sec. 3.4) of the singular system: p with
    A p = b - lam m and m^T p = 0, from the dense bordered system."""
    n = A.n
    S = A.to_scipy().toarray()
    B = np.zeros((n + 1, n + 1))
    B[:n, :n] = S
    B[:n, n] = m
    B[n, :n] = m
    rhs = np.concatenate([_f64(b), [0.0]])
    sol = np.linalg.solve(B, rhs)
    return sol[:n]


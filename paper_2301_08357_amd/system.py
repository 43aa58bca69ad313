"""Python binding of the C ABI: argument marshalling only.

Every computation happens in libpressure.so (host setup in C++, the
operator and the solver in HIP kernels).  PyTorch provides device memory
and streams: vectors are float64 CUDA tensors, and calls run on the
current stream unless a stream is given.
"""

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _lib
from ._lib import PmMesh, check, load


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class _MeshArgs:
    """Keeps the host arrays alive while the C call reads them."""

    def __init__(self, dim, coords, elems, dirichlet=None, lattice=None, period=None):
        self.coords = _np(coords, np.float64)
        self.elems = _np(elems, np.int32)
        self.dirichlet = None if dirichlet is None else _np(dirichlet, np.uint8)
        self.lattice = None if lattice is None else _np(lattice, np.int32)
        self.period = None if period is None else _np(period, np.float64)
        n = self.coords.shape[0]
        if self.coords.shape != (n, dim) or self.elems.ndim != 2 or self.elems.shape[1] != dim + 1:
            raise ValueError("coords must be [n, dim] and elems [m, dim+1]")
        if self.dirichlet is not None and self.dirichlet.shape != (n,):
            raise ValueError("dirichlet must have one entry per node")
        if self.lattice is not None and self.lattice.shape != (n, dim):
            raise ValueError("lattice must be [n, dim]")
        if self.period is not None and self.period.shape != (dim,):
            raise ValueError("period must have dim entries")
        self.struct = PmMesh(dim, 0, n, self.elems.shape[0], _ptr(self.coords), _ptr(self.elems),
                             _ptr(self.dirichlet), _ptr(self.lattice), _ptr(self.period))

    def ref(self):
        return ctypes.byref(self.struct)


def layout(dim, coords, elems, lattice=None, period=None):
    """The integer layout the library builds (host only, no GPU)."""
    m = _MeshArgs(dim, coords, elems, None, lattice, period)
    n, e = m.coords.shape[0], m.elems.shape[0]
    out = {
        "node_new2old": np.zeros(n, dtype=np.int32),
        "elem_new2old": np.zeros(e, dtype=np.int32),
        "elems_new": np.zeros((e, dim + 1), dtype=np.int32),
        "n2e_off": np.zeros(n + 1, dtype=np.int32),
        "n2e_ent": np.zeros(e * (dim + 1), dtype=np.int32),
    }
    st = load().pressure_layout(m.ref(), *[_ptr(out[k]) for k in
                                           ("node_new2old", "elem_new2old", "elems_new", "n2e_off", "n2e_ent")])
    return st, out


def footprint(dim, coords, elems, flags=_lib.PM_FP64, period=None):
    m = _MeshArgs(dim, coords, elems, period=period)
    b = ctypes.c_uint64(0)
    check(load().pressure_footprint(m.ref(), flags, ctypes.byref(b)), "pressure_footprint")
    return b.value


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, n, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError("%s must be a float64 CUDA tensor" % what)
    if t.numel() != n or not t.is_contiguous():
        raise ValueError("%s must be contiguous with %d entries" % (what, n))
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class SolveResult:
    p: object
    status: int
    iters: int
    hist: np.ndarray
    true_relres: float
    outer: int = 0


class PressureSystem:
    """The P1 pressure operator of one mesh, resident on the GPU.

    alpha * M + dt^2 * K_c with Dirichlet pressure nodes (see
    include/pressure_cg.h for the exact definition)."""

    def __init__(self, dim, coords, elems, coef, mass_coef, dt=1.0, dirichlet=None, lattice=None,
                 flags=_lib.PM_FP64, period=None):
        m = _MeshArgs(dim, coords, elems, dirichlet, lattice, period)
        c = _np(coef, np.float64)
        if c.shape != (m.elems.shape[0],):
            raise ValueError("coef must have one entry per element")
        h = ctypes.c_void_p(None)
        check(load().pressure_setup(m.ref(), _ptr(c), float(mass_coef), float(dt), int(flags),
                                    ctypes.byref(h)), "pressure_setup")
        self._h = h
        self.dim = dim
        self.n_nodes = m.coords.shape[0]
        self.n_elems = m.elems.shape[0]

    @classmethod
    def from_problem(cls, prob, flags=_lib.PM_FP64):
        m = prob.mesh
        if prob.extra.get("lumped"):
            flags |= _lib.PM_MASS_LUMPED
        return cls(m.dim, m.coords, m.elems, prob.coef, prob.alpha, float(np.sqrt(prob.beta)),
                   m.dirichlet, m.lattice, flags, getattr(m, "period", None))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().pressure_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update_coef(self, coef=None, mass_coef=None, dt=1.0):
        c = None if coef is None else _np(coef, np.float64)
        check(load().pressure_update_coef(self._h, _ptr(c), float(mass_coef), float(dt)),
              "pressure_update_coef")

    def set_variant(self, variant):
        check(load().pressure_set_variant(self._h, int(variant)), "pressure_set_variant")

    def set_mixed_mode(self, mode):
        check(load().pressure_set_mixed_mode(self._h, int(mode)), "pressure_set_mixed_mode")

    def apply(self, x, y=None, stream=None):
        import torch
        if y is None:
            y = torch.empty_like(x)
        check(load().pressure_apply(self._h, _dev_ptr(x, self.n_nodes, "x"), _dev_ptr(y, self.n_nodes, "y"),
                                    _stream_handle(stream)), "pressure_apply")
        return y

    def solve(self, rhs, x0=None, rtol=1e-10, max_iter=20000, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty_like(rhs)
        it = ctypes.c_int32(0)
        tr = ctypes.c_double(0.0)
        hist = np.empty(max_iter + 1)   # the library writes entries 0..iters
        st = load().pressure_solve(self._h, _dev_ptr(rhs, self.n_nodes, "rhs"),
                                   None if x0 is None else _dev_ptr(x0, self.n_nodes, "x0"),
                                   float(rtol), int(max_iter), _dev_ptr(out, self.n_nodes, "p"),
                                   ctypes.byref(it), _ptr(hist), ctypes.byref(tr), _stream_handle(stream))
        check(st, "pressure_solve")
        return SolveResult(out, st, it.value, hist[: it.value + 1].copy(), tr.value)

    def solve_noalloc(self, rhs, out, x0=None, rtol=1e-10, max_iter=20000, stream=None, hist=None):
        """pressure_solve_noalloc: solve without any device allocation (the
        library's static scratch holds the CG state).  The caller provides
        the output tensor `out` (and, optionally, the host array `hist` of at
        least max_iter + 1 doubles for the residual history)."""
        it = ctypes.c_int32(0)
        tr = ctypes.c_double(0.0)
        if hist is None:
            hist = np.empty(max_iter + 1)   # the library writes entries 0..iters
        elif hist.dtype != np.float64 or not hist.flags.c_contiguous or hist.size < max_iter + 1:
            raise ValueError("hist must be a contiguous float64 array of at least max_iter + 1 entries")
        st = load().pressure_solve_noalloc(self._h, _dev_ptr(rhs, self.n_nodes, "rhs"),
                                           None if x0 is None else _dev_ptr(x0, self.n_nodes, "x0"),
                                           float(rtol), int(max_iter), _dev_ptr(out, self.n_nodes, "p"),
                                           ctypes.byref(it), _ptr(hist), ctypes.byref(tr), _stream_handle(stream))
        check(st, "pressure_solve_noalloc")
        return SolveResult(out, st, it.value, hist[: it.value + 1].copy(), tr.value)

    def solve_mixed(self, rhs, x0=None, rtol=1e-10, inner_rtol=1e-2, max_iter=20000, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty_like(rhs)
        it = ctypes.c_int32(0)
        outer = ctypes.c_int32(0)
        tr = ctypes.c_double(0.0)
        hist = np.empty(max_iter + 1)   # the library writes entries 0..iters
        st = load().pressure_solve_mixed(self._h, _dev_ptr(rhs, self.n_nodes, "rhs"),
                                         None if x0 is None else _dev_ptr(x0, self.n_nodes, "x0"),
                                         float(rtol), float(inner_rtol), int(max_iter),
                                         _dev_ptr(out, self.n_nodes, "p"), ctypes.byref(it), ctypes.byref(outer),
                                         _ptr(hist), ctypes.byref(tr), _stream_handle(stream))
        check(st, "pressure_solve_mixed")
        return SolveResult(out, st, it.value, hist[: outer.value + 1].copy(), tr.value, outer.value)

    def timing_enable(self, on=True):
        check(load().pressure_timing_enable(self._h, 1 if on else 0), "pressure_timing_enable")

    def timing_read(self):
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        check(load().pressure_timing_read(self._h, ctypes.byref(n), ctypes.byref(ms)), "pressure_timing_read")
        return n.value, ms.value

    def dual_faces(self):
        """The dual cells (faces of the primal mesh in the library's
        numbering): (face_vertices [F, dim], face_elems [F, 2], n_boundary)."""
        nf = ctypes.c_int64(0)
        nb = ctypes.c_int64(0)
        check(load().pressure_dual_count(self._h, ctypes.byref(nf), ctypes.byref(nb)), "pressure_dual_count")
        fv = np.zeros((nf.value, self.dim), dtype=np.int32)
        fe = np.zeros((nf.value, 2), dtype=np.int32)
        check(load().pressure_dual_faces(self._h, _ptr(fv), _ptr(fe)), "pressure_dual_faces")
        return fv, fe, nb.value

    def projection(self, rho, we, wu, p, gamma, dt, pb=None, bflux=None, dp0=None, n_picard=2, rtol=1e-10,
                   max_iter=20000, p_out=None, wu_out=None, h_out=None, stream=None):
        """One projection stage (see pressure_projection in
        include/pressure_cg.h).  Dual-cell fields are float64 CUDA tensors
        in the face numbering of dual_faces(); returns
        (P^{n+1}, W_u^{n+1}, H^{n+1} per element, CG iterations per Picard
        iteration)."""
        import torch
        nf = ctypes.c_int64(0)
        check(load().pressure_dual_count(self._h, ctypes.byref(nf), None), "pressure_dual_count")
        F = nf.value
        args = [_dev_ptr(rho, F, "rho"), _dev_ptr(we, F, "we"), _dev_ptr(wu, F * self.dim, "wu"),
                _dev_ptr(p, self.n_nodes, "p"),
                None if pb is None else _dev_ptr(pb, self.n_nodes, "pb"),
                None if bflux is None else _dev_ptr(bflux, F, "bflux"),
                None if dp0 is None else _dev_ptr(dp0, self.n_nodes, "dp0")]
        if p_out is None:
            p_out = torch.empty_like(p)
        if wu_out is None:
            wu_out = torch.empty_like(wu)
        if h_out is None:
            h_out = torch.empty(self.n_elems, dtype=torch.float64, device=p.device)
        its = np.zeros(max(int(n_picard), 1), dtype=np.int32)
        st = load().pressure_projection(self._h, *args, float(gamma), float(dt), int(n_picard), float(rtol),
                                        int(max_iter), _dev_ptr(p_out, self.n_nodes, "p_out"),
                                        _dev_ptr(wu_out, F * self.dim, "wu_out"),
                                        _dev_ptr(h_out, self.n_elems, "h_out"), _ptr(its),
                                        _stream_handle(stream))
        if st < 0:
            check(st, "pressure_projection")
        return p_out, wu_out, h_out, its, st

    def post_projection(self, rho, we, wu, p, gamma, dt, we_out=None, stream=None):
        """The total energy W_E^{n+1} on the dual cells (see
        pressure_post_projection in include/pressure_cg.h)."""
        import torch
        nf = ctypes.c_int64(0)
        check(load().pressure_dual_count(self._h, ctypes.byref(nf), None), "pressure_dual_count")
        F = nf.value
        we_out = torch.empty_like(we) if we_out is None else we_out
        check(load().pressure_post_projection(self._h, _dev_ptr(rho, F, "rho"), _dev_ptr(we, F, "we"),
                                              _dev_ptr(wu, F * self.dim, "wu"), _dev_ptr(p, self.n_nodes, "p"),
                                              float(gamma), float(dt), _dev_ptr(we_out, F, "we_out"),
                                              _stream_handle(stream)), "pressure_post_projection")
        return we_out

    def transport(self, rho, wu, we, p, dt, gravity=None, c_alpha=0.0, mu=0.0, lam=0.0, r_gas=1.0, rho_out=None,
                  wu_out=None, we_out=None, stream=None, lader=False):
        """One transport step on the dual cells, first order (see
        pressure_transport in include/pressure_cg.h) or, with lader set, the
        second-order LADER step (pressure_transport_lader); returns
        (rho^{n+1}, double-tilde W_u, tilde W_E)."""
        import torch
        nf = ctypes.c_int64(0)
        check(load().pressure_dual_count(self._h, ctypes.byref(nf), None), "pressure_dual_count")
        F = nf.value
        rho_out = torch.empty_like(rho) if rho_out is None else rho_out
        wu_out = torch.empty_like(wu) if wu_out is None else wu_out
        we_out = torch.empty_like(we) if we_out is None else we_out
        g = None if gravity is None else _np(gravity, np.float64)
        if g is not None and g.shape != (self.dim,):
            raise ValueError("gravity must have dim entries")
        fn = load().pressure_transport_lader if lader else load().pressure_transport
        check(fn(self._h, _dev_ptr(rho, F, "rho"), _dev_ptr(wu, F * self.dim, "wu"),
                 _dev_ptr(we, F, "we"), _dev_ptr(p, self.n_nodes, "p"), _ptr(g),
                 float(c_alpha), float(mu), float(lam), float(r_gas), float(dt),
                 _dev_ptr(rho_out, F, "rho_out"),
                 _dev_ptr(wu_out, F * self.dim, "wu_out"), _dev_ptr(we_out, F, "we_out"),
                 _stream_handle(stream)), "pressure_transport_lader" if lader else "pressure_transport")
        return rho_out, wu_out, we_out

    def info(self):
        v = (ctypes.c_int64 * 9)()
        check(load().pressure_info(self._h, v, 9), "pressure_info")
        keys = ("n_nodes", "n_elems", "n_free", "dim", "apply_bytes", "device_bytes", "n_tiles", "n_instances",
                "one_launch_solve")
        return dict(zip(keys, list(v)))


class PressureBatch:
    """Several PressureSystem meshes solved together (batched launches
    replayed from a HIP graph).  Joining a batch fixes each system's launch
    grids to the batch's, so single solves on those systems reproduce the
    batched results bit for bit."""

    def __init__(self, systems, tiles_per_slot=4, nodes_per_lane=8, first_index=1, mixed=False, inner_rtol=1e-2):
        self.systems = list(systems)
        self.mixed = bool(mixed)
        n = len(self.systems)
        hs = (ctypes.c_void_p * n)(*[s._h.value for s in self.systems])
        params = (ctypes.c_int32 * 3)(int(tiles_per_slot), int(nodes_per_lane), int(first_index))
        b = ctypes.c_void_p(None)
        if self.mixed:
            check(load().pressure_batch_create_mixed(hs, n, params, float(inner_rtol), ctypes.byref(b)),
                  "pressure_batch_create_mixed")
        else:
            check(load().pressure_batch_create(hs, n, params, ctypes.byref(b)), "pressure_batch_create")
        self._b = b

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            load().pressure_batch_destroy(self._b)
        self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_graph(self, iterations_per_replay):
        check(load().pressure_batch_set_graph(self._b, int(iterations_per_replay)), "pressure_batch_set_graph")

    def set_persistent(self, persistent=True):
        """Run each step as one cooperative launch of the persistent kernel
        (grid barriers between the CG phases) instead of two launches per
        iteration."""
        check(load().pressure_batch_set_persistent(self._b, 1 if persistent else 0), "pressure_batch_set_persistent")

    def set_barrier_limit(self, microseconds):
        """Time limit of each grid-barrier wait of the persistent form (0: 2 s)."""
        check(load().pressure_batch_set_barrier_limit(self._b, int(microseconds)), "pressure_batch_set_barrier_limit")

    def solve(self, rhs, x0=None, rtol=1e-10, max_iter=20000, out=None, stream=None):
        """rhs, x0, out: lists of float64 CUDA tensors (one per system).
        Returns (overall status, list of SolveResult)."""
        import torch
        n = len(self.systems)
        if out is None:
            out = [torch.empty_like(r) for r in rhs]
        rp = (ctypes.c_void_p * n)(*[_dev_ptr(r, s.n_nodes, "rhs").value for r, s in zip(rhs, self.systems)])
        op = (ctypes.c_void_p * n)(*[_dev_ptr(o, s.n_nodes, "p").value for o, s in zip(out, self.systems)])
        xp = None
        if x0 is not None:
            xp = (ctypes.c_void_p * n)(*[None if x is None else _dev_ptr(x, s.n_nodes, "x0").value
                                         for x, s in zip(x0, self.systems)])
        its = np.zeros(n, dtype=np.int32)
        rel = np.zeros(n)
        st = np.zeros(n, dtype=np.int32)
        code = load().pressure_batch_solve(self._b, rp, xp, float(rtol), int(max_iter), op, _ptr(its), _ptr(rel),
                                           _ptr(st), _stream_handle(stream))
        check(code, "pressure_batch_solve")
        res = [SolveResult(out[m], int(st[m]), int(its[m]), None, float(rel[m])) for m in range(n)]
        return code, res

    # -- continuous batching -------------------------------------------------
    def next_index(self):
        k = ctypes.c_int32(0)
        check(load().pressure_batch_next_index(self._b, ctypes.byref(k)), "pressure_batch_next_index")
        return k.value

    def begin(self, m, rhs, x0=None, rtol=1e-10, max_iter=20000, stream=None):
        s = self.systems[m]
        check(load().pressure_batch_begin(self._b, int(m), _dev_ptr(rhs, s.n_nodes, "rhs"),
                                          None if x0 is None else _dev_ptr(x0, s.n_nodes, "x0"),
                                          float(rtol), int(max_iter), _stream_handle(stream)), "pressure_batch_begin")

    def step(self, stream=None):
        """One chunk of iterations for every solve in flight; returns the
        done flags (numpy bool array, True = idle or finished)."""
        done = np.zeros(len(self.systems), dtype=np.int32)
        check(load().pressure_batch_step(self._b, _ptr(done), _stream_handle(stream)), "pressure_batch_step")
        return done != 0

    def step_launch(self, stream=None):
        """Queue one step (as step) and return at once; step_wait() ends it."""
        check(load().pressure_batch_step_launch(self._b, _stream_handle(stream)), "pressure_batch_step_launch")

    def step_wait(self):
        """Wait for the step queued by step_launch; returns the done flags."""
        done = np.zeros(len(self.systems), dtype=np.int32)
        check(load().pressure_batch_step_wait(self._b, _ptr(done)), "pressure_batch_step_wait")
        return done != 0

    def step_poll(self):
        """The done flags if the step queued by step_launch has ended (as
        step_wait), else None."""
        done = np.zeros(len(self.systems), dtype=np.int32)
        code = load().pressure_batch_step_poll(self._b, _ptr(done))
        if code == _lib.PM_PENDING:
            return None
        check(code, "pressure_batch_step_poll")
        return done != 0

    def finish(self, m, rhs, rtol=1e-10, out=None, stream=None):
        import torch
        s = self.systems[m]
        if out is None:
            out = torch.empty_like(rhs)
        it = ctypes.c_int32(0)
        tr = ctypes.c_double(0.0)
        code = load().pressure_batch_finish(self._b, int(m), _dev_ptr(rhs, s.n_nodes, "rhs"), float(rtol),
                                            _dev_ptr(out, s.n_nodes, "p"), ctypes.byref(it), ctypes.byref(tr),
                                            _stream_handle(stream))
        check(code, "pressure_batch_finish")
        return SolveResult(out, code, it.value, None, tr.value)


def default_tune_cache():
    """Path of the autotuners' cache file: $PM_TUNE_CACHE, else
    ~/.cache/paper_2301_08357_amd/tune.txt."""
    import os
    p = os.environ.get("PM_TUNE_CACHE")
    if p:
        return p
    d = os.path.join(os.path.expanduser("~"), ".cache", "paper_2301_08357_amd")
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, "tune.txt")


def _cache_arg(cache):
    if cache is False:
        return None
    return (default_tune_cache() if cache is None else str(cache)).encode()


def tune_batch(systems, iters=64, cache=None):
    """Batch launch shape picked by the library's autotuner.  Returns
    (tiles_per_slot, nodes_per_lane, ms_per_iteration).  cache: None for the
    default file, False for none, or a path."""
    n = len(systems)
    hs = (ctypes.c_void_p * n)(*[s._h.value for s in systems])
    out = (ctypes.c_int32 * 2)()
    ms = ctypes.c_double(0.0)
    check(load().pressure_batch_tune(hs, n, int(iters), _cache_arg(cache), out, ctypes.byref(ms)),
          "pressure_batch_tune")
    return int(out[0]), int(out[1]), ms.value


def tune_tile(prob, flags=_lib.PM_FP64, iters=32, cache=None):
    """Tile-size flags picked by the library's autotuner for a synth
    Problem.  Returns (flags, ms_per_iteration)."""
    m = prob.mesh
    a = _MeshArgs(m.dim, m.coords, m.elems, m.dirichlet, m.lattice)
    c = _np(prob.coef, np.float64)
    f = ctypes.c_int32(0)
    ms = ctypes.c_double(0.0)
    check(load().pressure_tune_tile(a.ref(), _ptr(c), float(prob.alpha), float(np.sqrt(prob.beta)), int(flags),
                                    int(iters), _cache_arg(cache), ctypes.byref(f), ctypes.byref(ms)),
          "pressure_tune_tile")
    return int(f.value), ms.value

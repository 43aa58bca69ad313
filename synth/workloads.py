"""The synthetic workloads, with their sizes, seeds and value distributions.

  tgv2d_32   2D unit square, 32 x 32 cells x 2 triangles (mesh M2 of the
             paper's Table 1: 2048 triangles, 1089 vertices), jitter 0.2 h,
             c = 1, w = 1e-2, source of p = sin(pi x) sin(pi y), rtol 1e-12.
  cube64     3D unit cube, 64^3 cells x 6 tetrahedra (1,572,864 tets,
             274,625 nodes), no jitter, rho ~ U[0.5, 2], c = 1/rho,
             w in {1e-6, 1e-3, 1}, rtol 1e-10.
  cube160    3D unit cube, 160^3 x 6 (24,576,000 tets, 4,173,281 nodes),
             jitter 0.2 h, rho = exp(0.5 z), z ~ N(0, 1), c = 1/rho,
             w = 1e-4, rtol 1e-10.
  batch256   256 independent meshes: dim 2 or 3 with probability 1/2, node
             count log-uniform in [2e3, 2e5], w log-uniform in [1e-6, 1],
             jitter 0.2 h, rho ~ U[0.5, 2].
  serve10k   10,000 requests over the batch256 meshes, exponential
             inter-arrival times, uniform mesh choice, 1 % right-hand-side
             perturbation per request.
  periodic   meshes periodic along some axes with merged images (Sec. 3.6):
             the fully periodic square (sin 2 pi x sin 2 pi y, w = 1e-2),
             the channel periodic in x with Dirichlet walls in y
             (sin 2 pi x sin pi y), the fully periodic cube (lognormal rho),
             its alpha = 0 form (solved in V_0), and cube160p, the 160^3
             fully periodic cube of the cube160 recipe.
The non-periodic meshes carry Dirichlet pressure nodes on the whole
boundary, and the periodic ones on their open boundaries.
"""

from dataclasses import dataclass, field, replace

import numpy as np

from . import fields
from .mesh import periodic_mesh, structured_mesh
from .rng import MASTER_SEED, STREAM_ARRIVAL, STREAM_BATCH, STREAM_CHOICE, uniform


@dataclass
class Problem:
    name: str
    mesh: object
    coef: np.ndarray          # c_e > 0 per element
    alpha: float              # mass weight
    beta: float               # stiffness scale
    rtol: float
    seed: int
    extra: dict = field(default_factory=dict)


def tgv2d(n=32, seed=MASTER_SEED, w=1e-2):
    m = structured_mesh(2, n, jitter=0.2, seed=seed)
    coef = np.ones(m.n_elems)
    return Problem("tgv2d_%d" % n, m, coef, w, 1.0, 1e-12, seed,
                   extra={"source": fields.helmholtz_source(m.coords, w)})


def cube(n=64, seed=MASTER_SEED, w=1e-3, jitter=0.0, rho="uniform", rtol=1e-10):
    m = structured_mesh(3, n, jitter=jitter, seed=seed)
    if rho == "uniform":
        r = fields.rho_uniform(seed, m.n_elems)
    elif rho == "lognormal":
        r = fields.rho_lognormal(seed, m.n_elems, 0.5)
    else:
        raise ValueError(rho)
    return Problem("cube%d" % n, m, 1.0 / r, w, 1.0, rtol, seed,
                   extra={"xstar": fields.sine_product(m.coords)})


def cube64(w=1e-3, seed=MASTER_SEED):
    return cube(64, seed, w, 0.0, "uniform")


CUBE64_W = (1e-6, 1e-3, 1.0)


def cube160(seed=MASTER_SEED):
    return cube(160, seed, 1e-4, 0.2, "lognormal")


def batch_params(n_meshes=256, seed=MASTER_SEED):
    """(dim, n, w) of each mesh of the batched mix (stream 3)."""
    out = []
    for mi in range(n_meshes):
        u = uniform(seed, STREAM_BATCH, np.arange(4 * mi, 4 * mi + 3, dtype=np.uint64))
        dim = 2 if u[0] < 0.5 else 3
        target = np.exp(np.log(2e3) + u[1] * np.log(100.0))
        n = max(2, int(round(target ** (1.0 / dim))) - 1)
        w = float(np.exp(np.log(1e-6) + u[2] * np.log(1e6)))
        out.append((dim, n, w))
    return out


def batch_sample(k=16, params=None):
    """Indices of k meshes of the batched mix: its largest 2D and 3D meshes,
    its smallest one and its extreme mass weights, the rest spread evenly
    over the list (the same meshes every run)."""
    params = batch_params() if params is None else params
    size = [(n + 1) ** d for d, n, w in params]
    idx = set()
    for d in (2, 3):
        same = [i for i in range(len(params)) if params[i][0] == d]
        idx.add(max(same, key=lambda i: size[i]))
    idx.add(min(range(len(params)), key=lambda i: size[i]))
    idx.add(min(range(len(params)), key=lambda i: params[i][2]))
    idx.add(max(range(len(params)), key=lambda i: params[i][2]))
    for i in np.linspace(0, len(params) - 1, 2 * k).astype(int):
        if len(idx) >= k:
            break
        idx.add(int(i))
    return sorted(idx)


def batch_problem(mi, params, seed=MASTER_SEED):
    dim, n, w = params[mi]
    s = seed + 1 + mi
    m = structured_mesh(dim, n, jitter=0.2, seed=s)
    r = fields.rho_uniform(s, m.n_elems)
    return Problem("batch%d" % mi, m, 1.0 / r, w, 1.0, 1e-10, s,
                   extra={"xstar": fields.sine_product(m.coords)})


def arrivals(n_requests, rate, n_meshes, seed=MASTER_SEED):
    """Arrival times (s) of a Poisson stream of the given rate and the mesh
    each request targets."""
    k = np.arange(n_requests, dtype=np.uint64)
    gaps = -np.log1p(-uniform(seed, STREAM_ARRIVAL, k)) / rate
    choice = np.minimum((uniform(seed, STREAM_CHOICE, k) * n_meshes).astype(np.int64), n_meshes - 1)
    return np.cumsum(gaps), choice


def neumann_square(n=32, seed=MASTER_SEED, jitter=0.2):
    """The zero-Mach limit of the pressure system: alpha = 0, no Dirichlet
    node (the solve is posed in V_0), c = 1 on the unit square.  Source of
    p = cos(pi x) cos(pi y), which has zero mean and zero normal derivative:
    f = 2 pi^2 p.  rtol 1e-12."""
    m = structured_mesh(2, n, jitter=jitter, seed=seed)
    m.dirichlet[:] = 0
    p = np.cos(np.pi * m.coords[:, 0]) * np.cos(np.pi * m.coords[:, 1])
    return Problem("neumann_square_%d" % n, m, np.ones(m.n_elems), 0.0, 1.0, 1e-12, seed,
                   extra={"source": 2.0 * np.pi ** 2 * p, "exact": p})


def neumann_cube(n=10, seed=MASTER_SEED, jitter=0.2, rho="lognormal"):
    """alpha = 0 and no Dirichlet node on the unit cube, c = 1/rho; the rhs
    is b = A x* with x* = prod cos(pi x_i) (so b is compatible)."""
    m = structured_mesh(3, n, jitter=jitter, seed=seed)
    m.dirichlet[:] = 0
    r = fields.rho_lognormal(seed, m.n_elems, 0.5) if rho == "lognormal" else fields.rho_uniform(seed, m.n_elems)
    xs = np.prod(np.cos(np.pi * m.coords), axis=1)
    return Problem("neumann_cube_%d" % n, m, 1.0 / r, 0.0, 1.0, 1e-12, seed, extra={"xstar": xs})


def _sin2pi(coords):
    return np.prod(np.sin(2.0 * np.pi * coords), axis=1)


def periodic_square(n=32, seed=MASTER_SEED, w=1e-2, jitter=0.2):
    """Fully periodic unit square, c = 1, alpha = w: the source of
    p = sin(2 pi x) sin(2 pi y) for w p - Laplace p = f is f = (w + 8 pi^2) p.
    rtol 1e-12."""
    m = periodic_mesh(2, n, (0, 1), jitter=jitter, seed=seed)
    p = _sin2pi(m.coords)
    return Problem("periodic_square_%d" % n, m, np.ones(m.n_elems), w, 1.0, 1e-12, seed,
                   extra={"source": (w + 8.0 * np.pi ** 2) * p, "exact": p})


def periodic_channel(n=24, seed=MASTER_SEED, w=1e-2, jitter=0.2):
    """Unit square periodic in x, Dirichlet walls at y = 0 and y = 1, c = 1,
    alpha = w: p = sin(2 pi x) sin(pi y), f = (w + 5 pi^2) p.  rtol 1e-12."""
    m = periodic_mesh(2, n, (0,), jitter=jitter, seed=seed)
    p = np.sin(2.0 * np.pi * m.coords[:, 0]) * np.sin(np.pi * m.coords[:, 1])
    return Problem("periodic_channel_%d" % n, m, np.ones(m.n_elems), w, 1.0, 1e-12, seed,
                   extra={"source": (w + 5.0 * np.pi ** 2) * p, "exact": p})


def periodic_cube(n=12, seed=MASTER_SEED, w=1e-3, jitter=0.2, rho="lognormal", rtol=1e-10):
    """Fully periodic unit cube, c = 1/rho, alpha = w (w = 0: the solve is
    posed in V_0); b = A x* with x* = prod sin(2 pi x_i)."""
    m = periodic_mesh(3, n, (0, 1, 2), jitter=jitter, seed=seed)
    r = fields.rho_lognormal(seed, m.n_elems, 0.5) if rho == "lognormal" else fields.rho_uniform(seed, m.n_elems)
    return Problem("periodic_cube_%d" % n, m, 1.0 / r, w, 1.0, rtol, seed, extra={"xstar": _sin2pi(m.coords)})


def cube160p(seed=MASTER_SEED):
    """The cube160 recipe (jitter 0.2 h, lognormal rho, w = 1e-4) on the fully
    periodic 160^3 mesh: 4,096,000 merged nodes, 24,576,000 tetrahedra."""
    return periodic_cube(160, seed, 1e-4, 0.2, "lognormal", 1e-10)


def lumped(prob):
    """The same problem with the lumped (diagonal, row-sum) mass matrix in
    the operator; the right-hand side is unchanged."""
    return replace(prob, name=prob.name + "_lumped", extra=dict(prob.extra, lumped=True))

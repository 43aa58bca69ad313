"""Seeded synthetic inputs of the projection stage: the dual-cell fields a
transport stage would hand over (rho^{n+1}, tilde W_E, double-tilde W_u),
the vertex pressure P^n, prescribed boundary pressure and boundary normal
flux.  Nondimensional: P ~ 1/gamma (sound speed ~ 1), rho ~ 1, flow speed
~ mach.  Draws come from stream 7 of the counter generator (rng.py), one
block of 8 draws per face and per node.

The face list (vertex ids per face, elements per face) is an input: the
tests pass the oracle's numbering, which the library must reproduce.
"""

import numpy as np

from .rng import MASTER_SEED, uniform

STREAM_PROJ = 7


def _u(seed, base, n, k):
    return uniform(seed, STREAM_PROJ, np.uint64(base) + np.uint64(8) * np.arange(n, dtype=np.uint64) + np.uint64(k))


def fields(mesh, face_vertices, face_elems, seed=MASTER_SEED, gamma=1.4, mach=0.1, energy_noise=1e-2):
    """dict(p, rho_f, we_f, wu_f [F, dim], pb, bflux)."""
    dim = mesh.dim
    x = np.asarray(mesh.coords, dtype=np.float64)
    N, F = x.shape[0], face_vertices.shape[0]
    p0 = 1.0 / gamma
    s = np.sin(2.0 * np.pi * x)
    p = p0 * (1.0 + 0.05 * np.prod(s, axis=1) + 0.01 * (2.0 * _u(seed, 0, N, 0) - 1.0))
    c = x[np.asarray(face_vertices, dtype=np.int64)].mean(axis=1)          # face centroids
    base = 8 * N
    rho = 1.0 + 0.1 * np.cos(2.0 * np.pi * c[:, 0]) + 0.05 * (2.0 * _u(seed, base, F, 0) - 1.0)
    vel = np.zeros((F, dim))
    vel[:, 0] = np.sin(2.0 * np.pi * c[:, 1])
    vel[:, 1] = -np.sin(2.0 * np.pi * c[:, 0])
    if dim == 3:
        vel[:, 2] = 0.3 * np.sin(2.0 * np.pi * (c[:, 0] + c[:, 1]))
    for k in range(dim):
        vel[:, k] += 0.2 * (2.0 * _u(seed, base, F, 1 + k) - 1.0)
    wu = mach * rho[:, None] * vel
    pf = p[np.asarray(face_vertices, dtype=np.int64)].mean(axis=1)
    we = pf / (gamma - 1.0) + (wu * wu).sum(axis=1) / (2.0 * rho)
    we = we * (1.0 + energy_noise * (2.0 * _u(seed, base, F, 5) - 1.0))
    pb = p * (1.0 + 0.01 * np.cos(2.0 * np.pi * x[:, 0]))
    bflux = np.where(np.asarray(face_elems)[:, 1] < 0, 0.1 * mach * (2.0 * _u(seed, base, F, 6) - 1.0), 0.0)
    return {"p": p, "rho_f": rho, "we_f": we, "wu_f": wu, "pb": pb, "bflux": bflux}

"""Seeded coefficient fields and manufactured nodal fields.

Coefficient convention of the library: the operator is
    alpha * M + beta * K_c,   K_c the stiffness with per-element weight c_e,
which is the paper's pressure operator (Sec. 3.4, the weak problem) with
alpha = 1/(gamma-1), beta = dt^2 and c_e = H_e, or -- after division by
dt^2 -- alpha = w, beta = 1, c_e = 1/rho_e as in the synthetic workloads.
"""

import numpy as np

from .rng import STREAM_PERTURB, STREAM_RHO, normal, uniform


def rho_uniform(seed, n_elems, lo=0.5, hi=2.0):
    """Element density rho_e = lo + (hi - lo) * u, u from stream 2."""
    u = uniform(seed, STREAM_RHO, np.arange(n_elems, dtype=np.uint64))
    return lo + (hi - lo) * u


def rho_lognormal(seed, n_elems, sigma=0.5):
    """Element density rho_e = exp(sigma * z), z standard normal (stream 2)."""
    z = normal(seed, STREAM_RHO, np.arange(n_elems, dtype=np.uint64))
    return np.exp(sigma * z)


def sine_product(coords):
    """x* = prod_i sin(pi x_i) at the nodes (zero on the unit box boundary)."""
    out = np.ones(coords.shape[0])
    for ax in range(coords.shape[1]):
        out *= np.sin(np.pi * coords[:, ax])
    return out


def helmholtz_source(coords, w):
    """f = (w + d pi^2) prod sin(pi x_i): the source for which the continuous
    problem  w p - Laplace p = f  with p = 0 on the boundary has the solution
    p = prod sin(pi x_i)."""
    d = coords.shape[1]
    return (w + d * np.pi ** 2) * sine_product(coords)


def perturbation(seed, request_id, n_nodes):
    """Standard normal per-node draws for one serving request (stream 6,
    index request_id * 2**32 + node)."""
    idx = np.uint64(request_id) * np.uint64(1 << 32) + np.arange(n_nodes, dtype=np.uint64)
    return normal(seed, STREAM_PERTURB, idx)


def perturbation_torch(seed, request_id, n_nodes, device):
    """perturbation() generated on a torch device."""
    import torch
    from .rng import normal_torch
    idx = torch.arange(n_nodes, dtype=torch.int64, device=device) + (int(request_id) << 32)
    return normal_torch(seed, STREAM_PERTURB, idx)

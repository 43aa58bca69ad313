"""Counter-based random numbers: the SplitMix64 output function.

SplitMix64 is the generator of Steele, Lea and Flood, "Fast splittable
pseudorandom number generators" (OOPSLA 2014).  Its output function is used
here as a hash of a 64-bit counter, so draw number ``idx`` of stream
``stream`` is

    z   = seed + GOLDEN * (stream * 2**40 + idx + 1)          (mod 2**64)
    z  ^= z >> 30;  z *= M1;  z ^= z >> 27;  z *= M2;  z ^= z >> 31
    u   = (z >> 11) * 2**-53                                   in [0, 1)

with GOLDEN = 0x9E3779B97F4A7C15, M1 = 0xBF58476D1CE4E5B9,
M2 = 0x94D049BB133111EB.  Streams in use: 1 coordinate jitter, 2 element
density, 3 batched-mesh parameters, 4 arrival times, 5 mesh choice,
6 right-hand-side perturbation.
"""

import numpy as np

MASTER_SEED = 230108357

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)

STREAM_JITTER = 1
STREAM_RHO = 2
STREAM_BATCH = 3
STREAM_ARRIVAL = 4
STREAM_CHOICE = 5
STREAM_PERTURB = 6


def splitmix64_mix(z):
    """The SplitMix64 finaliser applied elementwise to a uint64 array."""
    z = np.asarray(z, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= M1
        z ^= z >> np.uint64(27)
        z *= M2
        z ^= z >> np.uint64(31)
    return z


def raw(seed, stream, idx):
    """uint64 draws ``idx`` (array) of ``stream`` under ``seed``."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        ctr = np.uint64(stream) * np.uint64(1 << 40) + idx + np.uint64(1)
        z = np.uint64(seed) + GOLDEN * ctr
    return splitmix64_mix(z)


def uniform(seed, stream, idx):
    """Uniform doubles in [0, 1) with 53 random bits."""
    return (raw(seed, stream, idx) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed, stream, idx):
    """Standard normal draws by Box-Muller from draws 2*idx and 2*idx+1.

    z = sqrt(-2 ln(1 - u1)) * cos(2 pi u2); 1 - u1 lies in (0, 1] so the log
    is finite.
    """
    idx = np.asarray(idx, dtype=np.uint64)
    u1 = uniform(seed, stream, np.uint64(2) * idx)
    u2 = uniform(seed, stream, np.uint64(2) * idx + np.uint64(1))
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)


def _i64(c):
    """A uint64 constant as the int64 with the same bits."""
    c = int(c)
    return c - (1 << 64) if c >= (1 << 63) else c


def uniform_torch(seed, stream, idx):
    """uniform() computed with torch int64 arithmetic on idx's device (the
    same bits: products wrap mod 2**64, right shifts are masked to logical
    shifts)."""
    import torch
    idx = idx.to(torch.int64)

    def srl(z, k):
        return (z >> k) & ((1 << (64 - k)) - 1)

    ctr = idx + (_i64(stream) << 40) + 1
    z = ctr * _i64(GOLDEN) + _i64(seed)
    z = z ^ srl(z, 30)
    z = z * _i64(M1)
    z = z ^ srl(z, 27)
    z = z * _i64(M2)
    z = z ^ srl(z, 31)
    return srl(z, 11).to(torch.float64) * (2.0 ** -53)


def normal_torch(seed, stream, idx):
    """normal() with torch on idx's device (Box-Muller with torch's log1p and
    cos, which may differ from numpy's in the last bit)."""
    import math
    import torch
    idx = idx.to(torch.int64)
    u1 = uniform_torch(seed, stream, 2 * idx)
    u2 = uniform_torch(seed, stream, 2 * idx + 1)
    return torch.sqrt(-2.0 * torch.log1p(-u1)) * torch.cos((2.0 * math.pi) * u2)

"""The seeded input generators: the torch form of the counter-based
generator gives the numpy form's draws (uniform bits exactly; normals to the
last bit of the libm calls), on any index range, including the serving
perturbation's request-id * 2**32 + node indices."""

import numpy as np
import pytest

from synth import fields, rng

torch = pytest.importorskip("torch")


def test_uniform_torch_bits_equal_numpy():
    idx = np.concatenate([np.arange(4096, dtype=np.uint64),
                          np.uint64(987654) * np.uint64(1 << 32) + np.arange(4096, dtype=np.uint64),
                          np.array([2 ** 63 - 1, 2 ** 62 + 17, 2 ** 40 - 1], dtype=np.uint64)])
    for stream in (1, 2, 6):
        a = rng.uniform(rng.MASTER_SEED, stream, idx)
        b = rng.uniform_torch(rng.MASTER_SEED, stream, torch.tensor(idx.astype(np.int64))).numpy()
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_perturbation_torch_matches_numpy():
    a = fields.perturbation(rng.MASTER_SEED, 4321, 30000)
    b = fields.perturbation_torch(rng.MASTER_SEED, 4321, 30000, "cpu").numpy()
    assert np.max(np.abs(a - b)) <= 4e-15 * max(1.0, np.max(np.abs(a)))
    # standard normal moments on 30000 draws
    assert abs(a.mean()) < 0.03 and abs(a.std() - 1.0) < 0.02

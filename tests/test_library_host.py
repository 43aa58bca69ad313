"""Host-side checks of the HIP library that need no GPU: the C ABI exports
every declared symbol, and the integer layout built by pressure_layout
(orientation, Morton order, element order, node-to-element lists) equals
the oracle's bit for bit."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2301_08357_amd as pm
from paper_2301_08357_amd import _lib
from synth import mesh as smesh
from synth import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "pressure_cg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(pressure_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 13
    L = ctypes.CDLL(_lib.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.SIGNATURES)


def test_strerror_and_footprint():
    L = pm.load()
    for code in (0, 1, -1, -2, -3, -4, -5):
        assert L.pressure_strerror(code)
    m = smesh.structured_mesh(3, 4)
    b = pm.footprint(3, m.coords, m.elems)
    assert b > 16 * m.n_elems + 48 * m.n_nodes


def _compare(dim, coords, elems, lattice):
    st, lay = pm.layout(dim, coords, elems, lattice)
    assert st == 0
    ost, el = oracle.orient(dim, coords, elems)
    assert ost == 0
    ol = oracle.layout(dim, coords, el, lattice)
    for k in ("node_new2old", "elem_new2old", "elems_new", "n2e_off", "n2e_ent"):
        assert np.array_equal(lay[k].ravel(), ol[k].ravel()), k


@pytest.mark.parametrize("dim,n,jit", [(2, 13, 0.2), (3, 6, 0.2), (2, 1, 0.0), (3, 1, 0.0), (3, 9, 0.0)])
def test_layout_matches_oracle(dim, n, jit):
    m = smesh.structured_mesh(dim, n, jitter=jit, seed=21)
    _compare(dim, m.coords, m.elems, m.lattice)
    _compare(dim, m.coords, m.elems, None)          # quantised coordinates


def test_layout_reorients_and_shuffles():
    rng = np.random.default_rng(5)
    m = smesh.structured_mesh(3, 5, jitter=0.2, seed=2)
    el = m.elems[rng.permutation(m.n_elems)].copy()
    flip = rng.random(m.n_elems) < 0.5
    el[flip, 1], el[flip, 2] = el[flip, 2].copy(), el[flip, 1].copy()
    # relabel nodes too
    perm = rng.permutation(m.n_nodes)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(m.n_nodes)
    coords = m.coords[perm]
    lat = m.lattice[perm]
    el2 = inv[el].astype(np.int32)
    _compare(3, coords, el2, lat)
    _compare(3, coords, el2, None)


def test_layout_full_size_tgv_and_cube64():
    p = workloads.tgv2d(32)
    _compare(2, p.mesh.coords, p.mesh.elems, p.mesh.lattice)
    m = smesh.structured_mesh(3, 64)
    _compare(3, m.coords, m.elems, m.lattice)


def test_layout_batch_mix_sample():
    params = workloads.batch_params()
    for mi in (0, 1, 2, 3):
        prob = workloads.batch_problem(mi, params)
        _compare(prob.mesh.dim, prob.mesh.coords, prob.mesh.elems, prob.mesh.lattice)


def test_layout_errors():
    m = smesh.structured_mesh(3, 3, jitter=0.2, seed=8)
    bad = m.elems.copy()
    bad[4, 3] = bad[4, 0]
    assert pm.layout(3, m.coords, bad)[0] == pm.PM_EDEGENERATE
    bad = m.elems.copy()
    bad[4, 3] = -1
    assert pm.layout(3, m.coords, bad)[0] == pm.PM_EINVAL
    lat = m.lattice.copy()
    lat[0, 0] = 1 << 21
    assert pm.layout(3, m.coords, m.elems, lat)[0] == pm.PM_EINVAL
    c = m.coords.copy()
    c[3, 1] = np.nan
    assert pm.layout(3, c, m.elems)[0] == pm.PM_EINVAL


@pytest.mark.parametrize("dim,n,axes", [(2, 7, (0, 1)), (2, 6, (1,)), (3, 5, (0, 1, 2)), (3, 4, (2,))])
def test_periodic_layout_matches_oracle(dim, n, axes):
    """Periodic meshes with merged images, every third element given with the
    opposite orientation: the library decides each sign from the
    minimum-image edge vectors; the oracle decides it on the unmerged mesh,
    where the images have their own coordinates, and then merges."""
    m = smesh.periodic_mesh(dim, n, axes, jitter=0.2, seed=8)
    flip = np.arange(m.n_elems) % 3 == 1
    el = m.elems.copy()
    el[flip, 1], el[flip, 2] = m.elems[flip, 2], m.elems[flip, 1]
    uel = m.unmerged.elems.copy()
    uel[flip, 1], uel[flip, 2] = m.unmerged.elems[flip, 2], m.unmerged.elems[flip, 1]
    for lat in (m.lattice, None):
        st, lay = pm.layout(dim, m.coords, el, lat, m.period)
        assert st == 0
        ost, uo = oracle.orient(dim, m.unmerged.coords, uel)
        assert ost == 0
        ol = oracle.layout(dim, m.coords, m.rep[uo].astype(np.int32), lat)
        for k in ("node_new2old", "elem_new2old", "elems_new", "n2e_off", "n2e_ent"):
            assert np.array_equal(lay[k].ravel(), ol[k].ravel()), k


def test_periodic_layout_errors():
    m = smesh.periodic_mesh(2, 4, (0, 1), jitter=0.2, seed=8)
    for bad in ([1.0, -1.0], [np.nan, 1.0], [np.inf, 0.0]):
        assert pm.layout(2, m.coords, m.elems, m.lattice, bad)[0] == pm.PM_EINVAL
    with pytest.raises(ValueError):
        pm.layout(2, m.coords, m.elems, m.lattice, [1.0, 1.0, 1.0])
    # an element whose two vertices are images of one node has no volume
    bad = m.elems.copy()
    bad[5, 2] = bad[5, 0]
    assert pm.layout(2, m.coords, bad, m.lattice, m.period)[0] == pm.PM_EDEGENERATE

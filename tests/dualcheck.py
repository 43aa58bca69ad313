"""A check of a dual-cell list against its definition (the oracle's
``projection.dual_faces``: every face of the primal mesh once, numbered by
the lexicographic order of its vertices' sorted Morton-rank tuples, with the
one or two elements that share it in ascending order), done without
building the list, so that it runs on the 49M faces of the 160^3 mesh."""

import numpy as np


def check_dual_faces(elems, fv, fe, rank, n_faces):
    """elems [E, d+1] (caller ids), fv [F, d] ascending caller node ids,
    fe [F, 2] ascending caller element ids (-1 = none), rank [N] the Morton
    rank of each caller node, n_faces the number of distinct faces of the
    mesh (from its counts).  Returns None or raises AssertionError.

    A list of n_faces entries in strictly increasing order of the sorted
    rank tuples, each one a face of every element it names, with every
    element named d+1 times, is exactly the definition: strictly increasing
    means distinct, n_faces distinct faces are all of them, and d+1 distinct
    faces per element are all of its faces."""
    E, nv = elems.shape
    d = nv - 1
    F = fv.shape[0]
    assert F == n_faces, (F, n_faces)
    assert fv.shape == (F, d) and fe.shape == (F, 2)
    assert np.all(np.diff(fv, axis=1) > 0)
    r = np.sort(np.asarray(rank, dtype=np.int64)[fv], axis=1)
    inc = np.zeros(F - 1, dtype=bool)
    tie = np.ones(F - 1, dtype=bool)
    for j in range(d):
        dj = np.diff(r[:, j])
        inc |= tie & (dj > 0)
        tie &= dj == 0
        del dj
    assert inc.all()
    del r, inc, tie
    assert np.all(fe[:, 0] >= 0)
    assert np.all((fe[:, 1] < 0) | (fe[:, 0] < fe[:, 1]))
    for slot in (0, 1):
        rows = np.nonzero(fe[:, slot] >= 0)[0]
        conn = elems[fe[rows, slot]]
        for j in range(d):
            assert (conn == fv[rows, j:j + 1]).any(axis=1).all()
        del conn
    named = fe[fe >= 0]
    assert np.array_equal(np.bincount(named, minlength=E), np.full(E, nv))

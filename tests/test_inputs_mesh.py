"""The whole-array box-mesh builder against an element-by-element build, and
the connectivity it produces against the geometry it describes.

The geometric check does not use the builder's rotation tables: for every
side it takes the physical coordinates of the master's face nodes, maps the
face-local indices with the side's orientation code (the convention stated
in include/dgx.h) to the slave's face nodes, and requires the same points
up to the box period.  A wrong face, orientation or master/slave pairing
fails it.
"""
import numpy as np
import pytest

from paper_2605_28627_amd import inputs as I
from mesh_bruteforce import box_mesh_loops

CASES = [((2, 2, 2), 1, 0.0, None), ((3, 2, 4), 1, 0.0, None), ((3, 2, 2), 3, 0.1, None),
         ((2, 2, 2), 1, 0.0, 3), ((3, 3, 2), 2, 0.0, 5), ((2, 3, 2), 3, 0.1, 11), ((3, 3, 3), 1, 0.0, 21),
         ((1, 1, 1), 1, 0.0, 7), ((4, 1, 1), 2, 0.0, None)]


@pytest.mark.parametrize("K,Ngeo,amp,rot", CASES)
def test_box_mesh_matches_loops(K, Ngeo, amp, rot):
    lo, hi = (-np.pi,) * 3, (np.pi,) * 3
    m = I.box_mesh(K, lo, hi, Ngeo=Ngeo, curved_amp=amp, rotate_seed=rot)
    X, se, sl, so = box_mesh_loops(K, lo, hi, Ngeo, amp, rot)
    assert np.array_equal(m.sideElem, se)
    assert np.array_equal(m.sideLoc, sl)
    assert np.array_equal(m.sideOrient, so)
    assert np.abs(m.X - X).max() <= 1e-14


def _face_point(X, e, f, p, q, Ngeo):
    """Physical position of geometry node (p, q) of local face f of element e."""
    r = f // 2
    end = Ngeo if f % 2 else 0
    idx = [0, 0, 0]
    t = [d for d in range(3) if d != r]
    idx[r], idx[t[0]], idx[t[1]] = end, p, q
    a, b, c = idx
    return X[:, e, c, b, a]


@pytest.mark.parametrize("K,Ngeo,amp,rot", CASES)
def test_connectivity_matches_geometry(K, Ngeo, amp, rot):
    lo, hi = np.array((0.0,) * 3), np.array((2.0, 3.0, 1.5))
    m = I.box_mesh(K, tuple(lo), tuple(hi), Ngeo=Ngeo, curved_amp=0.0, rotate_seed=rot)
    L = hi - lo
    for s in range(m.nSides):
        me, se = m.sideElem[2 * s], m.sideElem[2 * s + 1]
        mf, sf = m.sideLoc[2 * s], m.sideLoc[2 * s + 1]
        o = m.sideOrient[s]
        for p in range(Ngeo + 1):
            for q in range(Ngeo + 1):
                a, b = (q, p) if o & 4 else (p, q)
                if o & 1:
                    a = Ngeo - a
                if o & 2:
                    b = Ngeo - b
                xm = _face_point(m.X, me, mf, p, q, Ngeo)
                xs = _face_point(m.X, se, sf, a, b, Ngeo)
                dx = (xm - xs) / L
                assert np.abs(dx - np.round(dx)).max() < 1e-12, (s, p, q)


def test_large_box_is_fast():
    import time
    t0 = time.time()
    m = I.box_mesh((64, 64, 64), (-np.pi,) * 3, (np.pi,) * 3)
    assert time.time() - t0 < 10.0
    assert m.nSides == 3 * 64 ** 3 and m.X.shape == (3, 64 ** 3, 2, 2, 2)

"""Datum-plane oracle (oracle/datum.py) against closed forms: boxes whose
face areas and positions are known, config 1's faces from its documented
geometry (a 100 x 60 x 40 block, a 40 x 20 pocket 15 deep, two blind holes of
radius 4 with 160-gon rims), and the two tolerances of the reading (planes
link within 1e-6 x diagonal, faces count within 1e-4 rad of an axis)."""
import math

import numpy as np
import pytest

from oracle import datum as D
from oracle import oracle as O
from synth import parts as P


def box(lo, hi):
    """Closed box, outward triangles: 8 corners, 12 triangles."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    v = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]], np.float32)
    t = np.array([[0, 2, 1], [0, 3, 2],      # -Z
                  [4, 5, 6], [4, 6, 7],      # +Z
                  [0, 1, 5], [0, 5, 4],      # -Y
                  [3, 7, 6], [3, 6, 2],      # +Y
                  [0, 4, 7], [0, 7, 3],      # -X
                  [1, 2, 6], [1, 6, 5]],     # +X
                 np.int32)
    return v, t


def _area_ok(rec, area, n):
    # W x 2^-k lies within n units of 2^-k below the exact area
    _, k = O.area_weights(*_last_mesh)
    return area - n * 2.0 ** -k - 1e-9 <= rec["area"] <= area + 1e-9


_last_mesh = None


def _frames(v, t):
    global _last_mesh
    _last_mesh = (v, t)
    return D.datum_frames(v, t)


def test_box_closed_form():
    lo, hi = (1.0, 2.0, 3.0), (11.0, 22.0, 33.0)   # 10 x 20 x 30
    fr = _frames(*box(lo, hi))
    area = {0: 600.0, 1: 600.0, 2: 300.0, 3: 300.0, 4: 200.0, 5: 200.0}   # by direction
    coord = {0: 11.0, 1: 1.0, 2: 22.0, 3: 2.0, 4: 33.0, 5: 3.0}
    for a in range(6):
        prim, sec, ter = fr[a]
        assert prim["dir"] == a ^ 1
        assert prim["offset"] == coord[a ^ 1] and prim["n_tris"] == 2
        assert _area_ok(prim, area[a ^ 1], 2)
        # secondary: the largest face off a's axis, ties to the lower direction
        cands = [d for d in range(6) if d >> 1 != a >> 1]
        want = min(cands, key=lambda d: (-area[d], d))
        assert sec["dir"] == want and _area_ok(sec, area[want], 2)
        cands = [d for d in cands if d >> 1 != want >> 1]
        want3 = min(cands, key=lambda d: (-area[d], d))
        assert ter["dir"] == want3 and ter["offset"] == coord[want3]


def test_box_ties_to_lower_direction():
    fr = _frames(*box((0.0, 0.0, 0.0), (10.0, 10.0, 4.0)))
    # setup +Z: +X, -X, +Y, -Y faces are all 10 x 4; the secondary is +X,
    # the tertiary (off X) +Y
    prim, sec, ter = fr[4]
    assert (prim["dir"], sec["dir"], ter["dir"]) == (5, 0, 2)


def test_config1_natural_datums():
    m = P.config1_part()
    fr = _frames(m.verts, m.tris)
    k = 160
    hole = 0.5 * k * 16.0 * math.sin(2 * math.pi / k)     # the 160-gon rim, r = 4
    pl, _ = D.planes(m.verts, m.tris)
    by = {(p[0], p[1]): p for p in pl}
    # the planes the geometry fixes, by (direction, offset): area
    want = {(5, 0.0): 6000.0, (4, 40.0): 5200.0 - hole, (4, 25.0): 800.0, (4, 28.0): hole,
            (1, 0.0): 2400.0, (0, 100.0): 2400.0 - hole, (0, 88.0): hole, (0, 10.0): 300.0, (1, 50.0): 300.0,
            (2, 60.0): 4000.0, (3, 0.0): 4000.0, (2, 20.0): 600.0, (3, 40.0): 600.0}
    _, kk = O.area_weights(m.verts, m.tris)
    for key, area in want.items():
        assert key in by, key
        W = by[key][2] * 2.0 ** -kk
        # rims are 160-gons of FP32 vertices (about 4e-6 mm off the exact
        # circle points), so a rim area is good to about 1e-4 mm^2
        assert area - by[key][3] * 2.0 ** -kk - 2e-3 <= W <= area + 2e-3, (key, W, area)
    assert len(pl) == len(want)   # hole walls are 160-gon facets, none within 1e-4 rad of an axis
    # setups of config 1: {+X, +Z}
    p, s, t = fr[4]
    assert (p["dir"], p["offset"]) == (5, 0.0)
    assert (s["dir"], s["offset"]) == (2, 60.0)      # +Y and -Y tie at 4000: the lower direction
    assert (t["dir"], t["offset"]) == (1, 0.0)       # -X 2400 beats +X 2400 - hole
    p, s, t = fr[0]
    assert (p["dir"], p["offset"]) == (1, 0.0)
    assert (s["dir"], s["offset"]) == (5, 0.0)
    assert (t["dir"], t["offset"]) == (2, 60.0)


def _two_squares(dz):
    v = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                  [3, 0, dz], [4, 0, dz], [4, 1, dz], [3, 1, dz],
                  [0, 0, -50], [0.5, 0, -50], [0, 0.5, -50]], np.float32)   # a far face sets the diagonal
    t = np.array([[0, 1, 2], [0, 2, 3], [4, 5, 6], [4, 6, 7], [8, 10, 9]], np.int32)
    return v, t


@pytest.mark.parametrize("frac,linked", [(0.5, True), (2.0, False)])
def test_planes_link_within_tolerance(frac, linked):
    v, _ = _two_squares(0.0)
    _, diag, _ = O.mesh_info(v)
    dz = np.float32(frac * D.LINK_FRAC * diag)
    v, t = _two_squares(float(dz))
    assert float(v[4, 2]) > 0.0
    pl, k = D.planes(v, t)
    up = [p for p in pl if p[0] == 4]
    if linked:
        assert len(up) == 1 and up[0][3] == 4 and up[0][1] == 0.0
    else:
        assert len(up) == 2 and [p[3] for p in up] == [2, 2]
        assert up[0][1] == 0.0 and up[1][1] == float(v[4, 2])
        # equal areas: the lower offset is the primary of setup -Z
        assert D.datum_frames(v, t)[5][0]["offset"] == 0.0


@pytest.mark.parametrize("ang,facing", [(5e-5, True), (2e-4, False)])
def test_facing_angle(ang, facing):
    c, s = math.cos(ang), math.sin(ang)
    sq = np.array([[0, 0, 0], [10, 0, 0], [10, 10, 0], [0, 10, 0]], np.float64)
    rot = np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    v = (sq @ rot.T).astype(np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    d, _, _, _ = D.faces(v, t)
    assert ((d == 4).all() if facing else (d == -1).all())


def test_zero_area_faces_take_no_part():
    v, t = box((0.0, 0.0, 0.0), (2.0, 3.0, 4.0))
    t2 = np.vstack([t, [[0, 0, 1], [4, 5, 5]]]).astype(np.int32)
    assert D.planes(v, t2)[0] == D.planes(v, t)[0]


def test_planted_mistakes_fail(monkeypatch):
    """Mistakes planted in the oracle are caught by the pins above: a sign
    slip in the direction (d ^ 1 for every facing face), a linkage tolerance
    wide enough to merge planes 3 mm apart, and the roles chosen without
    their axis filters."""
    real_faces = D.faces

    def flipped(verts, tris):
        d, h, w, k = real_faces(verts, tris)
        return np.where(d >= 0, d ^ 1, d), h, w, k

    monkeypatch.setattr(D, "faces", flipped)
    with pytest.raises(AssertionError):
        test_box_closed_form()
    monkeypatch.setattr(D, "faces", real_faces)
    monkeypatch.setattr(D, "LINK_FRAC", 0.05)   # 6 mm: merges the pocket floor and the hole bottom
    with pytest.raises(AssertionError):
        test_config1_natural_datums()
    monkeypatch.setattr(D, "LINK_FRAC", 1e-6)
    real_best = D._best

    def any_axis(cands):   # ignores the axis filters by picking from all planes
        return real_best(cands + [p for p in D.planes(*_last_mesh)[0]])

    monkeypatch.setattr(D, "_best", any_axis)
    with pytest.raises(AssertionError):
        test_box_closed_form()

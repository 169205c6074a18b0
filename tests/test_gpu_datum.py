"""GPU parity of the datum planes per setup orientation (hra_datum_frames)
against the CPU oracle (oracle/datum.py) on the same parts.  Every value is
decided by integers or by FP64 arithmetic the two sides take in the same
order (normals, offsets, integer area weights, single linkage on sorted
offsets), so all eighteen records must match exactly: direction, face
count, integer area, offset and the scaled area."""
import sys

import numpy as np
import pytest

from oracle import datum as D
from synth import parts as P

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2609_05467_amd import hra
    assert torch.cuda.is_available()
    c = hra.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _same(got, want, label):
    for a in range(6):
        for r in range(3):
            g, w = got[a][r], want[a][r]
            assert g["dir"] == w["dir"], (label, a, r, g, w)
            if w["dir"] < 0:
                continue
            assert g["n_tris"] == w["n_tris"], (label, a, r, g, w)
            assert g["area_w"] == w["area_w"], (label, a, r, g, w)
            assert g["offset"] == w["offset"], (label, a, r, g, w)
            assert g["area"] == w["area"], (label, a, r, g, w)


def _check_one(ctx, v, t, label):
    _say("datum", label, len(t))
    bvh = ctx.build_bvh(v, t)
    try:
        got = ctx.datum_frames(bvh)
    finally:
        bvh.release()
    _same(got, D.datum_frames(v, t), label)
    return got


def _box(lo, hi):
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    v = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]], np.float32)
    t = np.array([[0, 2, 1], [0, 3, 2], [4, 5, 6], [4, 6, 7], [0, 1, 5], [0, 5, 4],
                  [3, 7, 6], [3, 6, 2], [0, 4, 7], [0, 7, 3], [1, 2, 6], [1, 6, 5]], np.int32)
    return v, t


def _mesh(m):
    return np.asarray(m.verts, np.float32), np.asarray(m.tris, np.int32)


def test_box_and_config1(ctx):
    fr = _check_one(ctx, *_box((1.0, 2.0, 3.0), (11.0, 22.0, 33.0)), "box 10x20x30")
    assert [f[0]["dir"] for f in fr] == [1, 0, 3, 2, 5, 4]
    fr = _check_one(ctx, *_mesh(P.config1_part()), "config1")
    assert (fr[4][0]["dir"], fr[4][0]["offset"]) == (5, 0.0)


@pytest.mark.parametrize("name", ["pocket", "l_bracket", "stacked", "thin_plate", "tetrahedron", "icosphere",
                                  "blind_hole", "box_part"])
def test_synthetic_shapes(ctx, name):
    m = {"pocket": P.pocket_part, "l_bracket": P.l_bracket, "stacked": P.stacked_boxes, "thin_plate": P.thin_plate,
         "tetrahedron": P.tetrahedron, "icosphere": P.icosphere, "blind_hole": P.blind_hole_part,
         "box_part": P.box_part}[name]()
    _check_one(ctx, *_mesh(m), name)


@pytest.mark.parametrize("seed,family,n", [(5, "pockets", 20_000), (6, "multiaxis", 30_000),
                                           (2, "pockets", 200_000)])
def test_procedural(ctx, seed, family, n):
    _check_one(ctx, *_mesh(P.procedural_part(seed, n, family)), f"{family} seed {seed} ~{n}")


def test_no_axis_facing_faces(ctx):
    """A rotated block faces no axis: every role is empty."""
    v, t = _mesh(P.config1_part())
    c, s = np.cos(0.3), np.sin(0.3)
    R = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]]) @ np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    v = (v.astype(np.float64) @ R.T).astype(np.float32)
    fr = _check_one(ctx, v, t, "rotated config1")
    assert all(r["dir"] == -1 for f in fr for r in f)


def test_ties_links_and_degenerate_faces(ctx):
    """Equal areas (ties to the lower direction, then the lower offset),
    two planes 0.5 and 2 linkage tolerances apart, faces tilted on both
    sides of the facing threshold, and zero-area faces."""
    v, t = _box((0.0, 0.0, 0.0), (10.0, 10.0, 4.0))
    _check_one(ctx, v, t, "tied box")
    for frac in (0.5, 2.0):
        base = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [3, 0, 0], [4, 0, 0], [4, 1, 0], [3, 1, 0],
                         [0, 0, -50], [0.5, 0, -50], [0, 0.5, -50]], np.float64)
        lo, hi = base.min(0), base.max(0)
        dz = np.float32(frac * D.LINK_FRAC * np.linalg.norm(hi - lo))
        base[4:8, 2] = dz
        tt = np.array([[0, 1, 2], [0, 2, 3], [4, 5, 6], [4, 6, 7], [8, 10, 9]], np.int32)
        _check_one(ctx, base.astype(np.float32), tt, f"two squares {frac} tol")
    for ang in (5e-5, 9.9e-5, 1.01e-4, 2e-4):
        c, s = np.cos(ang), np.sin(ang)
        sq = np.array([[0, 0, 0], [10, 0, 0], [10, 10, 0], [0, 10, 0], [0, 0, 5], [10, 0, 5], [10, 10, 5],
                       [0, 10, 5]], np.float64)
        rot = np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
        vv = (sq @ rot.T).astype(np.float32)
        tt = np.array([[0, 1, 2], [0, 2, 3], [4, 6, 5], [4, 7, 6]], np.int32)
        _check_one(ctx, vv, tt, f"tilt {ang}")
    t2 = np.vstack([t, [[0, 0, 1], [4, 5, 5], [2, 2, 2]]]).astype(np.int32)
    fr = _check_one(ctx, v, t2, "box with zero-area faces")
    assert fr[4][0]["n_tris"] == 2


def test_batch_hierarchy_parts(ctx):
    """Each part of a batch hierarchy against the oracle on that part alone."""
    meshes = [_mesh(P.config1_part()), _box((-5.0, -5.0, -5.0), (5.0, 7.0, 9.0)), _mesh(P.l_bracket()),
              _mesh(P.procedural_part(9, 15_000, "pockets"))]
    _say("datum batch of", len(meshes))
    bvh = ctx.build_bvh_batch(meshes)
    try:
        for i, (v, t) in enumerate(meshes):
            _same(ctx.datum_frames(bvh, part=i), D.datum_frames(v, t), f"batch part {i}")
        from paper_2609_05467_amd import hra
        for bad in (-1, len(meshes)):
            with pytest.raises(hra.HraError):
                ctx.datum_frames(bvh, part=bad)
    finally:
        bvh.release()

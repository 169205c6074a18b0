"""Pins of the tool-aware cast oracle (oracle.cast_tool, ball-end tool of
radius r touching the sample point): the half-line-to-triangle distance
against brute force on point clouds and closed forms, a convex face that
every tool reaches, the bottom of a blind hole against the clearance angle
of a tilted capsule, and monotonicity in the radius."""
import math

import numpy as np
import pytest

from synth import parts as P


def _brute_distance(tri, c, u, T=60.0, n=600):
    """Upper bound on the distance, from dense points on both sets."""
    a, b, cc = (np.asarray(x, np.float64) for x in tri)
    w = np.random.default_rng(0).dirichlet([1, 1, 1], 20000)
    pts = w[:, :1] * a + w[:, 1:2] * b + w[:, 2:] * cc
    # edges densely too
    s = np.linspace(0, 1, 2001)[:, None]
    pts = np.concatenate([pts, a + s * (b - a), b + s * (cc - b), cc + s * (a - cc)])
    t = np.linspace(0, T, n)[:, None]
    line = np.asarray(c) + t * np.asarray(u)
    best = np.inf
    for k in range(0, len(line), 50):
        d = np.linalg.norm(line[k:k + 50, None, :] - pts[None, :, :], axis=2)
        best = min(best, d.min())
    return best


def test_distance_closed_forms(orc):
    tri = np.array([[0, 0, 0], [10, 0, 0], [0, 10, 0]], np.float64)
    up, down = np.array([0, 0, 1.0]), np.array([0, 0, -1.0])
    assert orc.tool_distance(tri, [2, 2, 3], up) == pytest.approx(3.0, abs=1e-12)     # above the interior
    assert orc.tool_distance(tri, [2, 2, 3], down) == 0.0                            # meets it
    assert orc.tool_distance(tri, [-5, 2, 4], [1, 0, 0]) == pytest.approx(4.0, abs=1e-12)   # parallel, over it
    assert orc.tool_distance(tri, [-5, 2, 4], [-1, 0, 0]) == pytest.approx(math.hypot(5, 4), abs=1e-12)
    # nearest point on the hypotenuse edge: from (20,20,5) going up, distance to (5,5,0) in xy and z 5 below
    assert orc.tool_distance(tri, [20, 20, 5], up) == pytest.approx(math.sqrt(15 ** 2 * 2 + 25), abs=1e-9)
    # skew lines: the ray along y at height 3 over x = 15 misses the triangle's x range
    assert orc.tool_distance(tri, [15, -5, 3], [0, 1, 0]) == pytest.approx(math.hypot(5, 3), abs=1e-9)


def test_distance_against_brute_force(orc):
    rng = np.random.default_rng(4)
    for _ in range(12):
        tri = rng.uniform(-5, 5, (3, 3))
        c = rng.uniform(-8, 8, 3)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        d = orc.tool_distance(tri, c, u)
        bf = _brute_distance(tri, c, u)
        # the brute force is an upper bound within its sampling step
        assert d <= bf + 1e-9 and bf - d < 0.06, (d, bf)


def test_convex_face_every_direction_free(orc):
    m = P.box_part()
    s = orc.sample_centroid(m.verts, m.tris)
    top = np.nonzero(s["normal"][:, 2] > 0.5)[0][::7]
    sub = {k: v[top] for k, v in s.items()}
    for r in (0.5, 3.0):
        bits, amb = orc.cast_tool(m.verts, m.tris, sub, orc.fibonacci_dirs(150), r)
        assert amb.sum() == 0
        assert np.all(orc.counts(bits, 150) == 150), r
    # the six axes: -Z points into the material (culled); a horizontal tool
    # resting on the top face clears the box (its axis runs r above it)
    b6, _ = orc.cast_tool(m.verts, m.tris, sub, orc.axes6(), 2.0, kind=1)
    assert np.all(b6[:, 0] == 0b011111)


@pytest.mark.parametrize("r_tool", [1.0, 2.0, 3.5])
def test_blind_hole_bottom_clearance_angle(orc, r_tool):
    """A capsule from the hole bottom centre clears the rim iff
    R cos(theta) - (D - r) sin(theta) >= r - tol, theta the tilt from the
    hole axis (the rim point is the nearest wall point; a 160-gon lies
    between its inscribed and circumscribed circles)."""
    R, D, k = 4.0, 12.0, 160
    m = P.blind_hole_part(R, D, k)
    cu, cv, top = m.meta["centre"]
    s = {"point": np.array([[cu, cv, top - D]], np.float32), "normal": np.array([[0, 0, 1.0]], np.float32),
         "origin": np.array([[cu, cv, top - D]], np.float32), "tri": np.zeros(1, np.int32)}
    N = 2048
    dirs = orc.fibonacci_dirs(N)
    bits, amb = orc.cast_tool(m.verts, m.tris, s, dirs, r_tool)
    _, diag, _ = orc.mesh_info(m.verts)
    thr = r_tool - 1e-4 * diag
    th = np.arccos(np.clip(dirs[:, 2].astype(np.float64), -1, 1))
    free = (bits[0][np.arange(N) >> 5] >> (np.arange(N) & 31)) & 1
    r_in = R * math.cos(math.pi / k)
    sure_free = r_in * np.cos(th) - (D - r_tool) * np.sin(th) > thr + 1e-6
    sure_blocked = R * np.cos(th) - (D - r_tool) * np.sin(th) < thr - 1e-6
    assert np.all(free[sure_free] == 1) and np.all(free[sure_blocked] == 0)
    assert sure_free.sum() > 0 and sure_blocked.sum() > 0
    # the free cone shrinks as the tool grows: compare with the ideal circle's count
    ideal = np.sum(R * np.cos(th) - (D - r_tool) * np.sin(th) >= thr)
    assert abs(int(free.sum()) - int(ideal)) <= max(3, 0.05 * ideal)


def test_monotone_in_radius(orc):
    m = P.config1_part()
    s = orc.sample_area(m.verts, m.tris, 120, 3)
    dirs = orc.fibonacci_dirs(128)
    prev, prev_amb = None, None
    for r in (0.5, 1.5, 3.0, 6.0):
        bits, amb = orc.cast_tool(m.verts, m.tris, s, dirs, r)
        if prev is not None:
            sure = ~(amb | prev_amb)
            # a larger tool reaches a subset of the directions a smaller one does
            assert not np.any(bits & ~prev & sure)
            assert orc.counts(bits, 128).sum() <= orc.counts(prev, 128).sum()
        prev, prev_amb = bits, amb


# ---------------------------------------------------------------- holder (tool half-line + holder half-line)
def test_holder_distance_closed_forms(orc):
    """The tool is the half-line from the tip centre; the holder the
    half-line from L + R above it, so its rounded nose reaches down to L."""
    L, R, d = 10.0, 3.0, 2.0
    up = [0, 0, 1.0]
    g = L + R
    # a wall parallel to the axis over every axial position: both at d
    wall = [[d, -50, -5], [d, 50, -5], [d, 0, 500]]
    assert orc.tool_holder_distances(wall, [0, 0, 0], up, L, R) == pytest.approx((d, d), abs=1e-12)
    # a wall that stops at z = 4: the tool runs alongside it (d); the holder's
    # nearest point is the wall's top edge at (d, 0, 4), seen from (0, 0, L + R)
    low = [[d, -50, 4], [d, 50, 4], [d, 0, -100]]
    dc, dh = orc.tool_holder_distances(low, [0, 0, 0], up, L, R)
    assert dc == pytest.approx(d, abs=1e-12) and dh == pytest.approx(math.hypot(d, g - 4), abs=1e-12)
    # a plate the axis crosses at z = L/2: 0 for the tool, L/2 + R for the holder
    plate = lambda z: [[-20, -20, z], [20, -20, z], [0, 30, z]]
    assert orc.tool_holder_distances(plate(L / 2), [0, 0, 0], up, L, R) == pytest.approx((0.0, g - L / 2), abs=1e-12)
    # just below the end of the cutting length the holder's nose clears by a
    # little more than R; crossed beyond L + R, both are 0
    assert orc.tool_holder_distances(plate(L - 0.25), [0, 0, 0], up, L, R)[1] == pytest.approx(R + 0.25, abs=1e-12)
    assert orc.tool_holder_distances(plate(2 * g), [0, 0, 0], up, L, R) == pytest.approx((0.0, 0.0), abs=1e-12)
    # the holder's nose: a point-like triangle on the axis at the end of the
    # cutting length lies exactly R from the holder's half-line
    tiny = [[-1e-6, 0, L], [1e-6, 0, L], [0, 1e-6, L]]
    assert orc.tool_holder_distances(tiny, [0, 0, 0], up, L, R)[1] == pytest.approx(R, abs=1e-6)


def test_holder_distance_against_brute_force(orc):
    rng = np.random.default_rng(7)
    for _ in range(10):
        tri = rng.uniform(-5, 5, (3, 3))
        c = rng.uniform(-8, 8, 3)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        L, R = rng.uniform(1, 12), rng.uniform(1, 6)
        dc, dh = orc.tool_holder_distances(tri, c, u, L, R)
        bc = _brute_distance(tri, c, u)
        bh = _brute_distance(tri, c + (L + R) * u, u)
        assert dc <= bc + 1e-9 and bc - dc < 0.06, (dc, bc)
        assert dh <= bh + 1e-9 and bh - dh < 0.06, (dh, bh)


def test_holder_cast_reduces_to_plain_and_is_monotone(orc):
    """R = r is the plain tool (the holder lies inside it); a wider holder
    never frees a direction a narrower one blocks, and on config 1 (an 8 mm
    deep pocket, 4 mm holes) holders of 2.5, 4 and 6 mm at L = 8 keep
    directions free, strictly fewer as R grows."""
    m = P.config1_part()
    s = orc.sample_area(m.verts, m.tris, 80, 5)
    dirs = orc.fibonacci_dirs(96)
    r = 1.5
    plain, pa = orc.cast_tool(m.verts, m.tris, s, dirs, r)
    same, sa = orc.cast_tool_holder(m.verts, m.tris, s, dirs, r, 8.0, r)
    assert np.array_equal(plain, same) and np.array_equal(pa, sa)
    prev, prev_amb = same, sa
    counts = [int(orc.counts(same, 96).sum())]
    for R in (2.5, 4.0, 6.0):
        bits, amb = orc.cast_tool_holder(m.verts, m.tris, s, dirs, r, 8.0, R)
        assert not np.any(bits & ~prev & ~(amb | prev_amb))
        counts.append(int(orc.counts(bits, 96).sum()))
        prev, prev_amb = bits, amb
    assert counts[-1] > 0 and all(a > b for a, b in zip(counts, counts[1:])), counts

"""Pins for the CPU oracle: closed forms from the geometry, exact rational
arithmetic, invariants, published generator outputs and the paper's printed
indicator values.  Each test is chosen so that a plausible slip in the oracle
(a dropped term, a wrong sign or index, a transposed operand) fails it."""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from synth import parts as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- generator
def test_splitmix64_reference_outputs(orc):
    with open(os.path.join(GOLD, "splitmix64.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for r in rows:
        seed, want = int(r[0]), [int(x) for x in r[1:]]
        got = [int(x) for x in orc.splitmix64(seed, 0, 3)]
        assert got == want


def test_splitmix64_counter_is_sequential(orc):
    a = orc.splitmix64(99, 0, 10)
    b = orc.splitmix64(99, 5, 5)
    assert np.array_equal(a[5:], b)


# ---------------------------------------------------------------- directions
@pytest.mark.parametrize("n", [150, 512, 1024, 2048, 4096])
def test_fibonacci_hemisphere_properties(orc, n):
    d = orc.fibonacci_dirs(n).astype(np.float64)
    assert d.shape == (n, 3)
    assert np.all(d[:, 2] > 0) and np.all(d[:, 2] < 1)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=2e-7)
    # uniform in solid angle: z is uniform on (0,1) (Archimedes), the mean of z
    # over the hemisphere is 1/2 and the horizontal mean vanishes
    assert abs(d[:, 2].mean() - 0.5) < 1e-6
    assert abs(d[:, 0].mean()) < 3.0 / n and abs(d[:, 1].mean()) < 3.0 / n
    zs = np.sort(d[:, 2])
    assert np.allclose(np.diff(zs), 1.0 / n, atol=1e-6)
    # caps: count of points in random caps matches the solid-angle fraction
    rng = np.random.default_rng(n)
    for _ in range(20):
        c = rng.normal(size=3)
        c[2] = abs(c[2])
        c /= np.linalg.norm(c)
        ang = rng.uniform(0.3, 0.9)
        inside = (d @ c) > math.cos(ang)
        # exact solid angle of a cap clipped to z>0 is messy; use caps fully inside
        if c[2] < math.sin(ang) + 1e-9:
            continue
        frac = (1 - math.cos(ang)) / 1.0  # cap area / (2 pi) relative to hemisphere 2 pi
        assert abs(inside.sum() - n * frac) < 2.5 * math.sqrt(n) + 3
    # not cosine-weighted: the mean of z^2 over a uniform hemisphere is 1/3
    assert abs((d[:, 2] ** 2).mean() - 1.0 / 3.0) < 1e-3


GOLDEN_ANGLE = math.pi * (3.0 - math.sqrt(5.0))   # 137.5078 degrees


def _azimuth_walk_ok(d, n):
    """Point 0 lies at azimuth 0 (on the +x side of the x-z plane), point j
    at height 1 - (2j+1)/(2n), and each point lies one golden angle
    counter-clockwise from the one before (Section 3.1's uniform hemisphere
    read as the spherical Fibonacci lattice).  A mirrored set turns
    clockwise; a shifted index moves point 0 off azimuth 0 and every height."""
    d = np.asarray(d, np.float64)
    j = np.arange(n)
    if not np.all(np.abs(d[:, 2] - (1.0 - (2.0 * j + 1.0) / (2.0 * n))) <= 1.2e-7):
        return False
    phi = np.arctan2(d[:, 1], d[:, 0])
    if not (abs(phi[0]) < 1e-6 and d[0, 0] > 0):
        return False
    step = np.mod(np.diff(phi) - GOLDEN_ANGLE + math.pi, 2 * math.pi) - math.pi
    r = np.hypot(d[:, 0], d[:, 1])
    tol = 4e-7 / np.minimum(r[1:], r[:-1]) + 1e-6
    return bool(np.all(np.abs(step) <= tol))


@pytest.mark.parametrize("n", [1, 2, 150, 512, 4096, 8192])
def test_fibonacci_azimuth_walk(orc, n):
    d = orc.fibonacci_dirs(n)
    assert _azimuth_walk_ok(d, n)
    if n >= 2:
        # the check itself catches a mirror (phi -> -phi) and a shifted index
        mirrored = d * np.array([1, -1, 1], np.float32)
        assert not _azimuth_walk_ok(mirrored, n)
        assert not _azimuth_walk_ok(np.roll(d, 1, axis=0), n)


def test_axes6(orc):
    a = orc.axes6()
    assert np.array_equal(a, np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.float32))


# ---------------------------------------------------------------- frames
def test_frame_orthonormal_right_handed(orc):
    rng = np.random.default_rng(5)
    for _ in range(2000):
        n = rng.normal(size=3)
        n = (n / np.linalg.norm(n)).astype(np.float32)
        t, b = orc.frame(n)
        t, b, nn = t.astype(np.float64), b.astype(np.float64), n.astype(np.float64)
        assert abs(np.linalg.norm(t) - 1) < 2e-6 and abs(np.linalg.norm(b) - 1) < 2e-6
        assert abs(t @ b) < 2e-6 and abs(t @ nn) < 2e-6 and abs(b @ nn) < 2e-6
        assert np.allclose(np.cross(t, b), nn, atol=3e-6)


@pytest.mark.parametrize("n", [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)])
def test_frame_axis_normals_exact(orc, n):
    t, b = orc.frame(np.array(n, np.float32))
    for v in (t, b):
        assert set(np.abs(v).tolist()) <= {0.0, 1.0} and np.abs(v).sum() == 1.0
    assert np.array_equal(np.cross(t, b), np.array(n, np.float32))


def test_ray_dirs_plus_z_is_table(orc):
    d = orc.fibonacci_dirs(512)
    r = orc.ray_dirs(np.array([[0, 0, 1]], np.float32), d)
    assert np.array_equal(r[0], d)


# ---------------------------------------------------------------- sampling
def test_mesh_info_config1(orc):
    m = P.config1_part()
    bbox, diag, eps = orc.mesh_info(m.verts)
    assert np.array_equal(bbox, [0, 0, 0, 100, 60, 40])
    assert diag == math.sqrt(100 ** 2 + 60 ** 2 + 40 ** 2)
    assert eps == np.float32(1e-4 * math.sqrt(15200.0))


def test_area_weights_proportional(orc):
    m = P.config1_part()
    w, k = orc.area_weights(m.verts, m.tris)
    v = m.verts.astype(np.float64)[m.tris]
    area = 0.5 * np.linalg.norm(np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]), axis=1)
    assert int(w.sum()) < 2 ** 54
    rel = w.astype(np.float64) / 2.0 ** k
    assert np.allclose(rel, area, rtol=0, atol=2.0 ** -k * 1.01 + 1e-12 * area.max())


def test_samples_inside_their_triangles(orc):
    m = P.config1_part()
    s = orc.sample_area(m.verts, m.tris, 20000, 7)
    v = m.verts.astype(np.float64)[m.tris[s["tri"]]]
    p = s["point"].astype(np.float64)
    e1, e2, q = v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], p - v[:, 0]
    G = np.stack([e1, e2], 2)
    bc, *_ = zip(*[np.linalg.lstsq(G[i], q[i], rcond=None) for i in range(2000)])
    bc = np.array(bc)
    assert np.all(bc > -1e-5) and np.all(bc.sum(1) < 1 + 1e-5)
    resid = np.linalg.norm(np.einsum("nij,nj->ni", G[:2000], bc) - q[:2000], axis=1)
    assert resid.max() < 1e-4
    n = np.cross(e1, e2)
    n /= np.linalg.norm(n, axis=1)[:, None]
    assert np.allclose(s["normal"], n, atol=2e-6)
    _, _, eps = orc.mesh_info(m.verts)
    assert np.allclose(s["origin"] - s["point"], float(eps) * s["normal"], atol=1e-5)


def test_sampling_chi2_area(orc):
    from scipy import stats
    m = P.config1_part()
    n = 200_000
    s = orc.sample_area(m.verts, m.tris, n, 11)
    v = m.verts.astype(np.float64)[m.tris]
    area = 0.5 * np.linalg.norm(np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]), axis=1)
    cnt = np.bincount(s["tri"], minlength=len(area))
    # group consecutive triangles into ~60 bins of similar total area
    edges = np.searchsorted(np.cumsum(area) / area.sum(), np.linspace(0, 1, 61)[1:-1])
    obs = np.array([g.sum() for g in np.split(cnt, edges)])
    exp = np.array([g.sum() for g in np.split(area, edges)]) / area.sum() * n
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, len(obs) - 1) > 1e-4


def test_sampling_uniform_in_triangle(orc):
    m = P.tetrahedron()
    s = orc.sample_area(m.verts, m.tris, 60000, 3)
    sel = s["tri"] == 0
    v = m.verts.astype(np.float64)[m.tris[0]]
    p = s["point"][sel].astype(np.float64)
    # barycentric weight of v0; uniform density gives E[w0] = 1/3 and
    # P(w0 > 1/2) = 1/4 (the corner triangle scaled by 1/2)
    e1, e2 = v[1] - v[0], v[2] - v[0]
    G = np.stack([e1, e2], 1)
    bc = np.linalg.lstsq(G, (p - v[0]).T, rcond=None)[0].T
    w0 = 1 - bc.sum(1)
    assert abs(w0.mean() - 1 / 3) < 0.01
    assert abs((w0 > 0.5).mean() - 0.25) < 0.01


def test_sampling_deterministic(orc):
    m = P.config1_part()
    a = orc.sample_area(m.verts, m.tris, 500, 42)
    b = orc.sample_area(m.verts, m.tris, 500, 42)
    c = orc.sample_area(m.verts, m.tris, 500, 43)
    for k in a:
        assert np.array_equal(a[k], b[k])
    assert not np.array_equal(a["point"], c["point"])


def test_sample_centroid(orc):
    m = P.config1_part()
    s = orc.sample_centroid(m.verts, m.tris)
    assert len(s["tri"]) == m.n_tris
    c = m.verts.astype(np.float64)[m.tris].mean(1)
    assert np.allclose(s["point"], c, rtol=0, atol=1e-5)


# ---------------------------------------------------------------- decision vs exact arithmetic
def _exact_verdict(v, o, d):
    F = [[Fraction(float(x)) for x in row] for row in v]
    O = [Fraction(float(x)) for x in o]
    D = [Fraction(float(x)) for x in d]
    a, b, c = ([F[k][i] - O[i] for i in range(3)] for k in range(3))

    def cr(u, w):
        return [u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]]

    def dt(u, w):
        return u[0] * w[0] + u[1] * w[1] + u[2] * w[2]
    e = [dt(D, cr(b, c)), dt(D, cr(c, a)), dt(D, cr(a, b))]
    Pl = cr([b[i] - a[i] for i in range(3)], [c[i] - a[i] for i in range(3)])
    h, q = dt(a, Pl), dt(D, Pl)
    return e, h, q


def test_decision_matches_exact_arithmetic(orc):
    rng = np.random.default_rng(123)
    nhit = nmiss = namb = 0
    for it in range(3000):
        v = rng.uniform(-10, 10, (3, 3)).astype(np.float32)
        o = rng.uniform(-20, 20, 3).astype(np.float32)
        mode = it % 3
        if mode == 0:     # aim at a random point of the triangle
            w = rng.dirichlet([1, 1, 1])
            tgt = w @ v.astype(np.float64)
        elif mode == 1:   # aim at a point on an edge, slightly perturbed
            k = rng.integers(3)
            lam = rng.uniform()
            tgt = (1 - lam) * v[k].astype(np.float64) + lam * v[(k + 1) % 3]
            tgt = tgt + rng.normal(size=3) * 10.0 ** rng.uniform(-9, -3)
        else:
            tgt = rng.uniform(-10, 10, 3)
        d = tgt - o
        if rng.random() < 0.3:
            d = -d       # pointing away: the hit would be behind
        d = (d / np.linalg.norm(d)).astype(np.float32)
        r, _ = orc.decide_one(v.astype(np.float64), o.astype(np.float64), d.astype(np.float64))
        e, h, q = _exact_verdict(v, o, d)
        if r == 1:
            nhit += 1
            assert (all(x > 0 for x in e) or all(x < 0 for x in e)) and h * q > 0
        elif r == 0:
            nmiss += 1
            assert (any(x > 0 for x in e) and any(x < 0 for x in e)) or h * q <= 0
        else:
            namb += 1
            # an ambiguous verdict needs some quantity inside its band
            vv = v.astype(np.float64) - o.astype(np.float64)
            nb = np.linalg.norm(vv, axis=1)
            S = [np.linalg.norm(vv[2] - vv[1]) * max(nb[1], nb[2]),
                 np.linalg.norm(vv[0] - vv[2]) * max(nb[2], nb[0]),
                 np.linalg.norm(vv[1] - vv[0]) * max(nb[0], nb[1])]
            Pn = np.linalg.norm(np.cross(vv[1] - vv[0], vv[2] - vv[0]))
            near = [abs(float(e[i])) <= 1.01e-6 * S[i] for i in range(3)]
            near += [abs(float(h)) <= 1.01e-6 * Pn * nb.max(), abs(float(q)) <= 1.01e-6 * Pn]
            assert any(near)
    assert nhit > 300 and nmiss > 300 and namb > 10


def test_decision_two_sided(orc):
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float64)
    o = np.array([0.2, 0.2, 1.0])
    assert orc.decide_one(v, o, np.array([0, 0, -1.0]))[0] == 1
    assert orc.decide_one(v[::-1].copy(), o, np.array([0, 0, -1.0]))[0] == 1   # back face blocks too
    assert orc.decide_one(v, o, np.array([0, 0, 1.0]))[0] == 0                  # behind the origin
    assert orc.decide_one(v, np.array([0.2, 0.2, 0.0]), np.array([1.0, 0, 0]))[0] != 1  # in-plane


# ---------------------------------------------------------------- cast closed forms
def test_convex_box_sees_full_hemisphere(orc):
    m = P.box_part()
    s = orc.sample_area(m.verts, m.tris, 300, 5)
    d = orc.fibonacci_dirs(512)
    bits, gr, _ = orc.cast(m.verts, m.tris, s, d)
    assert gr.sum() == 0
    assert np.all(bits == 0xFFFFFFFF)


def test_box_axes6(orc):
    m = P.box_part()
    s = orc.sample_area(m.verts, m.tris, 200, 6)
    bits, gr, _ = orc.cast(m.verts, m.tris, s, orc.axes6(), kind=1)
    assert gr.sum() == 0
    n = s["normal"]
    for i in range(len(n)):
        want = 0
        for k, D in enumerate(orc.axes6()):
            if float(n[i] @ D) >= 0:
                want |= 1 << k
        assert bits[i, 0] == want
    top = np.all(n == np.array([0, 0, 1], np.float32), axis=1)
    assert np.all(bits[top, 0] == 0b011111)


def _hole_expected(rim, o, dirs, depth_to_rim):
    """Bottom-centre closed form: the ray escapes iff its crossing of the rim
    plane lies inside the convex rim polygon; directions whose crossing is
    within 1e-6 rad (relative) of the rim are excluded."""
    rim = rim.astype(np.float64)
    o = o.astype(np.float64)
    d = dirs.astype(np.float64)
    x = o[0] + depth_to_rim * d[:, 0] / d[:, 2]
    y = o[1] + depth_to_rim * d[:, 1] / d[:, 2]
    k = len(rim)
    inside = np.ones(len(d), bool)
    margin = np.full(len(d), np.inf)
    L = depth_to_rim / d[:, 2]
    for i in range(k):
        a, b = rim[i], rim[(i + 1) % k]
        ex, ey = b[0] - a[0], b[1] - a[1]
        cr = (ex * (y - a[1]) - ey * (x - a[0])) / math.hypot(ex, ey)
        inside &= cr > 0
        margin = np.minimum(margin, np.abs(cr) / L)
    return inside, margin > 1e-6


@pytest.mark.parametrize("n,circle", [(512, 26), (1024, 53), (2048, 105), (4096, 211)])
def test_blind_hole_bottom_centre(orc, n, circle):
    r, depth, k = 4.0, 12.0, 160
    m = P.blind_hole_part(r, depth, k)
    _, _, eps = orc.mesh_info(m.verts)
    cu, cv, top = m.meta["centre"]
    p = np.array([[cu, cv, top - depth]], np.float32)
    nn = np.array([[0, 0, 1]], np.float32)
    # origin = fma(eps, n, p): for n = +Z the exact sum rounded once
    o = p.copy()
    o[0, 2] = np.float32(np.float64(p[0, 2]) + np.float64(eps))
    s = {"point": p, "normal": nn, "origin": o, "tri": np.zeros(1, np.int32)}
    d = orc.fibonacci_dirs(n)
    bits, gr, _ = orc.cast(m.verts, m.tris, s, d)
    got = orc.unpack_bits(bits, n)[0]
    assert not orc.unpack_bits(gr, n)[0].any()
    zs = m.verts[:, 2]
    rim = m.verts[(np.abs(zs - top) < 1e-4) & (np.hypot(m.verts[:, 0] - cu, m.verts[:, 1] - cv) < r + 1e-3)]
    ang = np.arctan2(rim[:, 1] - cv, rim[:, 0] - cu)
    rim = rim[np.argsort(ang)]
    want, keep = _hole_expected(rim, o[0], d, float(top) - float(o[0, 2]))
    assert keep.sum() >= n - 2
    assert np.array_equal(got[keep], want[keep])
    # the polygon differs from the inscribed circle only near the rim
    assert abs(int(got.sum()) - circle) <= 3
    # continuum: cone of half-angle atan(r/d), solid-angle fraction 1 - cos
    assert abs(got.mean() - (1 - math.cos(math.atan(r / depth)))) < 0.01


def test_pocket_floor_closed_form(orc):
    m = P.pocket_part()
    x0, y0, x1, y1 = m.meta["rect"]
    depth, top = m.meta["depth"], m.meta["top"]
    _, _, eps = orc.mesh_info(m.verts)
    rng = np.random.default_rng(9)
    S = 24
    p = np.stack([rng.uniform(x0 + 0.5, x1 - 0.5, S), rng.uniform(y0 + 0.5, y1 - 0.5, S),
                  np.full(S, top - depth)], 1).astype(np.float32)
    nn = np.tile(np.array([0, 0, 1], np.float32), (S, 1))
    o = p.copy()
    o[:, 2] = (p[:, 2].astype(np.float64) + float(eps)).astype(np.float32)
    s = {"point": p, "normal": nn, "origin": o, "tri": np.zeros(S, np.int32)}
    N = 1024
    d = orc.fibonacci_dirs(N)
    bits, gr, _ = orc.cast(m.verts, m.tris, s, d)
    got = orc.unpack_bits(bits, N)
    dd = d.astype(np.float64)
    for i in range(S):
        h = float(top) - float(o[i, 2])
        x = float(o[i, 0]) + h * dd[:, 0] / dd[:, 2]
        y = float(o[i, 1]) + h * dd[:, 1] / dd[:, 2]
        want = (x > x0) & (x < x1) & (y > y0) & (y < y1)
        L = h / dd[:, 2]
        mg = np.minimum.reduce([np.abs(x - x0), np.abs(x - x1), np.abs(y - y0), np.abs(y - y1)]) / L
        keep = mg > 1e-6
        assert np.array_equal(got[i][keep], want[keep])


def test_watertight_interior_never_escapes(orc):
    m = P.config1_part()
    rng = np.random.default_rng(4)
    pts = np.array([[5, 5, 5], [95, 55, 5], [60, 10, 20], [20, 50, 35], [85, 45, 10]], np.float32)
    O = np.repeat(pts, 400, 0)
    D = rng.normal(size=(len(O), 3))
    D = (D / np.linalg.norm(D, axis=1)[:, None]).astype(np.float32)
    v = orc.cast_rays(m.verts, m.tris, O, D)
    assert not np.any(v == 1)


def test_grazing_through_shared_edge(orc):
    m = P.box_part()
    # the top cell [10,20]^2 is split along its diagonal x = y
    v = orc.cast_rays(m.verts, m.tris, np.array([[15, 15, 50], [15, 14, 50]], np.float32),
                      np.array([[0, 0, -1], [0, 0, -1]], np.float32))
    assert v[0] == 2 and v[1] == 0


def test_config1_full_cast_no_grazing(orc):
    m = P.config1_part()
    s = orc.sample_area(m.verts, m.tris, 200, 1)
    d = orc.fibonacci_dirs(512)
    bits, gr, _ = orc.cast(m.verts, m.tris, s, d)
    assert gr.sum() == 0
    cnt = orc.counts(bits, 512)
    # every sample on a bbox-plane face (no feature above) sees the full hemisphere
    bbox, diag, _ = orc.mesh_info(m.verts)
    on_box = orc.bbox_face_tris(m.verts, m.tris, bbox, diag)[s["tri"]]
    top_open = on_box & (s["normal"][:, 2] == 1)
    assert np.all(cnt[top_open] == 512)


# ---------------------------------------------------------------- directional statistics
def test_dirstats_flat_face(orc):
    m = P.box_part()
    s = orc.sample_area(m.verts, m.tris, 120, 8)
    N = 512
    d = orc.fibonacci_dirs(N)
    bits, _, _ = orc.cast(m.verts, m.tris, s, d)
    st = orc.dirstats(s, d, bits)
    n = s["normal"].astype(np.float64)
    ax = np.argmax(np.abs(n), 1)
    assert np.array_equal(st["axis"], ax)
    # continuum values for an open flat face: E|x| = E|y| = E|z| = 1/2 over a
    # uniform hemisphere, so c = 1/3, and the signed mean is n/2
    assert np.all(np.abs(st["conc"] - 1 / 3) < 2e-3)
    assert np.allclose(st["mean"], 0.5 * n, atol=1e-2)
    cnt = orc.counts(bits, N)
    assert int(st["hist"].sum()) == int(cnt.sum())
    top = n[:, 2] > 0.5
    stt = orc.dirstats({k: v[top] for k, v in s.items()}, d, bits[top])
    zb = np.arange(8192) // 128
    assert stt["hist"][zb < 32].sum() == 0


def test_dirstats_hole_bottom_cap(orc):
    r, depth = 4.0, 12.0
    m = P.blind_hole_part(r, depth, 160)
    _, _, eps = orc.mesh_info(m.verts)
    cu, cv, top = m.meta["centre"]
    p = np.array([[cu, cv, top - depth]], np.float32)
    s = {"point": p, "normal": np.array([[0, 0, 1]], np.float32),
         "origin": np.array([[cu, cv, np.float64(p[0, 2]) + np.float64(eps)]], np.float32),
         "tri": np.zeros(1, np.int32)}
    N = 4096
    d = orc.fibonacci_dirs(N)
    bits, _, _ = orc.cast(m.verts, m.tris, s, d)
    st = orc.dirstats(s, d, bits)
    a = math.atan(r / depth)
    # cap of half-angle a: m_z = (1 + cos a)/2; A_x = A_y = (2/pi) E[sin th];
    # with E[sin th] over the cap, c = A_z / (A_x + A_y + A_z)
    th = np.linspace(0, a, 200001)
    w = np.sin(th)
    esin = np.trapezoid(np.sin(th) * w, th) / np.trapezoid(w, th)
    ez = (1 + math.cos(a)) / 2
    c = ez / (ez + 2 * (2 / math.pi) * esin)
    assert st["axis"][0] == 2
    assert abs(st["mean"][0, 2] - ez) < 5e-3
    assert abs(st["conc"][0] - c) < 1e-2
    assert abs(c - 0.78312) < 1e-4


def test_dirstats_single_bit(orc):
    N = 64
    d = orc.fibonacci_dirs(N)
    n = np.array([[0.6, 0.0, 0.8]], np.float32)
    s = {"point": np.zeros((1, 3), np.float32), "normal": n, "origin": np.zeros((1, 3), np.float32),
         "tri": np.zeros(1, np.int32)}
    j = 37
    bits = np.zeros((1, 2), np.uint32)
    bits[0, j // 32] = 1 << (j % 32)
    st = orc.dirstats(s, d, bits)
    w = orc.ray_dirs(n, d)[0, j].astype(np.float64)
    assert np.allclose(st["mean"][0], w) and np.allclose(st["absmean"][0], np.abs(w))
    assert st["axis"][0] == int(np.argmax(np.abs(w)))
    zb = min(63, int((w[2] / np.linalg.norm(w) + 1) * 32))
    az = min(127, int((math.atan2(w[1], w[0]) + math.pi) / (2 * math.pi) * 128))
    assert st["hist"][zb * 128 + az] == 1 and st["hist"].sum() == 1


def test_dirstats_empty_row(orc):
    d = orc.fibonacci_dirs(64)
    s = {"normal": np.array([[0, 0, 1]], np.float32)}
    st = orc.dirstats(s, d, np.zeros((1, 2), np.uint32))
    assert st["axis"][0] == -1 and st["hist"].sum() == 0


# ---------------------------------------------------------------- classification
def test_paper_tables_verdicts(orc):
    with open(os.path.join(GOLD, "paper_tables.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for name, acc, sx, sy, sz, c, verdict in rows:
        ind = {"access": float(acc), "shares": [float(sx), float(sy), float(sz)], "conc": float(c)}
        multi, _ = orc.classify(ind)
        assert multi == (verdict == "multi"), name
        assert abs(sum(ind["shares"]) - 1.0) < 2e-3     # shares sum to 100 % (Section 3.3)


def test_indicators_shares_sum_to_one(orc):
    rng = np.random.default_rng(1)
    axis = rng.integers(-1, 3, 1000)
    ind = orc.indicators(rng.integers(0, 100, 1000), 100, axis, rng.uniform(1 / 3, 1, 1000))
    assert abs(sum(ind["shares"]) - 1.0) < 1e-12 and ind["n_blind"] == int((axis < 0).sum())


def _classify_part(orc, m, n_samples, N, seed):
    s = orc.sample_area(m.verts, m.tris, n_samples, seed)
    d = orc.fibonacci_dirs(N)
    bits, _, _ = orc.cast(m.verts, m.tris, s, d)
    st = orc.dirstats(s, d, bits)
    ind = orc.indicators(orc.counts(bits, N), N, st["axis"], st["conc"])
    return ind, orc.classify(ind)


def test_thin_plate_is_three_axis(orc):
    ind, (multi, _) = _classify_part(orc, P.thin_plate(), 300, 150, 2)
    assert ind["access"] == 1.0 and max(ind["shares"]) > 0.8 and not multi


def test_icosphere_is_multi_axis(orc):
    ind, (multi, tripped) = _classify_part(orc, P.icosphere(), 600, 150, 2)
    assert max(ind["shares"]) < 0.45 and multi and tripped & 2


# ---------------------------------------------------------------- reach, classes, setups
@pytest.fixture(scope="module")
def cfg1_axes(orc):
    m = P.config1_part()
    s = orc.sample_area(m.verts, m.tris, 1000, 1)
    bits, gr, _ = orc.cast(m.verts, m.tris, s, orc.axes6(), kind=1)
    bbox, diag, _ = orc.mesh_info(m.verts)
    btri = orc.bbox_face_tris(m.verts, m.tris, bbox, diag)
    return m, s, bits[:, 0], bbox, btri, gr


def test_config1_setups(orc, cfg1_axes):
    m, s, b6, bbox, btri, gr = cfg1_axes
    assert gr.sum() == 0
    cls, code = orc.reach_classes(s["point"], s["tri"], b6, bbox, btri, 50.0)
    h = orc.code_histogram(cls, code)
    assert orc.min_setups_exact(h) == (2, 0b010001)   # {+X, +Z}
    assert orc.min_setups_greedy(h)[0] == 2
    assert not np.any(cls == 2)


def test_config1_reach_thresholds(orc, cfg1_axes):
    m, s, b6, bbox, btri, _ = cfg1_axes
    p = s["point"].astype(np.float64)
    n = s["normal"]
    h1_floor = (np.abs(p[:, 2] - 28) < 1e-4) & (n[:, 2] == 1) & (np.hypot(p[:, 0] - 75, p[:, 1] - 30) < 4)
    pocket_floor = (np.abs(p[:, 2] - 25) < 1e-4) & (n[:, 2] == 1)
    assert h1_floor.sum() > 0 and pocket_floor.sum() > 0
    for L, h1_viable, pf_viable in [(11.99, False, False), (12.01, True, False), (14.99, True, False), (15.01, True, True)]:
        cls, _ = orc.reach_classes(s["point"], s["tri"], b6, bbox, btri, L)
        assert np.all((cls[h1_floor] == 0) == h1_viable)
        assert np.all((cls[pocket_floor] == 0) == pf_viable)
        assert np.all(cls[h1_floor | pocket_floor] != 2)


def test_setups_greedy_suboptimal(orc):
    C, A, B = 1, 2, 4         # directions 0 (+X), 1 (-X), 2 (+Y)
    h = np.zeros(64, np.int64)
    h[A | C] = 3              # x1, x2 and z: covered by A and by C
    h[A] = 2                  # x3, x4
    h[B | C] = 2              # y1, y2
    h[B] = 2                  # y3, y4
    # A and C both cover 5, the tie goes to C (lowest index); then A and B
    assert orc.min_setups_greedy(h) == (3, A | B | C)
    assert orc.min_setups_exact(h) == (2, A | B)


def test_setups_exact_small_cases(orc):
    h = np.zeros(64, np.int64)
    assert orc.min_setups_exact(h) == (0, 0)
    for c in (1, 2, 4):
        h[c] = 1
    assert orc.min_setups_exact(h) == (3, 7)
    h = np.zeros(64, np.int64)
    for c in (3, 6, 12, 24, 48, 33):   # a 6-cycle needs 3
        h[c] = 5
    assert orc.min_setups_exact(h) == (3, 0b010101)
    h = np.zeros(64, np.int64)
    h[63] = 10
    assert orc.min_setups_exact(h) == (1, 1)


def test_setups_exact_is_minimum_bruteforce(orc):
    rng = np.random.default_rng(3)
    for _ in range(200):
        h = np.zeros(64, np.int64)
        for c in rng.integers(1, 64, rng.integers(1, 8)):
            h[c] += 1
        k, mask = orc.min_setups_exact(h)
        codes = [c for c in range(64) if h[c]]
        assert all(c & mask for c in codes) and bin(mask).count("1") == k
        for sub in itertools.product([0, 1], repeat=6):
            mm = sum(b << i for i, b in enumerate(sub))
            if all(c & mm for c in codes):
                assert bin(mm).count("1") >= k
        g, gm = orc.min_setups_greedy(h)
        assert g >= k and all(c & gm for c in codes)


def _wedge():
    """Convex triangular prism: cross-section (0,0),(8,0),(0,6) in (x,z),
    extruded along y; its slanted face has normal (0.6, 0, 0.8)."""
    prof = [(0, 0), (8, 0), (0, 6)]
    v = np.array([[x, 0, z] for x, z in prof] + [[x, 10, z] for x, z in prof], np.float32)
    t = np.array([(0, 2, 1), (3, 4, 5), (0, 1, 4), (0, 4, 3), (1, 2, 5), (1, 5, 4), (2, 0, 3), (2, 3, 5)], np.int32)
    # convex: wind every triangle so its normal points away from the centre
    c = v.mean(0)
    tv = v[t]
    nrm = np.cross(tv[:, 1] - tv[:, 0], tv[:, 2] - tv[:, 0])
    flip = np.einsum("ij,ij->i", nrm, tv.mean(1) - c) < 0
    t[flip] = t[flip][:, ::-1]
    m = P.Mesh(v, t, "wedge")
    assert P.is_watertight(m)
    return m


def test_dirstats_tilted_open_face(orc):
    """A face of a convex part sees its whole hemisphere.  For the tilted
    normal n = (0.6, 0, 0.8) the continuum values are m = n/2 and
    A_k = E|d_k| over the hemisphere about n, found here by quadrature in
    spherical coordinates; directions of the hemisphere reach z < 0, so the
    mean of |d_z| differs from |m_z|."""
    m = _wedge()
    s = orc.sample_area(m.verts, m.tris, 3000, 4)
    sel = np.abs(s["normal"][:, 0] - 0.6) < 1e-5
    s = {k: v[sel][:40] for k, v in s.items()}
    N = 4096
    d = orc.fibonacci_dirs(N)
    bits, gr, _ = orc.cast(m.verts, m.tris, s, d)
    assert gr.sum() == 0 and np.all(bits == 0xFFFFFFFF)
    st = orc.dirstats(s, d, bits)
    n = np.array([0.6, 0.0, 0.8])
    e1 = np.array([0.8, 0.0, -0.6])
    e2 = np.cross(n, e1)
    th = (np.arange(2000) + 0.5) / 2000 * (np.pi / 2)
    ph = (np.arange(4000) + 0.5) / 4000 * (2 * np.pi)
    T, Ph = np.meshgrid(th, ph, indexing="ij")
    w = np.sin(T)
    D = (np.sin(T) * np.cos(Ph))[..., None] * e1 + (np.sin(T) * np.sin(Ph))[..., None] * e2 + np.cos(T)[..., None] * n
    A = (np.abs(D) * w[..., None]).sum((0, 1)) / w.sum()
    c = A[2] / A.sum()
    assert np.all(st["axis"] == 2)
    assert np.allclose(st["mean"], 0.5 * n, atol=2e-3)
    assert np.allclose(st["absmean"], A, atol=2e-3)
    assert np.all(np.abs(st["conc"] - c) < 2e-3)
    assert A[2] - 0.4 > 0.05      # the tilted face's |d_z| mean is not |m_z|


# ---------------------------------------------------------------- inclined bores
from closed_forms import bore_closed_form, bore_floor_sample  # noqa: E402


def test_inclined_bore_floor_closed_form(orc):
    # same seed and layout as the 1M-triangle multi-axis part, coarse tessellation
    m = P._procedural(3, 1.0, "multiaxis", None, None)
    bores = [f for f in m.meta["features"] if f["kind"] == "bore"]
    assert len(bores) >= 3
    N = 1024
    d = orc.fibonacci_dirs(N)
    for f in bores:
        s = bore_floor_sample(orc, m, f)
        assert np.allclose(s["normal"][0], np.array(f["axis"]) / np.linalg.norm(f["axis"]), atol=1e-5)
        bits, gr, _ = orc.cast(m.verts, m.tris, s, d)
        got = orc.unpack_bits(bits, N)[0]
        want, keep = bore_closed_form(f, s["origin"][0], orc.ray_dirs(s["normal"], d)[0])
        assert keep.sum() >= N - 3
        assert np.array_equal(got[keep], want[keep])
        assert want.sum() > 0

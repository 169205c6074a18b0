"""Input generator validity: watertight, outward-wound, non-overlapping
meshes (the premise of any-hit accessibility on a closed part)."""
import numpy as np
import pytest

from synth import parts as P

NAMED = [P.config1_part, P.box_part, P.blind_hole_part, P.pocket_part, P.tetrahedron,
         P.stacked_boxes, P.l_bracket, P.icosphere, P.thin_plate]


@pytest.mark.parametrize("fn", NAMED, ids=lambda f: f.__name__)
def test_named_parts_watertight(fn):
    m = fn()
    r = P.check_watertight(m)
    assert r["dup_directed_edges"] == 0 and r["unmatched_edges"] == 0, r
    assert r["zero_area"] == 0 and r["volume"] > 0, r


def test_config1_shape():
    m = P.config1_part()
    lo, hi = m.bbox()
    assert np.allclose(lo, 0) and np.allclose(hi, [100, 60, 40])
    assert 1400 <= m.n_tris <= 2000
    # volume = block - pocket - 2 holes (160-gon area = 0.5 k r^2 sin(2pi/k))
    k, r = 160, 4.0
    hole = 0.5 * k * r * r * np.sin(2 * np.pi / k) * 12.0
    want = 100 * 60 * 40 - 40 * 20 * 15 - 2 * hole
    assert abs(P.signed_volume(m.verts, m.tris) - want) < 1e-3 * want


@pytest.mark.parametrize("seed,family", [(7, "pockets"), (8, "multiaxis"), (9, "pockets"), (10, "multiaxis")])
def test_procedural_small_valid(seed, family):
    m = P._procedural(seed, 1.0, family, (120.0, 90.0, 60.0), (6, 10))
    assert P.is_watertight(m)
    cover, n = P.planar_overlap(m, 0.25)
    assert cover == 1 and n > 0


def test_procedural_interactive_size():
    m = P.procedural_part(2, 200_000, "pockets")
    assert P.is_watertight(m)
    assert abs(m.n_tris - 200_000) < 0.1 * 200_000


def test_planar_overlap_detects_overlap():
    m = P.box_part()
    dup = P.Mesh(m.verts, np.concatenate([m.tris, m.tris[:1]]), "dup")
    assert P.planar_overlap(dup, 0.5)[0] == 2


def test_generator_deterministic():
    a = P._procedural(11, 1.5, "multiaxis", None, None)
    b = P._procedural(11, 1.5, "multiaxis", None, None)
    assert np.array_equal(a.verts, b.verts) and np.array_equal(a.tris, b.tris)


def test_paper_shape_parts():
    """Stand-ins for the paper's two case-study shapes (Table 3 face counts)."""
    h = P.workload_parts("paper_housing_22k")[0]
    assert P.is_watertight(h) and abs(h.n_tris - 22_530) < 0.03 * 22_530
    m = P.workload_parts("paper_impeller_124k")[0]
    r = P.check_watertight(m)   # every shell closed: the hub and each blade
    assert r["dup_directed_edges"] == 0 and r["unmatched_edges"] == 0 and r["zero_area"] == 0, r
    assert abs(m.n_tris - 123_958) < 0.01 * 123_958
    # volume: the hub's k-gon annulus plus 12 blades of rectangular section
    # t x h(s) swept along the spiral centreline
    k = int(round(len(np.unique(np.round(np.arctan2(m.verts[:, 1], m.verts[:, 0])[m.verts[:, 2] == 0], 9)))))
    hub = 0.5 * k * (60.0 ** 2 - 10.0 ** 2) * np.sin(2 * np.pi / k) * 20.0
    s = np.linspace(0, 1, 20001)
    r_, th = 16.0 + 42.0 * s, np.radians(60.0) * s ** 1.5
    ds = np.hypot(np.gradient(r_ * np.cos(th), s), np.gradient(r_ * np.sin(th), s))
    blade = np.trapezoid(2.0 * (35.0 - 23.0 * s) * ds, s)
    want = hub + 12 * blade
    assert abs(P.signed_volume(m.verts, m.tris) - want) < 5e-3 * want, (P.signed_volume(m.verts, m.tris), want)
    lo, hi = m.bbox()
    assert np.allclose(lo[2], 0.0) and np.isclose(hi[2], 55.0)

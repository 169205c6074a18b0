"""The oracle's padded-hierarchy cast against its brute-force cast.

oracle.BVHCast must give the brute-force bits on every ray brute force
decides, flag a subset of its grazing rays (equal on every mesh here), and
carry the same informational exact-sign bit.  Cases: config 1 in full, the
tiny meshes, small procedural and batch parts (up to 20k triangles), the six
axes, crafted rays through lattice edges and vertices (many grazing rays),
interior origins, rows of the full-size interactive part, and a planted
mistake (boxes shrunk instead of grown) that the comparison must catch.
The full-size records written from this cast are checked against a fresh
oracle run on some of their blocks."""
import numpy as np
import pytest

import full_size as FS
from synth import parts as P


def _n(x):
    return int(np.unpackbits(np.ascontiguousarray(x).view(np.uint8)).sum())


def _same(orc, m, s, dirs, kind=0, b=None):
    ob, og, oi = orc.cast(m.verts, m.tris, s, dirs, kind=kind)
    own = b is None
    b = b or orc.BVHCast(m.verts, m.tris)
    bb, bg, bi = b.cast(s, dirs, kind=kind)
    if own:
        b.close()
    # the proven relation first: equal bits where brute force decides, a
    # subset of its grazing flags
    assert not ((ob ^ bb) & ~og).any()
    assert not (bg & ~og).any()
    # and, on these meshes, equality of everything
    assert np.array_equal(ob, bb) and np.array_equal(og, bg) and np.array_equal(oi & og, bi & bg)
    return _n(og)


def test_config1_full(orc):
    m = P.config1_part()
    s = orc.sample_area(m.verts, m.tris, 1000, 1)
    _same(orc, m, s, orc.fibonacci_dirs(512))
    _same(orc, m, s, orc.axes6(), kind=1)


@pytest.mark.parametrize("name", ["tetrahedron", "stacked_boxes", "l_bracket", "icosphere", "thin_plate",
                                  "blind_hole_part", "pocket_part", "box_part"])
def test_tiny_meshes(orc, name):
    m = getattr(P, name)()
    s = orc.sample_area(m.verts, m.tris, 150, 4)
    _same(orc, m, s, orc.fibonacci_dirs(256))
    _same(orc, m, s, orc.fibonacci_dirs(150))
    _same(orc, m, s, orc.axes6(), kind=1)


@pytest.mark.parametrize("which", ["pockets", "multiaxis", "batch0", "batch3", "batch5"])
def test_small_parts(orc, which):
    if which == "pockets":
        m = P._procedural(7, 1.0, "pockets", (120.0, 90.0, 60.0), (6, 10))
    elif which == "multiaxis":
        m = P._procedural(8, 1.0, "multiaxis", (120.0, 90.0, 60.0), (4, 8))
    else:
        m = P.batch_part(int(which[5:]))
    assert m.n_tris <= 20_000
    s = orc.sample_area(m.verts, m.tris, 120, 17)
    _same(orc, m, s, orc.fibonacci_dirs(512))
    _same(orc, m, s, orc.axes6(), kind=1)


def _lattice_samples(m, z_above, step):
    """Origins above the part at lattice positions (x, y multiples of
    `step`), normal -Z, so the -Z axis ray runs exactly through cell edges
    and vertices of the top and bottom faces, and +-X/+-Y rays along rows of
    cells at the origin's height."""
    lo, hi = m.verts.min(0), m.verts.max(0)
    xs = np.arange(lo[0], hi[0] + 1e-3, step, dtype=np.float32)
    ys = np.arange(lo[1], hi[1] + 1e-3, step, dtype=np.float32)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    o = np.stack([X.ravel(), Y.ravel(), np.full(X.size, z_above, np.float32)], 1).astype(np.float32)
    n = np.tile(np.array([[0, 0, -1]], np.float32), (len(o), 1))
    return {"point": o, "normal": n, "origin": o, "tri": np.zeros(len(o), np.int32)}


def test_crafted_grazing_rays(orc):
    """Rays exactly through shared edges and vertices: many grazing flags,
    and the two casts agree on every one."""
    m = P.box_part()
    s = _lattice_samples(m, 50.0, 5.0)
    g = _same(orc, m, s, orc.axes6(), kind=1)
    assert g > 50
    # origins at a lattice height inside the box's x-y range but above it:
    # the horizontal rays run along nothing; from inside the solid they hit
    s2 = _lattice_samples(m, 20.0, 10.0)
    _same(orc, m, s2, orc.axes6(), kind=1)
    m1 = P.config1_part()
    s3 = _lattice_samples(m1, 60.0, 2.5)
    assert _same(orc, m1, s3, orc.axes6(), kind=1) > 0


def test_interior_origins_blocked(orc):
    m = P.config1_part()
    pts = np.array([[5, 5, 5], [95, 55, 5], [60, 10, 20], [20, 50, 35], [85, 45, 10]], np.float32)
    rng = np.random.default_rng(2)
    nrm = rng.normal(size=(len(pts), 3))
    nrm = (nrm / np.linalg.norm(nrm, axis=1)[:, None]).astype(np.float32)
    s = {"point": pts, "normal": nrm, "origin": pts, "tri": np.zeros(len(pts), np.int32)}
    b = orc.BVHCast(m.verts, m.tris)
    bits, gr, _ = b.cast(s, orc.fibonacci_dirs(1024))
    assert not bits.any()   # (a ray through a shared edge may be flagged grazing instead)
    _same(orc, m, s, orc.fibonacci_dirs(1024), b=b)


def test_planted_shrunk_boxes_are_caught(orc):
    """Boxes shrunk by 1e-3 of the diagonal (a traversal that can skip
    triangles the ray meets) must disagree with brute force: the comparison
    above is sensitive to a pruning mistake."""
    m = P.config1_part()
    s = orc.sample_area(m.verts, m.tris, 300, 1)
    d = orc.fibonacci_dirs(512)
    ob, og, _ = orc.cast(m.verts, m.tris, s, d)
    bad = orc.BVHCast(m.verts, m.tris, pad_frac=-1e-3)
    bb, bg, _ = bad.cast(s, d)
    assert ((ob ^ bb) & ~og).any()


def test_zero_pad_keeps_the_proven_relation(orc):
    """With no growth at all the box test is still conservative: equal bits
    where brute force decides, grazing flags a subset."""
    m = P._procedural(7, 1.0, "pockets", (120.0, 90.0, 60.0), (6, 10))
    s = orc.sample_area(m.verts, m.tris, 100, 5)
    d = orc.fibonacci_dirs(512)
    ob, og, _ = orc.cast(m.verts, m.tris, s, d)
    b = orc.BVHCast(m.verts, m.tris, pad_frac=0.0)
    bb, bg, _ = b.cast(s, d)
    assert not ((ob ^ bb) & ~og).any() and not (bg & ~og).any()


def test_full_size_rows_interactive(orc):
    """Eight rows of the full-size interactive part (204.5k triangles, 4096
    directions): brute force and the hierarchy agree."""
    m = P.workload_parts("interactive_200k")[0]
    s = orc.sample_area(m.verts, m.tris, 100_000, 2)
    rows = np.sort(np.random.default_rng(11).choice(100_000, 8, replace=False))
    sub = {k: v[rows] for k, v in s.items()}
    _same(orc, m, sub, orc.fibonacci_dirs(4096))


@pytest.mark.parametrize("name", ["interactive_200k", "multiaxis_1m", "paper_housing_22k", "paper_impeller_124k",
                                  "batch64"])
def test_full_size_records_reproduce(orc, name):
    """A stored record is what the oracle computes: mesh and sample hashes,
    two blocks of rows re-cast, the grazing share within 1e-4, and the
    statistics' own invariants."""
    rec_all = FS.load(name)
    N = rec_all["n_dirs"]
    idx = [0, 41] if name == "batch64" else [0]
    for i in idx:
        rec = rec_all["parts"][i]
        m = P.batch_part(i) if name == "batch64" else P.workload_parts(name)[0]
        assert FS.array_sha256(m.verts, m.tris) == rec["mesh_sha256"]
        smp = rec["samples"]
        s = (orc.sample_area(m.verts, m.tris, smp["n"], smp["seed"]) if smp["mode"] == "area"
             else orc.sample_centroid(m.verts, m.tris))
        assert FS.array_sha256(s["point"], s["normal"], s["origin"], s["tri"]) == smp["sha256"]
        h = rec["hemi"]
        S = smp["n"]
        assert h["n_grazing"] <= 1e-4 * S * N and rec["axes"]["n_grazing"] <= 1e-4 * S * 6
        b = orc.BVHCast(m.verts, m.tris)
        nblk = len(h["digests"])
        for blk in sorted({0, nblk // 2, nblk - 1})[:2]:
            r0, r1 = blk * h["chunk"], min(S, (blk + 1) * h["chunk"])
            bits, gr, _ = b.cast(s, orc.fibonacci_dirs(N), s0=r0, s1=r1)
            gsel = [(r - r0, d) for r, d in zip(h["grazing_rows"], h["grazing_dirs"]) if r0 <= r < r1]
            rr, dd = FS.flagged(gr)
            assert sorted(zip(rr.tolist(), dd.tolist())) == sorted(gsel)
            assert FS.chunk_digests(FS.cleared(bits, rr, dd), h["chunk"])[0] == h["digests"][blk]
        b.close()
        st = rec["stats"]
        assert abs(sum(st["shares"]) - 1.0) < 1e-12 or st["n_included"] == 0
        if st["hist"] is not None:
            assert int(FS.unpack_hist(st["hist"]).sum()) == h["n_free"]
        assert abs(st["access"] - h["n_free"] / (S * N)) < 1e-15
        su = rec["setups"]
        assert sum(su["n_class"]) == S and sum(su["code_hist"]) == su["n_class"][0]

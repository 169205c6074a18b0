"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.  Bit-exact for direction tables, samples, rays, bits
(grazing rays excluded), classes and setups; FP tolerances as stated."""
import math
import sys

import numpy as np
import pytest

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


@pytest.fixture(scope="module")
def cfg1(ctx):
    m = P.config1_part()
    b = ctx.build_bvh(m.verts, m.tris, leaf_size=4)
    return m, b


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _np_samples(s):
    return {k: v.cpu().numpy() for k, v in s.items()}


# ---------------------------------------------------------------- tables, mesh, samples
@pytest.mark.parametrize("n", [1, 6, 33, 150, 512, 1000, 1024, 2048, 4096, 8192])
def test_direction_table_bit_exact(ctx, orc, n):
    _say("dirs", n)
    assert np.array_equal(ctx.dirs_table(n), orc.fibonacci_dirs(n))


def test_axes6_table(ctx, orc):
    from paper_2609_05467_amd import hra
    assert np.array_equal(ctx.dirs_table(6, hra.DIRS_AXES6), orc.axes6())


def test_bvh_info_config1(ctx, orc, cfg1):
    m, b = cfg1
    _say("bvh info config1")
    inf = b.info()
    bbox, diag, _ = orc.mesh_info(m.verts)
    assert list(inf.bbox) == list(bbox.astype(np.float32))
    assert inf.diag == diag
    assert inf.n_tris == m.n_tris and inf.n_degenerate == 0
    assert 1 <= inf.depth <= 64 and inf.n_nodes > 0


@pytest.mark.parametrize("name", ["config1", "pockets-small", "multiaxis-small", "tetrahedron"])
def test_area_samples_bit_exact(ctx, orc, name):
    m = {"config1": P.config1_part, "tetrahedron": P.tetrahedron,
         "pockets-small": lambda: P._procedural(7, 1.0, "pockets", (120.0, 90.0, 60.0), (6, 10)),
         "multiaxis-small": lambda: P._procedural(8, 1.0, "multiaxis", (120.0, 90.0, 60.0), (4, 8))}[name]()
    _say("samples", name, m.n_tris)
    b = ctx.build_bvh(m.verts, m.tris)
    for seed, n in [(1, 1000), (12345, 4097)]:
        s = _np_samples(ctx.sample_surface(b, n, seed))
        o = orc.sample_area(m.verts, m.tris, n, seed)
        for k in ("tri", "point", "normal", "origin"):
            assert np.array_equal(s[k], o[k]), (name, seed, k)


def test_centroid_samples_bit_exact(ctx, orc, cfg1):
    from paper_2609_05467_amd import hra
    m, b = cfg1
    s = _np_samples(ctx.sample_surface(b, 0, 0, mode=hra.SAMPLE_CENTROID))
    o = orc.sample_centroid(m.verts, m.tris)
    for k in ("tri", "point", "normal", "origin"):
        assert np.array_equal(s[k], o[k]), k


def test_debug_rays_bit_exact(ctx, orc, cfg1):
    m, b = cfg1
    s = ctx.sample_surface(b, 300, 3)
    N = 512
    idx = np.arange(0, 300, 7)
    r = ctx.debug_rays(s, N, idx).cpu().numpy()
    sn = _np_samples(s)
    want = orc.ray_dirs(sn["normal"][idx], orc.fibonacci_dirs(N))
    assert np.array_equal(r[:, :, 3:], want)
    assert np.array_equal(r[:, :, :3], np.repeat(sn["origin"][idx][:, None, :], N, 1))


# ---------------------------------------------------------------- casting
def _cast_parity(ctx, orc, m, b, S, N, seed, kind=0, s=None, max_grazing=1e-4):
    from paper_2609_05467_amd import hra
    if s is None:
        s = ctx.sample_surface(b, S, seed)
    sn = _np_samples(s)
    dirs = orc.fibonacci_dirs(N) if kind == 0 else orc.axes6()
    bits, cnt = ctx.cast(b, s, N, kind=hra.DIRS_HEMI if kind == 0 else hra.DIRS_AXES6)
    got = _u32(bits)
    ob, og, _ = orc.cast(m.verts, m.tris, sn, dirs, kind=kind)
    keep = ~og
    bad = (got ^ ob) & keep
    assert not bad.any(), f"{int(np.unpackbits(bad.view(np.uint8)).sum())} non-grazing rays differ"
    W = (N + 31) // 32
    tail = np.uint32((1 << (N % 32)) - 1) if N % 32 else np.uint32(0xFFFFFFFF)
    assert np.all(got[:, W - 1] & ~tail == 0), "bits beyond N must be zero"
    graze = int(np.unpackbits(og.view(np.uint8)).sum())
    assert graze <= max_grazing * S * N + 1e-9, graze
    popc = np.array([int(np.unpackbits(r.view(np.uint8)).sum()) for r in got])
    assert np.array_equal(_u32(cnt), popc.astype(np.uint32))
    return s, got, ob, og


def test_cast_config1_full(ctx, orc, cfg1):
    m, b = cfg1
    _say("cast config1 1000 x 512")
    _cast_parity(ctx, orc, m, b, 1000, 512, 1)


@pytest.mark.parametrize("N", [1, 33, 64, 100, 150, 1000])
def test_cast_ragged_direction_counts(ctx, orc, cfg1, N):
    m, b = cfg1
    _say("cast ragged N", N)
    _cast_parity(ctx, orc, m, b, 77, N, 5)


@pytest.mark.parametrize("leaf", [1, 2, 4, 8, 12, 16])
def test_cast_leaf_sizes(ctx, orc, leaf):
    m = P._procedural(9, 1.0, "pockets", (120.0, 90.0, 60.0), (6, 10))
    _say("leaf", leaf, m.n_tris)
    b = ctx.build_bvh(m.verts, m.tris, leaf_size=leaf)
    _cast_parity(ctx, orc, m, b, 120, 256, 2)


@pytest.mark.parametrize("name", ["tetrahedron", "stacked_boxes", "l_bracket", "icosphere", "box"])
def test_cast_tiny_meshes(ctx, orc, name):
    m = getattr(P, name if name != "box" else "box_part")()
    _say("tiny", name)
    b = ctx.build_bvh(m.verts, m.tris)
    _cast_parity(ctx, orc, m, b, 200, 256, 4)
    _cast_parity(ctx, orc, m, b, 200, 6, 4, kind=1)


def test_cast_multiaxis_part(ctx, orc):
    m = P._procedural(10, 1.0, "multiaxis", (120.0, 90.0, 60.0), (4, 8))
    _say("multiaxis part", m.n_tris)
    b = ctx.build_bvh(m.verts, m.tris)
    _cast_parity(ctx, orc, m, b, 150, 512, 6)
    _cast_parity(ctx, orc, m, b, 400, 6, 6, kind=1)


def test_cast_configs_identical(ctx, orc, cfg1):
    """Every launch shape and both traversal loops give the same bits, for
    the hemisphere and the six-axis casts, and the same work counts."""
    from paper_2609_05467_amd import hra
    m, b = cfg1
    s = ctx.sample_surface(b, 300, 8)
    ref = ref6 = None
    for trav in (hra.TRAVERSAL_STEP, hra.TRAVERSAL_LEAF_LOOP, hra.TRAVERSAL_REFILL):
        for rpw in (64, 128, 256):
            for st in (16, 20, 24, 32):
                _say("config", trav, rpw, st)
                ctx.set_cast_config(rpw, st, 0, trav)
                bits, _ = ctx.cast(b, s, 1000)
                b6, _ = ctx.cast(b, s, 6, kind=hra.DIRS_AXES6)
                g, g6 = _u32(bits), _u32(b6)
                if ref is None:
                    ref, ref6 = g, g6
                assert np.array_equal(g, ref), (trav, rpw, st)
                assert np.array_equal(g6, ref6), (trav, rpw, st)
    works = []
    for trav in (hra.TRAVERSAL_STEP, hra.TRAVERSAL_LEAF_LOOP, hra.TRAVERSAL_REFILL):
        ctx.set_cast_config(64, 20, 0, trav)
        wb, nf, nt = ctx.cast_work(b, s, 1000)
        assert np.array_equal(_u32(wb), ref)
        works.append((nf, nt))
    assert works[0] == works[1] == works[2] and works[0][0] > 0
    ctx.set_cast_config(64, 16, 0, hra.TRAVERSAL_STEP)


@pytest.mark.parametrize("N", [1, 7, 33, 100, 150, 255, 256])
def test_cast_grouped_matches_one_sample_per_workgroup(ctx, orc, cfg1, N):
    """Several samples per workgroup (chosen or forced) give the bits of one
    sample per workgroup, on a sample count no group size divides, and the
    same work counts."""
    from paper_2609_05467_amd import hra
    m, b = cfg1
    _say("grouped", N)
    s = ctx.sample_surface(b, 211, 12)
    ctx.set_cast_config(64, 16, 0, hra.TRAVERSAL_STEP, 1)
    ref, _ = ctx.cast(b, s, N)
    ref = _u32(ref)
    _, nf1, nt1 = ctx.cast_work(b, s, N)
    for trav in (hra.TRAVERSAL_STEP, hra.TRAVERSAL_REFILL):
        for g in (0, 1, 2, 3, 5, 16):
            ctx.set_cast_config(64, 16, 0, trav, g)
            got, cnt = ctx.cast(b, s, N)
            assert np.array_equal(_u32(got), ref), (trav, g)
            wb, nf, nt = ctx.cast_work(b, s, N)
            assert np.array_equal(_u32(wb), ref) and (nf, nt) == (nf1, nt1), (trav, g)
    ctx.set_cast_config(64, 16, 0, hra.TRAVERSAL_STEP, 0)
    _cast_parity(ctx, orc, m, b, 211, N, 12, s=s)


def test_convex_box_all_free(ctx):
    m = P.box_part()
    b = ctx.build_bvh(m.verts, m.tris)
    s = ctx.sample_surface(b, 500, 9)
    bits, cnt = ctx.cast(b, s, 4096)
    assert np.all(_u32(bits) == 0xFFFFFFFF) and np.all(_u32(cnt) == 4096)


def test_blind_hole_bottom_centre_gpu(ctx, orc):
    import torch
    r, depth = 4.0, 12.0
    m = P.blind_hole_part(r, depth, 160)
    b = ctx.build_bvh(m.verts, m.tris)
    _, _, eps = orc.mesh_info(m.verts)
    cu, cv, top = m.meta["centre"]
    p = np.array([[cu, cv, top - depth]], np.float32)
    o = p.copy()
    o[0, 2] = np.float32(np.float64(p[0, 2]) + np.float64(eps))
    dev = ctx.device
    s = {"point": torch.tensor(p, device=dev), "normal": torch.tensor([[0, 0, 1.0]], device=dev),
         "origin": torch.tensor(o, device=dev), "tri": torch.zeros(1, dtype=torch.int32, device=dev)}
    for N, circle in [(512, 26), (4096, 211)]:
        bits, cnt = ctx.cast(b, s, N)
        ob, og, _ = orc.cast(m.verts, m.tris, _np_samples(s), orc.fibonacci_dirs(N))
        assert og.sum() == 0 and np.array_equal(_u32(bits), ob)
        assert abs(int(_u32(cnt)[0]) - circle) <= 3


def test_watertight_interior_gpu(ctx):
    import torch
    m = P.config1_part()
    b = ctx.build_bvh(m.verts, m.tris)
    pts = np.array([[5, 5, 5], [95, 55, 5], [60, 10, 20], [20, 50, 35], [85, 45, 10]], np.float32)
    rng = np.random.default_rng(2)
    nrm = rng.normal(size=(len(pts), 3))
    nrm = (nrm / np.linalg.norm(nrm, axis=1)[:, None]).astype(np.float32)
    dev = ctx.device
    s = {"point": torch.tensor(pts, device=dev), "normal": torch.tensor(nrm, device=dev),
         "origin": torch.tensor(pts, device=dev), "tri": torch.zeros(len(pts), dtype=torch.int32, device=dev)}
    bits, cnt = ctx.cast(b, s, 4096)
    assert np.all(_u32(cnt) == 0)


def test_empty_and_single_sample(ctx, orc, cfg1):
    m, b = cfg1
    s0 = ctx.alloc_samples(0)
    bits, cnt = ctx.cast(b, s0, 512)
    assert bits.shape == (0, 16)
    _cast_parity(ctx, orc, m, b, 1, 512, 77)


def test_degenerate_triangle_counted(ctx, orc):
    m = P.box_part()
    v = np.concatenate([m.verts, m.verts[:1]])
    t = np.concatenate([m.tris, np.array([[0, 1, len(m.verts)]], np.int32)])   # zero area: vertex 0 twice
    b = ctx.build_bvh(v, t)
    inf = b.info()
    assert inf.n_degenerate == 1
    s = _np_samples(ctx.sample_surface(b, 2000, 3))
    assert not np.any(s["tri"] == len(t) - 1)
    o = orc.sample_area(v, t, 2000, 3)
    assert np.array_equal(s["point"], o["point"])


def test_bad_index_reported(ctx):
    from paper_2609_05467_amd import hra
    m = P.box_part()
    t = m.tris.copy()
    t[5, 1] = len(m.verts) + 10
    b = ctx.build_bvh(m.verts, t)
    with pytest.raises(hra.HraError) as e:
        b.info()
    assert e.value.status == -4


# ---------------------------------------------------------------- statistics, classification, setups
def _stats_parity(ctx, orc, m, b, S, N, seed):
    s = ctx.sample_surface(b, S, seed)
    sn = _np_samples(s)
    bits, cnt = ctx.cast(b, s, N)
    ob, og, _ = orc.cast(m.verts, m.tris, sn, orc.fibonacci_dirs(N))
    got = _u32(bits)
    # the statistics are compared on the GPU's own bits, and the oracle is fed
    # the same bits (identical on all non-grazing rays)
    st = ctx.dominant_axes(s, N, bits)
    o = orc.dirstats(sn, orc.fibonacci_dirs(N), got)
    mean, absmean = st["mean"].cpu().numpy(), st["absmean"].cpu().numpy()
    axis, conc = st["axis"].cpu().numpy(), st["conc"].cpu().numpy()
    assert np.allclose(mean, o["mean"], atol=1e-5, rtol=0)
    assert np.allclose(absmean, o["absmean"], atol=1e-5, rtol=0)
    sel = ~o["tie"]
    assert np.array_equal(axis[sel], o["axis"][sel])
    assert np.allclose(conc[sel], o["conc"][sel], atol=1e-4, rtol=0)
    h = st["hist"].cpu().numpy().view(np.uint32).astype(np.int64)
    oh = o["hist"].astype(np.int64)
    assert h.sum() == oh.sum() == int(_u32(cnt).astype(np.int64).sum())
    assert np.abs(h - oh).sum() <= 2e-4 * oh.sum()
    rep = ctx.classify(st, S, N)
    ind = orc.indicators(orc.counts(got, N), N, o["axis"], o["conc"])
    assert abs(rep["access"] - ind["access"]) < 1e-12
    # the GPU and the oracle read the same bits, so a sample's axis can differ
    # only where the oracle flags a tie: each share moves by at most
    # ties / included samples (0 without ties: then equal exactly)
    n_tie = int((~sel & (o["axis"] >= 0)).sum())
    bound = n_tie / max(1, ind["n_included"])
    assert max(abs(a - b) for a, b in zip(rep["shares"], ind["shares"])) <= bound + 1e-15
    assert abs(rep["conc"] - ind["conc"]) < 1e-4
    if not rep["near_tie"]:
        assert rep["multi_axis"] == orc.classify(ind)[0]
    return s, bits


def test_stats_config1(ctx, orc, cfg1):
    m, b = cfg1
    _say("stats config1")
    _stats_parity(ctx, orc, m, b, 1000, 512, 1)


def test_stats_multiaxis(ctx, orc):
    m = P._procedural(10, 1.0, "multiaxis", (120.0, 90.0, 60.0), (4, 8))
    b = ctx.build_bvh(m.verts, m.tris)
    _say("stats multiaxis")
    _stats_parity(ctx, orc, m, b, 300, 1024, 2)


def test_classify_thresholds_and_designed_parts(ctx, orc):
    for fn, multi in [(P.thin_plate, False), (P.icosphere, True)]:
        m = fn()
        b = ctx.build_bvh(m.verts, m.tris)
        s = ctx.sample_surface(b, 400, 2)
        bits, _ = ctx.cast(b, s, 150)
        st = ctx.dominant_axes(s, 150, bits)
        assert ctx.classify(st, 400, 150)["multi_axis"] == multi


@pytest.mark.parametrize("L", [11.99, 12.01, 14.99, 15.01, 50.0])
def test_setups_config1(ctx, orc, cfg1, L):
    from paper_2609_05467_amd import hra
    m, b = cfg1
    _say("setups", L)
    s = ctx.sample_surface(b, 1000, 1)
    a6, _ = ctx.cast(b, s, 6, kind=hra.DIRS_AXES6, counts=False)
    rep = ctx.min_setups(b, s, a6, L)
    sn = _np_samples(s)
    ob, og, _ = orc.cast(m.verts, m.tris, sn, orc.axes6(), kind=1)
    assert og.sum() == 0 and np.array_equal(_u32(a6)[:, 0], ob[:, 0])
    bbox, diag, _ = orc.mesh_info(m.verts)
    cls, code = orc.reach_classes(sn["point"], sn["tri"], ob[:, 0], bbox,
                                  orc.bbox_face_tris(m.verts, m.tris, bbox, diag), L)
    assert np.array_equal(rep["class"].cpu().numpy(), cls)
    h = orc.code_histogram(cls, code)
    assert rep["code_hist"] == list(h)
    assert (rep["min_count"], rep["min_mask"]) == orc.min_setups_exact(h)
    assert (rep["greedy_count"], rep["greedy_mask"]) == orc.min_setups_greedy(h)
    if L >= 15.01:
        assert (rep["min_count"], rep["min_mask"]) == (2, 0b010001)


# Full-size workloads: every row is compared with the oracle in
# test_gpu_full_size.py.


def test_cast_work_counts(ctx, cfg1):
    m, b = cfg1
    s = ctx.sample_surface(b, 200, 4)
    bits, _ = ctx.cast(b, s, 512)
    wbits, nodes, tests = ctx.cast_work(b, s, 512)
    assert np.array_equal(_u32(wbits), _u32(bits))
    assert nodes >= 200 * 512 and tests > 0


# ---------------------------------------------------------------- full size (multi-axis stress part)
def test_multiaxis_full_size(ctx, orc):
    """1M-triangle part, 250k samples x 2048 directions in one cast (every
    row is compared with the oracle in test_gpu_full_size.py): the histogram
    of each inclined bore's floor
    samples has the same peak as the oracle's on the same bits, and
    the rays from each bore's floor centre escape exactly when they cross
    the face plane inside the rim polygon (convex cavity closed form)."""
    import torch
    from paper_2609_05467_amd import hra
    m = P.workload_parts("multiaxis_1m")[0]
    S, N = 250_000, 2048
    _say("multiaxis full", m.n_tris, S, N)
    b = ctx.build_bvh(m.verts, m.tris)
    inf = b.info()
    assert inf.n_degenerate == 0
    s = ctx.sample_surface(b, S, 3)
    bits, cnt = ctx.cast(b, s, N)
    got = _u32(bits)
    sn = _np_samples(s)
    st = ctx.dominant_axes(s, N, bits)
    h = st["hist"].cpu().numpy().view(np.uint32)
    assert int(h.astype(np.int64).sum()) == int(_u32(cnt).astype(np.int64).sum())
    dirs = orc.fibonacci_dirs(N)
    checked = 0
    for f in m.meta["features"]:
        if f["kind"] != "bore":
            continue
        t0, t1 = f["floor_tris"]
        sel = np.nonzero((sn["tri"] >= t0) & (sn["tri"] < t1))[0]
        if len(sel) < 5:
            continue
        idx = torch.tensor(sel, device=ctx.device)
        sub = {k: v[idx].contiguous() for k, v in s.items()}
        sbits = bits[idx].contiguous()
        hs = ctx.dominant_axes(sub, N, sbits)["hist"].cpu().numpy().view(np.uint32)
        pk = hra.histogram_peaks(hs, 1)
        o = orc.dirstats({k: v[sel] for k, v in sn.items()}, dirs, got[sel])
        opk = orc.histogram_peaks(o["hist"], 1)
        assert pk["bins"] == opk["bins"]
        # exact visibility from the floor centre (convex cavity, oblique rim)
        from closed_forms import bore_closed_form, bore_floor_sample
        fs = bore_floor_sample(orc, m, f)
        ts = {k: torch.tensor(v, device=ctx.device) for k, v in fs.items()}
        fb, _ = ctx.cast(b, ts, N)
        want, keep = bore_closed_form(f, fs["origin"][0], orc.ray_dirs(fs["normal"], dirs)[0])
        gotf = orc.unpack_bits(_u32(fb), N)[0]
        assert keep.sum() >= N - 3 and np.array_equal(gotf[keep], want[keep]) and want.sum() > 0
        checked += 1
    assert checked >= 3

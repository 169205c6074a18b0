"""Batches of parts: every per-part result of a batch hierarchy and of the
one-call batch path equals the result of the same part alone (bit for bit:
hierarchy shape, samples, bitmasks, statistics, class, setups), and the
batch bitmasks agree with the oracle directly."""
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
def meshes():
    return [P.config1_part(), P.box_part(), P.blind_hole_part(),
            P._procedural(11, 1.0, "multiaxis", (100.0, 80.0, 50.0), (4, 8)), P.tetrahedron(), P.pocket_part(),
            P._procedural(12, 1.0, "pockets", (120.0, 90.0, 60.0), (6, 10))]


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _np(s):
    return {k: v.cpu().numpy() for k, v in s.items()}


def test_batch_hierarchy_parts_match_alone(ctx, meshes):
    from paper_2609_05467_amd import hra
    _say("batch hierarchy", [m.n_tris for m in meshes])
    bb = ctx.build_bvh_batch([(m.verts, m.tris) for m in meshes], leaf_size=4)
    assert bb.n_parts == len(meshes)
    for p, m in enumerate(meshes):
        _say("part", p, m.n_tris)
        ba = ctx.build_bvh(m.verts, m.tris, leaf_size=4)
        ia, ib = ba.info(), bb.info(part=p)
        for f in ("diag", "n_tris", "n_degenerate", "n_nodes", "depth", "leaf_size"):
            assert getattr(ia, f) == getattr(ib, f), (p, f)
        assert list(ia.bbox) == list(ib.bbox)
        n = 700 + 97 * p
        sa = ctx.sample_surface(ba, n, 5 + p)
        sb = ctx.sample_surface(bb, n, 5 + p, part=p)
        for k in ("point", "normal", "origin", "tri"):
            assert np.array_equal(sa[k].cpu().numpy(), sb[k].cpu().numpy()), (p, k)
        ca = ctx.sample_surface(ba, 0, 0, mode=hra.SAMPLE_CENTROID)
        cb = ctx.sample_surface(bb, 0, 0, mode=hra.SAMPLE_CENTROID, part=p)
        for k in ("point", "normal", "origin", "tri"):
            assert np.array_equal(ca[k].cpu().numpy(), cb[k].cpu().numpy()), (p, "centroid", k)
        for N in (300, 1024):
            xa, na = ctx.cast(ba, sa, N)
            xb, nb = ctx.cast(bb, sa, N, part=p)
            assert np.array_equal(_u32(xa), _u32(xb)), (p, N)
            assert np.array_equal(na.cpu().numpy(), nb.cpu().numpy()), (p, N)
        a6, _ = ctx.cast(ba, sa, 6, kind=hra.DIRS_AXES6)
        b6, _ = ctx.cast(bb, sa, 6, kind=hra.DIRS_AXES6, part=p)
        assert np.array_equal(_u32(a6), _u32(b6)), p
        ra = ctx.min_setups(ba, sa, a6, 30.0)
        rb = ctx.min_setups(bb, sa, b6, 30.0, part=p)
        for k in ("min_count", "min_mask", "greedy_count", "greedy_mask", "n_class", "code_hist"):
            assert ra[k] == rb[k], (p, k)
        assert np.array_equal(ra["class"].cpu().numpy(), rb["class"].cpu().numpy()), p
        ba.release()
    bb.release()


def test_batch_part_index_checked(ctx, meshes):
    from paper_2609_05467_amd import hra
    bb = ctx.build_bvh_batch([(m.verts, m.tris) for m in meshes[:2]])
    s = ctx.alloc_samples(10)
    with pytest.raises(hra.HraError):
        ctx.sample_surface(bb, 10, 1, part=2, out=s)
    with pytest.raises(hra.HraError):
        ctx.cast(bb, s, 64, part=-1)
    with pytest.raises(hra.HraError):
        bb.info(part=5)
    with pytest.raises(ValueError):
        bb.export()
    bb.release()


def _single(ctx, m, n, seed, N, tool, leaf=4):
    from paper_2609_05467_amd import hra
    b = ctx.build_bvh(m.verts, m.tris, leaf_size=leaf)
    s = ctx.sample_surface(b, n, seed)
    bits, _ = ctx.cast(b, s, N, counts=False)
    ds = ctx.dominant_axes(s, N, bits)
    rep = ctx.classify(ds, n, N)
    b6, _ = ctx.cast(b, s, 6, kind=hra.DIRS_AXES6, counts=False)
    su = ctx.min_setups(b, s, b6, tool, want_class=False)
    b.release()
    return s, bits, rep, su


@pytest.mark.parametrize("N", [150, 256, 1000])
def test_batch_run_matches_single_calls(ctx, meshes, N):
    import torch
    reqs = [{"verts": m.verts, "tris": m.tris, "n_samples": 500 + 311 * p, "seed": 100 + p,
             "tool_length": 20.0 + 5 * p} for p, m in enumerate(meshes)]
    _say("batch_run", N, [r["n_samples"] for r in reqs])
    W = (N + 31) // 32
    S = sum(r["n_samples"] for r in reqs)
    bits = torch.empty((S, W), dtype=torch.int32, device=ctx.device)
    res = ctx.batch_run(reqs, N, leaf_size=4, bits=bits)
    got = _u32(bits)
    off = 0
    for p, (m, r) in enumerate(zip(meshes, reqs)):
        _say("compare part", p)
        _, b1, rep, su = _single(ctx, m, r["n_samples"], r["seed"], N, r["tool_length"])
        n = r["n_samples"]
        assert np.array_equal(got[off:off + n], _u32(b1)), p
        assert res[p]["class"] == rep, p
        for k in ("min_count", "min_mask", "greedy_count", "greedy_mask", "n_class", "code_hist"):
            assert res[p]["setups"][k] == su[k], (p, k)
        off += n


def test_batch_run_bits_vs_oracle(ctx, orc, meshes):
    """Direct check of the batch bitmasks against the oracle (grazing rays
    excluded) for two parts of different size in one batch."""
    import torch
    ms = [meshes[0], meshes[3]]
    N = 512
    reqs = [{"verts": m.verts, "tris": m.tris, "n_samples": 400, "seed": 9 + p, "tool_length": 40.0}
            for p, m in enumerate(ms)]
    bits = torch.empty((800, N // 32), dtype=torch.int32, device=ctx.device)
    ctx.batch_run(reqs, N, bits=bits)
    got = _u32(bits)
    dirs = orc.fibonacci_dirs(N)
    for p, m in enumerate(ms):
        o = orc.sample_area(m.verts, m.tris, 400, 9 + p)
        ob, og, _ = orc.cast(m.verts, m.tris, o, dirs)
        bad = (got[400 * p:400 * (p + 1)] ^ ob) & ~og
        assert not bad.any(), p


def test_batch_run_single_part_and_limits(ctx, meshes):
    from paper_2609_05467_amd import hra
    m = meshes[0]
    r = ctx.batch_run([{"verts": m.verts, "tris": m.tris, "n_samples": 300, "seed": 4, "tool_length": 50.0}], 128)
    _, _, rep, su = _single(ctx, m, 300, 4, 128, 50.0)
    assert r[0]["class"] == rep and r[0]["setups"]["min_count"] == su["min_count"]
    with pytest.raises(hra.HraError):
        ctx.batch_run([{"verts": m.verts, "tris": m.tris, "n_samples": 0, "seed": 4, "tool_length": 50.0}], 128)
    with pytest.raises(hra.HraError):
        ctx.batch_run([], 128)


def _reqs(ms, base_n=400):
    return [{"verts": m.verts, "tris": m.tris, "n_samples": base_n + 137 * p, "seed": 50 + p,
             "tool_length": 25.0 + 3 * p} for p, m in enumerate(ms)]


@pytest.mark.parametrize("rpw,stack,leaf,trav", [(64, 24, 4, 1), (128, 16, 2, 2), (256, 32, 8, 1), (64, 20, 4, 2)])
def test_plan_eager_matches_batch_run(ctx, meshes, rpw, stack, leaf, trav):
    import torch
    reqs = _reqs(meshes)
    N = 777
    W = (N + 31) // 32
    S = sum(r["n_samples"] for r in reqs)
    _say("plan eager", rpw, stack, leaf, trav)
    b0 = torch.empty((S, W), dtype=torch.int32, device=ctx.device)
    b1 = torch.empty_like(b0)
    want = ctx.batch_run(reqs, N, leaf_size=4, bits=b0)
    pl = ctx.plan(reqs, N, leaf_size=leaf, rays_per_wave=rpw, stack_depth=stack, traversal=trav)
    got = pl.run(graph=False, bits=b1)
    assert got == want
    assert torch.equal(b0, b1)
    ms = pl.stage_ms()
    assert all(v >= 0 for v in ms.values()) and ms["cast"] > 0
    assert pl.bytes > 0
    pl.destroy()


def test_plan_graph_replays_match_eager(ctx, meshes):
    """Capture once, replay several times with other eager work and
    synchronisations between the replays; every replay equals the eager run."""
    import torch
    reqs = _reqs(meshes, 300)
    N = 512
    S = sum(r["n_samples"] for r in reqs)
    pl = ctx.plan(reqs, N)
    be = torch.empty((S, N // 32), dtype=torch.int32, device=ctx.device)
    want = pl.run(graph=False, bits=be)
    m = meshes[0]
    b = ctx.build_bvh(m.verts, m.tris)
    for k in range(4):
        _say("graph replay", k)
        bg = torch.full((S, N // 32), -1, dtype=torch.int32, device=ctx.device)
        got = pl.run(graph=True, bits=bg)
        torch.cuda.synchronize()
        assert got == want, k
        assert torch.equal(bg, be), k
        # eager work between replays
        s = ctx.sample_surface(b, 200, 7 + k)
        ctx.cast(b, s, 256)
        torch.cuda.synchronize()
    b.release()
    pl.destroy()


def test_autotune_picks_a_point_and_keeps_results(ctx, meshes):
    from paper_2609_05467_amd import hra
    reqs = _reqs(meshes[:3], 300)
    old = ctx.cast_config()
    _say("autotune")
    rep = ctx.autotune(reqs, 256, reps=1)
    assert len(rep["points"]) == 27
    assert {(p["rays_per_wave"], p["stack_depth"], p["leaf_size"]) for p in rep["points"]} == {
        (r, st, lf) for r in (64, 128, 256) for st in (16, 24, 32) for lf in (2, 4, 8)}
    assert {p["traversal"] for p in rep["points"]} == {old[3]}
    best = rep["best"]
    assert best["ms"] == min(p["ms"] for p in rep["points"])
    assert ctx.cast_config()[:4] == (best["rays_per_wave"], best["stack_depth"], best["leaf_size"], best["traversal"])
    # results of a single-part cast do not depend on the tuned shape
    m = meshes[0]
    b = ctx.build_bvh(m.verts, m.tris)
    s = ctx.sample_surface(b, 300, 3)
    x1, _ = ctx.cast(b, s, 256)
    ctx.set_cast_config(*old)
    b2 = ctx.build_bvh(m.verts, m.tris)
    x2, _ = ctx.cast(b2, s, 256)
    assert np.array_equal(_u32(x1), _u32(x2))
    b.release()
    b2.release()


def test_batch64_full_size_matches_single_parts(ctx, orc, tmp_path):
    """The 64-part workload at full size (2.9k-412k triangles, 1.5M samples
    x 1,024 directions) in one plan run replayed as a graph: every part's
    bits, class and setups equal its single-part run, and sampled rows of
    the smaller parts agree with the oracle (grazing rays excluded)."""
    import subprocess
    import torch
    from paper_2609_05467_amd import hra
    # generate in a child process (the generator forks workers; this process
    # has the GPU open)
    f = tmp_path / "parts.npz"
    code = ("import sys, numpy as np; sys.path.insert(0, %r); from synth import parts; "
            "ms = parts.batch_parts(workers=16); "
            "np.savez(%r, **{f'v{i}': m.verts for i, m in enumerate(ms)}, **{f't{i}': m.tris for i, m in enumerate(ms)})"
            % (str(P.__file__).rsplit("/synth/", 1)[0], str(f)))
    _say("generating the 64 parts")
    subprocess.run([sys.executable, "-c", code], check=True, timeout=600)
    z = np.load(f)
    meshes = [P.Mesh(z[f"v{i}"], z[f"t{i}"]) for i in range(64)]
    counts = P.batch_samples(meshes)
    N, tool = 1024, 50.0
    reqs = [{"verts": m.verts, "tris": m.tris, "n_samples": c, "seed": 400 + i, "tool_length": tool}
            for i, (m, c) in enumerate(zip(meshes, counts))]
    S = sum(counts)
    bits = torch.empty((S, N // 32), dtype=torch.int32, device=ctx.device)
    _say("plan", S, "samples")
    pl = ctx.plan(reqs, N)
    pl.run(graph=True)
    res = pl.run(graph=True, bits=bits)
    pl.destroy()
    got = _u32(bits)
    dirs = orc.fibonacci_dirs(N)
    off = 0
    for p, (m, c) in enumerate(zip(meshes, counts)):
        _say("part", p, m.n_tris, c)
        s, b1, rep, su = _single(ctx, m, c, 400 + p, N, tool)
        assert np.array_equal(got[off:off + c], _u32(b1)), p
        assert res[p]["class"] == rep, p
        for k in ("min_count", "min_mask", "greedy_count", "greedy_mask", "n_class", "code_hist"):
            assert res[p]["setups"][k] == su[k], (p, k)
        if m.n_tris < 20_000:
            rows = np.array([0, c // 2, c - 1])
            sn = {k: v.cpu().numpy()[rows] for k, v in s.items()}
            ob, og, _ = orc.cast(m.verts, m.tris, sn, dirs)
            assert not ((got[off + rows] ^ ob) & ~og).any(), p
        off += c

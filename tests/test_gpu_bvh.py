"""The hierarchy the GPU builds: a tree over every nonzero-area face, every
child box exactly the union of the triangle boxes below it, and the same
bytes on every rebuild.  The refit publishes boxes between threads of
different compute dies; a box read before its writer finished would show up
here as a box that is not the exact union, or as a difference between
builds."""
import sys

import numpy as np
import pytest

from synth import parts as P
from bvh_check import check_bvh

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


MESHES = {
    "config1": lambda: P.config1_part(),
    "icosphere": lambda: P.icosphere(subdiv=4),
    "multiaxis-small": lambda: P._procedural(21, 1.0, "multiaxis", (100.0, 80.0, 50.0), (4, 8)),
    "pockets-small": lambda: P._procedural(22, 1.0, "pockets", (120.0, 90.0, 60.0), (6, 10)),
}


def _export(ctx, m, leaf):
    b = ctx.build_bvh(m.verts, m.tris, leaf_size=leaf)
    out = b.export()
    b.release()
    return out


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("leaf", [1, 4, 8, 16])
def test_bvh_tight_and_identical_across_builds(ctx, name, leaf):
    m = MESHES[name]()
    _say("bvh", name, leaf, m.n_tris)
    nodes, tris, root, nv = _export(ctx, m, leaf)
    check_bvh(nodes, tris, root, nv, m.verts, m.tris, tight=True)
    for k in range(6):
        n2, t2, r2, nv2 = _export(ctx, m, leaf)
        assert (r2, nv2) == (root, nv), k
        assert np.array_equal(t2.view(np.uint32), tris.view(np.uint32)), k
        assert np.array_equal(n2.view(np.uint32), nodes.view(np.uint32)), k


def test_bvh_interactive_size_tight(ctx):
    m = P.workload_parts("interactive_200k")[0]
    _say("bvh interactive", m.n_tris)
    nodes, tris, root, nv = _export(ctx, m, 4)
    check_bvh(nodes, tris, root, nv, tight=True)
    for k in range(3):
        n2, t2, r2, _ = _export(ctx, m, 4)
        assert r2 == root and np.array_equal(n2.view(np.uint32), nodes.view(np.uint32)), k


def test_release_after_context_destroyed():
    """Handles may be freed after their context (Python collects them in any
    order): releasing a hierarchy and a plan then must leave no error behind
    for the next context's calls."""
    from paper_2609_05467_amd import hra
    m = P.config1_part()
    c1 = hra.Context(0)
    b = c1.build_bvh(m.verts, m.tris)
    b.info()
    pl = c1.plan([{"verts": m.verts, "tris": m.tris, "n_samples": 100, "seed": 1, "tool_length": 50.0}], 256)
    pl.run()
    c1.close()
    b.release()
    pl.destroy()
    c2 = hra.Context(0)
    b2 = c2.build_bvh(m.verts, m.tris)
    assert b2.info().n_tris == m.n_tris
    b2.release()
    c2.close()


def test_release_in_stream_order_while_work_is_queued(ctx):
    """A pipelined caller frees step k's hierarchy on its stream while step
    k + 1's build and cast are queued behind it: the arrays return to the
    pool in stream order, the next builds reuse them, and every step's bits
    equal those of a hierarchy nobody released early (the memory the pool
    hands back is never read by a stale reader, nor overwritten under a
    live one)."""
    import torch
    m = P.config1_part()
    S, N = 4000, 1024
    _say("release async", m.n_tris, S, N)
    ref_b = ctx.build_bvh(m.verts, m.tris)
    s = ctx.alloc_samples(S)
    ctx.sample_surface(ref_b, S, 3, out=s)
    ref, _ = ctx.cast(ref_b, s, N, counts=False)
    ref_nodes = _export(ctx, m, 4)[0]
    torch.cuda.synchronize()
    main = torch.cuda.current_stream()
    cur = ctx.build_bvh(m.verts, m.tris)
    outs = []
    for k in range(6):
        bits, _ = ctx.cast(cur, s, N, counts=False)
        outs.append(bits)
        nxt = ctx.build_bvh(m.verts, m.tris)       # queued behind the cast
        cur.release(stream=main)                    # no wait: freed after the cast in stream order
        assert cur.ptr is None
        cur = nxt
    n2 = _export(ctx, m, 4)[0]
    torch.cuda.synchronize()
    for k, bits in enumerate(outs):
        assert torch.equal(bits, ref), k
    assert np.array_equal(n2.view(np.uint32), ref_nodes.view(np.uint32))
    cur.release(stream=main)
    cur.release(stream=main)       # a second release of a freed handle does nothing
    ref_b.release()
    torch.cuda.synchronize()


def test_release_on_another_stream_waits(ctx):
    """A hierarchy built on one stream and released on another: the pool
    would give its blocks to the next build on the first stream before the
    second stream's queued work has run, so the release waits for the device
    instead, and a cast queued before it still reads an intact hierarchy."""
    import torch
    m = P.config1_part()
    S, N = 4000, 1024
    _say("release on another stream", m.n_tris, S, N)
    ref_b = ctx.build_bvh(m.verts, m.tris)
    s = ctx.alloc_samples(S)
    ctx.sample_surface(ref_b, S, 3, out=s)
    ref, _ = ctx.cast(ref_b, s, N, counts=False)
    torch.cuda.synchronize()
    other = torch.cuda.Stream()
    outs = []
    for k in range(4):
        b = ctx.build_bvh(m.verts, m.tris)           # built on the current stream
        other.wait_stream(torch.cuda.current_stream())
        bits, _ = ctx.cast(b, s, N, counts=False, stream=other)
        outs.append(bits)
        b.release(stream=other)                       # not the build stream: waits for the device
        assert b.ptr is None
    torch.cuda.synchronize()
    for k, bits in enumerate(outs):
        assert torch.equal(bits, ref), k
    ref_b.release()
    torch.cuda.synchronize()

"""Casting against global obstacles: a clamp block held 5 mm above the top
of the config-1 part.  Samples are drawn on the part's own hierarchy and
cast against a hierarchy of the part and the block together; the casts read
only a sample's point, origin and normal.  Parity with the oracle on the
combined mesh for the hemisphere and the tool-aware casts, and the block
only ever removes directions from the hemisphere cast (every triangle
decision is exact, so the part's triangles block the same rays in either
hierarchy)."""
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


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _combined():
    m = P.config1_part()
    v2, t2 = P._box_tris(len(m.verts), (20.0, 45.0, 45.0), (80.0, 70.0, 55.0))
    c = P.Mesh(np.vstack([m.verts, v2]).astype(np.float32), np.vstack([m.tris, t2]).astype(np.int32),
               "config1+clamp")
    return m, c


def _ones(x):
    return int(np.unpackbits(x.view(np.uint8)).sum())


def test_obstacle_hemisphere(ctx, orc):
    m, c = _combined()
    bp = ctx.build_bvh(m.verts, m.tris)
    bc = ctx.build_bvh(c.verts, c.tris)
    s = ctx.sample_surface(bp, 400, 9)
    sn = {k: v.cpu().numpy() for k, v in s.items()}
    N = 256
    _say("obstacle hemisphere", m.n_tris, c.n_tris, N)
    bits_p, _ = ctx.cast(bp, s, N)
    bits_c, cnt_c = ctx.cast(bc, s, N)
    gp, gc = _u32(bits_p), _u32(bits_c)
    ob, og, _ = orc.cast(c.verts, c.tris, sn, orc.fibonacci_dirs(N))
    assert not ((gc ^ ob) & ~og).any()
    assert np.array_equal(_u32(cnt_c), np.array([_ones(r) for r in gc], np.uint32))
    assert not (gc & ~gp).any()
    assert _ones(gp & ~gc) > 0.01 * _ones(gp)


def test_obstacle_tool(ctx, orc):
    m, c = _combined()
    bp = ctx.build_bvh(m.verts, m.tris)
    bc = ctx.build_bvh(c.verts, c.tris)
    s = ctx.sample_surface(bp, 150, 4)
    sn = {k: v.cpu().numpy() for k, v in s.items()}
    _say("obstacle tool")
    bits, _ = ctx.cast_tool(bc, s, 150, 2.0)
    got = _u32(bits)
    ob, oa = orc.cast_tool(c.verts, c.tris, sn, orc.fibonacci_dirs(150), 2.0)
    assert not ((got ^ ob) & ~oa).any()
    alone, _ = ctx.cast_tool(bp, s, 150, 2.0)
    assert _ones(_u32(alone) & ~got) > 0

"""The allocation-free directional statistics (hra_dominant_axes_noalloc)
through the C ABI against hra_dominant_axes on the same inputs: every output
bit for bit (the same kernels; per-sample values and integer histogram sums
do not depend on the launch), on two calls in a row, the second with fewer
samples and fewer directions, so that the scratch array's leftovers from the
first call must not reach the second; and the direction limit."""
import numpy as np
import pytest

from synth import parts as P

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2609_05467_amd import hra
    assert torch.cuda.is_available()
    c = hra.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _outputs(st):
    return {k: st[k].cpu().numpy().copy() for k in ("mean", "absmean", "axis", "conc", "hist")}


def _both(ctx, s, N, bits):
    import torch
    ref = ctx.dominant_axes(s, N, bits)
    got = ctx.dominant_axes(s, N, bits, noalloc=True)
    torch.cuda.synchronize()
    a, b = _outputs(ref), _outputs(got)
    for k in a:
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k
    n = s["origin"].shape[0]
    assert ctx.classify(ref, n, N) == ctx.classify(got, n, N)
    # part totals as written (the header's five counters and the FP64 sum,
    # then the per-sample FP64 concentrations and counts; the header's pad
    # and the buffer's slack are never written)
    ta, tb = ref["totals"].cpu().numpy(), got["totals"].cpu().numpy()
    assert np.array_equal(ta[:48], tb[:48])
    assert np.array_equal(ta[64:64 + 12 * n], tb[64:64 + 12 * n])
    return b


def test_noalloc_matches_dominant_axes_twice(ctx):
    m = P._procedural(7, 1.0, "pockets", (120.0, 90.0, 60.0), (6, 10))
    b = ctx.build_bvh(m.verts, m.tris)
    # first call: 9000 samples x 4096 directions (2250 four-sample blocks,
    # capped at the slice count)
    s1 = ctx.sample_surface(b, 9000, 3)
    bits1, _ = ctx.cast(b, s1, 4096)
    _say("noalloc 9000 x 4096")
    o1 = _both(ctx, s1, 4096, bits1)
    assert o1["hist"].view(np.uint32).sum() > 0
    # second call right after: fewer samples (fewer blocks) and directions
    s2 = ctx.sample_surface(b, 37, 4)
    bits2, cnt2 = ctx.cast(b, s2, 150)
    _say("noalloc 37 x 150")
    o2 = _both(ctx, s2, 150, bits2)
    assert int(o2["hist"].view(np.uint32).astype(np.int64).sum()) == int(cnt2.cpu().numpy().view(np.uint32).sum())
    # no samples at all
    s0 = ctx.alloc_samples(0)
    z = ctx.dominant_axes(s0, 512, bits2[:0], noalloc=True)
    assert not z["hist"].cpu().numpy().any()
    b.release()


def test_noalloc_direction_limit(ctx):
    from paper_2609_05467_amd import hra
    m = P.box_part()
    b = ctx.build_bvh(m.verts, m.tris)
    s = ctx.sample_surface(b, 10, 1)
    bits, _ = ctx.cast(b, s, 8192)
    _both(ctx, s, 8192, bits)
    big, _ = ctx.cast(b, s, 8193)
    with pytest.raises(hra.HraError) as e:
        ctx.dominant_axes(s, 8193, big, noalloc=True)
    assert e.value.status == -1
    b.release()

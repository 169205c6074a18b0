"""The spatial sample order the hemisphere cast follows (hra_samples.order):
the sampler's order is a permutation sorted by the Morton key of each
origin; bits do not depend on the order (the sampler's, the one the cast
forms itself, none below the size where it forms one, or a reversed one);
an order naming an index outside [0, n) is an error, not an access."""
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


def _morton21(o, lo, hi):
    code = np.zeros(len(o), np.uint32)
    for k in range(3):
        ext = np.float32(hi[k] - lo[k])
        t = (o[:, k] - np.float32(lo[k])) / ext
        q = np.clip(np.floor(np.float32(128.0) * t), 0, 127).astype(np.uint32)
        for b in range(7):
            code |= ((q >> b) & 1) << (3 * b + (2 - k))
    return code


@pytest.mark.parametrize("name,n,ndirs", [("config1", 20_000, 512), ("procedural", 12_000, 1024)])
def test_order_is_a_sorted_permutation_and_bits_do_not_depend_on_it(ctx, name, n, ndirs):
    import torch
    m = P.config1_part() if name == "config1" else P.procedural_part(7, 30_000, "pockets")
    _say("order", name, n, ndirs)
    b = ctx.build_bvh(m.verts, m.tris)
    try:
        s = ctx.alloc_samples(n)
        s["order"] = torch.empty((n,), dtype=torch.int32, device=ctx.device)
        ctx.sample_surface(b, n, 5, out=s)
        order = s["order"].cpu().numpy()
        assert np.array_equal(np.sort(order), np.arange(n))
        info = b.info()
        lo, hi = np.array(info.bbox[:3], np.float32), np.array(info.bbox[3:], np.float32)
        keys = _morton21(s["origin"].cpu().numpy(), lo, hi)[order]
        assert np.all(np.diff(keys.astype(np.int64)) >= 0)
        # stable: equal keys keep index order
        same = np.diff(keys.astype(np.int64)) == 0
        assert np.all(np.diff(order)[same] > 0)
        with_order, _ = ctx.cast(b, s, ndirs, counts=False)
        own = {k: v for k, v in s.items() if k != "order"}          # the cast forms its own order
        without, _ = ctx.cast(b, own, ndirs, counts=False)
        rev = dict(s)
        rev["order"] = torch.flip(s["order"], [0]).contiguous()      # any permutation gives the same bits
        reversed_bits, _ = ctx.cast(b, rev, ndirs, counts=False)
        small = {k: v[:3000].contiguous() for k, v in own.items()}  # below the size that forms an order
        small_bits, _ = ctx.cast(b, small, ndirs, counts=False)
        torch.cuda.synchronize()
        assert torch.equal(with_order, without)
        assert torch.equal(with_order, reversed_bits)
        assert torch.equal(with_order[:3000], small_bits)
    finally:
        b.release()


def test_order_outside_the_samples_is_an_error(ctx):
    import torch
    from paper_2609_05467_amd import hra
    m = P.config1_part()
    b = ctx.build_bvh(m.verts, m.tris)
    try:
        n = 5000
        s = ctx.alloc_samples(n)
        ctx.sample_surface(b, n, 5, out=s)
        bad = torch.arange(n, dtype=torch.int32, device=ctx.device)
        bad[17] = n + 3          # the kernel's own bound check turns it into the error word
        s["order"] = bad
        _say("order out of range")
        ctx.cast(b, s, 512, counts=False)
        with pytest.raises(hra.HraError, match="sample order"):
            b.info()   # a synchronising call reads (and clears) the context's error word
        # the context stays usable
        del s["order"]
        bits, _ = ctx.cast(b, s, 512, counts=False)
        b.info()
        torch.cuda.synchronize()
    finally:
        b.release()

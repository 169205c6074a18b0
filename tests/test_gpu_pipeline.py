"""The pipelined step that bench.py times, at a size the checks finish in
seconds: each step's hierarchy and samples made on a stream of their own
beside the previous step's cast, the casts queued behind the previous step's
statistics before the host reads its class, two sample buffers, and each
hierarchy freed in stream order on the stream that built it.  Every step's
bits, class and setups must equal those of the same step run alone."""
import sys

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


@pytest.mark.parametrize("name,S,N", [("config1", 6000, 1024), ("procedural", 5000, 2048)])
def test_pipelined_steps_equal_steps_alone(ctx, name, S, N):
    import torch
    from paper_2609_05467_amd import hra
    m = P.config1_part() if name == "config1" else P.procedural_part(11, 40_000, "pockets")
    dev = ctx.device
    verts = torch.tensor(m.verts, device=dev)
    tris = torch.tensor(m.tris, device=dev)
    W = (N + 31) // 32
    _say("pipeline", name, m.n_tris, S, N)

    # one step alone, everything on the current stream
    b = ctx.build_bvh(verts, tris)
    s = ctx.alloc_samples(S)
    s["order"] = torch.empty((S,), dtype=torch.int32, device=dev)
    ctx.sample_surface(b, S, 2, out=s)
    ref_bits, _ = ctx.cast(b, s, N, counts=False)
    ref_b6, _ = ctx.cast(b, s, 6, kind=hra.DIRS_AXES6, counts=False)
    ref_rep = ctx.classify(ctx.dominant_axes(s, N, ref_bits), S, N)
    ref_su = ctx.min_setups(b, s, ref_b6, 50.0, want_class=False)
    torch.cuda.synchronize()
    b.release()

    bufs = []
    for _ in range(2):
        sb = ctx.alloc_samples(S)
        sb["order"] = torch.empty((S,), dtype=torch.int32, device=dev)
        bufs.append(sb)
    bits = torch.empty((S, W), dtype=torch.int32, device=dev)
    bits6 = torch.empty((S, 1), dtype=torch.int32, device=dev)
    prep, side, cls = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    main = torch.cuda.current_stream()
    copies = []

    def prepare(i):
        with torch.cuda.stream(prep):
            bvh = ctx.build_bvh(verts, tris)
            ctx.sample_surface(bvh, S, 2, out=bufs[i % 2])
        return bvh, bufs[i % 2]

    def launch(cur):
        bvh, smp = cur
        main.wait_stream(prep)
        side.wait_stream(main)
        ctx.cast(bvh, smp, 6, kind=hra.DIRS_AXES6, counts=False, bits=bits6, stream=side)
        ctx.cast(bvh, smp, N, counts=False, bits=bits)
        copies.append(bits.clone())          # stream-ordered copy of this step's bits
        return cur

    steps = 6
    out = []
    cur = launch(prepare(0))
    for k in range(steps):
        bvh, smp = cur
        ds = ctx.dominant_axes(smp, N, bits)
        ev = torch.cuda.Event()
        ev.record()
        su = ctx.min_setups(bvh, smp, bits6, 50.0, want_class=False, stream=side)
        cls.wait_event(ev)
        cur = launch(prepare(k + 1)) if k + 1 < steps else None
        rep = ctx.classify(ds, S, N, stream=cls)
        prep.wait_event(ev)
        bvh.release(stream=prep)             # the build stream: no wait
        out.append((rep, su))
    torch.cuda.synchronize()
    assert len(copies) == steps
    for k in range(steps):
        assert torch.equal(copies[k], ref_bits), k
        assert out[k][0] == ref_rep, k
        assert out[k][1] == ref_su, k

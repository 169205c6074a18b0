"""Directional statistics (hra_dominant_axes, Section 3.3) on crafted bit rows
against the oracle's dirstats: rows with no free direction (blind), every
direction free, only the first or only the last direction free, and random
densities from sparse to dense, for direction counts below, at and just
past one 64-direction chunk and with a ragged tail.  The bits are inputs
here (drawn on the host), not cast results, so every row shape is reached."""
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


def _rows(N, S, seed):
    """S bit rows of N directions (unpacked, bool): the special rows first,
    then random densities."""
    rng = np.random.default_rng(seed)
    U = np.zeros((S, N), bool)
    U[1] = True
    U[2, 0] = True
    U[3, N - 1] = True
    dens = rng.choice([0.01, 0.1, 0.5, 0.9, 0.99], size=S)
    for i in range(4, S):
        U[i] = rng.random(N) < dens[i]
    return U


def _pack(U):
    S, N = U.shape
    W = (N + 31) // 32
    pad = np.zeros((S, W * 32), bool)
    pad[:, :N] = U
    w = pad.reshape(S, W, 32).astype(np.uint64) << np.arange(32, dtype=np.uint64)
    return w.sum(axis=2).astype(np.uint32)


@pytest.mark.parametrize("N", [1, 33, 64, 65, 150, 1000])
def test_dirstats_crafted_rows(ctx, orc, N):
    import torch
    m = P.icosphere(subdiv=2)
    b = ctx.build_bvh(m.verts, m.tris)
    S = 257
    s = ctx.sample_surface(b, S, 5)
    sn = {k: v.cpu().numpy() for k, v in s.items()}
    U = _rows(N, S, N)
    bits_np = _pack(U)
    bits = torch.from_numpy(bits_np.view(np.int32)).to(ctx.device)
    _say("dirstats crafted", N)
    st = ctx.dominant_axes(s, N, bits)
    o = orc.dirstats(sn, orc.fibonacci_dirs(N), bits_np)
    mean, absmean = st["mean"].cpu().numpy(), st["absmean"].cpu().numpy()
    axis, conc = st["axis"].cpu().numpy(), st["conc"].cpu().numpy()
    assert np.allclose(mean, o["mean"], atol=1e-5, rtol=0)
    assert np.allclose(absmean, o["absmean"], atol=1e-5, rtol=0)
    blind = ~U.any(axis=1)
    assert np.array_equal(axis[blind], np.full(blind.sum(), -1, np.int8)) and blind[0]
    assert np.all(mean[blind] == 0) and np.all(conc[blind] == 0)
    sel = ~o["tie"]
    assert np.array_equal(axis[sel], o["axis"][sel])
    assert np.allclose(conc[sel], o["conc"][sel], atol=1e-4, rtol=0)
    h = st["hist"].cpu().numpy().view(np.uint32).astype(np.int64)
    oh = o["hist"].astype(np.int64)
    assert h.sum() == oh.sum() == int(U.sum())
    assert np.abs(h - oh).sum() <= max(2, 2e-4 * oh.sum())
    # the whole-part counts agree with the rows
    rep = ctx.classify(st, S, N)
    assert rep["n_blind"] == int(blind.sum())
    assert rep["n_unobstructed"] == int(U.sum())

"""The FP32 azimuth sector the statistics kernel takes away from sector
edges: the pseudo-angle p = |y| / (|x| + |y|) looked up in the library's
boundary table (hra_debug_azimuth_table, host only) and compared with it in
float32 on the CPU, as the kernel does, must give the FP64 atan2 sector of
the histogram's definition wherever the kernel's guard lets FP32 decide, on
every quadrant, axis and diagonal; axes, zeros and exact boundaries must go
to the FP64 path."""
import ctypes as C

import numpy as np

from paper_2609_05467_amd import hra

CELLS = 128
EPS = np.float32(4e-6)      # guard in p units, as in the kernel


def _table():
    n = hra.lib().hra_debug_azimuth_table(None, 0)
    assert n == 4 * 4 * (CELLS + 1)
    buf = (C.c_float * n)()
    assert hra.lib().hra_debug_azimuth_table(buf, n) == n
    return np.frombuffer(buf, np.float32).reshape(4, CELLS + 1, 4).copy()


def _fp64_sector(x, y):
    az = np.floor((np.arctan2(y.astype(np.float64), x.astype(np.float64)) + np.pi) * 128.0 / (2 * np.pi))
    return np.clip(az, 0, 127).astype(np.int64)


def _kernel_sector(tab, x, y, rcp_ulps=0):
    """The kernel's FP32 steps; rcp_ulps moves the reciprocal by that many
    ulps (the hardware reciprocal is within one).  Returns (sector, clear)."""
    x = x.astype(np.float32)
    y = y.astype(np.float32)
    s = (np.abs(x) + np.abs(y)).astype(np.float32)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = (np.float32(1) / s).astype(np.float32)
    if rcp_ulps:
        r = np.nextafter(r, np.float32(np.inf) if rcp_ulps > 0 else np.float32(0)).astype(np.float32)
    with np.errstate(invalid="ignore"):
        p = (np.abs(y) * r).astype(np.float32)
        cell = np.where(np.isnan(p), 0, np.minimum((p * np.float32(CELLS)).astype(np.float64), 1e9)).astype(np.int64)
    cell = np.minimum(cell, CELLS)
    q = 2 * (np.signbit(x)).astype(np.int64) + np.signbit(y).astype(np.int64)
    e = tab[q, cell]
    with np.errstate(invalid="ignore"):
        clear = np.fmin(p - e[:, 0], np.abs(e[:, 1] - p)) >= EPS
        above = p >= e[:, 1]
    off = np.where(above, e[:, 3].view(np.uint32), e[:, 2].view(np.uint32)).astype(np.int64)
    assert (off % 4 == 0).all()
    return off // 4, clear


def test_table_boundaries_are_the_sector_edges():
    tab = _table()
    k = np.arange(33)
    a = k * np.pi / 64
    pk = np.where(k == 32, 1.0, np.sin(a) / (np.sin(a) + np.cos(a)))
    for q in range(4):
        for c in range(CELLS + 1):
            lo, nxt = tab[q, c, 0], tab[q, c, 1]
            kb = int(np.argmin(np.abs(pk - lo)))
            assert abs(pk[kb] - lo) < 1e-7 and pk[kb] <= c / CELLS + 1e-7
            assert kb == 31 or pk[kb + 1] > c / CELLS
            assert abs(pk[kb + 1] - nxt) < 1e-7


def test_sector_matches_atan2_where_fp32_decides():
    tab = _table()
    rng = np.random.default_rng(1)
    v = rng.normal(size=(1_000_000, 2))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    # directions crowded against every sector edge
    edges = (np.arange(128) * 2 * np.pi / 128 - np.pi)[:, None] + np.array([-1e-5, -2e-6, 0.0, 2e-6, 1e-5])[None, :]
    v = np.vstack([v, np.stack([np.cos(edges.ravel()), np.sin(edges.ravel())], 1)])
    x, y = v[:, 0].astype(np.float32), v[:, 1].astype(np.float32)
    want = _fp64_sector(x, y)
    for ulps in (0, 1, -1):
        got, clear = _kernel_sector(tab, x, y, ulps)
        assert np.array_equal(got[clear], want[clear]), ulps
        assert clear[:1_000_000].mean() > 0.999
        # a direction within the guard of an edge goes to FP64
        assert not clear[1_000_000:].reshape(128, 5)[:, 1:4].any()


def test_axes_zeros_and_diagonals_go_to_fp64_or_match():
    tab = _table()
    pts = np.array([[1, 0], [0, 1], [-1, 0], [0, -1], [0, 0], [-0.0, 0], [0, -0.0], [1, 1], [-1, 1], [-1, -1],
                    [1, -1], [0.3, 1e-30], [-0.3, 1e-30], [1e-30, -0.3]], np.float64)
    x, y = pts[:, 0].astype(np.float32), pts[:, 1].astype(np.float32)
    got, clear = _kernel_sector(tab, x, y)
    # on an axis (a sector edge) or at the origin the FP32 path must stand down
    assert not clear[:7].any()
    want = _fp64_sector(x, y)
    assert np.array_equal(got[clear], want[clear])

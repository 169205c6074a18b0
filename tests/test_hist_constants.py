"""The FP32 azimuth used for histogram bins on the GPU: the arctangent
coefficients in the kernel source, evaluated in float32 on the CPU, stay
within the error the kernel's edge guard assumes, and the octant mapping
reproduces atan2 on every quadrant, axis and diagonal."""
import os
import re

import numpy as np

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2609_05467_amd", "csrc", "stats.hip")
HIST_EDGE = 5e-4          # bins, the guard in the kernel
BIN = 2 * np.pi / 128     # radians per azimuth sector


def _coeffs():
    s = open(SRC).read()
    m = re.search(r"ATAN_C\[7\]\s*=\s*\{([^}]*)\}", s)
    assert m, "coefficient table not found"
    c = [float(x.strip().rstrip("f")) for x in m.group(1).split(",")]
    assert len(c) == 7
    return np.array(c, np.float32)


def _atan01(r):
    c = _coeffs()
    r = r.astype(np.float32)
    r2 = (r * r).astype(np.float32)
    p = np.full_like(r, c[6])
    for k in range(5, -1, -1):
        p = (p * r2 + c[k]).astype(np.float32)
    return (r * p).astype(np.float32)


def _azimuth_bins(x, y):
    x = x.astype(np.float32)
    y = y.astype(np.float32)
    ax, ay = np.abs(x), np.abs(y)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = (np.minimum(ax, ay) * (np.float32(1) / np.maximum(ax, ay))).astype(np.float32)
    a = _atan01(r)
    a = np.where(ay > ax, np.float32(1.57079637) - a, a).astype(np.float32)
    a = np.where(x < 0, np.float32(3.14159274) - a, a).astype(np.float32)
    a = np.where(y < 0, -a, a).astype(np.float32)
    return ((a + np.float32(3.14159274)) * np.float32(20.3718327)).astype(np.float32)


def test_arctangent_polynomial_error():
    r = np.linspace(0, 1, 1_000_001).astype(np.float32)
    err = np.abs(_atan01(r).astype(np.float64) - np.arctan(r.astype(np.float64)))
    assert err.max() < 4e-7
    # the guard is far wider than this error, in sector units
    assert err.max() / BIN < HIST_EDGE / 40


def test_azimuth_matches_atan2_in_every_octant():
    rng = np.random.default_rng(0)
    v = rng.normal(size=(400_000, 2))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    special = np.array([[1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1],
                        [0.3, 1e-7], [-0.3, 1e-7], [1e-7, -0.3]], np.float64)
    v = np.vstack([v, special])
    x, y = v[:, 0].astype(np.float32), v[:, 1].astype(np.float32)
    got = _azimuth_bins(x, y).astype(np.float64)
    want = (np.arctan2(y.astype(np.float64), x.astype(np.float64)) + np.pi) * 128.0 / (2 * np.pi)
    assert np.abs(got - want).max() < 1e-4
    # away from the guard band the sector is the FP64 one
    frac = got - np.floor(got)
    ok = (frac > HIST_EDGE) & (frac < 1 - HIST_EDGE)
    assert ok.mean() > 0.95
    assert np.array_equal(np.floor(got[ok]), np.floor(want[ok]))


def test_azimuth_origin_goes_to_fp64_path():
    # x = y = 0: the FP32 value is NaN, so the edge test fails and FP64 decides
    got = _azimuth_bins(np.zeros(2), np.array([0.0, -0.0]))
    assert np.isnan(got).all()

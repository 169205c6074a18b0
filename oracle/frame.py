"""CPU oracle: canonical machining frame.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the tests, the
smoke check and the benchmark's CPU-baseline leg use it.

Section 3.2 of the paper reorients every part into a canonical machining frame
before the six orthogonal casts, but does not say how the frame is found.  The
reading written out here (plain numpy, FP64, one step after another) is:

1. Faces.  For each triangle, the FP64 normal N = (B - A) x (C - A) of its FP32
   vertices, |N| = sqrt((Nx^2 + Ny^2) + Nz^2), area |N| / 2.  A face with
   |N| = 0 takes no part.  The unit normal n = N / |N| is folded onto the
   upper hemisphere (a face and its opposite face give the same machining
   axis): n -> -n when nz < 0, or nz = 0 and ny < 0, or nz = ny = 0 and nx < 0;
   zero components are then made +0, so that the bin of a direction such as
   (0, 0, 1) does not depend on the sign of a zero (atan2 tells -0 from +0).
2. Histogram.  Integer area weights w = floor(area * 2^s), s = 31 - e where
   the largest area is m * 2^e with m in [0.5, 1), summed into the 8192 bins
   of the direction histogram (`oracle.histogram_bin`).  Integer sums make the
   peak independent of summation order.
3. First axis.  b1 = the heaviest bin (lowest index on ties).  a1 starts as
   the normalised area-weighted mean of the normals in b1, then is refined
   twice: the normalised area-weighted mean of the normals within 5 degrees
   of it (each taken with the sign that agrees with the current axis), then
   within 2 degrees.
4. Second axis.  b2 = the heaviest bin whose centre is within 15 degrees of
   perpendicular to a1 (|centre . a1| <= cos 75 deg).  a2 is refined from b2
   like a1, each step followed by removing its a1 component.  Without such a
   bin, a2 is the world axis least aligned with a1 with its a1 component
   removed.  a3 = a1 x a2.
5. Labels.  Z = the axis with the most surface area on faces within 5 degrees
   of it (the largest planar faces: the fixture face); X = the remaining axis
   along which the vertices extend furthest; Y = Z x X.  Z and X are signed so
   that their largest component is positive.  Near-ties are decided the same
   way on every implementation: values within a relative 1e-9 count as equal
   and the earlier axis wins; a component within 1e-9 of the largest counts as
   the largest.
6. Confidence = the fraction of the surface area on faces within 5 degrees of
   one of the three axes (1 for a box, near 0 for a sphere).

Every dot product is (x0 y0 + x1 y1) + x2 y2, as the library computes it.
Pins: tests/test_frame_oracle.py (axis-aligned parts give the identity
exactly, known rotations are recovered, symmetric tilts average to the axis,
handedness, tie rules, a sphere has low confidence).
"""
from __future__ import annotations

import numpy as np

from .oracle import bin_centre, histogram_bin

CONE_WIDE = float(np.cos(np.radians(5.0)))     # refinement cone and "aligned" faces
CONE_FINE = float(np.cos(np.radians(2.0)))     # second refinement
PERP_COS = float(np.cos(np.radians(75.0)))     # second-axis candidates: within 15 deg of perpendicular
TIE_REL = 1e-9                                 # relative tie window for the Z and X choices
TIE_ABS = 1e-9                                 # absolute tie window for the sign component


def dot3(x, y):
    """(x0 y0 + x1 y1) + x2 y2; x may be a (k, 3) array."""
    x = np.asarray(x, np.float64)
    return (x[..., 0] * y[0] + x[..., 1] * y[1]) + x[..., 2] * y[2]


def normalise(x):
    L = np.sqrt((x[0] * x[0] + x[1] * x[1]) + x[2] * x[2])
    return x / L


def cross(a, b):
    return np.array([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


def orth(x, a):
    """x without its component along the unit vector a, normalised."""
    return normalise(x - dot3(x, a) * a)


def faces(verts, tris):
    """Step 1: folded unit normals, areas and the nonzero-area flag, FP64."""
    v = np.asarray(verts, np.float32).astype(np.float64)
    t = np.asarray(tris, np.int64)
    A, B, Cc = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    e1, e2 = B - A, Cc - A
    N = np.stack([e1[:, 1] * e2[:, 2] - e1[:, 2] * e2[:, 1],
                  e1[:, 2] * e2[:, 0] - e1[:, 0] * e2[:, 2],
                  e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]], 1)
    L = np.sqrt((N[:, 0] * N[:, 0] + N[:, 1] * N[:, 1]) + N[:, 2] * N[:, 2])
    ok = L > 0
    n = np.zeros_like(N)
    n[ok] = N[ok] / L[ok, None]
    flip = (n[:, 2] < 0) | ((n[:, 2] == 0) & ((n[:, 1] < 0) | ((n[:, 1] == 0) & (n[:, 0] < 0))))
    n[flip] = -n[flip]
    n = n + 0.0   # -0 -> +0: the azimuth of (0, 0, 1) must not depend on the sign of a zero
    return n, 0.5 * L, ok


def weights(area, ok):
    """Step 2: integer weights floor(area * 2^s), s = 31 - exponent of the largest area."""
    _, e = np.frexp(float(area[ok].max()))
    s = 31 - int(e)
    w = np.zeros(len(area), np.uint64)
    w[ok] = np.floor(np.ldexp(area[ok], s)).astype(np.uint64)
    return w, s


def face_bins(n, ok):
    b = np.full(len(n), -1, np.int64)
    for i in np.nonzero(ok)[0]:
        b[i] = histogram_bin(n[i])
    return b


def histogram(bins, w, ok):
    """Step 2: H[b] = sum of the weights of the faces in bin b."""
    H = np.zeros(8192, np.uint64)
    np.add.at(H, bins[ok], w[ok])
    return H


def bin_mean(n, area, bins, b):
    """Normalised area-weighted mean of the normals in bin b."""
    sel = bins == b
    S = (area[sel][:, None] * n[sel]).sum(0)
    return normalise(S)


def cone_mean(n, area, ok, c, cos_cone):
    """Normalised area-weighted mean of the normals within the cone about c,
    each signed to agree with c; c itself when no face is inside."""
    d = dot3(n, c)
    sel = ok & (np.abs(d) >= cos_cone)
    if not sel.any():
        return c
    S = ((area[sel] * np.sign(d[sel]))[:, None] * n[sel]).sum(0)
    return normalise(S)


def heaviest(H, mask):
    """Index of the largest H among mask (lowest index on ties), -1 if none."""
    idx = np.nonzero(mask & (H > 0))[0]
    if len(idx) == 0:
        return -1
    return int(idx[np.argmax(H[idx])])   # argmax returns the first maximum


def first_max(vals):
    """Index of the largest value, values within a relative TIE_REL of the
    current best counting as equal (the earlier index wins)."""
    best = 0
    for k in range(1, len(vals)):
        if vals[k] > vals[best] * (1 + TIE_REL):
            best = k
    return best


def sign_fix(a):
    """a or -a: the one whose largest-magnitude component (the first within
    TIE_ABS of the largest) is positive."""
    m = np.abs(a).max()
    k = int(np.nonzero(np.abs(a) >= m - TIE_ABS)[0][0])
    return -a if a[k] < 0 else a


def estimate(verts, tris):
    """The canonical frame of one mesh (steps 1-6 of the module docstring).

    Returns a dict: axes (3x3, rows X, Y, Z), confidence, aligned (surface
    area aligned with X, Y, Z), extent (vertex extent along X, Y, Z), total
    area, the peak bins (b1, b2), the refined axes a1, a2, a3, the weight
    shift s and the histogram."""
    v64 = np.asarray(verts, np.float32).astype(np.float64)
    n, area, ok = faces(verts, tris)
    if not ok.any():
        raise ValueError("no face with nonzero area")
    w, s = weights(area, ok)
    bins = face_bins(n, ok)
    H = histogram(bins, w, ok)
    b1 = heaviest(H, np.ones(8192, bool))
    a1 = bin_mean(n, area, bins, b1)
    a1 = cone_mean(n, area, ok, a1, CONE_WIDE)
    a1 = cone_mean(n, area, ok, a1, CONE_FINE)
    centres = np.array([bin_centre(b) for b in range(8192)])
    b2 = heaviest(H, np.abs(dot3(centres, a1)) <= PERP_COS)
    if b2 >= 0:
        a2 = orth(bin_mean(n, area, bins, b2), a1)
        a2 = orth(cone_mean(n, area, ok, a2, CONE_WIDE), a1)
        a2 = orth(cone_mean(n, area, ok, a2, CONE_FINE), a1)
    else:
        k = first_max(-np.abs(a1) + 2.0)   # least aligned world axis (ties: the earlier)
        a2 = orth(np.eye(3)[k], a1)
    a3 = normalise(cross(a1, a2))
    ax = [a1, a2, a3]
    aligned = np.array([area[ok & (np.abs(dot3(n, a)) >= CONE_WIDE)].sum() for a in ax])
    extent = np.array([dot3(v64, a).max() - dot3(v64, a).min() for a in ax])
    kz = first_max(aligned)
    i, j = [k for k in range(3) if k != kz]
    kx = j if extent[j] > extent[i] * (1 + TIE_REL) else i
    ky = 3 - kz - kx
    Z = sign_fix(ax[kz])
    X = sign_fix(ax[kx])
    Y = cross(Z, X)
    total = area[ok].sum()
    return {"axes": np.stack([X, Y, Z]), "confidence": float(aligned.sum() / total),
            "aligned": aligned[[kx, ky, kz]], "extent": extent[[kx, ky, kz]], "total_area": float(total),
            "peak_bins": (b1, b2), "a": np.stack(ax), "order": (kx, ky, kz), "shift": s, "hist": H}


def apply(axes, verts):
    """Vertices in the frame: v'_k = (f_k0 v_x + f_k1 v_y) + f_k2 v_z, in FP32
    with the frame rounded to FP32 (the rotation the library applies)."""
    f = np.asarray(axes, np.float64).astype(np.float32)
    v = np.asarray(verts, np.float32)
    out = np.empty_like(v)
    for k in range(3):
        out[:, k] = (f[k, 0] * v[:, 0] + f[k, 1] * v[:, 1]) + f[k, 2] * v[:, 2]
    return out

"""CPU oracle: datum planes per setup orientation.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the tests, the
smoke check and the benchmark's CPU-baseline leg use it.

Section 6 of the paper names the automatic identification of datum surfaces
for each setup orientation as future work (reference frames for the
tolerancing of each machining operation) and gives no method.  The reading
written out here (plain numpy, FP64, one step after another; the 3-2-1 rule
of fixturing applied to the part's axis-facing planes) is:

1. Axis-facing faces.  For each triangle, the FP64 normal N = (B - A) x (C - A)
   of its FP32 vertices, computed as (e1y e2z - e1z e2y, e1z e2x - e1x e2z,
   e1x e2y - e1y e2x) with q = (Nx^2 + Ny^2) + Nz^2 (the area rule of the
   sampler: a face with q = 0 takes no part).  Its dominant component c is
   the largest |N_c| (lowest c on ties); the face faces axis direction
   d = 2c + (N_c < 0) (the order +X, -X, +Y, -Y, +Z, -Z of the six-axis
   cast) when N_c^2 >= 0.99999999 q, i.e. its normal lies within 1e-4 rad
   of that axis.  Its offset is h = ((A_c + B_c) + C_c) / 3 in FP64 and its
   area the integer weight of the sampler, w = floor(area * 2^k).
2. Planes.  Axis-facing faces are ordered by (d, h with its three lowest
   bits dropped from its order-preserving 64-bit key, face index); a plane
   starts at the first face, at a change of d, and where h exceeds the
   previous face's h by more than 1e-6 x the bounding-box diagonal (single
   linkage).  A plane has direction d, offset h_min (its least h), area
   W = sum of w (exact: integers) and a face count.
3. Frames.  A setup is a tool approach direction a (0..5, as in the setup
   search).  The part rests on its opposite side, so its datum frame is:
   primary = the plane of direction a ^ 1 with the largest W; secondary =
   the plane with the largest W among those whose axis differs from a's;
   tertiary = the plane with the largest W among those whose axis differs
   from a's and the secondary's.  Ties: the lower direction, then the lower
   h_min.  A role with no candidate is empty (direction -1).

Areas are reported as W and as W x 2^-k (within n 2^-k of the plane's FP64
area, n its face count).
"""
from __future__ import annotations

import numpy as np

from . import oracle as O

FACING_COS2 = 0.99999999
LINK_FRAC = 1e-6


def faces(verts, tris):
    """Step 1: per triangle (direction or -1, offset h, weight w) and k."""
    v = np.asarray(verts, np.float32).astype(np.float64)
    t = np.asarray(tris, np.int64)
    A, B, C = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    e1, e2 = B - A, C - A
    nx = e1[:, 1] * e2[:, 2] - e1[:, 2] * e2[:, 1]
    ny = e1[:, 2] * e2[:, 0] - e1[:, 0] * e2[:, 2]
    nz = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    sx, sy, sz = nx * nx, ny * ny, nz * nz
    q = (sx + sy) + sz
    n = np.stack([nx, ny, nz], 1)
    s = np.stack([sx, sy, sz], 1)
    c = np.argmax(np.abs(n), axis=1)          # first index of the largest |N_c|
    rows = np.arange(len(t))
    nc, sc = n[rows, c], s[rows, c]
    facing = (q > 0.0) & (sc >= FACING_COS2 * q)
    d = np.where(facing, 2 * c + (nc < 0.0), -1).astype(np.int64)
    h = ((A[rows, c] + B[rows, c]) + C[rows, c]) / 3.0
    w, k = O.area_weights(verts, tris)
    return d, h, w.astype(np.uint64), k


def order_key(h):
    """Order-preserving 64-bit key of an FP64 value."""
    u = np.asarray(h, np.float64).view(np.uint64)
    neg = (u >> np.uint64(63)) == np.uint64(1)
    return np.where(neg, ~u, u | np.uint64(1 << 63))


def planes(verts, tris):
    """Step 2: list of planes (dir, h_min, W, count), and k."""
    d, h, w, k = faces(verts, tris)
    _, diag, _ = O.mesh_info(verts)
    tol = LINK_FRAC * diag
    idx = np.nonzero(d >= 0)[0]
    key = (d[idx].astype(np.uint64) << np.uint64(61)) | (order_key(h[idx]) >> np.uint64(3))
    idx = idx[np.lexsort((idx, key))]
    out = []
    for j, f in enumerate(idx):
        start = j == 0 or d[f] != d[idx[j - 1]] or (h[f] - h[idx[j - 1]]) > tol
        if start:
            out.append([int(d[f]), float(h[f]), 0, 0])
        p = out[-1]
        p[1] = min(p[1], float(h[f]))
        p[2] += int(w[f])
        p[3] += 1
    return [tuple(p) for p in out], k


def _best(cands):
    if not cands:
        return None
    return min(cands, key=lambda p: (-p[2], p[0], p[1]))


def datum_frames(verts, tris):
    """Step 3: for each approach direction a = 0..5, the (primary,
    secondary, tertiary) planes as dicts {dir, offset, area_w, area,
    n_tris} (dir -1: empty)."""
    pl, k = planes(verts, tris)
    scale = 2.0 ** -k

    def rec(p):
        if p is None:
            return {"dir": -1, "offset": 0.0, "area_w": 0, "area": 0.0, "n_tris": 0}
        return {"dir": p[0], "offset": p[1], "area_w": p[2], "area": p[2] * scale, "n_tris": p[3]}

    frames = []
    for a in range(6):
        ax = a >> 1
        prim = _best([p for p in pl if p[0] == (a ^ 1)])
        sec = _best([p for p in pl if (p[0] >> 1) != ax])
        ter = None
        if sec is not None:
            ter = _best([p for p in pl if (p[0] >> 1) != ax and (p[0] >> 1) != (sec[0] >> 1)])
        frames.append([rec(prim), rec(sec), rec(ter)])
    return frames

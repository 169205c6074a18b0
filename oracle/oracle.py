"""CPU oracle: Python side.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this module; the library never does, and this module
imports nothing from the library.  It wraps the plain C reference
(`hra_oracle.c`, brute force, FP64 decisions) and writes out the host-level
definitions (classification, reach, setups) directly from the paper.

Each function names the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import itertools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hra_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=False):
    """Compile the C oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math", "-fno-finite-math-only",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i64, i32, u64, f32 = C.c_int64, C.c_int32, C.c_uint64, C.c_float
        L.orc_splitmix64.argtypes = [u64, u64, i64, P]
        L.orc_cast_tool.argtypes = [P, P, i64, P, P, i64, i64, P, i32, i32, C.c_double, C.c_double, C.c_double,
                                    P, P, i32]
        L.orc_cast_tool.restype = C.c_int
        L.orc_tool_distance.argtypes = [P, P, P]
        L.orc_tool_distance.restype = C.c_double
        d = C.c_double
        L.orc_cast_tool_holder.argtypes = [P, P, i64, P, P, i64, i64, P, i32, i32, d, d, d, d, d, P, P, i32]
        L.orc_cast_tool_holder.restype = C.c_int
        L.orc_tool_holder_distances.argtypes = [P, P, P, d, d, P]
        L.orc_tool_holder_distances.restype = None
        L.orc_fibonacci_dirs.argtypes = [i32, P]
        L.orc_axes6.argtypes = [P]
        L.orc_frame.argtypes = [P, P, P]
        L.orc_ray_dirs.argtypes = [P, i64, P, i32, i32, P]
        L.orc_mesh_info.argtypes = [P, i64, P, P, P, f32]
        L.orc_area_weights.argtypes = [P, P, i64, P, P]
        L.orc_area_weights.restype = C.c_int
        L.orc_sample_area.argtypes = [P, i64, P, i64, i64, u64, f32, P, P, P, P]
        L.orc_sample_area.restype = C.c_int
        L.orc_sample_centroid.argtypes = [P, i64, P, i64, f32, P, P, P, P]
        L.orc_sample_centroid.restype = C.c_int64
        L.orc_cast.argtypes = [P, i64, P, i64, P, P, i64, i64, P, i32, i32, P, P, P, i32]
        L.orc_cast.restype = C.c_int
        L.orc_cast_rays.argtypes = [P, P, i64, P, P, i64, P, i32]
        L.orc_decide_one.argtypes = [P, P, P, P]
        L.orc_decide_one.restype = C.c_int
        L.orc_dirstats.argtypes = [P, i64, P, i32, P, P, P, P, P, P, P]
        L.orc_max_threads.restype = C.c_int32
        L.orc_bvh_build.argtypes = [P, i64, P, i64, C.c_double]
        L.orc_bvh_build.restype = C.c_void_p
        L.orc_bvh_free.argtypes = [P]
        L.orc_bvh_free.restype = None
        L.orc_bvh_shape.argtypes = [P, P]
        L.orc_bvh_shape.restype = None
        L.orc_bvh_cast.argtypes = [P, P, P, i64, i64, P, i32, i32, P, P, P, P, i32]
        L.orc_bvh_cast.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# --------------------------------------------------------------------------
# generator, directions, frames, rays
# --------------------------------------------------------------------------
def splitmix64(seed, c0, n):
    out = np.empty(n, np.uint64)
    lib().orc_splitmix64(seed, c0, n, _p(out))
    return out


def fibonacci_dirs(n):
    """Section 3.1 / Fig. 1: uniformly sampled hemisphere (spherical Fibonacci)."""
    out = np.empty((n, 3), np.float32)
    lib().orc_fibonacci_dirs(n, _p(out))
    return out


def axes6():
    """Section 3.2: the six principal directions +X,-X,+Y,-Y,+Z,-Z."""
    out = np.empty((6, 3), np.float32)
    lib().orc_axes6(_p(out))
    return out


def frame(n):
    n = _f32(n)
    t = np.empty(3, np.float32)
    b = np.empty(3, np.float32)
    lib().orc_frame(_p(n), _p(t), _p(b))
    return t, b


def ray_dirs(normals, dirs, kind=0):
    """World directions of every (sample, direction) ray, [S][N][3] FP32."""
    normals, dirs = _f32(normals), _f32(dirs)
    S, N = len(normals), len(dirs)
    out = np.empty((S, N, 3), np.float32)
    lib().orc_ray_dirs(_p(normals), S, _p(dirs), N, kind, _p(out))
    return out


# --------------------------------------------------------------------------
# mesh facts and sampling (Section 3.1)
# --------------------------------------------------------------------------
def mesh_info(verts, offset_frac=1e-4):
    v = _f32(verts)
    bbox = np.empty(6, np.float64)
    diag = np.empty(1, np.float64)
    eps = np.empty(1, np.float32)
    lib().orc_mesh_info(_p(v), len(v), _p(bbox), _p(diag), _p(eps), offset_frac)
    return bbox, float(diag[0]), eps[0]


def area_weights(verts, tris):
    v, t = _f32(verts), _i32(tris)
    w = np.empty(len(t), np.uint64)
    k = np.empty(1, np.int32)
    rc = lib().orc_area_weights(_p(v), _p(t), len(t), _p(w), _p(k))
    if rc != 0:
        raise ValueError("mesh has no triangle with nonzero area")
    return w, int(k[0])


def sample_area(verts, tris, n, seed, offset_frac=1e-4):
    """Area-weighted i.i.d. samples: returns dict(point, normal, origin, tri)."""
    v, t = _f32(verts), _i32(tris)
    P = np.empty((n, 3), np.float32)
    Nn = np.empty((n, 3), np.float32)
    O = np.empty((n, 3), np.float32)
    T = np.empty(n, np.int32)
    rc = lib().orc_sample_area(_p(v), len(v), _p(t), len(t), n, seed, offset_frac, _p(P), _p(Nn), _p(O), _p(T))
    if rc != 0:
        raise ValueError("mesh has no triangle with nonzero area")
    return {"point": P, "normal": Nn, "origin": O, "tri": T}


def sample_centroid(verts, tris, offset_frac=1e-4):
    """One sample per face with nonzero area, at its centroid (Section 3.1)."""
    v, t = _f32(verts), _i32(tris)
    n = len(t)
    P = np.empty((n, 3), np.float32)
    Nn = np.empty((n, 3), np.float32)
    O = np.empty((n, 3), np.float32)
    T = np.empty(n, np.int32)
    m = lib().orc_sample_centroid(_p(v), len(v), _p(t), n, offset_frac, _p(P), _p(Nn), _p(O), _p(T))
    return {"point": P[:m], "normal": Nn[:m], "origin": O[:m], "tri": T[:m]}


# --------------------------------------------------------------------------
# casting (Section 3.1 hemisphere, Section 3.2 principal directions)
# --------------------------------------------------------------------------
def cast(verts, tris, samples, dirs, kind=0, s0=0, s1=None, threads=0):
    """Brute-force cast.  Returns (bits, grazing, info), each uint32 [S][W]."""
    v, t = _f32(verts), _i32(tris)
    O, Nn, d = _f32(samples["origin"]), _f32(samples["normal"]), _f32(dirs)
    s1 = len(O) if s1 is None else s1
    N = len(d)
    W = (N + 31) // 32
    S = s1 - s0
    bits = np.empty((S, W), np.uint32)
    gr = np.empty((S, W), np.uint32)
    inf = np.empty((S, W), np.uint32)
    rc = lib().orc_cast(_p(v), len(v), _p(t), len(t), _p(O), _p(Nn), s0, s1, _p(d), N, kind,
                        _p(bits), _p(gr), _p(inf), threads)
    if rc != 0:
        raise MemoryError("oracle cast failed")
    return bits, gr, inf


def cast_rays(verts, tris, origins, dirs, threads=0):
    """Per-ray verdict for explicit (o, d): 0 occluded, 1 unobstructed, 2 grazing."""
    v, t = _f32(verts), _i32(tris)
    O, D = _f32(origins), _f32(dirs)
    out = np.empty(len(O), np.uint8)
    lib().orc_cast_rays(_p(v), _p(t), len(t), _p(O), _p(D), len(O), _p(out), threads)
    return out


BVH_PAD_FRAC = 1e-4     # outward growth of the oracle hierarchy's boxes: 1e-4 x bbox diagonal


class BVHCast:
    """The brute-force cast through a padded median-split hierarchy
    (hra_oracle.c, orc_bvh_cast): the same bits wherever brute force decides
    a ray, and a subset of its grazing flags (equal on every mesh the tests
    compare).  Holds its own copies of the mesh arrays."""

    def __init__(self, verts, tris, pad_frac=BVH_PAD_FRAC):
        self.v, self.t = _f32(verts).copy(), _i32(tris).copy()
        _, diag, _ = mesh_info(self.v)
        self.pad = float(pad_frac) * diag
        self.h = lib().orc_bvh_build(_p(self.v), len(self.v), _p(self.t), len(self.t), self.pad)
        if not self.h:
            raise MemoryError("oracle hierarchy build failed")
        sh = np.zeros(2, np.int64)
        lib().orc_bvh_shape(self.h, _p(sh))
        self.n_nodes, self.depth = int(sh[0]), int(sh[1])
        self.work = np.zeros(2, np.uint64)

    def cast(self, samples, dirs, kind=0, s0=0, s1=None, threads=0):
        """(bits, grazing, info), uint32 [s1 - s0][W], as oracle.cast."""
        O, Nn, d = _f32(samples["origin"]), _f32(samples["normal"]), _f32(dirs)
        s1 = len(O) if s1 is None else s1
        N = len(d)
        W = (N + 31) // 32
        S = s1 - s0
        bits = np.empty((S, W), np.uint32)
        gr = np.empty((S, W), np.uint32)
        inf = np.empty((S, W), np.uint32)
        if S > 0:
            rc = lib().orc_bvh_cast(self.h, _p(O), _p(Nn), s0, s1, _p(d), N, kind, _p(bits), _p(gr), _p(inf),
                                    _p(self.work), threads)
            if rc != 0:
                raise MemoryError("oracle hierarchy cast failed")
        return bits, gr, inf

    def close(self):
        if self.h:
            lib().orc_bvh_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cast_bvh(verts, tris, samples, dirs, kind=0, s0=0, s1=None, threads=0):
    """oracle.cast through the padded hierarchy (one-off build)."""
    b = BVHCast(verts, tris)
    try:
        return b.cast(samples, dirs, kind, s0, s1, threads)
    finally:
        b.close()


TOOL_TOL_FRAC = 1e-4    # tool clearance tolerance: 1e-4 x bbox diagonal
TOOL_BAND_FRAC = 1e-9   # decisions this close to the threshold (x diagonal) are ambiguous


def cast_tool(verts, tris, samples, dirs, radius, kind=0, s0=0, s1=None, threads=0):
    """Brute-force tool cast (ball-end tool of `radius` touching each sample
    point from outside).  Returns (bits, ambiguous), uint32 [S][W]."""
    v, t = _f32(verts), _i32(tris)
    Pt, Nn, d = _f32(samples["point"]), _f32(samples["normal"]), _f32(dirs)
    s1 = len(Pt) if s1 is None else s1
    N = len(d)
    W = (N + 31) // 32
    S = s1 - s0
    _, diag, _ = mesh_info(verts)
    bits = np.empty((S, W), np.uint32)
    amb = np.empty((S, W), np.uint32)
    lib().orc_cast_tool(_p(v), _p(t), len(t), _p(Pt), _p(Nn), s0, s1, _p(d), N, kind, float(radius),
                        TOOL_TOL_FRAC * diag, TOOL_BAND_FRAC * diag, _p(bits), _p(amb), threads)
    return bits, amb


def cast_tool_holder(verts, tris, samples, dirs, radius, cut_length, holder_radius, kind=0, threads=0):
    """Brute-force tool cast with a holder: the ball-end tool of `radius`
    (every point within radius of the approach half-line from the tip
    centre), and a holder of `holder_radius` about the half-line that starts
    cut_length + holder_radius above the tip centre, so that its rounded nose
    reaches down to the end of the cutting length.  Blocked when a triangle
    comes within radius - tol of the tool's half-line or within
    holder_radius - tol of the holder's.  Returns (bits, ambiguous)."""
    v, t = _f32(verts), _i32(tris)
    Pt, Nn, d = _f32(samples["point"]), _f32(samples["normal"]), _f32(dirs)
    S, N = len(Pt), len(d)
    W = (N + 31) // 32
    _, diag, _ = mesh_info(verts)
    bits = np.empty((S, W), np.uint32)
    amb = np.empty((S, W), np.uint32)
    lib().orc_cast_tool_holder(_p(v), _p(t), len(t), _p(Pt), _p(Nn), 0, S, _p(d), N, kind, float(radius),
                               float(cut_length), float(holder_radius), TOOL_TOL_FRAC * diag, TOOL_BAND_FRAC * diag,
                               _p(bits), _p(amb), threads)
    return bits, amb


def tool_holder_distances(tri9, c, u, cut_length, holder_radius):
    """FP64 (distance from the tool's half-line c + t u, t >= 0, distance
    from the holder's half-line from c + (cut_length + holder_radius) u) to
    a triangle."""
    a = np.ascontiguousarray(tri9, np.float64).reshape(9)
    out = np.zeros(2, np.float64)
    lib().orc_tool_holder_distances(_p(a), _p(np.ascontiguousarray(c, np.float64)),
                                    _p(np.ascontiguousarray(u, np.float64)), float(cut_length),
                                    float(holder_radius), _p(out))
    return float(out[0]), float(out[1])


def tool_distance(tri9, c, u):
    """FP64 distance between the half-line c + t u (t >= 0, u unit) and a triangle (9 coordinates)."""
    a = np.ascontiguousarray(tri9, np.float64).reshape(9)
    return lib().orc_tool_distance(_p(a), _p(np.ascontiguousarray(c, np.float64)),
                                   _p(np.ascontiguousarray(u, np.float64)))


def decide_one(tri9, o, d):
    """(decision, info) for one ray/triangle pair; decision 0 miss, 1 hit, 2 ambiguous."""
    v = np.ascontiguousarray(tri9, np.float64).reshape(9)
    o = np.ascontiguousarray(o, np.float64)
    d = np.ascontiguousarray(d, np.float64)
    info = np.zeros(1, np.int32)
    r = lib().orc_decide_one(_p(v), _p(o), _p(d), _p(info))
    return int(r), int(info[0])


def unpack_bits(words, n):
    """uint32 [S][W] -> bool [S][n], bit j%32 of word j/32 = direction j."""
    w = np.ascontiguousarray(words, np.uint32)
    b = np.unpackbits(w.view(np.uint8).reshape(w.shape[0], -1), axis=1, bitorder="little")
    return b[:, :n].astype(bool)


def counts(bits, n):
    """Section 3.1: number of unobstructed rays per sample."""
    return unpack_bits(bits, n).sum(1).astype(np.int64)


# --------------------------------------------------------------------------
# directional statistics (Section 3.3)
# --------------------------------------------------------------------------
def dirstats(samples, dirs, bits):
    Nn, d = _f32(samples["normal"]), _f32(dirs)
    S, N = len(Nn), len(d)
    b = np.ascontiguousarray(bits, np.uint32)
    mean = np.empty((S, 3), np.float64)
    absmean = np.empty((S, 3), np.float64)
    axis = np.empty(S, np.int8)
    conc = np.empty(S, np.float64)
    tie = np.empty(S, np.uint8)
    hist = np.empty(8192, np.uint64)
    lib().orc_dirstats(_p(Nn), S, _p(d), N, _p(b), _p(mean), _p(absmean), _p(axis), _p(conc), _p(tie), _p(hist))
    return {"mean": mean, "absmean": absmean, "axis": axis, "conc": conc, "tie": tie.astype(bool), "hist": hist}


DEFAULT_THRESHOLDS = {"min_access": 0.60, "min_share": 0.45, "max_conc": 0.40}


def indicators(cnt, n_dirs, axis, conc):
    """Section 3.3 indicators.  Overall accessibility = mean over samples of
    unobstructed/total (area-weighted by construction of the samples);
    dominant-axis shares over samples with at least one unobstructed ray
    (they sum to 1); mean concentration over the same samples."""
    cnt = np.asarray(cnt, np.int64)
    axis = np.asarray(axis)
    inc = axis >= 0
    n_inc = int(inc.sum())
    access = float(cnt.sum()) / float(len(cnt) * n_dirs) if len(cnt) else 0.0
    shares = [float((axis == k).sum()) / n_inc if n_inc else 0.0 for k in range(3)]
    cbar = float(np.sum(np.asarray(conc, np.float64)[inc])) / n_inc if n_inc else 0.0
    return {"access": access, "shares": shares, "conc": cbar, "n_included": n_inc,
            "n_blind": int(len(cnt) - n_inc)}


def classify(ind, th=None):
    """Section 3.3: multi-axis if any indicator crosses its threshold.
    Returns (is_multi_axis, tripped) with tripped a bitmask:
    1 = accessibility below min, 2 = max share below min, 4 = concentration above max."""
    th = dict(DEFAULT_THRESHOLDS, **(th or {}))
    tripped = 0
    if ind["access"] < th["min_access"]:
        tripped |= 1
    if max(ind["shares"]) < th["min_share"]:
        tripped |= 2
    if ind["conc"] > th["max_conc"]:
        tripped |= 4
    return tripped != 0, tripped


# --------------------------------------------------------------------------
# reach, fixture faces, classes, setups (Section 3.3, last paragraph)
# --------------------------------------------------------------------------
def bbox_face_tris(verts, tris, bbox, diag):
    """A triangle lies on the stock's bounding box (a fixture face) when all
    three vertices lie on the same bbox plane within 1e-6 x diag."""
    v = np.asarray(verts, np.float64)[np.asarray(tris)]
    tol = 1e-6 * diag
    out = np.zeros(len(tris), bool)
    for c in range(3):
        for lim in (bbox[c], bbox[3 + c]):
            out |= np.all(np.abs(v[:, :, c] - lim) <= tol, axis=1)
    return out


def reach_classes(points, tri, axes_bits, bbox, bbox_tri, tool_length):
    """travel along +k = bbox_max_k - p_k, along -k = p_k - bbox_min_k (FP64);
    direction k reachable iff accessible and travel <= tool length.
    class: 0 viable, 1 over-threshold, 2 inaccessible, 3 fixture face.
    Returns (class u8 [S], code u8 [S] of reachable directions)."""
    p = np.asarray(points, np.float64)
    ab = np.asarray(axes_bits, np.uint32).reshape(-1) & 63
    travel = np.stack([bbox[3] - p[:, 0], p[:, 0] - bbox[0], bbox[4] - p[:, 1], p[:, 1] - bbox[1],
                       bbox[5] - p[:, 2], p[:, 2] - bbox[2]], 1)
    acc = ((ab[:, None] >> np.arange(6)) & 1).astype(bool)
    reach = acc & (travel <= tool_length)
    code = (reach * (1 << np.arange(6))).sum(1).astype(np.uint8)
    cls = np.where(reach.any(1), 0, np.where(acc.any(1), 1, 2)).astype(np.uint8)
    cls[np.asarray(bbox_tri)[np.asarray(tri)]] = 3
    code[cls != 0] = 0
    return cls, code


def code_histogram(cls, code):
    h = np.zeros(64, np.int64)
    np.add.at(h, np.asarray(code)[np.asarray(cls) == 0].astype(np.int64), 1)
    return h


def min_setups_exact(hist):
    """Smallest set M of directions such that every occurring code meets M;
    ties -> numerically smallest mask.  Exhaustive over all 63 subsets."""
    codes = [c for c in range(64) if hist[c] > 0]
    if not codes:
        return 0, 0
    if any(c == 0 for c in codes):
        raise ValueError("a viable sample has no reachable direction")
    best = None
    for size in range(1, 7):
        for combo in itertools.combinations(range(6), size):
            m = sum(1 << k for k in combo)
            if all(c & m for c in codes):
                if best is None or m < best:
                    best = m
        if best is not None:
            return size, best
    raise AssertionError


def min_setups_greedy(hist):
    """The paper's greedy set cover: repeatedly take the direction that covers
    the most still-uncovered viable samples (ties -> lowest index)."""
    left = {c: int(hist[c]) for c in range(64) if hist[c] > 0}
    mask = 0
    n = 0
    while left:
        gain = [sum(v for c, v in left.items() if c >> k & 1) if not (mask >> k & 1) else -1 for k in range(6)]
        k = int(np.argmax(gain))
        if gain[k] <= 0:
            raise ValueError("uncoverable code")
        mask |= 1 << k
        n += 1
        left = {c: v for c, v in left.items() if not (c & mask)}
    return n, mask


def max_threads():
    return int(lib().orc_max_threads())


# --------------------------------------------------------------------------
# dominant directions from the direction histogram (the multi-axis workload)
# --------------------------------------------------------------------------
def bin_centre(b):
    """Centre direction of histogram bin b (64 equal-area z bands x 128 sectors)."""
    zb, az = b // 128, b % 128
    z = (zb + 0.5) / 32.0 - 1.0
    phi = (az + 0.5) * (2 * np.pi / 128) - np.pi
    r = np.sqrt(max(0.0, 1 - z * z))
    return np.array([r * np.cos(phi), r * np.sin(phi), z])


def histogram_bin(d):
    """Bin of a world direction, FP64 (the definition the statistics use)."""
    d = np.asarray(d, np.float64)
    zh = d[2] / np.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
    zb = min(63, max(0, int(np.floor((zh + 1.0) * 32.0))))
    az = min(127, max(0, int(np.floor((np.arctan2(d[1], d[0]) + np.pi) * 128.0 / (2 * np.pi)))))
    return zb * 128 + az


def histogram_peaks(hist, k=8):
    """Local maxima over the 3x3 bin window (azimuth wraps, lower bin wins
    ties), largest first; and the mass within 45 degrees of each axis."""
    h = np.asarray(hist, np.int64).reshape(64, 128)
    peaks = []
    for zb in range(64):
        for az in range(128):
            v = h[zb, az]
            if v == 0:
                continue
            b = zb * 128 + az
            ok = True
            for dz in (-1, 0, 1):
                z2 = zb + dz
                if z2 < 0 or z2 > 63:
                    continue
                for da in (-1, 0, 1):
                    if dz == 0 and da == 0:
                        continue
                    a2 = (az + da) % 128
                    b2 = z2 * 128 + a2
                    if h[z2, a2] > v or (h[z2, a2] == v and b2 < b):
                        ok = False
            if ok:
                peaks.append((-int(v), b))
    peaks.sort()
    peaks = peaks[:k]
    axis_mass = [0] * 6
    for b in np.nonzero(h.reshape(-1))[0]:
        c = bin_centre(b)
        for a in range(6):
            comp = -c[a // 2] if a % 2 else c[a // 2]
            if comp > np.sqrt(0.5):
                axis_mass[a] += int(h.reshape(-1)[b])
    return {"bins": [b for _, b in peaks], "mass": [-m for m, _ in peaks], "axis_mass": axis_mass}

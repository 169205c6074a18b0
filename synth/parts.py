"""Seeded procedural CAD-like parts: watertight, outward-wound triangle meshes.

This module only produces input geometry (vertex and triangle arrays); it holds
none of the accessibility method's arithmetic, so both the CPU oracle and the
GPU path can consume what it makes.

Construction.  A part is a block [0,W]x[0,D]x[0,H] (mm, min corner at the
origin).  Every block face is a rectangular lattice of square cells; a feature
(pocket, blind hole, T-slot, dovetail, inclined bore) replaces a rectangle of
cells (a "macro cell").  Vertices on the block surface are keyed by integer 3D
lattice coordinates, so faces that share a block edge share vertices exactly.
A feature's rim is either the macro cell boundary itself (full pockets) or a
convex polygon strictly inside it, joined to the boundary by an angular zipper
triangulation.  Walls are quad strips between rings with equal vertex counts;
floors are fans or nested lattices that can hold further features.  The result
has no T-junctions: every directed edge appears once and its reverse once.

Features hang from their face into the material and are confined to disjoint
columns (top-face features stay away from the side faces by more than the
side-feature depth), so they never intersect each other.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# ----------------------------------------------------------------------------
# mesh container
# ----------------------------------------------------------------------------
class MeshBuilder:
    def __init__(self):
        self._v: list[np.ndarray] = []
        self._t: list[np.ndarray] = []
        self.nv = 0
        self.nt = 0
        self.notes: list[dict] = []   # feature records (e.g. bore axes) for tests

    def add_verts(self, p) -> np.ndarray:
        p = np.asarray(p, dtype=np.float64).reshape(-1, 3)
        idx = np.arange(self.nv, self.nv + len(p), dtype=np.int64)
        self._v.append(p)
        self.nv += len(p)
        return idx

    def add_tris(self, t) -> None:
        t = np.asarray(t, dtype=np.int64).reshape(-1, 3)
        if len(t):
            self._t.append(t)
            self.nt += len(t)

    def arrays(self):
        """float32 vertices (unused ones dropped) and int32 triangles."""
        v = np.concatenate(self._v) if self._v else np.zeros((0, 3))
        t = np.concatenate(self._t) if self._t else np.zeros((0, 3), np.int64)
        used = np.zeros(len(v), bool)
        used[t.ravel()] = True
        remap = np.cumsum(used) - 1
        return v[used].astype(np.float32), remap[t].astype(np.int32)


@dataclass
class Mesh:
    verts: np.ndarray  # float32 [V,3]
    tris: np.ndarray   # int32 [T,3], counter-clockwise seen from outside
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_tris(self):
        return int(self.tris.shape[0])

    def bbox(self):
        return self.verts.min(0), self.verts.max(0)


# ----------------------------------------------------------------------------
# geometry helpers
# ----------------------------------------------------------------------------
class Frame:
    """Planar frame: origin + u*eu + v*ev + h*en (en = outward face normal)."""

    def __init__(self, origin, eu, ev, en):
        self.o = np.asarray(origin, np.float64)
        self.eu = np.asarray(eu, np.float64)
        self.ev = np.asarray(ev, np.float64)
        self.en = np.asarray(en, np.float64)

    def pos(self, u, v, h=0.0):
        u = np.asarray(u, np.float64)[..., None]
        v = np.asarray(v, np.float64)[..., None]
        h = np.asarray(h, np.float64)[..., None]
        return self.o + u * self.eu + v * self.ev + h * self.en


def _orient(a, b, c):
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])


def zipper(outer_ids, outer_uv, inner_ids, inner_uv, centre, flip=False):
    """Triangulate the annulus between two nested convex CCW rings (2D coords
    in the face frame).  Walks both rings in angular order about `centre`;
    a step that would make a bridge edge cut through the inner polygon is
    replaced by the other step, so every triangle lies in the annulus.
    Triangles are CCW in (u,v) unless `flip`."""
    c = np.asarray(centre, np.float64)
    O = np.asarray(outer_uv, np.float64)
    I = np.asarray(inner_uv, np.float64)
    no, ni = len(O), len(I)
    ao = np.arctan2(O[:, 1] - c[1], O[:, 0] - c[0])
    ai = np.arctan2(I[:, 1] - c[1], I[:, 0] - c[0])

    def sees(p, k):
        """p (outside I) sees inner vertex k without crossing I's interior."""
        km, kp = (k - 1) % ni, (k + 1) % ni
        return _orient(I[km], I[k], p) <= 0 or _orient(I[k], I[kp], p) <= 0

    so = int(np.argmin(ao))
    # inner start: visible vertex closest in angle to the outer start
    cand = [k for k in range(ni) if sees(O[so], k)]
    dang = [abs((ai[k] - ao[so] + math.pi) % (2 * math.pi) - math.pi) for k in cand]
    si = cand[int(np.argmin(dang))]

    def unwrap(a, s, ref):
        r = np.roll(a, -s).copy()
        r = ref + np.mod(r - ref, 2 * math.pi)
        out = np.empty(len(r) + 1)
        out[:-1] = r
        out[-1] = r[0] + 2 * math.pi
        for k in range(1, len(out)):
            while out[k] < out[k - 1]:
                out[k] += 2 * math.pi
        return out

    ref = min(ao[so], ai[si]) - 1e-12
    uo, ui = unwrap(ao, so, ref), unwrap(ai, si, ref)
    tris = []
    i = j = 0
    while i < no or j < ni:
        oi, oi1 = (so + i) % no, (so + i + 1) % no
        ij, ij1 = (si + j) % ni, (si + j + 1) % ni
        can_o = i < no and sees(O[oi1], ij) and _orient(O[oi], O[oi1], I[ij]) > 0
        can_i = j < ni and sees(O[oi], ij1) and _orient(I[ij1], I[ij], O[oi]) > 0
        if can_o and can_i:
            take_o = uo[i + 1] <= ui[j + 1]
        elif can_o or can_i:
            take_o = can_o
        else:
            raise RuntimeError("annulus triangulation failed")
        if take_o:
            tris.append((outer_ids[oi], outer_ids[oi1], inner_ids[ij]))
            i += 1
        else:
            tris.append((inner_ids[ij1], inner_ids[ij], outer_ids[oi]))
            j += 1
    t = np.asarray(tris, np.int64)
    if flip:
        t = t[:, ::-1]
    return t


def strip(r0, r1):
    """Quad strip between two rings of equal length (closed).  With r0 CCW
    (seen from the face's outward side) and r1 below it, the wall's outward
    normal points into the cavity enclosed by the rings."""
    r0 = np.asarray(r0)
    r1 = np.asarray(r1)
    a, b = r0, np.roll(r0, -1)
    c, d = np.roll(r1, -1), r1
    t1 = np.stack([a, b, c], 1)
    t2 = np.stack([a, c, d], 1)
    return np.concatenate([t1, t2])


def fan(mb, ring_ids, centre_xyz, flip=False):
    ci = mb.add_verts(centre_xyz)[0]
    r = np.asarray(ring_ids)
    t = np.stack([np.full(len(r), ci), r, np.roll(r, -1)], 1)
    if flip:
        t = t[:, ::-1]
    return t


def polygon_ccw(cu, cv, r, k, phase=0.0):
    ang = phase + 2 * math.pi * np.arange(k) / k
    return np.stack([cu + r * np.cos(ang), cv + r * np.sin(ang)], 1)


def rect_ring(u0, v0, u1, v1, nu, nv):
    """CCW ring of points on a rectangle with nu segments along u, nv along v."""
    us = u0 + (u1 - u0) * np.arange(nu) / nu
    vs = v0 + (v1 - v0) * np.arange(nv) / nv
    bottom = np.stack([us, np.full(nu, v0)], 1)
    right = np.stack([np.full(nv, u1), vs], 1)
    top = np.stack([u1 - (us - u0), np.full(nu, v1)], 1)
    left = np.stack([np.full(nv, u0), v1 - (vs - v0)], 1)
    return np.concatenate([bottom, right, top, left])


# ----------------------------------------------------------------------------
# lattice surfaces
# ----------------------------------------------------------------------------
class Surf:
    """A planar rectangle [0,U]x[0,V] in `frame`, split into nu x nv cells of
    M x M lattice sub-squares each.  `vid(a,b)` returns the vertex index of
    lattice point (a,b); `pos(a,b)` its local (u,v)."""

    def __init__(self, mb, frame, U, V, nu, nv, M, key=None, inset=0.0, h=0.0):
        self.mb, self.f = mb, frame
        self.U, self.V, self.nu, self.nv, self.M = U, V, nu, nv, M
        self.key = key          # optional (a,b) -> global key for shared vertices
        self.inset, self.h = inset, h
        self.local: dict = {}
        self.shared: dict | None = None
        self.occ = np.zeros((nu, nv), bool)
        self.features: list = []

    def uv(self, a, b):
        A, B = self.nu * self.M, self.nv * self.M
        u = self.inset + (self.U - 2 * self.inset) * (np.asarray(a, np.float64) / A)
        v = self.inset + (self.V - 2 * self.inset) * (np.asarray(b, np.float64) / B)
        return u, v

    def vid(self, a, b):
        if self.key is not None:
            k = self.key(a, b)
            d = self.shared
        else:
            k = (a, b)
            d = self.local
        i = d.get(k)
        if i is None:
            u, v = self.uv(a, b)
            i = int(self.mb.add_verts(self.f.pos(u, v, self.h))[0])
            d[k] = i
        return i

    def preassign(self, a, b, vid):
        self.local[(a, b)] = vid

    def boundary(self, a0, b0, a1, b1):
        """Lattice points on the rectangle boundary, CCW from (a0,b0)."""
        pts = [(a, b0) for a in range(a0, a1)] + [(a1, b) for b in range(b0, b1)] + \
              [(a, b1) for a in range(a1, a0, -1)] + [(a0, b) for b in range(b1, b0, -1)]
        return pts

    def free(self, c0, d0, c1, d1, gap=1):
        if c0 < 0 or d0 < 0 or c1 > self.nu or d1 > self.nv:
            return False
        return not self.occ[max(0, c0 - gap):c1 + gap, max(0, d0 - gap):d1 + gap].any()

    def add(self, c0, d0, c1, d1, feat):
        self.occ[c0:c1, d0:d1] = True
        self.features.append((c0, d0, c1, d1, feat))

    def cell_size(self):
        return (self.U - 2 * self.inset) / self.nu, (self.V - 2 * self.inset) / self.nv

    def lattice_ids(self):
        """Vertex ids of every lattice point, created in bulk (interior points
        of macro cells end up unused and are dropped when the mesh is built)."""
        A, B = self.nu * self.M, self.nv * self.M
        ids = np.empty((A + 1, B + 1), np.int64)
        aa, bb = np.meshgrid(np.arange(A + 1), np.arange(B + 1), indexing="ij")
        edge = (aa == 0) | (aa == A) | (bb == 0) | (bb == B)
        if self.key is not None or self.local:
            for a, b in zip(aa[edge], bb[edge]):
                ids[a, b] = self.vid(int(a), int(b))
        else:
            u, v = self.uv(aa[edge], bb[edge])
            ids[edge] = self.mb.add_verts(self.f.pos(u, v, self.h))
            for a, b, i in zip(aa[edge], bb[edge], ids[edge]):
                self.local[(int(a), int(b))] = int(i)
        inner = ~edge
        u, v = self.uv(aa[inner], bb[inner])
        ids[inner] = self.mb.add_verts(self.f.pos(u, v, self.h))
        return ids

    def emit(self):
        M, mb = self.M, self.mb
        ids = self.lattice_ids()
        self._ids = ids
        # plain cells, vectorised over lattice sub-squares
        free = ~np.repeat(np.repeat(self.occ, M, 0), M, 1)
        a, b = np.nonzero(free)
        p00, p10, p11, p01 = ids[a, b], ids[a + 1, b], ids[a + 1, b + 1], ids[a, b + 1]
        mb.add_tris(np.concatenate([np.stack([p00, p10, p11], 1), np.stack([p00, p11, p01], 1)]))
        for (c0, d0, c1, d1, feat) in self.features:
            pts = self.boundary(c0 * M, d0 * M, c1 * M, d1 * M)
            pa = np.array([p[0] for p in pts])
            pb = np.array([p[1] for p in pts])
            bids = ids[pa, pb]
            uv = np.stack(self.uv(pa, pb), 1)
            rect = (*self.uv(c0 * M, d0 * M), *self.uv(c1 * M, d1 * M))
            feat.emit(self, bids, uv, rect, (c1 - c0) * M, (d1 - d0) * M)


# ----------------------------------------------------------------------------
# features
# ----------------------------------------------------------------------------
@dataclass
class Hole:
    """Blind cylindrical hole: k-gon inscribed at radius r, flat floor."""
    cu: float
    cv: float
    r: float
    depth: float
    k: int
    phase: float = 0.0

    def emit(self, s: Surf, ids, uv, rect, nA, nB):
        mb, f = s.mb, s.f
        rim_uv = polygon_ccw(self.cu, self.cv, self.r, self.k, self.phase)
        rim = mb.add_verts(f.pos(rim_uv[:, 0], rim_uv[:, 1], s.h))
        mb.add_tris(zipper(ids, uv, rim, rim_uv, (self.cu, self.cv)))
        bot = mb.add_verts(f.pos(rim_uv[:, 0], rim_uv[:, 1], s.h - self.depth))
        mb.add_tris(strip(rim, bot))
        mb.add_tris(fan(mb, bot, f.pos(self.cu, self.cv, s.h - self.depth)))


@dataclass
class Pocket:
    """Pocket whose rim is the macro-cell boundary; vertical walls, optional
    quarter-round floor fillet of radius rf with nf segments, flat floor that
    is itself a lattice surface and may hold sub-features."""
    depth: float
    rf: float = 0.0
    nf: int = 0
    sub: list = field(default_factory=list)   # (c0,d0,c1,d1,feature) on the floor grid
    floor: Surf | None = None

    def make_floor(self, s: Surf, rect, nA, nB, nu, nv):
        u0, v0, u1, v1 = rect
        o = s.f.o + u0 * s.f.eu + v0 * s.f.ev
        fr = Frame(o, s.f.eu, s.f.ev, s.f.en)
        self.floor = Surf(s.mb, fr, u1 - u0, v1 - v0, nu, nv, nA // nu if nu else 1,
                          inset=self.rf, h=s.h - self.depth)
        return self.floor

    def emit(self, s: Surf, ids, uv, rect, nA, nB):
        mb, f = s.mb, s.f
        u0, v0, u1, v1 = rect
        fl = self.floor
        assert fl is not None and fl.nu * fl.M == nA and fl.nv * fl.M == nB
        # rings: rim -> (walls) -> fillet rings -> floor boundary
        rings = [ids]
        nfr = self.nf if self.rf > 0 else 0
        wall_bottom = self.depth - self.rf
        Wd, Hd = u1 - u0, v1 - v0
        a_rel = (uv[:, 0] - u0) / Wd
        b_rel = (uv[:, 1] - v0) / Hd

        def ring_at(inset, hdepth):
            uu = u0 + inset + (Wd - 2 * inset) * a_rel
            vv = v0 + inset + (Hd - 2 * inset) * b_rel
            return mb.add_verts(f.pos(uu, vv, s.h - hdepth))

        if self.rf > 0:
            rings.append(ring_at(0.0, wall_bottom))
            for q in range(1, nfr):
                th = 0.5 * math.pi * q / nfr
                rings.append(ring_at(self.rf * (1 - math.cos(th)), wall_bottom + self.rf * math.sin(th)))
        # floor boundary ring from the floor lattice (shared vertices)
        for (c0, d0, c1, d1, feat) in self.sub:
            fl.add(c0, d0, c1, d1, feat)
        fl.emit()
        pts = fl.boundary(0, 0, nA, nB)
        last = fl._ids[np.array([p[0] for p in pts]), np.array([p[1] for p in pts])]
        rings.append(last)
        for r0, r1 in zip(rings[:-1], rings[1:]):
            mb.add_tris(strip(r0, r1))


@dataclass
class TSlot:
    """Blind T-slot: a narrow neck from the face, then a wider chamber (an
    undercut).  Neck: rectangle [nu0,nu1]x[nv0,nv1], depth d1; chamber:
    rectangle [cu0,cu1]x[cv0,cv1] from d1 to d2."""
    neck: tuple
    chamber: tuple
    d1: float
    d2: float
    seg: int = 2

    def emit(self, s: Surf, ids, uv, rect, nA, nB):
        mb, f = s.mb, s.f
        n0, n1, n2, n3 = self.neck
        c0, c1, c2, c3 = self.chamber
        kn = max(1, self.seg)
        neck_uv = rect_ring(n0, n1, n2, n3, kn * 4, kn)
        ch_uv = rect_ring(c0, c1, c2, c3, kn * 4, kn * 2)
        cen = ((n0 + n2) / 2, (n1 + n3) / 2)
        rim = mb.add_verts(f.pos(neck_uv[:, 0], neck_uv[:, 1], s.h))
        mb.add_tris(zipper(ids, uv, rim, neck_uv, cen))
        neck_bot = mb.add_verts(f.pos(neck_uv[:, 0], neck_uv[:, 1], s.h - self.d1))
        mb.add_tris(strip(rim, neck_bot))
        ch_top = mb.add_verts(f.pos(ch_uv[:, 0], ch_uv[:, 1], s.h - self.d1))
        # ceiling of the chamber faces down into the cavity
        mb.add_tris(zipper(ch_top, ch_uv, neck_bot, neck_uv, cen, flip=True))
        ch_bot = mb.add_verts(f.pos(ch_uv[:, 0], ch_uv[:, 1], s.h - self.d2))
        mb.add_tris(strip(ch_top, ch_bot))
        mb.add_tris(fan(mb, ch_bot, f.pos(cen[0], cen[1], s.h - self.d2)))


@dataclass
class Dovetail:
    """Dovetail recess: rectangular rim, walls flaring outward by `flare`
    per side down to depth `depth` (an undercut), flat floor."""
    rim: tuple
    depth: float
    flare: float
    seg: int = 2

    def emit(self, s: Surf, ids, uv, rect, nA, nB):
        mb, f = s.mb, s.f
        r0, r1, r2, r3 = self.rim
        e = self.flare
        k = max(1, self.seg)
        top_uv = rect_ring(r0, r1, r2, r3, 3 * k, k)
        bot_uv = rect_ring(r0 - e, r1 - e, r2 + e, r3 + e, 3 * k, k)
        cen = ((r0 + r2) / 2, (r1 + r3) / 2)
        rim = mb.add_verts(f.pos(top_uv[:, 0], top_uv[:, 1], s.h))
        mb.add_tris(zipper(ids, uv, rim, top_uv, cen))
        bot = mb.add_verts(f.pos(bot_uv[:, 0], bot_uv[:, 1], s.h - self.depth))
        mb.add_tris(strip(rim, bot))
        mb.add_tris(fan(mb, bot, f.pos(cen[0], cen[1], s.h - self.depth)))


@dataclass
class Bore:
    """Blind cylindrical bore of radius r whose axis is tilted by `tilt` from
    the face normal at azimuth `azim`; its axis length from the rim centre
    is `length`; flat bottom perpendicular to the axis."""
    cu: float
    cv: float
    r: float
    length: float
    tilt: float
    azim: float
    k: int

    def axis_local(self):
        st, ct = math.sin(self.tilt), math.cos(self.tilt)
        return np.array([st * math.cos(self.azim), st * math.sin(self.azim), -ct])

    def footprint(self):
        """(umin, vmin, umax, vmax) of the rim and the bottom disk, projected."""
        a = self.axis_local()
        e1, e2 = _perp(a)
        ang = 2 * math.pi * np.arange(64) / 64
        circ = self.r * (np.cos(ang)[:, None] * e1 + np.sin(ang)[:, None] * e2)
        rim = self._rim_pts(circ, a)
        bot = np.array([self.cu, self.cv, 0.0]) + self.length * a + circ
        pts = np.concatenate([rim, bot])
        return pts[:, 0].min(), pts[:, 1].min(), pts[:, 0].max(), pts[:, 1].max(), -pts[:, 2].max() * -1

    def max_depth(self):
        a = self.axis_local()
        return self.length * (-a[2]) + self.r * math.sin(self.tilt)

    def _rim_pts(self, circ, a):
        p0 = np.array([self.cu, self.cv, 0.0]) + circ
        s = -p0[:, 2] / a[2]
        return p0 + s[:, None] * a

    def emit(self, s: Surf, ids, uv, rect, nA, nB):
        mb, f = s.mb, s.f
        a = self.axis_local()
        e1, e2 = _perp(a)
        ang = 2 * math.pi * np.arange(self.k) / self.k
        circ = self.r * (np.cos(ang)[:, None] * e1 + np.sin(ang)[:, None] * e2)
        rim_l = self._rim_pts(circ, a)
        rim_uv = rim_l[:, :2]
        # make the rim CCW in (u,v)
        area = 0.5 * np.sum(rim_uv[:, 0] * np.roll(rim_uv[:, 1], -1) - np.roll(rim_uv[:, 0], -1) * rim_uv[:, 1])
        order = np.arange(self.k) if area > 0 else np.arange(self.k)[::-1]
        rim_uv = rim_uv[order]
        circ = circ[order]
        bot_l = np.array([self.cu, self.cv, 0.0]) + self.length * a + circ
        rim = mb.add_verts(f.pos(rim_uv[:, 0], rim_uv[:, 1], s.h))
        mb.add_tris(zipper(ids, uv, rim, rim_uv, (self.cu, self.cv)))
        bot = mb.add_verts(f.pos(bot_l[:, 0], bot_l[:, 1], s.h + bot_l[:, 2]))
        mb.add_tris(strip(rim, bot))
        c = np.array([self.cu, self.cv, 0.0]) + self.length * a
        t0 = mb.nt
        mb.add_tris(fan(mb, bot, f.pos(c[0], c[1], s.h + c[2])))
        out_axis = -(a[0] * f.eu + a[1] * f.ev + a[2] * f.en)
        mb.notes.append({"kind": "bore", "floor_tris": (t0, mb.nt), "axis": out_axis.tolist(),
                         "floor_centre": f.pos(c[0], c[1], s.h + c[2]).tolist(), "r": self.r,
                         "tilt": self.tilt, "length": self.length,
                         "rim": f.pos(rim_uv[:, 0], rim_uv[:, 1], s.h).tolist(),
                         "face_normal": f.en.tolist(), "face_point": f.pos(0.0, 0.0, s.h).tolist(),
                         "face_axes": [f.eu.tolist(), f.ev.tolist()]})


def _perp(a):
    a = a / np.linalg.norm(a)
    t = np.array([1.0, 0, 0]) if abs(a[0]) < 0.9 else np.array([0, 1.0, 0])
    e1 = np.cross(a, t)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(a, e1)
    return e1, e2


# ----------------------------------------------------------------------------
# block with six lattice faces
# ----------------------------------------------------------------------------
class Block:
    def __init__(self, W, D, H, cs, M=1):
        self.W, self.D, self.H = W, D, H
        self.gx, self.gy, self.gz = int(round(W / cs)), int(round(D / cs)), int(round(H / cs))
        assert abs(self.gx * cs - W) < 1e-9 and abs(self.gy * cs - D) < 1e-9 and abs(self.gz * cs - H) < 1e-9
        self.cs, self.M = cs, M
        self.mb = MeshBuilder()
        self.shared: dict = {}
        NX, NY, NZ = self.gx * M, self.gy * M, self.gz * M
        self.N = (NX, NY, NZ)

        def mk(frame, U, V, nu, nv, keyf):
            s = Surf(self.mb, frame, U, V, nu, nv, M, key=keyf)
            s.shared = self.shared
            s.uv3 = None
            return s

        # global position from lattice key, identical for every face
        def posk(k):
            i, j, l = k
            return np.array([W * i / NX, D * j / NY, H * l / NZ])

        self._posk = posk
        self.faces = {
            "+Z": mk(Frame((0, 0, H), (1, 0, 0), (0, 1, 0), (0, 0, 1)), W, D, self.gx, self.gy,
                     lambda a, b: (a, b, NZ)),
            "-Z": mk(Frame((0, 0, 0), (0, 1, 0), (1, 0, 0), (0, 0, -1)), D, W, self.gy, self.gx,
                     lambda a, b: (b, a, 0)),
            "+X": mk(Frame((W, 0, 0), (0, 1, 0), (0, 0, 1), (1, 0, 0)), D, H, self.gy, self.gz,
                     lambda a, b: (NX, a, b)),
            "-X": mk(Frame((0, 0, 0), (0, 0, 1), (0, 1, 0), (-1, 0, 0)), H, D, self.gz, self.gy,
                     lambda a, b: (0, b, a)),
            "+Y": mk(Frame((0, D, 0), (0, 0, 1), (1, 0, 0), (0, 1, 0)), H, W, self.gz, self.gx,
                     lambda a, b: (b, NY, a)),
            "-Y": mk(Frame((0, 0, 0), (1, 0, 0), (0, 0, 1), (0, -1, 0)), W, H, self.gx, self.gz,
                     lambda a, b: (a, 0, b)),
        }
        # shared-vertex creation goes through the global key position
        for s in self.faces.values():
            s.vid = self._make_vid(s)

    def _make_vid(self, s):
        def vid(a, b):
            k = s.key(a, b)
            i = self.shared.get(k)
            if i is None:
                i = int(self.mb.add_verts(self._posk(k))[0])
                self.shared[k] = i
            return i
        return vid

    def build(self, name="", meta=None):
        for s in self.faces.values():
            s.emit()
        v, t = self.mb.arrays()
        meta = dict(meta or {})
        meta["features"] = self.mb.notes
        return Mesh(v, t, name, meta)


# ----------------------------------------------------------------------------
# named parts
# ----------------------------------------------------------------------------
def box_part(W=100.0, D=60.0, H=40.0, cs=10.0, M=1):
    return Block(W, D, H, cs, M).build("box", {"dims": (W, D, H)})


def config1_part(k=160):
    """100x60x40 mm block; top pocket x in [10,50], y in [20,40], floor z=25;
    top blind hole at (75,30), r=4, bottom z=28; +X-face blind hole at
    (y,z)=(30,20), r=4, bottom x=88.  Rims are k-gons."""
    b = Block(100.0, 60.0, 40.0, 10.0, 1)
    top = b.faces["+Z"]
    p = Pocket(depth=15.0)
    rect = (*top.uv(1, 2), *top.uv(5, 4))
    p.make_floor(top, rect, 4, 2, 4, 2)
    top.add(1, 2, 5, 4, p)
    top.add(7, 2, 8, 4, Hole(75.0, 30.0, 4.0, 12.0, k))
    px = b.faces["+X"]  # u = y, v = z
    px.add(2, 1, 4, 3, Hole(30.0, 20.0, 4.0, 12.0, k))
    return b.build("config1", {"pocket": (10, 20, 50, 40, 25), "holes": [(75, 30, 4, 12), (30, 20, 4, 12)]})


def blind_hole_part(r=4.0, depth=12.0, k=160, cell=10.0, size=(40.0, 40.0, 30.0)):
    """Block with one blind hole of radius r and depth d in the top face centre."""
    W, D, H = size
    b = Block(W, D, H, cell, 1)
    top = b.faces["+Z"]
    cu, cv = W / 2, D / 2
    c0, c1 = int((cu - cell) // cell), int((cu + cell) // cell)
    d0, d1 = int((cv - cell) // cell), int((cv + cell) // cell)
    top.add(c0, d0, c1, d1, Hole(cu, cv, r, depth, k))
    return b.build("blind_hole", {"centre": (cu, cv, H), "r": r, "depth": depth, "k": k})


def pocket_part(W=100.0, D=60.0, H=40.0, rect=(30.0, 20.0, 70.0, 40.0), depth=15.0, cs=10.0):
    b = Block(W, D, H, cs, 1)
    top = b.faces["+Z"]
    c0, d0, c1, d1 = [int(round(x / cs)) for x in rect]
    p = Pocket(depth=depth)
    p.make_floor(top, (*top.uv(c0, d0), *top.uv(c1, d1)), c1 - c0, d1 - d0, c1 - c0, d1 - d0)
    top.add(c0, d0, c1, d1, p)
    return b.build("pocket", {"rect": rect, "depth": depth, "top": H})


def tetrahedron():
    v = np.array([[0, 0, 0], [10, 0, 0], [0, 10, 0], [0, 0, 10]], np.float32)
    t = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], np.int32)
    return Mesh(v, t, "tetrahedron")


def _box_tris(base, lo, hi):
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    v = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]], np.float32)
    q = [(0, 3, 2, 1), (4, 5, 6, 7), (0, 1, 5, 4), (2, 3, 7, 6), (1, 2, 6, 5), (0, 4, 7, 3)]
    t = []
    for a, b, c, d in q:
        t += [(a, b, c), (a, c, d)]
    return v, np.array(t, np.int32) + base


def stacked_boxes(gap=1.0):
    v1, t1 = _box_tris(0, (0, 0, 0), (20, 20, 10))
    v2, t2 = _box_tris(8, (5, 5, 10 + gap), (15, 15, 20 + gap))
    return Mesh(np.concatenate([v1, v2]), np.concatenate([t1, t2]), "stacked_boxes")


def l_bracket(L=40.0, W=20.0, T=5.0, H=30.0):
    """L-shaped prism: profile in (x,z) = L-shape, extruded along y by W."""
    prof = np.array([[0, 0], [L, 0], [L, T], [T, T], [T, H], [0, H]], np.float64)
    n = len(prof)
    v = np.concatenate([np.stack([prof[:, 0], np.zeros(n), prof[:, 1]], 1),
                        np.stack([prof[:, 0], np.full(n, W), prof[:, 1]], 1)]).astype(np.float32)
    # profile is CCW in (x,z); seen from -y (the y=0 cap's outside) (x,z) is CW... build
    # caps by ear decomposition of the L: (0,1,2,3),(0,3,4,5)
    cap = [(0, 1, 2), (0, 2, 3), (0, 3, 4), (0, 4, 5)]
    t = []
    for a, b, c in cap:
        t.append((a, b, c))               # y=0 cap: normal -y for CCW-in-(x,z)
        t.append((a + n, c + n, b + n))   # y=W cap
    for i in range(n):
        j = (i + 1) % n
        t += [(i, i + n, j + n), (i, j + n, j)]
    t = np.array(t, np.int32)
    m = Mesh(v, t, "l_bracket")
    if signed_volume(m.verts, m.tris) < 0:
        m.tris = m.tris[:, ::-1].copy()
    return m


def icosphere(subdiv=2, radius=20.0, centre=(30.0, 30.0, 30.0)):
    p = (1 + 5 ** 0.5) / 2
    v = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0), (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
         (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
         (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    v = [np.array(x, np.float64) / np.linalg.norm(x) for x in v]
    for _ in range(subdiv):
        cache = {}
        nf = []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = (v[a] + v[b]) / 2
                v.append(m / np.linalg.norm(m))
                cache[key] = len(v) - 1
            return cache[key]
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    verts = (np.array(v) * radius + np.array(centre)).astype(np.float32)
    return Mesh(verts, np.array(f, np.int32), "icosphere")


def thin_plate(W=200.0, D=200.0, H=5.0):
    return Block(W, D, H, 5.0, 1).build("thin_plate")


# ----------------------------------------------------------------------------
# procedural families
# ----------------------------------------------------------------------------
def _kgon(r, seg, kmin=12, kmax=4096):
    return int(min(kmax, max(kmin, math.ceil(2 * math.pi * r / seg))))


def _layout_pockets(rng, W, D, H, cs, side_depth, n_pockets, n_holes):
    """Random feature plan for the 'pockets' family: rectangular pockets with
    floor fillets (80 % top, 20 % sides), blind holes on the top face, on
    pocket floors and on the sides."""
    plan = []
    gx, gy, gz = int(round(W / cs)), int(round(D / cs)), int(round(H / cs))
    mc = int(math.ceil((side_depth + 3.0) / cs))
    occ = {f: np.zeros(s, bool) for f, s in
           {"+Z": (gx, gy), "+X": (gy, gz), "-X": (gz, gy), "+Y": (gz, gx), "-Y": (gx, gz)}.items()}
    # allowed region per face (cells), top keeps away from the sides
    region = {"+Z": (mc, mc, gx - mc, gy - mc)}
    for f in ("+X", "-X", "+Y", "-Y"):
        nu, nv = occ[f].shape
        # along the horizontal axis keep away from the vertical block edges
        if f in ("+X",):
            region[f] = (mc, 1, nu - mc, nv - 1)
        elif f == "-X":
            region[f] = (1, mc, nu - 1, nv - mc)
        elif f == "+Y":
            region[f] = (1, mc, nu - 1, nv - mc)
        else:
            region[f] = (mc, 1, nu - mc, nv - 1)

    def place(face, wc, hc, tries=200):
        a0, b0, a1, b1 = region[face]
        o = occ[face]
        for _ in range(tries):
            if a1 - a0 - wc < 0 or b1 - b0 - hc < 0:
                return None
            c0 = int(rng.integers(a0, a1 - wc + 1))
            d0 = int(rng.integers(b0, b1 - hc + 1))
            if not o[max(0, c0 - 1):c0 + wc + 1, max(0, d0 - 1):d0 + hc + 1].any():
                o[c0:c0 + wc, d0:d0 + hc] = True
                return c0, d0
        return None

    for _ in range(n_pockets):
        top = rng.random() < 0.8
        face = "+Z" if top else ["+X", "-X", "+Y", "-Y"][int(rng.integers(4))]
        wmm, hmm = rng.uniform(10, 60), rng.uniform(10, 40)
        if rng.random() < 0.5:
            wmm, hmm = hmm, wmm
        wc, hc = max(2, int(round(wmm / cs))), max(2, int(round(hmm / cs)))
        if face != "+Z":
            nu, nv = occ[face].shape
            wc, hc = min(wc, max(2, nu - 2 * mc - 1)), min(hc, max(2, nv - 3))
        depth = rng.uniform(3, 25) if top else rng.uniform(3, min(25.0, side_depth))
        rf = min(rng.uniform(1, 3), depth * 0.5, cs * 0.3)
        at = place(face, wc, hc)
        if at is None:
            continue
        plan.append(("pocket", face, at[0], at[1], wc, hc, depth, rf))
    for _ in range(n_holes):
        u = rng.random()
        face = "+Z" if u < 0.55 else ("floor" if u < 0.8 else ["+X", "-X", "+Y", "-Y"][int(rng.integers(4))])
        r = rng.uniform(1, 8)
        dr = rng.uniform(1, 6)
        plan.append(("hole", face, r, dr))
    return plan


def procedural_part(seed, target_tris=200_000, family="pockets", dims=None, n_features=None):
    """Seeded procedural block part.

    family 'pockets': 20-60 rectangular pockets with floor fillets, blind holes
    (r 1-8 mm, depth/r 1-6) on the top face, pocket floors and sides.
    family 'multiaxis': T-slots, dovetail undercuts and inclined blind bores
    tilted 10-60 degrees at random azimuth, plus a few pockets and holes.
    Tessellation density is bisected so the triangle count lands near
    `target_tris`.
    """
    def build(density):
        return _procedural(seed, density, family, dims, n_features)

    lo, hi = 0.02, 64.0
    m = build(1.0)
    if target_tris is None:
        return m
    # bisection on density (log scale)
    best = m
    for _ in range(22):
        mid = math.sqrt(lo * hi)
        m = build(mid)
        if abs(m.n_tris - target_tris) < abs(best.n_tris - target_tris):
            best = m
        if m.n_tris < target_tris:
            lo = mid
        else:
            hi = mid
        if abs(m.n_tris - target_tris) <= 0.03 * target_tris:
            best = m
            break
    return best


def _procedural(seed, density, family, dims, n_features):
    rng = np.random.default_rng(seed)
    cs = 5.0
    if dims is None:
        W = cs * round(rng.uniform(200, 300) / cs)
        D = cs * round(rng.uniform(120, 200) / cs)
        H = cs * round(rng.uniform(60, 100) / cs)
    else:
        W, D, H = dims
    side_depth = 20.0
    # tessellation from density: circle segment length and lattice subdivision
    seg = 1.0 / density
    M = max(1, int(round(density * cs / 6.0)))
    b = Block(W, D, H, cs, M)
    F = b.faces
    n_p = n_features[0] if n_features else int(rng.integers(20, 61))
    n_h = n_features[1] if n_features else int(rng.integers(20, 61))
    if family == "pockets":
        plan = _layout_pockets(rng, W, D, H, cs, side_depth, n_p, n_h)
    else:
        plan = _layout_pockets(rng, W, D, H, cs, side_depth, max(4, n_p // 4), n_h // 2)
    pockets = []
    fnf = max(2, int(round(density * 2)))
    for item in plan:
        if item[0] != "pocket":
            continue
        _, face, c0, d0, wc, hc, depth, rf = item
        s = F[face]
        p = Pocket(depth=depth, rf=rf, nf=fnf)
        p.make_floor(s, (*s.uv(c0 * M, d0 * M), *s.uv((c0 + wc) * M, (d0 + hc) * M)), wc * M, hc * M, wc, hc)
        s.add(c0, d0, c0 + wc, d0 + hc, p)
        pockets.append((face, p, depth))
    mc = int(math.ceil((side_depth + 3.0) / cs))

    def region(face):
        s = F[face]
        nu, nv = s.nu, s.nv
        if face == "+Z":
            return mc, mc, nu - mc, nv - mc
        if face in ("+X", "-Y"):
            return mc, 1, nu - mc, nv - 1
        return 1, mc, nu - 1, nv - mc

    def try_place(s, wc, hc, reg, tries=60):
        a0, b0, a1, b1 = reg
        for _ in range(tries):
            if a1 - a0 - wc < 0 or b1 - b0 - hc < 0:
                return None
            c0 = int(rng.integers(a0, a1 - wc + 1))
            d0 = int(rng.integers(b0, b1 - hc + 1))
            if s.free(c0, d0, c0 + wc, d0 + hc, gap=1):
                return c0, d0
        return None

    if family == "multiaxis":   # inclined bores first, before holes take the room
        nb = int(rng.integers(16, 29))
        for _ in range(nb):        # inclined bores
            face = "+Z" if rng.random() < 0.75 else ["+X", "-X", "+Y", "-Y"][int(rng.integers(4))]
            s = F[face]
            r = rng.uniform(2, 6)
            tilt = math.radians(rng.uniform(10, 60))
            azim = rng.uniform(0, 2 * math.pi)
            maxd = (H - 8.0) if face == "+Z" else side_depth - 2.0
            length = rng.uniform(2.5 * r, 6 * r)
            bore = Bore(0.0, 0.0, r, length, tilt, azim, _kgon(r, seg))
            while bore.max_depth() > maxd and bore.length > r:
                bore.length *= 0.8
            if bore.max_depth() > maxd:
                continue
            fu0, fv0, fu1, fv1, _ = bore.footprint()
            wmm, hmm = fu1 - fu0 + 2.5, fv1 - fv0 + 2.5
            wc, hc = int(math.ceil(wmm / cs)) + 1, int(math.ceil(hmm / cs)) + 1
            at = try_place(s, wc, hc, region(face), tries=200)
            if at is None:
                continue
            c0, d0 = at
            u0, v0 = s.uv(c0 * M, d0 * M)
            u1, v1 = s.uv((c0 + wc) * M, (d0 + hc) * M)
            # centre the footprint in the macro cell
            bore.cu = (u0 + u1) / 2 - (fu0 + fu1) / 2
            bore.cv = (v0 + v1) / 2 - (fv0 + fv1) / 2
            s.add(c0, d0, c0 + wc, d0 + hc, bore)
    for item in plan:
        if item[0] != "hole":
            continue
        _, face, r, dr = item
        depth = r * dr
        if face == "floor":
            if not pockets:
                continue
            pf, p, pdepth = pockets[int(rng.integers(len(pockets)))]
            s = p.floor
            csu, csv = s.cell_size()
            ncell = int(math.ceil((2 * r + 2.0) / min(csu, csv)))
            if ncell > min(s.nu, s.nv):
                continue
            limit = (H - 8.0 - pdepth) if pf == "+Z" else (side_depth - pdepth)
            depth = min(depth, limit)
            if depth < max(1.0, r * 0.5):
                continue
            at = try_place(s, ncell, ncell, (0, 0, s.nu, s.nv))
            if at is None:
                continue
            c0, d0 = at
            cu, cv = [(x + y) / 2 for x, y in zip(s.uv(c0 * s.M, d0 * s.M), s.uv((c0 + ncell) * s.M, (d0 + ncell) * s.M))]
            p.sub.append((c0, d0, c0 + ncell, d0 + ncell, Hole(cu, cv, r, depth, _kgon(r, seg))))
            s.occ[c0:c0 + ncell, d0:d0 + ncell] = True
            continue
        s = F[face]
        ncell = int(math.ceil((2 * r + 2.0) / cs))
        limit = H - 8.0 if face == "+Z" else side_depth
        depth = min(depth, limit)
        at = try_place(s, ncell, ncell, region(face))
        if at is None:
            continue
        c0, d0 = at
        cu, cv = [(x + y) / 2 for x, y in zip(s.uv(c0 * M, d0 * M), s.uv((c0 + ncell) * M, (d0 + ncell) * M))]
        s.add(c0, d0, c0 + ncell, d0 + ncell, Hole(cu, cv, r, depth, _kgon(r, seg)))

    if family == "multiaxis":
        top = F["+Z"]
        reg = region("+Z")
        nsl = int(rng.integers(4, 9))
        for _ in range(nsl):       # T-slots: long in u or v
            along_u = rng.random() < 0.5
            L = int(rng.integers(6, 14))
            wc, hc = (L, 4) if along_u else (4, L)
            at = try_place(top, wc, hc, reg)
            if at is None:
                continue
            c0, d0 = at
            u0, v0 = top.uv(c0 * M, d0 * M)
            u1, v1 = top.uv((c0 + wc) * M, (d0 + hc) * M)
            nw = rng.uniform(4, 6)
            cw = rng.uniform(nw + 4, 16)
            d1 = rng.uniform(4, 10)
            d2 = d1 + rng.uniform(5, 10)
            if along_u:
                vc = (v0 + v1) / 2
                neck = (u0 + 2, vc - nw / 2, u1 - 2, vc + nw / 2)
                ch = (u0 + 1, vc - cw / 2, u1 - 1, vc + cw / 2)
            else:
                uc = (u0 + u1) / 2
                neck = (uc - nw / 2, v0 + 2, uc + nw / 2, v1 - 2)
                ch = (uc - cw / 2, v0 + 1, uc + cw / 2, v1 - 1)
            top.add(c0, d0, c0 + wc, d0 + hc, TSlot(neck, ch, d1, d2, seg=max(2, int(density * 8))))
        ndv = int(rng.integers(4, 9))
        for _ in range(ndv):       # dovetail undercuts on the top and the sides
            face = "+Z" if rng.random() < 0.5 else ["+X", "-X", "+Y", "-Y"][int(rng.integers(4))]
            s = F[face]
            wc, hc = int(rng.integers(3, 7)), int(rng.integers(3, 6))
            at = try_place(s, wc, hc, region(face))
            if at is None:
                continue
            c0, d0 = at
            u0, v0 = s.uv(c0 * M, d0 * M)
            u1, v1 = s.uv((c0 + wc) * M, (d0 + hc) * M)
            fl = rng.uniform(1.0, 2.0)
            rim = (u0 + fl + 1.0, v0 + fl + 1.0, u1 - fl - 1.0, v1 - fl - 1.0)
            depth = rng.uniform(4, 12) if face == "+Z" else rng.uniform(4, side_depth - 2)
            s.add(c0, d0, c0 + wc, d0 + hc, Dovetail(rim, depth, fl, seg=max(2, int(density * 6))))
    return b.build(f"{family}-{seed}", {"seed": seed, "family": family, "dims": (W, D, H), "density": density})


# ----------------------------------------------------------------------------
# validation (input sanity; not part of the method)
# ----------------------------------------------------------------------------
def signed_volume(v, t):
    v = v.astype(np.float64)
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


def check_watertight(mesh: Mesh):
    """Every directed edge appears exactly once and its reverse exactly once;
    positive enclosed volume; no zero-area triangle.  Returns a dict."""
    t = mesh.tris.astype(np.int64)
    V = int(mesh.verts.shape[0])
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    key = e[:, 0] * V + e[:, 1]
    rkey = e[:, 1] * V + e[:, 0]
    uk, cnt = np.unique(key, return_counts=True)
    dup = int((cnt > 1).sum())
    present = np.isin(rkey, uk)
    v = mesh.verts.astype(np.float64)
    n = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    area2 = np.einsum("ij,ij->i", n, n)
    return {
        "dup_directed_edges": dup,
        "unmatched_edges": int((~present).sum()),
        "volume": signed_volume(mesh.verts, mesh.tris),
        "zero_area": int((area2 == 0).sum()),
        "unused_verts": int(V - len(np.unique(t))),
    }


def is_watertight(mesh: Mesh) -> bool:
    r = check_watertight(mesh)
    return r["dup_directed_edges"] == 0 and r["unmatched_edges"] == 0 and r["volume"] > 0 and r["zero_area"] == 0


# ----------------------------------------------------------------------------
# impeller-like part (multi-axis: curved blades crowding a hub)
# ----------------------------------------------------------------------------
def _closed_shell(mb, v, t):
    """Add a closed shell, flipping its winding if its signed volume is negative."""
    v = np.asarray(v, np.float64)
    t = np.asarray(t, np.int64)
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0
    if vol < 0:
        t = t[:, [0, 2, 1]]
    idx = mb.add_verts(v)
    mb.add_tris(idx[t])


def _ring_grid(n_i, n_j):
    """Quads of an n_i x n_j grid periodic in both directions, as triangles."""
    i, j = np.meshgrid(np.arange(n_i), np.arange(n_j), indexing="ij")
    a = i * n_j + j
    b = ((i + 1) % n_i) * n_j + j
    c = ((i + 1) % n_i) * n_j + (j + 1) % n_j
    d = i * n_j + (j + 1) % n_j
    return np.concatenate([np.stack([a, b, c], -1).reshape(-1, 3), np.stack([a, c, d], -1).reshape(-1, 3)])


def _impeller(density, n_blades=12, R_hub=60.0, r_bore=10.0, H_hub=20.0, r_in=16.0, r_out=58.0,
              h_in=35.0, h_out=12.0, sweep_deg=60.0, thick=2.0):
    mb = MeshBuilder()
    k = max(24, int(round(192 * density)))
    n_r = max(2, int(round(8 * density)))
    n_z = max(2, int(round(4 * density)))
    # hub: an annular solid of revolution; the profile loop runs along the
    # bottom, up the outer side, back along the top and down the bore
    prof = [(r_bore + (R_hub - r_bore) * q / n_r, 0.0) for q in range(n_r)]
    prof += [(R_hub, H_hub * q / n_z) for q in range(n_z)]
    prof += [(R_hub - (R_hub - r_bore) * q / n_r, H_hub) for q in range(n_r)]
    prof += [(r_bore, H_hub - H_hub * q / n_z) for q in range(n_z)]
    phi = 2 * np.pi * np.arange(k) / k
    pr = np.array(prof)
    v = np.stack([pr[:, None, 0] * np.cos(phi)[None], pr[:, None, 0] * np.sin(phi)[None],
                  np.broadcast_to(pr[:, None, 1], (len(pr), k))], -1).reshape(-1, 3)
    _closed_shell(mb, v, _ring_grid(len(pr), k))
    # blades: thin walls on the hub top along a swept spiral, taller near the bore
    n_s = max(4, int(round(64 * density)))
    n_v = max(2, int(round(24 * density)))
    s = np.linspace(0.0, 1.0, n_s + 1)
    beta = np.radians(sweep_deg)
    for bl in range(n_blades):
        th0 = 2 * np.pi * bl / n_blades
        r = r_in + (r_out - r_in) * s
        th = th0 + beta * s ** 1.5
        P = np.stack([r * np.cos(th), r * np.sin(th)], -1)
        dr = r_out - r_in
        dth = 1.5 * beta * np.sqrt(s)
        T = np.stack([dr * np.cos(th) - r * np.sin(th) * dth, dr * np.sin(th) + r * np.cos(th) * dth], -1)
        T /= np.linalg.norm(T, axis=1, keepdims=True)
        N = np.stack([-T[:, 1], T[:, 0]], -1)
        h = h_in + (h_out - h_in) * s
        vk = np.arange(n_v + 1) / n_v
        # cross-section loop: (-,0), (+,v_0..v_n), (-,v_n..v_1)
        side = np.array([-1.0] + [1.0] * (n_v + 1) + [-1.0] * n_v)
        frac = np.concatenate([[0.0], vk, vk[::-1][:-1]])
        L = len(side)
        xy = P[:, None, :] + (0.5 * thick) * side[None, :, None] * N[:, None, :]
        z = H_hub + frac[None, :] * h[:, None]
        vb = np.concatenate([xy, z[..., None]], -1).reshape(-1, 3)
        i, j = np.meshgrid(np.arange(n_s), np.arange(L), indexing="ij")
        a = i * L + j
        b = (i + 1) * L + j
        c = (i + 1) * L + (j + 1) % L
        d = i * L + (j + 1) % L
        tri = [np.stack([a, b, c], -1).reshape(-1, 3), np.stack([a, c, d], -1).reshape(-1, 3)]
        pk = 1 + np.arange(n_v + 1)
        mk = np.array([0] + [2 * n_v + 2 - q for q in range(1, n_v + 1)])
        for base, flip in ((0, False), (n_s * L, True)):
            cap = np.concatenate([np.stack([mk[:-1], pk[:-1], pk[1:]], -1), np.stack([mk[:-1], pk[1:], mk[1:]], -1)])
            tri.append(base + (cap[:, [0, 2, 1]] if flip else cap))
        _closed_shell(mb, vb, np.concatenate(tri))
    v, t = mb.arrays()
    return Mesh(v, t, "impeller", {"blades": n_blades})


def impeller_part(target_tris=124_000, n_blades=12):
    """Impeller-like part: an annular hub with `n_blades` thin curved blades
    (a 60-degree swept spiral, 35 mm tall at the bore side, 12 mm at the rim).
    Closed shells: the hub and each blade (the blades stand on the hub top).
    Tessellation density is bisected so the triangle count lands near
    `target_tris`."""
    lo, hi = 0.05, 16.0
    best = _impeller(1.0, n_blades)
    for _ in range(30):
        mid = math.sqrt(lo * hi)
        m = _impeller(mid, n_blades)
        if abs(m.n_tris - target_tris) < abs(best.n_tris - target_tris):
            best = m
        if m.n_tris < target_tris:
            lo = mid
        else:
            hi = mid
        if abs(m.n_tris - target_tris) <= 0.01 * target_tris:
            break
    return best


# ----------------------------------------------------------------------------
# the workloads (names follow the configurations they stand for)
# ----------------------------------------------------------------------------
def workload_parts(name: str):
    """Return a list of meshes for a named workload."""
    if name == "single_block_1k5":
        return [config1_part()]
    if name == "interactive_200k":
        return [procedural_part(2, 200_000, "pockets")]
    if name == "multiaxis_1m":
        return [procedural_part(3, 1_000_000, "multiaxis")]
    # stand-ins of the shape of the paper's two case studies (Table 3): a
    # housing-like block with a few top and side features (22,512 faces) and
    # an impeller-like part (about 124k faces)
    if name == "paper_housing_22k":
        return [procedural_part(13, 22_530, "pockets", dims=(150.0, 100.0, 50.0), n_features=(5, 10))]
    if name == "paper_impeller_124k":
        return [impeller_part(123_958)]
    if name.startswith("batch64"):
        return batch_parts()
    raise KeyError(name)


def batch_sizes(n=64, lo=2_000, hi=500_000, seed=400):
    rng = np.random.default_rng(seed)
    return [int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))))) for _ in range(n)]


def batch_part(i, n=64, lo=2_000, hi=500_000, seed0=400):
    """Part i of the batch: seed seed0 + i, triangle target log-uniform in
    [lo, hi]; every third part is of the multi-axis family."""
    tt = batch_sizes(n, lo, hi, seed0)[i]
    fam = "pockets" if i % 3 else "multiaxis"
    dims = (100.0, 80.0, 50.0) if tt < 20_000 else None
    return procedural_part(seed0 + i, tt, fam, dims=dims, n_features=(6, 10) if tt < 20_000 else None)


def batch_parts(n=64, lo=2_000, hi=500_000, seed0=400, workers=1):
    """The batch of uneven parts (optionally generated by `workers`
    processes; the parts do not depend on it)."""
    if workers <= 1:
        return [batch_part(i, n, lo, hi, seed0) for i in range(n)]
    import concurrent.futures as cf
    import multiprocessing as mp
    from functools import partial
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        return list(ex.map(partial(batch_part, n=n, lo=lo, hi=hi, seed0=seed0), range(n)))


def surface_area(mesh):
    v = mesh.verts.astype(np.float64)
    t = mesh.tris
    c = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    return 0.5 * float(np.linalg.norm(c, axis=1).sum())


def batch_samples(meshes, smin=1_000, smax=50_000):
    """Samples per part proportional to surface area, the largest part
    getting smax, clamped to [smin, smax]."""
    a = np.array([surface_area(m) for m in meshes])
    return [int(min(smax, max(smin, round(smax * x / a.max())))) for x in a]


def planar_overlap(mesh: Mesh, res=0.25, min_group=1):
    """Largest number of triangles covering one point of an axis-aligned
    plane (sampled on a grid of spacing `res`, offset so that grid points do
    not fall on lattice edges).  A valid surface covers each point at most
    once from each side.  Returns (max_cover, n_points_checked)."""
    v = mesh.verts.astype(np.float64)
    t = mesh.tris
    P = v[t]
    worst, checked = 0, 0
    for ax in range(3):
        same = (P[:, 0, ax] == P[:, 1, ax]) & (P[:, 1, ax] == P[:, 2, ax])
        idx = np.nonzero(same)[0]
        if len(idx) == 0:
            continue
        u, w = [(ax + 1) % 3, (ax + 2) % 3]
        n = np.cross(P[idx, 1] - P[idx, 0], P[idx, 2] - P[idx, 0])[:, ax]
        key = np.stack([P[idx, 0, ax], np.sign(n)], 1)
        groups = {}
        for i, k in zip(idx, map(tuple, key)):
            groups.setdefault(k, []).append(i)
        for k, g in groups.items():
            g = np.array(g)
            if len(g) < min_group:
                continue
            Q = P[g][:, :, [u, w]]
            lo, hi = Q.reshape(-1, 2).min(0), Q.reshape(-1, 2).max(0)
            xs = np.arange(lo[0] + 0.3719 * res, hi[0], res)
            ys = np.arange(lo[1] + 0.6173 * res, hi[1], res)
            cover = np.zeros((len(xs), len(ys)), np.int32)
            for q in Q:
                a, b, c = q
                x0, x1 = np.searchsorted(xs, min(a[0], b[0], c[0])), np.searchsorted(xs, max(a[0], b[0], c[0]))
                y0, y1 = np.searchsorted(ys, min(a[1], b[1], c[1])), np.searchsorted(ys, max(a[1], b[1], c[1]))
                if x1 <= x0 or y1 <= y0:
                    continue
                X, Y = np.meshgrid(xs[x0:x1], ys[y0:y1], indexing="ij")
                def ed(p, q_):
                    return (q_[0] - p[0]) * (Y - p[1]) - (q_[1] - p[1]) * (X - p[0])
                e0, e1, e2 = ed(a, b), ed(b, c), ed(c, a)
                s = np.sign((b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]))
                tol = 1e-9
                inside = (s * e0 > tol) & (s * e1 > tol) & (s * e2 > tol)
                cover[x0:x1, y0:y1] += inside
            worst = max(worst, int(cover.max()))
            checked += cover.size
    return worst, checked

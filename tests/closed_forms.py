"""Closed-form visibility of geometric features of the procedural parts
(test helpers; pure numpy)."""
import numpy as np


def bore_floor_sample(orc, m, f):
    """Sample at the centre of a bore's flat floor: the mesh's own floor
    centre vertex, the floor triangles' normal, origin offset by eps."""
    t0, t1 = f["floor_tris"]
    tri = m.tris[t0]
    v = m.verts[tri].astype(np.float64)
    n = np.cross(v[1] - v[0], v[2] - v[0])
    n /= np.linalg.norm(n)
    c = m.verts[tri[0]]          # fan triangles start at the floor centre vertex
    _, _, eps = orc.mesh_info(m.verts)
    p = c.astype(np.float32)[None]
    nn = n.astype(np.float32)[None]
    o = (p.astype(np.float64) + np.float64(eps) * nn.astype(np.float64)).astype(np.float32)
    return {"point": p, "normal": nn, "origin": o, "tri": np.array([t0], np.int32)}


def bore_closed_form(f, o, dirs_world):
    """From a point inside the convex bore cavity, a ray escapes iff its
    crossing of the face plane lies inside the rim polygon (the cavity is
    the prism over the rim cut by the floor and face planes; outside the
    face there is nothing).  Returns (escapes, keep) with directions whose
    crossing lies within 1e-6 rad of the rim excluded."""
    nf = np.array(f["face_normal"])
    c = nf @ np.array(f["face_point"])
    eu, ev = (np.array(a) for a in f["face_axes"])
    rim = np.array(f["rim"], np.float32).astype(np.float64)
    R = np.stack([rim @ eu, rim @ ev], 1)
    o = np.asarray(o, np.float64)
    d = np.asarray(dirs_world, np.float64)
    den = d @ nf
    t = np.where(den > 0, (c - nf @ o) / np.where(den > 0, den, 1), -1)
    X = o + t[:, None] * d
    x, y = X @ eu, X @ ev
    inside = t > 0
    margin = np.full(len(d), np.inf)
    area = np.sum(R[:, 0] * np.roll(R[:, 1], -1) - np.roll(R[:, 0], -1) * R[:, 1])
    sgn = 1.0 if area > 0 else -1.0
    for i in range(len(R)):
        a, b = R[i], R[(i + 1) % len(R)]
        e = b - a
        cr = sgn * (e[0] * (y - a[1]) - e[1] * (x - a[0])) / np.hypot(*e)
        inside &= cr > 0
        margin = np.minimum(margin, np.abs(cr) / np.maximum(t, 1e-30))
    keep = (margin > 1e-6) | (den <= 0)
    return inside, keep

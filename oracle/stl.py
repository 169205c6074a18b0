"""CPU oracle: STL mesh files.

TEST INFRASTRUCTURE ONLY: used by the tests, never by the library.

A plain reader written from the STL format's definition, with the reading
the library documents: binary when the file size is exactly 84 + 50 x (the
little-endian uint32 at byte 80), otherwise ASCII; ASCII numbers are parsed
to the nearest FP64 value and rounded to FP32; vertices are welded by equal
FP32 coordinates (-0 as +0) in order of first appearance; facet normals are
ignored.  Writers for both forms make the test files.
"""
from __future__ import annotations

import struct

import numpy as np


class StlError(ValueError):
    pass


def _weld(corners):
    """corners: float32 [m*3][3] in facet order -> (verts, tris)."""
    index = {}
    verts = []
    tris = np.empty(len(corners), np.int64)
    for k, c in enumerate(corners):
        c = [float(np.float32(x)) + 0.0 for x in c]    # -0 -> +0
        if not all(np.isfinite(c)):
            raise StlError(f"facet {k // 3}: non-finite coordinate")
        key = tuple(np.float32(x).tobytes() for x in c)
        if key not in index:
            index[key] = len(verts)
            verts.append(c)
        tris[k] = index[key]
    return np.array(verts, np.float32).reshape(-1, 3), tris.reshape(-1, 3).astype(np.int32)


def read(path):
    """(verts float32 [n][3], tris int32 [m][3]) of an STL file; StlError if malformed."""
    data = open(path, "rb").read()
    try:
        return _read(data)
    except StlError:
        raise
    except (ValueError, IndexError) as e:
        raise StlError(f"malformed STL: {e}") from e


def _read(data):
    if len(data) >= 84:
        (count,) = struct.unpack_from("<I", data, 80)
        if len(data) == 84 + 50 * count:
            rec = np.frombuffer(data, dtype=np.dtype([("n", "<f4", 3), ("v", "<f4", (3, 3)), ("a", "<u2")]),
                                count=count, offset=84)
            if count == 0:
                raise StlError("no facets")
            return _weld(rec["v"].reshape(-1, 3))
    words = data.decode("ascii", errors="replace").split()
    if not words or words[0] != "solid":
        raise StlError("neither binary nor ASCII STL")
    # the solid's name runs to the end of the line that holds "solid"
    line_end = data.find(b"\n", data.find(b"solid"))
    words = data[line_end + 1:].decode("ascii", errors="replace").split() if line_end >= 0 else []
    corners, i = [], 0
    while True:
        if i >= len(words):
            raise StlError("missing endsolid")
        w = words[i]
        if w == "endsolid":
            break
        if w != "facet":
            raise StlError(f"expected facet, found {w!r}")
        i += 1
        if words[i] == "normal":
            [float(x) for x in words[i + 1:i + 4]]
            i += 4
        if words[i:i + 2] != ["outer", "loop"]:
            raise StlError("expected outer loop")
        i += 2
        for _ in range(3):
            if words[i] != "vertex":
                raise StlError("expected vertex")
            corners.append([np.float32(float(x)) for x in words[i + 1:i + 4]])
            i += 4
        if words[i:i + 2] != ["endloop", "endfacet"]:
            raise StlError("expected endloop endfacet")
        i += 2
    if not corners:
        raise StlError("no facets")
    return _weld(np.array(corners, np.float32))


def write_binary(path, verts, tris, header=b"hra test mesh"):
    v = np.asarray(verts, np.float32)
    t = np.asarray(tris, np.int64)
    rec = np.zeros(len(t), dtype=np.dtype([("n", "<f4", 3), ("v", "<f4", (3, 3)), ("a", "<u2")]))
    rec["v"] = v[t]
    with open(path, "wb") as f:
        f.write(header[:80].ljust(80, b" "))
        f.write(struct.pack("<I", len(t)))
        f.write(rec.tobytes())


def write_ascii(path, verts, tris, name="part"):
    """ASCII STL with coordinates printed exactly (repr of the FP32 value as FP64 round-trips)."""
    v = np.asarray(verts, np.float32)
    with open(path, "w") as f:
        f.write(f"solid {name}\n")
        for a, b, c in np.asarray(tris, np.int64):
            f.write("  facet normal 0 0 0\n    outer loop\n")
            for k in (a, b, c):
                f.write("      vertex " + " ".join(repr(float(x)) for x in v[k]) + "\n")
            f.write("    endloop\n  endfacet\n")
        f.write(f"endsolid {name}\n")

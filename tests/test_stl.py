"""STL reading: the oracle reader (oracle/stl.py) pinned by a hand-written
cube and by round trips of generated parts, and the library's reader
(hra_stl_read, host code in libhra.so, no GPU) equal to it byte for byte."""
import os

import numpy as np
import pytest

from oracle import stl as S
from synth import parts as P

HERE = os.path.dirname(os.path.abspath(__file__))
CUBE = os.path.join(HERE, "golden", "cube_ascii.stl")


def _lib_read(path):
    from paper_2609_05467_amd import hra
    return hra.read_stl(path)


def _corners(v, t):
    return np.asarray(v, np.float32)[np.asarray(t, np.int64)]


def test_cube_fixture():
    v, t = S.read(CUBE)
    assert v.shape == (8, 3) and t.shape == (12, 3)
    m = P.Mesh(v, t, "cube")
    assert P.is_watertight(m)
    assert abs(P.signed_volume(v, t) - 1.0) < 1e-12
    # first appearance order: (0,0,0), (1,1,0), (1,0,0), ...
    assert np.array_equal(v[:3], [[0, 0, 0], [1, 1, 0], [1, 0, 0]])


@pytest.mark.parametrize("form", ["binary", "ascii"])
@pytest.mark.parametrize("name", ["config1", "impeller-small"])
def test_round_trip(tmp_path, form, name):
    m = P.config1_part() if name == "config1" else P._impeller(0.3)
    f = str(tmp_path / f"m.{form}.stl")
    (S.write_binary if form == "binary" else S.write_ascii)(f, m.verts, m.tris)
    v, t = S.read(f)
    # the same facets, corner for corner, bit for bit
    assert np.array_equal(_corners(v, t).view(np.uint32), _corners(m.verts, m.tris).view(np.uint32))
    # welding: one vertex per distinct coordinate, numbered by first appearance
    assert len(v) == len(np.unique(m.verts, axis=0))
    first = np.unique(t.reshape(-1), return_index=True)[1]
    assert np.all(np.diff(first) > 0)
    lv, lt = _lib_read(f)
    assert np.array_equal(lv.view(np.uint32), v.view(np.uint32)) and np.array_equal(lt, t)


def test_binary_header_starting_with_solid(tmp_path):
    m = P.box_part()
    f = str(tmp_path / "solidheader.stl")
    S.write_binary(f, m.verts, m.tris, header=b"solid but binary")
    v, t = S.read(f)
    assert len(t) == m.n_tris
    lv, lt = _lib_read(f)
    assert np.array_equal(lv, v) and np.array_equal(lt, t)


def test_negative_zero_welds(tmp_path):
    f = str(tmp_path / "z.stl")
    with open(f, "w") as fh:
        fh.write("solid z\nfacet normal 0 0 1\nouter loop\nvertex 0 0 0\nvertex 1 0 0\nvertex 0 1 0\nendloop\n"
                 "endfacet\nfacet\nouter loop\nvertex -0 0 -0.0\nvertex 0 1 0\nvertex -1 0 0\nendloop\nendfacet\n"
                 "endsolid z\n")
    v, t = S.read(f)
    assert len(v) == 4 and t[1, 0] == 0 and not np.any(np.signbit(v) & (v == 0))
    lv, lt = _lib_read(f)
    assert np.array_equal(lv.view(np.uint32), v.view(np.uint32)) and np.array_equal(lt, t)
    # the library matches the cube fixture too
    lv, lt = _lib_read(CUBE)
    cv, ct = S.read(CUBE)
    assert np.array_equal(lv, cv) and np.array_equal(lt, ct)


@pytest.mark.parametrize("case", ["empty", "truncated", "nan", "no_endsolid", "garbage", "missing"])
def test_errors(tmp_path, case):
    from paper_2609_05467_amd import hra
    f = str(tmp_path / f"{case}.stl")
    m = P.tetrahedron()
    if case == "empty":
        open(f, "wb").close()
    elif case == "truncated":
        S.write_binary(f, m.verts, m.tris)
        data = open(f, "rb").read()
        open(f, "wb").write(b"\x00" + data[1:-7])
    elif case == "nan":
        v = m.verts.copy()
        v[1, 2] = np.nan
        S.write_binary(f, v, m.tris)
    elif case == "no_endsolid":
        S.write_ascii(f, m.verts, m.tris)
        txt = open(f).read()
        open(f, "w").write(txt[:txt.rindex("endsolid")])
    elif case == "garbage":
        open(f, "w").write("solid x\nfacet normal 0 0 1\nouter loop\nvertex 0 0 zero\n")
    if case != "missing":
        with pytest.raises(S.StlError):
            S.read(f)
    with pytest.raises(hra.HraError) as e:
        _lib_read(f)
    assert e.value.status == -1 and str(e.value)

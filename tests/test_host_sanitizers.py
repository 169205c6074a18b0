"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the C oracle, the STL reader and the server's scheduling core, each built
with gcc/g++ and the sanitizers, driven by a small program under
tests/sanitize/, and required to exit cleanly with no sanitizer report."""
import os
import struct
import subprocess

import numpy as np
import pytest

from synth import parts as P

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")


def _build(tmp, out, cmd):
    exe = str(tmp / out)
    subprocess.run(cmd + ["-o", exe], check=True, capture_output=True, text=True)
    return exe


def _run(args):
    r = subprocess.run(args, capture_output=True, text=True, env=ENV, timeout=300)
    report = ("ERROR: AddressSanitizer" in r.stderr or "runtime error:" in r.stderr
              or "ERROR: LeakSanitizer" in r.stderr)
    assert r.returncode == 0 and not report, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = _build(tmp_path, "oracle_main", ["gcc", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math"] + SAN +
                 [os.path.join(ROOT, "oracle", "hra_oracle.c"), os.path.join(HERE, "sanitize", "oracle_main.c"), "-lm"])
    m = P.config1_part()
    v, t = tmp_path / "v.f32", tmp_path / "t.i32"
    m.verts.astype(np.float32).tofile(v)
    m.tris.astype(np.int32).tofile(t)
    out = _run([exe, str(v), str(len(m.verts)), str(t), str(m.n_tris)])
    assert "oracle ok" in out


def _binary_stl(path, verts, tris, count=None):
    with open(path, "wb") as f:
        f.write(b"\0" * 80)
        f.write(struct.pack("<I", len(tris) if count is None else count))
        for tri in tris:
            f.write(struct.pack("<3f", 0, 0, 0))
            for k in tri:
                f.write(struct.pack("<3f", *verts[k]))
            f.write(b"\0\0")


def test_stl_reader_under_sanitizers(tmp_path):
    exe = _build(tmp_path, "stl_main", ["g++", "-std=c++17", "-x", "c++"] + SAN +
                 [os.path.join(ROOT, "paper_2609_05467_amd", "csrc", "stl.hip"), "-x", "none",
                  os.path.join(HERE, "sanitize", "stl_main.cpp")])
    m = P.box_part()
    files = {}
    files["ascii"] = os.path.join(HERE, "golden", "cube_ascii.stl")
    files["binary"] = str(tmp_path / "box.stl")
    _binary_stl(files["binary"], m.verts, m.tris)
    files["truncated"] = str(tmp_path / "trunc.stl")
    with open(files["binary"], "rb") as f:
        data = f.read()
    with open(files["truncated"], "wb") as f:
        f.write(data[:len(data) - 17])
    files["huge_count"] = str(tmp_path / "huge.stl")
    _binary_stl(files["huge_count"], m.verts, m.tris[:3], count=0xFFFFFFFF)
    files["empty"] = str(tmp_path / "empty.stl")
    open(files["empty"], "wb").close()
    files["garbage"] = str(tmp_path / "garbage.stl")
    with open(files["garbage"], "wb") as f:
        f.write(bytes(np.random.default_rng(3).integers(0, 256, 5000, dtype=np.uint8)))
    files["nan"] = str(tmp_path / "nan.stl")
    with open(files["nan"], "w") as f:
        f.write("solid x\nfacet normal 0 0 1\nouter loop\nvertex 0 0 0\nvertex 1 0 nan\nvertex 0 1 0\n"
                "endloop\nendfacet\nendsolid x\n")
    files["unterminated"] = str(tmp_path / "unterminated.stl")
    with open(files["unterminated"], "w") as f:
        f.write("solid x\nfacet normal 0 0 1\nouter loop\nvertex 0 0 0\nvertex 1 0 0\n")
    names = list(files)
    out = _run([exe] + [files[n] for n in names]).splitlines()
    got = dict(zip(names, out))
    assert got["ascii"].startswith("ok") and got["binary"] == f"ok {len(m.verts)} {m.n_tris}"
    for n in ("truncated", "huge_count", "empty", "garbage", "nan", "unterminated"):
        assert got[n].startswith("err -1"), (n, got[n])


def test_scheduler_under_sanitizers(tmp_path):
    exe = _build(tmp_path, "sched_main", ["g++", "-std=c++17"] + SAN + [os.path.join(HERE, "sanitize", "sched_main.cpp")])
    assert "sched ok" in _run([exe])

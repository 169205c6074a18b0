"""Whole-bitmask parity at full size: digests of bit rows.

The full-size workloads (4.1e8 rays and more) are cast once by the CPU
oracle's padded hierarchy (oracle.BVHCast, identical to brute force wherever
brute force decides a ray) in `tests/golden/full_size/make_digests.py`, which
stores per workload: the rays the oracle flags as grazing, a digest of every
block of CHUNK rows with those rays cleared, and the oracle's statistics,
class and setups.  A GPU test clears the same rays in its own bits and
compares every block digest, so every non-grazing ray of every row is
compared; a differing block is then re-cast by the oracle to name the rays.

Nothing here computes any part of the method: it hashes, masks and reads
files.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

CHUNK = 512     # rows per digest block
GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size")


def golden_path(name):
    return os.path.join(GOLDEN_DIR, f"{name}.json")


def load(name):
    with open(golden_path(name)) as f:
        return json.load(f)


def array_sha256(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def flagged(gr):
    """(row, direction) of every set bit of uint32 [S][W] rows, row-major."""
    gr = np.ascontiguousarray(gr, np.uint32)
    rows, words = np.nonzero(gr)
    out_r, out_d = [], []
    for r, w in zip(rows.tolist(), words.tolist()):
        v = int(gr[r, w])
        while v:
            b = (v & -v).bit_length() - 1
            out_r.append(r)
            out_d.append(32 * w + b)
            v &= v - 1
    return np.array(out_r, np.int64), np.array(out_d, np.int64)


def cleared(bits, rows, dirs):
    """Copy of uint32 [S][W] bits with the listed (row, direction) bits set to 0."""
    b = np.array(bits, dtype=np.uint32, copy=True)
    if len(rows):
        rows = np.asarray(rows, np.int64)
        dirs = np.asarray(dirs, np.int64)
        np.bitwise_and.at(b, (rows, dirs >> 5), ~(np.uint32(1) << (dirs & 31).astype(np.uint32)))
    return b


def chunk_digests(bits, chunk=CHUNK):
    b = np.ascontiguousarray(bits, np.uint32)
    return [hashlib.blake2b(b[i:i + chunk].tobytes(), digest_size=8).hexdigest() for i in range(0, len(b), chunk)]


def pack_hist(h):
    """uint32 [8192] histogram as base64 text of its zlib-compressed bytes."""
    import base64
    import zlib
    return base64.b64encode(zlib.compress(np.asarray(h, np.uint32).tobytes(), 9)).decode()


def unpack_hist(txt):
    import base64
    import zlib
    return np.frombuffer(zlib.decompress(base64.b64decode(txt)), np.uint32).astype(np.int64)


def compare(bits, rec):
    """Blocks of `bits` (uint32 [S][W], the GPU's) whose digest, with the
    record's grazing rays cleared, differs from the oracle's.  rec: the
    record of one cast ({'grazing_rows', 'grazing_dirs', 'digests', ...})."""
    got = chunk_digests(cleared(bits, rec["grazing_rows"], rec["grazing_dirs"]), rec["chunk"])
    want = rec["digests"]
    if len(got) != len(want):
        raise AssertionError(f"{len(got)} blocks against {len(want)}")
    return [i for i, (g, w) in enumerate(zip(got, want)) if g != w]

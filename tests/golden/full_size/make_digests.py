"""Write the oracle's full-size records (tests/golden/full_size/*.json).

Calls only the CPU oracle (oracle/) and the seeded part generator (synth/):
for every part of the full-size workloads it draws the samples with the
oracle's sampler, casts the hemisphere and the six axes through the
oracle's padded hierarchy (oracle.BVHCast, bit-identical to brute force on
every ray brute force decides), and stores
  - the mesh and sample hashes (the GPU test checks its inputs against them),
  - the rays flagged grazing and a digest of every CHUNK rows with those rays
    cleared (tests/full_size.py),
  - the part statistics, class (Section 3.3) and setups (Section 3.3, last
    paragraph) computed by the oracle from its own bits.

Usage (from the repository root; about 8 minutes on 8 cores):
    python tests/golden/full_size/make_digests.py [workload ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import numpy as np  # noqa: E402

import full_size as FS  # noqa: E402
import oracle_records as OR  # noqa: E402
from oracle import oracle as orc  # noqa: E402
from synth import parts as P  # noqa: E402

TOOL_LENGTH = 50.0
# name: (parts, sample mode, sampling seed(s), samples, directions); the
# single-part entries are the benchmark's workloads as it runs them
WORKLOADS = {
    "interactive_200k": ("interactive_200k", "area", 2, 100_000, 4096),
    "multiaxis_1m": ("multiaxis_1m", "area", 2, 250_000, 2048),
    "batch64": ("batch64", "area", 400, None, 1024),
    "paper_housing_22k": ("paper_housing_22k", "centroid", 0, None, 150),
    "paper_impeller_124k": ("paper_impeller_124k", "centroid", 0, None, 150),
}


def log(*a):
    print(*a, flush=True)


def cast_record(bvh, samples, dirs, kind):
    bits, gr, inf = bvh.cast(samples, dirs, kind=kind)
    rows, dd = FS.flagged(gr)
    info = [int(inf[r, d >> 5] >> (d & 31) & 1) for r, d in zip(rows.tolist(), dd.tolist())]
    rec = {"n_dirs": len(dirs), "chunk": FS.CHUNK, "grazing_rows": rows.tolist(), "grazing_dirs": dd.tolist(),
           "grazing_info": info, "n_grazing": len(rows), "n_free": int(orc.counts(bits, len(dirs)).sum()),
           "digests": FS.chunk_digests(FS.cleared(bits, rows, dd))}
    return rec, bits


def part_record(m, mode, seed, S, N, keep_hist=True):
    t0 = time.perf_counter()
    if mode == "area":
        s = orc.sample_area(m.verts, m.tris, S, seed)
    else:
        s = orc.sample_centroid(m.verts, m.tris)
    S = len(s["origin"])
    rec = {"n_tris": int(m.n_tris), "mesh_sha256": FS.array_sha256(m.verts, m.tris),
           "samples": {"mode": mode, "seed": seed, "n": S,
                       "sha256": FS.array_sha256(s["point"], s["normal"], s["origin"], s["tri"])}}
    bvh = orc.BVHCast(m.verts, m.tris)
    dirs = orc.fibonacci_dirs(N)
    rec["hemi"], bits = cast_record(bvh, s, dirs, 0)
    rec["hemi"]["oracle_work_per_ray"] = (bvh.work / float(S * N)).tolist()
    t1 = time.perf_counter()
    rec["stats"], hist = OR.stats_record(orc, s, dirs, bits, rec["hemi"]["grazing_rows"], hist=keep_hist)
    # the batch results carry no histogram: kept for single parts
    rec["stats"]["hist"] = FS.pack_hist(hist) if keep_hist else None
    rec["axes"], a6 = cast_record(bvh, s, orc.axes6(), 1)
    rec["setups"] = OR.setups_record(orc, m, s, a6, TOOL_LENGTH)
    bvh.close()
    log(f"  {m.n_tris} triangles, {S} samples x {N}: cast {t1 - t0:.1f} s, stats {time.perf_counter() - t1:.1f} s, "
        f"grazing {rec['hemi']['n_grazing']} + {rec['axes']['n_grazing']} (axes)")
    return rec


def make(name):
    parts_name, mode, seed, S, N = WORKLOADS[name]
    log(f"[{name}]")
    if parts_name == "batch64":
        meshes = P.batch_parts(workers=min(8, os.cpu_count() or 1))
        counts = P.batch_samples(meshes)
        recs = [part_record(m, mode, seed + i, c, N, keep_hist=False) for i, (m, c) in enumerate(zip(meshes, counts))]
    else:
        recs = [part_record(P.workload_parts(parts_name)[0], mode, seed, S, N)]
    out = {"workload": name, "generator": "tests/golden/full_size/make_digests.py",
           "oracle": "oracle.BVHCast (padded median-split hierarchy, FP64 decisions), oracle.dirstats, "
                     "oracle.indicators/classify, oracle.reach_classes/min_setups_exact/min_setups_greedy",
           "pad_frac": orc.BVH_PAD_FRAC, "n_dirs": N, "parts": recs}
    with open(FS.golden_path(name), "w") as f:
        json.dump(out, f, separators=(",", ":"))
        f.write("\n")


if __name__ == "__main__":
    names = sys.argv[1:] or list(WORKLOADS)
    for n in names:
        make(n)

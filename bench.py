"""Benchmark: any-hit hemisphere rays/s of the whole accessibility path.

One step = one pass of the hot path over one part whose mesh is already in
HBM: build the BVH, draw the surface samples, cast the hemisphere, the
directional statistics and classification, the six-axis cast and the setup
search.  `value` is hemisphere rays per second over the timed steps.

Default workload: the single part at interactive size (seeded procedural
block with pockets, holes and fillets, ~200k triangles), 100k area-weighted
samples, 4096 Fibonacci-hemisphere directions (4.1e8 rays per step).

Prints one JSON line.  Extra keys: parts/s, per-stage milliseconds, BVH
facts, the traversal work per ray, the roofline of the cast kernel (HIP
events over the timed region), the CPU oracle timed on a bounded sample, and
the canonical machining frame of the part (estimate and reorientation, timed
apart from the step: the workload parts are generated in that frame).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (part builder, samples, directions)
    "interactive_200k": ("interactive_200k", 100_000, 4096),
    "single_block_1k5": ("single_block_1k5", 1_000, 512),
    "multiaxis_1m": ("multiaxis_1m", 250_000, 2048),
    # 64 uneven parts (2k-500k triangles), samples by area in [1k, 50k]
    "batch64": ("batch64", None, 1024),
    # Poisson arrivals of analyses of parts drawn from the batch64 pool
    "serve": ("batch64", None, 1024),
    # the shape of the paper's case studies (Table 3): one ray origin per
    # face (offset centroid), 150 directions, on a housing-like 22.5k-face
    # part and an impeller-like 124k-face part, one after the other
    "paper_shape": (("paper_housing_22k", "paper_impeller_124k"), "centroid", 150),
}
# the paper's own times for its two cases (Table 3; GTX 1650, PyTorch + Warp):
# context for paper_shape, never a target
PAPER_TABLE3 = {"paper_housing_22k": {"faces": 22_530, "seconds": 0.18},
                "paper_impeller_124k": {"faces": 123_958, "seconds": 4.50}}
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
NODE_BYTES, TRI_BYTES = 64, 48  # one interior-node record, one leaf triangle
# FP32 vector operations the cast performs: per node visit two slab tests
# (22 each: 6 differences, 6 products, 9 min/max, the widening product and the
# compare) and the leaf decoding (6); per triangle test 54 (the translated
# vertex and two edges, 9; the largest component, 5; the two bounds, 4; the
# cross products P and Q, 12; U, V, det and Tn, 12; the third edge, 2; the
# compares, 10); per ray 20 (rotation 9, three guarded reciprocals 9, the
# bound factor 2).
NODE_OPS, TRI_OPS, RAY_OPS = 50, 54, 20
# Floating-point operations of the hemisphere cast, counted from its source
# with a fused multiply-add as two and a min, max, compare or reciprocal as
# one (sign flips, absolute values and selects not counted): per node visit
# two slab tests of 25 (six differences, six products, eleven min/max, the
# widening product, the compare) and the near-far compare; per triangle test
# 71 (translated vertex and edges 9, largest component 9, the squared and
# bound products 2, cross products P and Q 18, U, V, det and Tn 20, the
# third edge 2, its bound 1, the plane bound 2, compares 8); per ray 24
# (rotation 15, three guarded reciprocals 6, the bound factor 3).
NODE_FLOPS, TRI_FLOPS, RAY_FLOPS = 51, 71, 24
# MI355X published vector FP32 peak (counts an FMA as two flops and packed
# FP32 as two lanes; this build issues no packed FP32, so 78.6 TFLOP/s is
# the most it can reach with FMAs only, and 39.3 T/s with single operations)
FP32_PEAK_TFLOPS = 157.3
FP32_UNPACKED_FMA_TFLOPS = 78.6
# VALU lane operations per second: 256 CUs x 64 lanes x 2.4 GHz, one
# operation per lane per clock without packed FP32 (the issue limit of the
# instructions this build emits).
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
TRAVERSAL = {"step": 1, "leaf_loop": 2, "refill": 3}     # hra.h HRA_TRAVERSAL_*
# the traversal loop measured faster on each workload's part: the step loop,
# except for the paper-shape parts (150 directions), whose hemisphere cast
# runs faster with refilled lanes (impeller 6.45 -> 5.6 ms per cast)
DEFAULT_TRAVERSAL = {"interactive_200k": "step", "single_block_1k5": "step", "multiaxis_1m": "step",
                     "batch64": "step", "serve": "step", "paper_shape": "refill"}
# (rays per wave, leaf size) measured faster per workload; (64, 4) elsewhere.
# On the 1M-triangle part (samples in spatial order) leaves of up to 16
# triangles cast in 23.1 ms, up to 8 in 24.1, up to 4 in 26.6; 256 rays per
# wave a little faster than 64.  The 64-part batch plan: 61.4 ms with leaves
# of up to 16, 61.7 with 8, 62.7 with 4.  On the interactive part every shape
# from leaves of 2 to 16 and 64 to 256 rays per wave lies within 1 %
# (10.70-10.81 ms).
DEFAULT_SHAPE = {"multiaxis_1m": (256, 16), "batch64": (64, 16)}
# Whether a step's build and sample run on a stream of their own beside the
# previous step's cast: they do on the parts whose cast takes milliseconds
# (interactive part 12.05 -> 11.70 ms per step, 1M-triangle part 27.9 ->
# 26.5 ms); on the 1.8k-triangle part every stage lasts tens of microseconds
# and the cross-stream waits cost more than the overlap returns (0.65 ->
# 0.84 ms), so its steps stay on one stream.
PREP_STREAM = {"single_block_1k5": False}


def roofline(nodes, tests, rays, W, N, cast_ms, traffic, l2_hit, kernel="k_cast_rows"):
    """Roofline of the hemisphere cast kernel against the published FP32
    peak (the kernel is bound by vector-ALU issue: its node and triangle data
    live in L2 and the MALL), with the issue-rate and cache-served byte views
    beside it.  nodes, tests: node visits and triangle tests over `rays`
    (the instrumented build of the same kernel)."""
    flops_per_ray = (nodes * NODE_FLOPS + tests * TRI_FLOPS) / rays + RAY_FLOPS
    ops_per_ray = (nodes * NODE_OPS + tests * TRI_OPS) / rays + RAY_OPS
    bytes_per_ray = (nodes * NODE_BYTES + tests * TRI_BYTES) / rays + W * 4 / N
    t = cast_ms * 1e-3
    achieved = flops_per_ray * rays / t / 1e12
    ops = ops_per_ray * rays / t / 1e12
    gbs = bytes_per_ray * rays / t / 1e9
    return {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS, "traffic": traffic, "kernel": kernel,
            "avg_launch_ms": cast_ms, "flops_per_launch": flops_per_ray * rays, "flops_per_ray": flops_per_ray,
            "frac_of_unpacked_fma_peak": achieved / FP32_UNPACKED_FMA_TFLOPS,
            "issue_view": {"ops_per_ray": ops_per_ray, "achieved_tops": ops, "peak_tops": ALU_PEAK_TOPS,
                           "frac": ops / ALU_PEAK_TOPS,
                           "note": "FP32 operations as issued (no packed FP32, FMA as one) against "
                                   "256 CUs x 64 lanes x 2.4 GHz"},
            "cache_served_bytes_view": {"algorithmic_bytes": bytes_per_ray * rays, "bytes_per_ray": bytes_per_ray,
                                        "achieved_gbs": gbs, "hbm_peak_gbs": HBM_PEAK_GBS,
                                        "ratio_to_hbm_peak": gbs / HBM_PEAK_GBS,
                                        "measured_hbm_traffic_bytes": traffic, "l2_hit_rate": l2_hit,
                                        "note": "node and triangle bytes per ray x rays / time; above the HBM "
                                                "peak because L2 and the MALL serve them"}}


# Tool-aware cast (hra_cast_tool), flops counted from its source as for the
# hemisphere cast: FP32 per node visit 51 (two slab tests against boxes
# grown through shifted origins, 25 each, and the near-far compare), per
# screened triangle 57 (the bounding-sphere screen every candidate takes:
# centroid 8, farthest-vertex radius 18, distance from the axis 28, the
# compare 3; the plane screen some also take is not counted); FP64 per
# distance test 352 (the half-line meeting test 64, the squared point-triangle
# distance 70, three squared edge distances 72 each, without early exits).
TOOL_NODE_FLOPS, TOOL_SCREEN_FLOPS, TOOL_TEST_FLOPS = 51, 57, 352
FP64_PEAK_TFLOPS = 78.6
TOOL_RADIUS_MM = 3.0
CUT_LENGTH_MM, HOLDER_RADIUS_MM = 20.0, 8.0   # a 6 mm ball-end cutter, 20 mm of flute, a 16 mm holder


def tool_extra(ctx, bvh, samples, N, reps=3):
    """Tool-aware cast (ball-end tool of TOOL_RADIUS_MM) over the same samples
    and directions: time by HIP events, work per direction, ALU roofline."""
    import torch
    S = samples["origin"].shape[0]
    bits, cnt = ctx.cast_tool(bvh, samples, N, TOOL_RADIUS_MM)
    free = int(cnt.to(torch.int64).sum())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.cast_tool(bvh, samples, N, TOOL_RADIUS_MM, counts=False, bits=bits)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    wb, nv, nt, ns = ctx.cast_tool_work(bvh, samples, N, TOOL_RADIUS_MM)
    rays = S * N
    # the same ball with a holder: HOLDER_RADIUS_MM from CUT_LENGTH_MM above the tip centre
    _, hc = ctx.cast_tool_holder(bvh, samples, N, TOOL_RADIUS_MM, CUT_LENGTH_MM, HOLDER_RADIUS_MM)
    e0.record()
    ctx.cast_tool_holder(bvh, samples, N, TOOL_RADIUS_MM, CUT_LENGTH_MM, HOLDER_RADIUS_MM, counts=False)
    e1.record()
    torch.cuda.synchronize()
    hms = e0.elapsed_time(e1)
    holder = {"cut_length_mm": CUT_LENGTH_MM, "holder_radius_mm": HOLDER_RADIUS_MM, "ms": hms,
              "dirs_per_s": rays / (hms * 1e-3), "free_fraction": int(hc.to(torch.int64).sum()) / rays}
    f32 = nv * TOOL_NODE_FLOPS + ns * TOOL_SCREEN_FLOPS
    f64 = nt * TOOL_TEST_FLOPS
    t = ms * 1e-3
    return {"radius_mm": TOOL_RADIUS_MM, "ms": ms, "dirs_per_s": rays / t,
            "node_visits_per_dir": nv / rays, "screened_tris_per_dir": ns / rays, "distance_tests_per_dir": nt / rays,
            "instrumented_bits_identical": bool(torch.equal(wb, bits)), "free_fraction": free / rays, "holder": holder,
            "roofline": {"bound": "alu", "achieved": (f32 + f64) / t / 1e12, "unit": "TFLOP/s",
                         "peak": FP32_PEAK_TFLOPS, "fp32_tflops": f32 / t / 1e12, "fp64_tflops": f64 / t / 1e12,
                         "frac": f32 / t / 1e12 / FP32_PEAK_TFLOPS + f64 / t / 1e12 / FP64_PEAK_TFLOPS,
                         "note": "frac = FP32 flops / 157.3 TFLOP/s + FP64 flops / 78.6 TFLOP/s over the launch",
                         "fp32_flops_per_dir": f32 / rays, "fp64_flops_per_dir": f64 / rays}}


# Canonical frame (hra_frame_estimate), algorithmic HBM bytes: per face the
# indices (12), the record and bin written (36), the histogram pass (bin and
# area, 12), two bin-mean passes (bins, 8), four cone passes (records, 128)
# and the aligned-area pass (32); per vertex the vertices read twice (24).
FRAME_FACE_BYTES, FRAME_VERT_BYTES = 228, 24


def frame_extra(ctx, verts, tris, mesh, reps=20, oracle=True):
    """Canonical machining frame of the workload's part: the estimate and the
    reorientation timed with HIP events on the stream they run on, their HBM
    rooflines, and the oracle's time for the same estimate."""
    import numpy as np
    import torch
    fr, _ = ctx.estimate_frame(verts, tris)
    out = torch.empty_like(verts)
    ctx.apply_frame(fr, verts, out=out)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(reps):
        fr, _ = ctx.estimate_frame(verts, tris)
    e[1].record()
    for _ in range(reps):
        ctx.apply_frame(fr, verts, out=out)
    e[2].record()
    torch.cuda.synchronize()
    est_ms = e[0].elapsed_time(e[1]) / reps
    app_ms = e[1].elapsed_time(e[2]) / reps
    g = ctx.read_frame(fr)
    nt, nv = mesh.n_tris, len(mesh.verts)
    eb = FRAME_FACE_BYTES * nt + FRAME_VERT_BYTES * nv
    ab = 24 * nv
    res = {"triangles": nt, "vertices": nv, "estimate_ms": est_ms, "apply_ms": app_ms,
           "axes": np.round(g["axes"], 12).tolist(), "confidence": g["confidence"], "peak_bins": g["peak_bins"],
           "reoriented_identical": bool(torch.equal(out, verts)),
           "roofline_estimate": {"bound": "hbm", "achieved": eb / (est_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": eb / (est_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                 "algorithmic_bytes": eb, "launches": 10},
           "roofline_apply": {"bound": "hbm", "achieved": ab / (app_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": ab / (app_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "algorithmic_bytes": ab}}
    if oracle:
        from oracle import frame as F
        t0 = time.perf_counter()
        o = F.estimate(mesh.verts, mesh.tris)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": nt / dt, "unit": "faces/s", "cores": 1, "kind": "oracle",
                               "sample": f"the whole part ({nt} triangles), numpy FP64", "seconds": round(dt, 3)}
        res["matches_oracle"] = bool(np.allclose(g["axes"], o["axes"], rtol=0, atol=1e-9)
                                     and g["peak_bins"] == o["peak_bins"])
    return res


DATUM_FACE_BYTES = 60   # per triangle: its three float4 vertices, leaf position and weight prefix, read once


def datum_extra(ctx, verts, tris, mesh, reps=20, oracle=True):
    """Datum planes of the part's six setup orientations: the call timed
    (it synchronises, so host wall clock per call, and HIP events around
    the same calls), its HBM roofline, and the oracle's time for the same
    frames, with their equality."""
    import torch
    bvh = ctx.build_bvh(verts, tris)
    got = ctx.datum_frames(bvh)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    t0 = time.perf_counter()
    e[0].record()
    for _ in range(reps):
        got = ctx.datum_frames(bvh)
    e[1].record()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) / reps * 1e3
    dev_ms = e[0].elapsed_time(e[1]) / reps
    bvh.release()
    nt = mesh.n_tris
    b = DATUM_FACE_BYTES * nt
    res = {"triangles": nt, "call_ms": wall_ms, "event_ms": dev_ms,
           "frame_pz": [(r["dir"], r["offset"]) for r in got[4]],
           "roofline": {"bound": "hbm", "achieved": b / (dev_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": b / (dev_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes": b}}
    if oracle:
        from oracle import datum as D
        t0 = time.perf_counter()
        want = D.datum_frames(mesh.verts, mesh.tris)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": nt / dt, "unit": "faces/s", "cores": 1, "kind": "oracle",
                               "sample": f"the whole part ({nt} triangles), numpy FP64", "seconds": round(dt, 3)}
        res["matches_oracle"] = got == want
    return res


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _popcount(a):
    import numpy as np
    return int(np.unpackbits(np.ascontiguousarray(a).view(np.uint8)).sum())


def cpu_baseline(mesh, samples_np, n_dirs, gpu_bits, budget_s=40.0, brute=False):
    """The CPU oracle on the same samples and directions, timed on the host
    cores: its padded-hierarchy cast (bit-identical to brute force wherever
    brute force decides a ray), or brute force itself with brute=True.  All
    rows when the whole run fits budget_s (estimated from a first slice),
    else the leading rows that do.  Every GPU row it covers is compared
    with it: the rays that differ outside the oracle's grazing set (must be
    0) and the grazing share."""
    import numpy as np
    from oracle import oracle as orc
    threads = orc.max_threads()
    dirs = orc.fibonacci_dirs(n_dirs)
    S = len(samples_np["origin"])
    if brute:
        def cast(r0, r1):
            return orc.cast(mesh.verts, mesh.tris, samples_np, dirs, s0=r0, s1=r1, threads=threads)
        t_build = 0.0
    else:
        t0 = time.perf_counter()
        h = orc.BVHCast(mesh.verts, mesh.tris)
        t_build = time.perf_counter() - t0

        def cast(r0, r1):
            return h.cast(samples_np, dirs, s0=r0, s1=r1, threads=threads)
    probe = min(S, max(4 * threads, S // 100))
    t0 = time.perf_counter()
    cast(0, probe)
    tp = time.perf_counter() - t0
    rows = S if tp * S / probe <= budget_s else max(probe, int(probe * budget_s / max(tp, 1e-6)))
    t0 = time.perf_counter()
    bits, gr, _ = cast(0, rows)
    dt = time.perf_counter() - t0
    n_diff = _popcount((np.asarray(gpu_bits[:rows]) ^ bits) & ~gr)
    n_gr = _popcount(gr)
    rays = rows * n_dirs
    kind = "brute force (every ray against every triangle)" if brute else \
        "padded median-split hierarchy (FP64 decisions, bit-identical to brute force where it decides)"
    base = {"value": rays / dt, "unit": "rays/s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{'all ' if rows == S else 'the first '}{rows} of {S} samples x {n_dirs} directions "
                      f"({rays} rays) of the same part ({mesh.n_tris} triangles); {kind}",
            "seconds": round(dt, 3), "hierarchy_build_s": round(t_build, 3)}
    parity = {"rows_compared": rows, "rays_compared": rays, "rays_differing_outside_grazing": n_diff,
              "grazing_rays": n_gr, "grazing_fraction": n_gr / rays if rays else 0.0,
              "status": "equal" if n_diff == 0 else "DIFFERENT", "oracle": "brute force" if brute else "padded hierarchy"}
    return base, parity


def measured_traffic(workload):
    """HBM bytes per launch of the hemisphere cast kernel and its L2 hit rate
    from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when
    the kernel source has changed since those counters were taken (or none
    were taken for this workload)."""
    import hashlib
    f = os.path.join(ROOT, "profiles", f"k_cast_rows_{workload}_traffic.txt")
    if not os.path.exists(f):
        return None, None
    kv = dict(l.strip().split("=", 1) for l in open(f) if "=" in l and not l.startswith("#"))
    h = hashlib.sha256()
    for src in ("paper_2609_05467_amd/csrc/cast.hip", "paper_2609_05467_amd/csrc/common.hpp"):
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest() != kv.get("source_sha256"):
        return None, None
    return float(kv["traffic_bytes"]), float(kv.get("l2_hit_rate", "nan"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps (each step a whole pass; the queue stays full between steps)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="interactive_200k", choices=sorted(WORKLOADS))
    ap.add_argument("--tool-length", type=float, default=50.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rays-per-wave", type=int, default=None, help="default: the workload's measured best")
    ap.add_argument("--stack", type=int, default=None,
                    help="LDS stack entries per lane (default 16: nine workgroups fit in LDS)")
    ap.add_argument("--leaf", type=int, default=None, help="default: the workload's measured best")
    ap.add_argument("--traversal", choices=("step", "leaf_loop", "refill"), default=None,
                    help="traversal loop of the casts (same results; see hra.h); default: the one measured "
                         "faster for the workload's part")
    ap.add_argument("--autotune", action="store_true", help="batch64: sweep the launch shape first")
    ap.add_argument("--rates", default="100,500,1000", help="serve: arrival rates (requests/s)")
    ap.add_argument("--requests", type=int, default=2000, help="serve: requests per rate and mode")
    ap.add_argument("--budget-gib", type=float, default=200.0, help="serve: device memory budget")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="processes generating the batch parts (before any GPU work)")
    ap.add_argument("--no-extras", action="store_true",
                    help="single-part workloads: skip the 64-part batch and serving comparisons")
    ap.add_argument("--no-frame", action="store_true",
                    help="single-part workloads: skip the canonical-frame and datum-plane measurements")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before timing, copy this many MiB device to device (a kernel of known traffic for "
                         "scaling hardware byte counters)")
    args = ap.parse_args()
    if args.traversal is None:
        args.traversal = DEFAULT_TRAVERSAL[args.workload]
    if args.stack is None:
        args.stack = 16
    rpw0, leaf0 = DEFAULT_SHAPE.get(args.workload, (64, 4))
    if args.rays_per_wave is None:
        args.rays_per_wave = rpw0
    if args.leaf is None:
        args.leaf = leaf0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the path would shard by part "
              "and by samples, with no bulk exchange between GPUs)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch64":
        return run_batch(args)
    if args.workload == "paper_shape":
        return run_paper_shape(args)
    if args.workload == "serve":
        return run_serve(args)
    extras = None
    if not args.no_extras and args.workload == "interactive_200k":
        extras = gen_batch(args)   # before any GPU work (the generator forks)
    out = run_single(args, args.workload, cpu_budget_s=40.0, frame=not args.no_frame,
                     brute=args.workload == "single_block_1k5")
    if extras is not None:
        out["workloads"] = {}
        for name in ("single_block_1k5", "multiaxis_1m"):
            log(f"[bench] extra workload {name}")
            w = run_single(workload_args(args, name), name, cpu_budget_s=12.0, frame=False,
                           brute=name == "single_block_1k5")
            out["workloads"][name] = {k: w[k] for k in ("value", "unit", "ms_per_step", "steps", "warmup", "config",
                                                        "parts_per_s", "stage_ms", "side_stream_elapsed_ms",
                                                        "secondary_alone_ms", "cast_rays_per_s", "bvh",
                                                        "work_per_ray", "result", "roofline", "cpu_baseline",
                                                        "parity") if k in w}
        meshes, counts = extras
        log("[bench] 64-part batch against the plain per-part path")
        b = batch_compare(args, meshes, counts, 2)
        out["batch64"] = {k: b[k] for k in ("config", "batched_graph", "batched_eager", "plain", "speedup_vs_plain",
                                            "results_identical", "stage_ms")}
        log("[bench] serving: served against plain at 100, 500 and 1000 requests/s, and an eviction run")
        out["serve"] = serve_extra(args, meshes, counts)
    print(json.dumps(out), flush=True)


def workload_args(args, name):
    """Launch shape of a workload: its measured-best rays per wave, leaf size
    and traversal loop unless given on the command line for the main one."""
    import copy
    a = copy.copy(args)
    a.workload = name
    a.rays_per_wave, a.leaf = DEFAULT_SHAPE.get(name, (64, 4))
    a.traversal = DEFAULT_TRAVERSAL[name]
    a.stack = 16
    return a


def run_single(args, workload, cpu_budget_s=40.0, frame=True, brute=False):
    """One part per step (build, sample, hemisphere cast, statistics and
    class, six-axis cast, setups), timed over args.steps steps with the mesh
    resident; then the work counts, the roofline, and the CPU oracle over the
    same samples with parity of every row it covers."""
    import numpy as np
    import torch
    from paper_2609_05467_amd import hra
    from synth import parts

    part_name, S, N = WORKLOADS[workload]
    log(f"[bench] generating {part_name}")
    mesh = parts.workload_parts(part_name)[0]
    ctx = hra.Context(0)
    ctx.set_cast_config(args.rays_per_wave, args.stack, 0, TRAVERSAL[args.traversal])
    dev = ctx.device
    verts = torch.tensor(mesh.verts, device=dev)
    tris = torch.tensor(mesh.tris, device=dev)
    # outputs reused across steps (allocated outside the timed region)
    W = (N + 31) // 32
    bits = torch.empty((S, W), dtype=torch.int32, device=dev)
    bits6 = torch.empty((S, 1), dtype=torch.int32, device=dev)
    # two sample buffers: the next step samples into one while this step's
    # six-axis cast and setups still read the other.  The sampler also writes
    # a spatial order of the samples, which the hemisphere cast follows
    # (nearby samples at the same time share the hierarchy's nodes in L2; the
    # results do not depend on it)
    sample_bufs = []
    for _ in range(2):
        sb = ctx.alloc_samples(S)
        sb["order"] = torch.empty((S,), dtype=torch.int32, device=dev)
        sample_bufs.append(sb)
    samples = sample_bufs[0]

    ev = {k: [] for k in ("build", "sample", "cast", "stats", "axes", "setups")}

    # the six-axis cast and the setups need only the samples and the
    # hierarchy: they run on a second stream beside the hemisphere cast and
    # its statistics (default priority, as every stream here)
    side = torch.cuda.Stream()

    pending = []   # each timed step's events, read after the timed loop
    cls_stream = torch.cuda.Stream()

    # the build and the sample of a step run on a third stream, beside the
    # previous step's hemisphere cast; a hierarchy is freed on the stream it
    # was built on, after the statistics that last read it (the pool gives a
    # block back to the next allocation on its own stream in that stream's
    # order only)
    prep = torch.cuda.Stream() if PREP_STREAM.get(workload, True) else torch.cuda.current_stream()

    def prepare(i):
        """Step i's hierarchy and samples, enqueued on the prep stream."""
        b = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        with torch.cuda.stream(prep):
            b[0].record()
            bvh = ctx.build_bvh(verts, tris, leaf_size=args.leaf)
            b[1].record()
            smp = sample_bufs[i % 2]
            b[2].record()
            ctx.sample_surface(bvh, S, 2, out=smp)
            b[3].record()
        return bvh, smp, b

    def launch(cur):
        """Enqueue a step's six-axis cast (side stream) and hemisphere cast
        (main stream) on the hierarchy and samples `cur`, after the prep
        stream's build and sample."""
        bvh, smp, b = cur
        main = torch.cuda.current_stream()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        f = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        main.wait_stream(prep)
        side.wait_stream(main)
        f[0].record(side)
        ctx.cast(bvh, smp, 6, kind=hra.DIRS_AXES6, counts=False, bits=bits6, stream=side)
        f[1].record(side)
        e[0].record()
        ctx.cast(bvh, smp, N, counts=False, bits=bits)
        e[1].record()
        return bvh, smp, b, e, f

    def step(record, cur, i, prefetch):
        """Finish analysis step i, whose casts `cur` are enqueued: its
        statistics (main stream) and setups (side stream), then its class.
        With prefetch, step i + 1's build, sample and casts are enqueued
        behind this step's statistics before the host waits for them, so
        the device is not idle while the host finishes this step; every step
        still builds its own hierarchy, draws its own samples and casts
        them."""
        bvh, smp, b, e, f = cur
        main = torch.cuda.current_stream()
        ds = ctx.dominant_axes(smp, N, bits)
        e[2].record()
        # the setups return a host report: the host waits for the side
        # stream here, while the cast and the statistics queued on the main
        # one run, then for the statistics in classify
        su = ctx.min_setups(bvh, smp, bits6, args.tool_length, want_class=False, stream=side)
        f[2].record(side)
        # the class is read on a stream that waits for the statistics only,
        # so the host does not also wait for the work queued behind them
        cls_stream.wait_event(e[2])
        nxt = launch(prepare(i + 1)) if prefetch else None
        rep = ctx.classify(ds, S, N, stream=cls_stream)
        if record:
            pending.append((b, e, f))
        # the last readers of this step's hierarchy are the statistics (the
        # side stream's work ended before the setups returned): it goes back
        # to the pool on the stream it was built on, behind the next step's
        # build and sample there and after the statistics, without a wait
        prep.wait_event(e[2])
        bvh.release(stream=prep)
        return rep, su, nxt

    if args.copy_calibration_mib:
        src = torch.ones(args.copy_calibration_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log(f"[bench] {workload}: {mesh.n_tris} triangles, {S} samples x {N} directions; warmup {args.warmup}")
    for w in range(args.warmup):
        step(False, launch(prepare(w)), w, False)
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    # exactly K builds, K samplings and K steps inside the timed region
    t0 = time.perf_counter()
    cur = launch(prepare(0))
    reports = []
    for k in range(args.steps):
        rep, su, cur = step(True, cur, k, k + 1 < args.steps)
        reports.append((rep, su))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # every step analyses the same part with the same seeded samples, so
    # every step's class and setups must be the same, bit for bit, however
    # the steps overlap on the device
    steps_identical = all(r == reports[0] for r in reports)
    for b, e, f in pending:
        ev["build"].append(b[0].elapsed_time(b[1]))
        ev["sample"].append(b[2].elapsed_time(b[3]))
        ev["cast"].append(e[0].elapsed_time(e[1]))
        ev["stats"].append(e[1].elapsed_time(e[2]))
        ev["axes"].append(f[0].elapsed_time(f[1]))
        ev["setups"].append(f[1].elapsed_time(f[2]))
    ms = dt / args.steps * 1e3
    rays = S * N
    value = rays * args.steps / dt
    gpu_bits = bits.cpu().numpy().view(np.uint32)

    # traversal work per ray (instrumented build of the same kernel, outside the timed region)
    bvh = ctx.build_bvh(verts, tris, leaf_size=args.leaf)
    info = bvh.info()
    ctx.sample_surface(bvh, S, 2, out=samples)
    # the secondary stages alone on the main stream (inside the step they
    # overlap the hemisphere cast, so their stage times there include waiting)
    alone = {}
    for name, fn in (("dominant_axes", lambda: ctx.dominant_axes(samples, N, bits)),
                     ("six_axis_cast", lambda: ctx.cast(bvh, samples, 6, kind=hra.DIRS_AXES6, counts=False,
                                                         bits=bits6)),
                     ("setups", lambda: ctx.min_setups(bvh, samples, bits6, args.tool_length, want_class=False))):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(5):
            fn()
        b.record()
        torch.cuda.synchronize()
        alone[name] = a.elapsed_time(b) / 5
    wbits, nodes, tests = ctx.cast_work(bvh, samples, N)
    same = bool(torch.equal(wbits, bits))
    bytes_per_ray = (nodes * NODE_BYTES + tests * TRI_BYTES) / rays + W * 4 / N
    cast_ms = float(np.mean(ev["cast"]))
    samples_np = {k: v.cpu().numpy() for k, v in samples.items()}
    bvh.release()
    traffic, l2_hit = measured_traffic(workload)

    out = {
        "metric": "any-hit hemisphere rays/s",
        "value": value,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "triangles": mesh.n_tris, "samples": S, "directions": N,
                   "rays_per_step": rays, "leaf_size": args.leaf, "rays_per_wave": args.rays_per_wave,
                   "stack_depth": args.stack, "traversal": args.traversal, "tool_length_mm": args.tool_length},
        "parts_per_s": args.steps / dt,
        # each stage's interval on its stream: cast and statistics on the main
        # stream (the step's critical path); build and sample on the prep
        # stream, where they share the GPU with the previous step's cast ...
        "stage_ms": {k: round(float(np.mean(ev[k])), 3) for k in ("build", "sample", "cast", "stats")},
        # ... and the side stream's intervals, which share the GPU with the cast running beside them
        "side_stream_elapsed_ms": {k: round(float(np.mean(ev[k])), 3) for k in ("axes", "setups")},
        "stage_streams": {"main": ["cast", "stats"],
                          ("prep, beside the previous step's cast" if PREP_STREAM.get(workload, True)
                           else "main, before the cast"): ["build", "sample"],
                          "side, after sample": ["axes", "setups"],
                          "pipelining": "each step's build and sample run on the prep stream beside the "
                                        "previous step's cast (parts whose cast takes milliseconds), and its "
                                        "casts are enqueued behind the previous "
                                        "step's statistics, before the host waits for them (two sample "
                                        "buffers)"},
        # each secondary stage timed alone on an idle GPU, outside the steps
        "secondary_alone_ms": {k: round(v, 4) for k, v in alone.items()},
        "cast_rays_per_s": rays / (cast_ms * 1e-3),
        "bvh": {"depth": info.depth, "nodes": info.n_nodes, "bytes": info.bytes},
        "work_per_ray": {"node_fetches": nodes / rays, "tri_tests": tests / rays, "bytes": bytes_per_ray,
                         "instrumented_bits_identical": same},
        "result": {"access": rep["access"], "multi_axis": rep["multi_axis"], "shares": rep["shares"],
                   "mean_conc": rep["conc"], "min_setups": su["min_count"], "greedy_setups": su["greedy_count"],
                   "all_steps_identical": steps_identical},
        "roofline": roofline(nodes, tests, rays, W, N, cast_ms, traffic, l2_hit),
    }
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle on the same samples ({'brute force' if brute else 'padded hierarchy'})")
        out["cpu_baseline"], out["parity"] = cpu_baseline(mesh, samples_np, N, gpu_bits, cpu_budget_s, brute)
        log(f"[bench]   {out['parity']['rows_compared']} rows: {out['parity']['status']}, grazing "
            f"{out['parity']['grazing_rays']} ({out['parity']['grazing_fraction']:.2e})")
    if frame:
        log("[bench] canonical frame of the part")
        out["frame"] = frame_extra(ctx, verts, tris, mesh, oracle=not args.no_cpu_baseline)
        log("[bench] datum planes of the part")
        out["datum"] = datum_extra(ctx, verts, tris, mesh, oracle=not args.no_cpu_baseline)
    ctx.close()
    return out


def run_paper_shape(args):
    """The paper's workload shape: per part, build, one offset-centroid
    sample per face, 150 hemisphere directions, statistics and class, the
    six-axis casts and the setup search; the two parts one after the other
    make one step.  value = hemisphere rays per second over both."""
    import numpy as np
    import torch
    from paper_2609_05467_amd import hra
    from synth import parts

    names, _, N = WORKLOADS["paper_shape"]
    meshes = [parts.workload_parts(n)[0] for n in names]
    ctx = hra.Context(0)
    ctx.set_cast_config(args.rays_per_wave, args.stack, 0, TRAVERSAL[args.traversal])
    dev = ctx.device
    W = (N + 31) // 32
    per = []
    for m in meshes:
        v = torch.tensor(m.verts, device=dev)
        t = torch.tensor(m.tris, device=dev)
        b = ctx.build_bvh(v, t, leaf_size=args.leaf)
        S = m.n_tris - b.info().n_degenerate
        b.release()
        per.append({"mesh": m, "v": v, "t": t, "S": S, "samples": ctx.alloc_samples(S),
                    "bits": torch.empty((S, W), dtype=torch.int32, device=dev),
                    "bits6": torch.empty((S, 1), dtype=torch.int32, device=dev), "ms": []})

    def one(p, record):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record()
        bvh = ctx.build_bvh(p["v"], p["t"], leaf_size=args.leaf)
        ctx.sample_surface(bvh, p["S"], 0, mode=hra.SAMPLE_CENTROID, out=p["samples"])
        ctx.cast(bvh, p["samples"], N, counts=False, bits=p["bits"])
        ds = ctx.dominant_axes(p["samples"], N, p["bits"])
        rep = ctx.classify(ds, p["S"], N)
        ctx.cast(bvh, p["samples"], 6, kind=hra.DIRS_AXES6, counts=False, bits=p["bits6"])
        su = ctx.min_setups(bvh, p["samples"], p["bits6"], args.tool_length, want_class=False)
        e[1].record()
        if record:
            torch.cuda.synchronize()
            p["ms"].append(e[0].elapsed_time(e[1]))
        bvh.release()
        p["rep"], p["su"] = rep, su

    log(f"[bench] paper_shape: {[p['mesh'].n_tris for p in per]} faces, {N} directions; warmup {args.warmup}")
    for _ in range(args.warmup):
        for p in per:
            one(p, False)
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for p in per:
            one(p, True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rays = sum(p["S"] for p in per) * N
    out = {
        "metric": "any-hit hemisphere rays/s",
        "value": rays * args.steps / dt,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "paper_shape", "parts": list(names), "samples": "offset centroid of every face",
                   "directions": N, "rays_per_step": rays, "leaf_size": args.leaf,
                   "rays_per_wave": args.rays_per_wave, "stack_depth": args.stack, "traversal": args.traversal,
                   "tool_length_mm": args.tool_length},
        "parts": {},
    }
    for n, p in zip(names, per):
        ms = float(np.mean(p["ms"]))
        b = ctx.build_bvh(p["v"], p["t"], leaf_size=args.leaf)
        ctx.sample_surface(b, p["S"], 0, mode=hra.SAMPLE_CENTROID, out=p["samples"])
        log(f"[bench] tool cast on {n}")
        tool = tool_extra(ctx, b, p["samples"], N)
        b.release()
        out["parts"][n] = {
            "faces": p["mesh"].n_tris, "samples": p["S"], "ms": ms, "rays_per_s": p["S"] * N / (ms * 1e-3),
            "result": {"access": p["rep"]["access"], "multi_axis": p["rep"]["multi_axis"],
                       "shares": p["rep"]["shares"], "mean_conc": p["rep"]["conc"],
                       "min_setups": p["su"]["min_count"], "greedy_setups": p["su"]["greedy_count"]},
            "paper_table3_context": dict(PAPER_TABLE3[n], hardware="GeForce GTX 1650 (another machine, another part)"),
            "tool": tool,
        }
    if not args.no_cpu_baseline:
        import numpy as np
        log("[bench] CPU oracle on the housing part's samples")
        p = per[0]
        out["cpu_baseline"], out["parity"] = cpu_baseline(
            p["mesh"], {k: x.cpu().numpy() for k, x in p["samples"].items()}, N,
            p["bits"].cpu().numpy().view(np.uint32), 30.0)
    ctx.close()
    print(json.dumps(out), flush=True)


def gen_batch(args):
    """The 64-part pool and its sample counts (host only; call before any GPU
    work, the generator forks worker processes)."""
    from synth import parts
    log(f"[bench] generating 64 parts with {args.workers} processes")
    t0 = time.perf_counter()
    meshes = parts.batch_parts(workers=args.workers)
    counts = parts.batch_samples(meshes)
    log(f"[bench] generated in {time.perf_counter() - t0:.1f} s: {sum(m.n_tris for m in meshes)} triangles, "
        f"{sum(counts)} samples")
    return meshes, counts


def run_batch(args):
    """64 uneven parts: the plain path (one part after another, each stage
    its own launches, synchronising per part) against the batch plan (one
    hierarchy, one launch per stage for all parts) eager and as a replayed
    HIP graph.  value = hemisphere rays/s of the graph runs."""
    meshes, counts = gen_batch(args)
    out = batch_compare(args, meshes, counts, args.steps, work=True)
    print(json.dumps(out), flush=True)


def batch_compare(args, meshes, counts, steps, work=False):
    import numpy as np
    N = WORKLOADS["batch64"][2]
    import torch
    from paper_2609_05467_amd import hra
    ctx = hra.Context(0)
    dev = ctx.device
    ctx.set_cast_config(args.rays_per_wave, args.stack, args.leaf, TRAVERSAL[args.traversal])
    dm = [(torch.tensor(m.verts, device=dev), torch.tensor(m.tris, device=dev)) for m in meshes]
    reqs = [{"verts": v, "tris": t, "n_samples": c, "seed": 400 + i, "tool_length": args.tool_length}
            for i, ((v, t), c) in enumerate(zip(dm, counts))]
    S = sum(counts)
    rays = S * N
    tune = None
    if args.autotune:
        log("[bench] autotune sweep (27 points)")
        tune = ctx.autotune(reqs, N, reps=1)
        log(f"[bench] best {tune['best']}")
    rpw, stack, leaf, trav, _ = ctx.cast_config()

    # plain: one part after another
    W = (N + 31) // 32
    bufs = [(ctx.alloc_samples(c), torch.empty((c, W), dtype=torch.int32, device=dev),
             torch.empty((c, 1), dtype=torch.int32, device=dev)) for c in counts]

    def plain_pass():
        out = []
        for i, ((v, t), c) in enumerate(zip(dm, counts)):
            smp, bits, b6 = bufs[i]
            b = ctx.build_bvh(v, t, leaf_size=leaf)
            ctx.sample_surface(b, c, 400 + i, out=smp)
            ctx.cast(b, smp, N, counts=False, bits=bits)
            ds = ctx.dominant_axes(smp, N, bits)
            rep = ctx.classify(ds, c, N)
            ctx.cast(b, smp, 6, kind=hra.DIRS_AXES6, counts=False, bits=b6)
            su = ctx.min_setups(b, smp, b6, args.tool_length, want_class=False)
            b.release()
            out.append((rep, su))
        return out

    log("[bench] plain warmup")
    plain_res = plain_pass()
    torch.cuda.synchronize()
    log(f"[bench] plain timing {steps} passes")
    t0 = time.perf_counter()
    for _ in range(steps):
        plain_pass()
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / steps

    pl = ctx.plan(reqs, N)
    log(f"[bench] plan holds {pl.bytes / 2**30:.2f} GiB; eager warmup")
    res = pl.run(graph=False)
    same_plain = all(r["class"] == p[0] and all(r["setups"][k] == p[1][k] for k in
                                                  ("min_count", "min_mask", "n_class", "code_hist"))
                     for r, p in zip(res, plain_res))
    stage = {k: [] for k in ("build", "sample", "cast", "stats", "axes", "setups")}
    t0 = time.perf_counter()
    for _ in range(steps):
        pl.run(graph=False)
        for k, v in pl.stage_ms().items():
            stage[k].append(v)
    eager_s = (time.perf_counter() - t0) / steps
    log("[bench] graph capture + replays")
    res_g = pl.run(graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res_g = pl.run(graph=True)
    torch.cuda.synchronize()
    graph_s = (time.perf_counter() - t0) / steps
    same_graph = res_g == res
    pl.destroy()

    # traversal work per ray (instrumented single-part casts, outside the timed region)
    W = (N + 31) // 32
    nodes = tests = 0
    if work:
        for i, ((v, t), c) in enumerate(zip(dm, counts)):
            smp = bufs[i][0]
            b = ctx.build_bvh(v, t, leaf_size=leaf)
            ctx.sample_surface(b, c, 400 + i, out=smp)
            _, nf, nt = ctx.cast_work(b, smp, N)
            nodes += nf
            tests += nt
            b.release()
    cast_ms = float(np.mean(stage["cast"]))
    out = {
        "metric": "any-hit hemisphere rays/s",
        "value": rays / graph_s,
        "unit": "rays/s",
        "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": graph_s * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch64", "parts": len(meshes), "triangles": int(sum(m.n_tris for m in meshes)),
                   "triangles_min_max": [int(min(m.n_tris for m in meshes)), int(max(m.n_tris for m in meshes))],
                   "samples": S, "samples_min_max": [min(counts), max(counts)], "directions": N,
                   "rays_per_step": rays, "leaf_size": leaf, "rays_per_wave": rpw, "stack_depth": stack,
                   "traversal": {v: k for k, v in TRAVERSAL.items()}[trav], "tool_length_mm": args.tool_length},
        "parts_per_s": len(meshes) / graph_s,
        "batched_graph": {"ms": graph_s * 1e3, "parts_per_s": len(meshes) / graph_s, "rays_per_s": rays / graph_s},
        "batched_eager": {"ms": eager_s * 1e3, "parts_per_s": len(meshes) / eager_s, "rays_per_s": rays / eager_s},
        "plain": {"ms": plain_s * 1e3, "parts_per_s": len(meshes) / plain_s, "rays_per_s": rays / plain_s},
        "speedup_vs_plain": plain_s / graph_s,
        "results_identical": {"batch_vs_plain": bool(same_plain), "graph_vs_eager": bool(same_graph)},
        "stage_ms": {k: round(float(np.mean(v)), 3) for k, v in stage.items()},
    }
    if work:
        out["work_per_ray"] = {"node_fetches": nodes / rays, "tri_tests": tests / rays}
        out["roofline"] = roofline(nodes, tests, rays, W, N, cast_ms, *measured_traffic("batch64"))
    if tune is not None:
        out["autotune"] = tune
    ctx.close()
    return out


def serve_run(hra, pool, counts, schedule, N, mode, budget, tool):
    """Submit `schedule` [(t_arrival_s, part index, seed)] at its arrival
    times; returns per-request records and the server statistics."""
    sv = hra.Server(0, n_dirs=N, mode=mode, budget_bytes=budget)
    tickets = []
    t0 = time.perf_counter()
    for (ta, k, seed) in schedule:
        dt = t0 + ta - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        v, t = pool[k]
        tickets.append(sv.submit(k, v, t, counts[k], seed, tool))
    recs = [sv.wait(tk, 600_000) for tk in tickets]
    st = sv.stats()
    sv.close()
    return recs, st


def serve_summary(recs, N, counts, schedule):
    import numpy as np
    ok = [r for r in recs if r and r["status"] == 0]
    lat = np.array([(r["t_done_ns"] - r["t_submit_ns"]) * 1e-6 for r in ok])
    t_first = min(r["t_submit_ns"] for r in ok)
    t_last = max(r["t_done_ns"] for r in ok)
    span = (t_last - t_first) * 1e-9
    rays = sum(counts[k] for (_, k, _) in schedule) * N
    return {"requests": len(recs), "ok": len(ok), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
            "parts_per_s": len(ok) / span, "rays_per_s": rays / span, "span_s": span,
            "resident_hit_frac": float(np.mean([r["resident_hit"] for r in ok])),
            "mean_batch": float(np.mean([r["batch_size"] for r in ok]))}


def run_serve(args):
    """Poisson arrivals of part analyses (Zipf(1.1) popularity over the
    64-part pool, samples by area) served with continuous batching and
    resident hierarchies, against the plain mode (one request at a time,
    rebuilt every time), on the same arrival schedule per rate."""
    meshes, counts = gen_batch(args)
    rates = [float(x) for x in args.rates.split(",")]
    out_rates = serve_compare(args, meshes, counts, rates, args.requests)
    top = out_rates[-1]
    out = {
        "metric": "p99 per-part latency, served",
        "value": top["served"]["p99_ms"], "unit": "ms", "n_gpus": 1, "steps": args.requests, "warmup": 0,
        "ms_per_step": top["served"]["mean_ms"], "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serve", "pool_parts": len(meshes), "directions": WORKLOADS["serve"][2],
                   "popularity": "zipf 1.1", "rates_per_s": rates, "requests_per_rate": args.requests,
                   "budget_gib": args.budget_gib, "samples_min_max": [min(counts), max(counts)]},
        "rates": out_rates,
    }
    print(json.dumps(out), flush=True)


SERVE_RATES = (100.0, 500.0, 1000.0)   # requests/s; plain mode keeps up with about 270 parts/s
SERVE_REQUESTS = 2000
EVICT_BUDGET_GIB = 0.25   # below the pool's ~0.7 GB of hierarchies, above its largest request


def serve_extra(args, meshes, counts):
    """Served against plain at three arrival rates, the upper two past plain
    mode's capacity, 2000 requests each; then the served mode under a small
    budget (256 MiB, below the ~0.7 GB the pool's hierarchies take), which
    forces hierarchies out of residency (LRU)."""
    import numpy as np
    rates = serve_compare(args, meshes, counts, list(SERVE_RATES), SERVE_REQUESTS)
    from paper_2609_05467_amd import hra
    N = WORKLOADS["serve"][2]
    import torch
    pool = [(torch.from_numpy(m.verts).pin_memory(), torch.from_numpy(m.tris).pin_memory()) for m in meshes]
    rng = np.random.default_rng(55)
    zipf = 1.0 / np.arange(1, len(meshes) + 1) ** 1.1
    zipf /= zipf.sum()
    order = rng.permutation(len(meshes))
    lam = 500.0
    gaps = rng.exponential(1.0 / lam, SERVE_REQUESTS)
    ta = np.cumsum(gaps) - gaps[0]
    ks = order[rng.choice(len(meshes), SERVE_REQUESTS, p=zipf)]
    schedule = [(float(t), int(k), 9000 + i) for i, (t, k) in enumerate(zip(ta, ks))]
    log(f"[bench] eviction run: {lam}/s, {SERVE_REQUESTS} requests, {EVICT_BUDGET_GIB} GiB budget")
    recs, st = serve_run(hra, pool, counts, schedule, N, hra.SERVE_CONTINUOUS, int(EVICT_BUDGET_GIB * 2 ** 30),
                         args.tool_length)
    ev = serve_summary(recs, N, counts, schedule)
    ev.update({"rate": lam, "budget_gib": EVICT_BUDGET_GIB, "builds": st["builds"], "evictions": st["evictions"],
               "peak_used_bytes": st["peak_used_bytes"]})
    log(f"[bench]   p50 {ev['p50_ms']:.2f} ms p99 {ev['p99_ms']:.2f} ms {ev['parts_per_s']:.1f} parts/s, "
        f"{st['evictions']} evictions")
    return {"popularity": "zipf 1.1 over the 64-part pool", "requests_per_rate": SERVE_REQUESTS,
            "budget_gib": args.budget_gib, "rates": rates, "eviction_run": ev}


def serve_compare(args, meshes, counts, rates, n_requests):
    import numpy as np
    import torch
    from paper_2609_05467_amd import hra
    N = WORKLOADS["serve"][2]
    # meshes in pinned host memory, as a client would hand them over
    pool = [(torch.from_numpy(m.verts).pin_memory(), torch.from_numpy(m.tris).pin_memory()) for m in meshes]
    rng = np.random.default_rng(5)
    zipf = 1.0 / np.arange(1, len(meshes) + 1) ** 1.1
    zipf /= zipf.sum()
    order = rng.permutation(len(meshes))          # popularity rank -> part
    budget = int(args.budget_gib * 2 ** 30)
    out_rates = []
    for lam in rates:
        gaps = rng.exponential(1.0 / lam, n_requests)
        ta = np.cumsum(gaps) - gaps[0]
        ks = order[rng.choice(len(meshes), n_requests, p=zipf)]
        schedule = [(float(t), int(k), 9000 + i) for i, (t, k) in enumerate(zip(ta, ks))]
        row = {"rate": lam}
        for name, mode in (("served", hra.SERVE_CONTINUOUS), ("plain", hra.SERVE_PLAIN)):
            log(f"[bench] rate {lam}/s, {n_requests} requests, {name}")
            recs, st = serve_run(hra, pool, counts, schedule, N, mode, budget, args.tool_length)
            row[name] = serve_summary(recs, N, counts, schedule)
            row[name]["builds"] = st["builds"]
            row[name]["evictions"] = st["evictions"]
            log(f"[bench]   p50 {row[name]['p50_ms']:.2f} ms p99 {row[name]['p99_ms']:.2f} ms "
                f"{row[name]['parts_per_s']:.1f} parts/s")
        out_rates.append(row)
    return out_rates


if __name__ == "__main__":
    main()

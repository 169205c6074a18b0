"""Python binding of libhra.so (ctypes).

Argument marshalling only: torch tensors provide device memory and the HIP
stream; every step runs in the library's HIP kernels.  The library must be
built (`python -m paper_2609_05467_amd.build`); importing this module fails
loudly if it is missing or if no GPU is present when a context is made.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhra.so")

HRA_OK = 0
STATUS = {0: "OK", -1: "INVALID_ARG", -2: "OUT_OF_MEMORY", -3: "DEVICE", -4: "BAD_MESH", -5: "OVER_BUDGET",
          -6: "NOT_READY"}
SAMPLE_AREA, SAMPLE_CENTROID = 0, 1
SERVE_CONTINUOUS, SERVE_PLAIN = 0, 1
DIRS_HEMI, DIRS_AXES6 = 0, 1
TRAVERSAL_STEP, TRAVERSAL_LEAF_LOOP, TRAVERSAL_REFILL = 1, 2, 3
CLASS_VIABLE, CLASS_OVER, CLASS_INACCESSIBLE, CLASS_FIXTURE = 0, 1, 2, 3


class HraError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hra error {STATUS.get(status, status)}: {msg}")
        self.status = status


class BvhOpts(C.Structure):
    _fields_ = [("leaf_size", C.c_int32)]


class BvhInfo(C.Structure):
    _fields_ = [("bbox", C.c_float * 6), ("diag", C.c_double), ("n_tris", C.c_int64), ("n_degenerate", C.c_int64),
                ("n_nodes", C.c_int64), ("bytes", C.c_int64), ("depth", C.c_int32), ("leaf_size", C.c_int32)]


class Samples(C.Structure):
    _fields_ = [("point", C.c_void_p), ("normal", C.c_void_p), ("origin", C.c_void_p), ("tri", C.c_void_p),
                ("n", C.c_int64), ("order", C.c_void_p)]


class Dirs(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32)]


class CastConfig(C.Structure):
    _fields_ = [("rays_per_wave", C.c_int32), ("stack_depth", C.c_int32), ("leaf_size", C.c_int32),
                ("traversal", C.c_int32), ("samples_per_group", C.c_int32)]


class DirStats(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("absmean", C.c_void_p), ("axis", C.c_void_p), ("conc", C.c_void_p),
                ("hist", C.c_void_p), ("totals", C.c_void_p)]


class Thresholds(C.Structure):
    _fields_ = [("min_access", C.c_double), ("min_share", C.c_double), ("max_conc", C.c_double)]


class ClassReport(C.Structure):
    _fields_ = [("access", C.c_double), ("share", C.c_double * 3), ("mean_conc", C.c_double),
                ("n_samples", C.c_int64), ("n_blind", C.c_int64), ("n_unobstructed", C.c_uint64),
                ("multi_axis", C.c_int32), ("tripped", C.c_int32), ("near_tie", C.c_int32)]


class HistPeaks(C.Structure):
    _fields_ = [("n_peaks", C.c_int32), ("bin", C.c_int32 * 16), ("mass", C.c_uint32 * 16),
                ("dir", (C.c_float * 3) * 16), ("axis_mass", C.c_uint64 * 6)]


class SetupReport(C.Structure):
    _fields_ = [("min_count", C.c_int32), ("min_mask", C.c_int32), ("greedy_count", C.c_int32),
                ("greedy_mask", C.c_int32), ("n_class", C.c_int64 * 4), ("code_hist", C.c_uint32 * 64)]


class Mesh(C.Structure):
    _fields_ = [("d_verts", C.c_void_p), ("n_verts", C.c_int64), ("d_tris", C.c_void_p), ("n_tris", C.c_int64)]


class Frame(C.Structure):
    _fields_ = [("axes", (C.c_double * 3) * 3), ("confidence", C.c_double), ("aligned", C.c_double * 3),
                ("extent", C.c_double * 3), ("total_area", C.c_double), ("peak_bin", C.c_int32 * 2),
                ("shift", C.c_int32), ("error", C.c_uint32)]


class DatumFrame(C.Structure):
    _fields_ = [("dir", C.c_int32 * 3), ("n_tris", C.c_int32 * 3), ("offset", C.c_double * 3),
                ("area", C.c_double * 3), ("area_w", C.c_uint64 * 3)]


class PartRequest(C.Structure):
    _fields_ = [("mesh", Mesh), ("n_samples", C.c_int64), ("seed", C.c_uint64), ("tool_length", C.c_double)]


class BatchOpts(C.Structure):
    _fields_ = [("n_dirs", C.c_int32), ("leaf_size", C.c_int32), ("rays_per_wave", C.c_int32),
                ("stack_depth", C.c_int32), ("traversal", C.c_int32), ("offset_frac", C.c_float),
                ("thresholds", C.POINTER(Thresholds))]


class TunePoint(C.Structure):
    _fields_ = [("rays_per_wave", C.c_int32), ("stack_depth", C.c_int32), ("leaf_size", C.c_int32),
                ("traversal", C.c_int32), ("ms", C.c_float)]


class TuneReport(C.Structure):
    _fields_ = [("n_points", C.c_int32), ("best", C.c_int32), ("points", TunePoint * 27)]


class PartResult(C.Structure):
    _fields_ = [("cls", ClassReport), ("setups", SetupReport)]


class ServerOpts(C.Structure):
    _fields_ = [("budget_bytes", C.c_int64), ("mode", C.c_int32), ("max_batch", C.c_int32),
                ("max_inflight", C.c_int32), ("keep_resident", C.c_int32), ("n_dirs", C.c_int32),
                ("leaf_size", C.c_int32), ("offset_frac", C.c_float), ("thresholds", C.POINTER(Thresholds))]


class Request(C.Structure):
    _fields_ = [("part_key", C.c_uint64), ("h_verts", C.c_void_p), ("n_verts", C.c_int64), ("h_tris", C.c_void_p),
                ("n_tris", C.c_int64), ("n_samples", C.c_int64), ("seed", C.c_uint64), ("tool_length", C.c_double)]


class RequestResult(C.Structure):
    _fields_ = [("status", C.c_int), ("resident_hit", C.c_int32), ("batch_size", C.c_int32), ("pad", C.c_int32),
                ("batch_id", C.c_int64), ("t_submit_ns", C.c_int64), ("t_admit_ns", C.c_int64),
                ("t_launch_ns", C.c_int64), ("t_done_ns", C.c_int64), ("result", PartResult)]


class ServerStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("submitted", "completed", "failed", "batches", "builds", "evictions",
                                         "resident_hits", "resident_bytes", "used_bytes", "peak_used_bytes")] + \
               [(n, C.c_int32) for n in ("resident_parts", "pending", "inflight", "pad")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2609_05467_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, i32, i64, u64, f32, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_float, C.c_double
        sig = {
            "hra_ctx_create": ([i32, C.POINTER(P)], C.c_int),
            "hra_ctx_destroy": ([P], None),
            "hra_last_error": ([P], C.c_char_p),
            "hra_version": ([], C.c_char_p),
            "hra_build_bvh": ([P, P, i64, P, i64, C.POINTER(BvhOpts), P, C.POINTER(P)], C.c_int),
            "hra_bvh_get_info": ([P, P, C.POINTER(BvhInfo)], C.c_int),
            "hra_bvh_release": ([P], None),
            "hra_bvh_release_async": ([P, P], C.c_int),
            "hra_bvh_export": ([P, P, P, P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
            "hra_sample_surface": ([P, P, i32, u64, f32, C.POINTER(Samples), P], C.c_int),
            "hra_dirs_table": ([P, Dirs, P], C.c_int),
            "hra_cast_hemisphere": ([P, P, C.POINTER(Samples), Dirs, P, P, P], C.c_int),
            "hra_set_cast_config": ([P, C.POINTER(CastConfig)], C.c_int),
            "hra_cast_work": ([P, P, C.POINTER(Samples), Dirs, P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), P],
                              C.c_int),
            "hra_get_cast_config": ([P, C.POINTER(CastConfig)], C.c_int),
            "hra_debug_rays": ([P, C.POINTER(Samples), Dirs, P, i64, P, P], C.c_int),
            "hra_dirstats_bytes": ([i64], i64),
            "hra_debug_azimuth_table": ([P, i32], i32),
            "hra_dominant_axes": ([P, C.POINTER(Samples), Dirs, P, C.POINTER(DirStats), P], C.c_int),
            "hra_dominant_axes_noalloc": ([P, C.POINTER(Samples), Dirs, P, C.POINTER(DirStats), P], C.c_int),
            "hra_classify": ([P, C.POINTER(DirStats), i64, i32, C.POINTER(Thresholds), C.POINTER(ClassReport), P],
                             C.c_int),
            "hra_min_setups": ([P, P, C.POINTER(Samples), P, f64, P, C.POINTER(SetupReport), P], C.c_int),
            "hra_histogram_peaks": ([P, i32, C.POINTER(HistPeaks)], C.c_int),
            "hra_build_bvh_batch": ([P, C.POINTER(Mesh), i32, C.POINTER(BvhOpts), P, C.POINTER(P)], C.c_int),
            "hra_bvh_parts": ([P], i32),
            "hra_bvh_part_info": ([P, i32, P, C.POINTER(BvhInfo)], C.c_int),
            "hra_sample_part": ([P, P, i32, i32, u64, f32, C.POINTER(Samples), P], C.c_int),
            "hra_cast_part": ([P, P, i32, C.POINTER(Samples), Dirs, P, P, P], C.c_int),
            "hra_min_setups_part": ([P, P, i32, C.POINTER(Samples), P, f64, P, C.POINTER(SetupReport), P],
                                    C.c_int),
            "hra_batch_run": ([P, C.POINTER(PartRequest), i32, C.POINTER(BatchOpts), C.POINTER(PartResult), P, P],
                              C.c_int),
            "hra_plan_create": ([P, C.POINTER(PartRequest), i32, C.POINTER(BatchOpts), C.POINTER(P)], C.c_int),
            "hra_plan_run": ([P, i32, C.POINTER(PartResult), P, P], C.c_int),
            "hra_plan_stage_ms": ([P, C.POINTER(C.c_float)], C.c_int),
            "hra_plan_bytes": ([P], i64),
            "hra_plan_bits": ([P], P),
            "hra_plan_destroy": ([P], None),
            "hra_autotune": ([P, C.POINTER(PartRequest), i32, C.POINTER(BatchOpts), i32, C.POINTER(TuneReport), P],
                             C.c_int),
            "hra_now_ns": ([], i64),
            "hra_server_create": ([i32, C.POINTER(ServerOpts), C.POINTER(P)], C.c_int),
            "hra_server_submit": ([P, C.POINTER(Request), C.POINTER(u64)], C.c_int),
            "hra_server_poll": ([P, u64, C.POINTER(RequestResult)], C.c_int),
            "hra_server_wait": ([P, u64, i64, C.POINTER(RequestResult)], C.c_int),
            "hra_server_drain": ([P, i64], C.c_int),
            "hra_server_get_stats": ([P, C.POINTER(ServerStats)], C.c_int),
            "hra_server_destroy": ([P], None),
            "hra_frame_estimate": ([P, C.POINTER(Mesh), P, P, P], C.c_int),
            "hra_frame_ws_bytes": ([i64], i64),
            "hra_frame_apply": ([P, P, P, P, i64, P], C.c_int),
            "hra_datum_frames": ([P, P, i32, C.POINTER(DatumFrame), P], C.c_int),
            "hra_stl_read": ([C.c_char_p, C.POINTER(P), C.POINTER(i64), C.POINTER(i64)], C.c_int),
            "hra_stl_copy": ([P, P, P], C.c_int),
            "hra_stl_free": ([P], None),
            "hra_stl_error": ([], C.c_char_p),
            "hra_cast_tool": ([P, P, i32, C.POINTER(Samples), Dirs, f64, P, P, P], C.c_int),
            "hra_cast_tool_holder": ([P, P, i32, C.POINTER(Samples), Dirs, f64, f64, f64, P, P, P], C.c_int),
            "hra_cast_tool_work": ([P, P, i32, C.POINTER(Samples), Dirs, f64, P, C.POINTER(u64), C.POINTER(u64),
                                    C.POINTER(u64), P], C.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


EXPORTS = ["hra_ctx_create", "hra_ctx_destroy", "hra_last_error", "hra_version", "hra_build_bvh",
           "hra_bvh_get_info", "hra_bvh_release", "hra_bvh_export", "hra_sample_surface", "hra_dirs_table", "hra_cast_hemisphere",
           "hra_set_cast_config", "hra_get_cast_config", "hra_cast_work", "hra_debug_rays", "hra_dirstats_bytes",
           "hra_dominant_axes", "hra_classify", "hra_min_setups", "hra_histogram_peaks", "hra_build_bvh_batch",
           "hra_bvh_parts", "hra_bvh_part_info", "hra_sample_part", "hra_cast_part", "hra_min_setups_part",
           "hra_batch_run", "hra_plan_create", "hra_plan_run", "hra_plan_stage_ms", "hra_plan_bytes", "hra_plan_bits",
           "hra_plan_destroy", "hra_autotune", "hra_now_ns", "hra_server_create", "hra_server_submit",
           "hra_server_poll", "hra_server_wait", "hra_server_drain", "hra_server_get_stats", "hra_server_destroy",
           "hra_frame_estimate", "hra_frame_ws_bytes", "hra_frame_apply", "hra_stl_read", "hra_stl_copy",
           "hra_stl_free", "hra_stl_error", "hra_cast_tool", "hra_cast_tool_work",
           "hra_cast_tool_holder", "hra_dominant_axes_noalloc", "hra_debug_azimuth_table",
           "hra_datum_frames", "hra_bvh_release_async"]
FRAME_BAD_INDEX, FRAME_EMPTY = 1, 2


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_tensor(x, dtype, device):
    t = torch.as_tensor(x)
    return t.to(device=device, dtype=dtype).contiguous()


class Context:
    """A library context on one GPU (one per host thread)."""

    def __init__(self, device=0):
        if not torch.cuda.is_available():
            raise RuntimeError("hra needs a ROCm GPU; none is visible")
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        p = C.c_void_p()
        st = lib().hra_ctx_create(device, C.byref(p))
        if st != HRA_OK:
            raise HraError(st, f"context creation on device {device} failed")
        self.ptr = p

    def _check(self, st):
        if st != HRA_OK:
            msg = lib().hra_last_error(self.ptr)
            raise HraError(st, (msg or b"").decode())

    def close(self):
        if getattr(self, "ptr", None):
            lib().hra_ctx_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- mesh
    def build_bvh(self, verts, tris, leaf_size=0, stream=None):
        v = _dev_tensor(verts, torch.float32, self.device)
        t = _dev_tensor(tris, torch.int32, self.device)
        out = C.c_void_p()
        opts = BvhOpts(leaf_size)
        self._check(lib().hra_build_bvh(self.ptr, _ptr(v), v.shape[0], _ptr(t), t.shape[0], C.byref(opts),
                                        _stream(stream), C.byref(out)))
        return Bvh(self, out, (v, t), stream)

    def build_bvh_batch(self, meshes, leaf_size=0, stream=None):
        """One hierarchy over several parts; `meshes` is a list of (verts, tris)."""
        keep, arr = [], (Mesh * len(meshes))()
        for i, (verts, tris) in enumerate(meshes):
            v = _dev_tensor(verts, torch.float32, self.device)
            t = _dev_tensor(tris, torch.int32, self.device)
            keep += [v, t]
            arr[i] = Mesh(_ptr(v), v.shape[0], _ptr(t), t.shape[0])
        out = C.c_void_p()
        self._check(lib().hra_build_bvh_batch(self.ptr, arr, len(meshes), C.byref(BvhOpts(leaf_size)),
                                              _stream(stream), C.byref(out)))
        return Bvh(self, out, keep, stream)

    def _requests(self, parts):
        n = len(parts)
        reqs = (PartRequest * n)()
        keep = []
        for i, q in enumerate(parts):
            v = _dev_tensor(q["verts"], torch.float32, self.device)
            t = _dev_tensor(q["tris"], torch.int32, self.device)
            keep += [v, t]
            reqs[i] = PartRequest(Mesh(_ptr(v), v.shape[0], _ptr(t), t.shape[0]), int(q["n_samples"]),
                                  int(q["seed"]), float(q["tool_length"]))
        return reqs, keep

    @staticmethod
    def _batch_opts(n_dirs, leaf_size=0, rays_per_wave=0, stack_depth=0, offset_frac=0.0, thresholds=None,
                    traversal=0):
        th = Thresholds(*thresholds) if thresholds is not None else None
        o = BatchOpts(n_dirs, leaf_size, rays_per_wave, stack_depth, traversal, offset_frac,
                      C.pointer(th) if th is not None else None)
        return o, th

    def batch_run(self, parts, n_dirs, leaf_size=0, offset_frac=0.0, thresholds=None, bits=None, stream=None):
        """The whole path for many parts: `parts` is a list of dicts with
        verts, tris (device or host), n_samples, seed, tool_length.  Returns
        one result dict per part (classification and setups)."""
        reqs, keep = self._requests(parts)
        opts, th = self._batch_opts(n_dirs, leaf_size, 0, 0, offset_frac, thresholds)
        res = (PartResult * len(parts))()
        self._check(lib().hra_batch_run(self.ptr, reqs, len(parts), C.byref(opts), res, _ptr(bits), _stream(stream)))
        return [_result_dict(r) for r in res]

    def plan(self, parts, n_dirs, leaf_size=0, rays_per_wave=0, stack_depth=0, offset_frac=0.0, thresholds=None,
             traversal=0):
        """A batch plan (all buffers allocated once; runs may replay a graph)."""
        reqs, keep = self._requests(parts)
        opts, th = self._batch_opts(n_dirs, leaf_size, rays_per_wave, stack_depth, offset_frac, thresholds,
                                    traversal)
        out = C.c_void_p()
        self._check(lib().hra_plan_create(self.ptr, reqs, len(parts), C.byref(opts), C.byref(out)))
        return Plan(self, out, len(parts), sum(int(q["n_samples"]) for q in parts), n_dirs, keep)

    def autotune(self, parts, n_dirs, reps=2, offset_frac=0.0, stream=None):
        """Sweep (rays per wave, traversal, leaf size) on this batch; the
        fastest point becomes the context's cast configuration."""
        reqs, keep = self._requests(parts)
        opts, th = self._batch_opts(n_dirs, 0, 0, 0, offset_frac, None)
        rep = TuneReport()
        self._check(lib().hra_autotune(self.ptr, reqs, len(parts), C.byref(opts), reps, C.byref(rep),
                                       _stream(stream)))
        pts = [{"rays_per_wave": p.rays_per_wave, "stack_depth": p.stack_depth, "leaf_size": p.leaf_size,
                "traversal": p.traversal, "ms": p.ms} for p in rep.points[:rep.n_points]]
        return {"points": pts, "best": pts[rep.best]}

    def dirs_table(self, n, kind=DIRS_HEMI):
        import numpy as np
        out = np.empty((n, 3), np.float32)
        self._check(lib().hra_dirs_table(self.ptr, Dirs(kind, n), out.ctypes.data_as(C.c_void_p)))
        return out

    def set_cast_config(self, rays_per_wave=64, stack_depth=16, leaf_size=0, traversal=0, samples_per_group=0):
        """Launch shape of the casts (0 for leaf_size or traversal keeps the current value;
        samples_per_group 0 chooses it from the direction count)."""
        self._check(lib().hra_set_cast_config(self.ptr, C.byref(CastConfig(rays_per_wave, stack_depth, leaf_size,
                                                                            traversal, samples_per_group))))

    def cast_config(self):
        """(rays_per_wave, stack_depth, leaf_size, traversal, samples_per_group)."""
        c = CastConfig()
        self._check(lib().hra_get_cast_config(self.ptr, C.byref(c)))
        return c.rays_per_wave, c.stack_depth, c.leaf_size, c.traversal, c.samples_per_group

    # ---------------------------------------------------------------- samples
    def alloc_samples(self, n):
        d = self.device
        return {"point": torch.empty((n, 3), dtype=torch.float32, device=d),
                "normal": torch.empty((n, 3), dtype=torch.float32, device=d),
                "origin": torch.empty((n, 3), dtype=torch.float32, device=d),
                "tri": torch.empty((n,), dtype=torch.int32, device=d)}

    @staticmethod
    def _samples_struct(s):
        n = s["origin"].shape[0]
        for k in ("point", "normal", "origin"):
            if k in s and s[k] is not None:
                assert s[k].is_contiguous() and s[k].dtype == torch.float32 and s[k].shape == (n, 3), k
        order = s.get("order")
        if order is not None:
            assert order.is_contiguous() and order.dtype == torch.int32 and order.shape == (n,), "order"
        return Samples(_ptr(s.get("point")), _ptr(s.get("normal")), _ptr(s.get("origin")), _ptr(s.get("tri")), n,
                       _ptr(order))

    def sample_surface(self, bvh, n, seed, mode=SAMPLE_AREA, offset_frac=1e-4, stream=None, out=None, part=0):
        if mode == SAMPLE_CENTROID:
            info = bvh.info(stream, part)
            n = info.n_tris - info.n_degenerate
        s = out if out is not None else self.alloc_samples(n)
        assert s["origin"].shape[0] == n
        st = self._samples_struct(s)
        self._check(lib().hra_sample_part(self.ptr, bvh.ptr, part, mode, seed, offset_frac, C.byref(st),
                                          _stream(stream)))
        return s

    # ---------------------------------------------------------------- cast
    def cast(self, bvh, samples, n_dirs, kind=DIRS_HEMI, counts=True, stream=None, bits=None, part=0):
        n = samples["origin"].shape[0]
        W = (n_dirs + 31) // 32
        if bits is None:
            bits = torch.empty((n, W), dtype=torch.int32, device=self.device)
        cnt = torch.empty((n,), dtype=torch.int32, device=self.device) if counts else None
        st = self._samples_struct(samples)
        self._check(lib().hra_cast_part(self.ptr, bvh.ptr, part, C.byref(st), Dirs(kind, n_dirs), _ptr(bits),
                                        _ptr(cnt), _stream(stream)))
        return bits, cnt

    def cast_tool(self, bvh, samples, n_dirs, radius, kind=DIRS_HEMI, counts=True, stream=None, bits=None, part=0):
        """Tool-aware cast (hra_cast_tool): ball-end tool of `radius` mm."""
        n = samples["origin"].shape[0]
        W = (n_dirs + 31) // 32
        if bits is None:
            bits = torch.empty((n, W), dtype=torch.int32, device=self.device)
        cnt = torch.empty((n,), dtype=torch.int32, device=self.device) if counts else None
        st = self._samples_struct(samples)
        self._check(lib().hra_cast_tool(self.ptr, bvh.ptr, part, C.byref(st), Dirs(kind, n_dirs), float(radius),
                                        _ptr(bits), _ptr(cnt), _stream(stream)))
        return bits, cnt

    def cast_tool_holder(self, bvh, samples, n_dirs, radius, cut_length, holder_radius, kind=DIRS_HEMI, counts=True,
                         stream=None, part=0):
        """Tool cast with a holder (hra_cast_tool_holder): cutter of `radius` over
        `cut_length` mm from the tip centre, holder of `holder_radius` beyond."""
        n = samples["origin"].shape[0]
        bits = torch.empty((n, (n_dirs + 31) // 32), dtype=torch.int32, device=self.device)
        cnt = torch.empty((n,), dtype=torch.int32, device=self.device) if counts else None
        st = self._samples_struct(samples)
        self._check(lib().hra_cast_tool_holder(self.ptr, bvh.ptr, part, C.byref(st), Dirs(kind, n_dirs),
                                               float(radius), float(cut_length), float(holder_radius), _ptr(bits),
                                               _ptr(cnt), _stream(stream)))
        return bits, cnt

    def cast_tool_work(self, bvh, samples, n_dirs, radius, kind=DIRS_HEMI, stream=None, part=0):
        """Instrumented tool cast: (bits, node visits, FP64 distance tests, screened triangles)."""
        n = samples["origin"].shape[0]
        bits = torch.empty((n, (n_dirs + 31) // 32), dtype=torch.int32, device=self.device)
        nv, nt, ns = C.c_uint64(), C.c_uint64(), C.c_uint64()
        st = self._samples_struct(samples)
        self._check(lib().hra_cast_tool_work(self.ptr, bvh.ptr, part, C.byref(st), Dirs(kind, n_dirs), float(radius),
                                             _ptr(bits), C.byref(nv), C.byref(nt), C.byref(ns), _stream(stream)))
        return bits, nv.value, nt.value, ns.value

    def cast_work(self, bvh, samples, n_dirs, kind=DIRS_HEMI, stream=None):
        """Instrumented cast: (bits, node fetches, triangle tests) over all rays."""
        n = samples["origin"].shape[0]
        bits = torch.empty((n, (n_dirs + 31) // 32), dtype=torch.int32, device=self.device)
        nf, nt = C.c_uint64(), C.c_uint64()
        st = self._samples_struct(samples)
        self._check(lib().hra_cast_work(self.ptr, bvh.ptr, C.byref(st), Dirs(kind, n_dirs), _ptr(bits), C.byref(nf),
                                        C.byref(nt), _stream(stream)))
        return bits, nf.value, nt.value

    def debug_rays(self, samples, n_dirs, idx, kind=DIRS_HEMI, stream=None):
        idx = _dev_tensor(idx, torch.int64, self.device)
        out = torch.empty((idx.shape[0], n_dirs, 6), dtype=torch.float32, device=self.device)
        st = self._samples_struct(samples)
        self._check(lib().hra_debug_rays(self.ptr, C.byref(st), Dirs(kind, n_dirs), _ptr(idx), idx.shape[0], _ptr(out),
                                         _stream(stream)))
        return out

    # ---------------------------------------------------------------- frame
    def estimate_frame(self, verts, tris, want_hist=False, stream=None):
        """Canonical machining frame (hra_frame_estimate), enqueued on the
        stream.  Returns the device record (a uint8 tensor holding one
        hra_frame; read it with read_frame) and the uint64 [8192] weighted
        histogram, or None."""
        v = _dev_tensor(verts, torch.float32, self.device)
        t = _dev_tensor(tris, torch.int32, self.device)
        fr = torch.empty((C.sizeof(Frame),), dtype=torch.uint8, device=self.device)
        hist = torch.empty((8192,), dtype=torch.int64, device=self.device) if want_hist else None
        m = Mesh(_ptr(v), v.shape[0], _ptr(t), t.shape[0])
        self._check(lib().hra_frame_estimate(self.ptr, C.byref(m), _ptr(hist), _ptr(fr), _stream(stream)))
        if stream is not None:   # copies made here are freed only after that stream passes the call
            v.record_stream(stream)
            t.record_stream(stream)
        return fr, hist

    @staticmethod
    def read_frame(fr):
        """The hra_frame in a device record as a dict (waits for the record)."""
        import numpy as np
        r = Frame.from_buffer_copy(bytes(fr.cpu().numpy().tobytes()))
        return {"axes": np.array([list(row) for row in r.axes]), "confidence": r.confidence,
                "aligned": np.array(list(r.aligned)), "extent": np.array(list(r.extent)),
                "total_area": r.total_area, "peak_bins": (r.peak_bin[0], r.peak_bin[1]), "shift": r.shift,
                "error": r.error}

    def apply_frame(self, fr, verts, out=None, stream=None):
        """Vertices in the frame (hra_frame_apply): float32 [n][3] on the device."""
        v = _dev_tensor(verts, torch.float32, self.device)
        if out is None:
            out = torch.empty_like(v)
        self._check(lib().hra_frame_apply(self.ptr, _ptr(fr), _ptr(v), _ptr(out), v.shape[0], _stream(stream)))
        return out

    def datum_frames(self, bvh, part=0, stream=None):
        """Datum planes per approach direction (hra_datum_frames): six lists
        (a = +X, -X, +Y, -Y, +Z, -Z) of three dicts, primary, secondary and
        tertiary, each {dir, offset, area_w, area, n_tris} (dir -1: empty)."""
        out = (DatumFrame * 6)()
        self._check(lib().hra_datum_frames(self.ptr, bvh.ptr, int(part), out, _stream(stream)))
        return [[{"dir": f.dir[r], "offset": f.offset[r], "area_w": int(f.area_w[r]), "area": f.area[r],
                  "n_tris": f.n_tris[r]} for r in range(3)] for f in out]

    # ---------------------------------------------------------------- stats
    def dominant_axes(self, samples, n_dirs, bits, stream=None, noalloc=False):
        """hra_dominant_axes, or with noalloc=True hra_dominant_axes_noalloc
        (same outputs; the library allocates nothing for the call)."""
        n = samples["origin"].shape[0]
        d = self.device
        out = {"mean": torch.empty((n, 3), dtype=torch.float32, device=d),
               "absmean": torch.empty((n, 3), dtype=torch.float32, device=d),
               "axis": torch.empty((n,), dtype=torch.int8, device=d),
               "conc": torch.empty((n,), dtype=torch.float32, device=d),
               "hist": torch.empty((8192,), dtype=torch.int32, device=d),
               "totals": torch.empty((int(lib().hra_dirstats_bytes(n)),), dtype=torch.uint8, device=d)}
        ds = DirStats(*[_ptr(out[k]) for k in ("mean", "absmean", "axis", "conc", "hist", "totals")])
        st = self._samples_struct(samples)
        fn = lib().hra_dominant_axes_noalloc if noalloc else lib().hra_dominant_axes
        self._check(fn(self.ptr, C.byref(st), Dirs(DIRS_HEMI, n_dirs), _ptr(bits), C.byref(ds), _stream(stream)))
        out["_struct"] = ds
        return out

    def classify(self, stats, n, n_dirs, thresholds=None, stream=None):
        rep = ClassReport()
        th = C.byref(Thresholds(*thresholds)) if thresholds is not None else None
        self._check(lib().hra_classify(self.ptr, C.byref(stats["_struct"]), n, n_dirs, th, C.byref(rep),
                                       _stream(stream)))
        return _class_dict(rep)

    def min_setups(self, bvh, samples, axes_bits, tool_length, want_class=True, stream=None, part=0):
        n = samples["origin"].shape[0]
        cls = torch.empty((n,), dtype=torch.uint8, device=self.device) if want_class else None
        rep = SetupReport()
        st = self._samples_struct(samples)
        ab = axes_bits.reshape(-1).contiguous()
        self._check(lib().hra_min_setups_part(self.ptr, bvh.ptr, part, C.byref(st), _ptr(ab), float(tool_length),
                                              _ptr(cls), C.byref(rep), _stream(stream)))
        out = _setup_dict(rep)
        out["class"] = cls
        return out


def _class_dict(rep):
    return {"access": rep.access, "shares": list(rep.share), "conc": rep.mean_conc, "n_blind": rep.n_blind,
            "n_unobstructed": rep.n_unobstructed, "multi_axis": bool(rep.multi_axis), "tripped": rep.tripped,
            "near_tie": bool(rep.near_tie)}


def _result_dict(r):
    return {"class": _class_dict(r.cls), "setups": _setup_dict(r.setups)}


class Plan:
    """A batch plan: run() returns one result dict per part."""

    def __init__(self, ctx, ptr, n_parts, n_samples, n_dirs, keep):
        self.ctx, self.ptr, self.n_parts, self.n_samples, self.n_dirs = ctx, ptr, n_parts, n_samples, n_dirs
        self._keep = keep

    def run(self, graph=False, bits=None, stream=None):
        res = (PartResult * self.n_parts)()
        self.ctx._check(lib().hra_plan_run(self.ptr, 1 if graph else 0, res, _ptr(bits), _stream(stream)))
        return [_result_dict(r) for r in res]

    def stage_ms(self):
        ms = (C.c_float * 6)()
        self.ctx._check(lib().hra_plan_stage_ms(self.ptr, ms))
        return dict(zip(("build", "sample", "cast", "stats", "axes", "setups"), list(ms)))

    @property
    def bytes(self):
        return int(lib().hra_plan_bytes(self.ptr))

    def destroy(self):
        if self.ptr:
            lib().hra_plan_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _setup_dict(rep):
    return {"min_count": rep.min_count, "min_mask": rep.min_mask, "greedy_count": rep.greedy_count,
            "greedy_mask": rep.greedy_mask, "n_class": list(rep.n_class), "code_hist": list(rep.code_hist)}


def histogram_peaks(hist, k=8):
    """Top-k local maxima of an 8192-bin direction histogram and the six
    45-degree axis-cone masses (library host function)."""
    import numpy as np
    h = np.ascontiguousarray(np.asarray(hist).reshape(-1).view(np.uint32) if hasattr(hist, "view") and
                             np.asarray(hist).dtype != np.uint32 else np.asarray(hist, np.uint32))
    out = HistPeaks()
    st = lib().hra_histogram_peaks(h.ctypes.data_as(C.c_void_p), k, C.byref(out))
    if st != HRA_OK:
        raise HraError(st, "histogram_peaks")
    n = out.n_peaks
    return {"bins": [out.bin[i] for i in range(n)], "mass": [out.mass[i] for i in range(n)],
            "dirs": [list(out.dir[i]) for i in range(n)], "axis_mass": list(out.axis_mass)}


class Bvh:
    def __init__(self, ctx, ptr, keep, stream):
        self.ctx, self.ptr = ctx, ptr
        self._keep = keep   # inputs stay alive until the build has run
        # the stream the build was queued on
        self._stream = stream if stream is not None else torch.cuda.current_stream(ctx.device)

    def _drop_inputs(self):
        """Let the build's input tensors go without waiting: the caching
        allocator reuses their memory only after the work queued so far on
        the build's stream (the build included) has run."""
        keep, self._keep = self._keep, None
        if keep is not None:
            for x in keep:
                x.record_stream(self._stream)

    @property
    def n_parts(self):
        return int(lib().hra_bvh_parts(self.ptr))

    def info(self, stream=None, part=0):
        inf = BvhInfo()
        self.ctx._check(lib().hra_bvh_part_info(self.ptr, part, _stream(stream), C.byref(inf)))
        self._drop_inputs()
        return inf

    def export(self, stream=None):
        """Host copy of a one-part hierarchy: (nodes float32 [nn,16] with
        int32 children in columns 12-13, tris float32 [n_valid,3,4], root,
        n_valid)."""
        import numpy as np
        if self.n_parts != 1:
            raise ValueError("export covers one-part hierarchies")
        inf = self.info(stream)
        nn = max(1, inf.n_tris - 1)
        nodes = np.empty((nn, 16), np.float32)
        tris = np.empty((inf.n_tris, 3, 4), np.float32)
        root, nv = C.c_int32(), C.c_int32()
        self.ctx._check(lib().hra_bvh_export(self.ptr, _stream(stream), nodes.ctypes.data_as(C.c_void_p),
                                             tris.ctypes.data_as(C.c_void_p), C.byref(root), C.byref(nv)))
        return nodes, tris[:nv.value], root.value, nv.value

    def release(self, stream=None):
        """Free the hierarchy.  With the stream it was built on: in stream
        order, without waiting (every other reader must be ordered before
        the work queued on that stream so far); with another stream or none:
        after the device's queued work."""
        self._drop_inputs()
        if self.ptr:
            p, self.ptr = self.ptr, None
            if stream is None:
                lib().hra_bvh_release(p)
            else:
                st = lib().hra_bvh_release_async(p, _stream(stream))
                if st != 0:
                    raise HraError(st, "hierarchy release failed")

    def __del__(self):
        try:
            self._drop_inputs()
            self.release()
        except Exception:
            pass


def read_stl(path):
    """Read a binary or ASCII STL file (hra_stl_read, host only): welded
    float32 vertices [n][3] and int32 triangles [m][3] as numpy arrays."""
    import numpy as np
    m = C.c_void_p()
    nv, nt = C.c_int64(), C.c_int64()
    st = lib().hra_stl_read(os.fsencode(path), C.byref(m), C.byref(nv), C.byref(nt))
    if st != HRA_OK:
        raise HraError(st, (lib().hra_stl_error() or b"").decode())
    try:
        v = np.empty((nv.value, 3), np.float32)
        t = np.empty((nt.value, 3), np.int32)
        st = lib().hra_stl_copy(m, v.ctypes.data_as(C.c_void_p), t.ctypes.data_as(C.c_void_p))
        if st != HRA_OK:
            raise HraError(st, "hra_stl_copy")
    finally:
        lib().hra_stl_free(m)
    return v, t


def now_ns():
    """The server's monotonic clock (nanoseconds)."""
    return int(lib().hra_now_ns())


class Server:
    """Analysis server on one device (its own context and worker thread).
    submit() takes host meshes (numpy or pinned torch tensors), kept alive
    here until their result has been taken."""

    def __init__(self, device=0, n_dirs=1024, mode=SERVE_CONTINUOUS, budget_bytes=0, max_batch=0, max_inflight=0,
                 keep_resident=True, leaf_size=0, offset_frac=0.0, thresholds=None):
        self._th = Thresholds(*thresholds) if thresholds is not None else None
        o = ServerOpts(int(budget_bytes), mode, max_batch, max_inflight, int(keep_resident), n_dirs, leaf_size,
                       offset_frac, C.pointer(self._th) if self._th is not None else None)
        p = C.c_void_p()
        st = lib().hra_server_create(device, C.byref(o), C.byref(p))
        if st != HRA_OK:
            raise HraError(st, "server creation failed")
        self.ptr = p
        self._keep = {}

    @staticmethod
    def _host(x, dtype):
        if isinstance(x, torch.Tensor):
            assert x.device.type == "cpu" and x.is_contiguous() and x.dtype == dtype
            return x, x.data_ptr()
        import numpy as np
        a = np.ascontiguousarray(x, dtype={torch.float32: np.float32, torch.int32: np.int32}[dtype])
        return a, a.ctypes.data

    def submit(self, part_key, verts, tris, n_samples, seed, tool_length):
        v, vp = self._host(verts, torch.float32)
        t, tp = self._host(tris, torch.int32)
        r = Request(int(part_key), vp, v.shape[0], tp, t.shape[0], int(n_samples), int(seed), float(tool_length))
        tk = C.c_uint64()
        st = lib().hra_server_submit(self.ptr, C.byref(r), C.byref(tk))
        if st != HRA_OK:
            raise HraError(st, "submit rejected")
        self._keep[tk.value] = (v, t)
        return tk.value

    def _out(self, tk, r):
        self._keep.pop(tk, None)
        d = {"status": r.status, "resident_hit": bool(r.resident_hit), "batch_size": r.batch_size,
             "batch_id": r.batch_id, "t_submit_ns": r.t_submit_ns, "t_admit_ns": r.t_admit_ns,
             "t_launch_ns": r.t_launch_ns, "t_done_ns": r.t_done_ns}
        if r.status == HRA_OK:
            d.update(_result_dict(r.result))
        return d

    def poll(self, ticket):
        r = RequestResult()
        st = lib().hra_server_poll(self.ptr, ticket, C.byref(r))
        if st == -6:
            return None
        if st != HRA_OK:
            raise HraError(st, f"poll of ticket {ticket}")
        return self._out(ticket, r)

    def wait(self, ticket, timeout_ms=-1):
        r = RequestResult()
        st = lib().hra_server_wait(self.ptr, ticket, int(timeout_ms), C.byref(r))
        if st == -6:
            return None
        if st != HRA_OK:
            raise HraError(st, f"wait for ticket {ticket}")
        return self._out(ticket, r)

    def drain(self, timeout_ms=-1):
        st = lib().hra_server_drain(self.ptr, int(timeout_ms))
        if st != HRA_OK:
            raise HraError(st, "drain timed out")

    def stats(self):
        s = ServerStats()
        lib().hra_server_get_stats(self.ptr, C.byref(s))
        return {n: getattr(s, n) for n, _ in ServerStats._fields_ if n != "pad"}

    def close(self):
        if getattr(self, "ptr", None):
            lib().hra_server_destroy(self.ptr)
            self.ptr = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

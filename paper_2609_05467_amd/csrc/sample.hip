// Surface samples (Section 3.1: per-face centroid, normal and area; rays
// leave a slightly offset point).  FP32 throughout, in a fixed order of
// single IEEE operations; the triangle choice is exact integer work.
//
// One launch serves any number of sampling jobs (a part of a hierarchy, a
// mode, a seed, an output range), so a batch of parts is sampled at once.
#include "common.hpp"
#include "prims.hpp"

namespace hra {

// Unit geometric normal N / |N| with N = (v1 - v0) x (v2 - v0), FP32.
__device__ inline float3 face_normal32(float4 a, float4 b, float4 c) {
    const float e1x = b.x - a.x, e1y = b.y - a.y, e1z = b.z - a.z;
    const float e2x = c.x - a.x, e2y = c.y - a.y, e2z = c.z - a.z;
    const float p1 = e1y * e2z, p2 = e1z * e2y;
    const float nx = p1 - p2;
    const float p3 = e1z * e2x, p4 = e1x * e2z;
    const float ny = p3 - p4;
    const float p5 = e1x * e2y, p6 = e1y * e2x;
    const float nz = p5 - p6;
    const float sx = nx * nx, sy = ny * ny, sz = nz * nz;
    const float sxy = sx + sy;
    const float len = sqrtf(sxy + sz);
    return make_float3(nx / len, ny / len, nz / len);
}

__device__ inline void write_sample(const SampleArgs &S, int64_t i, float3 p, float3 n, float eps, int32_t f) {
    S.point[3 * i + 0] = p.x;
    S.point[3 * i + 1] = p.y;
    S.point[3 * i + 2] = p.z;
    S.normal[3 * i + 0] = n.x;
    S.normal[3 * i + 1] = n.y;
    S.normal[3 * i + 2] = n.z;
    S.origin[3 * i + 0] = fmaf(eps, n.x, p.x);
    S.origin[3 * i + 1] = fmaf(eps, n.y, p.y);
    S.origin[3 * i + 2] = fmaf(eps, n.z, p.z);
    S.tri[i] = f;
}

// Area mode: face = first f of the part whose inclusive weight prefix
// exceeds r = floor(x0 * total / 2^64) (searched as base + r in the global
// prefix); point = the area-uniform square-root parametrisation with u1, u2
// the top 24 bits of the next two generator outputs.
// Centroid mode: one sample per nonzero-area face at ((v0 + v1) + v2) / 3,
// in face order.
__global__ void k_sample(SampleArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_threads) return;
    SampleJob J = a.job0;
    if (a.jobs) {
        int lo = 0, hi = a.n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.jobs[mid].thread_base <= i) lo = mid;
            else hi = mid - 1;
        }
        J = a.jobs[lo];
    }
    const int64_t li = i - J.thread_base;
    if (li < 0 || li >= J.n_threads) return;
    const PartMeta &P = *J.meta;
    const double e = (double)J.offset_frac * P.diag;
    const float eps = (float)e;
    if (J.mode == HRA_SAMPLE_AREA) {
        if (li >= J.n_out) return;
        if (P.total_w == 0) {
            // a part without nonzero-area faces (the build reports it): a
            // defined null sample, face -1
            write_sample(a, J.out_base + li, make_float3(0.0f, 0.0f, 0.0f), make_float3(0.0f, 0.0f, 0.0f), 0.0f, -1);
            return;
        }
        const uint64_t x0 = splitmix64_at(J.seed, 3ull * (uint64_t)li);
        const uint64_t x1 = splitmix64_at(J.seed, 3ull * (uint64_t)li + 1);
        const uint64_t x2 = splitmix64_at(J.seed, 3ull * (uint64_t)li + 2);
        const uint64_t r = P.base_w + __umul64hi(x0, P.total_w);
        int64_t lo = P.tri_start, hi = P.tri_start + P.n_tris - 1;
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if (J.prefix[mid] > r) hi = mid;
            else lo = mid + 1;
        }
        const int32_t p = J.leaf_pos[lo];
        if (p < 0) return;
        const float4 A = J.tris[3 * (int64_t)p], B = J.tris[3 * (int64_t)p + 1], C = J.tris[3 * (int64_t)p + 2];
        const float u1 = (float)(uint32_t)(x1 >> 40) * 0x1p-24f;
        const float u2 = (float)(uint32_t)(x2 >> 40) * 0x1p-24f;
        const float su = sqrtf(u1);
        const float w0 = 1.0f - su;
        const float omu2 = 1.0f - u2;
        const float w1 = su * omu2;
        const float w2 = su * u2;
        float3 pt;
        pt.x = fmaf(w2, C.x, fmaf(w1, B.x, w0 * A.x));
        pt.y = fmaf(w2, C.y, fmaf(w1, B.y, w0 * A.y));
        pt.z = fmaf(w2, C.z, fmaf(w1, B.z, w0 * A.z));
        write_sample(a, J.out_base + li, pt, face_normal32(A, B, C), eps, (int32_t)(lo - P.tri_start));
    } else {
        const int64_t g = P.tri_start + li;
        const int32_t rk = J.valid_rank[g];
        if (rk < 0 || rk >= J.n_out) return;
        const int32_t p = J.leaf_pos[g];
        if (p < 0) return;
        const float4 A = J.tris[3 * (int64_t)p], B = J.tris[3 * (int64_t)p + 1], C = J.tris[3 * (int64_t)p + 2];
        float3 pt;
        pt.x = ((A.x + B.x) + C.x) / 3.0f;
        pt.y = ((A.y + B.y) + C.y) / 3.0f;
        pt.z = ((A.z + B.z) + C.z) / 3.0f;
        write_sample(a, J.out_base + rk, pt, face_normal32(A, B, C), eps, (int32_t)li);
    }
}

SampleJob make_sample_job(const hra_bvh *bvh, int32_t part, int32_t mode, uint64_t seed, float frac, int64_t n_out,
                          int64_t thread_base, int64_t out_base) {
    SampleJob J;
    J.meta = bvh->parts + part;
    J.tris = bvh->tris;
    J.leaf_pos = bvh->leaf_pos;
    J.prefix = bvh->prefix;
    J.valid_rank = bvh->valid_rank;
    J.thread_base = thread_base;
    J.n_threads = mode == HRA_SAMPLE_AREA ? n_out : bvh->part_tris[part];
    J.out_base = out_base;
    J.n_out = n_out;
    J.seed = seed;
    J.offset_frac = frac;
    J.mode = mode;
    return J;
}

hipError_t launch_sample(const SampleJob *d_jobs, int32_t n_jobs, const SampleJob &job0, int64_t n_threads,
                         float *point, float *normal, float *origin, int32_t *tri, hipStream_t s) {
    if (n_threads <= 0) return hipSuccess;
    SampleArgs a;
    a.jobs = d_jobs;
    a.n_jobs = n_jobs;
    a.job0 = job0;
    a.n_threads = n_threads;
    a.point = point;
    a.normal = normal;
    a.origin = origin;
    a.tri = tri;
    k_sample<<<blocks_for(n_threads, 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace hra

using namespace hra;

namespace hra {
// The order changes only which samples a cast runs at the same time (nearby
// ones share the hierarchy's nodes in L2); each sample's result is the same
// in any order.
// Morton code of a point in the part's box, ORDER_AXIS_BITS bits per axis
constexpr int ORDER_AXIS_BITS = 7, ORDER_BITS = 3 * ORDER_AXIS_BITS;
__device__ inline uint32_t morton_code(const float *p, const PartMeta &P) {
    constexpr float cells = (float)(1 << ORDER_AXIS_BITS);
    uint32_t code = 0;
    for (int k = 0; k < 3; ++k) {
        const float lo = P.bbox[k], ext = P.bbox[3 + k] - lo;
        const float t = ext > 0.0f ? (p[k] - lo) / ext : 0.0f;
        const uint32_t q = (uint32_t)fminf(fmaxf(t * cells, 0.0f), cells - 1.0f);   // NaN -> 0
        for (int b = 0; b < ORDER_AXIS_BITS; ++b) code |= ((q >> b) & 1u) << (3 * b + (2 - k));
    }
    return code;
}

__global__ void k_order_keys(const float *origin, int64_t n, const PartMeta *meta, uint64_t *keys, uint32_t *vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = morton_code(origin + 3 * i, *meta);
    vals[i] = (uint32_t)i;
}

__global__ void k_order_keys_jobs(const CastJob *jobs, int32_t n_jobs, CastJob job0, int64_t n, uint64_t *keys,
                                  uint32_t *vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int j = 0;
    if (jobs) {   // the last job whose first item is at most i
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].item_base <= i) lo = mid;
            else hi = mid - 1;
        }
        j = lo;
    }
    const CastJob &J = jobs ? jobs[j] : job0;
    keys[i] = ((uint64_t)j << ORDER_BITS) | morton_code(J.origin + 3 * (i - J.item_base), *J.meta);
    vals[i] = (uint32_t)i;
}

hipError_t sample_order_jobs(const CastJob *d_jobs, int32_t n_jobs, const CastJob &job0, int64_t n, uint64_t *k0,
                             uint32_t *v0, uint64_t *k1, uint32_t *v1, uint32_t *ws, hipStream_t s,
                             const int32_t **order) {
    *order = nullptr;
    if (n <= 0) return hipSuccess;
    int jb = 0;
    while (jb < 31 && ((int64_t)1 << jb) < n_jobs) ++jb;
    const int passes = (ORDER_BITS + jb + 7) / 8;
    k_order_keys_jobs<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(d_jobs, n_jobs, job0, n, k0, v0);
    hipError_t e = hipGetLastError();
    bool in1 = false;
    if (e == hipSuccess) e = sort_pairs(k0, v0, k1, v1, n, ws, s, &in1, passes);
    if (e == hipSuccess) *order = (const int32_t *)(in1 ? v1 : v0);
    return e;
}

size_t sample_order_ws_bytes(int64_t n) { return (size_t)n * 20 + (size_t)sort_pairs_ws_elems(n) * 4 + 64; }

hipError_t sample_order(const float *origin, int64_t n, const PartMeta *meta, int32_t *order, void *ws, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    constexpr int passes = (ORDER_BITS + 7) / 8;
    uint64_t *k0 = (uint64_t *)ws, *k1 = k0 + n;
    uint32_t *vt = (uint32_t *)(k1 + n), *sw = vt + n;
    // the values start in the array the result does not land in: with an
    // odd number of passes the sort ends in (k1, v1), so v1 is the order
    uint32_t *v0 = (passes & 1) ? vt : (uint32_t *)order, *v1 = (passes & 1) ? (uint32_t *)order : vt;
    k_order_keys<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(origin, n, meta, k0, v0);
    hipError_t e = hipGetLastError();
    bool in1 = false;
    if (e == hipSuccess) e = sort_pairs(k0, v0, k1, v1, n, sw, s, &in1, passes);
    if (e == hipSuccess && in1 != (bool)(passes & 1)) e = hipErrorUnknown;
    return e;
}

}  // namespace hra

extern "C" hra_status hra_sample_part(hra_ctx *ctx, const hra_bvh *bvh, int32_t part, int32_t mode, uint64_t seed,
                                      float offset_frac, const hra_samples *out, void *stream) {
    if (!ctx || !bvh || !out) return HRA_ERR_INVALID_ARG;
    if (part < 0 || part >= bvh->n_parts) return ctx->fail(HRA_ERR_INVALID_ARG, "part index out of range");
    if (out->n < 0) return ctx->fail(HRA_ERR_INVALID_ARG, "negative sample count");
    if (!(offset_frac > 0.0f && offset_frac <= 0.01f))
        return ctx->fail(HRA_ERR_INVALID_ARG, "offset_frac must be in (0, 0.01]");
    if (mode != HRA_SAMPLE_AREA && mode != HRA_SAMPLE_CENTROID)
        return ctx->fail(HRA_ERR_INVALID_ARG, "unknown sampling mode");
    if (out->n == 0) return HRA_OK;
    if (!out->point || !out->normal || !out->origin || !out->tri)
        return ctx->fail(HRA_ERR_INVALID_ARG, "sample arrays must be non-null");
    HRA_HIP(hipSetDevice(ctx->device));
    const SampleJob J = make_sample_job(bvh, part, mode, seed, offset_frac, out->n, 0, 0);
    hipStream_t s = (hipStream_t)stream;
    HRA_HIP(launch_sample(nullptr, 1, J, J.n_threads, out->point, out->normal, out->origin, out->tri, s));
    if (out->order) {
        void *ws = nullptr;
        HRA_HIP(hipMallocAsync(&ws, sample_order_ws_bytes(out->n), s));
        const hipError_t e = sample_order(out->origin, out->n, bvh->parts + part, out->order, ws, s);
        const hipError_t ef = hipFreeAsync(ws, s);
        if (e != hipSuccess || ef != hipSuccess)
            return ctx->fail(HRA_ERR_DEVICE, "sample order", hipGetErrorString(e != hipSuccess ? e : ef));
    }
    return HRA_OK;
}

extern "C" hra_status hra_sample_surface(hra_ctx *ctx, const hra_bvh *bvh, int32_t mode, uint64_t seed,
                                         float offset_frac, const hra_samples *out, void *stream) {
    return hra_sample_part(ctx, bvh, 0, mode, seed, offset_frac, out, stream);
}

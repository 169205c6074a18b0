// Surface samples (Section 3.1: per-face centroid, normal and area; rays
// leave a slightly offset point).  FP32 throughout, in a fixed order of
// single IEEE operations; the triangle choice is exact integer work.
#include "common.hpp"

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

__device__ inline float offset_eps(const BvhMeta *meta, float offset_frac) {
    const double e = (double)offset_frac * meta->diag;
    return (float)e;
}

__device__ inline void write_sample(const hra_samples &S, int64_t i, float3 p, float3 n, float eps, int32_t f) {
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

// Area-weighted i.i.d. points.  Face: first f whose inclusive weight prefix
// exceeds r = floor(x0 * total / 2^64); point: the area-uniform square-root
// parametrisation with u1, u2 the top 24 bits of the next two outputs.
__global__ void k_sample_area(const float4 *tri4, const int32_t *leaf_pos, const uint64_t *prefix, int64_t nt,
                              const BvhMeta *meta, uint64_t seed, float offset_frac, hra_samples S) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.n || meta->total_w == 0) return;  // empty mesh: reported by the build
    const uint64_t x0 = splitmix64_at(seed, 3ull * (uint64_t)i);
    const uint64_t x1 = splitmix64_at(seed, 3ull * (uint64_t)i + 1);
    const uint64_t x2 = splitmix64_at(seed, 3ull * (uint64_t)i + 2);
    const uint64_t r = __umul64hi(x0, meta->total_w);
    int64_t lo = 0, hi = nt - 1;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (prefix[mid] > r) hi = mid;
        else lo = mid + 1;
    }
    const int32_t f = (int32_t)lo;
    const int32_t p = leaf_pos[f];
    if (p < 0) return;
    const float4 a = tri4[3 * (int64_t)p], b = tri4[3 * (int64_t)p + 1], c = tri4[3 * (int64_t)p + 2];
    const float u1 = (float)(uint32_t)(x1 >> 40) * 0x1p-24f;
    const float u2 = (float)(uint32_t)(x2 >> 40) * 0x1p-24f;
    const float su = sqrtf(u1);
    const float w0 = 1.0f - su;
    const float omu2 = 1.0f - u2;
    const float w1 = su * omu2;
    const float w2 = su * u2;
    float3 pt;
    pt.x = fmaf(w2, c.x, fmaf(w1, b.x, w0 * a.x));
    pt.y = fmaf(w2, c.y, fmaf(w1, b.y, w0 * a.y));
    pt.z = fmaf(w2, c.z, fmaf(w1, b.z, w0 * a.z));
    write_sample(S, i, pt, face_normal32(a, b, c), offset_eps(meta, offset_frac), f);
}

// One sample per nonzero-area face, at its centroid ((v0 + v1) + v2) / 3.
__global__ void k_sample_centroid(const float4 *tri4, const int32_t *leaf_pos, const int32_t *valid_rank, int64_t nt,
                                  const BvhMeta *meta, float offset_frac, hra_samples S) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nt) return;
    const int32_t rk = valid_rank[f];
    if (rk < 0 || rk >= S.n) return;
    const int32_t p = leaf_pos[f];
    const float4 a = tri4[3 * (int64_t)p], b = tri4[3 * (int64_t)p + 1], c = tri4[3 * (int64_t)p + 2];
    float3 pt;
    pt.x = ((a.x + b.x) + c.x) / 3.0f;
    pt.y = ((a.y + b.y) + c.y) / 3.0f;
    pt.z = ((a.z + b.z) + c.z) / 3.0f;
    write_sample(S, rk, pt, face_normal32(a, b, c), offset_eps(meta, offset_frac), (int32_t)f);
}

}  // namespace hra

using namespace hra;

extern "C" hra_status hra_sample_surface(hra_ctx *ctx, const hra_bvh *bvh, int32_t mode, uint64_t seed,
                                         float offset_frac, const hra_samples *out, void *stream) {
    if (!ctx || !bvh || !out) return HRA_ERR_INVALID_ARG;
    if (out->n < 0) return ctx->fail(HRA_ERR_INVALID_ARG, "negative sample count");
    if (!(offset_frac > 0.0f && offset_frac <= 0.01f))
        return ctx->fail(HRA_ERR_INVALID_ARG, "offset_frac must be in (0, 0.01]");
    if (out->n == 0) return HRA_OK;
    if (!out->point || !out->normal || !out->origin || !out->tri)
        return ctx->fail(HRA_ERR_INVALID_ARG, "sample arrays must be non-null");
    hipStream_t s = (hipStream_t)stream;
    HRA_HIP(hipSetDevice(ctx->device));
    if (mode == HRA_SAMPLE_AREA) {
        k_sample_area<<<blocks_for(out->n, 256), 256, 0, s>>>(bvh->tris, bvh->leaf_pos, bvh->prefix, bvh->n_tris,
                                                             bvh->meta, seed, offset_frac, *out);
    } else if (mode == HRA_SAMPLE_CENTROID) {
        k_sample_centroid<<<blocks_for(bvh->n_tris, 256), 256, 0, s>>>(bvh->tris, bvh->leaf_pos, bvh->valid_rank,
                                                                      bvh->n_tris, bvh->meta, offset_frac, *out);
    } else {
        return ctx->fail(HRA_ERR_INVALID_ARG, "unknown sampling mode");
    }
    HRA_HIP(hipGetLastError());
    return HRA_OK;
}

// Datum planes per setup orientation.  The paper names the automatic
// identification of datum surfaces for each setup as future work (Section
// 6: reference frames for the tolerancing of each machining operation) and
// gives no method; this is the library's, the 3-2-1 rule of fixturing
// applied to the part's axis-facing planes:
//   faces: a triangle faces axis direction d = 2c + (N_c < 0) (+X, -X, +Y,
//     -Y, +Z, -Z, the order of the six-axis cast) when its FP64 normal
//     N = (B - A) x (C - A) has N_c^2 >= 0.99999999 |N|^2 for its dominant
//     component c (within 1e-4 rad of the axis); its offset is
//     h = ((A_c + B_c) + C_c) / 3 and its area the sampler's integer weight;
//   planes: faces sorted by (d, h with the three lowest bits of its
//     order-preserving key dropped, face index), linked while consecutive
//     offsets differ by at most 1e-6 x the bounding-box diagonal; a plane's
//     area is the sum of its weights (exact integers), its offset the least h;
//   frames: for a tool approach direction a, primary = the largest plane of
//     direction a ^ 1 (the side the part rests on), secondary = the largest
//     plane off a's axis, tertiary = the largest off both axes; ties to the
//     lower direction, then the lower offset.
//
// One launch per step over the part's faces: keys, the hierarchy build's
// radix sort, run starts, an inclusive scan of them (run ids), integer
// atomics per run (exact, so their order does not matter), and one block
// that picks the eighteen planes in a fixed order.
#include "common.hpp"
#include "prims.hpp"

#include <cmath>
#include <cstring>

namespace hra {
namespace {

constexpr int DT_TB = 256;
constexpr uint64_t DT_NONE = ~0ull;   // key of a face that faces no axis: sorts last
constexpr double DT_FACING = 0.99999999;
constexpr double DT_LINK = 1e-6;

struct DatumRun {
    unsigned long long area_w;   // sum of the faces' integer weights
    unsigned long long h_key;    // least order key of the faces' offsets
    uint32_t count;
    int32_t dir;
};

__device__ inline uint64_t order_key(double h) {
    const uint64_t u = (uint64_t)__double_as_longlong(h);
    return (u >> 63) ? ~u : (u | (1ull << 63));
}

// Axis direction (or -1) and offset of the triangle (A, B, C): the sampler's
// FP64 normal and its squared length, operation for operation.
__device__ inline int face_dir(float4 A, float4 B, float4 C, double &h) {
    const double e1x = (double)B.x - (double)A.x, e1y = (double)B.y - (double)A.y, e1z = (double)B.z - (double)A.z;
    const double e2x = (double)C.x - (double)A.x, e2y = (double)C.y - (double)A.y, e2z = (double)C.z - (double)A.z;
    const double p1 = e1y * e2z, p2 = e1z * e2y;
    const double nx = p1 - p2;
    const double p3 = e1z * e2x, p4 = e1x * e2z;
    const double ny = p3 - p4;
    const double p5 = e1x * e2y, p6 = e1y * e2x;
    const double nz = p5 - p6;
    const double sx = nx * nx, sy = ny * ny, sz = nz * nz;
    const double sxy = sx + sy;
    const double q = sxy + sz;
    int c = 0;
    double nc = nx, sc = sx, ac = fabs(nx);
    if (fabs(ny) > ac) {
        c = 1;
        nc = ny;
        sc = sy;
        ac = fabs(ny);
    }
    if (fabs(nz) > ac) {
        c = 2;
        nc = nz;
        sc = sz;
    }
    const double a = c == 0 ? (double)A.x : (c == 1 ? (double)A.y : (double)A.z);
    const double b = c == 0 ? (double)B.x : (c == 1 ? (double)B.y : (double)B.z);
    const double cc = c == 0 ? (double)C.x : (c == 1 ? (double)C.y : (double)C.z);
    h = ((a + b) + cc) / 3.0;
    if (!(q > 0.0) || !(sc >= DT_FACING * q)) return -1;
    return 2 * c + (nc < 0.0 ? 1 : 0);
}

__device__ inline int face_of(const float4 *tris, const int32_t *leaf_pos, int64_t g, double &h) {
    const int32_t p = leaf_pos[g];
    h = 0.0;
    if (p < 0) return -1;
    return face_dir(tris[3 * (int64_t)p], tris[3 * (int64_t)p + 1], tris[3 * (int64_t)p + 2], h);
}

__global__ void k_datum_keys(const float4 *tris, const int32_t *leaf_pos, int64_t tri_start, int64_t n,
                             uint64_t *keys, uint32_t *vals) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n) return;
    double h;
    const int d = face_of(tris, leaf_pos, tri_start + f, h);
    keys[f] = d < 0 ? DT_NONE : (((uint64_t)d << 61) | (order_key(h) >> 3));
    vals[f] = (uint32_t)f;
}

// flags[i] = 1 where a plane starts in sorted order
__global__ void k_datum_starts(const uint64_t *keys, const uint32_t *vals, const float4 *tris, const int32_t *leaf_pos,
                               int64_t tri_start, int64_t n, const PartMeta *meta, uint32_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = keys[i];
    if (k == DT_NONE) {
        flags[i] = 0u;
        return;
    }
    bool start = i == 0 || (keys[i - 1] >> 61) != (k >> 61);
    if (!start) {
        double h, hp;
        face_of(tris, leaf_pos, tri_start + vals[i], h);
        face_of(tris, leaf_pos, tri_start + vals[i - 1], hp);
        start = (h - hp) > DT_LINK * meta->diag;
    }
    flags[i] = start ? 1u : 0u;
}

__global__ void k_datum_clear(DatumRun *runs, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    runs[i].area_w = 0ull;
    runs[i].h_key = ~0ull;
    runs[i].count = 0u;
    runs[i].dir = -1;
}

// rid: inclusive scan of the starts (run index + 1)
__global__ void k_datum_accum(const uint64_t *keys, const uint32_t *vals, const uint32_t *flags, const uint32_t *rid,
                              const float4 *tris, const int32_t *leaf_pos, const uint64_t *prefix, int64_t tri_start,
                              int64_t n, DatumRun *runs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = keys[i];
    if (k == DT_NONE) return;
    const int64_t g = tri_start + vals[i];
    double h;
    face_of(tris, leaf_pos, g, h);
    const uint64_t w = prefix[g] - (g > 0 ? prefix[g - 1] : 0ull);
    DatumRun &R = runs[rid[i] - 1u];
    atomicAdd(&R.area_w, (unsigned long long)w);
    atomicAdd(&R.count, 1u);
    atomicMin(&R.h_key, (unsigned long long)order_key(h));
    if (flags[i]) R.dir = (int32_t)(k >> 61);
}

// (area desc, direction asc, offset asc): true when run x is better than y
__device__ inline bool better(const DatumRun &x, const DatumRun &y) {
    if (x.area_w != y.area_w) return x.area_w > y.area_w;
    if (x.dir != y.dir) return x.dir < y.dir;
    return x.h_key < y.h_key;
}

// One block: for each approach direction a and role r, the best run under
// the role's filter; sel[3 a + r] = run index or -1.
__global__ __launch_bounds__(DT_TB) void k_datum_select(const DatumRun *runs, const uint32_t *rid_last, int32_t *sel) {
    __shared__ int32_t best[DT_TB];
    __shared__ int32_t axis_sec;
    const int t = threadIdx.x;
    const int64_t nr = *rid_last;
    for (int a = 0; a < 6; ++a) {
        for (int r = 0; r < 3; ++r) {
            const int ax = a >> 1;
            const int sec_axis = r == 2 ? axis_sec : -1;
            int32_t b = -1;
            for (int64_t j = t; j < nr; j += DT_TB) {
                const DatumRun &R = runs[j];
                bool ok;
                if (r == 0) ok = R.dir == (a ^ 1);
                else if (r == 1) ok = (R.dir >> 1) != ax;
                else ok = sec_axis >= 0 && (R.dir >> 1) != ax && (R.dir >> 1) != sec_axis;
                if (ok && (b < 0 || better(R, runs[b]))) b = (int32_t)j;
            }
            best[t] = b;
            __syncthreads();
            for (int off = DT_TB / 2; off > 0; off >>= 1) {
                if (t < off) {
                    const int32_t o = best[t + off], m = best[t];
                    if (o >= 0 && (m < 0 || better(runs[o], runs[m]))) best[t] = o;
                }
                __syncthreads();
            }
            if (t == 0) {
                sel[3 * a + r] = best[0];
                if (r == 1) axis_sec = best[0] >= 0 ? (runs[best[0]].dir >> 1) : -1;
            }
            __syncthreads();
        }
    }
}

__global__ void k_datum_gather(const DatumRun *runs, const int32_t *sel, DatumRun *out) {
    const int i = threadIdx.x;
    if (i >= 18) return;
    const int32_t j = sel[i];
    if (j >= 0) {
        out[i] = runs[j];
    } else {
        out[i].area_w = 0ull;
        out[i].h_key = ~0ull;
        out[i].count = 0u;
        out[i].dir = -1;
    }
}

double from_order_key(uint64_t k) {
    const uint64_t u = (k >> 63) ? (k & ~(1ull << 63)) : ~k;
    double h;
    std::memcpy(&h, &u, sizeof h);
    return h;
}

}  // namespace
}  // namespace hra

using namespace hra;

extern "C" hra_status hra_datum_frames(hra_ctx *ctx, const hra_bvh *bvh, int32_t part, hra_datum_frame *out,
                                       void *stream) {
    if (!ctx || !bvh || !out) return HRA_ERR_INVALID_ARG;
    if (part < 0 || part >= bvh->n_parts) return ctx->fail(HRA_ERR_INVALID_ARG, "part index out of range");
    hipStream_t s = (hipStream_t)stream;
    HRA_HIP(hipSetDevice(ctx->device));
    const int64_t n = bvh->part_tris[part], t0 = bvh->part_start[part];
    for (int a = 0; a < 6; ++a) {
        for (int r = 0; r < 3; ++r) {
            out[a].dir[r] = -1;
            out[a].n_tris[r] = 0;
            out[a].offset[r] = 0.0;
            out[a].area[r] = 0.0;
            out[a].area_w[r] = 0;
        }
    }
    if (n <= 0) return HRA_OK;
    if (n >= ((int64_t)1 << 31)) return ctx->fail(HRA_ERR_INVALID_ARG, "part too large for the datum search");
    PartMeta P;
    HRA_HIP(hipMemcpyAsync(&P, bvh->parts + part, sizeof(P), hipMemcpyDeviceToHost, s));
    // workspace: keys x2, values x2, starts, run ids, runs, sort and scan
    // space, selection and its gathered runs
    const int64_t sort_ws = sort_pairs_ws_elems(n), scan_ws = scan_u32_ws_elems(n);
    const size_t bytes = 16 * (size_t)n + 8 * (size_t)n + 8 * (size_t)n + sizeof(DatumRun) * (size_t)n +
                         4 * (size_t)(sort_ws + scan_ws) + 4 * 18 + sizeof(DatumRun) * 18 + 256;
    char *ws = nullptr;
    HRA_HIP(hipMallocAsync((void **)&ws, bytes, s));
    char *q = ws;
    auto take = [&](size_t b) {
        char *r = q;
        q += (b + 15) & ~(size_t)15;
        return r;
    };
    uint64_t *k0 = (uint64_t *)take(8 * n), *k1 = (uint64_t *)take(8 * n);
    uint32_t *v0 = (uint32_t *)take(4 * n), *v1 = (uint32_t *)take(4 * n);
    uint32_t *flags = (uint32_t *)take(4 * n), *rid = (uint32_t *)take(4 * n);
    DatumRun *runs = (DatumRun *)take(sizeof(DatumRun) * n);
    uint32_t *sws = (uint32_t *)take(4 * sort_ws), *cws = (uint32_t *)take(4 * scan_ws);
    int32_t *sel = (int32_t *)take(4 * 18);
    DatumRun *picked = (DatumRun *)take(sizeof(DatumRun) * 18);
    const unsigned nb = (unsigned)((n + DT_TB - 1) / DT_TB);
    hipError_t e = hipSuccess;
    k_datum_keys<<<nb, DT_TB, 0, s>>>(bvh->tris, bvh->leaf_pos, t0, n, k0, v0);
    bool in_k1 = false;
    e = hipGetLastError();
    if (e == hipSuccess) e = sort_pairs(k0, v0, k1, v1, n, sws, s, &in_k1);
    const uint64_t *ks = in_k1 ? k1 : k0;
    const uint32_t *vs = in_k1 ? v1 : v0;
    if (e == hipSuccess) {
        k_datum_starts<<<nb, DT_TB, 0, s>>>(ks, vs, bvh->tris, bvh->leaf_pos, t0, n, bvh->parts + part, flags);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = scan_u32(flags, rid, n, true, cws, s);
    if (e == hipSuccess) {
        k_datum_clear<<<nb, DT_TB, 0, s>>>(runs, n);
        k_datum_accum<<<nb, DT_TB, 0, s>>>(ks, vs, flags, rid, bvh->tris, bvh->leaf_pos, bvh->prefix, t0, n, runs);
        k_datum_select<<<1, DT_TB, 0, s>>>(runs, rid + (n - 1), sel);
        k_datum_gather<<<1, 64, 0, s>>>(runs, sel, picked);
        e = hipGetLastError();
    }
    DatumRun h[18];
    if (e == hipSuccess) e = hipMemcpyAsync(h, picked, sizeof(h), hipMemcpyDeviceToHost, s);
    const hipError_t ef = hipFreeAsync(ws, s);
    if (e == hipSuccess) e = ef;
    if (e != hipSuccess) return ctx->fail(HRA_ERR_DEVICE, "datum search launch failed", hipGetErrorString(e));
    hra_status st = check_error_word(ctx, s);   // synchronises the stream
    if (st != HRA_OK) return st;
    const double scale = std::ldexp(1.0, -P.k_scale);
    for (int a = 0; a < 6; ++a) {
        for (int r = 0; r < 3; ++r) {
            const DatumRun &R = h[3 * a + r];
            if (R.dir < 0) continue;
            out[a].dir[r] = R.dir;
            out[a].n_tris[r] = (int32_t)R.count;
            out[a].offset[r] = from_order_key(R.h_key);
            out[a].area_w[r] = R.area_w;
            out[a].area[r] = (double)R.area_w * scale;
        }
    }
    return HRA_OK;
}

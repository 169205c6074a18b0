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

// Per face (index f within the part): its sort key and index, and its
// offset and integer weight for the later passes.
__global__ void k_datum_keys(const float4 *tris, const int32_t *leaf_pos, const uint64_t *prefix, int64_t tri_start,
                             int64_t n, uint64_t *keys, uint32_t *vals, double *hf, uint64_t *wf) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n) return;
    const int64_t g = tri_start + f;
    double h;
    const int d = face_of(tris, leaf_pos, g, h);
    keys[f] = d < 0 ? DT_NONE : (((uint64_t)d << 61) | (order_key(h) >> 3));
    vals[f] = (uint32_t)f;
    hf[f] = h;
    wf[f] = prefix[g] - (g > 0 ? prefix[g - 1] : 0ull);
}

// flags[i] = 1 where a plane starts in sorted order
__global__ void k_datum_starts(const uint64_t *keys, const uint32_t *vals, const double *hf, int64_t n,
                               const PartMeta *meta, uint32_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = keys[i];
    if (k == DT_NONE) {
        flags[i] = 0u;
        return;
    }
    bool start = i == 0 || (keys[i - 1] >> 61) != (k >> 61);
    if (!start) start = (hf[vals[i]] - hf[vals[i - 1]]) > DT_LINK * meta->diag;
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

constexpr int DT_ACC_TILES = 16;   // consecutive 64-element tiles per wave in k_datum_accum

__device__ inline void run_flush(DatumRun *runs, int64_t r, unsigned long long w, uint32_t c, unsigned long long hk) {
    DatumRun &R = runs[r];
    atomicAdd(&R.area_w, w);
    atomicAdd(&R.count, c);
    atomicMin(&R.h_key, hk);
}

// rid: inclusive scan of the starts (run index + 1).  Runs are contiguous
// in sorted order.  Each wave walks DT_ACC_TILES consecutive tiles of 64
// elements; in a tile its lanes fold their values per run (a segmented
// inclusive scan over shuffles), runs that end inside the tile go to their
// totals from their last lane, and the run still open at lane 63 is carried
// to the next tile in registers.  A plane of a million faces then costs one
// atomic per 1,024 faces, not one per face; all sums are integers and the
// offset a minimum, so the order of the atomics does not matter.
__global__ __launch_bounds__(DT_TB) void k_datum_accum(const uint64_t *keys, const uint32_t *vals, const uint32_t *flags,
                                                       const uint32_t *rid, const double *hf, const uint64_t *wf,
                                                       int64_t n, DatumRun *runs) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * DT_TB + threadIdx.x) >> 6;
    const int64_t base = wave * 64 * DT_ACC_TILES;
    // Every value that reaches a shuffle is formed by selects, never
    // assigned under a lane-dependent branch (the compiler has mis-merged
    // such values across divergent regions); the trip counts are uniform.
    int64_t cr = -1;   // carried run (-1: none) and its partial totals, the same in every lane
    unsigned long long cw = 0ull, chk = ~0ull;
    uint32_t cc = 0u;
    for (int it = 0; it < DT_ACC_TILES; ++it) {
        const int64_t i = base + 64 * it + lane;
        const bool inb = i < n;
        const int64_t ic = inb ? i : 0;   // n >= 1: element 0 is readable
        const uint64_t k = keys[ic];
        const bool valid = inb && k != DT_NONE;
        const uint32_t f = vals[ic];      // a face index of the part, < n
        const unsigned long long wv = wf[f], hv = order_key(hf[f]);
        // run index, -1: no run (past the end, or a face that faces no axis)
        int64_t r = valid ? (int64_t)rid[ic] - 1 : -1;
        unsigned long long w = valid ? wv : 0ull, hk = valid ? hv : ~0ull;
        uint32_t cnt = valid ? 1u : 0u;
        if (valid && flags[ic]) runs[r].dir = (int32_t)(k >> 61);
        // a carried run that does not continue into this tile is complete
        const int64_t r0 = __shfl(r, 0, 64);
        const bool close = cr >= 0 && r0 != cr;
        if (close && lane == 0) run_flush(runs, cr, cw, cc, chk);
        cr = close ? -1 : cr;
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t r_o = __shfl_up(r, off, 64);
            const unsigned long long w_o = __shfl_up(w, off, 64), hk_o = __shfl_up(hk, off, 64);
            const uint32_t c_o = __shfl_up(cnt, off, 64);
            const bool m = lane >= off && r_o == r;
            w = m ? w + w_o : w;
            cnt = m ? cnt + c_o : cnt;
            hk = (m && hk_o < hk) ? hk_o : hk;
        }
        // the tile's first run continues the carried one
        const bool cont = r >= 0 && r == cr;
        w = cont ? w + cw : w;
        cnt = cont ? cnt + cc : cnt;
        hk = (cont && chk < hk) ? chk : hk;
        const int64_t r_next = __shfl_down(r, 1, 64);
        if (r >= 0 && lane != 63 && r_next != r) run_flush(runs, r, w, cnt, hk);
        cr = __shfl(r, 63, 64);
        cw = __shfl(w, 63, 64);
        chk = __shfl(hk, 63, 64);
        cc = __shfl(cnt, 63, 64);
    }
    if (cr >= 0 && lane == 0) run_flush(runs, cr, cw, cc, chk);
}

// (area desc, direction asc, offset asc): true when run x is better than y
__device__ inline bool better(const DatumRun &x, const DatumRun &y) {
    if (x.area_w != y.area_w) return x.area_w > y.area_w;
    if (x.dir != y.dir) return x.dir < y.dir;
    return x.h_key < y.h_key;
}

__device__ inline int32_t pick(const DatumRun *runs, int32_t x, int32_t y) {
    if (x < 0) return y;
    if (y < 0) return x;
    return better(runs[y], runs[x]) ? y : x;
}

// One block.  Under a total order the best plane of a set of directions is
// the best of the directions' own bests, so one pass finds the best run of
// each direction and thread 0 forms the eighteen roles from those six:
// sel[3 a + r] = run index or -1.
__global__ __launch_bounds__(DT_TB) void k_datum_select(const DatumRun *runs, const uint32_t *rid_last, int32_t *sel) {
    __shared__ int32_t best[6][DT_TB];
    const int t = threadIdx.x;
    const int64_t nr = *rid_last;
    int32_t b[6] = {-1, -1, -1, -1, -1, -1};
    for (int64_t j = t; j < nr; j += DT_TB) {
        const int d = runs[j].dir;
        for (int q = 0; q < 6; ++q)
            if (q == d) b[q] = pick(runs, b[q], (int32_t)j);
    }
    for (int q = 0; q < 6; ++q) best[q][t] = b[q];
    __syncthreads();
    for (int off = DT_TB / 2; off > 0; off >>= 1) {
        if (t < off)
            for (int q = 0; q < 6; ++q) best[q][t] = pick(runs, best[q][t], best[q][t + off]);
        __syncthreads();
    }
    if (t != 0) return;
    for (int a = 0; a < 6; ++a) {
        const int ax = a >> 1;
        const int32_t prim = best[a ^ 1][0];
        int32_t sec = -1;
        for (int d = 0; d < 6; ++d)
            if ((d >> 1) != ax) sec = pick(runs, sec, best[d][0]);
        int32_t ter = -1;
        if (sec >= 0) {
            const int sx = runs[sec].dir >> 1;
            for (int d = 0; d < 6; ++d)
                if ((d >> 1) != ax && (d >> 1) != sx) ter = pick(runs, ter, best[d][0]);
        }
        sel[3 * a] = prim;
        sel[3 * a + 1] = sec;
        sel[3 * a + 2] = ter;
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
    // workspace: keys x2, values x2, starts, run ids, runs, per-face offsets
    // and weights, sort and scan space, selection and its gathered runs
    const int64_t sort_ws = sort_pairs_ws_elems(n), scan_ws = scan_u32_ws_elems(n);
    // (thirteen pieces, each padded to a multiple of 16 bytes)
    const size_t bytes = 16 * (size_t)n + 8 * (size_t)n + 8 * (size_t)n + 16 * (size_t)n +
                         sizeof(DatumRun) * (size_t)n + 4 * (size_t)(sort_ws + scan_ws) + 4 * 18 +
                         sizeof(DatumRun) * 18 + 13 * 16;
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
    double *hf = (double *)take(8 * n);
    uint64_t *wf = (uint64_t *)take(8 * n);
    uint32_t *sws = (uint32_t *)take(4 * sort_ws), *cws = (uint32_t *)take(4 * scan_ws);
    int32_t *sel = (int32_t *)take(4 * 18);
    DatumRun *picked = (DatumRun *)take(sizeof(DatumRun) * 18);
    const unsigned nb = (unsigned)((n + DT_TB - 1) / DT_TB);
    hipError_t e = hipSuccess;
    k_datum_keys<<<nb, DT_TB, 0, s>>>(bvh->tris, bvh->leaf_pos, bvh->prefix, t0, n, k0, v0, hf, wf);
    bool in_k1 = false;
    e = hipGetLastError();
    if (e == hipSuccess) e = sort_pairs(k0, v0, k1, v1, n, sws, s, &in_k1);
    const uint64_t *ks = in_k1 ? k1 : k0;
    const uint32_t *vs = in_k1 ? v1 : v0;
    if (e == hipSuccess) {
        k_datum_starts<<<nb, DT_TB, 0, s>>>(ks, vs, hf, n, bvh->parts + part, flags);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = scan_u32(flags, rid, n, true, cws, s);
    if (e == hipSuccess) {
        k_datum_clear<<<nb, DT_TB, 0, s>>>(runs, n);
        const int64_t acc_waves = (n + 64 * DT_ACC_TILES - 1) / (64 * DT_ACC_TILES);
        k_datum_accum<<<(unsigned)((acc_waves + DT_TB / 64 - 1) / (DT_TB / 64)), DT_TB, 0, s>>>(ks, vs, flags, rid, hf,
                                                                                              wf, n, runs);
        k_datum_select<<<1, DT_TB, 0, s>>>(runs, rid + (n - 1), sel);
        k_datum_gather<<<1, 64, 0, s>>>(runs, sel, picked);
        e = hipGetLastError();
    }
    // both results through the context's pinned staging, after every launch
    static_assert(sizeof(DatumRun) * 18 + 16 + sizeof(PartMeta) <= STAGE_BYTES - STAGE_USER, "staging too small");
    DatumRun *h = (DatumRun *)stage_user(ctx);
    PartMeta *hp = (PartMeta *)((char *)h + ((sizeof(DatumRun) * 18 + 15) & ~(size_t)15));
    if (e == hipSuccess) e = hipMemcpyAsync(h, picked, sizeof(DatumRun) * 18, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hp, bvh->parts + part, sizeof(PartMeta), hipMemcpyDeviceToHost, s);
    const hipError_t ef = hipFreeAsync(ws, s);
    if (e == hipSuccess) e = ef;
    if (e != hipSuccess) return ctx->fail(HRA_ERR_DEVICE, "datum search launch failed", hipGetErrorString(e));
    hra_status st = check_error_word(ctx, s);   // synchronises the stream
    if (st != HRA_OK) return st;
    const double scale = std::ldexp(1.0, -hp->k_scale);
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

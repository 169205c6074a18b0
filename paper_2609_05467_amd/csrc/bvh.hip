// Mesh ingest and LBVH construction, all on the device.
//
// Stages (one stream, no host round trip):
//   1. per-triangle prep: index check, FP64 doubled-area-squared, area,
//      nonzero-area flag;
//   2. vertex bbox, largest area (two-pass reductions) -> BvhMeta;
//   3. integer area weights and their inclusive prefix (for the sampler),
//      ranks of nonzero-area faces (for centroid samples);
//   4. 63-bit Morton codes of centroids; zero-area faces get the largest key;
//   5. LSD radix sort, 8 passes of 8 bits, LDS digit counts and a stable
//      LDS-ranked scatter;
//   6. binary radix tree over the sorted codes (Karras, "Maximizing
//      Parallelism in the Construction of BVHs, Octrees, and k-d Trees", HPG
//      2012), ties between equal codes broken by position;
//   7. bottom-up box refit: the second thread to reach a node merges it;
//   8. leaf collapse (subtrees with <= leaf_size triangles become one leaf
//      over a contiguous run) and emission of 64-byte nodes.
#include "common.hpp"

#include <algorithm>

namespace hra {

constexpr int TB = 256;

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------- scans
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = TB * SCAN_ITEMS;

template <typename T>
__global__ void k_scan_tile(const T *in, T *out, int64_t n, T *block_sums, int inclusive) {
    __shared__ T s[TB];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)tid * SCAN_ITEMS;
    T v[SCAN_ITEMS];
    T tot = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t i = base + k;
        v[k] = i < n ? in[i] : (T)0;
        tot += v[k];
    }
    s[tid] = tot;
    __syncthreads();
    for (int off = 1; off < TB; off <<= 1) {
        T add = tid >= off ? s[tid - off] : (T)0;
        __syncthreads();
        s[tid] += add;
        __syncthreads();
    }
    T run = s[tid] - tot;  // exclusive prefix of this thread's items
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t i = base + k;
        const T x = v[k];
        if (i < n) out[i] = inclusive ? run + x : run;
        run += x;
    }
    if (block_sums && tid == TB - 1) block_sums[blockIdx.x] = s[TB - 1];
}

template <typename T>
__global__ void k_scan_add(T *out, int64_t n, const T *block_prefix) {
    const T add = block_prefix[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    for (int k = threadIdx.x; k < SCAN_TILE; k += TB) {
        const int64_t i = base + k;
        if (i < n) out[i] += add;
    }
}

template <typename T>
static hipError_t scan(const T *in, T *out, int64_t n, bool inclusive, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        k_scan_tile<T><<<1, TB, 0, s>>>(in, out, n, (T *)nullptr, inclusive ? 1 : 0);
        return hipGetLastError();
    }
    T *sums = nullptr;
    hipError_t e = hipMallocAsync((void **)&sums, sizeof(T) * nb, s);
    if (e != hipSuccess) return e;
    k_scan_tile<T><<<(unsigned)nb, TB, 0, s>>>(in, out, n, sums, inclusive ? 1 : 0);
    e = scan<T>(sums, sums, nb, false, s);
    if (e == hipSuccess) {
        k_scan_add<T><<<(unsigned)nb, TB, 0, s>>>(out, n, sums);
        e = hipGetLastError();
    }
    hipFreeAsync(sums, s);
    return e;
}

// ---------------------------------------------------------------- ingest
// FP64 doubled area squared, fixed order (twice the area is |(v1-v0)x(v2-v0)|).
__device__ inline double tri_q64(const float *a, const float *b, const float *c) {
    const double e1x = (double)b[0] - (double)a[0], e1y = (double)b[1] - (double)a[1], e1z = (double)b[2] - (double)a[2];
    const double e2x = (double)c[0] - (double)a[0], e2y = (double)c[1] - (double)a[1], e2z = (double)c[2] - (double)a[2];
    const double p1 = e1y * e2z, p2 = e1z * e2y;
    const double nx = p1 - p2;
    const double p3 = e1z * e2x, p4 = e1x * e2z;
    const double ny = p3 - p4;
    const double p5 = e1x * e2y, p6 = e1y * e2x;
    const double nz = p5 - p6;
    const double sx = nx * nx, sy = ny * ny, sz = nz * nz;
    const double sxy = sx + sy;
    return sxy + sz;
}

__global__ void k_tri_prep(const float *verts, int64_t nv, const int32_t *tris, int64_t nt, double *area,
                           uint32_t *valid, uint32_t *err) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nt) return;
    const int32_t i0 = tris[3 * f], i1 = tris[3 * f + 1], i2 = tris[3 * f + 2];
    if (i0 < 0 || i1 < 0 || i2 < 0 || i0 >= nv || i1 >= nv || i2 >= nv) {
        atomicOr(err, ERR_BAD_INDEX);
        area[f] = 0.0;
        valid[f] = 0;
        return;
    }
    const double q = tri_q64(verts + 3 * (int64_t)i0, verts + 3 * (int64_t)i1, verts + 3 * (int64_t)i2);
    const bool ok = q > 0.0;
    area[f] = ok ? 0.5 * sqrt(q) : 0.0;
    valid[f] = ok ? 1u : 0u;
}

constexpr int RED_BLOCKS = 256;

// partial[b] = {min xyz, max xyz, max area}
__global__ void k_reduce_partial(const float *verts, int64_t nv, const double *area, int64_t nt, double *partial) {
    __shared__ double s[7][TB];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double amax = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride)
        for (int c = 0; c < 3; ++c) {
            const float x = verts[3 * i + c];
            lo[c] = fminf(lo[c], x);
            hi[c] = fmaxf(hi[c], x);
        }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nt; i += stride) amax = fmax(amax, area[i]);
    const int t = threadIdx.x;
    for (int c = 0; c < 3; ++c) {
        s[c][t] = lo[c];
        s[3 + c][t] = hi[c];
    }
    s[6][t] = amax;
    __syncthreads();
    for (int off = TB / 2; off > 0; off >>= 1) {
        if (t < off) {
            for (int c = 0; c < 3; ++c) {
                s[c][t] = fmin(s[c][t], s[c][t + off]);
                s[3 + c][t] = fmax(s[3 + c][t], s[3 + c][t + off]);
            }
            s[6][t] = fmax(s[6][t], s[6][t + off]);
        }
        __syncthreads();
    }
    if (t == 0)
        for (int k = 0; k < 7; ++k) partial[7 * blockIdx.x + k] = s[k][0];
}

__global__ void k_reduce_final(const double *partial, int nparts, int64_t nt, BvhMeta *meta) {
    if (threadIdx.x != 0) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, amax = 0.0;
    for (int b = 0; b < nparts; ++b) {
        for (int c = 0; c < 3; ++c) {
            lo[c] = fmin(lo[c], partial[7 * b + c]);
            hi[c] = fmax(hi[c], partial[7 * b + 3 + c]);
        }
        amax = fmax(amax, partial[7 * b + 6]);
    }
    for (int c = 0; c < 3; ++c) {
        meta->bbox[c] = (float)lo[c];
        meta->bbox[3 + c] = (float)hi[c];
    }
    const double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    const double sx = dx * dx, sy = dy * dy, sz = dz * dz;
    const double sxy = sx + sy;
    meta->diag = sqrt(sxy + sz);
    meta->amax = amax;
    // weights floor(area * 2^k) with k = 62 - (ilogb(amax) + 1) - bitlen(nt)
    // keep the weight sum below 2^62
    int tb = 0;
    while (tb < 63 && ((int64_t)1 << tb) <= nt) ++tb;
    meta->k_scale = amax > 0.0 ? 62 - (ilogb(amax) + 1) - tb : 0;
    meta->root = 0;
    meta->depth = 0;
    meta->n_nodes = 0;
}

__global__ void k_weights(const double *area, int64_t nt, const BvhMeta *meta, uint64_t *w) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nt) return;
    w[f] = (uint64_t)floor(ldexp(area[f], meta->k_scale));
}

__global__ void k_ranks(const uint32_t *valid, const uint32_t *excl, int64_t nt, int32_t *rank, const uint64_t *prefix,
                        BvhMeta *meta, uint32_t *err) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nt) return;
    rank[f] = valid[f] ? (int32_t)excl[f] : -1;
    if (f == nt - 1) {
        const int32_t nvld = (int32_t)(excl[f] + valid[f]);
        meta->n_valid = nvld;
        meta->total_w = prefix[f];
        if (nvld == 0) atomicOr(err, ERR_EMPTY_MESH);
    }
}

// ---------------------------------------------------------------- Morton
__device__ inline uint64_t spread21(uint32_t x) {
    uint64_t v = x & 0x1FFFFFu;
    v = (v | (v << 32)) & 0x001F00000000FFFFull;
    v = (v | (v << 16)) & 0x001F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ inline uint32_t quant21(float c, float lo, float hi) {
    const float ext = hi - lo;
    float x = ext > 0.0f ? (c - lo) / ext : 0.5f;
    x = fminf(fmaxf(x, 0.0f), 1.0f);
    const uint32_t q = (uint32_t)(x * 2097152.0f);
    return q > 2097151u ? 2097151u : q;
}

__global__ void k_morton(const float *verts, const int32_t *tris, int64_t nt, const uint32_t *valid,
                         const BvhMeta *meta, uint64_t *keys, uint32_t *vals) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nt) return;
    vals[f] = (uint32_t)f;
    if (!valid[f]) {
        keys[f] = ~0ull;
        return;
    }
    const float *a = verts + 3 * (int64_t)tris[3 * f];
    const float *b = verts + 3 * (int64_t)tris[3 * f + 1];
    const float *c = verts + 3 * (int64_t)tris[3 * f + 2];
    uint64_t code = 0;
    for (int k = 0; k < 3; ++k) {
        const float s = (a[k] + b[k]) + c[k];
        const float m = s * (1.0f / 3.0f);
        code |= spread21(quant21(m, meta->bbox[k], meta->bbox[3 + k])) << (2 - k);
    }
    keys[f] = code;
}

// ---------------------------------------------------------------- radix sort
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = TB * RS_ITEMS;

__global__ void k_rs_hist(const uint64_t *keys, int64_t n, int shift, uint32_t *hist, int nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int i = threadIdx.x; i < RS_TILE; i += TB) {
        const int64_t idx = base + i;
        if (idx < n) atomicAdd(&h[(uint32_t)(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: keys of a tile are ranked in index order.  Each round
// handles 256 consecutive keys; inside a wave, peers with the same digit are
// found with eight ballots (one per digit bit).
__global__ void k_rs_scatter(const uint64_t *kin, const uint32_t *vin, uint64_t *kout, uint32_t *vout, int64_t n,
                             int shift, const uint32_t *offs, int nblocks) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[TB / 64][256];
    __shared__ uint32_t boff[256];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    boff[tid] = offs[(int64_t)tid * nblocks + blockIdx.x];
    run[tid] = 0;
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int round = 0; round < RS_ITEMS; ++round) {
        const int64_t idx = base + (int64_t)round * TB + tid;
        const bool ok = idx < n;
        const uint64_t key = ok ? kin[idx] : 0ull;
        const uint32_t val = ok ? vin[idx] : 0u;
        const uint32_t digit = (uint32_t)(key >> shift) & 255u;
        for (int k = tid; k < (TB / 64) * 256; k += TB) (&wcnt[0][0])[k] = 0;
        __syncthreads();
        uint64_t peers = __ballot(ok);
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = (digit >> bit) & 1u;
            const uint64_t bb = __ballot(set);
            peers &= set ? bb : ~bb;
        }
        const uint64_t lower = peers & lt_mask;
        const uint32_t rank = (uint32_t)__popcll(lower);
        if (ok && lower == 0) wcnt[wave][digit] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (ok) {
            uint32_t pre = run[digit];
            for (int w = 0; w < wave; ++w) pre += wcnt[w][digit];
            const uint32_t pos = boff[digit] + pre + rank;
            if (pos < (uint64_t)n) {
                kout[pos] = key;
                vout[pos] = val;
            }
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < TB / 64; ++w) add += wcnt[w][tid];
        run[tid] += add;
        __syncthreads();
    }
}

static hipError_t radix_sort(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n, hipStream_t s,
                             bool *result_in_k1) {
    const int nb = (int)((n + RS_TILE - 1) / RS_TILE);
    uint32_t *hist = nullptr;
    hipError_t e = hipMallocAsync((void **)&hist, sizeof(uint32_t) * 256 * (size_t)nb, s);
    if (e != hipSuccess) return e;
    uint64_t *ka = k0, *kb = k1;
    uint32_t *va = v0, *vb = v1;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 8 * pass;
        k_rs_hist<<<nb, TB, 0, s>>>(ka, n, shift, hist, nb);
        e = scan<uint32_t>(hist, hist, (int64_t)256 * nb, false, s);
        if (e != hipSuccess) break;
        k_rs_scatter<<<nb, TB, 0, s>>>(ka, va, kb, vb, n, shift, hist, nb);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    hipFreeAsync(hist, s);
    *result_in_k1 = (ka == k1);
    if (e == hipSuccess) e = hipGetLastError();
    return e;
}

// ---------------------------------------------------------------- gather
__global__ void k_gather(const float *verts, const int32_t *tris, const uint32_t *sorted_vals, const BvhMeta *meta,
                         float4 *tri4, int32_t *leaf_pos) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= meta->n_valid) return;
    const uint32_t f = sorted_vals[p];
    for (int k = 0; k < 3; ++k) {
        const float *v = verts + 3 * (int64_t)tris[3 * (int64_t)f + k];
        tri4[3 * p + k] = make_float4(v[0], v[1], v[2], __int_as_float((int)f));
    }
    leaf_pos[f] = (int32_t)p;
}

// ---------------------------------------------------------------- Karras
constexpr uint32_t KLEAF = 0x80000000u;

__device__ inline int kdelta(const uint64_t *keys, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    const uint64_t a = keys[i], b = keys[j];
    if (a == b) return 64 + __clz((uint32_t)(i ^ j));
    return __clzll(a ^ b);
}

__global__ void k_karras(const uint64_t *keys, const BvhMeta *meta, int32_t *left, int32_t *right, int32_t *first,
                         int32_t *last, int32_t *parent_int, int32_t *parent_leaf) {
    const int n = meta->n_valid;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (kdelta(keys, n, i, i + 1) - kdelta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = kdelta(keys, n, i, i - d);
    int lmax = 2;
    while (kdelta(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (kdelta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = kdelta(keys, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (kdelta(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int g = i + s * d + (d < 0 ? d : 0);
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    int32_t L, R;
    if (lo == g) {
        L = (int32_t)(KLEAF | (uint32_t)g);
        parent_leaf[g] = i;
    } else {
        L = g;
        parent_int[g] = i;
    }
    if (hi == g + 1) {
        R = (int32_t)(KLEAF | (uint32_t)(g + 1));
        parent_leaf[g + 1] = i;
    } else {
        R = g + 1;
        parent_int[g + 1] = i;
    }
    left[i] = L;
    right[i] = R;
    first[i] = lo;
    last[i] = hi;
    if (i == 0) parent_int[0] = -1;
}

// ---------------------------------------------------------------- refit
__device__ inline void tri_box(const float4 *tri4, int p, float *bx) {
    const float4 a = tri4[3 * p], b = tri4[3 * p + 1], c = tri4[3 * p + 2];
    bx[0] = fminf(fminf(a.x, b.x), c.x);
    bx[1] = fminf(fminf(a.y, b.y), c.y);
    bx[2] = fminf(fminf(a.z, b.z), c.z);
    bx[3] = fmaxf(fmaxf(a.x, b.x), c.x);
    bx[4] = fmaxf(fmaxf(a.y, b.y), c.y);
    bx[5] = fmaxf(fmaxf(a.z, b.z), c.z);
}

__device__ inline void load_box(const float *box_int, int node, float *bx) {
    const uint32_t *src = reinterpret_cast<const uint32_t *>(box_int) + 6 * (int64_t)node;
    for (int k = 0; k < 6; ++k)
        bx[k] = __uint_as_float(__hip_atomic_load(src + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

__device__ inline void child_box(const float4 *tri4, const float *box_int, int32_t c, float *bx) {
    if ((uint32_t)c & KLEAF)
        tri_box(tri4, (int)((uint32_t)c & ~KLEAF), bx);
    else
        load_box(box_int, c, bx);
}

__global__ void k_refit(const float4 *tri4, const int32_t *parent_leaf, const int32_t *parent_int, const int32_t *left,
                        const int32_t *right, float *box_int, uint32_t *flags, const BvhMeta *meta) {
    const int n = meta->n_valid;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n || n < 2) return;
    int node = parent_leaf[p];
    int steps = 0;
    while (node >= 0 && node < n - 1 && ++steps <= n) {
        __threadfence();
        const uint32_t old = atomicAdd(&flags[node], 1u);
        if (old == 0) return;  // the sibling subtree is not done yet
        __threadfence();
        float a[6], b[6];
        child_box(tri4, box_int, left[node], a);
        child_box(tri4, box_int, right[node], b);
        uint32_t *dst = reinterpret_cast<uint32_t *>(box_int) + 6 * (int64_t)node;
        for (int k = 0; k < 3; ++k) {
            __hip_atomic_store(dst + k, __float_as_uint(fminf(a[k], b[k])), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(dst + 3 + k, __float_as_uint(fmaxf(a[3 + k], b[3 + k])), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        node = parent_int[node];
    }
}

// ---------------------------------------------------------------- emit
// Every node slot starts as a sentinel: boxes spanning all space and both
// children 0x7fffffff, an index past any node array.  A traversal that ever
// reaches an unwritten slot steps to that index, which the traversal's
// bounds guard reports as an error instead of reading out of bounds.
constexpr int32_t SENTINEL_CHILD = 0x7fffffff;
__global__ void k_fill_sentinel_nodes(Node *nodes, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float inf = INFINITY;
    Node nd;
    nd.a = make_float4(-inf, -inf, -inf, inf);
    nd.b = make_float4(inf, inf, -inf, -inf);
    nd.c = make_float4(-inf, inf, inf, inf);
    nd.d = make_int4(SENTINEL_CHILD, SENTINEL_CHILD, 0, 0);
    nodes[i] = nd;
}

__global__ void k_emit(const float4 *tri4, const int32_t *left, const int32_t *right, const int32_t *first,
                       const int32_t *last, const int32_t *parent_int, const float *box_int, int leaf_size,
                       Node *nodes, BvhMeta *meta) {
    const int n = meta->n_valid;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) meta->root = (n <= leaf_size) ? leaf_code(0, n) : 0;
    if (i >= n - 1) return;
    if (last[i] - first[i] + 1 <= leaf_size) return;
    float bx[2][6];
    int32_t code[2];
    const int32_t ch[2] = {left[i], right[i]};
    for (int k = 0; k < 2; ++k) {
        const int32_t c = ch[k];
        if ((uint32_t)c & KLEAF) {
            const int p = (int)((uint32_t)c & ~KLEAF);
            tri_box(tri4, p, bx[k]);
            code[k] = leaf_code(p, 1);
        } else {
            load_box(box_int, c, bx[k]);
            const int cnt = last[c] - first[c] + 1;
            code[k] = cnt <= leaf_size ? leaf_code(first[c], cnt) : c;
        }
    }
    Node nd;
    nd.a = make_float4(bx[0][0], bx[0][1], bx[0][2], bx[0][3]);
    nd.b = make_float4(bx[0][4], bx[0][5], bx[1][0], bx[1][1]);
    nd.c = make_float4(bx[1][2], bx[1][3], bx[1][4], bx[1][5]);
    nd.d = make_int4(code[0], code[1], 0, 0);
    nodes[i] = nd;
    atomicAdd(&meta->n_nodes, 1);
    int depth = 1;
    for (int a = parent_int[i]; a >= 0 && a < n - 1 && depth <= n; a = parent_int[a]) ++depth;
    atomicMax(&meta->depth, depth);
}

}  // namespace hra

using namespace hra;

extern "C" hra_status hra_build_bvh(hra_ctx *ctx, const float *d_verts, int64_t n_verts, const int32_t *d_tris,
                                    int64_t n_tris, const hra_bvh_opts *opts, void *stream, hra_bvh **out) {
    if (!ctx || !out) return HRA_ERR_INVALID_ARG;
    *out = nullptr;
    if (!d_verts || !d_tris || n_verts < 3 || n_tris < 1)
        return ctx->fail(HRA_ERR_INVALID_ARG, "mesh needs at least 3 vertices and 1 triangle");
    if (n_tris >= (int64_t)1 << 27 || n_verts >= (int64_t)1 << 31)
        return ctx->fail(HRA_ERR_INVALID_ARG, "mesh too large (max 2^27 triangles)");
    int leaf = opts && opts->leaf_size ? opts->leaf_size : 4;
    if (leaf < 1 || leaf > 8) return ctx->fail(HRA_ERR_INVALID_ARG, "leaf_size must be in 1..8");
    hipStream_t s = (hipStream_t)stream;
    HRA_HIP(hipSetDevice(ctx->device));

    hra_bvh *b = new hra_bvh();
    b->ctx = ctx;
    b->n_tris = n_tris;
    b->n_verts = n_verts;
    b->leaf_size = leaf;
    const int64_t T = n_tris;
    const int64_t nn = T > 1 ? T - 1 : 1;
    size_t bytes = 0;
    auto alloc = [&](void **p, size_t n) -> bool {
        bytes += n;
        return hipMalloc(p, n) == hipSuccess;
    };
    if (!alloc((void **)&b->nodes, sizeof(Node) * nn) || !alloc((void **)&b->tris, sizeof(float4) * 3 * T) ||
        !alloc((void **)&b->leaf_pos, sizeof(int32_t) * T) || !alloc((void **)&b->valid_rank, sizeof(int32_t) * T) ||
        !alloc((void **)&b->prefix, sizeof(uint64_t) * T) || !alloc((void **)&b->meta, sizeof(BvhMeta))) {
        hra_bvh_release(b);
        return ctx->fail(HRA_ERR_OUT_OF_MEMORY, "BVH allocation failed");
    }
    b->bytes = (int64_t)bytes;

    // temporaries, stream ordered
    double *area = nullptr, *partial = nullptr;
    uint32_t *valid = nullptr, *excl = nullptr, *vals0 = nullptr, *vals1 = nullptr, *flags = nullptr;
    uint64_t *w = nullptr, *keys0 = nullptr, *keys1 = nullptr;
    int32_t *L = nullptr, *R = nullptr, *F = nullptr, *La = nullptr, *PI = nullptr, *PL = nullptr;
    float *box = nullptr;
    hipError_t e = hipSuccess;
#define TMP(p, n)                                                   \
    if (e == hipSuccess) e = hipMallocAsync((void **)&(p), (n), s);
    TMP(area, sizeof(double) * T);
    TMP(partial, sizeof(double) * 7 * RED_BLOCKS);
    TMP(valid, sizeof(uint32_t) * T);
    TMP(excl, sizeof(uint32_t) * T);
    TMP(w, sizeof(uint64_t) * T);
    TMP(keys0, sizeof(uint64_t) * T);
    TMP(keys1, sizeof(uint64_t) * T);
    TMP(vals0, sizeof(uint32_t) * T);
    TMP(vals1, sizeof(uint32_t) * T);
    TMP(L, sizeof(int32_t) * nn);
    TMP(R, sizeof(int32_t) * nn);
    TMP(F, sizeof(int32_t) * nn);
    TMP(La, sizeof(int32_t) * nn);
    TMP(PI, sizeof(int32_t) * nn);
    TMP(PL, sizeof(int32_t) * T);
    TMP(flags, sizeof(uint32_t) * nn);
    TMP(box, sizeof(float) * 6 * nn);
#undef TMP
    if (e == hipSuccess) {
        const int gT = blocks_for(T, TB), gN = blocks_for(nn, TB);
        int rb = blocks_for(std::max(n_verts, T), TB);
        rb = std::min(rb, RED_BLOCKS);
        k_fill_i32<<<gT, TB, 0, s>>>(b->leaf_pos, T, -1);
        k_fill_sentinel_nodes<<<gN, TB, 0, s>>>(b->nodes, nn);
        k_fill_u32<<<gN, TB, 0, s>>>(flags, nn, 0u);
        k_fill_i32<<<gN, TB, 0, s>>>(PI, nn, -1);
        k_tri_prep<<<gT, TB, 0, s>>>(d_verts, n_verts, d_tris, T, area, valid, ctx->d_err);
        k_reduce_partial<<<rb, TB, 0, s>>>(d_verts, n_verts, area, T, partial);
        k_reduce_final<<<1, 64, 0, s>>>(partial, rb, T, b->meta);
        k_weights<<<gT, TB, 0, s>>>(area, T, b->meta, w);
        e = scan<uint64_t>(w, b->prefix, T, true, s);
        if (e == hipSuccess) e = scan<uint32_t>(valid, excl, T, false, s);
        if (e == hipSuccess) {
            k_ranks<<<gT, TB, 0, s>>>(valid, excl, T, b->valid_rank, b->prefix, b->meta, ctx->d_err);
            k_morton<<<gT, TB, 0, s>>>(d_verts, d_tris, T, valid, b->meta, keys0, vals0);
            bool in1 = false;
            e = radix_sort(keys0, vals0, keys1, vals1, T, s, &in1);
            uint64_t *ks = in1 ? keys1 : keys0;
            uint32_t *vs = in1 ? vals1 : vals0;
            if (e == hipSuccess) {
                k_gather<<<gT, TB, 0, s>>>(d_verts, d_tris, vs, b->meta, b->tris, b->leaf_pos);
                k_karras<<<gN, TB, 0, s>>>(ks, b->meta, L, R, F, La, PI, PL);
                k_refit<<<gT, TB, 0, s>>>(b->tris, PL, PI, L, R, box, flags, b->meta);
                k_emit<<<gN, TB, 0, s>>>(b->tris, L, R, F, La, PI, box, leaf, b->nodes, b->meta);
                e = hipGetLastError();
            }
        }
    }
    for (void *p : {(void *)area, (void *)partial, (void *)valid, (void *)excl, (void *)w, (void *)keys0,
                    (void *)keys1, (void *)vals0, (void *)vals1, (void *)L, (void *)R, (void *)F, (void *)La,
                    (void *)PI, (void *)PL, (void *)flags, (void *)box})
        if (p) hipFreeAsync(p, s);
    if (e != hipSuccess) {
        hipStreamSynchronize(s);
        hra_bvh_release(b);
        return ctx->fail(HRA_ERR_DEVICE, "BVH build launch failed", hipGetErrorString(e));
    }
    *out = b;
    return HRA_OK;
}

extern "C" hra_status hra_bvh_get_info(hra_bvh *b, void *stream, hra_bvh_info *out) {
    if (!b || !out) return HRA_ERR_INVALID_ARG;
    hra_ctx *ctx = b->ctx;
    hra_status st = check_error_word(ctx, (hipStream_t)stream);
    if (st != HRA_OK) return st;
    BvhMeta m;
    HRA_HIP(hipMemcpy(&m, b->meta, sizeof(m), hipMemcpyDeviceToHost));
    for (int k = 0; k < 6; ++k) out->bbox[k] = m.bbox[k];
    out->diag = m.diag;
    out->n_tris = b->n_tris;
    out->n_degenerate = b->n_tris - m.n_valid;
    out->n_nodes = m.n_nodes;
    out->bytes = b->bytes;
    out->depth = m.depth;
    out->leaf_size = b->leaf_size;
    return HRA_OK;
}

extern "C" hra_status hra_bvh_export(hra_bvh *b, void *stream, void *host_nodes, void *host_tris, int32_t *root,
                                     int32_t *n_valid) {
    if (!b || !host_nodes || !host_tris || !root || !n_valid) return HRA_ERR_INVALID_ARG;
    hra_ctx *ctx = b->ctx;
    hra_status st = check_error_word(ctx, (hipStream_t)stream);
    if (st != HRA_OK) return st;
    BvhMeta m;
    HRA_HIP(hipMemcpy(&m, b->meta, sizeof(m), hipMemcpyDeviceToHost));
    const int64_t nn = b->n_tris > 1 ? b->n_tris - 1 : 1;
    HRA_HIP(hipMemcpy(host_nodes, b->nodes, sizeof(Node) * nn, hipMemcpyDeviceToHost));
    HRA_HIP(hipMemcpy(host_tris, b->tris, sizeof(float4) * 3 * b->n_tris, hipMemcpyDeviceToHost));
    *root = m.root;
    *n_valid = m.n_valid;
    return HRA_OK;
}

extern "C" void hra_bvh_release(hra_bvh *b) {
    if (!b) return;
    if (b->ctx) hipSetDevice(b->ctx->device);
    hipFree(b->nodes);
    hipFree(b->tris);
    hipFree(b->leaf_pos);
    hipFree(b->valid_rank);
    hipFree(b->prefix);
    hipFree(b->meta);
    delete b;
}

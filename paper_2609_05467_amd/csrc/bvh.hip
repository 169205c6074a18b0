// Mesh ingest and LBVH construction for one or many parts at once, all on
// the device.
//
// Every part's triangles are concatenated; a 64-bit key puts the part index
// in the top 8 bits and a 54-bit Morton code (18 bits per axis, in the part's
// own bounding box) below, so one global sort lays every part out as a
// contiguous run, and in the binary radix tree over the sorted keys each
// run is exactly one subtree (the keys of a part share its 8-bit prefix, so
// their lowest common ancestor holds no other key).  Traversal of part p
// starts at that subtree's root; nodes spanning two parts are never used.
//
// Stages (one stream, no host round trip):
//   1. per-triangle prep: part lookup, index check, FP64 doubled area
//      squared, area, nonzero-area flag, a copy of the three vertices;
//   2. per-part vertex bbox and largest area (a 2D grid of blocks per part,
//      exact atomic min/max), then diagonal and weight scale;
//   3. integer area weights, their global inclusive prefix (the sampler
//      searches a part's range), ranks of nonzero-area faces;
//   4. keys (part, Morton of the centroid); zero-area faces get the
//      largest key;
//   5. LSD radix sort, 8 passes of 8 bits, LDS digit counts and a stable
//      LDS-ranked scatter;
//   6. binary radix tree over the sorted keys (Karras, "Maximizing
//      Parallelism in the Construction of BVHs, Octrees, and k-d Trees", HPG
//      2012), ties between equal keys broken by position within the part;
//      part roots;
//   7. bottom-up box refit: the second thread to reach a node merges it and
//      records its height;
//   8. leaf collapse (subtrees of one part with <= leaf_size triangles become
//      one leaf over a contiguous run) and emission of 64-byte nodes; node
//      counts per part and each part's depth (its root's height).
#include "common.hpp"
#include "prims.hpp"

#include <algorithm>
#include <vector>

namespace hra {

constexpr int TB = 256;

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

// Elements of scratch a scan of n elements needs (block sums, recursively).
static int64_t scan_ws_elems(int64_t n) {
    if (n <= SCAN_TILE) return 0;
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    return nb + scan_ws_elems(nb);
}

// Exclusive or inclusive prefix sum; `ws` holds scan_ws_elems(n) elements.
template <typename T>
static hipError_t scan(const T *in, T *out, int64_t n, bool inclusive, T *ws, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        k_scan_tile<T><<<1, TB, 0, s>>>(in, out, n, (T *)nullptr, inclusive ? 1 : 0);
        return hipGetLastError();
    }
    T *sums = ws;
    k_scan_tile<T><<<(unsigned)nb, TB, 0, s>>>(in, out, n, sums, inclusive ? 1 : 0);
    hipError_t e = scan<T>(sums, sums, nb, false, ws + nb, s);
    if (e == hipSuccess) {
        k_scan_add<T><<<(unsigned)nb, TB, 0, s>>>(out, n, sums);
        e = hipGetLastError();
    }
    return e;
}

// ---------------------------------------------------------------- ingest
// Part of global triangle g: the last part whose tri_start <= g.
__device__ inline int part_of(const MeshIn *mesh, int n_parts, int64_t g) {
    int lo = 0, hi = n_parts - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (mesh[mid].tri_start <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

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

// tv: the triangle's three vertices (9 floats), tpart: its part.
__global__ void k_tri_prep(const MeshIn *mesh, int n_parts, int64_t T, double *area, uint32_t *valid, float *tv,
                           uint8_t *tpart, uint32_t *err) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= T) return;
    const int p = part_of(mesh, n_parts, g);
    const MeshIn m = mesh[p];
    const int64_t f = g - m.tri_start;
    tpart[g] = (uint8_t)p;
    const int32_t i0 = m.t[3 * f], i1 = m.t[3 * f + 1], i2 = m.t[3 * f + 2];
    if (i0 < 0 || i1 < 0 || i2 < 0 || i0 >= m.nv || i1 >= m.nv || i2 >= m.nv) {
        atomicOr(err, ERR_BAD_INDEX);
        area[g] = 0.0;
        valid[g] = 0;
        for (int k = 0; k < 9; ++k) tv[9 * g + k] = 0.0f;
        return;
    }
    const float *a = m.v + 3 * (int64_t)i0, *b = m.v + 3 * (int64_t)i1, *c = m.v + 3 * (int64_t)i2;
    for (int k = 0; k < 3; ++k) {
        tv[9 * g + k] = a[k];
        tv[9 * g + 3 + k] = b[k];
        tv[9 * g + 6 + k] = c[k];
    }
    const double q = tri_q64(a, b, c);
    const bool ok = q > 0.0;
    area[g] = ok ? 0.5 * sqrt(q) : 0.0;
    valid[g] = ok ? 1u : 0u;
}

// Per-part facts from many blocks at once: blocks (b, p) of a 2D grid take
// slices of part p's vertices and triangles and fold their bounding box and
// largest area into per-part accumulators with atomics (exact: min, max).
// Floats are folded as order-preserving unsigned keys.
struct PartAcc {
    uint32_t lo[3], hi[3];   // ordered keys of the vertex bbox
    unsigned long long amax; // bits of the largest area (non-negative double)
    int32_t pad[2];
};
constexpr int FACT_BLOCKS = 64;

__device__ inline uint32_t fkey(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float fkey_inv(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__global__ void k_part_facts(const MeshIn *mesh, const double *area, PartAcc *acc) {
    __shared__ uint32_t slo[3], shi[3];
    __shared__ unsigned long long samax;
    const int p = blockIdx.y, t = threadIdx.x;
    const MeshIn m = mesh[p];
    if (t < 3) {
        slo[t] = 0xffffffffu;
        shi[t] = 0u;
    }
    if (t == 0) samax = 0ull;
    __syncthreads();
    const int64_t vchunk = (m.nv + FACT_BLOCKS - 1) / FACT_BLOCKS, tchunk = (m.nt + FACT_BLOCKS - 1) / FACT_BLOCKS;
    const int64_t v0 = blockIdx.x * vchunk, v1 = v0 + vchunk < m.nv ? v0 + vchunk : m.nv;
    const int64_t t0 = blockIdx.x * tchunk, t1 = t0 + tchunk < m.nt ? t0 + tchunk : m.nt;
    uint32_t lo[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, hi[3] = {0u, 0u, 0u};
    for (int64_t i = v0 + t; i < v1; i += blockDim.x)
        for (int c = 0; c < 3; ++c) {
            const uint32_t k = fkey(m.v[3 * i + c]);
            lo[c] = k < lo[c] ? k : lo[c];
            hi[c] = k > hi[c] ? k : hi[c];
        }
    unsigned long long am = 0ull;
    for (int64_t i = t0 + t; i < t1; i += blockDim.x) {
        const unsigned long long b = (unsigned long long)__double_as_longlong(area[m.tri_start + i]);
        am = b > am ? b : am;
    }
    for (int c = 0; c < 3; ++c) {
        atomicMin(&slo[c], lo[c]);
        atomicMax(&shi[c], hi[c]);
    }
    atomicMax(&samax, am);
    __syncthreads();
    if (t < 3) {
        atomicMin(&acc[p].lo[t], slo[t]);
        atomicMax(&acc[p].hi[t], shi[t]);
    }
    if (t == 0) atomicMax(&acc[p].amax, samax);
}

// One thread per part: bbox, diagonal, largest area and the weight scale
// k = 54 - (ilogb(amax) + 1) - bitlen(n_tris), which keeps each part's weight
// sum below 2^54 and the sum over up to 1024 parts below 2^64.
__global__ void k_part_finalize(const MeshIn *mesh, const PartAcc *acc, int n_parts, PartMeta *meta) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_parts) return;
    const MeshIn m = mesh[p];
    const PartAcc &A = acc[p];
    PartMeta &P = meta[p];
    double lo[3], hi[3];
    for (int c = 0; c < 3; ++c) {
        lo[c] = fkey_inv(A.lo[c]);
        hi[c] = fkey_inv(A.hi[c]);
        P.bbox[c] = (float)lo[c];
        P.bbox[3 + c] = (float)hi[c];
    }
    const double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    const double sx = dx * dx, sy = dy * dy, sz = dz * dz;
    const double sxy = sx + sy;
    P.diag = sqrt(sxy + sz);
    P.amax = __longlong_as_double((long long)A.amax);
    int tb = 0;
    while (tb < 63 && ((int64_t)1 << tb) <= m.nt) ++tb;
    P.k_scale = P.amax > 0.0 ? 54 - (ilogb(P.amax) + 1) - tb : 0;
    P.tri_start = m.tri_start;
    P.n_tris = (int32_t)m.nt;
    P.n_verts = m.nv;
    P.root = 0;
    P.depth = 0;
    P.n_nodes = 0;
}

__global__ void k_weights(const double *area, const uint8_t *tpart, int64_t T, const PartMeta *meta, uint64_t *w) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= T) return;
    w[g] = (uint64_t)floor(ldexp(area[g], meta[tpart[g]].k_scale));
}

// Per part: weight base and total, nonzero-area count, first leaf position.
// Single thread: at most MAX_PARTS parts.
__global__ void k_part_counts(const uint64_t *prefix, const uint32_t *excl, const uint32_t *valid, int n_parts,
                              int64_t T, PartMeta *meta, int32_t *n_valid_total, uint32_t *err) {
    if (threadIdx.x != 0) return;
    int32_t leaf = 0;
    for (int p = 0; p < n_parts; ++p) {
        PartMeta &P = meta[p];
        const int64_t a = P.tri_start, b = P.tri_start + P.n_tris;
        P.base_w = a > 0 ? prefix[a - 1] : 0;
        P.total_w = prefix[b - 1] - P.base_w;
        const uint32_t ea = excl[a], eb = b < T ? excl[b] : excl[T - 1] + valid[T - 1];
        P.n_valid = (int32_t)(eb - ea);
        P.leaf_lo = leaf;
        leaf += P.n_valid;
        if (P.n_valid == 0) atomicOr(err, ERR_EMPTY_MESH);
    }
    *n_valid_total = leaf;
}

// ---------------------------------------------------------------- keys
__device__ inline uint64_t spread18(uint32_t x) {
    uint64_t v = x & 0x3FFFFu;
    v = (v | (v << 32)) & 0x001F00000000FFFFull;
    v = (v | (v << 16)) & 0x001F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ inline uint32_t quant18(float c, float lo, float hi) {
    const float ext = hi - lo;
    float x = ext > 0.0f ? (c - lo) / ext : 0.5f;
    x = fminf(fmaxf(x, 0.0f), 1.0f);
    const uint32_t q = (uint32_t)(x * 262144.0f);
    return q > 262143u ? 262143u : q;
}

// Per triangle: its rank among its part's nonzero-area faces (-1 for a
// zero-area one) and its sort key and index.
__global__ void k_ranks_keys(const uint32_t *valid, const uint32_t *excl, const float *tv, const uint8_t *tpart,
                             int64_t T, const PartMeta *meta, int32_t *rank, uint64_t *keys, uint32_t *vals) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= T) return;
    rank[g] = valid[g] ? (int32_t)(excl[g] - excl[meta[tpart[g]].tri_start]) : -1;
    vals[g] = (uint32_t)g;
    if (!valid[g]) {
        keys[g] = ~0ull;
        return;
    }
    const int p = tpart[g];
    const PartMeta &P = meta[p];
    const float *v = tv + 9 * g;
    uint64_t code = 0;
    for (int k = 0; k < 3; ++k) {
        const float s = (v[k] + v[3 + k]) + v[6 + k];
        const float m = s * (1.0f / 3.0f);
        code |= spread18(quant18(m, P.bbox[k], P.bbox[3 + k])) << (2 - k);
    }
    keys[g] = ((uint64_t)p << 56) | code;
}

// ---------------------------------------------------------------- radix sort
// Keys per workgroup: TB x items.  Large tiles keep the digit histogram
// (256 counters per tile) and its scan small; small tiles give a short
// sort enough workgroups to fill the device (204.5k keys in 4096-key tiles
// made 50 workgroups, each running 16 rounds of barriers).
__host__ __device__ inline int rs_items(int64_t n) {
    return n >= ((int64_t)4 << 20) ? 16 : (n >= ((int64_t)1 << 20) ? 8 : (n >= ((int64_t)1 << 18) ? 4 : 2));
}

__global__ void k_rs_hist(const uint64_t *keys, int64_t n, int shift, uint32_t *hist, int nblocks, int items) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int tile = TB * items;
    const int64_t base = (int64_t)blockIdx.x * tile;
    for (int i = threadIdx.x; i < tile; i += TB) {
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
                             int shift, const uint32_t *offs, int nblocks, int items, const uint32_t *totals) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[TB / 64][256];
    __shared__ uint32_t boff[256];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    // this block's first position per digit: the keys of lower digits (an
    // exclusive scan of the digit totals) plus this digit's keys in earlier
    // blocks (k_rs_digit_scan)
    run[tid] = totals[tid];
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t v = tid >= off ? run[tid - off] : 0u;
        __syncthreads();
        run[tid] += v;
        __syncthreads();
    }
    boff[tid] = (tid > 0 ? run[tid - 1] : 0u) + offs[(int64_t)tid * nblocks + blockIdx.x];
    __syncthreads();
    run[tid] = 0;
    const int64_t base = (int64_t)blockIdx.x * TB * items;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int round = 0; round < items; ++round) {
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

// Exclusive prefix over the blocks of each digit's counts, in place
// (digit-major layout hist[d * nb + b]); one workgroup per digit, which also
// writes the digit's total.
__global__ __launch_bounds__(TB) void k_rs_digit_scan(uint32_t *hist, int nb, uint32_t *totals) {
    __shared__ uint32_t part[TB];
    uint32_t *h = hist + (int64_t)blockIdx.x * nb;
    const int t = threadIdx.x;
    const int per = (nb + TB - 1) / TB;
    const int b0 = min(t * per, nb), b1 = min(b0 + per, nb);
    uint32_t sum = 0;
    for (int b = b0; b < b1; ++b) sum += h[b];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < TB; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t acc = t > 0 ? part[t - 1] : 0u;
    for (int b = b0; b < b1; ++b) {
        const uint32_t c = h[b];
        h[b] = acc;
        acc += c;
    }
    if (t == TB - 1) totals[blockIdx.x] = part[TB - 1];
}

static_assert(TB == 256, "one thread per digit in the radix sort");

static int64_t radix_ws_elems(int64_t n) {
    const int64_t tile = (int64_t)TB * rs_items(n);
    const int64_t nb = (n + tile - 1) / tile;
    return 256 * nb + 256;
}

// `ws` holds radix_ws_elems(n) uint32 elements.  The keys are ordered by
// their low 8 x passes bits (three launches per pass).
static hipError_t radix_sort(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n, uint32_t *ws,
                             hipStream_t s, bool *result_in_k1, int passes = 8) {
    const int items = rs_items(n);
    const int64_t tile = (int64_t)TB * items;
    const int nb = (int)((n + tile - 1) / tile);
    uint32_t *hist = ws, *totals = ws + 256 * (int64_t)nb;
    uint64_t *ka = k0, *kb = k1;
    uint32_t *va = v0, *vb = v1;
    hipError_t e = hipSuccess;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = 8 * pass;
        k_rs_hist<<<nb, TB, 0, s>>>(ka, n, shift, hist, nb, items);
        k_rs_digit_scan<<<256, TB, 0, s>>>(hist, nb, totals);
        k_rs_scatter<<<nb, TB, 0, s>>>(ka, va, kb, vb, n, shift, hist, nb, items, totals);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    *result_in_k1 = (ka == k1);
    if (e == hipSuccess) e = hipGetLastError();
    return e;
}

// ---------------------------------------------------------------- gather
__global__ void k_gather(const float *tv, const uint32_t *sorted_vals, const uint8_t *tpart, const PartMeta *meta,
                         const int32_t *n_valid_total, float4 *tri4, int32_t *leaf_pos) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= *n_valid_total) return;
    const uint32_t g = sorted_vals[q];
    const int32_t f = (int32_t)(g - meta[tpart[g]].tri_start);   // face index within its part
    const float *v = tv + 9 * (int64_t)g;
    for (int k = 0; k < 3; ++k) tri4[3 * q + k] = make_float4(v[3 * k], v[3 * k + 1], v[3 * k + 2], __int_as_float(f));
    leaf_pos[g] = (int32_t)q;
}

// The sort and the scan for other translation units (declared in prims.hpp).
int64_t sort_pairs_ws_elems(int64_t n) { return radix_ws_elems(n); }
hipError_t sort_pairs(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n, uint32_t *ws, hipStream_t s,
                      bool *result_in_k1, int passes) {
    return radix_sort(k0, v0, k1, v1, n, ws, s, result_in_k1, passes);
}
int64_t scan_u32_ws_elems(int64_t n) { return scan_ws_elems(n); }
hipError_t scan_u32(const uint32_t *in, uint32_t *out, int64_t n, bool inclusive, uint32_t *ws, hipStream_t s) {
    return scan<uint32_t>(in, out, n, inclusive, ws, s);
}

// ---------------------------------------------------------------- Karras
constexpr uint32_t KLEAF = 0x80000000u;

// Common-prefix length of keys i and j (-1 outside [0, n)).  Equal keys
// (same part, same cell) fall back to the indices within the part, so a
// part's subtree is the same whether it is built alone or in a batch.
__device__ inline int kdelta(const uint64_t *keys, const PartMeta *meta, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    const uint64_t a = keys[i], b = keys[j];
    if (a == b) {
        const int s = meta[a >> 56].leaf_lo;
        return 64 + __clz((uint32_t)((i - s) ^ (j - s)));
    }
    return __clzll(a ^ b);
}

__global__ void k_karras(const uint64_t *keys, const int32_t *n_valid_total, int32_t *left, int32_t *right,
                         int32_t *first, int32_t *last, int32_t *parent_int, int32_t *parent_leaf, PartMeta *meta) {
    const int n = *n_valid_total;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (kdelta(keys, meta, n, i, i + 1) - kdelta(keys, meta, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = kdelta(keys, meta, n, i, i - d);
    int lmax = 2;
    while (kdelta(keys, meta, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (kdelta(keys, meta, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = kdelta(keys, meta, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (kdelta(keys, meta, n, i, i + (s + t) * d) > dnode) s += t;
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
    // the node holding exactly one part's run is that part's subtree root
    const int p = (int)(keys[lo] >> 56);
    if ((int)(keys[hi] >> 56) == p && keys[lo] != ~0ull) {
        PartMeta &P = meta[p];
        if (lo == P.leaf_lo && hi == P.leaf_lo + P.n_valid - 1) P.root = i;
    }
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

// Bottom-up box refit: each leaf's thread walks towards the root; at every
// node the first arrival stops and the second (which then sees both
// children done) merges the boxes and goes on.  The same walk records each
// node's height in emitted interior nodes (a node whose subtree holds at
// most leaf_size triangles becomes a leaf: height 0).
//
// Publication between the two children's threads, which may run on
// different compute dies with separate L2 caches: every box and height
// this kernel shares is written and read with agent-scope atomic stores and
// loads, which the compiler issues as device-coherent accesses (they do not
// hit a die's own L2 copy).  A thread waits until all its earlier memory
// operations have completed (s_waitcnt 0) before it increments the node's
// counter, so the box and height it wrote are visible device-wide before
// its sibling can see the increment; the sibling's loads come after the
// increment's returned value (control dependence, in-order issue).  An
// acquire-release increment would order the same accesses, but it also
// writes back and invalidates the whole L2 at every step (about six times
// slower for the whole build); nothing here needs that, since no plain
// (L2-cached) store is shared.  The compiler fences keep the shared
// accesses on their side of the increment.
// Relative costs of the traversal's two units of work for the collapse
// decision: one interior-node visit (both child boxes) and one ray-triangle
// test, in VALU operations.
constexpr float SAH_NODE = 50.0f, SAH_TRI = 54.0f;

__device__ inline float half_area(const float *bx) {
    const float dx = bx[3] - bx[0], dy = bx[4] - bx[1], dz = bx[5] - bx[2];
    return (dx * dy + dy * dz) + dz * dx;
}

__device__ inline float child_cost(const float4 *tri4, const float *cost, int32_t c) {
    if ((uint32_t)c & KLEAF) {
        float bx[6];
        tri_box(tri4, (int)((uint32_t)c & ~KLEAF), bx);
        return SAH_TRI * half_area(bx);
    }
    return __uint_as_float(__hip_atomic_load(reinterpret_cast<const uint32_t *>(cost) + c, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT));
}

__global__ void k_refit(const float4 *tri4, const uint64_t *keys, const int32_t *parent_leaf, const int32_t *parent_int,
                        const int32_t *left, const int32_t *right, const int32_t *first, const int32_t *last,
                        int leaf_size, float *box_int, float *cost, int32_t *leafy, int32_t *height, uint32_t *flags,
                        const int32_t *n_valid_total) {
    const int n = *n_valid_total;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n || n < 2) return;
    int node = parent_leaf[p];
    int steps = 0;
    while (node >= 0 && node < n - 1 && ++steps <= n) {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        const uint32_t old = __hip_atomic_fetch_add(&flags[node], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (old == 0) return;  // the sibling subtree is not done yet
        float a[6], b[6], u[6];
        const int32_t l = left[node], r = right[node];
        child_box(tri4, box_int, l, a);
        child_box(tri4, box_int, r, b);
        uint32_t *dst = reinterpret_cast<uint32_t *>(box_int) + 6 * (int64_t)node;
        for (int k = 0; k < 3; ++k) {
            u[k] = fminf(a[k], b[k]);
            u[3 + k] = fmaxf(a[3 + k], b[3 + k]);
            __hip_atomic_store(dst + k, __float_as_uint(u[k]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(dst + 3 + k, __float_as_uint(u[3 + k]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // Surface-area cost: a subtree of at most leaf_size triangles (all of
        // one part) becomes a single leaf when testing its triangles costs
        // less than traversing it.
        const int cnt = last[node] - first[node] + 1;
        const float A = half_area(u);
        const float keep = (SAH_NODE * A + child_cost(tri4, cost, l)) + child_cost(tri4, cost, r);
        const float as_leaf = (SAH_TRI * (float)cnt) * A;
        const bool one_part = (keys[first[node]] >> 56) == (keys[last[node]] >> 56);
        const bool col = cnt <= leaf_size && one_part && as_leaf <= keep;
        __hip_atomic_store(reinterpret_cast<uint32_t *>(cost) + node, __float_as_uint(col ? as_leaf : keep),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(leafy + node, col ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int h = 0;
        if (!col) {
            const int hl = ((uint32_t)l & KLEAF) ? 0 : __hip_atomic_load(height + l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int hr = ((uint32_t)r & KLEAF) ? 0 : __hip_atomic_load(height + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            h = 1 + (hl > hr ? hl : hr);
        }
        __hip_atomic_store(height + node, h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        node = parent_int[node];
    }
}

// ---------------------------------------------------------------- emit
// Every node slot starts as a sentinel: boxes spanning all space and both
// children 0x7fffffff, an index past any node array.  A traversal that ever
// reaches an unwritten slot steps to that index, which the traversal's
// bounds guard reports as an error instead of reading out of bounds.
constexpr int32_t SENTINEL_CHILD = 0x7fffffff;
// Every fill a build starts with, in one launch: leaf positions -1,
// sentinel nodes, cleared refit counters, parent indices -1 and the per-part
// accumulators of k_part_facts.
__global__ void k_build_init(int32_t *leaf_pos, int64_t T, Node *nodes, uint32_t *flags, int32_t *PI, int64_t nn,
                             PartAcc *acc, int n_parts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < T) leaf_pos[i] = -1;
    if (i < nn) {
        const float inf = INFINITY;
        Node nd;
        nd.a = make_float4(-inf, -inf, -inf, inf);
        nd.b = make_float4(inf, inf, -inf, -inf);
        nd.c = make_float4(-inf, inf, inf, inf);
        nd.d = make_int4(SENTINEL_CHILD, SENTINEL_CHILD, 0, 0);
        nodes[i] = nd;
        flags[i] = 0u;
        PI[i] = -1;
    }
    if (i < n_parts) {
        for (int c = 0; c < 3; ++c) {
            acc[i].lo[c] = 0xffffffffu;
            acc[i].hi[c] = 0u;
        }
        acc[i].amax = 0ull;
    }
}

// Roots of parts too small for an interior node of their own: one leaf.
__global__ void k_small_roots(PartMeta *meta, int n_parts, int leaf_size) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_parts) return;
    PartMeta &P = meta[p];
    if (P.n_valid >= 1 && P.n_valid <= leaf_size) P.root = leaf_code(P.leaf_lo, P.n_valid);
}

__global__ void k_emit(const float4 *tri4, const uint64_t *keys, const int32_t *left, const int32_t *right,
                       const int32_t *first, const int32_t *last, const int32_t *parent_int, const int32_t *leafy,
                       const float *box_int, int leaf_size, const int32_t *n_valid_total, Node *nodes,
                       uint8_t *emitted) {
    const int n = *n_valid_total;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    emitted[i] = 0;
    if (last[i] - first[i] + 1 <= leaf_size) {
        // inside a collapsed subtree (this node, or an ancestor of at most
        // leaf_size triangles that became the leaf) it is not a node at all
        if (leafy[i]) return;
        for (int p = parent_int[i], g = 0; p >= 0 && g < 16; p = parent_int[p], ++g) {
            if (last[p] - first[p] + 1 > leaf_size) break;
            if (leafy[p]) return;
        }
    }
    const int p = (int)(keys[first[i]] >> 56);
    if ((int)(keys[last[i]] >> 56) != p) return;   // spans two parts: never traversed
    float bx[2][6];
    int32_t code[2];
    const int32_t ch[2] = {left[i], right[i]};
    for (int k = 0; k < 2; ++k) {
        const int32_t c = ch[k];
        if ((uint32_t)c & KLEAF) {
            const int q = (int)((uint32_t)c & ~KLEAF);
            tri_box(tri4, q, bx[k]);
            code[k] = leaf_code(q, 1);
        } else {
            load_box(box_int, c, bx[k]);
            code[k] = leafy[c] ? leaf_code(first[c], last[c] - first[c] + 1) : c;
        }
    }
    Node nd;
    nd.a = make_float4(bx[0][0], bx[0][1], bx[0][2], bx[0][3]);
    nd.b = make_float4(bx[0][4], bx[0][5], bx[1][0], bx[1][1]);
    nd.c = make_float4(bx[1][2], bx[1][3], bx[1][4], bx[1][5]);
    nd.d = make_int4(code[0], code[1], 0, 0);
    nodes[i] = nd;
    emitted[i] = 1;
}

// Interior nodes and depth of every part.  In the radix tree each internal
// node's index is an end of its key range, so part p's interior nodes have
// indices in [leaf_lo, leaf_lo + n_valid - 1]; the other indices there
// belong to nodes spanning two parts, which are never emitted.  Blocks (b,
// p) count slices of that range; the depth is the root's height.
__global__ void k_part_nodes(const uint8_t *emitted, const int32_t *height, const int32_t *n_valid_total,
                             PartMeta *meta) {
    __shared__ int cnt;
    const int p = blockIdx.y, t = threadIdx.x;
    const int n = *n_valid_total;
    PartMeta &P = meta[p];
    if (t == 0) cnt = 0;
    __syncthreads();
    const int64_t a = P.leaf_lo;
    int64_t b = (int64_t)P.leaf_lo + P.n_valid;   // exclusive
    if (b > n - 1) b = n - 1;
    const int64_t len = b > a ? b - a : 0;
    const int64_t chunk = (len + FACT_BLOCKS - 1) / FACT_BLOCKS;
    const int64_t c0 = a + blockIdx.x * chunk, c1 = c0 + chunk < b ? c0 + chunk : b;
    int c = 0;
    for (int64_t i = c0 + t; i < c1; i += blockDim.x) c += emitted[i];
    if (c) atomicAdd(&cnt, c);
    __syncthreads();
    if (t == 0 && cnt) atomicAdd(&P.n_nodes, cnt);
    if (t == 0 && blockIdx.x == 0) P.depth = is_leaf(P.root) || P.n_valid < 2 ? 0 : height[P.root];
}

}  // namespace hra

using namespace hra;

namespace hra {

// Scratch of one build, carved from one allocation (256-byte aligned
// pieces), so a build can run in memory the caller set aside (graphs).
struct BuildWs {
    MeshIn *mesh;
    double *area;
    uint32_t *valid, *excl, *vals0, *vals1, *flags, *rs_ws;
    uint64_t *w, *keys0, *keys1, *scan64_ws;
    uint32_t *scan32_ws;
    int32_t *L, *R, *F, *La, *PI, *PL, *nvt, *height, *leafy;
    float *box, *tv, *cost;
    uint8_t *tpart, *emitted;
    PartAcc *acc;
};

static size_t carve(char *base, int64_t T, int n_parts, BuildWs *w) {
    const int64_t nn = T > 1 ? T - 1 : 1;
    size_t off = 0;
    auto take = [&](void **p, size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        if (base) *p = base + off;
        off += bytes;
    };
    BuildWs d;
    take((void **)&d.mesh, sizeof(MeshIn) * n_parts);
    take((void **)&d.area, sizeof(double) * T);
    take((void **)&d.valid, sizeof(uint32_t) * T);
    take((void **)&d.excl, sizeof(uint32_t) * T);
    take((void **)&d.w, sizeof(uint64_t) * T);
    take((void **)&d.keys0, sizeof(uint64_t) * T);
    take((void **)&d.keys1, sizeof(uint64_t) * T);
    take((void **)&d.vals0, sizeof(uint32_t) * T);
    take((void **)&d.vals1, sizeof(uint32_t) * T);
    take((void **)&d.tv, sizeof(float) * 9 * T);
    take((void **)&d.tpart, sizeof(uint8_t) * T);
    take((void **)&d.L, sizeof(int32_t) * nn);
    take((void **)&d.R, sizeof(int32_t) * nn);
    take((void **)&d.F, sizeof(int32_t) * nn);
    take((void **)&d.La, sizeof(int32_t) * nn);
    take((void **)&d.PI, sizeof(int32_t) * nn);
    take((void **)&d.PL, sizeof(int32_t) * T);
    take((void **)&d.flags, sizeof(uint32_t) * nn);
    take((void **)&d.box, sizeof(float) * 6 * nn);
    take((void **)&d.height, sizeof(int32_t) * nn);
    take((void **)&d.leafy, sizeof(int32_t) * nn);
    take((void **)&d.cost, sizeof(float) * nn);
    take((void **)&d.emitted, sizeof(uint8_t) * nn);
    take((void **)&d.acc, sizeof(PartAcc) * n_parts);
    take((void **)&d.nvt, sizeof(int32_t));
    take((void **)&d.scan64_ws, sizeof(uint64_t) * (scan_ws_elems(T) + 1));
    take((void **)&d.scan32_ws, sizeof(uint32_t) * (scan_ws_elems(T) + 1));
    take((void **)&d.rs_ws, sizeof(uint32_t) * radix_ws_elems(T));
    if (w) *w = d;
    return (off + 255) & ~(size_t)255;
}

size_t build_ws_bytes(int64_t T, int n_parts) { return carve(nullptr, T, n_parts, nullptr); }

MeshIn *build_ws_mesh_table(void *ws, int64_t T, int n_parts) {
    BuildWs w;
    carve((char *)ws, T, n_parts, &w);
    return w.mesh;
}

// Check the meshes and lay out the concatenated triangle ranges.
hra_status check_meshes(hra_ctx *ctx, const hra_mesh *meshes, int32_t n_parts, int32_t leaf,
                        std::vector<MeshIn> *hm, int64_t *T_out) {
    if (n_parts < 1 || n_parts > MAX_PARTS) return ctx->fail(HRA_ERR_INVALID_ARG, "1..255 parts per hierarchy");
    if (leaf < 1 || leaf > 16) return ctx->fail(HRA_ERR_INVALID_ARG, "leaf_size must be in 1..16");
    int64_t T = 0, V = 0;
    hm->resize(n_parts);
    for (int p = 0; p < n_parts; ++p) {
        const hra_mesh &m = meshes[p];
        if (!m.d_verts || !m.d_tris || m.n_verts < 3 || m.n_tris < 1)
            return ctx->fail(HRA_ERR_INVALID_ARG, "each mesh needs at least 3 vertices and 1 triangle");
        if (m.n_verts >= (int64_t)1 << 31) return ctx->fail(HRA_ERR_INVALID_ARG, "too many vertices in a mesh");
        (*hm)[p] = MeshIn{m.d_verts, m.d_tris, m.n_verts, m.n_tris, T, V};
        T += m.n_tris;
        V += m.n_verts;
    }
    if (T >= (int64_t)1 << 27) return ctx->fail(HRA_ERR_INVALID_ARG, "too many triangles (max 2^27 per hierarchy)");
    *T_out = T;
    return HRA_OK;
}

// The hierarchy's own arrays (no kernel work).
int64_t bvh_bytes(int64_t T, int n_parts) {
    const int64_t nn = T > 1 ? T - 1 : 1;
    return (int64_t)(sizeof(Node) * nn + sizeof(float4) * 3 * T + sizeof(int32_t) * 2 * T + sizeof(uint64_t) * T +
                     sizeof(PartMeta) * n_parts);
}

__global__ void k_put_mesh(MeshIn *dst, MeshIn m) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = m;
}

hipError_t put_mesh_table(MeshIn *dst, const MeshIn &m, hipStream_t s) {
    k_put_mesh<<<1, 64, 0, s>>>(dst, m);
    return hipGetLastError();
}

hra_status alloc_bvh(hra_ctx *ctx, const std::vector<MeshIn> &hm, int64_t T, int32_t leaf, hra_bvh **out,
                     hipStream_t stream, BvhAlloc mode) {
    const int n_parts = (int)hm.size();
    hra_bvh *b = new hra_bvh();
    b->ctx = ctx;
    b->device = ctx->device;
    b->n_parts = n_parts;
    b->n_tris = T;
    b->leaf_size = leaf;
    for (int p = 0; p < n_parts; ++p) {
        b->part_tris.push_back(hm[p].nt);
        b->part_start.push_back(hm[p].tri_start);
    }
    const int64_t nn = T > 1 ? T - 1 : 1;
    size_t bytes = 0;
    b->alloc_stream = mode == BVH_POOL_KEEP ? stream : nullptr;
    b->pooled = mode != BVH_PLAIN;
    b->build_stream = stream;
    auto alloc = [&](void **p, size_t n) -> bool {
        bytes += n;
        return (b->pooled ? hipMallocAsync(p, n, stream) : hipMalloc(p, n)) == hipSuccess;
    };
    if (!alloc((void **)&b->nodes, sizeof(Node) * nn) || !alloc((void **)&b->tris, sizeof(float4) * 3 * T) ||
        !alloc((void **)&b->leaf_pos, sizeof(int32_t) * T) || !alloc((void **)&b->valid_rank, sizeof(int32_t) * T) ||
        !alloc((void **)&b->prefix, sizeof(uint64_t) * T) || !alloc((void **)&b->parts, sizeof(PartMeta) * n_parts)) {
        hra_bvh_release(b);
        return ctx->fail(HRA_ERR_OUT_OF_MEMORY, "BVH allocation failed");
    }
    b->bytes = (int64_t)bytes;
    *out = b;
    return HRA_OK;
}

// Enqueue the whole build on `s`: kernels only (no allocation, copy or
// memset), reading the mesh table already in the workspace.
hipError_t enqueue_build(hra_ctx *ctx, hra_bvh *b, void *ws_base, hipStream_t s, uint32_t *err) {
    const int64_t T = b->n_tris;
    const int n_parts = b->n_parts;
    const int leaf = b->leaf_size;
    const int64_t nn = T > 1 ? T - 1 : 1;
    BuildWs W;
    carve((char *)ws_base, T, n_parts, &W);
    const int gT = blocks_for(T, TB), gN = blocks_for(nn, TB);
    k_build_init<<<blocks_for(std::max<int64_t>(std::max<int64_t>(T, nn), n_parts), TB), TB, 0, s>>>(
        b->leaf_pos, T, b->nodes, W.flags, W.PI, nn, W.acc, n_parts);
    k_tri_prep<<<gT, TB, 0, s>>>(W.mesh, n_parts, T, W.area, W.valid, W.tv, W.tpart, err);
    k_part_facts<<<dim3(FACT_BLOCKS, n_parts), 256, 0, s>>>(W.mesh, W.area, W.acc);
    k_part_finalize<<<blocks_for(n_parts, 64), 64, 0, s>>>(W.mesh, W.acc, n_parts, b->parts);
    k_weights<<<gT, TB, 0, s>>>(W.area, W.tpart, T, b->parts, W.w);
    hipError_t e = scan<uint64_t>(W.w, b->prefix, T, true, W.scan64_ws, s);
    if (e == hipSuccess) e = scan<uint32_t>(W.valid, W.excl, T, false, W.scan32_ws, s);
    if (e != hipSuccess) return e;
    k_part_counts<<<1, 64, 0, s>>>(b->prefix, W.excl, W.valid, n_parts, T, b->parts, W.nvt, err);
    k_ranks_keys<<<gT, TB, 0, s>>>(W.valid, W.excl, W.tv, W.tpart, T, b->parts, b->valid_rank, W.keys0, W.vals0);
    bool in1 = false;
    // keys are (part << 56) | a 54-bit Morton code, ~0 for a zero-area face:
    // with one part every key that matters differs in its low 56 bits
    e = radix_sort(W.keys0, W.vals0, W.keys1, W.vals1, T, W.rs_ws, s, &in1, n_parts == 1 ? 7 : 8);
    if (e != hipSuccess) return e;
    uint64_t *ks = in1 ? W.keys1 : W.keys0;
    uint32_t *vs = in1 ? W.vals1 : W.vals0;
    k_gather<<<gT, TB, 0, s>>>(W.tv, vs, W.tpart, b->parts, W.nvt, b->tris, b->leaf_pos);
    k_karras<<<gN, TB, 0, s>>>(ks, W.nvt, W.L, W.R, W.F, W.La, W.PI, W.PL, b->parts);
    k_small_roots<<<blocks_for(n_parts, 64), 64, 0, s>>>(b->parts, n_parts, leaf);
    k_refit<<<gT, TB, 0, s>>>(b->tris, ks, W.PL, W.PI, W.L, W.R, W.F, W.La, leaf, W.box, W.cost, W.leafy, W.height,
                              W.flags, W.nvt);
    k_emit<<<gN, TB, 0, s>>>(b->tris, ks, W.L, W.R, W.F, W.La, W.PI, W.leafy, W.box, leaf, W.nvt, b->nodes,
                             W.emitted);
    k_part_nodes<<<dim3(FACT_BLOCKS, n_parts), 256, 0, s>>>(W.emitted, W.height, W.nvt, b->parts);
    return hipGetLastError();
}

}  // namespace hra

static hra_status build_parts(hra_ctx *ctx, const hra_mesh *meshes, int32_t n_parts, const hra_bvh_opts *opts,
                              hipStream_t s, hra_bvh **out) {
    if (!ctx || !out || !meshes) return HRA_ERR_INVALID_ARG;
    *out = nullptr;
    const int leaf = opts && opts->leaf_size ? opts->leaf_size : ctx->leaf_default;
    std::vector<MeshIn> hm;
    int64_t T = 0;
    hra_status st = check_meshes(ctx, meshes, n_parts, leaf, &hm, &T);
    if (st != HRA_OK) return st;
    HRA_HIP(hipSetDevice(ctx->device));
    hra_bvh *b = nullptr;
    // from the device's stream-ordered pool (once the pool holds the memory, no
    // allocation goes to the operating system); the caller's stream is not
    // kept, since it may be destroyed before the hierarchy is released
    st = alloc_bvh(ctx, hm, T, leaf, &b, s, BVH_POOL);
    if (st != HRA_OK) return st;
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, build_ws_bytes(T, n_parts), s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(build_ws_mesh_table(ws, T, n_parts), hm.data(), sizeof(MeshIn) * n_parts,
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = enqueue_build(ctx, b, ws, s, ctx->d_err);
    if (ws) hipFreeAsync(ws, s);
    if (e != hipSuccess) {
        hipStreamSynchronize(s);
        hra_bvh_release(b);
        return ctx->fail(HRA_ERR_DEVICE, "BVH build launch failed", hipGetErrorString(e));
    }
    *out = b;
    return HRA_OK;
}

extern "C" hra_status hra_build_bvh(hra_ctx *ctx, const float *d_verts, int64_t n_verts, const int32_t *d_tris,
                                    int64_t n_tris, const hra_bvh_opts *opts, void *stream, hra_bvh **out) {
    if (!ctx || !out) return HRA_ERR_INVALID_ARG;
    const hra_mesh m = {d_verts, n_verts, d_tris, n_tris};
    return build_parts(ctx, &m, 1, opts, (hipStream_t)stream, out);
}

extern "C" hra_status hra_build_bvh_batch(hra_ctx *ctx, const hra_mesh *meshes, int32_t n_parts,
                                          const hra_bvh_opts *opts, void *stream, hra_bvh **out) {
    if (!ctx) return HRA_ERR_INVALID_ARG;
    return build_parts(ctx, meshes, n_parts, opts, (hipStream_t)stream, out);
}

extern "C" int32_t hra_bvh_parts(const hra_bvh *b) { return b ? b->n_parts : 0; }

extern "C" hra_status hra_bvh_part_info(hra_bvh *b, int32_t part, void *stream, hra_bvh_info *out) {
    if (!b || !out || part < 0 || part >= b->n_parts) return HRA_ERR_INVALID_ARG;
    hra_ctx *ctx = b->ctx;
    hipStream_t s = (hipStream_t)stream;
    hra_status st = check_error_word(ctx, s);
    if (st != HRA_OK) return st;
    PartMeta m;
    HRA_HIP(hipMemcpyAsync(&m, b->parts + part, sizeof(m), hipMemcpyDeviceToHost, s));
    HRA_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < 6; ++k) out->bbox[k] = m.bbox[k];
    out->diag = m.diag;
    out->n_tris = m.n_tris;
    out->n_degenerate = m.n_tris - m.n_valid;
    out->n_nodes = m.n_nodes;
    out->bytes = b->bytes;
    out->depth = m.depth;
    out->leaf_size = b->leaf_size;
    return HRA_OK;
}

extern "C" hra_status hra_bvh_get_info(hra_bvh *b, void *stream, hra_bvh_info *out) {
    return hra_bvh_part_info(b, 0, stream, out);
}

extern "C" hra_status hra_bvh_export(hra_bvh *b, void *stream, void *host_nodes, void *host_tris, int32_t *root,
                                     int32_t *n_valid) {
    if (!b || !host_nodes || !host_tris || !root || !n_valid) return HRA_ERR_INVALID_ARG;
    hra_ctx *ctx = b->ctx;
    hipStream_t s = (hipStream_t)stream;
    hra_status st = check_error_word(ctx, s);
    if (st != HRA_OK) return st;
    PartMeta m;
    const int64_t nn = b->n_tris > 1 ? b->n_tris - 1 : 1;
    HRA_HIP(hipMemcpyAsync(&m, b->parts, sizeof(m), hipMemcpyDeviceToHost, s));
    HRA_HIP(hipMemcpyAsync(host_nodes, b->nodes, sizeof(Node) * nn, hipMemcpyDeviceToHost, s));
    HRA_HIP(hipMemcpyAsync(host_tris, b->tris, sizeof(float4) * 3 * b->n_tris, hipMemcpyDeviceToHost, s));
    HRA_HIP(hipStreamSynchronize(s));
    *root = m.root;
    *n_valid = m.n_valid;
    return HRA_OK;
}

static void free_bvh_arrays(hra_bvh *b, hipStream_t s, bool async) {
    for (void *p : {(void *)b->nodes, (void *)b->tris, (void *)b->leaf_pos, (void *)b->valid_rank, (void *)b->prefix,
                    (void *)b->parts}) {
        if (!p) continue;
        if (async) (void)hipFreeAsync(p, s);
        else (void)hipFree(p);
    }
}

extern "C" void hra_bvh_release(hra_bvh *b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->alloc_stream) {
        free_bvh_arrays(b, b->alloc_stream, true);
    } else if (b->pooled) {
        // as a plain free does: the device's work ends first, then the
        // arrays go back to the pool
        (void)hipDeviceSynchronize();
        free_bvh_arrays(b, nullptr, true);
    } else {
        free_bvh_arrays(b, nullptr, false);
    }
    delete b;
}

extern "C" hra_status hra_bvh_release_async(hra_bvh *b, void *stream) {
    if (!b) return HRA_OK;
    if (hipSetDevice(b->device) != hipSuccess) {
        delete b;   // the handle is invalid on return; its arrays stay with the device
        return HRA_ERR_DEVICE;
    }
    // The pool hands a block freed on another stream, before that stream's
    // queued work has run, to the next allocation on the stream that first
    // allocated it (measured: no dependency is inserted).  A stream-ordered
    // free is therefore safe only on the stream the arrays came from; on any
    // other stream the device's work ends first, as in hra_bvh_release.
    const hipStream_t s = (hipStream_t)stream;
    if (b->pooled && s == b->build_stream) {
        free_bvh_arrays(b, s, true);
    } else {
        (void)hipDeviceSynchronize();
        free_bvh_arrays(b, b->alloc_stream, b->pooled);
    }
    delete b;
    return HRA_OK;
}

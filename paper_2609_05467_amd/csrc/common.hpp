// Internal declarations shared by the libhra translation units.
//
// All device code here is compiled with -ffp-contract=off and correctly
// rounded FP32 division and square root, so every FP32 expression below is
// the sequence of IEEE operations it spells out; fused multiply-adds appear
// only where written as fmaf.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hra.h"

namespace hra {

// ---------------------------------------------------------------- errors
enum : uint32_t {
    ERR_BAD_INDEX = 1u << 0,     // a triangle index outside [0, n_verts)
    ERR_EMPTY_MESH = 1u << 1,    // no triangle with nonzero area
    ERR_STACK = 1u << 2,         // traversal stack exhausted
    ERR_BAD_SAMPLE_TRI = 1u << 3, // a sample names a face that is not in the mesh
    ERR_TOOL_RADIUS = 1u << 4,    // a tool radius below twice the clearance tolerance
    ERR_BAD_ORDER = 1u << 5       // a sample order names an index outside [0, n)
};

#define HRA_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) return ctx->fail(HRA_ERR_DEVICE, #call, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------- node layout
// Binary node, 64 bytes = four 16-byte loads: both child boxes and both
// child references.  A child reference >= 0 is an interior node index;
// with bit 31 set it is a leaf: bits 27..30 hold count-1, bits 0..26 the
// first triangle of a contiguous run in the leaf-ordered triangle array.
struct alignas(16) Node {
    float4 a;  // lo0.x lo0.y lo0.z hi0.x
    float4 b;  // hi0.y hi0.z lo1.x lo1.y
    float4 c;  // lo1.z hi1.x hi1.y hi1.z
    int4 d;    // child0 child1 (unused) (unused)
};
static_assert(sizeof(Node) == 64, "node is 64 bytes");

__host__ __device__ inline int32_t leaf_code(int32_t first, int32_t count) {
    return (int32_t)(0x80000000u | ((uint32_t)(count - 1) << 27) | (uint32_t)first);
}
__host__ __device__ inline bool is_leaf(int32_t c) { return c < 0; }
__host__ __device__ inline int32_t leaf_first(int32_t c) { return c & 0x07FFFFFF; }
__host__ __device__ inline int32_t leaf_count(int32_t c) { return (int32_t)(((uint32_t)c >> 27) & 15u) + 1; }

// Per-part facts written by the build kernels and read by later kernels,
// so that no host round trip is needed between stages.  A hierarchy holds
// one or more parts; part p's input triangles are [tri_start, tri_start +
// n_tris) of the concatenated input, its nonzero-area triangles occupy
// [leaf_lo, leaf_lo + n_valid) of the leaf-ordered triangle array, and its
// own subtree starts at `root`.
struct PartMeta {
    float bbox[6];       // vertex bbox: min xyz, max xyz
    double diag;         // |max - min| in FP64
    double amax;         // largest triangle area
    uint64_t base_w;     // inclusive weight prefix just before the part
    uint64_t total_w;    // sum of the part's integer area weights
    int64_t tri_start;   // first triangle in the concatenated input
    int64_t n_verts;
    int32_t n_tris;
    int32_t k_scale;     // weights = floor(area * 2^k_scale)
    int32_t n_valid;     // nonzero-area triangles
    int32_t leaf_lo;     // first leaf-order position
    int32_t root;        // root reference (interior index or leaf code)
    int32_t depth;       // interior-node depth of the part's subtree
    int32_t n_nodes;     // emitted interior nodes of the part
    int32_t pad;
};

// Device view of one input mesh of a build.
struct MeshIn {
    const float *v;
    const int32_t *t;
    int64_t nv;
    int64_t nt;
    int64_t tri_start;    // first triangle of the part in the concatenation
    int64_t vert_start;   // first vertex of the part in the concatenation
};

// Largest number of parts in one hierarchy (the part index takes the top
// 8 bits of the 64-bit Morton key).
constexpr int MAX_PARTS = 255;

}  // namespace hra

// ---------------------------------------------------------------- handles
struct hra_ctx {
    int32_t device = 0;
    int32_t n_cu = 0;
    uint32_t *d_err = nullptr;        // device error word
    uint32_t *d_counter = nullptr;    // work counters for persistent kernels (64 words)
    // pinned host staging for small readbacks on the caller's stream (a copy
    // into pageable memory, or a blocking copy, can wait on other streams):
    // bytes [0, 64) take the error word, [64, STAGE_BYTES) a call's results
    void *h_stage = nullptr;
    hipStream_t own = nullptr;        // internal stream for table builds
    int32_t cast_rpw = 64;            // directions per wave work item
    int32_t cast_stack = 16;          // LDS stack entries per lane
    int32_t cast_traversal = HRA_TRAVERSAL_STEP;   // traversal loop (hra.h)
    int32_t cast_group = 0;           // samples per hemisphere work item (0: chosen from the direction count)
    int32_t leaf_default = 4;         // leaf size of builds whose options give 0
    std::string err;
    std::map<std::pair<int, int>, float4 *> dir_tables;  // (kind, n) -> device float4 [n]
    std::mutex mu;

    hra_status fail(hra_status s, const char *what, const char *detail = nullptr) {
        err = what ? what : "";
        if (detail) {
            err += ": ";
            err += detail;
        }
        return s;
    }
    hra_status ok() { return HRA_OK; }
};

struct hra_bvh {
    hra_ctx *ctx = nullptr;          // valid while the context lives (release does not use it)
    int32_t device = 0;              // the context's device, for release after the context has gone
    int32_t n_parts = 0;
    int64_t n_tris = 0;              // all parts
    int32_t leaf_size = 4;
    hra::Node *nodes = nullptr;      // [max(1, n_tris - 1)]
    float4 *tris = nullptr;          // [n_tris][3], leaf order, w = face index within its part
    int32_t *leaf_pos = nullptr;     // [n_tris] position in leaf order, -1 if zero area
    int32_t *valid_rank = nullptr;   // [n_tris] rank among the part's nonzero-area faces, -1 if zero area
    uint64_t *prefix = nullptr;      // [n_tris] inclusive prefix of the integer area weights
    hra::PartMeta *parts = nullptr;  // device [n_parts]
    std::vector<int64_t> part_tris;  // host: triangles per part
    std::vector<int64_t> part_start; // host: first triangle per part
    int64_t bytes = 0;
    hipStream_t alloc_stream = nullptr;  // arrays from the stream-ordered allocator on this stream, freed there
    bool pooled = false;                 // arrays from the stream-ordered allocator (else hipMalloc)
    hipStream_t build_stream = nullptr;  // the stream the pooled arrays were allocated on (compared, never used)
};

namespace hra {

// ---------------------------------------------------------------- job tables
// A sampling job: one part of a hierarchy, a mode, a seed and an output
// range; one launch runs any number of them (k_sample, sample.hip).
struct SampleJob {
    const PartMeta *meta;      // the part (device)
    const float4 *tris;        // hierarchy arrays
    const int32_t *leaf_pos;
    const uint64_t *prefix;
    const int32_t *valid_rank;
    int64_t thread_base;       // first global thread of this job
    int64_t n_threads;         // area mode: samples; centroid mode: the part's triangles
    int64_t out_base;          // first output row
    int64_t n_out;             // output rows of this job
    uint64_t seed;
    float offset_frac;
    int32_t mode;
};

struct SampleArgs {
    const SampleJob *jobs;     // device table, or null: job0 only
    int32_t n_jobs;
    SampleJob job0;
    int64_t n_threads;
    float *point, *normal, *origin;
    int32_t *tri;
};

// A cast job: the samples of one part against that part's subtree (k_cast,
// cast.hip).  Work item = (sample, chunk of directions); jobs are laid out
// back to back in item space.
struct CastJob {
    const Node *nodes;
    const float4 *tris;
    const PartMeta *meta;
    const float *origin;       // this job's first sample
    const float *normal;
    uint32_t *bits;            // this job's first row
    int64_t n_samples;
    int64_t item_base;         // first global item of this job
    int32_t n_nodes_alloc;     // node array length (bounds guard)
    int32_t pad;
};

struct CastArgs {
    const CastJob *jobs;       // device table, or null: job0 only
    int32_t n_jobs;
    CastJob job0;
    const float4 *dirs;        // canonical order
    const float4 *dirs_order;  // hemisphere: traversal order, w = canonical index (int bits)
    int32_t n_dirs;
    int32_t kind;              // 0: rotate hemisphere onto the normal, 1: world axes (cull n.D < 0)
    int32_t W;                 // words per row
    int64_t n_items;           // cast_items(kind, samples, group)
    int32_t group;             // hemisphere cast: samples per work item (cast_group)
    uint32_t *err;
    unsigned long long *work;  // instrumented variant: {node fetches, triangle tests}
    // one-sample hemisphere cast of one job: the work item of each workgroup
    // (the samples in a spatial order), or null: the workgroup's own index
    const int32_t *order = nullptr;
};

SampleJob make_sample_job(const hra_bvh *bvh, int32_t part, int32_t mode, uint64_t seed, float frac, int64_t n_out,
                          int64_t thread_base, int64_t out_base);
hipError_t launch_sample(const SampleJob *d_jobs, int32_t n_jobs, const SampleJob &job0, int64_t n_threads,
                         float *point, float *normal, float *origin, int32_t *tri, hipStream_t s);
CastJob make_cast_job(const hra_bvh *bvh, int32_t part, const float *origin, const float *normal, uint32_t *bits,
                      int64_t n_samples, int64_t item_base);
hipError_t launch_cast_any(const CastArgs &a, int rpw, int stack, int traversal, bool stats, hipStream_t s);
// Work items of a cast over n samples: one per sample (hemisphere), one per
// ten samples (six axes).
// Work items of a cast: hemisphere, ceil(n_samples / group); six-axis,
// ceil(n_samples / AX_PER_WAVE).
int64_t cast_items(int32_t kind, int64_t n_samples, int32_t group);
// Samples per hemisphere work item for n_dirs directions: `setting` if
// nonzero, else the count in 1..16 that leaves the fewest of a workgroup's
// 256 lanes idle (1 from 256 directions on).
int32_t cast_group(int32_t n_dirs, int32_t setting);

// ---------------------------------------------------------------- builds
// A build in three steps, so that it can run in memory set aside earlier
// (batch plans, graphs, the server): check and lay out the meshes, allocate
// the hierarchy's arrays, then enqueue kernels only, reading the mesh table
// from the workspace (build_ws_mesh_table) that the caller has filled.
hra_status check_meshes(hra_ctx *ctx, const hra_mesh *meshes, int32_t n_parts, int32_t leaf,
                        std::vector<MeshIn> *hm, int64_t *T_out);
// How a hierarchy's arrays are allocated: BVH_PLAIN with hipMalloc;
// BVH_POOL_KEEP from the stream-ordered allocator on `stream` and released
// there (the stream outlives the hierarchy); BVH_POOL from the stream-ordered
// allocator on `stream` (the null stream included) with no stream kept:
// hra_bvh_release waits for the device, hra_bvh_release_async frees on the
// stream it is given.
enum BvhAlloc { BVH_PLAIN = 0, BVH_POOL_KEEP = 1, BVH_POOL = 2 };
hra_status alloc_bvh(hra_ctx *ctx, const std::vector<MeshIn> &hm, int64_t T, int32_t leaf, hra_bvh **out,
                     hipStream_t stream = nullptr, BvhAlloc mode = BVH_PLAIN);
size_t build_ws_bytes(int64_t T, int n_parts);
MeshIn *build_ws_mesh_table(void *ws, int64_t T, int n_parts);
// Device bytes a hierarchy over T triangles in n_parts parts holds.
int64_t bvh_bytes(int64_t T, int n_parts);
// err: device error word the build reports to (index out of range, no
// nonzero-area triangle).
hipError_t enqueue_build(hra_ctx *ctx, hra_bvh *b, void *ws, hipStream_t s, uint32_t *err);
// Write one mesh table entry into device memory with a kernel (no host
// buffer to keep alive; can be captured).
hipError_t put_mesh_table(MeshIn *dst, const MeshIn &m, hipStream_t s);

// ---------------------------------------------------------------- helpers
hra_status dir_table(hra_ctx *ctx, hra_dirs dirs, const float4 **out);
// The canonical Fibonacci hemisphere table of n directions (the values
// dir_table caches) written to out[0, n) on stream s.
hipError_t launch_fibonacci(int32_t n, float4 *out, hipStream_t s);
// Look up, once per device, the address of the statistics' allocation-free
// scratch array; called by hra_ctx_create with `device` current.
hipError_t noalloc_setup(int device);
// Upload, once per device, the statistics' azimuth boundary table to its
// device array; called by hra_ctx_create with `device` current.
hipError_t stats_setup(int device);
hra_status check_error_word(hra_ctx *ctx, hipStream_t s);
constexpr size_t STAGE_BYTES = 4096, STAGE_USER = 64;
// ctx->h_stage + STAGE_USER: where a call copies its small results before
// check_error_word synchronises the stream.
inline void *stage_user(hra_ctx *ctx) { return (char *)ctx->h_stage + STAGE_USER; }
int blocks_for(int64_t n, int threads);

// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based stream: output
// c of stream `seed` mixes seed + (c + 1) * golden gamma.
__host__ __device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t c) {
    uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Orthonormal basis (t, b, n) from a unit normal: Duff, Burgess,
// Christensen, Hery, Kensler, Liani, Villemin, "Building an Orthonormal
// Basis, Revisited" (JCGT 2017), branchless form, FP32, in a fixed order.
__device__ inline void onb_frame(float nx, float ny, float nz, float3 &t, float3 &b) {
    const float sign = copysignf(1.0f, nz);
    const float a = -1.0f / (sign + nz);
    const float nxny = nx * ny;
    const float bb = nxny * a;
    const float snx = sign * nx;
    const float snxnx = snx * nx;
    const float snxnxa = snxnx * a;
    t.x = 1.0f + snxnxa;
    t.y = sign * bb;
    t.z = -(sign * nx);
    const float nyny = ny * ny;
    const float nynya = nyny * a;
    b.x = bb;
    b.y = sign + nynya;
    b.z = -ny;
}

// World direction of the local hemisphere point l: d_c = l.x t_c + l.y b_c
// + l.z n_c evaluated as fma(l.x, t_c, fma(l.y, b_c, l.z * n_c)).
__device__ inline float3 rotate_dir(const float3 &t, const float3 &b, float nx, float ny, float nz, float lx,
                                    float ly, float lz) {
    float3 d;
    const float zx = lz * nx, zy = lz * ny, zz = lz * nz;
    d.x = fmaf(lx, t.x, fmaf(ly, b.x, zx));
    d.y = fmaf(lx, t.y, fmaf(ly, b.y, zy));
    d.z = fmaf(lx, t.z, fmaf(ly, b.z, zz));
    return d;
}

}  // namespace hra

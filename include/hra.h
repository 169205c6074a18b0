/*
 * hra.h - hemispherical ray-casting accessibility on MI355X (gfx950).
 *
 * C ABI of libhra.so.  Every entry point follows the method of
 * "Hemispherical Ray-Casting Analysis for Milling Configuration
 * Classification and Machinability Assessment" (Baltadouros, Lauwers,
 * Duflou); the section of the paper that defines each operation is cited
 * beside it.
 *
 * Conventions shared by all calls
 *  - Return value: hra_status, 0 (HRA_OK) on success, negative on error.
 *    Calls never throw and never exit.  hra_last_error() gives the text of
 *    the last error of a context.
 *  - Pointers prefixed d_ are device pointers (HIP global memory on the
 *    context's device).  Other pointers are host pointers.
 *  - Ownership: the caller owns every array passed in or out and keeps it
 *    alive until the work enqueued on `stream` has finished.  hra_ctx and
 *    hra_bvh are opaque and owned by the library (create/destroy pairs).
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Calls enqueue their kernels on it and return without waiting,
 *    except the ones marked "synchronises", which wait for the stream.
 *  - Errors found by kernels (an index out of range, a traversal stack
 *    overflow) are recorded in a per-context device error word and reported
 *    as HRA_ERR_BAD_MESH or HRA_ERR_DEVICE by the next synchronising call.
 *  - A context is not thread-safe; use one per host thread.
 *  - Layouts: float [n][3] arrays are packed xyz triples.  Direction bitmask
 *    rows have W = ceil(n_dirs / 32) uint32 words; bit (j % 32) of word
 *    (j / 32) is direction j; 1 = unobstructed.
 */
#ifndef HRA_H
#define HRA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HRA_OK = 0,
    HRA_ERR_INVALID_ARG = -1,
    HRA_ERR_OUT_OF_MEMORY = -2,
    HRA_ERR_DEVICE = -3,
    HRA_ERR_BAD_MESH = -4,
    HRA_ERR_OVER_BUDGET = -5,
    HRA_ERR_NOT_READY = -6
} hra_status;

typedef struct hra_ctx hra_ctx;
typedef struct hra_bvh hra_bvh;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`.  Allocates the device error word
 * and the direction-table cache.  *out is set on success. */
hra_status hra_ctx_create(int32_t device, hra_ctx **out);
void hra_ctx_destroy(hra_ctx *ctx);
/* Text of the last error on this context ("" if none).  Valid until the next
 * call on the context. */
const char *hra_last_error(const hra_ctx *ctx);
/* Library version string. */
const char *hra_version(void);

/* -------------------------------------------------------------- mesh + BVH */

typedef struct {
    int32_t leaf_size; /* most triangles per BVH leaf: 1..16; 0 = default (4).  A subtree
                          that small becomes one leaf only where testing its triangles
                          costs less than traversing it (surface-area cost) */
} hra_bvh_opts;

/* Mesh ingest and acceleration structure (Section 3.1: the part is a
 * triangulated mesh; for each face its centroid, normal and area are
 * computed).  d_verts: float [n_verts][3] in mm; d_tris: int32 [n_tris][3]
 * vertex indices, counter-clockwise seen from outside.  The library copies
 * what it needs; the inputs may be freed once the stream passes the call.
 * Zero-area triangles are kept out of the hierarchy (never sampled, never
 * hit) and counted.  Enqueues the build on `stream`; the hierarchy's
 * arrays come from the device's stream-ordered pool, allocated on `stream`
 * (see hra_bvh_release_async).  Index errors surface as HRA_ERR_BAD_MESH at
 * the next synchronising call; a mesh without any nonzero-area triangle
 * fails there too. */
hra_status hra_build_bvh(hra_ctx *ctx, const float *d_verts, int64_t n_verts, const int32_t *d_tris,
                         int64_t n_tris, const hra_bvh_opts *opts, void *stream, hra_bvh **out);

/* One input mesh: device vertex and triangle arrays as for hra_build_bvh. */
typedef struct {
    const float *d_verts;   /* float [n_verts][3], mm */
    int64_t n_verts;
    const int32_t *d_tris;  /* int32 [n_tris][3], counter-clockwise seen from outside */
    int64_t n_tris;
} hra_mesh;

/* Build one hierarchy over several parts at once (1..255 parts, at most
 * 2^27 triangles in all): one sort and one tree, each part a subtree of its
 * own.  Part p of the handle is meshes[p]; every per-part entry point takes
 * the part index.  Same ownership, errors and stream rules as
 * hra_build_bvh (which is this call with one part). */
hra_status hra_build_bvh_batch(hra_ctx *ctx, const hra_mesh *meshes, int32_t n_parts, const hra_bvh_opts *opts,
                               void *stream, hra_bvh **out);
/* Number of parts in a hierarchy. */
int32_t hra_bvh_parts(const hra_bvh *bvh);

typedef struct {
    float bbox[6];         /* min xyz, max xyz of the vertices (the stock box) */
    double diag;           /* |max - min| */
    int64_t n_tris;        /* triangles given */
    int64_t n_degenerate;  /* zero-area triangles (not in the hierarchy) */
    int64_t n_nodes;       /* interior nodes of the hierarchy */
    int64_t bytes;         /* device bytes held by the handle */
    int32_t depth;         /* longest root-to-leaf path of interior nodes */
    int32_t leaf_size;
} hra_bvh_info;

/* Copy the summary of part 0 (hra_bvh_get_info) or of part `part` to the
 * host.  Synchronises `stream`. */
hra_status hra_bvh_get_info(hra_bvh *bvh, void *stream, hra_bvh_info *out);
hra_status hra_bvh_part_info(hra_bvh *bvh, int32_t part, void *stream, hra_bvh_info *out);

/* Copy the hierarchy to host memory, for inspection and invariant checks.
 * host_nodes: n_tris - 1 (at least 1) records of 64 bytes: float lo0[3],
 * hi0.x | hi0.yz, lo1.xy | lo1.z, hi1[3] | int32 child0, child1, 0, 0; a
 * child >= 0 is a node index, < 0 a leaf: bits 27..30 = count - 1, bits
 * 0..26 = first triangle; slots that are not part of the tree hold children
 * 0x7fffffff.  host_tris: n_tris x 48 bytes, the first n_valid used: float4
 * v0, v1, v2 in leaf order, w = face index (int32 bits).  *root: the root
 * reference; *n_valid: triangles in the hierarchy (part 0 of a batch
 * hierarchy; its other parts follow in the same arrays).  Synchronises. */
hra_status hra_bvh_export(hra_bvh *bvh, void *stream, void *host_nodes, void *host_tris, int32_t *root,
                          int32_t *n_valid);
/* Free a hierarchy.  The arrays of one from hra_build_bvh or
 * hra_build_bvh_batch come from the device's stream-ordered pool: the call
 * first waits for the device's queued work, as a plain free does, then
 * returns them to the pool.  Allowed after its context has been destroyed,
 * so that garbage-collected handles may go in any order; every other call
 * on a hierarchy needs its context alive. */
void hra_bvh_release(hra_bvh *bvh);
/* Free a hierarchy in stream order, without waiting, when `stream` is the
 * stream it was built on (still alive): its arrays return to the device's
 * pool once the work queued on `stream` so far has run.  The caller orders
 * every other reader of the hierarchy before that point (on `stream`
 * itself, through an event that `stream` waits on, or by having waited for
 * it).  With any other stream the call waits for the device first, as
 * hra_bvh_release does: this runtime's pool gives a block freed on one
 * stream to the next allocation on the stream that allocated it, before
 * the freeing stream's queued work has run.  The handle is invalid on
 * return, also on error.  HRA_ERR_DEVICE if the device cannot be made
 * current.  For the pipelined caller whose device must not drain between
 * steps (a host wait for one step's result while the next one's work is
 * queued).  Allowed after its context has been destroyed. */
hra_status hra_bvh_release_async(hra_bvh *bvh, void *stream);

/* ----------------------------------------------------------------- samples */

typedef struct {
    float *point;   /* device float [n][3]: surface point p */
    float *normal;  /* device float [n][3]: unit geometric normal of its face */
    float *origin;  /* device float [n][3]: ray origin p + eps * normal */
    int32_t *tri;   /* device int32 [n]: index of its face in the input mesh */
    int64_t n;      /* number of samples */
    int32_t *order; /* device int32 [n] or NULL: a spatial order of the samples, a permutation of
                       [0, n) (indices sorted stably by a 21-bit Morton code of the origin in the part's
                       box).  The
                       samplers write it when it is non-NULL; the hemisphere cast reads it, or forms one
                       itself when it is NULL.  Results do not depend on it: it only groups nearby
                       samples in time.  An index outside [0, n) sets HRA_ERR_INVALID_ARG at the next
                       synchronising call; an order that repeats an index leaves rows unwritten. */
} hra_samples;

enum { HRA_SAMPLE_AREA = 0, HRA_SAMPLE_CENTROID = 1 };

/* Surface points to cast from (Section 3.1: rays leave a slightly offset
 * face centroid).  mode HRA_SAMPLE_CENTROID: one sample per nonzero-area
 * face, in face order (out->n must equal n_tris - n_degenerate).
 * mode HRA_SAMPLE_AREA: out->n i.i.d. points with density proportional to
 * area, drawn with the counter-based SplitMix64 stream `seed`.  The offset is
 * eps = offset_frac x bbox diagonal (offset_frac in (0, 0.01]; 1e-4 is the
 * usual value) along the face normal.  Caller allocates the four arrays. */
hra_status hra_sample_surface(hra_ctx *ctx, const hra_bvh *bvh, int32_t mode, uint64_t seed,
                              float offset_frac, const hra_samples *out, void *stream);
/* The same for part `part` of a batch hierarchy (face indices are the
 * part's own). */
hra_status hra_sample_part(hra_ctx *ctx, const hra_bvh *bvh, int32_t part, int32_t mode, uint64_t seed,
                           float offset_frac, const hra_samples *out, void *stream);

/* -------------------------------------------------------------- directions */

enum { HRA_DIRS_HEMI_FIBONACCI = 0, HRA_DIRS_AXES6 = 1 };

typedef struct {
    int32_t kind; /* HRA_DIRS_HEMI_FIBONACCI or HRA_DIRS_AXES6 */
    int32_t n;    /* number of directions: 1..65536 (AXES6: 6) */
} hra_dirs;

/* Direction set (Section 3.1, Fig. 1: uniformly sampled hemisphere;
 * Section 3.2: the six principal directions).  Writes the exact FP32 values
 * the cast kernel uses to host_out[n][3]: local hemisphere points
 * (x, y, z > 0) for the Fibonacci set, world +X,-X,+Y,-Y,+Z,-Z for AXES6.
 * Synchronises the context's internal stream. */
hra_status hra_dirs_table(hra_ctx *ctx, hra_dirs dirs, float *host_out);

/* ------------------------------------------------------------------ casting */

/* Any-hit accessibility cast (Section 3.1: rays over the hemisphere rotated
 * onto each face normal, from the offset point; a ray obstructed by any
 * triangle is not counted; Section 3.2: rays along the six principal
 * directions with the same kernel).  For HEMI_FIBONACCI the local direction
 * l is rotated onto the sample normal with the orthonormal basis of Duff et
 * al. (2017); for AXES6 the world direction is used and a direction with
 * normal . D < 0 is not cast (bit 0).  Triangles block from both sides; rays
 * extend over t in (0, inf).  Only the samples' origin and normal are read
 * (not their triangle index), so samples drawn on one mesh may be cast
 * against a hierarchy of that mesh together with other geometry (fixtures,
 * clamps, a machine envelope): the obstacles then block rays as well.
 * d_bits: uint32 [samples->n][W] (written in full); d_counts: uint32
 * [samples->n] popcount of each row, or NULL. */
hra_status hra_cast_hemisphere(hra_ctx *ctx, const hra_bvh *bvh, const hra_samples *samples, hra_dirs dirs,
                               uint32_t *d_bits, uint32_t *d_counts, void *stream);
/* The same against part `part` of a batch hierarchy. */
hra_status hra_cast_part(hra_ctx *ctx, const hra_bvh *bvh, int32_t part, const hra_samples *samples, hra_dirs dirs,
                         uint32_t *d_bits, uint32_t *d_counts, void *stream);

/* Traversal loops of the casts.  Both visit the same nodes and test the same
 * triangles in the same order, so results are identical; which is faster
 * depends on the part (the autotuner measures it).
 *   HRA_TRAVERSAL_STEP: one unit of work per lane and loop iteration, a
 *     triangle test or a stack pop and node visit (lanes at a leaf and lanes
 *     inside the tree advance together);
 *   HRA_TRAVERSAL_LEAF_LOOP: one node visit per iteration, then the
 *     triangles of its hit leaf children (lanes stay in step on the tree). */
#define HRA_TRAVERSAL_STEP 1
#define HRA_TRAVERSAL_LEAF_LOOP 2
/*   HRA_TRAVERSAL_REFILL: the step loop, with lanes whose ray has ended
 *     taking the next rays of their work item's list (hemisphere casts; the
 *     six-axis cast uses the step loop). */
#define HRA_TRAVERSAL_REFILL 3

typedef struct {
    int32_t rays_per_wave; /* directions per work item of one wavefront: 64, 128 or 256 */
    int32_t stack_depth;   /* traversal stack entries per lane held in LDS: 16, 20, 24 or
                              32, default 16 (deeper paths overflow into private memory) */
    int32_t leaf_size;     /* triangles per leaf of builds whose options give 0: 1..16
                              (0 in hra_set_cast_config: keep the current value) */
    int32_t traversal;     /* HRA_TRAVERSAL_STEP or HRA_TRAVERSAL_LEAF_LOOP
                              (0 in hra_set_cast_config: keep the current value) */
    int32_t samples_per_group; /* samples per workgroup of the hemisphere cast,
                              1..16; 0 (default) = chosen from the direction count:
                              1 from 256 directions on, else the count that leaves
                              the fewest of the workgroup's 256 lanes idle (5 for
                              150 directions).  Plans and servers take the value in
                              force when they are created. */
} hra_cast_config;

/* Launch shape of hra_cast_hemisphere and default leaf size for this
 * context (defaults 64 / 16 / 4 / HRA_TRAVERSAL_STEP).  Results do not depend on it; only speed
 * does. */
hra_status hra_set_cast_config(hra_ctx *ctx, const hra_cast_config *cfg);
hra_status hra_get_cast_config(const hra_ctx *ctx, hra_cast_config *cfg);

/* Tool-aware accessibility (the paper's rays are infinitely thin; its
 * Section 3.3 reach test and its limitations concern the real tool).  A
 * ball-end tool of radius tool_radius (mm) touches each sample point p from
 * outside: tip centre c = p + r n (FP64 from the FP32 point and normal),
 * and the tool, shank included, fills every point within r of the
 * half-line from c along the approach direction (the direction normalised
 * in FP64).  Direction j is free (bit 1) iff no triangle of the part comes
 * closer to that half-line than r - tol, tol = 1e-4 x the part's
 * bounding-box diagonal.  Directions as in hra_cast_part: the Fibonacci
 * hemisphere rotated onto each normal, or HRA_DIRS_AXES6 (an axis with
 * n . D < 0 is not cast: bit 0).  Uses samples->point and ->normal; the
 * origin and triangle index are not used (obstacles as for
 * hra_cast_hemisphere: cast against a hierarchy that includes them; tol
 * then follows that hierarchy's diagonal).  d_bits: uint32 [n][ceil(N/32)], d_counts: uint32
 * [n] or NULL.  A radius of at most 2 tol sets the error word
 * (HRA_ERR_INVALID_ARG at the next synchronising call); a non-positive or
 * non-finite one fails at once.  Enqueues on `stream`. */
hra_status hra_cast_tool(hra_ctx *ctx, const hra_bvh *bvh, int32_t part, const hra_samples *samples, hra_dirs dirs,
                         double tool_radius, uint32_t *d_bits, uint32_t *d_counts, void *stream);
/* The tool cast with a holder (an extension of the same reading: Section
 * 3.3 names tool reach, and a real cutter sits in a wider holder).  The
 * tool, as in hra_cast_tool, is every point within tool_radius of the
 * approach half-line from the tip centre c; the holder is every point within
 * holder_radius of the half-line from c + (cut_length + holder_radius) u, a
 * cylinder whose rounded nose reaches down exactly to c + cut_length u (the
 * end of the cutting length) and never below it.  Direction free iff no
 * triangle comes closer than tool_radius - tol to the tool's half-line nor
 * closer than holder_radius - tol to the holder's (tol and the ambiguity
 * band as for hra_cast_tool).  cut_length must be positive and finite and
 * holder_radius finite and >= tool_radius (HRA_ERR_INVALID_ARG otherwise);
 * holder_radius == tool_radius gives hra_cast_tool's bits.  Outputs,
 * directions and stream as for hra_cast_tool. */
hra_status hra_cast_tool_holder(hra_ctx *ctx, const hra_bvh *bvh, int32_t part, const hra_samples *samples,
                                hra_dirs dirs, double tool_radius, double cut_length, double holder_radius,
                                uint32_t *d_bits, uint32_t *d_counts, void *stream);
/* The same tool cast (identical bits) in an instrumented build that also
 * counts, over all directions, the interior nodes visited, the FP64
 * triangle-distance tests made and the triangles that reached the FP32
 * screens ahead of them.  Synchronises `stream`. */
hra_status hra_cast_tool_work(hra_ctx *ctx, const hra_bvh *bvh, int32_t part, const hra_samples *samples,
                              hra_dirs dirs, double tool_radius, uint32_t *d_bits, uint64_t *node_visits,
                              uint64_t *tri_tests, uint64_t *tri_screened, void *stream);

/* The same cast as hra_cast_hemisphere (identical bits) in an instrumented
 * build of the traversal that also counts, over all rays, the interior
 * nodes fetched and the ray-triangle tests made.  These counts give the
 * algorithmic memory traffic per ray (64 bytes per node, 48 per triangle).
 * Synchronises `stream`. */
hra_status hra_cast_work(hra_ctx *ctx, const hra_bvh *bvh, const hra_samples *samples, hra_dirs dirs,
                         uint32_t *d_bits, uint64_t *node_fetches, uint64_t *tri_tests, void *stream);

/* The rays exactly as the cast kernel forms them, for checking: for the
 * samples listed in d_sample_idx (int64 [n_idx]) writes
 * d_out float [n_idx][n_dirs][6] = (origin xyz, direction xyz). */
hra_status hra_debug_rays(hra_ctx *ctx, const hra_samples *samples, hra_dirs dirs, const int64_t *d_sample_idx,
                          int64_t n_idx, float *d_out, void *stream);

/* ------------------------------------------------- directional statistics */

typedef struct {
    float *mean;      /* device float [n][3]: signed mean of unobstructed world directions */
    float *absmean;   /* device float [n][3]: mean of their absolute components */
    int8_t *axis;     /* device int8 [n]: dominant axis 0/1/2, -1 if no ray is unobstructed */
    float *conc;      /* device float [n]: axis concentration absmean[axis] / sum(absmean) */
    uint32_t *hist;   /* device uint32 [8192]: world-direction histogram of unobstructed rays */
    void *totals;     /* device scratch of hra_dirstats_bytes() bytes: part totals */
} hra_dirstats;

/* The azimuth boundary table hra_dominant_axes bins with, for checking
 * (host only, no device or context): 4 quadrants (index 2 * (x < 0) +
 * (y < 0), sign bits) x 129 cells over the pseudo-angle p = |y| / (|x| +
 * |y|) in [0, 1] (cell floor(128 p)), each 4 floats: the last sector
 * boundary in p at or below the cell's start, the next boundary, and the
 * sectors (bit patterns of uint32 byte offsets, 4 x sector) below and at or
 * above that next boundary.  Returns the float count (2064); writes `out`
 * only when capacity is at least that. */
int32_t hra_debug_azimuth_table(float *out, int32_t capacity);

/* Bytes needed for hra_dirstats.totals for n samples. */
int64_t hra_dirstats_bytes(int64_t n);

/* Directional variability (Section 3.3: dominant axis alignment and
 * directional concentration of each face from its unobstructed rays).
 * Per sample with set U of unobstructed directions d_j (world frame, as
 * cast): mean m = sum d_j / |U|, absmean A_k = sum |d_jk| / |U|; dominant
 * axis = smallest k with |m_k| >= (1 - 1e-5) max |m|; concentration
 * A_axis / (A_x + A_y + A_z).  m is the frame applied in FP64 to the FP64
 * sum of the local-frame directions; A is summed in FP32 over at most 64
 * terms per lane and 4096-direction chunk, then in FP64 (relative error
 * below 4e-6).  Histogram bin = zb * 128 + az with zb = min(63,
 * floor((d_z/|d| + 1) 32)) and az = min(127, floor((atan2(d_y, d_x) + pi)
 * 128 / (2 pi))) as in FP64: taken in FP32 where the coordinates lie clear
 * of a bin edge, else by that FP64 formula.
 * Part totals (counts per axis, blind samples, total unobstructed rays, and
 * the concentrations summed as integers round(c 2^32), so the same on every
 * run) go to out->totals for hra_classify. */
hra_status hra_dominant_axes(hra_ctx *ctx, const hra_samples *samples, hra_dirs dirs, const uint32_t *d_bits,
                             const hra_dirstats *out, void *stream);

/* hra_dominant_axes for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same outputs, bit for bit, with no allocation.  What
 * hra_dominant_axes allocates (its cached direction table and per-block
 * histogram slices) sits instead in a device array of the library, 32 MiB +
 * 130 KiB per device, held from the first context on that device until the
 * process ends.  dirs.n must be 1..8192 (HRA_ERR_INVALID_ARG beyond).  Every
 * call on one device shares that array: calls that overlap on a device (two
 * streams, two threads) race and must be ordered by the caller.  Arguments,
 * outputs and stream as for hra_dominant_axes. */
hra_status hra_dominant_axes_noalloc(hra_ctx *ctx, const hra_samples *samples, hra_dirs dirs, const uint32_t *d_bits,
                                     const hra_dirstats *out, void *stream);

typedef struct {
    double min_access; /* multi-axis if overall accessibility < this (default 0.60) */
    double min_share;  /* multi-axis if the largest dominant-axis share < this (default 0.45) */
    double max_conc;   /* multi-axis if the mean axis concentration > this (default 0.40) */
} hra_thresholds;

typedef struct {
    double access;          /* overall accessibility: unobstructed / (n * n_dirs) */
    double share[3];        /* fraction of non-blind samples per dominant axis (sums to 1) */
    double mean_conc;       /* mean concentration over non-blind samples */
    int64_t n_samples;
    int64_t n_blind;        /* samples with no unobstructed ray */
    uint64_t n_unobstructed;
    int32_t multi_axis;     /* 1 = multi-axis, 0 = 3-axis */
    int32_t tripped;        /* bit 0 access, bit 1 share, bit 2 concentration */
    int32_t near_tie;       /* an indicator lies within 1e-9 of its threshold */
} hra_class_report;

/* 3-axis versus multi-axis (Section 3.3: three indicators; if any
 * threshold is exceeded the part needs multi-axis machining).  thresholds
 * NULL = defaults.  Reads the totals written by hra_dominant_axes for the
 * same n and n_dirs.  Synchronises `stream`. */
hra_status hra_classify(hra_ctx *ctx, const hra_dirstats *stats, int64_t n, int32_t n_dirs,
                        const hra_thresholds *thresholds, hra_class_report *out, void *stream);

typedef struct {
    int32_t n_peaks;        /* local maxima found (<= k requested) */
    int32_t bin[16];        /* their bins, largest mass first */
    uint32_t mass[16];
    float dir[16][3];       /* bin-centre world directions */
    uint64_t axis_mass[6];  /* histogram mass within 45 degrees of +X,-X,+Y,-Y,+Z,-Z */
} hra_hist_peaks;

/* Dominant directions of a part from its direction histogram (host
 * function, no device work): the k (<= 16) largest local maxima of the
 * 64 x 128 (z band x azimuth) bins, a bin counting as a maximum when no
 * neighbour in the 3 x 3 window (azimuth wraps) holds more (ties: the lower
 * bin index wins), and the mass inside 45-degree cones about the six axes.
 * host_hist: uint32 [8192] as written by hra_dominant_axes. */
hra_status hra_histogram_peaks(const uint32_t *host_hist, int32_t k, hra_hist_peaks *out);

/* ------------------------------------------------------------------ setups */

enum { HRA_CLASS_VIABLE = 0, HRA_CLASS_OVER = 1, HRA_CLASS_INACCESSIBLE = 2, HRA_CLASS_FIXTURE = 3 };

typedef struct {
    int32_t min_count;   /* exact minimum number of setup directions */
    int32_t min_mask;    /* its directions, bit k: +X,-X,+Y,-Y,+Z,-Z; smallest mask on ties */
    int32_t greedy_count;/* the greedy set cover's count */
    int32_t greedy_mask;
    int64_t n_class[4];  /* samples per class: viable, over-threshold, inaccessible, fixture */
    uint32_t code_hist[64]; /* viable samples per 6-bit reachable-direction code */
} hra_setup_report;

/* Reachability and minimum setups (Section 3.3, last paragraph: for each
 * accessible principal direction the tool travel is checked against the
 * usable tool length; bounding-box faces are fixture faces; remaining faces
 * are viable, over-threshold or inaccessible; a set cover over viable faces
 * gives the setup count).  d_axes_bits: uint32 [n] from hra_cast_hemisphere
 * with HRA_DIRS_AXES6.  Travel along +k is bbox_max_k - p_k, along -k
 * p_k - bbox_min_k (FP64); reachable iff accessible and travel <= tool
 * length.  A fixture face has all three vertices on one bbox plane within
 * 1e-6 x diag.  The minimum is exact (all 63 subsets); the greedy count is
 * reported beside it.  d_class: uint8 [n] or NULL.  Synchronises. */
hra_status hra_min_setups(hra_ctx *ctx, const hra_bvh *bvh, const hra_samples *samples,
                          const uint32_t *d_axes_bits, double tool_length, uint8_t *d_class,
                          hra_setup_report *out, void *stream);
/* The same for part `part` of a batch hierarchy. */
hra_status hra_min_setups_part(hra_ctx *ctx, const hra_bvh *bvh, int32_t part, const hra_samples *samples,
                               const uint32_t *d_axes_bits, double tool_length, uint8_t *d_class,
                               hra_setup_report *out, void *stream);

/* ------------------------------------------------------------------- files */

typedef struct hra_stl hra_stl;

/* Read an STL file into host memory (the paper analyses parts given as
 * STEP/STL geometry, Sections 1 and 3.1).  Binary when the file size is
 * exactly 84 + 50 x (the uint32 at byte 80), otherwise ASCII ("solid",
 * facets of "facet [normal ...] outer loop", three "vertex x y z",
 * "endloop endfacet", then "endsolid"; numbers parsed to the nearest FP64
 * value, then rounded to FP32).  Vertices are welded: equal FP32
 * coordinates (-0 taken as +0) share an index, numbered by first
 * appearance; facets keep file order and vertex order, and stored facet
 * normals are ignored.  Host only: no device, no context.  *out holds the
 * mesh until hra_stl_free; *n_verts and *n_tris give the array sizes for
 * hra_stl_copy.  HRA_ERR_INVALID_ARG for an unreadable, malformed or empty
 * file or a non-finite coordinate; hra_stl_error() has the text (per host
 * thread). */
hra_status hra_stl_read(const char *path, hra_stl **out, int64_t *n_verts, int64_t *n_tris);
/* Copy the welded mesh to host_verts float [n_verts][3] and host_tris int32
 * [n_tris][3], ready for hra_build_bvh once on the device. */
hra_status hra_stl_copy(const hra_stl *m, float *host_verts, int32_t *host_tris);
void hra_stl_free(hra_stl *m);
/* Text of the last hra_stl_read error on this host thread. */
const char *hra_stl_error(void);

/* ------------------------------------------------------------ machining frame */

#define HRA_FRAME_BAD_INDEX 1u  /* a triangle index outside [0, n_verts) */
#define HRA_FRAME_EMPTY 2u      /* no triangle with nonzero area */

typedef struct {
    double axes[3][3];     /* rows X, Y, Z: unit vectors in world coordinates, right-handed */
    double confidence;     /* share of the surface area on faces within 5 degrees of an axis */
    double aligned[3];     /* that area per axis X, Y, Z (mm^2) */
    double extent[3];      /* vertex extent along X, Y, Z (mm) */
    double total_area;     /* area of the nonzero-area faces (mm^2) */
    int32_t peak_bin[2];   /* histogram bins the first and second axes came from (-1: none) */
    int32_t shift;         /* histogram weights are floor(area * 2^shift) */
    uint32_t error;        /* 0, or HRA_FRAME_BAD_INDEX | HRA_FRAME_EMPTY (axes are then the identity) */
} hra_frame;

/* Canonical machining frame of a part (Section 3.2: parts are reoriented
 * into a canonical machining frame before the orthogonal casts; the paper
 * gives no method, this is the library's).  Per face, the FP64 unit normal
 * of the FP32 vertices, folded so that opposite faces agree, and the area.
 * Integer area weights floor(area * 2^shift), shift = 31 - e for the largest
 * area m 2^e (m in [0.5, 1)), go into the 8192 bins of the direction
 * histogram (64 z bands x 128 azimuth sectors, as hra_dominant_axes).  The
 * heaviest bin (lowest index on ties) seeds the first axis: the
 * area-weighted mean normal of the bin, then of the faces within 5 degrees,
 * then within 2 degrees (each normal signed to agree with the axis).  The
 * heaviest bin whose centre lies within 15 degrees of perpendicular seeds
 * the second axis the same way, made orthogonal to the first after each
 * step; without one, the world axis least aligned with the first is used.
 * The third is their cross product.  Z is the axis with the most area on
 * faces within 5 degrees of it, X the remaining one of larger vertex
 * extent, Y = Z x X; Z and X have their largest component positive.
 * Values within a relative 1e-9 count as tied; the earlier axis wins.
 *
 * mesh: device arrays as for hra_build_bvh (n_tris in [1, 2^31 - 256]).
 * d_frame: device hra_frame, written when the stream reaches it.  d_hist:
 * device uint64 [8192] that receives the weighted histogram, or NULL.  Index
 * errors and meshes without a nonzero-area face set d_frame->error and the
 * context's error word (HRA_ERR_BAD_MESH at the next synchronising call).
 * Enqueues on `stream`; the workspace (hra_frame_ws_bytes) is taken from and
 * returned to the stream-ordered allocator.  The result is the same on every
 * run (fixed reduction order). */
hra_status hra_frame_estimate(hra_ctx *ctx, const hra_mesh *mesh, uint64_t *d_hist, hra_frame *d_frame,
                              void *stream);
/* Device workspace hra_frame_estimate takes for n_tris triangles. */
int64_t hra_frame_ws_bytes(int64_t n_tris);

/* Vertices in the frame: out_k = (f_k0 x + f_k1 y) + f_k2 z in FP32, f =
 * d_frame->axes rounded to FP32 (so a part reoriented with it can go through
 * every other call unchanged).  d_in and d_out: float [n_verts][3], may be
 * the same array.  A frame with an error copies the vertices unchanged.
 * Enqueues on `stream`. */
hra_status hra_frame_apply(hra_ctx *ctx, const hra_frame *d_frame, const float *d_in, float *d_out, int64_t n_verts,
                           void *stream);

/* ------------------------------------------------------------- datum planes */

typedef struct {
    int32_t dir[3];      /* primary, secondary, tertiary: axis direction 0..5 (+X,-X,+Y,-Y,+Z,-Z), -1 empty */
    int32_t n_tris[3];   /* faces of each plane */
    double offset[3];    /* the plane's coordinate along its axis: the least face offset (mm) */
    double area[3];      /* area_w x 2^-k, k the part's weight scale (mm^2) */
    uint64_t area_w[3];  /* sum of the faces' integer area weights floor(area x 2^k) */
} hra_datum_frame;

/* Datum planes of each setup orientation (Section 6 names reference frames
 * for the tolerancing of each setup as future work and gives no method; this
 * is the library's, the 3-2-1 rule of fixturing on axis-facing planes).
 * A face faces direction d = 2c + (N_c < 0) when its FP64 normal N = (B - A)
 * x (C - A) of the FP32 vertices has its dominant component c (lowest on
 * ties) with N_c^2 >= 0.99999999 |N|^2, i.e. within 1e-4 rad of the axis;
 * its offset is h = ((A_c + B_c) + C_c) / 3 in FP64.  Faces sorted by (d, h
 * with the three low bits of its order-preserving 64-bit key dropped, face
 * index) form planes, linked while consecutive offsets differ by at most
 * 1e-6 x the bounding-box diagonal.  For approach direction a (out[a], a =
 * 0..5): primary = the plane of direction a ^ 1 of largest area (the side
 * the part rests on), secondary = the largest plane whose axis is not a's,
 * tertiary = the largest plane whose axis is neither a's nor the
 * secondary's; ties to the lower direction, then the lower offset.  Areas
 * are the sampler's integer weights, so sums and choices are exact.
 *
 * bvh: a hierarchy from hra_build_bvh(_batch); part: its part index.  out:
 * host hra_datum_frame [6].  A part without axis-facing faces yields empty
 * roles.  Enqueues on `stream` with a stream-ordered workspace of about
 * 76 bytes per triangle, then synchronises it.  HRA_ERR_INVALID_ARG for a
 * null argument or a part index outside [0, parts). */
hra_status hra_datum_frames(hra_ctx *ctx, const hra_bvh *bvh, int32_t part, hra_datum_frame *out, void *stream);

/* ------------------------------------------------------------- batches */

typedef struct {
    hra_mesh mesh;          /* the part's mesh (device arrays, caller-owned) */
    int64_t n_samples;      /* area-weighted samples to draw (>= 1) */
    uint64_t seed;          /* their SplitMix64 stream */
    double tool_length;     /* usable tool length for the setup search, mm */
} hra_part_request;

typedef struct {
    int32_t n_dirs;                     /* hemisphere directions for every part */
    int32_t leaf_size;                  /* 0 = default (4) */
    int32_t rays_per_wave;              /* 0 = the context's cast configuration */
    int32_t stack_depth;                /* 0 = the context's cast configuration */
    int32_t traversal;                  /* 0 = the context's cast configuration */
    float offset_frac;                  /* 0 = 1e-4 */
    const hra_thresholds *thresholds;   /* NULL = defaults */
} hra_batch_opts;

typedef struct {
    hra_class_report cls;
    hra_setup_report setups;
} hra_part_result;

/* The whole path for many parts at once: one hierarchy for all meshes
 * (hra_build_bvh_batch), then one launch each for sampling, the hemisphere
 * cast, the directional statistics, the part totals, the six-axis cast and
 * the setup counts, every launch covering all parts.  Per part, the
 * results equal those of the single-part calls on the same inputs (the same
 * samples, bits, statistics, class and setups).  results: host
 * [n_parts].  Synchronises `stream`.  If d_bits_out is not NULL it receives
 * the hemisphere bitmasks of all parts, part after part: uint32
 * [sum n_samples][ceil(n_dirs / 32)].  Equivalent to hra_plan_create,
 * hra_plan_run without a graph, hra_plan_destroy. */
hra_status hra_batch_run(hra_ctx *ctx, const hra_part_request *parts, int32_t n_parts, const hra_batch_opts *opts,
                         hra_part_result *results, uint32_t *d_bits_out, void *stream);

/* A batch plan: every device buffer of one batch (hierarchy, build
 * scratch, samples, bitmasks, statistics, job tables) and pinned host
 * slots for its results, allocated once.  The part meshes are read at each
 * run, so they must stay allocated (their contents may change, their sizes
 * may not) until the plan is destroyed.  The launch shape (rays per wave,
 * stack depth, leaf size, traversal) is fixed at creation. */
typedef struct hra_plan hra_plan;
hra_status hra_plan_create(hra_ctx *ctx, const hra_part_request *parts, int32_t n_parts, const hra_batch_opts *opts,
                           hra_plan **out);
/* Run the plan after the work already on `stream`: build, sample, cast,
 * statistics, six-axis cast, setups; results as for hra_batch_run.  With
 * use_graph != 0 the first call captures the sequence (kernels and three
 * copies into pinned memory; no allocation, memset or host callback) in a
 * HIP graph on the plan's own streams (the six-axis cast and the setups on
 * a second stream beside the cast, forked and joined by events) and every
 * call replays it.  Without a
 * graph the per-stage times are kept (hra_plan_stage_ms).  Runs of one plan
 * must not overlap: the call synchronises before it returns. */
hra_status hra_plan_run(hra_plan *plan, int32_t use_graph, hra_part_result *results, uint32_t *d_bits_out,
                        void *stream);
/* Milliseconds of the last run without a graph: build, sample, cast,
 * statistics and totals, six-axis cast, setups.  The six-axis cast and the
 * setups run on a second stream of the plan beside the cast and the
 * statistics: their times are that stream's intervals from the end of the
 * sampling, and they share the device with the cast meanwhile. */
hra_status hra_plan_stage_ms(const hra_plan *plan, float *ms6);
/* Device bytes the plan holds. */
int64_t hra_plan_bytes(const hra_plan *plan);
/* The plan's own bitmask array (valid until the next run or destroy). */
const uint32_t *hra_plan_bits(const hra_plan *plan);
/* Free a plan; allowed after its context has been destroyed. */
void hra_plan_destroy(hra_plan *plan);

typedef struct {
    int32_t rays_per_wave;
    int32_t stack_depth;
    int32_t leaf_size;
    int32_t traversal;
    float ms;              /* mean time of one whole run of the batch (build to setups) */
} hra_tune_point;

typedef struct {
    int32_t n_points;
    int32_t best;          /* index of the fastest point */
    hra_tune_point points[27];   /* the first n_points are used */
} hra_tune_report;

/* Autotuner for a batch: sweeps rays per wave {64, 128, 256} x LDS stack
 * depth {16, 24, 32} x leaf size {2, 4, 8} (27 points; the traversal loop
 * is opts->traversal, 0 = the context's), times `reps` runs of a plan for
 * each point after one warm-up run, checks that every point gives the same
 * results, and stores the fastest point in the context's cast
 * configuration (hra_get_cast_config).  opts: as for hra_plan_create (its
 * launch-shape fields are overridden).  Synchronises `stream`. */
hra_status hra_autotune(hra_ctx *ctx, const hra_part_request *parts, int32_t n_parts, const hra_batch_opts *opts,
                        int32_t reps, hra_tune_report *out, void *stream);

/* -------------------------------------------------------------- server */

/* Serving part analyses as they arrive (the method's use case is interactive
 * feedback while a part is designed, Section 1).  A server owns a context
 * and a worker thread on one device.  Continuous mode: requests are
 * admitted in arrival order while the device memory they need (a resident
 * hierarchy, build scratch, samples, bitmasks, statistics) fits the budget,
 * evicting resident hierarchies that no request uses, least recently used
 * first; hierarchies of new parts are built on a stream of their own while
 * earlier batches run; all admitted requests ready at a launch go into one
 * batch (one launch per stage, as hra_batch_run), with up to max_inflight
 * batches on the device.  Plain mode: one request at a time in arrival
 * order, built, cast and finished before the next starts, nothing kept
 * resident.  Each result equals that of the single-part calls on the same
 * inputs. */
typedef struct hra_server hra_server;

enum { HRA_SERVE_CONTINUOUS = 0, HRA_SERVE_PLAIN = 1 };

typedef struct {
    int64_t budget_bytes;    /* device memory for hierarchies and admitted work; 0 = 200 GiB */
    int32_t mode;            /* HRA_SERVE_CONTINUOUS or HRA_SERVE_PLAIN */
    int32_t max_batch;       /* requests per launch batch, 1..255; 0 = 64 */
    int32_t max_inflight;    /* batches on the device at once, 1..4; 0 = 2 */
    int32_t keep_resident;   /* continuous mode: keep hierarchies after their requests (LRU) */
    int32_t n_dirs;          /* hemisphere directions of every analysis */
    int32_t leaf_size;       /* 0 = the context default (4) */
    float offset_frac;       /* 0 = 1e-4 */
    const hra_thresholds *thresholds;   /* NULL = defaults; copied */
} hra_server_opts;

typedef struct {
    uint64_t part_key;       /* equal keys name the same mesh: its hierarchy is reused while resident */
    const float *h_verts;    /* host float [n_verts][3] (pinned memory uploads fastest) */
    int64_t n_verts;
    const int32_t *h_tris;   /* host int32 [n_tris][3] */
    int64_t n_tris;
    int64_t n_samples;       /* area-weighted samples (>= 1) */
    uint64_t seed;
    double tool_length;      /* mm */
} hra_request;

typedef struct {
    hra_status status;       /* HRA_OK, HRA_ERR_BAD_MESH (index out of range or no nonzero-area
                                triangle), HRA_ERR_OVER_BUDGET (cannot fit even alone),
                                HRA_ERR_DEVICE */
    int32_t resident_hit;    /* its hierarchy was resident and built when it was admitted */
    int32_t batch_size;      /* requests in its launch batch */
    int32_t pad;
    int64_t batch_id;
    int64_t t_submit_ns, t_admit_ns, t_launch_ns, t_done_ns;   /* hra_now_ns clock */
    hra_part_result result;
} hra_request_result;

typedef struct {
    int64_t submitted, completed, failed, batches, builds, evictions, resident_hits;
    int64_t resident_bytes, used_bytes, peak_used_bytes;
    int32_t resident_parts, pending, inflight, pad;
} hra_server_stats;

/* Monotonic clock of the server's time stamps, in nanoseconds. */
int64_t hra_now_ns(void);
hra_status hra_server_create(int32_t device, const hra_server_opts *opts, hra_server **out);
/* Queue one analysis; returns at once with a ticket.  The host mesh arrays
 * must stay valid until the request has ended (poll or wait returns it).
 * Argument errors are returned here; mesh errors come with the result. */
hra_status hra_server_submit(hra_server *sv, const hra_request *req, uint64_t *ticket);
/* HRA_ERR_NOT_READY until the request has ended; then HRA_OK with its
 * result (taken: a ticket is returned once).  HRA_ERR_INVALID_ARG for an
 * unknown ticket. */
hra_status hra_server_poll(hra_server *sv, uint64_t ticket, hra_request_result *out);
/* As poll, waiting up to timeout_ms (< 0: no limit). */
hra_status hra_server_wait(hra_server *sv, uint64_t ticket, int64_t timeout_ms, hra_request_result *out);
/* Wait until every submitted request has ended (HRA_ERR_NOT_READY on time-out). */
hra_status hra_server_drain(hra_server *sv, int64_t timeout_ms);
hra_status hra_server_get_stats(hra_server *sv, hra_server_stats *out);
/* Stops the worker after the batches on the device have finished; requests
 * not yet launched are dropped. */
void hra_server_destroy(hra_server *sv);

#ifdef __cplusplus
}
#endif

#endif /* HRA_H */

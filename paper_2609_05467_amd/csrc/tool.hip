// Tool-aware accessibility.  The paper's rays are infinitely thin; a real
// cutter is not (Section 3.3 checks tool reach along the six axes; tool
// geometry is listed as a limitation).  Here a ball-end tool of radius r
// touches each sample point p from outside: its tip centre is c = p + r n
// and the tool, shank included, fills every point within r of the half-line
// L = {c + t u, t >= 0}, u the approach direction.  A direction is free iff
// no triangle of the part comes closer to L than r - tol, tol = 1e-4 x the
// part's bounding-box diagonal (the tool touches its own face at exactly r).
//
// One lane per (sample, direction) at a time, the directions of a sample
// on consecutive lanes in traversal order (neighbouring rays, shared
// nodes), each lane taking the next direction of its wave's range when its
// own is settled.
// The hierarchy is walked with FP32 slab tests against boxes grown by r and
// a margin (conservative: the capsule inside a grown box's sweep), and each
// candidate triangle's distance to L is computed in FP64: the plain
// definition (0 if L meets the triangle, else the least of the distance
// from c to the triangle and the three edge-to-L distances).
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace hra {
namespace {

constexpr int TOOL_THREADS = 256;
constexpr int TOOL_STACK = 24;    // LDS entries per lane
constexpr int TOOL_SPILL = 64;    // private overflow

struct ToolArgs {
    const Node *nodes;
    const float4 *tris;
    const PartMeta *meta;
    const float *point, *normal;
    const float4 *dirs;           // hemisphere: traversal order, w = canonical index bits; axes: the six axes
    int32_t n_dirs, kind, W, n_nodes_alloc;
    int64_t n_samples, n_rays;
    int32_t rays_per_lane;        // a wave's range: 64 x this consecutive directions
    int32_t pad;
    double radius;
    double hlen, hrad;            // holder: cutter length from the tip centre and holder radius (HOLDER only)
    uint32_t *bits;               // [n_samples][W], cleared first
    uint32_t *err;
    unsigned long long *work;     // instrumented launch: {node visits, FP64 distance tests, screened triangles}
};

struct D3 {
    double x, y, z;
};
__device__ inline D3 mk(double x, double y, double z) { return D3{x, y, z}; }
__device__ inline D3 operator-(D3 a, D3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ inline D3 operator+(D3 a, D3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ inline D3 operator*(double s, D3 a) { return mk(s * a.x, s * a.y, s * a.z); }
__device__ inline double dot(D3 a, D3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ inline D3 cross(D3 a, D3 b) { return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
__device__ inline double norm(D3 a) { return sqrt(dot(a, a)); }
__device__ inline D3 f4d(float4 v) { return mk(v.x, v.y, v.z); }

// Squared distances: every test compares a distance with a threshold, so
// the comparisons take squares and no square root is computed.  The
// decision changes only for distances within a few units of 2^-53 of the
// threshold, far inside the band (1e-9 x diagonal) where the oracle calls a
// direction ambiguous.

// squared distance from x to the segment [a, b]
__device__ inline double seg_dist2(D3 x, D3 a, D3 b) {
    const D3 e = b - a, w = x - a;
    const double ee = dot(e, e), we = dot(w, e);
    if (!(we > 0.0) || !(ee > 0.0)) return dot(w, w);     // nearest: a
    if (we >= ee) {                                        // nearest: b
        const D3 q = x - b;
        return dot(q, q);
    }
    const D3 q = w - (we / ee) * e;
    return dot(q, q);
}

// squared distance from x to the half-line c + t u (u unit)
__device__ inline double ray_dist2(D3 c, D3 u, D3 x) {
    const D3 w = x - c;
    double t = dot(w, u);
    t = t < 0.0 ? 0.0 : t;
    const D3 q = w - t * u;
    return dot(q, q);
}

// squared distance between the half-line and the segment: an end point of
// one of them, or the common perpendicular when it falls inside both
__device__ inline double ray_seg_dist2(D3 c, D3 u, D3 a, D3 b) {
    double best = fmin(fmin(ray_dist2(c, u, a), ray_dist2(c, u, b)), seg_dist2(c, a, b));
    const D3 e = b - a, w = c - a;
    const double B = dot(u, e), C = dot(e, e), D = dot(u, w), E = dot(e, w);
    const double den = C - B * B;
    if (den > 1e-300 * (C > 1.0 ? C : 1.0)) {
        // the feet t = tn / den on the half-line and s = sn / den on the
        // segment lie inside both when tn > 0 and 0 < sn < den (den > 0)
        const double tn = B * E - C * D, sn = E - B * D;
        if (tn > 0.0 && sn > 0.0 && sn < den) {
            const D3 q = (w + (tn / den) * u) - (sn / den) * e;
            best = fmin(best, dot(q, q));
        }
    }
    return best;
}

// squared distance from x to the triangle: to its plane when x projects
// inside it, else to the nearest edge
__device__ inline double tri_dist2(D3 x, D3 a, D3 b, D3 c) {
    const D3 e1 = b - a, e2 = c - a, w = x - a;
    const D3 nrm = cross(e1, e2);
    const double nn = dot(nrm, nrm);
    if (nn > 0.0) {
        const double d11 = dot(e1, e1), d12 = dot(e1, e2), d22 = dot(e2, e2), w1 = dot(w, e1), w2 = dot(w, e2);
        // barycentric numerators over the Gram determinant den > 0: inside
        // iff both are >= 0 and their sum is <= den
        const double den = d11 * d22 - d12 * d12;
        const double n1 = d22 * w1 - d12 * w2, n2 = d11 * w2 - d12 * w1;
        if (den > 0.0 && n1 >= 0.0 && n2 >= 0.0 && n1 + n2 <= den) {
            const double h = dot(w, nrm);
            return h * h / nn;
        }
    }
    return fmin(fmin(seg_dist2(x, a, b), seg_dist2(x, b, c)), seg_dist2(x, c, a));
}

// the half-line meets the closed triangle (signed volumes about c)
__device__ inline bool ray_meets(D3 c, D3 u, D3 A, D3 B, D3 C) {
    const D3 a = A - c, b = B - c, cc = C - c;
    const double e0 = dot(u, cross(b, cc)), e1 = dot(u, cross(cc, a)), e2 = dot(u, cross(a, b));
    const bool inside = (e0 >= 0.0 && e1 >= 0.0 && e2 >= 0.0) || (e0 <= 0.0 && e1 <= 0.0 && e2 <= 0.0);
    const D3 P = cross(b - a, cc - a);
    const double h = dot(a, P), q = dot(u, P);
    return inside && ((h >= 0.0 && q > 0.0) || (h <= 0.0 && q < 0.0));
}

// Hardware square root (within 1 ulp, 1.2e-7 relative): the screens below
// compare distances of at most a few diagonals with margins of 1e-5 x the
// diagonal beyond the threshold, far above its error, so a correctly rounded
// root (a dozen instructions more, five times per screened triangle) would
// change no decision.
__device__ inline float hsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Cheap FP32 screen: the triangle lies inside the sphere about its centroid
// m of radius rho (its farthest vertex), so it is at least
// |axis to m| - rho from the axis.  When that exceeds thr by the margin
// (far above the FP32 rounding of these few operations), it cannot block.
__device__ inline bool far_from_axis(float cx, float cy, float cz, float ux, float uy, float uz, float4 A, float4 B,
                                     float4 C, float thr_hi) {
    const float mx = ((A.x + B.x) + C.x) * (1.0f / 3.0f), my = ((A.y + B.y) + C.y) * (1.0f / 3.0f),
                mz = ((A.z + B.z) + C.z) * (1.0f / 3.0f);
    const float ax = A.x - mx, ay = A.y - my, az = A.z - mz, bx = B.x - mx, by = B.y - my, bz = B.z - mz;
    const float qx = C.x - mx, qy = C.y - my, qz = C.z - mz;
    const float rho2 = fmaxf(fmaxf((ax * ax + ay * ay) + az * az, (bx * bx + by * by) + bz * bz),
                             (qx * qx + qy * qy) + qz * qz);
    const float wx = mx - cx, wy = my - cy, wz = mz - cz;
    const float t = fmaxf((wx * ux + wy * uy) + wz * uz, 0.0f);
    const float px = wx - t * ux, py = wy - t * uy, pz = wz - t * uz;
    const float d = hsqrt((px * px + py * py) + pz * pz);
    if (d - hsqrt(rho2) > thr_hi) return true;
    // Second screen, for the faces around the sample: when the axis does not
    // approach the triangle's plane (it moves away or runs parallel), every
    // point of the axis is at least as far from the plane as the tip centre,
    // so a plane distance above thr_hi rules the triangle out.  Only for
    // triangles whose smallest-angle bound |N| > 0.05 |e1||e2| holds (about 3
    // degrees): their FP32 unit normal is good to a few 1e-6 rad, so the plane
    // distance is good to a few 1e-6 x diagonal, inside the margin of thr_hi;
    // a tiny approach rate (1e-6) costs at most 2e-6 x diagonal over the part.
    const float e1x = B.x - A.x, e1y = B.y - A.y, e1z = B.z - A.z, e2x = C.x - A.x, e2y = C.y - A.y, e2z = C.z - A.z;
    const float Nx = e1y * e2z - e1z * e2y, Ny = e1z * e2x - e1x * e2z, Nz = e1x * e2y - e1y * e2x;
    const float nn = hsqrt((Nx * Nx + Ny * Ny) + Nz * Nz);
    const float l1 = hsqrt((e1x * e1x + e1y * e1y) + e1z * e1z), l2 = hsqrt((e2x * e2x + e2y * e2y) + e2z * e2z);
    if (!(nn > 0.05f * (l1 * l2))) return false;
    const float s0 = ((cx - A.x) * Nx + (cy - A.y) * Ny) + (cz - A.z) * Nz;
    const float s1 = (ux * Nx + uy * Ny) + uz * Nz;
    const float away = s0 >= 0.0f ? s1 : -s1;
    return away >= -1e-6f * nn && fabsf(s0) > thr_hi * nn;
}

// The screens of far_from_axis for a tool with a holder: the tool's
// half-line from c with thr_hi and the holder's half-line from
// g = c + glen u (glen = cutting length + holder radius) with thr_h_hi.  The
// bounding sphere (centroid m, radius rho) must clear both, or, for the faces
// around the sample, the axis must not approach the plane and both c and g
// clear it (conditions and margins as in far_from_axis).
__device__ inline bool far_from_holder_tool(float cx, float cy, float cz, float ux, float uy, float uz, float glen,
                                            float4 A, float4 B, float4 C, float thr_hi, float thr_h_hi) {
    const float mx = ((A.x + B.x) + C.x) * (1.0f / 3.0f), my = ((A.y + B.y) + C.y) * (1.0f / 3.0f),
                mz = ((A.z + B.z) + C.z) * (1.0f / 3.0f);
    const float ax = A.x - mx, ay = A.y - my, az = A.z - mz, bx = B.x - mx, by = B.y - my, bz = B.z - mz;
    const float qx = C.x - mx, qy = C.y - my, qz = C.z - mz;
    const float rho = hsqrt(fmaxf(fmaxf((ax * ax + ay * ay) + az * az, (bx * bx + by * by) + bz * bz),
                                  (qx * qx + qy * qy) + qz * qz));
    const float wx = mx - cx, wy = my - cy, wz = mz - cz;
    const float t = (wx * ux + wy * uy) + wz * uz;
    const float ts = fmaxf(t, 0.0f), th = fmaxf(t, glen);
    const float sx = wx - ts * ux, sy = wy - ts * uy, sz = wz - ts * uz;
    const float hx = wx - th * ux, hy = wy - th * uy, hz = wz - th * uz;
    if (hsqrt((sx * sx + sy * sy) + sz * sz) - rho > thr_hi && hsqrt((hx * hx + hy * hy) + hz * hz) - rho > thr_h_hi)
        return true;
    const float e1x = B.x - A.x, e1y = B.y - A.y, e1z = B.z - A.z, e2x = C.x - A.x, e2y = C.y - A.y, e2z = C.z - A.z;
    const float Nx = e1y * e2z - e1z * e2y, Ny = e1z * e2x - e1x * e2z, Nz = e1x * e2y - e1y * e2x;
    const float nn = hsqrt((Nx * Nx + Ny * Ny) + Nz * Nz);
    const float l1 = hsqrt((e1x * e1x + e1y * e1y) + e1z * e1z), l2 = hsqrt((e2x * e2x + e2y * e2y) + e2z * e2z);
    if (!(nn > 0.05f * (l1 * l2))) return false;
    const float s0 = ((cx - A.x) * Nx + (cy - A.y) * Ny) + (cz - A.z) * Nz;
    const float s1 = (ux * Nx + uy * Ny) + uz * Nz;
    const float away = s0 >= 0.0f ? s1 : -s1;
    return away >= -1e-6f * nn && fabsf(s0) > thr_hi * nn && fabsf(s0 + glen * s1) > thr_h_hi * nn;
}

// true when the triangle comes closer than sqrt(thr2) to the half-line
// c + t u: it meets the half-line, or c lies that near it, or one of its
// edges does (each evaluated in turn, the first near one decides)
__device__ inline bool tool_blocked(D3 c, D3 u, float4 A4, float4 B4, float4 C4, double thr2) {
    const D3 A = f4d(A4), B = f4d(B4), C = f4d(C4);
    if (ray_meets(c, u, A, B, C)) return true;
    if (tri_dist2(c, A, B, C) < thr2) return true;
    if (ray_seg_dist2(c, u, A, B) < thr2) return true;
    if (ray_seg_dist2(c, u, B, C) < thr2) return true;
    return ray_seg_dist2(c, u, C, A) < thr2;
}

// Tool with a holder: the tool is the half-line from c (squared threshold
// thr2), the holder the half-line from g = c + (cutting length + holder
// radius) u (thr_h2): its rounded nose reaches down to the end of the
// cutting length.
// The plain tool's batch calls the test out of line: inlined, its
// temporaries pushed the walk's per-direction state (grown-box origins)
// into scratch, reloaded at every node visit (impeller 92 -> 61 ms).
__device__ __noinline__ bool tool_blocked_call(D3 c, D3 u, float4 A4, float4 B4, float4 C4, double thr2) {
    return tool_blocked(c, u, A4, B4, C4, thr2);
}

__device__ inline bool tool_blocked_holder(D3 c, D3 g, D3 u, float4 A4, float4 B4, float4 C4, double thr2,
                                           double thr_h2) {
    return tool_blocked(c, u, A4, B4, C4, thr2) || tool_blocked(g, u, A4, B4, C4, thr_h2);
}

// FP32 slab test against a box grown by pad on every side.  The growth is
// carried by the origin, shifted per ray: lo - pad - o = lo - (o + pad) and
// hi + pad - o = hi - (o - pad), with (o + pad) and (o - pad) formed once
// (their rounding, a few units of 2^-24 of the coordinates, lies far inside
// the margin the pad carries beyond the radius).
struct Shifted {
    float lx, ly, lz, hx, hy, hz;   // o + pad (for low faces), o - pad (for high faces)
};
__device__ inline Shifted shift(float ox, float oy, float oz, float pad) {
    return Shifted{ox + pad, oy + pad, oz + pad, ox - pad, oy - pad, oz - pad};
}
__device__ inline bool grown_slab(float lx, float ly, float lz, float hx, float hy, float hz, const Shifted &o, float ix,
                                  float iy, float iz, float &tn) {
    const float tx0 = (lx - o.lx) * ix, tx1 = (hx - o.hx) * ix;
    const float ty0 = (ly - o.ly) * iy, ty1 = (hy - o.hy) * iy;
    const float tz0 = (lz - o.lz) * iz, tz1 = (hz - o.hz) * iz;
    const float tmin = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
    const float tmax = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1));
    tn = tmin;
    return tmin <= tmax * 1.0000006f;
}

// Box test of a tool with a holder: the box grown by the tool's pad meets
// the ray anywhere on it, or the box grown by the holder's pad meets it at
// some t >= g_lo (a little below the holder's start, so a doubt means a
// visit).  tn orders the children.
__device__ inline bool holder_slab(float lx, float ly, float lz, float hx, float hy, float hz, const Shifted &oc,
                                   const Shifted &oh, float g_lo, float ix, float iy, float iz, float &tn) {
    float tc, th;
    const bool hc = grown_slab(lx, ly, lz, hx, hy, hz, oc, ix, iy, iz, tc);
    const float tx0 = (lx - oh.lx) * ix, tx1 = (hx - oh.hx) * ix;
    const float ty0 = (ly - oh.ly) * iy, ty1 = (hy - oh.hy) * iy;
    const float tz0 = (lz - oh.lz) * iz, tz1 = (hz - oh.hz) * iz;
    th = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
    const float tmax = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1)) * 1.0000006f;
    const bool hh = th <= tmax && tmax >= g_lo;
    tn = hc ? tc : th;
    return hc || hh;
}

__device__ inline float rcp_guarded(float x) { return fabsf(x) > 1e-30f ? 1.0f / x : copysignf(1e30f, x); }

// The cast's cost lies in the FP64 distance tests (a few hundred
// instructions each, about ten per direction on a part with deep pockets):
// run inside each lane's traversal they execute with one or two lanes of the
// wave active.  Here a lane only walks the hierarchy and screens candidate
// triangles in FP32, one unit of work per loop iteration (a node visit or a
// screen, in the visit order of a plain recursive walk); a triangle that
// survives its screen goes to the wave's queue in LDS, and whenever 64
// wait, or no lane walks, or enough lanes wait on their queued tests, the
// whole wave runs up to 64
// FP64 tests at once, each against the tip centre and direction its owner
// stored in LDS.  A test that finds its owner blocked sets the owner's bit
// in the wave's blocked mask; the owner then stops walking and the wave
// skips its queued tests.
//
// Each wave owns a range of 64 x TOOL_RAYS_PER_LANE consecutive directions
// (a sample's directions in traversal order, then the next sample's).  A
// lane whose direction is settled (walk ended and every test it queued
// done, or blocked and its queued entries passed) writes its bit and takes
// the next direction of the range from a counter in LDS, so the wave runs
// for about the mean walk of its directions instead of the longest one.  A
// lane takes a new direction only once the queue head has passed its last
// entry, so no queued entry ever names a lane's earlier direction.  The
// loop ends when no lane holds a direction (the range is used up, and
// every lane settled, so the queue is empty).  Lanes coordinate through
// LDS words read by the whole wave at the top of each iteration, never
// through cross-lane instructions, and every lane stays in the loop to its
// end.
//
// Four waves per SIMD (128 VGPRs, the FP64 test inline in the batch).
// HOLDER: the tool and the holder of tool_blocked_holder; boxes, screens
// and tests take each with its own radius and half-line.
constexpr int TOOL_WAVES = TOOL_THREADS / 64;
constexpr int TOOL_Q = 128;   // queue entries per wave: at most 63 wait after a batch, at most 64 join per iteration
constexpr int TOOL_RAYS_PER_LANE = 8;   // the most directions per lane (the launch picks fewer for small casts)
constexpr int TOOL_BATCH_WAIT = 16;   // a batch also runs once this many lanes wait on queued tests
enum : int { TS_IDLE = 0, TS_WALK = 1, TS_WAIT = 2 };

template <bool STATS, bool HOLDER>
__global__ __launch_bounds__(TOOL_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_cast_tool(ToolArgs a) {
    __shared__ int stk[TOOL_STACK * TOOL_THREADS];
    __shared__ int32_t q_tri[TOOL_WAVES][TOOL_Q];
    __shared__ uint8_t q_own[TOOL_WAVES][TOOL_Q];
    __shared__ double cu[TOOL_WAVES][64][6];       // per lane: tip centre c, unit direction u
    __shared__ int ctl[TOOL_WAVES][6];             // per wave: queue head, queue tail, walking lanes,
                                                   // lanes holding a direction, next direction of the
                                                   // range, lanes whose walk ended and that wait
    __shared__ unsigned long long blk[TOOL_WAVES]; // per wave: lanes whose direction is blocked
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wave_id = (int64_t)blockIdx.x * TOOL_WAVES + wv;
    const int64_t range0 = wave_id * (64 * (int64_t)a.rays_per_lane);
    const int64_t range1 = min(range0 + 64 * (int64_t)a.rays_per_lane, a.n_rays);
    const PartMeta &P = *a.meta;
    const double r = a.radius, tol = 1e-4 * P.diag, thr = r - tol;
    const double rr = HOLDER ? fmax(r, a.hrad) : r, thr_h = HOLDER ? a.hrad - tol : thr;
    const double glen = a.hlen + a.hrad;          // HOLDER: the holder's half-line starts at c + glen u
    const double thr2 = thr * thr, thr_h2 = thr_h * thr_h;
    const int32_t root = P.root, n_valid = P.n_valid, n_tris_alloc = P.leaf_lo + P.n_valid;
    // FP32 box tests from the rounded tip centre; the margin covers the
    // rounding of the centre and of the grown box faces
    const float pad = (float)(rr * 1.0001) + (float)(1e-5 * P.diag);
    const float pad_c = (float)(r * 1.0001) + (float)(1e-5 * P.diag);   // the cutter's (HOLDER)
    const float gl = (float)glen;
    const double gap = glen;   // the holder's start along u, for the batch's tests
    if (lane == 0) {
        ctl[wv][0] = 0;
        ctl[wv][1] = 0;
        ctl[wv][2] = 0;
        ctl[wv][3] = 0;
        ctl[wv][4] = 64;
        ctl[wv][5] = 0;
        blk[wv] = 0ull;
    }
    __syncthreads();

    // the lane's direction: sample s, bit index idx; tip centre and
    // direction for the FP32 walk; the traversal state
    int64_t s = 0;
    int32_t idx = 0;
    bool cast = false, bad = false;
    float cx = 0.f, cy = 0.f, cz = 0.f, ux = 0.f, uy = 0.f, uz = 0.f, ix = 0.f, iy = 0.f, iz = 0.f;
    float thr_hi = 0.f, thr_c_hi = 0.f;
    Shifted so{}, so_c{};
    int spill[TOOL_SPILL];
    int sp = 0;
    int32_t node = -1, ti = 0, tn = 0, budget = 0;
    int state = TS_IDLE;
    int last = 0;   // queue position after this direction's last entry
    uint32_t n_nodes = 0, n_tests = 0, n_cands = 0;

    // Take direction g of the range: set the lane up to walk it (or to
    // settle at once, when it is not cast).
    auto begin = [&](int64_t g) {
        s = g / a.n_dirs;
        const int32_t j = (int32_t)(g - s * a.n_dirs);
        const float px = a.point[3 * s], py = a.point[3 * s + 1], pz = a.point[3 * s + 2];
        const float nx = a.normal[3 * s], ny = a.normal[3 * s + 1], nz = a.normal[3 * s + 2];
        const float4 l = a.dirs[j];
        float3 d;
        cast = true;
        if (a.kind == 0) {
            float3 t, b;
            onb_frame(nx, ny, nz, t, b);
            d = rotate_dir(t, b, nx, ny, nz, l.x, l.y, l.z);
            idx = __float_as_int(l.w);
        } else {
            d = make_float3(l.x, l.y, l.z);
            idx = j;
            // into the material: not cast, bit 0
            cast = !((nx * d.x + ny * d.y) + nz * d.z < 0.0f);
        }
        if (cast && !(thr > tol)) {   // a tool thinner than twice the tolerance is not meaningful
            atomicOr(a.err, ERR_TOOL_RADIUS);
            cast = false;
        }
        const D3 c = mk((double)px + r * (double)nx, (double)py + r * (double)ny, (double)pz + r * (double)nz);
        const double dl = sqrt(((double)d.x * d.x + (double)d.y * d.y) + (double)d.z * d.z);
        const D3 u = mk(d.x / dl, d.y / dl, d.z / dl);
        cu[wv][lane][0] = c.x;
        cu[wv][lane][1] = c.y;
        cu[wv][lane][2] = c.z;
        cu[wv][lane][3] = u.x;
        cu[wv][lane][4] = u.y;
        cu[wv][lane][5] = u.z;
        cx = (float)c.x;
        cy = (float)c.y;
        cz = (float)c.z;
        ix = rcp_guarded(d.x);
        iy = rcp_guarded(d.y);
        iz = rcp_guarded(d.z);
        so = shift(cx, cy, cz, pad);
        so_c = shift(cx, cy, cz, pad_c);
        // unit direction and threshold for the FP32 screen; the margin
        // (1e-5 x diagonal, plus 1e-6 of the coordinates' magnitude for a
        // part far from the origin) is far above the screen's rounding
        ux = (float)u.x;
        uy = (float)u.y;
        uz = (float)u.z;
        const double cmax = fmax(fmax(fabs(c.x), fabs(c.y)), fabs(c.z)) + P.diag;
        thr_hi = (float)(fmax(thr, thr_h) + 1e-5 * P.diag + 1e-6 * cmax);
        thr_c_hi = (float)(thr + 1e-5 * P.diag + 1e-6 * cmax);
        sp = 0;
        node = is_leaf(root) ? -1 : root;
        ti = is_leaf(root) ? leaf_first(root) : 0;
        tn = is_leaf(root) ? leaf_count(root) : 0;
        budget = 2 * a.n_nodes_alloc + 64;
        bad = false;
        last = 0;
        if (cast && n_valid > 0) {
            state = TS_WALK;
            atomicAdd(&ctl[wv][2], 1);
        } else {
            state = TS_WAIT;
        }
    };

    // A lane's first direction is range0 + lane, later ones come from the
    // range's counter.  The plain tool starts every lane settled on no
    // direction (cast false, nothing queued), so the first one comes from
    // the set-up site in the loop; the holder's sets it up here as well.
    // Both orders give the same directions; they differ only in how the
    // compiler allocates registers (measured: plain 61 against 66 ms,
    // holder 188 against 214 ms on the impeller-like part).
    bool first = !HOLDER, walked = false;
    if constexpr (HOLDER) {
        if (range0 + lane < range1) {
            atomicAdd(&ctl[wv][3], 1);
            begin(range0 + lane);
        }
    } else {
        state = TS_WAIT;
        if (lane == 0) ctl[wv][3] = 64;
    }
    __syncthreads();
    while (true) {
        const int head = __hip_atomic_load(&ctl[wv][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const int tail = __hip_atomic_load(&ctl[wv][1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const int n_walk = __hip_atomic_load(&ctl[wv][2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const int n_busy = __hip_atomic_load(&ctl[wv][3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const int n_wait = __hip_atomic_load(&ctl[wv][5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const int qn = tail - head;
        if (qn > 0 && (qn >= 64 || n_walk == 0 || n_wait >= TOOL_BATCH_WAIT)) {
            // a batch of FP64 tests, one per lane
            if (lane < qn) {
                const int slot = (head + lane) & (TOOL_Q - 1);
                const int own = q_own[wv][slot];
                const int32_t f = q_tri[wv][slot];
                const unsigned long long bm =
                    __hip_atomic_load(&blk[wv], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (!((bm >> own) & 1ull)) {
                    const D3 oc = mk(cu[wv][own][0], cu[wv][own][1], cu[wv][own][2]);
                    const D3 ou = mk(cu[wv][own][3], cu[wv][own][4], cu[wv][own][5]);
                    const float4 *t = a.tris + 3 * (int64_t)f;
                    const float4 A4 = t[0], B4 = t[1], C4 = t[2];
                    if (STATS) ++n_tests;
                    const bool hit = HOLDER ? tool_blocked_holder(oc, oc + gap * ou, ou, A4, B4, C4, thr2, thr_h2)
                                            : tool_blocked_call(oc, ou, A4, B4, C4, thr2);
                    if (hit) atomicOr(&blk[wv], 1ull << own);
                }
            }
            // every lane stores the same new head
            ctl[wv][0] = head + (qn < 64 ? qn : 64);
            __builtin_amdgcn_wave_barrier();
            continue;
        }
        if (n_busy == 0) break;
        const unsigned long long bm = __hip_atomic_load(&blk[wv], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (state == TS_WALK) {
            bool end = ((bm >> lane) & 1ull) != 0ull;
            if (!end && tn > 0) {
                // screen one triangle of the current leaf
                if ((uint32_t)ti >= (uint32_t)n_tris_alloc) {
                    bad = true;
                } else {
                    const float4 *t = a.tris + 3 * (int64_t)ti;
                    const float4 A4 = t[0], B4 = t[1], C4 = t[2];
                    if (STATS) ++n_cands;
                    const bool far = HOLDER ? far_from_holder_tool(cx, cy, cz, ux, uy, uz, gl, A4, B4, C4, thr_c_hi, thr_hi)
                                            : far_from_axis(cx, cy, cz, ux, uy, uz, A4, B4, C4, thr_hi);
                    if (!far) {
                        const int pos = atomicAdd(&ctl[wv][1], 1);
                        const int slot = pos & (TOOL_Q - 1);
                        q_tri[wv][slot] = ti;
                        q_own[wv][slot] = (uint8_t)lane;
                        last = pos + 1;
                    }
                }
                ++ti;
                --tn;
            } else if (!end) {
                bool visit = true;
                if (node < 0) {
                    if (sp == 0) {
                        end = true;
                        visit = false;
                    } else {
                        --sp;
                        const int32_t itm = sp < TOOL_STACK ? stk[sp * TOOL_THREADS + threadIdx.x] : spill[sp - TOOL_STACK];
                        if (is_leaf(itm)) {
                            ti = leaf_first(itm);
                            tn = leaf_count(itm);
                            visit = false;
                        } else {
                            node = itm;
                        }
                    }
                }
                if (visit) {
                    if ((uint32_t)node >= (uint32_t)a.n_nodes_alloc || --budget < 0) {
                        bad = true;
                    } else {
                        const Node nd = a.nodes[node];
                        if (STATS) ++n_nodes;
                        float t0, t1;
                        bool h0, h1;
                        if (HOLDER) {
                            h0 = holder_slab(nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, so_c, so, gl * 0.99f, ix, iy,
                                             iz, t0);
                            h1 = holder_slab(nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, so_c, so, gl * 0.99f, ix, iy,
                                             iz, t1);
                        } else {
                            h0 = grown_slab(nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, so, ix, iy, iz, t0);
                            h1 = grown_slab(nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, so, ix, iy, iz, t1);
                        }
                        const int32_t c0 = nd.d.x, c1 = nd.d.y;
                        const bool l0 = h0 && is_leaf(c0), l1 = h1 && is_leaf(c1);
                        const bool g0 = h0 && !is_leaf(c0), g1 = h1 && !is_leaf(c1);
                        if (l0 || l1) {
                            const int32_t lc = l0 ? c0 : c1;
                            ti = leaf_first(lc);
                            tn = leaf_count(lc);
                        }
                        // at most one push per visit: the second leaf, or the
                        // farther of two interior children
                        const bool push = (l0 && l1) || (g0 && g1);
                        const int32_t pv = (l0 && l1) ? c1 : (t0 <= t1 ? c1 : c0);
                        node = (g0 && g1) ? (t0 <= t1 ? c0 : c1) : (g0 ? c0 : (g1 ? c1 : -1));
                        if (push) {
                            if (sp < TOOL_STACK) stk[sp * TOOL_THREADS + threadIdx.x] = pv;
                            else if (sp < TOOL_STACK + TOOL_SPILL) spill[sp - TOOL_STACK] = pv;
                            else bad = true;
                            ++sp;
                        }
                    }
                }
            }
            if (end || bad) {
                state = TS_WAIT;
                walked = true;
                atomicSub(&ctl[wv][2], 1);
                atomicAdd(&ctl[wv][5], 1);
            }
        } else if (state == TS_WAIT && head >= last) {
            // settled: every entry this direction queued has been tested or
            // skipped, so its blocked bit is final
            const bool blocked = ((bm >> lane) & 1ull) != 0ull;
            if (bad) atomicOr(a.err, ERR_STACK);
            if (cast && !bad && !blocked) atomicOr(&a.bits[s * a.W + (idx >> 5)], 1u << (idx & 31));
            if (blocked) atomicAnd(&blk[wv], ~(1ull << lane));
            if (walked) atomicSub(&ctl[wv][5], 1);
            walked = false;
            const int64_t g = range0 + (first ? lane : atomicAdd(&ctl[wv][4], 1));
            first = false;
            if (g < range1) {
                begin(g);
            } else {
                state = TS_IDLE;
                atomicSub(&ctl[wv][3], 1);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (STATS) {
        atomicAdd(a.work, (unsigned long long)n_nodes);
        atomicAdd(a.work + 1, (unsigned long long)n_tests);
        atomicAdd(a.work + 2, (unsigned long long)n_cands);
    }
}

__global__ void k_tool_zero(uint32_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void k_tool_popcount(const uint32_t *bits, int64_t n, int32_t W, uint32_t *counts) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    uint32_t c = 0;
    for (int32_t w = 0; w < W; ++w) c += __popc(bits[s * W + w]);
    counts[s] = c;
}

}  // namespace
}  // namespace hra

using namespace hra;

static hra_status tool_common(hra_ctx *ctx, const hra_bvh *bvh, int32_t part, const hra_samples *samples,
                               hra_dirs dirs, double tool_radius, uint32_t *d_bits, uint32_t *d_counts,
                               unsigned long long *work, hipStream_t s, double cut_length = 0.0,
                               double holder_radius = 0.0) {
    const bool holder = cut_length != 0.0;
    if (!ctx || !bvh || !samples) return HRA_ERR_INVALID_ARG;
    if (part < 0 || part >= bvh->n_parts) return ctx->fail(HRA_ERR_INVALID_ARG, "part index out of range");
    if (samples->n < 0) return ctx->fail(HRA_ERR_INVALID_ARG, "negative sample count");
    if (!(tool_radius > 0.0) || !std::isfinite(tool_radius))
        return ctx->fail(HRA_ERR_INVALID_ARG, "tool radius must be positive and finite");
    if (holder && (!(cut_length > 0.0) || !std::isfinite(cut_length)))
        return ctx->fail(HRA_ERR_INVALID_ARG, "cutting length must be positive and finite");
    if (holder && (!(holder_radius >= tool_radius) || !std::isfinite(holder_radius)))
        return ctx->fail(HRA_ERR_INVALID_ARG, "holder radius must be finite and at least the tool radius");
    const float4 *table = nullptr;
    hra_status st = dir_table(ctx, dirs, &table);
    if (st != HRA_OK) return st;
    if (samples->n == 0) return HRA_OK;
    if (!d_bits || !samples->point || !samples->normal)
        return ctx->fail(HRA_ERR_INVALID_ARG, "bits, points and normals must be non-null");
    HRA_HIP(hipSetDevice(ctx->device));
    ToolArgs a;
    a.nodes = bvh->nodes;
    a.tris = bvh->tris;
    a.meta = bvh->parts + part;
    a.point = samples->point;
    a.normal = samples->normal;
    a.kind = dirs.kind == HRA_DIRS_AXES6 ? 1 : 0;
    a.dirs = a.kind == 1 ? table : table + dirs.n;
    a.n_dirs = dirs.n;
    a.W = (dirs.n + 31) / 32;
    a.n_nodes_alloc = (int32_t)(bvh->n_tris > 1 ? bvh->n_tris - 1 : 1);
    a.n_samples = samples->n;
    a.n_rays = samples->n * (int64_t)dirs.n;
    a.radius = tool_radius;
    a.hlen = cut_length;
    a.hrad = holder ? holder_radius : tool_radius;
    a.bits = d_bits;
    a.err = ctx->d_err;
    a.work = work;
    const int64_t words = samples->n * (int64_t)a.W;
    // longer ranges balance a wave's lanes better, shorter ones give more
    // waves: ranges grow only while the grid keeps about 64 waves per
    // compute unit (four times what fits at once)
    const int64_t per_range = 64 * (int64_t)std::max(ctx->n_cu, 1) * 64;
    a.rays_per_lane = (int32_t)std::min<int64_t>(TOOL_RAYS_PER_LANE, std::max<int64_t>(1, a.n_rays / per_range));
    a.pad = 0;
    const int64_t rays_per_block = (int64_t)TOOL_THREADS * a.rays_per_lane;
    const int64_t blocks = (a.n_rays + rays_per_block - 1) / rays_per_block;
    if (blocks >= ((int64_t)1 << 31)) return ctx->fail(HRA_ERR_INVALID_ARG, "too many rays for one call");
    k_tool_zero<<<(unsigned)((words + 255) / 256), 256, 0, s>>>(d_bits, words);
    if (holder) {
        if (work) k_cast_tool<true, true><<<(unsigned)blocks, TOOL_THREADS, 0, s>>>(a);
        else k_cast_tool<false, true><<<(unsigned)blocks, TOOL_THREADS, 0, s>>>(a);
    } else {
        if (work) k_cast_tool<true, false><<<(unsigned)blocks, TOOL_THREADS, 0, s>>>(a);
        else k_cast_tool<false, false><<<(unsigned)blocks, TOOL_THREADS, 0, s>>>(a);
    }
    if (d_counts) k_tool_popcount<<<(unsigned)((samples->n + 255) / 256), 256, 0, s>>>(d_bits, samples->n, a.W, d_counts);
    HRA_HIP(hipGetLastError());
    return HRA_OK;
}

extern "C" hra_status hra_cast_tool(hra_ctx *ctx, const hra_bvh *bvh, int32_t part, const hra_samples *samples,
                                    hra_dirs dirs, double tool_radius, uint32_t *d_bits, uint32_t *d_counts,
                                    void *stream) {
    return tool_common(ctx, bvh, part, samples, dirs, tool_radius, d_bits, d_counts, nullptr, (hipStream_t)stream);
}

extern "C" hra_status hra_cast_tool_holder(hra_ctx *ctx, const hra_bvh *bvh, int32_t part, const hra_samples *samples,
                                           hra_dirs dirs, double tool_radius, double cut_length,
                                           double holder_radius, uint32_t *d_bits, uint32_t *d_counts, void *stream) {
    if (!(cut_length != 0.0)) {
        if (!ctx) return HRA_ERR_INVALID_ARG;
        return ctx->fail(HRA_ERR_INVALID_ARG, "cutting length must be positive and finite");
    }
    return tool_common(ctx, bvh, part, samples, dirs, tool_radius, d_bits, d_counts, nullptr, (hipStream_t)stream,
                       cut_length, holder_radius);
}

extern "C" hra_status hra_cast_tool_work(hra_ctx *ctx, const hra_bvh *bvh, int32_t part, const hra_samples *samples,
                                         hra_dirs dirs, double tool_radius, uint32_t *d_bits, uint64_t *node_visits,
                                         uint64_t *tri_tests, uint64_t *tri_screened, void *stream) {
    if (!ctx) return HRA_ERR_INVALID_ARG;
    if (!node_visits || !tri_tests || !tri_screened)
        return ctx->fail(HRA_ERR_INVALID_ARG, "counter outputs must be non-null");
    *node_visits = *tri_tests = *tri_screened = 0;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *w = nullptr;
    HRA_HIP(hipMallocAsync((void **)&w, 3 * sizeof(unsigned long long), s));
    k_tool_zero<<<1, 256, 0, s>>>(reinterpret_cast<uint32_t *>(w), 6);
    hra_status st = tool_common(ctx, bvh, part, samples, dirs, tool_radius, d_bits, nullptr, w, s);
    unsigned long long h[3] = {0, 0, 0};
    hipError_t e = hipSuccess;
    if (st == HRA_OK) e = hipMemcpyAsync(h, w, sizeof(h), hipMemcpyDeviceToHost, s);
    const hipError_t e2 = hipFreeAsync(w, s);
    const hipError_t e3 = hipStreamSynchronize(s);
    if (st != HRA_OK) return st;
    if (e != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
        return ctx->fail(HRA_ERR_DEVICE, "tool work counters", hipGetErrorString(e != hipSuccess ? e : (e2 != hipSuccess ? e2 : e3)));
    *node_visits = h[0];
    *tri_tests = h[1];
    *tri_screened = h[2];
    return check_error_word(ctx, s);
}

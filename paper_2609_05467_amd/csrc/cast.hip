// Any-hit accessibility cast: BVH traversal with a short per-lane stack in
// LDS, robust slab tests, an FP32 triangle test with error bounds and an FP64
// fallback, and wave-ballot packing of direction bits.
//
// Decision per (ray, triangle), origin o, direction d, a,b,c = v - o:
//   e0 = d.(b x c), e1 = d.(c x a), e2 = d.(a x b)   (side of each edge)
//   h  = a.(b x c)                                  (side of the plane)
// The ray meets the triangle at t > 0 iff all e_i share a sign s (edges
// inclusive) and h has the sign s.  In FP32 the same four numbers come, up to
// sign, from the translated-origin form T = o - A, E1 = B - A, E2 = C - A,
// P = d x E2, Q = T x E1:
//   U = T.P = -e1,  V = d.Q = -e2,  det - U - V = -e0 (det = E1.P),  E2.Q = -h
// (scalar triple products; the identities are exact in real arithmetic).
// Each FP32 value is trusted only when its magnitude exceeds a bound on its
// rounding error, written from the largest component M of T, E1, E2 and the
// largest direction component; otherwise the edge or plane function is
// recomputed in FP64 from the FP32 inputs.  A sign trusted this way is the
// exact sign, so a ray whose verdict is not on a knife edge gets the exact
// answer, and two triangles sharing an edge see it on opposite sides (exact
// signs are antisymmetric, and so is the FP64 value), so no ray slips
// between them.
#include "common.hpp"
#include "prims.hpp"

namespace hra {

// 16 units of 2^-24 per bounded product term: U, V, det and E2.Q carry at
// most 7 to 8 roundings each (the translated inputs, the cross product, the
// dot product), and the recombined third edge function (det - U - V) about 26
// of the 64 units it is given.
constexpr float TRI_K = 16.0f * 5.9604645e-8f;
constexpr int SPILL = 64;           // private overflow entries per lane beyond the LDS stack

__device__ __noinline__ int edge_sign64(float ox, float oy, float oz, float dx, float dy, float dz, float4 P, float4 Q) {
    const double bx = (double)P.x - (double)ox, by = (double)P.y - (double)oy, bz = (double)P.z - (double)oz;
    const double cx = (double)Q.x - (double)ox, cy = (double)Q.y - (double)oy, cz = (double)Q.z - (double)oz;
    const double p1 = by * cz, p2 = bz * cy, p3 = bz * cx, p4 = bx * cz, p5 = bx * cy, p6 = by * cx;
    const double X = p1 - p2, Y = p3 - p4, Z = p5 - p6;
    const double t0 = (double)dx * X, t1 = (double)dy * Y, t2 = (double)dz * Z;
    const double e = (t0 + t1) + t2;
    return (e > 0.0) - (e < 0.0);
}

__device__ __noinline__ int plane_sign64(float ox, float oy, float oz, float4 A, float4 B, float4 C) {
    const double ax = (double)A.x - (double)ox, ay = (double)A.y - (double)oy, az = (double)A.z - (double)oz;
    const double bx = (double)B.x - (double)ox, by = (double)B.y - (double)oy, bz = (double)B.z - (double)oz;
    const double cx = (double)C.x - (double)ox, cy = (double)C.y - (double)oy, cz = (double)C.z - (double)oz;
    const double X = by * cz - bz * cy, Y = bz * cx - bx * cz, Z = bx * cy - by * cx;
    const double h = (ax * X + ay * Y) + az * Z;
    return (h > 0.0) - (h < 0.0);
}

// kd = 6 * TRI_K * max|d_i|, a per-ray constant.  Every product term of U,
// V and det is at most max|d_i| * M^2 and there are six of them; those of
// E2.Q at most M^3.  M has a floor so that a bound never underflows below the
// absolute error of subnormal results.
// The decision when some FP32 sign is uncertain (value 2): the uncertain
// edge functions, and the plane side if the edges agree, in FP64; the rule
// is the one tri_hit applies to trusted signs.  Out of line: rare, and its
// FP64 registers stay out of the traversal loop.
__device__ __noinline__ bool tri_hit_fp64(float ox, float oy, float oz, float dx, float dy, float dz, float4 A, float4 B,
                                          float4 C, int s0, int s1, int s2, int hs) {
    if (s0 == 2) s0 = edge_sign64(ox, oy, oz, dx, dy, dz, B, C);
    if (s1 == 2) s1 = edge_sign64(ox, oy, oz, dx, dy, dz, C, A);
    if (s2 == 2) s2 = edge_sign64(ox, oy, oz, dx, dy, dz, A, B);
    int s;
    if (s0 >= 0 && s1 >= 0 && s2 >= 0 && (s0 | s1 | s2)) s = 1;
    else if (s0 <= 0 && s1 <= 0 && s2 <= 0 && (s0 | s1 | s2)) s = -1;
    else return false;
    if (hs == 2) hs = plane_sign64(ox, oy, oz, A, B, C);
    return hs == s;
}

__device__ inline bool tri_hit(float ox, float oy, float oz, float dx, float dy, float dz, float kd, float4 A, float4 B,
                               float4 C) {
    const float tx = ox - A.x, ty = oy - A.y, tz = oz - A.z;
    const float e1x = B.x - A.x, e1y = B.y - A.y, e1z = B.z - A.z;
    const float e2x = C.x - A.x, e2y = C.y - A.y, e2z = C.z - A.z;
    const float M = fmaxf(fmaxf(fmaxf(fmaxf(fabsf(tx), fabsf(ty)), fmaxf(fabsf(tz), 1e-12f)),
                                fmaxf(fmaxf(fabsf(e1x), fabsf(e1y)), fabsf(e1z))),
                          fmaxf(fmaxf(fabsf(e2x), fabsf(e2y)), fabsf(e2z)));
    const float MM = M * M;
    const float bd = kd * MM;
    const float px = fmaf(dy, e2z, -(dz * e2y)), py = fmaf(dz, e2x, -(dx * e2z)), pz = fmaf(dx, e2y, -(dy * e2x));
    const float U = fmaf(tz, pz, fmaf(ty, py, tx * px));
    const float qx = fmaf(ty, e1z, -(tz * e1y)), qy = fmaf(tz, e1x, -(tx * e1z)), qz = fmaf(tx, e1y, -(ty * e1x));
    const float V = fmaf(dz, qz, fmaf(dy, qy, dx * qx));
    const float det = fmaf(e1z, pz, fmaf(e1y, py, e1x * px));
    const float W = (det - U) - V;
    const float bw = 4.0f * bd;
    const float Tn = fmaf(e2z, qz, fmaf(e2y, qy, e2x * qx));
    const float bt = (6.0f * TRI_K) * MM * M;
    // certain signs as lane masks: P = certainly positive (sign code -1),
    // N = certainly negative (code 1), neither = uncertain (code 2, NaN too)
    const bool uP = U > bd, uN = U < -bd, vP = V > bd, vN = V < -bd;
    const bool wP = W > bw, wN = W < -bw, tP = Tn > bt, tN = Tn < -bt;
    // two certain, opposite edge signs: the line misses the triangle
    const bool miss = (uN || vN || wN) && (uP || vP || wP);
    const bool sure = (uP || uN) && (vP || vN) && (wP || wN) && (tP || tN);
    // no miss and nothing uncertain: the three edges share W's certain sign,
    // and the plane side must equal it
    bool hit = !miss && sure && tP == wP;
    if (!miss && !sure) {
        const int s1 = uP ? -1 : (uN ? 1 : 2), s2 = vP ? -1 : (vN ? 1 : 2);
        const int s0 = wP ? -1 : (wN ? 1 : 2), hs = tP ? -1 : (tN ? 1 : 2);
        hit = tri_hit_fp64(ox, oy, oz, dx, dy, dz, A, B, C, s0, s1, s2, hs);
    }
    return hit;
}

// Slab test, conservative: exact-ray intersections are never rejected.  The
// inverse direction comes from the hardware reciprocal (at most 1 ulp off);
// a component below 1e-30 in magnitude is replaced by +-1e30 in the inverse,
// so no NaN or infinity arises.  Each distance (bound - o) * inv then carries
// at most 4 units of 2^-24 relative error (subtraction, reciprocal,
// product), so tmin and tmax together 8, and the product with the widening
// factor one more: the far distance is widened by 6e-7 > 9 * 2^-24 (cf. Ize
// 2013, "Robust BVH Ray Traversal").
__device__ inline bool slab(float lx, float ly, float lz, float hx, float hy, float hz, float ox, float oy, float oz,
                            float ix, float iy, float iz, float &tn) {
    const float tx0 = (lx - ox) * ix, tx1 = (hx - ox) * ix;
    const float ty0 = (ly - oy) * iy, ty1 = (hy - oy) * iy;
    const float tz0 = (lz - oz) * iz, tz1 = (hz - oz) * iz;
    const float tmin = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
    const float tmax = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1));
    tn = tmin;
    return tmin <= tmax * 1.0000006f;
}

// 1/x for the slab test (see above).
__device__ inline float safe_rcp(float x) {
    return fabsf(x) > 1e-30f ? __builtin_amdgcn_rcpf(x) : copysignf(1e30f, x);
}

// The hierarchy lives in global memory: 16-byte loads through a global
// address-space pointer (global loads rather than flat ones).
typedef float v4f __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));
__device__ inline float4 gload_f4(const void *p) {
    const v4f v = *(const __attribute__((address_space(1))) v4f *)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ inline int4 gload_i4(const void *p) {
    const v4i v = *(const __attribute__((address_space(1))) v4i *)p;
    return make_int4(v.x, v.y, v.z, v.w);
}

struct WorkCount {
    uint32_t nodes = 0;   // interior nodes fetched
    uint32_t tris = 0;    // triangle tests
};

template <bool STATS>
__device__ inline bool leaf_hit(const float4 *__restrict__ tris, int32_t code, float ox, float oy, float oz, float dx,
                                float dy, float dz, float kd, int32_t n_tris_alloc, uint32_t *err, WorkCount &wc) {
    const int first = leaf_first(code), cnt = leaf_count(code);
    if (first + cnt > n_tris_alloc) {
        atomicOr(err, ERR_STACK);
        return true;
    }
    for (int k = 0; k < cnt; ++k) {
        const float4 *t = tris + 3 * (int64_t)(first + k);
        if (STATS) ++wc.tris;
        if (tri_hit(ox, oy, oz, dx, dy, dz, kd, gload_f4(t), gload_f4(t + 1), gload_f4(t + 2))) return true;
    }
    return false;
}

// The per-lane stack is addressed through an LDS-typed pointer: a pop then
// stays an LDS read with a 32-bit address, and cannot be merged with the
// private overflow read into one generic (flat) access.
typedef __attribute__((address_space(3))) int lds_int;

// Guards: a node index outside the array, a leaf run outside the triangle
// array, or more node visits than twice the node count set the error word
// and end the ray, so a malformed hierarchy cannot fault or spin.
template <int STACK, bool STATS>
__device__ inline bool occluded_step(const Node *__restrict__ nodes, const float4 *__restrict__ tris, int32_t root,
                                     float ox, float oy, float oz, float dx, float dy, float dz, lds_int *lds, int lane,
                                     uint32_t *err, int32_t n_nodes_alloc, int32_t n_tris_alloc, WorkCount &wc) {
    const float kd = (6.0f * TRI_K) * fmaxf(fmaxf(fabsf(dx), fabsf(dy)), fabsf(dz));
    if (is_leaf(root)) return leaf_hit<STATS>(tris, root, ox, oy, oz, dx, dy, dz, kd, n_tris_alloc, err, wc);
    if (n_nodes_alloc <= 0) {
        atomicOr(err, ERR_STACK);
        return true;
    }
    const float ix = safe_rcp(dx), iy = safe_rcp(dy), iz = safe_rcp(dz);
    int spill[SPILL];
    int sp = 0;
    int32_t node = root;      // next interior node to visit, or -1: take the stack
    // the leaf under test as a leaf code whose first-triangle and count
    // fields advance together: negative while triangles remain (the count
    // field holds count - 1, so taking a triangle adds 1 - 2^27; after the
    // last one the borrow clears the leaf bit).  A hierarchy holds fewer
    // than 2^27 triangles, so the first-triangle field never carries.
    int32_t tc = 0;
    // A valid hierarchy takes at most one iteration per node visit, stack
    // pop and triangle test, plus the last: fewer than 2 x nodes + triangles
    // + 1.  The count is the wave's (every lane still in the loop has taken
    // each iteration), so it lives in a scalar register; reaching the cap
    // means a cycle or a corrupt index.
    const int64_t cap = 2 * (int64_t)n_nodes_alloc + (int64_t)n_tris_alloc + 64;
    const uint32_t iter_cap = cap < 0xffffffffll ? (uint32_t)cap : 0xffffffffu;
    uint32_t iter = 0;
    const uint32_t last_node = (uint32_t)n_nodes_alloc - 1u, last_tri = (uint32_t)max(n_tris_alloc, 1) - 1u;
    bool hit = false, done = false, bad = false;
    // One unit of work per iteration: a triangle test while the lane holds a
    // leaf, otherwise a stack pop and/or a node visit.  Lanes at a leaf and
    // lanes inside the tree thus advance in the same iteration instead of the
    // tree lanes idling through a leaf loop.  The loop has a single back edge
    // and a single exit (hit, finished or a guard tripped), so the compiler
    // keeps it one loop; the guards (node index, visit budget, leaf run,
    // stack) only set a flag, and an out-of-range node index reads node 0
    // instead, whose contents the exit then discards.  The visit order is that
    // of a plain recursive traversal: hit leaf children first (child 0 before
    // child 1; a second leaf waits on top of the stack), then the nearer
    // interior child, the farther one pushed.
    while (true) {
        // the empty asm hides tc's value from the optimiser, which would
        // otherwise thread "triangles remain" back into an inner loop
        asm volatile("" : "+v"(tc));
        if (tc < 0) {
            // a leaf run outside the triangle array: a clamped (in-range)
            // read, whose verdict the exit below discards
            const uint32_t ti = (uint32_t)tc & 0x07FFFFFFu;
            bad = ti > last_tri;
            const float4 *t = tris + 3 * (uint64_t)min(ti, last_tri);
            if (STATS) ++wc.tris;
            hit = tri_hit(ox, oy, oz, dx, dy, dz, kd, gload_f4(t), gload_f4(t + 1), gload_f4(t + 2));
            tc = (int32_t)((uint32_t)tc + (1u - (1u << 27)));
        } else {
            bool visit = true;
            if (node < 0) {
                if (sp == 0) {
                    done = true;
                    visit = false;
                } else {
                    --sp;
                    int32_t item;
                    if (sp < STACK) item = lds[sp * 64 + lane];
                    else item = spill[sp - STACK];
                    if (is_leaf(item)) {
                        tc = item;
                        visit = false;
                    } else {
                        node = item;
                    }
                }
            }
            if (visit) {
                bad = (uint32_t)node > last_node;
                const Node *nd = nodes + min((uint32_t)node, last_node);
                if (STATS) ++wc.nodes;
                const float4 A = gload_f4(&nd->a), B = gload_f4(&nd->b), C = gload_f4(&nd->c);
                const int4 D = gload_i4(&nd->d);
                float t0, t1;
                const bool h0 = slab(A.x, A.y, A.z, A.w, B.x, B.y, ox, oy, oz, ix, iy, iz, t0);
                const bool h1 = slab(B.z, B.w, C.x, C.y, C.z, C.w, ox, oy, oz, ix, iy, iz, t1);
                const int32_t c0 = D.x, c1 = D.y;
                const bool l0 = h0 && is_leaf(c0), l1 = h1 && is_leaf(c1);
                // hit and interior: l implies h, so h != l (mask logic, no
                // second compare of the child codes)
                const bool g0 = h0 != l0, g1 = h1 != l1;
                if (l0 || l1) tc = l0 ? c0 : c1;
                // at most one push per visit: the second leaf, or the farther
                // of two interior children (a node with two leaf children has
                // no interior one)
                const bool push = (l0 && l1) || (g0 && g1);
                const int32_t pv = (l0 && l1) ? c1 : (t0 <= t1 ? c1 : c0);
                node = (g0 && g1) ? (t0 <= t1 ? c0 : c1) : (g0 ? c0 : (g1 ? c1 : -1));
                if (push) {
                    if (sp < STACK) lds[sp * 64 + lane] = pv;
                    else if (sp < STACK + SPILL) spill[sp - STACK] = pv;
                    else bad = true;
                    ++sp;
                }
            }
        }
        ++iter;
        const bool over = iter > iter_cap;
        bad = bad || over;
        if (hit || done || bad) break;
    }
    if (bad) atomicOr(err, ERR_STACK);
    return hit || bad;
}

// One node visit per iteration, then the triangles of its hit leaf children.
template <int STACK, bool STATS>
__device__ inline bool occluded_leafloop(const Node *__restrict__ nodes, const float4 *__restrict__ tris, int32_t root, float ox,
                                float oy, float oz, float dx, float dy, float dz, lds_int *lds, int lane, uint32_t *err,
                                int32_t n_nodes_alloc, int32_t n_tris_alloc, WorkCount &wc) {
    const float kd = (6.0f * TRI_K) * fmaxf(fmaxf(fabsf(dx), fabsf(dy)), fabsf(dz));
    if (is_leaf(root)) return leaf_hit<STATS>(tris, root, ox, oy, oz, dx, dy, dz, kd, n_tris_alloc, err, wc);
    const float ix = safe_rcp(dx), iy = safe_rcp(dy), iz = safe_rcp(dz);
    int spill[SPILL];
    int sp = 0;
    int32_t node = root;
    int32_t budget = 2 * n_nodes_alloc + 64;
    while (true) {
        if ((uint32_t)node >= (uint32_t)n_nodes_alloc || --budget < 0) {
            atomicOr(err, ERR_STACK);
            return true;
        }
        const Node *nd = nodes + node;
        if (STATS) ++wc.nodes;
        const float4 A = gload_f4(&nd->a), B = gload_f4(&nd->b), C = gload_f4(&nd->c);
        const int4 D = gload_i4(&nd->d);
        float t0, t1;
        const bool h0 = slab(A.x, A.y, A.z, A.w, B.x, B.y, ox, oy, oz, ix, iy, iz, t0);
        const bool h1 = slab(B.z, B.w, C.x, C.y, C.z, C.w, ox, oy, oz, ix, iy, iz, t1);
        const int32_t c0 = D.x, c1 = D.y;
        // the triangles of both hit leaf children in one loop, [f0, f0 + n0)
        // then [f1, f1 + n1): lanes with a leaf on either side test together
        const int32_t n0 = h0 && is_leaf(c0) ? leaf_count(c0) : 0;
        const int32_t n1 = h1 && is_leaf(c1) ? leaf_count(c1) : 0;
        const int32_t f0 = leaf_first(c0), f1 = leaf_first(c1);
        if ((n0 && f0 + n0 > n_tris_alloc) || (n1 && f1 + n1 > n_tris_alloc)) {
            atomicOr(err, ERR_STACK);
            return true;
        }
        for (int32_t k = 0; k < n0 + n1; ++k) {
            const float4 *t = tris + 3 * (int64_t)(k < n0 ? f0 + k : f1 + (k - n0));
            if (STATS) ++wc.tris;
            if (tri_hit(ox, oy, oz, dx, dy, dz, kd, gload_f4(t), gload_f4(t + 1), gload_f4(t + 2))) return true;
        }
        const bool g0 = h0 && !is_leaf(c0), g1 = h1 && !is_leaf(c1);
        if (g0 && g1) {
            const int32_t nearc = t0 <= t1 ? c0 : c1, farc = t0 <= t1 ? c1 : c0;
            if (sp < STACK) lds[sp * 64 + lane] = farc;
            else if (sp < STACK + SPILL) spill[sp - STACK] = farc;
            else {
                atomicOr(err, ERR_STACK);
                return true;
            }
            ++sp;
            node = nearc;
        } else if (g0) {
            node = c0;
        } else if (g1) {
            node = c1;
        } else {
            if (sp == 0) return false;
            --sp;
            if (sp < STACK) node = lds[sp * 64 + lane];
            else node = spill[sp - STACK];
        }
    }
}

// true if some triangle blocks the ray.  Two traversal loops give the same
// visits in the same order and the same results; they differ in how a wave's
// lanes share iterations (HRA_TRAVERSAL_STEP: one unit of work per lane and
// iteration; HRA_TRAVERSAL_LEAF_LOOP: a node visit per iteration followed by
// the hit leaves' triangles).  Which is faster depends on the part.
template <int STACK, bool STATS, bool STEP>
__device__ inline bool occluded(const Node *__restrict__ nodes, const float4 *__restrict__ tris, int32_t root, float ox,
                                float oy, float oz, float dx, float dy, float dz, lds_int *lds, int lane, uint32_t *err,
                                int32_t n_nodes_alloc, int32_t n_tris_alloc, WorkCount &wc) {
    if constexpr (STEP)
        return occluded_step<STACK, STATS>(nodes, tris, root, ox, oy, oz, dx, dy, dz, lds, lane, err, n_nodes_alloc,
                                           n_tris_alloc, wc);
    else
        return occluded_leafloop<STACK, STATS>(nodes, tris, root, ox, oy, oz, dx, dy, dz, lds, lane, err,
                                               n_nodes_alloc, n_tris_alloc, wc);
}

// A value that is the same in every lane, moved to a scalar register.
__device__ inline float uni(float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); }

__device__ inline int32_t uni_i(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline int64_t uni_l(int64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class T> __device__ inline T *uni_p(T *p) { return (T *)uni_l((int64_t)p); }

// A job's fields are wave-uniform; the compiler cannot prove it for values
// loaded from the job table, so they are moved to scalar registers here (the
// hierarchy pointers, sizes and root then cost no vector registers).
__device__ inline CastJob uni_job(const CastJob &j) {
    CastJob u;
    u.nodes = uni_p(j.nodes);
    u.tris = uni_p(j.tris);
    u.meta = uni_p(j.meta);
    u.origin = uni_p(j.origin);
    u.normal = uni_p(j.normal);
    u.bits = uni_p(j.bits);
    u.n_samples = uni_l(j.n_samples);
    u.item_base = uni_l(j.item_base);
    u.n_nodes_alloc = uni_i(j.n_nodes_alloc);
    u.pad = 0;
    return u;
}

// Job of a wave-uniform work item: the last job whose item_base <= item.
__device__ inline CastJob job_of(const CastArgs &a, int64_t item) {
    if (!a.jobs) return a.job0;
    int lo = 0, hi = a.n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.jobs[mid].item_base <= item) lo = mid;
        else hi = mid - 1;
    }
    return a.jobs[lo];
}

// Hemisphere cast.  One work item = one sample, all N directions, on one
// workgroup of four wavefronts.  The directions are walked in the table's
// traversal order (a space-filling curve over the hemisphere) in steps of
// 256: the four waves take four neighbouring 64-direction patches, so every
// ray in flight in the workgroup starts at the same origin with a nearby
// direction and they traverse nearly the same nodes (shared in L1, little
// divergence).  Each lane ORs its verdict into the sample's bit row in LDS
// at the direction's canonical index; the finished row is stored with
// coalesced writes.  The item index is the block index, uniform over the
// workgroup, so both barriers are reached by every thread, and the kernel
// has no cross-lane operation.  The step loop runs at eight waves per SIMD
// (64 VGPRs, none spilled; with the default 16-entry stack nine workgroups
// fit in LDS, 16.6 KB each), the leaf loop at seven (72 VGPRs; at eight it
// spills and is slower).
template <int RPW, int STACK, bool STATS, bool STEP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(STEP ? 8 : 7))) void k_cast_rows(CastArgs a) {
    extern __shared__ int dyn_lds[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if ((int64_t)blockIdx.x >= a.n_items) return;  // the whole workgroup leaves together
    // workgroups running at the same time take nearby samples when an order
    // is given, and so share the hierarchy's nodes in L2
    const int64_t item = a.order ? (int64_t)uni_i(a.order[blockIdx.x]) : (int64_t)blockIdx.x;
    if ((uint64_t)item >= (uint64_t)a.n_items) {   // not a permutation of the items: an error, no access
        if (threadIdx.x == 0) atomicOr(a.err, ERR_BAD_ORDER);
        return;
    }
    lds_int *lds = (lds_int *)(dyn_lds + wv * (STACK * 64));
    uint32_t *row = (uint32_t *)(dyn_lds + 4 * STACK * 64);
    const CastJob J = uni_job(job_of(a, item));
    const PartMeta &P = *J.meta;
    const int32_t root = uni_i(P.root);
    const int32_t n_valid = uni_i(P.n_valid);
    const bool empty = n_valid <= 0;
    const int32_t n_tris_alloc = uni_i(P.leaf_lo) + n_valid;   // end of this part's leaf run
    const int64_t s = item - J.item_base;
    // the sample, its normal and frame are the same for the whole
    // workgroup: keep them in scalar registers
    const float ox = uni(J.origin[3 * s]), oy = uni(J.origin[3 * s + 1]), oz = uni(J.origin[3 * s + 2]);
    const float nx = uni(J.normal[3 * s]), ny = uni(J.normal[3 * s + 1]), nz = uni(J.normal[3 * s + 2]);
    float3 t0, b0;
    onb_frame(nx, ny, nz, t0, b0);
    const float3 t = make_float3(uni(t0.x), uni(t0.y), uni(t0.z)), b = make_float3(uni(b0.x), uni(b0.y), uni(b0.z));
    for (int32_t w = threadIdx.x; w < a.W; w += 256) row[w] = 0u;
    __syncthreads();
    WorkCount wc;
    for (int32_t c = 0; c < a.n_dirs; c += 4 * RPW) {
#pragma unroll
        for (int r = 0; r < RPW / 64; ++r) {
            const int32_t j = c + r * 256 + wv * 64 + lane;
            uint32_t bit = 0u;
            int32_t idx = 0;
            if (j < a.n_dirs) {
                const float4 l = a.dirs_order[j];
                idx = __float_as_int(l.w);
                const float3 d = rotate_dir(t, b, nx, ny, nz, l.x, l.y, l.z);
                const bool free_ray = empty || !occluded<STACK, STATS, STEP>(J.nodes, J.tris, root, ox, oy, oz, d.x, d.y,
                                                                      d.z, lds, lane, a.err, J.n_nodes_alloc,
                                                                      n_tris_alloc, wc);
                bit = (uint32_t)free_ray << (idx & 31);
            }
            atomicOr(&row[idx >> 5], bit);
        }
    }
    __syncthreads();
    for (int32_t w = threadIdx.x; w < a.W; w += 256) J.bits[s * a.W + w] = row[w];
    if (STATS) {
        atomicAdd(a.work, (unsigned long long)wc.nodes);
        atomicAdd(a.work + 1, (unsigned long long)wc.tris);
    }
}

// Hemisphere cast with several samples per workgroup, for direction counts
// that would leave lanes of a one-sample workgroup idle (150 directions fill
// 150 of 256 lanes; five samples fill 750 of 768).  Work item = `group`
// consecutive samples of one job; lane k of the workgroup takes rays k,
// k + 256, ... of the flattened (sample, direction) list, so a wave's lanes
// hold consecutive directions of one sample, or of two at a boundary.  The
// origin is per lane here, not per workgroup; the rays, the test and the
// bits are those of k_cast_rows.
template <int STACK, bool STATS, bool STEP>
// Seven waves per SIMD: the per-lane origin takes three more registers than
// k_cast_rows, which at eight waves (64 registers) would spill.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) void k_cast_rows_grouped(CastArgs a) {
    extern __shared__ int dyn_lds[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t item = blockIdx.x;
    if (item >= a.n_items) return;  // the whole workgroup leaves together
    lds_int *lds = (lds_int *)(dyn_lds + wv * (STACK * 64));
    uint32_t *row = (uint32_t *)(dyn_lds + 4 * STACK * 64);
    const CastJob J = uni_job(job_of(a, item));
    const PartMeta &P = *J.meta;
    const int32_t root = uni_i(P.root);
    const int32_t n_valid = uni_i(P.n_valid);
    const bool empty = n_valid <= 0;
    const int32_t n_tris_alloc = uni_i(P.leaf_lo) + n_valid;
    const int32_t G = uni_i(a.group), N = uni_i(a.n_dirs), W = uni_i(a.W);
    const int64_t s0 = (item - J.item_base) * G;
    const int64_t left = J.n_samples - s0;
    const int32_t g_n = uni_i((int32_t)(left < G ? left : G));   // samples of this item
    const int32_t total = g_n * N;
    for (int32_t w = threadIdx.x; w < g_n * W; w += 256) row[w] = 0u;
    __syncthreads();
    WorkCount wc;
    for (int32_t c = 0; c < total; c += 256) {
        const int32_t jf = c + wv * 64 + lane;
        uint32_t bit = 0u;
        int32_t pos = 0;   // bit position in the workgroup's rows: word pos >> 5, bit pos & 31
        if (jf < total) {
            const int32_t g = jf / N;
            const int32_t j = jf - g * N;
            const int64_t s = s0 + g;
            const float ox = J.origin[3 * s], oy = J.origin[3 * s + 1], oz = J.origin[3 * s + 2];
            const float nx = J.normal[3 * s], ny = J.normal[3 * s + 1], nz = J.normal[3 * s + 2];
            float3 t, b;
            onb_frame(nx, ny, nz, t, b);
            const float4 l = a.dirs_order[j];
            pos = g * W * 32 + __float_as_int(l.w);
            const float3 d = rotate_dir(t, b, nx, ny, nz, l.x, l.y, l.z);
            const bool free_ray = empty || !occluded<STACK, STATS, STEP>(J.nodes, J.tris, root, ox, oy, oz, d.x, d.y,
                                                                  d.z, lds, lane, a.err, J.n_nodes_alloc,
                                                                  n_tris_alloc, wc);
            bit = (uint32_t)free_ray << (pos & 31);
        }
        atomicOr(&row[pos >> 5], bit);
    }
    __syncthreads();
    for (int32_t w = threadIdx.x; w < g_n * W; w += 256) J.bits[s0 * W + w] = row[w];
    if (STATS) {
        atomicAdd(a.work, (unsigned long long)wc.nodes);
        atomicAdd(a.work + 1, (unsigned long long)wc.tris);
    }
}

// One unit of the step loop for a lane's current ray in the refilled casts:
// a triangle test while the lane holds a leaf, else a stack pop and/or a node
// visit, in the visit order of occluded_step.  `win` bounds the near
// distance of a box that is entered (WINDOW; otherwise unbounded), in units
// of the ray's direction; triangles take the exact half-line test.  Sets
// hit, done (stack empty) or bad (a guard tripped).
template <int STACK, bool STATS, bool WINDOW>
__device__ __forceinline__ void step_unit(const CastJob &J, float ox, float oy, float oz, float dx, float dy, float dz,
                                          float ix, float iy, float iz, float kd, float win, lds_int *lds, int lane,
                                          int *spill, uint32_t last_node, uint32_t last_tri, int32_t &node, int32_t &sp,
                                          int32_t &ti, int32_t &tn, WorkCount &wc, bool &hit, bool &done, bool &bad) {
    asm volatile("" : "+v"(tn));
    if (tn > 0) {
        bad = (uint32_t)ti > last_tri;
        const float4 *tp = J.tris + 3 * (uint64_t)min((uint32_t)ti, last_tri);
        if (STATS) ++wc.tris;
        hit = tri_hit(ox, oy, oz, dx, dy, dz, kd, gload_f4(tp), gload_f4(tp + 1), gload_f4(tp + 2));
        ++ti;
        --tn;
        return;
    }
    bool visit = true;
    if (node < 0) {
        if (sp == 0) {
            done = true;
            visit = false;
        } else {
            --sp;
            int32_t itm;
            if (sp < STACK) itm = lds[sp * 64 + lane];
            else itm = spill[sp - STACK];
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
        bad = (uint32_t)node > last_node;
        const Node *nd = J.nodes + min((uint32_t)node, last_node);
        if (STATS) ++wc.nodes;
        const float4 A = gload_f4(&nd->a), B = gload_f4(&nd->b), C = gload_f4(&nd->c);
        const int4 D = gload_i4(&nd->d);
        float t0, t1;
        bool h0 = slab(A.x, A.y, A.z, A.w, B.x, B.y, ox, oy, oz, ix, iy, iz, t0);
        bool h1 = slab(B.z, B.w, C.x, C.y, C.z, C.w, ox, oy, oz, ix, iy, iz, t1);
        if (WINDOW) {
            h0 = h0 && t0 <= win;
            h1 = h1 && t1 <= win;
        }
        const int32_t c0 = D.x, c1 = D.y;
        const bool l0 = h0 && is_leaf(c0), l1 = h1 && is_leaf(c1);
        const bool g0 = h0 != l0, g1 = h1 != l1;   // hit and interior (l implies h)
        if (l0 || l1) {
            const int32_t lc = l0 ? c0 : c1;
            ti = leaf_first(lc);
            tn = leaf_count(lc);
        }
        const bool push = (l0 && l1) || (g0 && g1);
        const int32_t pv = (l0 && l1) ? c1 : (t0 <= t1 ? c1 : c0);
        node = (g0 && g1) ? (t0 <= t1 ? c0 : c1) : (g0 ? c0 : (g1 ? c1 : -1));
        if (push) {
            if (sp < STACK) lds[sp * 64 + lane] = pv;
            else if (sp < STACK + SPILL) spill[sp - STACK] = pv;
            else bad = true;
            ++sp;
        }
    }
}

// Hemisphere cast with refilled lanes.  The work item's rays (one sample's
// directions in traversal order, or `group` samples' in a row) form a list
// behind a workgroup counter in LDS.  A lane runs the step loop above on one
// ray at a time; when its ray ends it records the bit and goes idle, and the
// idle lanes of a wave take the next rays of the list together once at
// least REFILL_K of them wait (or the whole wave does).  A wave thus stops
// waiting for its slowest ray before the next 64 start, while rays that
// start together stay neighbours on the hemisphere.  Lanes coordinate only
// through LDS words (the list counter and one idle count per wave, read by
// the whole wave at the top of each iteration), never through cross-lane
// instructions.  Each ray keeps the step loop's visit order, work counts and
// guards (its own iteration cap), so bits and counts equal those of
// k_cast_rows and k_cast_rows_grouped.
constexpr int REFILL_K = 8;

__device__ inline int lds_peek(int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }

template <int STACK, bool STATS, bool GROUPED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GROUPED ? 7 : 8))) void k_cast_refill(CastArgs a) {
    extern __shared__ int dyn_lds[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t item = blockIdx.x;
    if (item >= a.n_items) return;  // the whole workgroup leaves together
    lds_int *lds = (lds_int *)(dyn_lds + wv * (STACK * 64));
    const CastJob J = uni_job(job_of(a, item));
    const PartMeta &P = *J.meta;
    const int32_t root = uni_i(P.root);
    const int32_t n_valid = uni_i(P.n_valid);
    const bool empty = n_valid <= 0;
    const int32_t n_tris_alloc = uni_i(P.leaf_lo) + n_valid;
    const int32_t N = uni_i(a.n_dirs), W = uni_i(a.W);
    const int32_t G = GROUPED ? uni_i(a.group) : 1;
    const int64_t s0 = (item - J.item_base) * G;
    int32_t g_n = 1;
    if (GROUPED) {
        const int64_t left = J.n_samples - s0;
        g_n = uni_i((int32_t)(left < G ? left : G));
    }
    const int32_t total = g_n * N;
    uint32_t *row = (uint32_t *)(dyn_lds + 4 * STACK * 64);
    int *ctr = dyn_lds + 4 * STACK * 64 + g_n * W;   // [0] next ray, [1 + w] idle lanes of wave w
    for (int32_t w = threadIdx.x; w < g_n * W; w += 256) row[w] = 0u;
    if (threadIdx.x == 0) ctr[0] = 0;
    if (threadIdx.x < 4) ctr[1 + threadIdx.x] = 64;
    // one sample per item: origin and frame are the workgroup's, in scalar
    // registers
    float uox = 0.f, uoy = 0.f, uoz = 0.f, unx = 0.f, uny = 0.f, unz = 1.f;
    float3 ut = make_float3(1.f, 0.f, 0.f), ub = make_float3(0.f, 1.f, 0.f);
    if (!GROUPED) {
        uox = uni(J.origin[3 * s0]);
        uoy = uni(J.origin[3 * s0 + 1]);
        uoz = uni(J.origin[3 * s0 + 2]);
        unx = uni(J.normal[3 * s0]);
        uny = uni(J.normal[3 * s0 + 1]);
        unz = uni(J.normal[3 * s0 + 2]);
        float3 t0, b0;
        onb_frame(unx, uny, unz, t0, b0);
        ut = make_float3(uni(t0.x), uni(t0.y), uni(t0.z));
        ub = make_float3(uni(b0.x), uni(b0.y), uni(b0.z));
    }
    // reciprocal of N for splitting a list position into (sample, direction)
    const float rN = 1.0f / (float)N;
    __syncthreads();
    WorkCount wc;
    if (empty) {
        // no triangle: every ray is free
        for (int32_t q = threadIdx.x; q < total; q += 256) {
            int32_t g = GROUPED ? (int32_t)((float)q * rN) : 0;
            g -= (g * N > q);
            g += ((g + 1) * N <= q);
            const int32_t j = q - g * N;
            const int32_t pos = g * W * 32 + __float_as_int(a.dirs_order[j].w);
            atomicOr(&row[pos >> 5], 1u << (pos & 31));
        }
    } else {
        const float ZERO = 0.0f;
        const int64_t cap = 2 * (int64_t)J.n_nodes_alloc + (int64_t)n_tris_alloc + 64;
        const uint32_t iter_cap = cap < 0xffffffffll ? (uint32_t)cap : 0xffffffffu;
        const uint32_t last_node = (uint32_t)J.n_nodes_alloc - 1u, last_tri = (uint32_t)max(n_tris_alloc, 1) - 1u;
        const bool root_leaf = is_leaf(root);
        bool active = false;
        float ox = uox, oy = uoy, oz = uoz, dx = ZERO, dy = ZERO, dz = ZERO, ix = ZERO, iy = ZERO, iz = ZERO, kd = ZERO;
        int32_t node = -1, sp = 0, ti = 0, tn = 0, pos = 0;
        uint32_t iter = 0;
        int spill[SPILL];
        while (true) {
            const int n_idle = lds_peek(ctr + 1 + wv);
            const int nxt = lds_peek(ctr);
            if (nxt >= total && n_idle == 64) break;
            if (n_idle >= REFILL_K && nxt < total && !active) {
                const int32_t q = atomicAdd(ctr, 1);
                if (q < total) {
                    int32_t g = 0;
                    float px = uox, py = uoy, pz = uoz, nx = unx, ny = uny, nz = unz;
                    float3 t = ut, b = ub;
                    if (GROUPED) {
                        g = (int32_t)((float)q * rN);
                        g -= (g * N > q);
                        g += ((g + 1) * N <= q);
                        const int64_t smp = s0 + g;
                        px = J.origin[3 * smp];
                        py = J.origin[3 * smp + 1];
                        pz = J.origin[3 * smp + 2];
                        nx = J.normal[3 * smp];
                        ny = J.normal[3 * smp + 1];
                        nz = J.normal[3 * smp + 2];
                        onb_frame(nx, ny, nz, t, b);
                    }
                    const int32_t j = q - g * N;
                    const float4 l = a.dirs_order[j];
                    pos = g * W * 32 + __float_as_int(l.w);
                    const float3 d = rotate_dir(t, b, nx, ny, nz, l.x, l.y, l.z);
                    if (GROUPED) {
                        ox = px;
                        oy = py;
                        oz = pz;
                    }
                    dx = d.x;
                    dy = d.y;
                    dz = d.z;
                    kd = (6.0f * TRI_K) * fmaxf(fmaxf(fabsf(dx), fabsf(dy)), fabsf(dz));
                    ix = safe_rcp(dx);
                    iy = safe_rcp(dy);
                    iz = safe_rcp(dz);
                    // a root that is a leaf: its triangles first, no node
                    node = root_leaf ? -1 : root;
                    ti = root_leaf ? leaf_first(root) : 0;
                    tn = root_leaf ? leaf_count(root) : 0;
                    sp = 0;
                    iter = 0;
                    active = true;
                    atomicSub(ctr + 1 + wv, 1);
                }
            }
            if (active) {
                // one sample per item: the origin stays in scalar registers
                const float rox = GROUPED ? ox : uox, roy = GROUPED ? oy : uoy, roz = GROUPED ? oz : uoz;
                bool hit = false, done = false, bad = false;
                step_unit<STACK, STATS, false>(J, rox, roy, roz, dx, dy, dz, ix, iy, iz, kd, 0.0f, lds, lane, spill,
                                               last_node, last_tri, node, sp, ti, tn, wc, hit, done, bad);
                ++iter;
                bad = bad || iter > iter_cap;
                if (hit || done || bad) {
                    if (!(hit || bad)) atomicOr(&row[pos >> 5], 1u << (pos & 31));
                    if (bad) atomicOr(a.err, ERR_STACK);
                    active = false;
                    atomicAdd(ctr + 1 + wv, 1);
                }
            }
        }
    }
    __syncthreads();
    for (int32_t w = threadIdx.x; w < g_n * W; w += 256) J.bits[s0 * W + w] = row[w];
    if (STATS) {
        atomicAdd(a.work, (unsigned long long)wc.nodes);
        atomicAdd(a.work + 1, (unsigned long long)wc.tris);
    }
}

// Six-axis cast.  Axis rays are few (six per sample) but some are long: a
// ray that runs along a wall, tangent to it, passes one box after another for
// hundreds of node visits, while the median ray takes one step.  Cast one
// ray per lane, a wavefront would iterate until its slowest lane ended, with
// a few lanes busy: the kernel would be bound by issue slots spent on idle
// lanes and then by a handful of dependent chains.  Here a workgroup takes
// AX_GROUP samples and runs two phases, each over a list in LDS from which
// every lane takes the next entry when its own ends (as in k_cast_refill):
//   1. every cast ray (n . D >= 0; a ray pointing into the material is not
//      cast), whole, for at most AX_BUDGET iterations of the step loop; a ray
//      still undecided then is marked open;
//   2. every open ray, cut into AX_SEGS pieces.
// Each sample's six verdicts sit in an LDS word (bit k set while ray k is
// free, bit 8 + k while it is open).
//
// Piece s of the ray o + t e (e = +-e_c) starts at o_s, equal to o but for
// its c coordinate o_c + sign * t_exit s / AX_SEGS in FP32 (t_exit the
// distance from o to the part's box face along e), so o_s lies on the ray at
// or beyond o; it is the half-line from o_s whose boxes are entered within
// win_s = |o_{s+1,c} - o_{s,c}| (1 + 1e-6) (the last piece: unbounded).
// Consecutive pieces meet exactly (the same FP32 expression) and win_s
// exceeds the slab test's relative error, so the windows cover the ray.  A
// triangle a piece reports is hit by the half-line from o_s, hence by the
// ray.  A triangle the ray hits at t is reported by the piece whose window
// holds t: an axis ray's edge functions do not involve o_c (the c column of
// the direction's cross products is zero), so they equal the unsplit ray's,
// and only the plane side depends on the origin, which decides as for the
// unsplit ray when o_s lies before the hit (a hit exactly at o_s is reported
// by the piece before).  So the bits equal those of one unsplit cast.
constexpr int AX_GROUP = 128;
constexpr uint32_t AX_BUDGET = 48;
constexpr int AX_SEGS = 16;
// Most samples in one work item of the grouped hemisphere cast.
constexpr int MAX_GROUP = 16;

// One phase of k_cast_axes: the `total` entries of the phase's list, taken
// by refilled lanes.  SPLIT: entry = (open ray, piece), else a whole ray.
template <int STACK, bool STATS, bool SPLIT>
__device__ __forceinline__ void axes_phase(const CastArgs &a, const CastJob &J, const PartMeta &P, int64_t s0,
                                           const int32_t *list, int32_t total, uint32_t *word, int *ctr, lds_int *lds,
                                           int lane, int wv, int32_t root, uint32_t iter_cap, uint32_t last_node,
                                           uint32_t last_tri, WorkCount &wc) {
    const bool root_leaf = is_leaf(root);
    const float inv_segs = 1.0f / (float)AX_SEGS;
    const float ZERO = 0.0f;
    bool active = false;
    float ox = ZERO, oy = ZERO, oz = ZERO, dx = ZERO, dy = ZERO, dz = ZERO, ix = ZERO, iy = ZERO, iz = ZERO;
    float kd = ZERO, win = ZERO;
    int32_t node = -1, sp = 0, ti = 0, tn = 0, g = 0, k = 0;
    uint32_t iter = 0;
    int spill[SPILL];
    while (true) {
        const int n_idle = lds_peek(ctr + 2 + wv);
        const int nxt = lds_peek(ctr + 1);
        if (nxt >= total && n_idle == 64) break;
        if (!active && nxt < total) {
            const int32_t q = atomicAdd(ctr + 1, 1);
            if (q < total) {
                const int32_t e = SPLIT ? q / AX_SEGS : q, seg = SPLIT ? q - e * AX_SEGS : 0;
                const int32_t code = list[e];
                g = code >> 3;
                k = code & 7;
                const int64_t smp = s0 + g;
                const float4 l = a.dirs[k];
                const float px = J.origin[3 * smp], py = J.origin[3 * smp + 1], pz = J.origin[3 * smp + 2];
                bool run = true;
                ox = px;
                oy = py;
                oz = pz;
                win = 1e30f;
                if (SPLIT) {
                    run = ((uint32_t)__hip_atomic_load(word + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >> k) & 1u;
                    const int c = l.x != 0.0f ? 0 : (l.y != 0.0f ? 1 : 2);
                    const float sg = c == 0 ? l.x : (c == 1 ? l.y : l.z);
                    const float oc = c == 0 ? px : (c == 1 ? py : pz);
                    const float t_exit = sg > 0.0f ? P.bbox[3 + c] - oc : oc - P.bbox[c];
                    if (!(t_exit > 0.0f)) {
                        // the origin is on or past the box face: one unbounded piece
                        run = run && seg == 0;
                    } else {
                        const float oa = oc + sg * (t_exit * ((float)seg * inv_segs));
                        const float ob = oc + sg * (t_exit * ((float)(seg + 1) * inv_segs));
                        if (seg != AX_SEGS - 1) win = fabsf(ob - oa) * 1.000001f;
                        ox = c == 0 ? oa : px;
                        oy = c == 1 ? oa : py;
                        oz = c == 2 ? oa : pz;
                    }
                }
                if (run) {
                    dx = l.x;
                    dy = l.y;
                    dz = l.z;
                    kd = (6.0f * TRI_K) * fmaxf(fmaxf(fabsf(dx), fabsf(dy)), fabsf(dz));
                    ix = safe_rcp(dx);
                    iy = safe_rcp(dy);
                    iz = safe_rcp(dz);
                    node = root_leaf ? -1 : root;
                    ti = root_leaf ? leaf_first(root) : 0;
                    tn = root_leaf ? leaf_count(root) : 0;
                    sp = 0;
                    iter = 0;
                    active = true;
                    atomicSub(ctr + 2 + wv, 1);
                }
            }
        }
        if (active) {
            bool hit = false, done = false, bad = false;
            step_unit<STACK, STATS, SPLIT>(J, ox, oy, oz, dx, dy, dz, ix, iy, iz, kd, win, lds, lane, spill, last_node,
                                           last_tri, node, sp, ti, tn, wc, hit, done, bad);
            ++iter;
            bad = bad || iter > iter_cap;
            const bool open = !SPLIT && !(hit || done || bad) && iter >= AX_BUDGET;
            if (hit || done || bad || open) {
                if (hit || bad) atomicAnd(word + g, ~(1u << k));
                if (open) atomicOr(word + g, 1u << (8 + k));
                if (bad) atomicOr(a.err, ERR_STACK);
                active = false;
                atomicAdd(ctr + 2 + wv, 1);
            }
        }
    }
}

template <int STACK, bool STATS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_cast_axes(CastArgs a) {
    __shared__ int stk[4 * STACK * 64];
    __shared__ uint32_t word[AX_GROUP];
    __shared__ int32_t list[6 * AX_GROUP];   // the phase's rays: 8 * sample + axis
    __shared__ int ctr[6];                   // [0] list length, [1] next entry, [2 + w] idle lanes of wave w
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t item = blockIdx.x;
    if (item >= a.n_items) return;  // the whole workgroup leaves together
    lds_int *lds = (lds_int *)(stk + wv * (STACK * 64));
    const CastJob J = uni_job(job_of(a, item));
    const PartMeta &P = *J.meta;
    const int32_t root = uni_i(P.root);
    const int32_t n_valid = uni_i(P.n_valid);
    const bool empty = n_valid <= 0;
    const int32_t n_tris_alloc = uni_i(P.leaf_lo) + n_valid;
    const int64_t s0 = (item - J.item_base) * AX_GROUP;
    const int64_t left = J.n_samples - s0;
    const int32_t g_n = uni_i((int32_t)(left < AX_GROUP ? left : AX_GROUP));
    if (threadIdx.x < AX_GROUP) word[threadIdx.x] = 0u;
    if (threadIdx.x < 6) ctr[threadIdx.x] = threadIdx.x < 2 ? 0 : 64;
    __syncthreads();
    for (int32_t q = threadIdx.x; q < 6 * g_n; q += 256) {
        const int32_t g = q / 6, k = q - 6 * g;
        const int64_t smp = s0 + g;
        const float4 l = a.dirs[k];
        const float q0 = J.normal[3 * smp] * l.x, q1 = J.normal[3 * smp + 1] * l.y, q2 = J.normal[3 * smp + 2] * l.z;
        if (!(((q0 + q1) + q2) < 0.0f)) {
            atomicOr(word + g, 1u << k);
            list[atomicAdd(ctr, 1)] = 8 * g + k;
        }
    }
    __syncthreads();
    WorkCount wc;
    if (!empty) {
        const int64_t cap = 2 * (int64_t)J.n_nodes_alloc + (int64_t)n_tris_alloc + 64;
        const uint32_t iter_cap = cap < 0xffffffffll ? (uint32_t)cap : 0xffffffffu;
        const uint32_t last_node = (uint32_t)J.n_nodes_alloc - 1u, last_tri = (uint32_t)max(n_tris_alloc, 1) - 1u;
        axes_phase<STACK, STATS, false>(a, J, P, s0, list, uni_i(ctr[0]), word, ctr, lds, lane, wv, root, iter_cap,
                                        last_node, last_tri, wc);
        __syncthreads();
        if (threadIdx.x < 6) ctr[threadIdx.x] = threadIdx.x < 2 ? 0 : 64;
        __syncthreads();
        for (int32_t q = threadIdx.x; q < 6 * g_n; q += 256) {
            const int32_t g = q / 6, k = q - 6 * g;
            if ((word[g] >> (8 + k)) & 1u) list[atomicAdd(ctr, 1)] = 8 * g + k;
        }
        __syncthreads();
        const int32_t n_open = uni_i(ctr[0]);
        if (n_open > 0)   // uniform: every thread reads the same count after the barrier
            axes_phase<STACK, STATS, true>(a, J, P, s0, list, n_open * AX_SEGS, word, ctr, lds, lane, wv, root,
                                           iter_cap, last_node, last_tri, wc);
    }
    __syncthreads();
    for (int32_t w = threadIdx.x; w < g_n; w += 256) J.bits[s0 + w] = word[w] & 63u;
    if (STATS) {
        atomicAdd(a.work, (unsigned long long)wc.nodes);
        atomicAdd(a.work + 1, (unsigned long long)wc.tris);
    }
}

__global__ void k_popcount_rows(const uint32_t *bits, int64_t n, int32_t W, uint32_t *counts) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    uint32_t c = 0;
    for (int32_t w = 0; w < W; ++w) c += __popc(bits[s * W + w]);
    counts[s] = c;
}

template <int STACK, bool STATS>
static hipError_t launch_refill(const CastArgs &args, hipStream_t s) {
    const int64_t blocks = args.n_items;
    if (blocks >= ((int64_t)1 << 31) || args.group > MAX_GROUP) return hipErrorInvalidValue;
    const size_t lds = sizeof(int) * (4 * STACK * 64 + (size_t)args.W * (args.group > 1 ? args.group : 1) + 8);
    if (args.group > 1) k_cast_refill<STACK, STATS, true><<<(unsigned)blocks, 256, lds, s>>>(args);
    else k_cast_refill<STACK, STATS, false><<<(unsigned)blocks, 256, lds, s>>>(args);
    return hipGetLastError();
}

template <int RPW, int STACK, bool STATS, bool STEP>
static hipError_t launch_cast(const CastArgs &args, hipStream_t s) {
    if (args.kind == 1) {
        const int64_t blocks = args.n_items;             // AX_GROUP samples per block
        if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
        k_cast_axes<STACK, STATS><<<(unsigned)blocks, 256, 0, s>>>(args);
    } else if (args.group > 1) {
        const int64_t blocks = args.n_items;             // `group` samples per block
        if (blocks >= ((int64_t)1 << 31) || args.group > MAX_GROUP) return hipErrorInvalidValue;
        const size_t lds = sizeof(int) * (4 * STACK * 64 + (size_t)args.W * args.group);
        k_cast_rows_grouped<STACK, STATS, STEP><<<(unsigned)blocks, 256, lds, s>>>(args);
    } else {
        const int64_t blocks = args.n_items;             // one sample per block
        if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
        const size_t lds = sizeof(int) * (4 * STACK * 64 + (size_t)args.W);
        k_cast_rows<RPW, STACK, STATS, STEP><<<(unsigned)blocks, 256, lds, s>>>(args);
    }
    return hipGetLastError();
}

template <int RPW, bool STATS, bool STEP>
static hipError_t launch_rpw(const CastArgs &a, int stack, hipStream_t s) {
    switch (stack) {
        case 16: return launch_cast<RPW, 16, STATS, STEP>(a, s);
        case 20: return launch_cast<RPW, 20, STATS, STEP>(a, s);
        case 32: return launch_cast<RPW, 32, STATS, STEP>(a, s);
        default: return launch_cast<RPW, 24, STATS, STEP>(a, s);
    }
}

template <bool STEP>
static hipError_t launch_mode(const CastArgs &a, int rpw, int stack, bool stats, hipStream_t s) {
    if (stats) return launch_rpw<64, true, STEP>(a, stack, s);
    switch (rpw) {
        case 128: return launch_rpw<128, false, STEP>(a, stack, s);
        case 256: return launch_rpw<256, false, STEP>(a, stack, s);
        default: return launch_rpw<64, false, STEP>(a, stack, s);
    }
}

hipError_t launch_cast_any(const CastArgs &a, int rpw, int stack, int traversal, bool stats, hipStream_t s) {
    if (traversal == HRA_TRAVERSAL_REFILL && a.kind == 0) {
        // the hemisphere cast with refilled lanes (the six-axis cast keeps
        // the step loop: ten samples per wave, no list to refill from)
        switch (stack) {
            case 16: return stats ? launch_refill<16, true>(a, s) : launch_refill<16, false>(a, s);
            case 20: return stats ? launch_refill<20, true>(a, s) : launch_refill<20, false>(a, s);
            case 32: return stats ? launch_refill<32, true>(a, s) : launch_refill<32, false>(a, s);
            default: return stats ? launch_refill<24, true>(a, s) : launch_refill<24, false>(a, s);
        }
    }
    return traversal == HRA_TRAVERSAL_LEAF_LOOP ? launch_mode<false>(a, rpw, stack, stats, s)
                                                : launch_mode<true>(a, rpw, stack, stats, s);
}

int32_t cast_group(int32_t n_dirs, int32_t setting) {
    if (setting > 0) return setting;
    if (n_dirs <= 0 || n_dirs >= 256) return 1;
    int32_t best = 1;
    double best_fill = 0.0;
    for (int32_t g = 1; g <= MAX_GROUP; ++g) {
        const int64_t rays = (int64_t)g * n_dirs, slots = (rays + 255) / 256 * 256;
        const double fill = (double)rays / (double)slots;
        if (fill > best_fill + 1e-12) {
            best_fill = fill;
            best = g;
        }
    }
    return best;
}

int64_t cast_items(int32_t kind, int64_t n_samples, int32_t group) {
    if (kind == 1) return (n_samples + AX_GROUP - 1) / AX_GROUP;
    return group > 1 ? (n_samples + group - 1) / group : n_samples;
}

// The rays as the cast forms them: out[i][j] = (o, d).
__global__ void k_debug_rays(const float *origin, const float *normal, const int64_t *idx, int64_t n_idx, int64_t n_samples,
                             const float4 *dirs, int32_t n_dirs, int32_t kind, float *out) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_idx * n_dirs) return;
    const int64_t k = g / n_dirs;
    const int32_t j = (int32_t)(g % n_dirs);
    const int64_t s = idx[k];
    float *o6 = out + 6 * g;
    if (s < 0 || s >= n_samples) {
        for (int q = 0; q < 6; ++q) o6[q] = __int_as_float(0x7fc00000);
        return;
    }
    const float nx = normal[3 * s], ny = normal[3 * s + 1], nz = normal[3 * s + 2];
    float3 t, b;
    onb_frame(nx, ny, nz, t, b);
    const float4 l = dirs[j];
    float3 d = kind == 0 ? rotate_dir(t, b, nx, ny, nz, l.x, l.y, l.z) : make_float3(l.x, l.y, l.z);
    o6[0] = origin[3 * s];
    o6[1] = origin[3 * s + 1];
    o6[2] = origin[3 * s + 2];
    o6[3] = d.x;
    o6[4] = d.y;
    o6[5] = d.z;
}

}  // namespace hra

using namespace hra;

extern "C" hra_status hra_set_cast_config(hra_ctx *ctx, const hra_cast_config *cfg) {
    if (!ctx || !cfg) return HRA_ERR_INVALID_ARG;
    if (cfg->rays_per_wave != 64 && cfg->rays_per_wave != 128 && cfg->rays_per_wave != 256)
        return ctx->fail(HRA_ERR_INVALID_ARG, "rays_per_wave must be 64, 128 or 256");
    if (cfg->stack_depth != 16 && cfg->stack_depth != 20 && cfg->stack_depth != 24 && cfg->stack_depth != 32)
        return ctx->fail(HRA_ERR_INVALID_ARG, "stack_depth must be 16, 20, 24 or 32");
    if (cfg->leaf_size < 0 || cfg->leaf_size > 16) return ctx->fail(HRA_ERR_INVALID_ARG, "leaf_size must be in 0..16");
    if (cfg->traversal != 0 && cfg->traversal != HRA_TRAVERSAL_STEP && cfg->traversal != HRA_TRAVERSAL_LEAF_LOOP &&
        cfg->traversal != HRA_TRAVERSAL_REFILL)
        return ctx->fail(HRA_ERR_INVALID_ARG,
                         "traversal must be 0, HRA_TRAVERSAL_STEP, HRA_TRAVERSAL_LEAF_LOOP or HRA_TRAVERSAL_REFILL");
    if (cfg->samples_per_group < 0 || cfg->samples_per_group > MAX_GROUP)
        return ctx->fail(HRA_ERR_INVALID_ARG, "samples_per_group must be in 0..16");
    ctx->cast_rpw = cfg->rays_per_wave;
    ctx->cast_group = cfg->samples_per_group;
    ctx->cast_stack = cfg->stack_depth;
    if (cfg->leaf_size) ctx->leaf_default = cfg->leaf_size;
    if (cfg->traversal) ctx->cast_traversal = cfg->traversal;
    return HRA_OK;
}

extern "C" hra_status hra_get_cast_config(const hra_ctx *ctx, hra_cast_config *cfg) {
    if (!ctx || !cfg) return HRA_ERR_INVALID_ARG;
    cfg->rays_per_wave = ctx->cast_rpw;
    cfg->stack_depth = ctx->cast_stack;
    cfg->leaf_size = ctx->leaf_default;
    cfg->traversal = ctx->cast_traversal;
    cfg->samples_per_group = ctx->cast_group;
    return HRA_OK;
}

CastJob hra::make_cast_job(const hra_bvh *bvh, int32_t part, const float *origin, const float *normal, uint32_t *bits,
                      int64_t n_samples, int64_t item_base) {
    CastJob J;
    J.nodes = bvh->nodes;
    J.tris = bvh->tris;
    J.meta = bvh->parts + part;
    J.origin = origin;
    J.normal = normal;
    J.bits = bits;
    J.n_samples = n_samples;
    J.item_base = item_base;
    J.n_nodes_alloc = (int32_t)(bvh->n_tris > 1 ? bvh->n_tris - 1 : 1);
    J.pad = 0;
    return J;
}

// The one-sample hemisphere cast (k_cast_rows) takes its samples in a
// spatial order: the one the sampler wrote, or one formed here for at least
// this many samples.
constexpr int64_t ORDER_MIN_SAMPLES = 4096;

static hra_status cast_common(hra_ctx *ctx, const hra_bvh *bvh, int32_t part, const hra_samples *samples, hra_dirs dirs,
                              uint32_t *d_bits, uint32_t *d_counts, unsigned long long *work, int rpw, hipStream_t s) {
    if (!ctx || !bvh || !samples) return HRA_ERR_INVALID_ARG;
    if (part < 0 || part >= bvh->n_parts) return ctx->fail(HRA_ERR_INVALID_ARG, "part index out of range");
    if (samples->n < 0) return ctx->fail(HRA_ERR_INVALID_ARG, "negative sample count");
    const float4 *table = nullptr;
    hra_status st = dir_table(ctx, dirs, &table);
    if (st != HRA_OK) return st;
    if (samples->n == 0) return HRA_OK;   // nothing to cast; arrays may be null
    if (!d_bits || !samples->origin || !samples->normal)
        return ctx->fail(HRA_ERR_INVALID_ARG, "bits, origins and normals must be non-null");
    HRA_HIP(hipSetDevice(ctx->device));
    CastArgs a;
    a.jobs = nullptr;
    a.n_jobs = 1;
    a.job0 = make_cast_job(bvh, part, samples->origin, samples->normal, d_bits, samples->n, 0);
    a.dirs = table;
    a.dirs_order = dirs.kind == HRA_DIRS_AXES6 ? table : table + dirs.n;
    a.n_dirs = dirs.n;
    a.kind = dirs.kind == HRA_DIRS_AXES6 ? 1 : 0;
    a.W = (dirs.n + 31) / 32;
    a.group = a.kind == 0 ? cast_group(dirs.n, ctx->cast_group) : 1;
    a.n_items = cast_items(a.kind, samples->n, a.group);
    a.err = ctx->d_err;
    a.work = work;
    if (a.n_items >= ((int64_t)1 << 31)) return ctx->fail(HRA_ERR_INVALID_ARG, "too many samples for one call");
    void *ows = nullptr;
    const int64_t n = samples->n;
    if (a.kind == 0 && a.group == 1 && ctx->cast_traversal != HRA_TRAVERSAL_REFILL) {
        if (samples->order) {
            a.order = samples->order;
        } else if (n >= ORDER_MIN_SAMPLES) {
            const size_t ob = (sizeof(int32_t) * (size_t)n + 255) & ~(size_t)255;
            HRA_HIP(hipMallocAsync(&ows, ob + sample_order_ws_bytes(n), s));
            const hipError_t e = sample_order(samples->origin, n, bvh->parts + part, (int32_t *)ows, (char *)ows + ob, s);
            if (e != hipSuccess) {
                const hipError_t ef = hipFreeAsync(ows, s);
                (void)ef;
                return ctx->fail(HRA_ERR_DEVICE, "sample order", hipGetErrorString(e));
            }
            a.order = (const int32_t *)ows;
        }
    }
    const hipError_t el = launch_cast_any(a, rpw, ctx->cast_stack, ctx->cast_traversal, work != nullptr, s);
    if (ows) {
        const hipError_t ef = hipFreeAsync(ows, s);
        if (el == hipSuccess && ef != hipSuccess) return ctx->fail(HRA_ERR_DEVICE, "hipFreeAsync", hipGetErrorString(ef));
    }
    HRA_HIP(el);
    if (d_counts) {
        k_popcount_rows<<<blocks_for(samples->n, 256), 256, 0, s>>>(d_bits, samples->n, a.W, d_counts);
        HRA_HIP(hipGetLastError());
    }
    return HRA_OK;
}

extern "C" hra_status hra_cast_part(hra_ctx *ctx, const hra_bvh *bvh, int32_t part, const hra_samples *samples,
                                    hra_dirs dirs, uint32_t *d_bits, uint32_t *d_counts, void *stream) {
    if (!ctx) return HRA_ERR_INVALID_ARG;
    return cast_common(ctx, bvh, part, samples, dirs, d_bits, d_counts, nullptr, ctx->cast_rpw, (hipStream_t)stream);
}

extern "C" hra_status hra_cast_hemisphere(hra_ctx *ctx, const hra_bvh *bvh, const hra_samples *samples, hra_dirs dirs,
                                          uint32_t *d_bits, uint32_t *d_counts, void *stream) {
    return hra_cast_part(ctx, bvh, 0, samples, dirs, d_bits, d_counts, stream);
}

__global__ void k_zero_work(unsigned long long *w) {
    if (threadIdx.x < 2) w[threadIdx.x] = 0;
}

extern "C" hra_status hra_cast_work(hra_ctx *ctx, const hra_bvh *bvh, const hra_samples *samples, hra_dirs dirs,
                                    uint32_t *d_bits, uint64_t *node_fetches, uint64_t *tri_tests, void *stream) {
    if (!ctx || !node_fetches || !tri_tests) return HRA_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *w = nullptr;
    HRA_HIP(hipMallocAsync((void **)&w, 2 * sizeof(unsigned long long), s));
    k_zero_work<<<1, 64, 0, s>>>(w);
    hra_status st = cast_common(ctx, bvh, 0, samples, dirs, d_bits, nullptr, w, 64, s);
    unsigned long long h[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(h, w, sizeof(h), hipMemcpyDeviceToHost, s);
    const hipError_t ef = hipFreeAsync(w, s);
    if (e == hipSuccess) e = ef;
    if (st != HRA_OK) return st;
    if (e != hipSuccess) return ctx->fail(HRA_ERR_DEVICE, "work counter copy failed", hipGetErrorString(e));
    st = check_error_word(ctx, s);
    if (st != HRA_OK) return st;
    *node_fetches = h[0];
    *tri_tests = h[1];
    return HRA_OK;
}

extern "C" hra_status hra_debug_rays(hra_ctx *ctx, const hra_samples *samples, hra_dirs dirs, const int64_t *d_sample_idx,
                                     int64_t n_idx, float *d_out, void *stream) {
    if (!ctx || !samples || !d_sample_idx || !d_out || n_idx < 0) return HRA_ERR_INVALID_ARG;
    const float4 *table = nullptr;
    hra_status st = dir_table(ctx, dirs, &table);
    if (st != HRA_OK) return st;
    if (n_idx == 0) return HRA_OK;
    hipStream_t s = (hipStream_t)stream;
    HRA_HIP(hipSetDevice(ctx->device));
    const int64_t total = n_idx * dirs.n;
    k_debug_rays<<<blocks_for(total, 256), 256, 0, s>>>(samples->origin, samples->normal, d_sample_idx, n_idx, samples->n,
                                                       table, dirs.n, dirs.kind == HRA_DIRS_AXES6 ? 1 : 0, d_out);
    HRA_HIP(hipGetLastError());
    return HRA_OK;
}

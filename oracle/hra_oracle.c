/*
 * CPU oracle for hemispherical ray-casting accessibility.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the library never does.  It
 * shares no code with the GPU path.
 *
 * Method (paper, Section 3.1): from a point on each face, offset slightly
 * along the normal, rays are cast over a uniformly sampled hemisphere that is
 * rotated onto the face normal; a ray is unobstructed if it hits no triangle
 * of the part.  The result here is the plain definition: every ray is tested
 * against every triangle with FP64 edge functions (brute force), and each
 * (ray, triangle) pair is decided HIT / MISS / AMBIGUOUS with a relative band
 * tau = 1e-6 so that rays grazing an edge are flagged rather than guessed.
 *
 * Loop order: for one sample the direction-independent factors of every
 * triangle (translated vertices, edge cross products, edge scales, plane) are
 * formed once and then dotted with each direction.  This changes no value:
 * each quantity is the same IEEE expression whichever loop runs outside.
 *
 * Readings taken where the paper is silent (listed in the design notes):
 *  - directions: spherical Fibonacci hemisphere, uniform in solid angle,
 *    computed in FP64 and rounded once to FP32;
 *  - rotation onto the normal: branchless orthonormal basis of Duff et al.
 *    (2017, "Building an Orthonormal Basis, Revisited"), FP32, fixed order;
 *  - offset: eps = 1e-4 x bbox diagonal along the unit normal (FP32 fma);
 *  - triangles block from both sides; rays extend over t in (0, inf);
 *  - an occluded ray is not unobstructed; the denominator is always N.
 *
 * Built with -ffp-contract=off and without fast-math so every FP32 step is a
 * single IEEE operation; fmaf is the C library's correctly rounded fma.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TAU 1e-6

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood 2014), used as a counter-based generator:
 * output number c of stream `seed` is the mix of seed + (c+1) * golden gamma. */
static inline uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline uint64_t sm64_at(uint64_t seed, uint64_t c) {
    return sm64_mix(seed + (c + 1ULL) * 0x9E3779B97F4A7C15ULL);
}

void orc_splitmix64(uint64_t seed, uint64_t c0, int64_t n, uint64_t *out) {
    for (int64_t i = 0; i < n; ++i) out[i] = sm64_at(seed, c0 + (uint64_t)i);
}

/* ------------------------------------------------------------------------ */
/* Direction sets (Section 3.1: uniformly sampled hemisphere, Fig. 1).
 * Spherical Fibonacci points on the open upper hemisphere:
 *   z_j = 1 - (2j+1)/(2N),  r_j = sqrt(1 - z_j^2),
 *   phi_j = 2 pi frac(j g),  g = (3 - sqrt 5)/2  (golden angle / 2 pi),
 * evaluated in FP64 and rounded once to FP32. */
void orc_fibonacci_dirs(int32_t n, float *out) {
    const double g = (3.0 - sqrt(5.0)) / 2.0;
    const double two_pi = 6.283185307179586476925286766559;
    for (int32_t j = 0; j < n; ++j) {
        double z = 1.0 - (2.0 * j + 1.0) / (2.0 * n);
        double r = sqrt(1.0 - z * z);
        double jg = (double)j * g;
        double f = jg - floor(jg);
        double phi = two_pi * f;
        out[3 * j + 0] = (float)(r * cos(phi));
        out[3 * j + 1] = (float)(r * sin(phi));
        out[3 * j + 2] = (float)z;
    }
}

/* The six principal directions of Section 3.2, world frame: +X,-X,+Y,-Y,+Z,-Z. */
void orc_axes6(float *out) {
    static const float a[18] = {1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1};
    memcpy(out, a, sizeof a);
}

/* ------------------------------------------------------------------------ */
/* Section 3.1: hemisphere rotated to the face normal.  Basis (t, b, n) from
 * the unit normal, Duff et al. 2017, evaluated in FP32 step by step. */
void orc_frame(const float *n, float *t, float *b) {
    float sign = copysignf(1.0f, n[2]);
    float a = -1.0f / (sign + n[2]);
    float nxny = n[0] * n[1];
    float bb = nxny * a;
    float snx = sign * n[0];
    float snxnx = snx * n[0];
    float snxnxa = snxnx * a;
    t[0] = 1.0f + snxnxa;
    t[1] = sign * bb;
    t[2] = -(sign * n[0]);
    float nyny = n[1] * n[1];
    float nynya = nyny * a;
    b[0] = bb;
    b[1] = sign + nynya;
    b[2] = -n[1];
}

/* World direction of local hemisphere point l = (x, y, z) for normal n:
 * d_c = fma(x, t_c, fma(y, b_c, z * n_c)), FP32, not renormalised. */
static inline void world_dir(const float *t, const float *b, const float *n, const float *l, float *d) {
    for (int c = 0; c < 3; ++c) {
        float zn = l[2] * n[c];
        d[c] = fmaf(l[0], t[c], fmaf(l[1], b[c], zn));
    }
}

/* Rays exactly as the method forms them.  kind 0: hemisphere rotated onto
 * each sample normal; kind 1: world-frame directions as given (the six
 * principal axes).  out: [S][N][3]. */
void orc_ray_dirs(const float *nrm, int64_t S, const float *dirs, int32_t N, int32_t kind, float *out) {
    for (int64_t s = 0; s < S; ++s) {
        const float *n = nrm + 3 * s;
        float t[3], b[3];
        orc_frame(n, t, b);
        for (int32_t j = 0; j < N; ++j) {
            float *d = out + 3 * (s * N + j);
            if (kind == 0) world_dir(t, b, n, dirs + 3 * j, d);
            else memcpy(d, dirs + 3 * j, 3 * sizeof(float));
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Mesh facts (Section 3.1: centroid, normal and area of each face). */
static inline void tri_verts(const float *V, const int32_t *T, int64_t f, double v[3][3]) {
    for (int k = 0; k < 3; ++k)
        for (int c = 0; c < 3; ++c) v[k][c] = (double)V[3 * (int64_t)T[3 * f + k] + c];
}

/* twice-area squared in FP64: q = |(v1-v0) x (v2-v0)|^2, fixed order */
static inline double tri_q(const double v[3][3]) {
    double e1x = v[1][0] - v[0][0], e1y = v[1][1] - v[0][1], e1z = v[1][2] - v[0][2];
    double e2x = v[2][0] - v[0][0], e2y = v[2][1] - v[0][1], e2z = v[2][2] - v[0][2];
    double p1 = e1y * e2z, p2 = e1z * e2y;
    double nx = p1 - p2;
    double p3 = e1z * e2x, p4 = e1x * e2z;
    double ny = p3 - p4;
    double p5 = e1x * e2y, p6 = e1y * e2x;
    double nz = p5 - p6;
    double sx = nx * nx, sy = ny * ny, sz = nz * nz;
    double s = sx + sy;
    return s + sz;
}

/* bbox[6] = min xyz, max xyz; returns diag (FP64) and eps (FP32). */
void orc_mesh_info(const float *V, int64_t nv, double *bbox, double *diag, float *eps, float offset_frac) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < nv; ++i)
        for (int c = 0; c < 3; ++c) {
            double x = V[3 * i + c];
            if (x < lo[c]) lo[c] = x;
            if (x > hi[c]) hi[c] = x;
        }
    double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    double sx = dx * dx, sy = dy * dy, sz = dz * dz;
    double s = sx + sy;
    s = s + sz;
    double d = sqrt(s);
    for (int c = 0; c < 3; ++c) { bbox[c] = lo[c]; bbox[3 + c] = hi[c]; }
    *diag = d;
    double e = (double)offset_frac * d;
    *eps = (float)e;
}

/* FP32 unit geometric normal of a triangle: N = (v1-v0) x (v2-v0), N/|N|. */
static inline void tri_normal32(const float *V, const int32_t *T, int64_t f, float *n) {
    const float *a = V + 3 * (int64_t)T[3 * f], *b = V + 3 * (int64_t)T[3 * f + 1], *c = V + 3 * (int64_t)T[3 * f + 2];
    float e1x = b[0] - a[0], e1y = b[1] - a[1], e1z = b[2] - a[2];
    float e2x = c[0] - a[0], e2y = c[1] - a[1], e2z = c[2] - a[2];
    float p1 = e1y * e2z, p2 = e1z * e2y;
    float nx = p1 - p2;
    float p3 = e1z * e2x, p4 = e1x * e2z;
    float ny = p3 - p4;
    float p5 = e1x * e2y, p6 = e1y * e2x;
    float nz = p5 - p6;
    float sx = nx * nx, sy = ny * ny, sz = nz * nz;
    float s = sx + sy;
    s = s + sz;
    float len = sqrtf(s);
    n[0] = nx / len;
    n[1] = ny / len;
    n[2] = nz / len;
}

static inline void offset_origin(const float *p, const float *n, float eps, float *o) {
    for (int c = 0; c < 3; ++c) o[c] = fmaf(eps, n[c], p[c]);
}

/* Area weights as integers so the choice of triangle is exact integer work:
 * w_f = floor(area_f * 2^k), k = 54 - (ilogb(max area) + 1) - bitlen(T),
 * which keeps sum(w) < 2^54 (room for many parts' weights in one 64-bit
 * running sum). Zero-area triangles get weight 0. */
int orc_area_weights(const float *V, const int32_t *T, int64_t nt, uint64_t *w, int32_t *k_out) {
    double amax = 0.0;
    double *area = (double *)malloc(sizeof(double) * (nt > 0 ? nt : 1));
    for (int64_t f = 0; f < nt; ++f) {
        double v[3][3];
        tri_verts(V, T, f, v);
        double q = tri_q(v);
        double a = 0.5 * sqrt(q);
        area[f] = a;
        if (a > amax) amax = a;
    }
    if (amax <= 0.0) { free(area); return -1; }
    int E = ilogb(amax);
    int tb = 0;
    while (tb < 63 && ((int64_t)1 << tb) <= nt) ++tb;
    int k = 54 - (E + 1) - tb;
    for (int64_t f = 0; f < nt; ++f) w[f] = (uint64_t)floor(ldexp(area[f], k));
    free(area);
    *k_out = k;
    return 0;
}

/* Section 3.1 (per-face attributes) with area-weighted i.i.d. points:
 * triangle chosen with probability proportional to its (quantised) area by
 * an upper-bound search of r = floor(x0 * total / 2^64) in the inclusive
 * prefix sums; the point is the area-uniform square-root parametrisation
 *   p = (1 - sqrt u1) v0 + sqrt u1 (1 - u2) v1 + sqrt u1 u2 v2,
 * with u1, u2 the top 24 bits of the next two generator outputs.  FP32. */
int orc_sample_area(const float *V, int64_t nv, const int32_t *T, int64_t nt, int64_t n, uint64_t seed,
                    float offset_frac, float *P, float *Nrm, float *O, int32_t *tri) {
    uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * (nt > 0 ? nt : 1));
    int32_t k;
    if (orc_area_weights(V, T, nt, w, &k) != 0) { free(w); return -1; }
    uint64_t *C = (uint64_t *)malloc(sizeof(uint64_t) * nt);
    uint64_t acc = 0;
    for (int64_t f = 0; f < nt; ++f) { acc += w[f]; C[f] = acc; }
    double bbox[6], diag;
    float eps;
    orc_mesh_info(V, nv, bbox, &diag, &eps, offset_frac);
    for (int64_t i = 0; i < n; ++i) {
        uint64_t x0 = sm64_at(seed, 3 * (uint64_t)i), x1 = sm64_at(seed, 3 * (uint64_t)i + 1),
                 x2 = sm64_at(seed, 3 * (uint64_t)i + 2);
        uint64_t r = (uint64_t)(((unsigned __int128)x0 * acc) >> 64);
        int64_t lo = 0, hi = nt - 1;           /* first f with C[f] > r */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (C[mid] > r) hi = mid; else lo = mid + 1;
        }
        int64_t f = lo;
        float u1 = (float)(x1 >> 40) * 0x1p-24f;
        float u2 = (float)(x2 >> 40) * 0x1p-24f;
        float su = sqrtf(u1);
        float w0 = 1.0f - su;
        float omu2 = 1.0f - u2;
        float w1 = su * omu2;
        float w2 = su * u2;
        const float *a = V + 3 * (int64_t)T[3 * f], *b = V + 3 * (int64_t)T[3 * f + 1], *c = V + 3 * (int64_t)T[3 * f + 2];
        float *p = P + 3 * i;
        for (int q = 0; q < 3; ++q) {
            float t0 = w0 * a[q];
            p[q] = fmaf(w2, c[q], fmaf(w1, b[q], t0));
        }
        tri_normal32(V, T, f, Nrm + 3 * i);
        offset_origin(p, Nrm + 3 * i, eps, O + 3 * i);
        tri[i] = (int32_t)f;
    }
    free(w);
    free(C);
    return 0;
}

/* Section 3.1 as printed: one sample at the centroid of every face with
 * nonzero area, in face order.  Returns the number of samples written. */
int64_t orc_sample_centroid(const float *V, int64_t nv, const int32_t *T, int64_t nt, float offset_frac,
                            float *P, float *Nrm, float *O, int32_t *tri) {
    double bbox[6], diag;
    float eps;
    orc_mesh_info(V, nv, bbox, &diag, &eps, offset_frac);
    int64_t m = 0;
    for (int64_t f = 0; f < nt; ++f) {
        double v[3][3];
        tri_verts(V, T, f, v);
        if (!(tri_q(v) > 0.0)) continue;
        const float *a = V + 3 * (int64_t)T[3 * f], *b = V + 3 * (int64_t)T[3 * f + 1], *c = V + 3 * (int64_t)T[3 * f + 2];
        float *p = P + 3 * m;
        for (int q = 0; q < 3; ++q) {
            float s = a[q] + b[q];
            s = s + c[q];
            p[q] = s / 3.0f;
        }
        tri_normal32(V, T, f, Nrm + 3 * m);
        offset_origin(p, Nrm + 3 * m, eps, O + 3 * m);
        tri[m] = (int32_t)f;
        ++m;
    }
    return m;
}

/* ------------------------------------------------------------------------ */
/* The per (ray, triangle) decision, FP64 (Section 3.1, ray-triangle tests).
 * a, b, c = vertices minus the ray origin.  Edge functions
 *   e0 = d.(b x c), e1 = d.(c x a), e2 = d.(a x b)
 * have the sign of the side of each edge the ray line passes; they all share
 * a sign iff the line meets the triangle.  With edge scales
 *   S0 = |c - b| max(|b|,|c|)  (and cyclically)
 * e_i / S_i is about the angle between the ray and edge i as seen from the
 * origin, so a band |e_i| <= tau S_i marks a grazing pass.  Plane:
 * P = (b-a) x (c-a), h = a.P, q = d.P; the hit lies at t = h/q, in front iff
 * h and q share a sign.  Definite: |h| > tau |P| max(|a|,|b|,|c|),
 * |q| > tau |P|. */
enum { DEC_MISS = 0, DEC_HIT = 1, DEC_AMB = 2 };

typedef struct {
    double X0[3], X1[3], X2[3], P[3];
    double S0, S1, S2, h, Pn, amax;
    int degenerate;
} tri_pre;

static inline void cross3(const double *u, const double *v, double *w) {
    double p1 = u[1] * v[2], p2 = u[2] * v[1];
    double p3 = u[2] * v[0], p4 = u[0] * v[2];
    double p5 = u[0] * v[1], p6 = u[1] * v[0];
    w[0] = p1 - p2;
    w[1] = p3 - p4;
    w[2] = p5 - p6;
}
static inline double dot3(const double *u, const double *v) {
    double p = u[0] * v[0], q = u[1] * v[1], r = u[2] * v[2];
    double s = p + q;
    return s + r;
}
static inline double norm3(const double *u) { return sqrt(dot3(u, u)); }

static void tri_prepare(const double v[3][3], const double *o, tri_pre *t) {
    double a[3], b[3], c[3], cb[3], ac[3], ba[3], ca[3];
    for (int k = 0; k < 3; ++k) {
        a[k] = v[0][k] - o[k];
        b[k] = v[1][k] - o[k];
        c[k] = v[2][k] - o[k];
    }
    cross3(b, c, t->X0);
    cross3(c, a, t->X1);
    cross3(a, b, t->X2);
    for (int k = 0; k < 3; ++k) {
        cb[k] = c[k] - b[k];
        ac[k] = a[k] - c[k];
        ba[k] = b[k] - a[k];
        ca[k] = c[k] - a[k];
    }
    double na = norm3(a), nb = norm3(b), nc = norm3(c);
    t->S0 = norm3(cb) * fmax(nb, nc);
    t->S1 = norm3(ac) * fmax(nc, na);
    t->S2 = norm3(ba) * fmax(na, nb);
    cross3(ba, ca, t->P);
    t->h = dot3(a, t->P);
    t->Pn = norm3(t->P);
    t->amax = fmax(na, fmax(nb, nc));
    t->degenerate = (t->P[0] == 0.0 && t->P[1] == 0.0 && t->P[2] == 0.0);
}

static inline int sgn_band(double e, double S) {
    if (e > TAU * S) return 1;
    if (e < -TAU * S) return -1;
    return 0;
}

/* Returns DEC_*; *info gets the exact inclusive-sign decision (1 = hit). */
static inline int decide(const tri_pre *t, const double *d, int *info) {
    double e0 = dot3(d, t->X0), e1 = dot3(d, t->X1), e2 = dot3(d, t->X2);
    double q = dot3(d, t->P);
    /* informational exact-sign verdict (inclusive edges, t > 0) */
    int ge = (e0 >= 0 && e1 >= 0 && e2 >= 0), le = (e0 <= 0 && e1 <= 0 && e2 <= 0);
    int allz = (e0 == 0 && e1 == 0 && e2 == 0);
    *info = ((ge || le) && !allz && ((t->h > 0 && q > 0) || (t->h < 0 && q < 0))) ? 1 : 0;

    int s0 = sgn_band(e0, t->S0), s1 = sgn_band(e1, t->S1), s2 = sgn_band(e2, t->S2);
    int hdef = fabs(t->h) > TAU * t->Pn * t->amax;
    int qdef = fabs(q) > TAU * t->Pn;
    int same = (t->h > 0) == (q > 0);
    int front = hdef && qdef && same;
    int behind = (q == 0.0) || (hdef && qdef && !same);
    int pos = (s0 > 0) + (s1 > 0) + (s2 > 0), neg = (s0 < 0) + (s1 < 0) + (s2 < 0);
    if ((pos == 3 || neg == 3) && front) return DEC_HIT;
    if ((pos > 0 && neg > 0) || behind) return DEC_MISS;
    return DEC_AMB;
}

/* Brute-force cast.  For every sample s and direction j:
 *   bit 1 = unobstructed (no triangle HIT and none AMBIGUOUS),
 *   bit 0 = occluded (some triangle HIT) or culled,
 *   grazing bit 1 = no HIT but some AMBIGUOUS (excluded from comparisons;
 *   `info` then holds the exact inclusive-sign verdict, 1 = unobstructed).
 * kind 0: hemisphere directions rotated onto each normal;
 * kind 1: world directions; a direction with n.D < 0 is culled (bit 0,
 *         not cast), n.D = 0 is cast (Section 3.2 reading).
 * Rows are W = ceil(N/32) words, bit j%32 of word j/32 is direction j.
 * Only samples in [s0, s1) are computed (for bounded subsets). */
int orc_cast(const float *V, int64_t nv, const int32_t *T, int64_t nt, const float *O, const float *Nrm,
             int64_t s0, int64_t s1, const float *dirs, int32_t N, int32_t kind,
             uint32_t *bits, uint32_t *grazing, uint32_t *info, int32_t nthreads) {
    (void)nv;
    const int32_t W = (N + 31) / 32;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int err = 0;
#pragma omp parallel
    {
        double (*D)[3] = (double (*)[3])malloc(sizeof(double) * 3 * N);
        unsigned char *st = (unsigned char *)malloc(N);   /* 0 free, 1 hit, 2 amb */
        unsigned char *inf = (unsigned char *)malloc(N);
        unsigned char *cull = (unsigned char *)malloc(N);
        if (!D || !st || !inf || !cull) err = 1;
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = s0; s < s1; ++s) {
            if (err) continue;
            const float *n = Nrm + 3 * s;
            float t3[3], b3[3];
            orc_frame(n, t3, b3);
            for (int32_t j = 0; j < N; ++j) {
                float d[3];
                if (kind == 0) world_dir(t3, b3, n, dirs + 3 * j, d);
                else { d[0] = dirs[3 * j]; d[1] = dirs[3 * j + 1]; d[2] = dirs[3 * j + 2]; }
                D[j][0] = d[0]; D[j][1] = d[1]; D[j][2] = d[2];
                st[j] = 0;
                inf[j] = 0;
                cull[j] = 0;
                if (kind == 1) {
                    /* n.D with D a signed unit axis is exactly +-n_k */
                    float nd = n[0] * d[0] + n[1] * d[1] + n[2] * d[2];
                    if (nd < 0.0f) { cull[j] = 1; st[j] = 1; }
                }
            }
            double o[3] = {O[3 * s], O[3 * s + 1], O[3 * s + 2]};
            for (int64_t f = 0; f < nt; ++f) {
                double v[3][3];
                tri_verts(V, T, f, v);
                tri_pre tp;
                tri_prepare(v, o, &tp);
                if (tp.degenerate) continue;   /* q = 0 for every ray: MISS */
                for (int32_t j = 0; j < N; ++j) {
                    if (st[j] == 1) continue;
                    int ib;
                    int dcs = decide(&tp, D[j], &ib);
                    if (ib) inf[j] = 1;          /* an inclusive-sign hit was seen */
                    if (dcs == DEC_HIT) st[j] = 1;
                    else if (dcs == DEC_AMB) st[j] = 2;
                }
            }
            uint32_t *rb = bits + (s - s0) * W, *rg = grazing + (s - s0) * W, *ri = info + (s - s0) * W;
            for (int32_t w = 0; w < W; ++w) rb[w] = rg[w] = ri[w] = 0;
            for (int32_t j = 0; j < N; ++j) {
                uint32_t m = 1u << (j & 31);
                if (st[j] == 0) rb[j >> 5] |= m;
                if (st[j] == 2) rg[j >> 5] |= m;
                if (st[j] == 2 && !inf[j]) ri[j >> 5] |= m;
            }
        }
        free(D);
        free(st);
        free(inf);
        free(cull);
    }
    return err ? -1 : 0;
}

/* Single-ray decision for arbitrary FP32 (o, d) pairs against all triangles:
 * out[i] = 0 occluded, 1 unobstructed, 2 grazing. */
int orc_cast_rays(const float *V, const int32_t *T, int64_t nt, const float *O, const float *D, int64_t nr,
                  uint8_t *out, int32_t nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < nr; ++r) {
        double o[3] = {O[3 * r], O[3 * r + 1], O[3 * r + 2]};
        double d[3] = {D[3 * r], D[3 * r + 1], D[3 * r + 2]};
        int st = 0;
        for (int64_t f = 0; f < nt && st != 1; ++f) {
            double v[3][3];
            tri_verts(V, T, f, v);
            tri_pre tp;
            tri_prepare(v, o, &tp);
            if (tp.degenerate) continue;
            int ib;
            int dcs = decide(&tp, d, &ib);
            if (dcs == DEC_HIT) st = 1;
            else if (dcs == DEC_AMB) st = 2;
        }
        out[r] = (uint8_t)(st == 1 ? 0 : (st == 2 ? 2 : 1));
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The same cast through a padded bounding-volume hierarchy, for inputs where
 * brute force takes too long.  Section 3.1 defines the result as "does any
 * triangle block the ray"; a hierarchy only skips triangles, so it reaches
 * the same result provided it never skips one that matters.
 *
 * Tree: top-down median split.  A range of triangles is split at its median
 * centroid along the axis where the centroids spread most (ties by index);
 * ranges of at most 4 triangles are leaves.  Boxes are the exact FP64 bounds
 * of their triangles' FP32 vertices, then grown outward by `pad` (and one
 * more ulp, so the rounding of the growth cannot shrink them).
 *
 * Box test: the slab intervals in FP64 from 1/d, accepted when the largest
 * entry distance is at most the smallest exit distance plus a slack of 1e-9
 * of their magnitudes (each computed distance is within a few units of
 * 2^-53 of the exact one) and the exit distance is not negative (signs are
 * exact under rounding).  A zero direction component keeps the slab when the
 * origin lies inside it.  So a box the exact ray meets is never rejected.
 *
 * Leaves: every triangle is decided by decide() on tri_prepare()'s factors,
 * the very routines of the brute-force cast.  Consequences:
 *  - a HIT needs three definite edge signs and a definite plane side, which
 *    only a ray meeting the closed triangle can give (the band is 1e-6, far
 *    above FP64 rounding), so every HIT triangle lies in a box the ray meets
 *    and is tested: bit 0 exactly where brute force has bit 0;
 *  - with no HIT, a ray is grazing here iff some tested triangle is
 *    AMBIGUOUS.  Tested triangles are a subset of all, so the grazing set is
 *    a subset of brute force's, and where brute force flags a ray that this
 *    cast clears, every ambiguous triangle lies outside a box grown by `pad`
 *    around it: the exact ray misses it, so 1 is the exact answer;
 *  - the informational exact-sign bit of a grazing ray is the same (an
 *    inclusive-sign hit lies on the closed triangle, inside its box).
 * With pad = 1e-4 x diagonal the grazing sets have been equal on every mesh
 * compared (the tests).
 *
 * The per-sample factors of a triangle (tri_prepare: translated vertices,
 * cross products, scales, plane) depend on the origin only, so each thread
 * keeps them for the current sample and reuses them across its directions,
 * as the brute-force loop does. */
typedef struct {
    double lo[3], hi[3];
    int32_t left, right;   /* children (interior), or -1 */
    int32_t first, count;  /* leaf: triangles ord[first .. first+count) */
} obvh_node;

typedef struct {
    const float *V;
    const int32_t *T;
    int64_t nt;
    int32_t *ord;          /* triangle order, leaves contiguous */
    obvh_node *nodes;
    int64_t n_nodes;
    int32_t depth;
    double *cen;           /* centroids [nt][3] (build only) */
    int sort_axis;
} obvh;

static obvh *g_sort_bvh;   /* comparator context (the build runs on one thread) */

static int obvh_cmp(const void *pa, const void *pb) {
    const int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    const double ca = g_sort_bvh->cen[3 * (int64_t)a + g_sort_bvh->sort_axis];
    const double cb = g_sort_bvh->cen[3 * (int64_t)b + g_sort_bvh->sort_axis];
    if (ca < cb) return -1;
    if (ca > cb) return 1;
    return (a > b) - (a < b);
}

static int32_t obvh_build_range(obvh *h, int64_t first, int64_t count, double pad, int32_t level) {
    const int32_t id = (int32_t)h->n_nodes++;
    obvh_node *nd = &h->nodes[id];
    if (level > h->depth) h->depth = level;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = first; i < first + count; ++i) {
        const int64_t f = h->ord[i];
        for (int k = 0; k < 3; ++k) {
            const double x = (double)h->V[3 * (int64_t)h->T[3 * f + k] + 0], y = (double)h->V[3 * (int64_t)h->T[3 * f + k] + 1],
                         z = (double)h->V[3 * (int64_t)h->T[3 * f + k] + 2];
            const double p[3] = {x, y, z};
            for (int c = 0; c < 3; ++c) {
                if (p[c] < lo[c]) lo[c] = p[c];
                if (p[c] > hi[c]) hi[c] = p[c];
            }
        }
        for (int c = 0; c < 3; ++c) {
            const double m = h->cen[3 * f + c];
            if (m < clo[c]) clo[c] = m;
            if (m > chi[c]) chi[c] = m;
        }
    }
    for (int c = 0; c < 3; ++c) {
        nd->lo[c] = nextafter(lo[c] - pad, -INFINITY);
        nd->hi[c] = nextafter(hi[c] + pad, INFINITY);
    }
    if (count <= 4) {
        nd->left = nd->right = -1;
        nd->first = (int32_t)first;
        nd->count = (int32_t)count;
        return id;
    }
    int axis = 0;
    for (int c = 1; c < 3; ++c)
        if (chi[c] - clo[c] > chi[axis] - clo[axis]) axis = c;
    g_sort_bvh = h;
    h->sort_axis = axis;
    qsort(h->ord + first, (size_t)count, sizeof(int32_t), obvh_cmp);
    const int64_t half = count / 2;
    nd->first = -1;
    nd->count = 0;
    const int32_t l = obvh_build_range(h, first, half, pad, level + 1);
    const int32_t r = obvh_build_range(h, first + half, count - half, pad, level + 1);
    h->nodes[id].left = l;     /* nd may have moved: index again */
    h->nodes[id].right = r;
    return id;
}

/* Build over all triangles of the mesh (zero-area ones included: decide()
 * treats them exactly as brute force does).  pad: outward growth of every
 * box in mm.  Returns NULL for an empty mesh or on allocation failure. */
void *orc_bvh_build(const float *V, int64_t nv, const int32_t *T, int64_t nt, double pad) {
    (void)nv;
    if (nt <= 0) return NULL;
    obvh *h = (obvh *)calloc(1, sizeof(obvh));
    h->V = V;
    h->T = T;
    h->nt = nt;
    h->ord = (int32_t *)malloc(sizeof(int32_t) * nt);
    h->nodes = (obvh_node *)malloc(sizeof(obvh_node) * (2 * nt));
    h->cen = (double *)malloc(sizeof(double) * 3 * nt);
    if (!h->ord || !h->nodes || !h->cen) {
        free(h->ord); free(h->nodes); free(h->cen); free(h);
        return NULL;
    }
    for (int64_t f = 0; f < nt; ++f) {
        h->ord[f] = (int32_t)f;
        double v[3][3];
        tri_verts(V, T, f, v);
        for (int c = 0; c < 3; ++c) h->cen[3 * f + c] = (v[0][c] + v[1][c] + v[2][c]) / 3.0;
    }
    obvh_build_range(h, 0, nt, pad, 1);
    free(h->cen);
    h->cen = NULL;
    return h;
}

void orc_bvh_free(void *p) {
    obvh *h = (obvh *)p;
    if (!h) return;
    free(h->ord);
    free(h->nodes);
    free(h);
}

/* out[0] nodes, out[1] depth */
void orc_bvh_shape(const void *p, int64_t *out) {
    const obvh *h = (const obvh *)p;
    out[0] = h->n_nodes;
    out[1] = h->depth;
}

static inline int obvh_box(const obvh_node *nd, const double *o, const double *d, const double *inv) {
    double tmin = -INFINITY, tmax = INFINITY;
    for (int k = 0; k < 3; ++k) {
        if (d[k] == 0.0) {
            if (o[k] < nd->lo[k] || o[k] > nd->hi[k]) return 0;
            continue;
        }
        double t0 = (nd->lo[k] - o[k]) * inv[k], t1 = (nd->hi[k] - o[k]) * inv[k];
        if (t0 > t1) { const double t = t0; t0 = t1; t1 = t; }
        if (t0 > tmin) tmin = t0;
        if (t1 < tmax) tmax = t1;
    }
    if (!(tmax >= 0.0)) return 0;
    return tmin <= tmax + 1e-9 * (fabs(tmin) + fabs(tmax));
}

typedef struct {
    tri_pre *pre;      /* [nt] factors for the current sample */
    int64_t *stamp;    /* [nt] sample whose factors pre[] holds, -1 none */
    int32_t *stack;    /* [2 * depth + 8] */
    uint64_t nodes, tris;
} obvh_scratch;

/* One ray: returns 0 free, 1 occluded, 2 grazing; *info = exact-sign bit
 * seen (as in orc_cast). */
static int obvh_ray(const obvh *h, obvh_scratch *w, int64_t s, const double *o, const double *d, int *info) {
    double inv[3];
    for (int k = 0; k < 3; ++k) inv[k] = d[k] != 0.0 ? 1.0 / d[k] : 0.0;
    int sp = 0, amb = 0;
    *info = 0;
    w->stack[sp++] = 0;
    while (sp > 0) {
        const obvh_node *nd = &h->nodes[w->stack[--sp]];
        ++w->nodes;
        if (!obvh_box(nd, o, d, inv)) continue;
        if (nd->left < 0) {
            for (int32_t i = nd->first; i < nd->first + nd->count; ++i) {
                const int64_t f = h->ord[i];
                if (w->stamp[f] != s) {
                    double v[3][3];
                    tri_verts(h->V, h->T, f, v);
                    tri_prepare(v, o, &w->pre[f]);
                    w->stamp[f] = s;
                }
                if (w->pre[f].degenerate) continue;
                ++w->tris;
                int ib;
                const int dcs = decide(&w->pre[f], d, &ib);
                if (ib) *info = 1;
                if (dcs == DEC_HIT) return 1;
                if (dcs == DEC_AMB) amb = 1;
            }
        } else {
            w->stack[sp++] = nd->right;
            w->stack[sp++] = nd->left;
        }
    }
    return amb ? 2 : 0;
}

/* orc_cast through the hierarchy: same arguments and outputs (bits,
 * grazing, info rows for samples [s0, s1)), plus work[2] += node box tests
 * and triangle decisions (may be NULL). */
int orc_bvh_cast(const void *ph, const float *O, const float *Nrm, int64_t s0, int64_t s1, const float *dirs, int32_t N,
                 int32_t kind, uint32_t *bits, uint32_t *grazing, uint32_t *info, uint64_t *work, int32_t nthreads) {
    const obvh *h = (const obvh *)ph;
    const int32_t W = (N + 31) / 32;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int err = 0;
    uint64_t tot_nodes = 0, tot_tris = 0;
#pragma omp parallel reduction(+ : tot_nodes, tot_tris)
    {
        obvh_scratch w;
        w.pre = (tri_pre *)malloc(sizeof(tri_pre) * h->nt);
        w.stamp = (int64_t *)malloc(sizeof(int64_t) * h->nt);
        w.stack = (int32_t *)malloc(sizeof(int32_t) * (2 * (size_t)h->depth + 8));
        w.nodes = w.tris = 0;
        if (!w.pre || !w.stamp || !w.stack) {
#pragma omp atomic write
            err = 1;
        } else {
            for (int64_t f = 0; f < h->nt; ++f) w.stamp[f] = -1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = s0; s < s1; ++s) {
            if (err) continue;
            const float *n = Nrm + 3 * s;
            float t3[3], b3[3];
            orc_frame(n, t3, b3);
            const double o[3] = {O[3 * s], O[3 * s + 1], O[3 * s + 2]};
            uint32_t *rb = bits + (s - s0) * W, *rg = grazing + (s - s0) * W, *ri = info + (s - s0) * W;
            for (int32_t q = 0; q < W; ++q) rb[q] = rg[q] = ri[q] = 0;
            for (int32_t j = 0; j < N; ++j) {
                float df[3];
                if (kind == 0) world_dir(t3, b3, n, dirs + 3 * j, df);
                else { df[0] = dirs[3 * j]; df[1] = dirs[3 * j + 1]; df[2] = dirs[3 * j + 2]; }
                if (kind == 1) {
                    const float nd = n[0] * df[0] + n[1] * df[1] + n[2] * df[2];
                    if (nd < 0.0f) continue;   /* culled: bit 0 */
                }
                const double d[3] = {df[0], df[1], df[2]};
                int ib;
                const int st = obvh_ray(h, &w, s, o, d, &ib);
                const uint32_t m = 1u << (j & 31);
                if (st == 0) rb[j >> 5] |= m;
                if (st == 2) rg[j >> 5] |= m;
                if (st == 2 && !ib) ri[j >> 5] |= m;
            }
        }
        tot_nodes += w.nodes;
        tot_tris += w.tris;
        free(w.pre);
        free(w.stamp);
        free(w.stack);
    }
    if (work) {
        work[0] += tot_nodes;
        work[1] += tot_tris;
    }
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Tool-aware accessibility (the tool-geometry row next to Section 3.3's
 * reach test; the paper's rays are infinitely thin).  A ball-end tool of
 * radius r touches the surface point p from outside: its tip centre is
 * c = p + r n (FP64 from the FP32 p and n), and the tool, shank included,
 * fills every point within r of the half-line L = {c + t u, t >= 0}, u the
 * direction normalised in FP64.  The direction is free iff no triangle comes
 * closer to L than thr = r - tol.  Distance between L and a triangle, the
 * plain definition: 0 if L meets the triangle, else the least of the
 * distance from c to the triangle and the distances from L to its three
 * edges (for convex sets the nearest pair has an end point of one set, or
 * lies in both interiors, which for a line and a triangle means L meets it
 * or runs parallel to it and the edge distances attain it). */
static double seg_point(const double *x, const double *a, const double *b) {
    /* distance from x to the segment [a, b] */
    double e[3], w[3], q[3];
    for (int k = 0; k < 3; ++k) { e[k] = b[k] - a[k]; w[k] = x[k] - a[k]; }
    double ee = dot3(e, e), s = ee > 0 ? dot3(w, e) / ee : 0.0;
    if (s < 0) s = 0;
    if (s > 1) s = 1;
    for (int k = 0; k < 3; ++k) q[k] = w[k] - s * e[k];
    return norm3(q);
}

static double ray_point(const double *c, const double *u, const double *x) {
    /* distance from x to the half-line c + t u, t >= 0 (u unit) */
    double w[3], q[3];
    for (int k = 0; k < 3; ++k) w[k] = x[k] - c[k];
    double t = dot3(w, u);
    if (t < 0) t = 0;
    for (int k = 0; k < 3; ++k) q[k] = w[k] - t * u[k];
    return norm3(q);
}

static double ray_segment(const double *c, const double *u, const double *a, const double *b) {
    double best = ray_point(c, u, a);
    double d2 = ray_point(c, u, b);
    if (d2 < best) best = d2;
    d2 = seg_point(c, a, b);
    if (d2 < best) best = d2;
    /* both interiors: the common perpendicular of the two lines */
    double e[3], w[3];
    for (int k = 0; k < 3; ++k) { e[k] = b[k] - a[k]; w[k] = c[k] - a[k]; }
    double B = dot3(u, e), Cc = dot3(e, e), D = dot3(u, w), E = dot3(e, w);
    double den = Cc - B * B;   /* |u| = 1 */
    if (den > 1e-300 * (Cc > 1 ? Cc : 1)) {
        double t = (B * E - Cc * D) / den, sp = (E - B * D) / den;
        if (t > 0 && sp > 0 && sp < 1) {
            double q[3];
            for (int k = 0; k < 3; ++k) q[k] = w[k] + t * u[k] - sp * e[k];
            d2 = norm3(q);
            if (d2 < best) best = d2;
        }
    }
    return best;
}

static double tri_point(const double *x, const double v[3][3]) {
    /* distance from x to the triangle: the plane when x projects inside it,
     * else the nearest edge */
    double e1[3], e2[3], w[3], nrm[3];
    for (int k = 0; k < 3; ++k) { e1[k] = v[1][k] - v[0][k]; e2[k] = v[2][k] - v[0][k]; w[k] = x[k] - v[0][k]; }
    cross3(e1, e2, nrm);
    double nn = dot3(nrm, nrm);
    if (nn > 0) {
        /* barycentric coordinates of the projection */
        double d11 = dot3(e1, e1), d12 = dot3(e1, e2), d22 = dot3(e2, e2), dw1 = dot3(w, e1), dw2 = dot3(w, e2);
        double den = d11 * d22 - d12 * d12;
        double b1 = (d22 * dw1 - d12 * dw2) / den, b2 = (d11 * dw2 - d12 * dw1) / den;
        if (b1 >= 0 && b2 >= 0 && b1 + b2 <= 1) return fabs(dot3(w, nrm)) / sqrt(nn);
    }
    double best = seg_point(x, v[0], v[1]), d;
    if ((d = seg_point(x, v[1], v[2])) < best) best = d;
    if ((d = seg_point(x, v[2], v[0])) < best) best = d;
    return best;
}

static int ray_meets(const double *c, const double *u, const double v[3][3]) {
    /* the half-line meets the (closed) triangle: signed volumes */
    double a[3], b[3], cc[3], X[3];
    for (int k = 0; k < 3; ++k) { a[k] = v[0][k] - c[k]; b[k] = v[1][k] - c[k]; cc[k] = v[2][k] - c[k]; }
    cross3(b, cc, X);
    double e0 = dot3(u, X);
    cross3(cc, a, X);
    double e1 = dot3(u, X);
    cross3(a, b, X);
    double e2 = dot3(u, X);
    if (!((e0 >= 0 && e1 >= 0 && e2 >= 0) || (e0 <= 0 && e1 <= 0 && e2 <= 0))) return 0;
    double ba[3], ca[3], P[3];
    for (int k = 0; k < 3; ++k) { ba[k] = b[k] - a[k]; ca[k] = cc[k] - a[k]; }
    cross3(ba, ca, P);
    double h = dot3(a, P), q = dot3(u, P);
    return (h >= 0 && q > 0) || (h <= 0 && q < 0);
}

double orc_tool_distance(const double *v9, const double *c, const double *u) {
    double v[3][3];
    memcpy(v, v9, sizeof(v));
    if (ray_meets(c, u, v)) return 0.0;
    double best = tri_point(c, v), d;
    for (int k = 0; k < 3; ++k)
        if ((d = ray_segment(c, u, v[k], v[(k + 1) % 3])) < best) best = d;
    return best;
}

/* Distances of a ball-end tool with a holder (Section 3.3 names tool reach;
 * the holder is this library's extension).  The cutter and its shank are the
 * plain tool, every point within r of the half-line from the tip centre c
 * along u; the holder is every point within R of the half-line from
 * g = c + (len + R) u: a cylinder of radius R whose rounded nose reaches down
 * exactly to c + len u, the end of the cutting length, and never below it.
 * out[0] = distance from the tool's half-line to the triangle, out[1] =
 * distance from the holder's half-line.  With R = r the holder lies inside
 * the tool, so the pair decides as the plain tool does. */
void orc_tool_holder_distances(const double *v9, const double *c, const double *u, double len, double R,
                               double *out) {
    double g[3];
    for (int k = 0; k < 3; ++k) g[k] = c[k] + (len + R) * u[k];
    out[0] = orc_tool_distance(v9, c, u);
    out[1] = orc_tool_distance(v9, g, u);
}

/* bits: 1 = free; amb: 1 = some triangle within +-band of thr and none below
 * thr - band (excluded from comparisons).  kind as in orc_cast. */
int orc_cast_tool_holder(const float *V, const int32_t *T, int64_t nt, const float *Pt, const float *Nrm,
                         int64_t s0, int64_t s1, const float *dirs, int32_t N, int32_t kind, double r, double len,
                         double R, double tol, double band, uint32_t *bits, uint32_t *amb, int32_t nthreads) {
    const int32_t W = (N + 31) / 32;
    const double thr = r - tol, thr_h = R - tol;
    const int holder = len > 0.0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = s0; s < s1; ++s) {
        const float *n = Nrm + 3 * s, *p = Pt + 3 * s;
        float t3[3], b3[3];
        orc_frame(n, t3, b3);
        double c[3];
        for (int k = 0; k < 3; ++k) c[k] = (double)p[k] + r * (double)n[k];
        uint32_t *rb = bits + (s - s0) * W, *ra = amb + (s - s0) * W;
        for (int32_t w = 0; w < W; ++w) rb[w] = ra[w] = 0;
        for (int32_t j = 0; j < N; ++j) {
            float d[3];
            if (kind == 0) world_dir(t3, b3, n, dirs + 3 * j, d);
            else { d[0] = dirs[3 * j]; d[1] = dirs[3 * j + 1]; d[2] = dirs[3 * j + 2]; }
            if (kind == 1 && n[0] * d[0] + n[1] * d[1] + n[2] * d[2] < 0.0f) continue;   /* culled */
            double dd[3] = {d[0], d[1], d[2]};
            double L = sqrt((dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2]);
            double u[3] = {dd[0] / L, dd[1] / L, dd[2] / L};
            int blocked = 0, near = 0;
            for (int64_t f = 0; f < nt && !blocked; ++f) {
                double v[3][3];
                tri_verts(V, T, f, v);
                if (!holder) {
                    double dist = orc_tool_distance(&v[0][0], c, u);
                    if (dist < thr - band) blocked = 1;
                    else if (dist <= thr + band) near = 1;
                } else {
                    double dd2[2];
                    orc_tool_holder_distances(&v[0][0], c, u, len, R, dd2);
                    if (dd2[0] < thr - band || dd2[1] < thr_h - band) blocked = 1;
                    else if (dd2[0] <= thr + band || dd2[1] <= thr_h + band) near = 1;
                }
            }
            uint32_t m = 1u << (j & 31);
            if (!blocked && !near) rb[j >> 5] |= m;
            if (!blocked && near) ra[j >> 5] |= m;
        }
    }
    return 0;
}

int orc_cast_tool(const float *V, const int32_t *T, int64_t nt, const float *Pt, const float *Nrm, int64_t s0,
                  int64_t s1, const float *dirs, int32_t N, int32_t kind, double r, double tol, double band,
                  uint32_t *bits, uint32_t *amb, int32_t nthreads) {
    return orc_cast_tool_holder(V, T, nt, Pt, Nrm, s0, s1, dirs, N, kind, r, 0.0, r, tol, band, bits, amb, nthreads);
}

/* Decision of one (ray, triangle) pair, for tests: returns DEC_* and the
 * informational exact-sign verdict. */
int orc_decide_one(const double *v9, const double *o, const double *d, int32_t *info) {
    double v[3][3];
    for (int k = 0; k < 3; ++k)
        for (int c = 0; c < 3; ++c) v[k][c] = v9[3 * k + c];
    tri_pre tp;
    tri_prepare(v, o, &tp);
    int ib = 0;
    int r = tp.degenerate ? DEC_MISS : decide(&tp, d, &ib);
    *info = ib;
    return r;
}

/* ------------------------------------------------------------------------ */
/* Section 3.3 directional statistics per sample.  U = set bits of the row,
 * d_j the world direction of ray j (as cast).  In FP64, in direction order:
 *   m = (1/|U|) sum d_j (signed mean), A_k = (1/|U|) sum |d_jk|;
 * dominant axis k* = smallest k with |m_k| >= (1 - 1e-5) max |m|;
 * concentration c = A_k* / (A_x + A_y + A_z).  |U| = 0 -> axis -1.
 * tie[s] = 1 if the two largest |m_k| lie within 2e-5 relative.
 * Histogram: bin = zb*128 + az, zb = min(63, floor((z/|d| + 1) * 32)),
 * az = min(127, floor((atan2(y, x) + pi) * 128 / (2 pi))), FP64, counting
 * every unobstructed ray. */
void orc_dirstats(const float *Nrm, int64_t S, const float *dirs, int32_t N, const uint32_t *bits,
                  double *mean, double *absmean, int8_t *axis, double *conc, uint8_t *tie, uint64_t *hist) {
    const int32_t W = (N + 31) / 32;
    const double pi = 3.14159265358979323846264338327950288;
    for (int b = 0; b < 8192; ++b) hist[b] = 0;
    for (int64_t s = 0; s < S; ++s) {
        const float *n = Nrm + 3 * s;
        float t3[3], b3[3];
        orc_frame(n, t3, b3);
        double sm[3] = {0, 0, 0}, sa[3] = {0, 0, 0};
        int64_t cnt = 0;
        for (int32_t j = 0; j < N; ++j) {
            if (!((bits[s * W + (j >> 5)] >> (j & 31)) & 1u)) continue;
            float d[3];
            world_dir(t3, b3, n, dirs + 3 * j, d);
            for (int c = 0; c < 3; ++c) {
                sm[c] += (double)d[c];
                sa[c] += fabs((double)d[c]);
            }
            ++cnt;
            double dx = d[0], dy = d[1], dz = d[2];
            double len = sqrt(dx * dx + dy * dy + dz * dz);
            double zh = dz / len;
            int zb = (int)floor((zh + 1.0) * 32.0);
            if (zb > 63) zb = 63;
            if (zb < 0) zb = 0;
            int az = (int)floor((atan2(dy, dx) + pi) * 128.0 / (2.0 * pi));
            if (az > 127) az = 127;
            if (az < 0) az = 0;
            hist[zb * 128 + az] += 1;
        }
        if (cnt == 0) {
            for (int c = 0; c < 3; ++c) mean[3 * s + c] = absmean[3 * s + c] = 0.0;
            axis[s] = -1;
            conc[s] = 0.0;
            tie[s] = 0;
            continue;
        }
        double am[3];
        for (int c = 0; c < 3; ++c) {
            mean[3 * s + c] = sm[c] / (double)cnt;
            absmean[3 * s + c] = sa[c] / (double)cnt;
            am[c] = fabs(mean[3 * s + c]);
        }
        double mx = fmax(am[0], fmax(am[1], am[2]));
        int k = 0;
        while (k < 2 && !(am[k] >= (1.0 - 1e-5) * mx)) ++k;
        axis[s] = (int8_t)k;
        double den = absmean[3 * s] + absmean[3 * s + 1] + absmean[3 * s + 2];
        conc[s] = absmean[3 * s + k] / den;
        double sorted[3] = {am[0], am[1], am[2]};
        for (int i = 0; i < 2; ++i)
            for (int j2 = 0; j2 < 2 - i; ++j2)
                if (sorted[j2] < sorted[j2 + 1]) { double t = sorted[j2]; sorted[j2] = sorted[j2 + 1]; sorted[j2 + 1] = t; }
        tie[s] = (sorted[0] - sorted[1] <= 2e-5 * sorted[0]) ? 1 : 0;
    }
}

/* Number of OpenMP threads the oracle will use. */
int32_t orc_max_threads(void) {
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

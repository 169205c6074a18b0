// Canonical machining frame of a part (Section 3.2: every part is turned into
// a canonical machining frame before the six orthogonal casts; the paper does
// not give the method).  The frame used here:
//
//   faces    FP64 unit normal of each nonzero-area face from its FP32
//            vertices, folded onto the upper hemisphere (a face and the face
//            opposite it name the same machining axis), and its area;
//   peak     integer area weights floor(area * 2^s) summed into the 8192
//            bins of the direction histogram; the heaviest bin (lowest index
//            on ties) is exact and independent of summation order;
//   a1       the area-weighted mean normal of that bin, refined by the mean
//            of the normals within 5 degrees, then within 2 degrees, each
//            normal signed to agree with the current axis;
//   a2       the same from the heaviest bin within 15 degrees of
//            perpendicular to a1, with its a1 component removed after every
//            step (the world axis least aligned with a1 if no such bin);
//   labels   Z = the axis with the most area on faces within 5 degrees of it,
//            X = the remaining axis of largest vertex extent, Y = Z x X; Z
//            and X have their largest component positive.
//
// Data flow, all on the caller's stream, ten launches: per-face records
// (normal, area) and bins are written once; each later pass streams them and
// leaves one partial per workgroup.  The fixed grid of FR_GRID workgroups and
// the fixed reduction order make every sum independent of scheduling, so the
// result is the same on every run.  A pass that needs the previous pass's
// result (an axis, a peak bin) derives it itself from that pass's partials or
// from the histogram: every workgroup computes the same value, so each step
// is one launch with no grid-wide synchronisation.  The histogram is built
// in LDS per workgroup and merged with one global atomic per nonzero bin:
// the faces of a CAD part crowd into a few bins, and per-face global atomics
// on those bins serialise.
#include "common.hpp"

namespace hra {
namespace {

constexpr int FR_BINS = 8192;      // 64 z bands x 128 azimuth sectors
constexpr int FR_THREADS = 256;
constexpr int FR_GRID = 256;       // workgroups of every reduction pass (fixed)
constexpr double FR_TIE_REL = 1e-9;
constexpr double FR_TIE_ABS = 1e-9;

enum : uint32_t { FR_BAD_INDEX = 1u, FR_EMPTY = 2u };

// Results of the steps, kept on the device between launches.
struct FrameState {
    double ax[6][3];              // ax[k]: the axis refinement step k used (k = 1, 2, 4, 5)
    double a[3][3];               // a1, a2, a3
    double amax;                  // largest face area
    int32_t b1, b2;
    int32_t shift;
    uint32_t err;
};

struct FacePart {                 // per workgroup of the face pass
    double amax;
    uint32_t err;
    uint32_t pad;
};

struct FinalPart {
    double s[4];                  // area aligned with a1, a2, a3; total area
    double lo[3], hi[3];          // vertex extent along a1, a2, a3
};

struct FrameWs {
    double4 *rec;                 // [nt] folded unit normal and area (all zero for a face of zero area)
    int32_t *bin;                 // [nt], -1 for a face of zero area
    unsigned long long *hist;     // [FR_BINS]
    FrameState *st;
    FacePart *fpart;              // [FR_GRID]
    double4 *part;                // [6][FR_GRID]
    FinalPart *fin;               // [FR_GRID]
};

__device__ inline double dot3(const double *x, const double *y) { return (x[0] * y[0] + x[1] * y[1]) + x[2] * y[2]; }

__device__ inline void normalise(double *x) {
    const double L = sqrt((x[0] * x[0] + x[1] * x[1]) + x[2] * x[2]);
    x[0] = x[0] / L;
    x[1] = x[1] / L;
    x[2] = x[2] / L;
}

// x without its component along the unit vector a, normalised.
__device__ inline void orth(double *x, const double *a) {
    const double d = dot3(x, a);
    x[0] = x[0] - d * a[0];
    x[1] = x[1] - d * a[1];
    x[2] = x[2] - d * a[2];
    normalise(x);
}

__device__ inline void cross3(const double *a, const double *b, double *o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// Bin of a unit direction (the direction histogram's definition, FP64):
// z band floor((z / |d| + 1) * 32), azimuth sector floor((atan2(y, x) + pi) *
// 128 / (2 pi)), both clamped to the table.
__device__ inline int32_t dir_bin64(double x, double y, double z) {
    const double zh = z / sqrt((x * x + y * y) + z * z);
    double fz = floor((zh + 1.0) * 32.0);
    fz = fz < 0.0 ? 0.0 : (fz > 63.0 ? 63.0 : fz);
    double fa = floor((atan2(y, x) + M_PI) * 128.0 / (2.0 * M_PI));
    fa = fa < 0.0 ? 0.0 : (fa > 127.0 ? 127.0 : fa);
    return (int32_t)fz * 128 + (int32_t)fa;
}

// Sum of a double4 across the workgroup in a fixed order (every thread's
// value enters the same tree position on every run); the result is returned
// to every thread.
__device__ double4 block_sum4(double4 v, double4 *lds) {
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int o = FR_THREADS / 2; o > 0; o >>= 1) {
        if (t < o) {
            double4 a = lds[t], b = lds[t + o];
            lds[t] = make_double4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
        }
        __syncthreads();
    }
    double4 r = lds[0];
    __syncthreads();
    return r;
}

// Sum of FR_GRID partials, the same fixed order in every workgroup.
__device__ double4 reduce_parts(const double4 *p, double4 *lds) {
    return block_sum4(p[threadIdx.x], lds);   // FR_GRID == FR_THREADS
}
static_assert(FR_GRID == FR_THREADS, "one partial per thread in the reductions");
static_assert(FR_BINS % FR_GRID == 0, "histogram zeroing by slices");

// Heaviest histogram bin among those `take` accepts (lowest index on ties),
// -1 if none holds weight; the same answer in every workgroup.
template <class Take>
__device__ int32_t heaviest_bin(const unsigned long long *hist, Take take, unsigned long long *sv, int32_t *sb) {
    const int t = threadIdx.x;
    unsigned long long best = 0ull;
    int32_t bb = -1;
    for (int b = t; b < FR_BINS; b += FR_THREADS) {   // b rises: the first maximum of the thread stays
        const unsigned long long h = hist[b];
        if (h > best && take(b)) {
            best = h;
            bb = b;
        }
    }
    sv[t] = best;
    sb[t] = bb;
    __syncthreads();
    for (int o = FR_THREADS / 2; o > 0; o >>= 1) {
        if (t < o) {
            const unsigned long long v2 = sv[t + o];
            const int32_t b2 = sb[t + o];
            if (b2 >= 0 && (sb[t] < 0 || v2 > sv[t] || (v2 == sv[t] && b2 < sb[t]))) {
                sv[t] = v2;
                sb[t] = b2;
            }
        }
        __syncthreads();
    }
    const int32_t r = sb[0];
    __syncthreads();
    return r;
}

// The normalised sum S, or `keep` when no face was selected (empty cone).
__device__ inline void axis_from(const double4 &S, const double *keep, double *x) {
    if (S.w > 0.0) {
        x[0] = S.x;
        x[1] = S.y;
        x[2] = S.z;
        normalise(x);
    } else {
        x[0] = keep[0];
        x[1] = keep[1];
        x[2] = keep[2];
    }
}

// Per face: bounds check, FP64 normal and area, fold, bin; per workgroup the
// largest area and the error bits.  Also clears the global histogram.
__global__ __launch_bounds__(FR_THREADS) void k_fr_faces(const float *v, int64_t nv, const int32_t *t, int64_t nt,
                                                          FrameWs w) {
    __shared__ double smax[FR_THREADS];
    __shared__ uint32_t serr[FR_THREADS];
    const int tid = threadIdx.x;
    for (int b = blockIdx.x * (FR_BINS / FR_GRID) + tid; b < (blockIdx.x + 1) * (FR_BINS / FR_GRID); b += FR_THREADS)
        w.hist[b] = 0ull;
    double amax = 0.0;
    uint32_t err = 0;
    for (int64_t i = (int64_t)blockIdx.x * FR_THREADS + tid; i < nt; i += (int64_t)FR_GRID * FR_THREADS) {
        const int32_t i0 = t[3 * i], i1 = t[3 * i + 1], i2 = t[3 * i + 2];
        double4 r = make_double4(0.0, 0.0, 0.0, 0.0);
        int32_t bin = -1;
        if (i0 < 0 || i1 < 0 || i2 < 0 || i0 >= nv || i1 >= nv || i2 >= nv) {
            err |= FR_BAD_INDEX;
        } else {
            const double ax = v[3 * (int64_t)i0], ay = v[3 * (int64_t)i0 + 1], az = v[3 * (int64_t)i0 + 2];
            const double e1x = v[3 * (int64_t)i1] - ax, e1y = v[3 * (int64_t)i1 + 1] - ay,
                         e1z = v[3 * (int64_t)i1 + 2] - az;
            const double e2x = v[3 * (int64_t)i2] - ax, e2y = v[3 * (int64_t)i2 + 1] - ay,
                         e2z = v[3 * (int64_t)i2 + 2] - az;
            const double Nx = e1y * e2z - e1z * e2y;
            const double Ny = e1z * e2x - e1x * e2z;
            const double Nz = e1x * e2y - e1y * e2x;
            const double L = sqrt((Nx * Nx + Ny * Ny) + Nz * Nz);
            if (L > 0.0) {
                double nx = Nx / L, ny = Ny / L, nz = Nz / L;
                // Fold by a select, not a branch: the short-circuit form of
                // this test, with the negation under it, was compiled for
                // gfx950 so that lanes with nz == 0 kept the unfolded normal.
                const bool flip = (nz < 0.0) | ((nz == 0.0) & ((ny < 0.0) | ((ny == 0.0) & (nx < 0.0))));
                const double sg = flip ? -1.0 : 1.0;
                // times -1 is exact; + 0 turns -0 into +0 (not an identity
                // under IEEE rules, so it stays): the azimuth of (0, 0, 1)
                // must not depend on a zero's sign
                nx = nx * sg + 0.0;
                ny = ny * sg + 0.0;
                nz = nz * sg + 0.0;
                const double area = 0.5 * L;
                r = make_double4(nx, ny, nz, area);
                bin = dir_bin64(nx, ny, nz);
                amax = fmax(amax, area);
            }
        }
        w.rec[i] = r;
        w.bin[i] = bin;
    }
    smax[tid] = amax;
    serr[tid] = err;
    __syncthreads();
    for (int o = FR_THREADS / 2; o > 0; o >>= 1) {
        if (tid < o) {
            smax[tid] = fmax(smax[tid], smax[tid + o]);
            serr[tid] |= serr[tid + o];
        }
        __syncthreads();
    }
    if (tid == 0) {
        FacePart f;
        f.amax = smax[0];
        f.err = serr[0];
        f.pad = 0;
        w.fpart[blockIdx.x] = f;
    }
}

// Integer weights into a workgroup histogram in LDS, then one global atomic
// per nonzero bin.  Every workgroup first reduces the face pass's partials
// (largest area, error bits); workgroup 0 also resets the state.
__global__ __launch_bounds__(FR_THREADS) void k_fr_hist(int64_t nt, FrameWs w) {
    __shared__ unsigned long long h[FR_BINS];
    __shared__ double smax[FR_THREADS];
    __shared__ uint32_t serr[FR_THREADS];
    const int tid = threadIdx.x;
    const FacePart f = w.fpart[tid];
    smax[tid] = f.amax;
    serr[tid] = f.err;
    for (int b = tid; b < FR_BINS; b += FR_THREADS) h[b] = 0ull;
    __syncthreads();
    for (int o = FR_THREADS / 2; o > 0; o >>= 1) {
        if (tid < o) {
            smax[tid] = fmax(smax[tid], smax[tid + o]);
            serr[tid] |= serr[tid + o];
        }
        __syncthreads();
    }
    const double amax = smax[0];
    int e = 0;
    frexp(amax, &e);                      // amax = m 2^e, m in [0.5, 1)
    const int s = 31 - e;
    if (blockIdx.x == 0 && tid == 0) {
        FrameState z = {};
        z.amax = amax;
        z.b1 = -1;
        z.b2 = -1;
        z.shift = s;
        z.err = serr[0];
        *w.st = z;
    }
    for (int64_t i = (int64_t)blockIdx.x * FR_THREADS + tid; i < nt; i += (int64_t)FR_GRID * FR_THREADS) {
        const int32_t b = w.bin[i];
        if (b < 0) continue;
        const unsigned long long wt = (unsigned long long)floor(ldexp(w.rec[i].w, s));
        if (wt) atomicAdd(&h[b], wt);
    }
    __syncthreads();
    for (int b = tid; b < FR_BINS; b += FR_THREADS)
        if (h[b]) atomicAdd(&w.hist[b], h[b]);
}

// One refinement pass.  Steps:
//   0  peak b1 from the histogram, mean of bin b1
//   1  cone 5 deg about a1 from step 0
//   2  cone 2 deg about a1 from step 1
//   3  a1 from step 2, peak b2 among the bins within 15 degrees of
//      perpendicular to it, mean of bin b2
//   4  cone 5 deg about a2 from step 3
//   5  cone 2 deg about a2 from step 4
// Partial: sum of area * sign * n over the selected faces, w = their area.
struct PassArgs {
    int step;
    double cos_cone;       // steps 1, 2, 4, 5
    double perp_cos;       // step 3
    const double4 *prev;   // partials of the previous step (steps 1 to 5)
    double4 *out;
};

__global__ __launch_bounds__(FR_THREADS) void k_fr_pass(int64_t nt, FrameWs w, PassArgs p) {
    __shared__ double4 lds[FR_THREADS];
    __shared__ unsigned long long sv[FR_THREADS];
    __shared__ int32_t sb[FR_THREADS];
    __shared__ double sec_c[128], sec_s[128], band_z[64], band_r[64];
    FrameState *st = w.st;
    const int tid = threadIdx.x;
    const bool lead = blockIdx.x == 0 && tid == 0;
    double c[3] = {0.0, 0.0, 0.0};
    int32_t bsel = -1;
    if (p.step == 0) {
        bsel = heaviest_bin(w.hist, [](int) { return true; }, sv, sb);
        if (lead) {
            st->b1 = bsel;
            if (bsel < 0) st->err |= FR_EMPTY;
        }
        if (bsel < 0) return;            // no face with nonzero area
    } else if (p.step == 3) {
        if (st->b1 < 0) return;
        double a1[3];
        const double4 S = reduce_parts(p.prev, lds);
        axis_from(S, st->ax[2], a1);
        if (tid < 128) {
            const double phi = (tid + 0.5) * (2.0 * M_PI / 128.0) - M_PI;
            sec_c[tid] = cos(phi);
            sec_s[tid] = sin(phi);
        } else if (tid < 192) {
            const double z = ((tid - 128) + 0.5) / 32.0 - 1.0;
            const double r2 = 1.0 - z * z;
            band_z[tid - 128] = z;
            band_r[tid - 128] = sqrt(r2 > 0.0 ? r2 : 0.0);
        }
        __syncthreads();
        // candidates: bin centres (r cos phi, r sin phi, z) with |centre . a1| <= cos 75 deg
        bsel = heaviest_bin(
            w.hist,
            [&](int b) {
                const double r = band_r[b >> 7], ctr[3] = {r * sec_c[b & 127], r * sec_s[b & 127], band_z[b >> 7]};
                return !(fabs(dot3(ctr, a1)) > p.perp_cos);
            },
            sv, sb);
        if (lead) {
            for (int k = 0; k < 3; ++k) st->a[0][k] = a1[k];
            st->b2 = bsel;
        }
        if (bsel < 0) return;            // no second peak: a2 is taken from the world axes
    } else {
        const int second = p.step > 3;
        if (st->b1 < 0 || (second && st->b2 < 0)) return;
        // every workgroup derives the same axis; the fallback for an empty
        // cone is the previous step's axis, written by an earlier launch
        const double4 S = reduce_parts(p.prev, lds);
        axis_from(S, st->ax[p.step - 1], c);
        if (second) orth(c, st->a[0]);
        if (lead)
            for (int k = 0; k < 3; ++k) st->ax[p.step][k] = c[k];
    }
    double4 acc = make_double4(0.0, 0.0, 0.0, 0.0);
    if (bsel >= 0) {                     // mean of one bin
        for (int64_t i = (int64_t)blockIdx.x * FR_THREADS + tid; i < nt; i += (int64_t)FR_GRID * FR_THREADS) {
            if (w.bin[i] != bsel) continue;
            const double4 r = w.rec[i];
            acc.x += r.w * r.x;
            acc.y += r.w * r.y;
            acc.z += r.w * r.z;
            acc.w += r.w;
        }
    } else {                             // cone about c
        for (int64_t i = (int64_t)blockIdx.x * FR_THREADS + tid; i < nt; i += (int64_t)FR_GRID * FR_THREADS) {
            const double4 r = w.rec[i];
            if (r.w == 0.0) continue;
            const double n[3] = {r.x, r.y, r.z};
            const double d = dot3(n, c);
            if (fabs(d) < p.cos_cone) continue;
            const double ws = r.w * (d > 0.0 ? 1.0 : -1.0);
            acc.x += ws * r.x;
            acc.y += ws * r.y;
            acc.z += ws * r.z;
            acc.w += r.w;
        }
    }
    const double4 S = block_sum4(acc, lds);
    if (tid == 0) p.out[blockIdx.x] = S;
}

// Index of the largest of three values; values within a relative FR_TIE_REL
// of the current best count as equal and the earlier index wins.
__device__ inline int first_max3(const double *v) {
    int best = 0;
    for (int k = 1; k < 3; ++k)
        if (v[k] > v[best] * (1.0 + FR_TIE_REL)) best = k;
    return best;
}

// a or -a: the one whose largest component (the first within FR_TIE_ABS of
// the largest magnitude) is positive.
__device__ inline void sign_fix(double *a) {
    const double m = fmax(fmax(fabs(a[0]), fabs(a[1])), fabs(a[2]));
    int k = 0;
    while (k < 2 && !(fabs(a[k]) >= m - FR_TIE_ABS)) ++k;
    if (a[k] < 0.0) {
        a[0] = -a[0];
        a[1] = -a[1];
        a[2] = -a[2];
    }
}

// Last pass: a2 and a3 finished, then per workgroup the area aligned with
// each axis (faces within 5 degrees), the total area and the vertex extent
// along each axis.
__global__ __launch_bounds__(FR_THREADS) void k_fr_aligned(const float *v, int64_t nv, int64_t nt, FrameWs w,
                                                            const double4 *prev, double cos_wide) {
    __shared__ double4 lds[FR_THREADS];
    __shared__ double red[6][FR_THREADS];
    FrameState *st = w.st;
    double a[3][3];
    for (int k = 0; k < 3; ++k) a[0][k] = st->a[0][k];
    if (st->b2 >= 0) {
        const double4 S = reduce_parts(prev, lds);
        axis_from(S, st->ax[5], a[1]);
        orth(a[1], a[0]);
    } else {
        // the world axis least aligned with a1 (ties: the earlier axis)
        double val[3];
        for (int k = 0; k < 3; ++k) val[k] = -fabs(a[0][k]) + 2.0;
        const int k = first_max3(val);
        a[1][0] = k == 0 ? 1.0 : 0.0;
        a[1][1] = k == 1 ? 1.0 : 0.0;
        a[1][2] = k == 2 ? 1.0 : 0.0;
        orth(a[1], a[0]);
    }
    cross3(a[0], a[1], a[2]);
    normalise(a[2]);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int j = 1; j < 3; ++j)
            for (int k = 0; k < 3; ++k) st->a[j][k] = a[j][k];

    double4 acc = make_double4(0.0, 0.0, 0.0, 0.0);
    for (int64_t i = (int64_t)blockIdx.x * FR_THREADS + threadIdx.x; i < nt; i += (int64_t)FR_GRID * FR_THREADS) {
        const double4 r = w.rec[i];
        if (r.w == 0.0) continue;
        const double n[3] = {r.x, r.y, r.z};
        if (fabs(dot3(n, a[0])) >= cos_wide) acc.x += r.w;
        if (fabs(dot3(n, a[1])) >= cos_wide) acc.y += r.w;
        if (fabs(dot3(n, a[2])) >= cos_wide) acc.z += r.w;
        acc.w += r.w;
    }
    const double4 S = block_sum4(acc, lds);

    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * FR_THREADS + threadIdx.x; i < nv; i += (int64_t)FR_GRID * FR_THREADS) {
        const double p[3] = {v[3 * i], v[3 * i + 1], v[3 * i + 2]};
        for (int k = 0; k < 3; ++k) {
            const double d = dot3(p, a[k]);
            lo[k] = fmin(lo[k], d);
            hi[k] = fmax(hi[k], d);
        }
    }
    const int t = threadIdx.x;
    for (int k = 0; k < 3; ++k) {
        red[k][t] = lo[k];
        red[3 + k][t] = hi[k];
    }
    __syncthreads();
    for (int o = FR_THREADS / 2; o > 0; o >>= 1) {
        if (t < o)
            for (int k = 0; k < 3; ++k) {
                red[k][t] = fmin(red[k][t], red[k][t + o]);
                red[3 + k][t] = fmax(red[3 + k][t], red[3 + k][t + o]);
            }
        __syncthreads();
    }
    if (t == 0) {
        FinalPart f;
        f.s[0] = S.x;
        f.s[1] = S.y;
        f.s[2] = S.z;
        f.s[3] = S.w;
        for (int k = 0; k < 3; ++k) {
            f.lo[k] = red[k][0];
            f.hi[k] = red[3 + k][0];
        }
        w.fin[blockIdx.x] = f;
    }
}

// Labels and the output record (one workgroup).
__global__ __launch_bounds__(FR_THREADS) void k_fr_final(FrameWs w, hra_frame *out, uint32_t *ctx_err) {
    __shared__ double4 lds[FR_THREADS];
    __shared__ double red[6][FR_THREADS];
    const int t = threadIdx.x;
    const FinalPart f = w.fin[t];
    const double4 S = block_sum4(make_double4(f.s[0], f.s[1], f.s[2], f.s[3]), lds);
    for (int k = 0; k < 3; ++k) {
        red[k][t] = f.lo[k];
        red[3 + k][t] = f.hi[k];
    }
    __syncthreads();
    for (int o = FR_THREADS / 2; o > 0; o >>= 1) {
        if (t < o)
            for (int k = 0; k < 3; ++k) {
                red[k][t] = fmin(red[k][t], red[k][t + o]);
                red[3 + k][t] = fmax(red[3 + k][t], red[3 + k][t + o]);
            }
        __syncthreads();
    }
    if (t != 0) return;
    const FrameState *st = w.st;
    hra_frame r = {};
    r.error = st->err;
    r.peak_bin[0] = st->b1;
    r.peak_bin[1] = st->b2;
    r.shift = st->shift;
    if (st->err) {
        for (int k = 0; k < 3; ++k) r.axes[k][k] = 1.0;
        *out = r;
        atomicOr(ctx_err, (st->err & FR_BAD_INDEX ? ERR_BAD_INDEX : 0u) | (st->err & FR_EMPTY ? ERR_EMPTY_MESH : 0u));
        return;
    }
    double a[3][3];
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) a[j][k] = st->a[j][k];
    const double al[3] = {S.x, S.y, S.z};
    double ext[3];
    for (int k = 0; k < 3; ++k) ext[k] = red[3 + k][0] - red[k][0];
    const int kz = first_max3(al);
    const int i = kz == 0 ? 1 : 0, j = kz == 2 ? 1 : 2;
    const int kx = ext[j] > ext[i] * (1.0 + FR_TIE_REL) ? j : i;
    const int ky = 3 - kz - kx;
    double X[3], Y[3], Z[3];
    for (int k = 0; k < 3; ++k) {
        X[k] = a[kx][k];
        Z[k] = a[kz][k];
    }
    sign_fix(Z);
    sign_fix(X);
    cross3(Z, X, Y);
    for (int k = 0; k < 3; ++k) {
        r.axes[0][k] = X[k];
        r.axes[1][k] = Y[k];
        r.axes[2][k] = Z[k];
    }
    r.aligned[0] = al[kx];
    r.aligned[1] = al[ky];
    r.aligned[2] = al[kz];
    r.extent[0] = ext[kx];
    r.extent[1] = ext[ky];
    r.extent[2] = ext[kz];
    r.total_area = S.w;
    r.confidence = ((al[0] + al[1]) + al[2]) / S.w;
    *out = r;
}

// v' = F v in FP32, F the frame rounded to FP32: v'_k = (f_k0 x + f_k1 y) + f_k2 z.
// A frame that carries an error leaves the vertices unchanged.
__global__ __launch_bounds__(FR_THREADS) void k_fr_apply(const hra_frame *fr, const float *in, float *out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * FR_THREADS + threadIdx.x;
    if (i >= n) return;
    const float x = in[3 * i], y = in[3 * i + 1], z = in[3 * i + 2];
    if (fr->error) {
        out[3 * i] = x;
        out[3 * i + 1] = y;
        out[3 * i + 2] = z;
        return;
    }
    float o[3];
    for (int k = 0; k < 3; ++k) {
        const float f0 = (float)fr->axes[k][0], f1 = (float)fr->axes[k][1], f2 = (float)fr->axes[k][2];
        o[k] = (f0 * x + f1 * y) + f2 * z;
    }
    out[3 * i] = o[0];
    out[3 * i + 1] = o[1];
    out[3 * i + 2] = o[2];
}

int64_t blocks_for(int64_t n) { return (n + FR_THREADS - 1) / FR_THREADS; }

}  // namespace

// Enqueue the whole estimate on s with workspace ws (frame_ws_bytes(nt)).
size_t frame_ws_bytes(int64_t nt) {
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return up(sizeof(double4) * nt) + up(sizeof(int32_t) * nt) + up(sizeof(unsigned long long) * FR_BINS) +
           up(sizeof(FrameState)) + up(sizeof(FacePart) * FR_GRID) + up(sizeof(double4) * 6 * FR_GRID) +
           up(sizeof(FinalPart) * FR_GRID);
}

hipError_t enqueue_frame(const float *v, int64_t nv, const int32_t *t, int64_t nt, void *ws, unsigned long long *hist,
                         hra_frame *out, uint32_t *ctx_err, hipStream_t s) {
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char *p = (char *)ws;
    FrameWs w;
    w.rec = (double4 *)p;
    p += up(sizeof(double4) * nt);
    w.bin = (int32_t *)p;
    p += up(sizeof(int32_t) * nt);
    w.hist = (unsigned long long *)p;
    p += up(sizeof(unsigned long long) * FR_BINS);
    if (hist) w.hist = hist;
    w.st = (FrameState *)p;
    p += up(sizeof(FrameState));
    w.fpart = (FacePart *)p;
    p += up(sizeof(FacePart) * FR_GRID);
    w.part = (double4 *)p;
    p += up(sizeof(double4) * 6 * FR_GRID);
    w.fin = (FinalPart *)p;

    const double cos_wide = cos(5.0 * (M_PI / 180.0));
    const double cos_fine = cos(2.0 * (M_PI / 180.0));
    const double perp_cos = cos(75.0 * (M_PI / 180.0));

    k_fr_faces<<<FR_GRID, FR_THREADS, 0, s>>>(v, nv, t, nt, w);
    k_fr_hist<<<FR_GRID, FR_THREADS, 0, s>>>(nt, w);
    for (int step = 0; step < 6; ++step) {
        PassArgs a;
        a.step = step;
        a.cos_cone = step % 3 == 2 ? cos_fine : cos_wide;
        a.perp_cos = perp_cos;
        a.prev = step == 0 ? nullptr : w.part + (step - 1) * FR_GRID;
        a.out = w.part + step * FR_GRID;
        k_fr_pass<<<FR_GRID, FR_THREADS, 0, s>>>(nt, w, a);
    }
    k_fr_aligned<<<FR_GRID, FR_THREADS, 0, s>>>(v, nv, nt, w, w.part + 5 * FR_GRID, cos_wide);
    k_fr_final<<<1, FR_THREADS, 0, s>>>(w, out, ctx_err);
    return hipGetLastError();
}

}  // namespace hra

using namespace hra;

extern "C" {

int64_t hra_frame_ws_bytes(int64_t n_tris) { return n_tris > 0 ? (int64_t)frame_ws_bytes(n_tris) : 0; }

hra_status hra_frame_estimate(hra_ctx *ctx, const hra_mesh *mesh, uint64_t *d_hist, hra_frame *d_frame, void *stream) {
    if (!ctx) return HRA_ERR_INVALID_ARG;
    if (!mesh || !d_frame || !mesh->d_verts || !mesh->d_tris) return ctx->fail(HRA_ERR_INVALID_ARG, "frame: null argument");
    if (mesh->n_tris <= 0 || mesh->n_verts <= 0 || mesh->n_tris > ((int64_t)1 << 31) - FR_THREADS)
        return ctx->fail(HRA_ERR_INVALID_ARG, "frame: n_tris must be in [1, 2^31 - 256], n_verts >= 1");
    hipStream_t s = (hipStream_t)stream;
    void *ws = nullptr;
    HRA_HIP(hipMallocAsync(&ws, frame_ws_bytes(mesh->n_tris), s));
    hipError_t e = enqueue_frame(mesh->d_verts, mesh->n_verts, mesh->d_tris, mesh->n_tris, ws,
                                 (unsigned long long *)d_hist, d_frame, ctx->d_err, s);
    hipError_t e2 = hipFreeAsync(ws, s);
    if (e != hipSuccess) return ctx->fail(HRA_ERR_DEVICE, "frame kernels", hipGetErrorString(e));
    if (e2 != hipSuccess) return ctx->fail(HRA_ERR_DEVICE, "hipFreeAsync", hipGetErrorString(e2));
    return HRA_OK;
}

hra_status hra_frame_apply(hra_ctx *ctx, const hra_frame *d_frame, const float *d_in, float *d_out, int64_t n_verts,
                           void *stream) {
    if (!ctx) return HRA_ERR_INVALID_ARG;
    if (!d_frame || !d_in || !d_out || n_verts < 0) return ctx->fail(HRA_ERR_INVALID_ARG, "frame apply: bad argument");
    if (n_verts == 0) return HRA_OK;
    hipStream_t s = (hipStream_t)stream;
    k_fr_apply<<<(unsigned)blocks_for(n_verts), FR_THREADS, 0, s>>>(d_frame, d_in, d_out, n_verts);
    HRA_HIP(hipGetLastError());
    return HRA_OK;
}

}  // extern "C"

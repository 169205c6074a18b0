// Directional statistics, classification, reachability and setups
// (Section 3.3).
#include "common.hpp"
#include "stages.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>
#include <map>
#include <mutex>

namespace hra {

struct DirTotals {
    unsigned long long n_axis[3];
    unsigned long long n_blind;
    unsigned long long n_unob;
    unsigned long long conc_fx;   // sum of round(concentration x 2^32): an integer, so any order gives it
    double pad[2];
};

constexpr int HIST_BINS = 8192;
constexpr float HIST_EDGE = 5e-4f;   // zenith bins: distance from an edge below which FP64 decides

// Azimuth sectors.  Within a quadrant the pseudo-angle p = |y| / (|x| + |y|)
// rises strictly with a = atan2(|y|, |x|) in [0, pi/2], so the sector
// boundaries a_k = k pi / 64 (k = 0..32) are boundaries p_k of p.  A table
// of AZ_CELLS + 1 cells per quadrant over p in [0, 1] holds, for each cell,
// the last boundary at or below the cell's start, the next boundary, and the
// sector (as a byte offset into a histogram row) on either side of that next
// boundary.  Boundaries lie at least 0.5 pi/64 = 0.0245 apart in p (dp/da
// is 1 / (cos a + sin a)^2 >= 1/2), more than a cell's width, so a cell holds
// at most one.  The FP32 p (one add, the hardware reciprocal, one multiply)
// is within 2e-7 of the exact value and the table's FP32 boundaries within
// 6e-8, so wherever p lies at least AZ_EPS from both boundaries the FP32
// comparison gives the sector of the exact angle.
constexpr int AZ_CELLS = 128;
constexpr int AZ_TAB = 4 * (AZ_CELLS + 1);
constexpr float AZ_EPS = 4e-6f;
static __device__ float4 az_table[AZ_TAB];

// Directions per wave whose bin is taken in FP64 after the sample (beyond
// this many, in place).
constexpr int EDGE_Q = 64;
constexpr int DS_WAVES = 8;           // waves per k_dirstats block
constexpr int DS_BLOCKS_PER_CU = 3;   // LDS: 3 x 46.3 KiB of the 160 KiB

__device__ inline bool near_zenith_edge(float xz) {
    const float f = __builtin_amdgcn_fractf(xz);
    return !(fabsf(f - 0.5f) < 0.5f - HIST_EDGE);
}

// Histogram bin of direction d by the definition, in FP64.
__device__ __noinline__ int hist_bin_fp64(float fx, float fy, float fz) {
    const double pi = 3.14159265358979323846264338327950288;
    const double dx = fx, dy = fy, dz = fz;
    int zb = (int)floor((dz / sqrt(dx * dx + dy * dy + dz * dz) + 1.0) * 32.0);
    int az = (int)floor((atan2(dy, dx) + pi) * 128.0 / (2.0 * pi));
    zb = zb > 63 ? 63 : (zb < 0 ? 0 : zb);
    az = az > 127 ? 127 : (az < 0 ? 0 : az);
    return zb * 128 + az;
}

// One wavefront per sample, DS_WAVES per block.  Per 4096-direction chunk the
// wave stages the row's bit words in LDS (zero past the last direction) and
// each lane takes directions lane, lane + 64, ...; for a free direction l
// (local frame) it adds l to FP64 sums, rotates it to d = R l and adds
// |d| to FP32 sums (at most 64 terms per lane per chunk, folded into FP64 at
// the chunk's end: relative error below 4e-6), and bins d.  The world mean
// is R applied once, in FP64, to the local sum: the same quantity as the sum
// of the rotated directions, without their per-term rounding.
//
// Zenith: (d_z + 1) 32 in FP32 without renormalising d.  |d| is 1 within
// 6e-7 for a unit normal (|n|^2 within 1e-6 of 1, as sampled) and a table of
// unit directions, so the FP32 coordinate is within 3e-5 bins of the FP64
// one (d_z / |d| + 1) 32; outside HIST_EDGE of an edge both give one bin.
// Azimuth: the pseudo-angle table above.  A direction near an edge, or of a
// sample whose normal is not unit, goes to a per-wave LDS queue and is binned
// by the FP64 definition after the sample's loop, with all lanes.
//
// The histogram is privatised in LDS per block and written out without
// atomics to a per-block slice; k_hist_reduce sums the slices (integer sums:
// the same in any order).  Part totals are formed afterwards from the
// per-sample outputs by k_part_totals.
__global__ __launch_bounds__(64 * DS_WAVES) __attribute__((amdgpu_waves_per_eu(6))) void k_dirstats(const float *normal, int64_t n, const float4 *dirs,
                                                            int32_t N, int32_t W, const uint32_t *bits,
                                                            hra_dirstats out, double *conc64, uint32_t *cnt_out,
                                                            uint32_t *hist_part, const float4 *az_tab_g) {
    __shared__ uint32_t h[HIST_BINS];
    __shared__ float4 az_tab[AZ_TAB];
    __shared__ uint32_t rowbuf[DS_WAVES][128];
    __shared__ int32_t edgeq[DS_WAVES][EDGE_Q];
    __shared__ int32_t edgen[DS_WAVES];
    const bool want_hist = hist_part != nullptr;
    if (want_hist) {
        for (int k = threadIdx.x; k < HIST_BINS; k += blockDim.x) h[k] = 0;
        for (int k = threadIdx.x; k < AZ_TAB; k += blockDim.x) az_tab[k] = az_tab_g[k];
        __syncthreads();
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * DS_WAVES;
    for (int64_t s = (int64_t)blockIdx.x * DS_WAVES + wv; s < n; s += nwaves) {
        const float nx = normal[3 * s], ny = normal[3 * s + 1], nz = normal[3 * s + 2];
        float3 t, b;
        onb_frame(nx, ny, nz, t, b);
        const float nn = fmaf(nx, nx, fmaf(ny, ny, nz * nz));
        const bool unit = fabsf(nn - 1.0f) <= 1e-6f;
        double sl0 = 0, sl1 = 0, sl2 = 0, sa0 = 0, sa1 = 0, sa2 = 0;
        uint32_t cnt = 0;
        edgen[wv] = 0;
        for (int32_t c = 0; c < W; c += 128) {
            const int32_t cw = W - c < 128 ? W - c : 128;
            // an odd word count leaves the upper half-wave of the chunk's
            // last step one word past the row: that word is staged as zero
            const int32_t cwp = (cw + 1) & ~1;
            __builtin_amdgcn_wave_barrier();
            for (int32_t k = lane; k < cwp; k += 64) {
                uint32_t wd = k < cw ? bits[s * W + c + k] : 0u;
                if (c + k == W - 1 && (N & 31)) wd &= (1u << (N & 31)) - 1u;
                rowbuf[wv][k] = wd;
                cnt += __popc(wd);
            }
            __builtin_amdgcn_wave_barrier();
            const int32_t j0 = 32 * c;
            const int32_t nj = N - j0 < 4096 ? N - j0 : 4096;
            float fa0 = 0.f, fa1 = 0.f, fa2 = 0.f;
            // the table is readable DIR_TABLE_PAD entries past N, so neither
            // read is clamped and both address from a uniform base
            const float4 *dp = dirs + j0;
            float4 lnext = dp[lane];
            for (int32_t i = 0; i < nj; i += 64) {
                const int32_t j = j0 + i + lane;
                const float4 l = lnext;
                lnext = (dp + i + 64)[lane];
                const uint32_t wd = rowbuf[wv][(i >> 5) + (lane >> 5)];
                if ((wd >> (lane & 31)) & 1u) {
                    sl0 += (double)l.x;
                    sl1 += (double)l.y;
                    sl2 += (double)l.z;
                    const float3 d = rotate_dir(t, b, nx, ny, nz, l.x, l.y, l.z);
                    fa0 += fabsf(d.x);
                    fa1 += fabsf(d.y);
                    fa2 += fabsf(d.z);
                    if (want_hist) {
                        const float xz = fmaf(d.z, 32.0f, 32.0f);
                        const float p = fabsf(d.y) * __builtin_amdgcn_rcpf(fabsf(d.x) + fabsf(d.y));
                        const uint32_t cell = (uint32_t)(p * (float)AZ_CELLS);
                        const uint32_t q = ((__float_as_uint(d.x) >> 31) << 1) | (__float_as_uint(d.y) >> 31);
                        const float4 e = az_tab[q * (AZ_CELLS + 1) + (cell < AZ_CELLS ? cell : AZ_CELLS)];
                        // NaN p (x = y = 0) fails the comparison: FP64 path
                        const bool clear = fminf(p - e.x, fabsf(e.y - p)) >= AZ_EPS;
                        if (unit && clear && !near_zenith_edge(xz)) {
                            const uint32_t zb = min((uint32_t)xz, 63u);
                            const uint32_t az4 = __float_as_uint(p >= e.y ? e.w : e.z);
                            atomicAdd((uint32_t *)((char *)h + (zb << 9) + az4), 1u);
                        } else {
                            const int slot = atomicAdd(&edgen[wv], 1);
                            if (slot < EDGE_Q) edgeq[wv][slot] = j;
                            else atomicAdd(&h[hist_bin_fp64(d.x, d.y, d.z)], 1u);
                        }
                    }
                }
            }
            sa0 += (double)fa0;
            sa1 += (double)fa1;
            sa2 += (double)fa2;
        }
        __builtin_amdgcn_wave_barrier();
        if (want_hist) {
            const int32_t qn = edgen[wv];
            const int32_t ne = qn < EDGE_Q ? qn : EDGE_Q;
            for (int32_t k = lane; k < ne; k += 64) {
                const int32_t j = edgeq[wv][k];
                const float4 l = dirs[j];
                const float3 d = rotate_dir(t, b, nx, ny, nz, l.x, l.y, l.z);
                atomicAdd(&h[hist_bin_fp64(d.x, d.y, d.z)], 1u);
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            sl0 += __shfl_xor(sl0, off);
            sl1 += __shfl_xor(sl1, off);
            sl2 += __shfl_xor(sl2, off);
            sa0 += __shfl_xor(sa0, off);
            sa1 += __shfl_xor(sa1, off);
            sa2 += __shfl_xor(sa2, off);
            cnt += __shfl_xor(cnt, off);
        }
        // every lane holds the totals after the butterfly; all lanes store the
        // same values, with no lane-dependent branch ahead of the next
        // iteration's shuffles
        const double tx = t.x, ty = t.y, tz = t.z, bx = b.x, by = b.y, bz = b.z;
        const double sm0 = tx * sl0 + bx * sl1 + (double)nx * sl2;
        const double sm1 = ty * sl0 + by * sl1 + (double)ny * sl2;
        const double sm2 = tz * sl0 + bz * sl1 + (double)nz * sl2;
        const bool blind = cnt == 0;
        const double cd = blind ? 1.0 : (double)cnt;
        const double m[3] = {sm0 / cd, sm1 / cd, sm2 / cd}, A[3] = {sa0 / cd, sa1 / cd, sa2 / cd};
        const double am[3] = {fabs(m[0]), fabs(m[1]), fabs(m[2])};
        const double mx = fmax(am[0], fmax(am[1], am[2]));
        int k = 0;
        while (k < 2 && !(am[k] >= (1.0 - 1e-5) * mx)) ++k;
        const double den = A[0] + A[1] + A[2];
        const double cc = blind ? 0.0 : A[k] / den;
        const int qq = lane % 3;
        out.mean[3 * s + qq] = blind ? 0.0f : (float)m[qq];
        out.absmean[3 * s + qq] = blind ? 0.0f : (float)A[qq];
        out.axis[s] = blind ? (int8_t)-1 : (int8_t)k;
        out.conc[s] = (float)cc;
        conc64[s] = cc;
        cnt_out[s] = cnt;
    }
    if (want_hist) {
        __syncthreads();
        uint32_t *dst = hist_part + (int64_t)blockIdx.x * HIST_BINS;
        for (int k = threadIdx.x; k < HIST_BINS; k += blockDim.x) dst[k] = h[k];
    }
}

// The azimuth table, in FP64 on the host: boundary p_k = sin a_k / (sin a_k
// + cos a_k), and for quadrant (sign of x, sign of y) the sector of a
// quadrant angle in [a_k, a_k+1): a = phi (x, y >= 0), pi - phi (x < 0 <= y),
// phi + pi (x, y < 0), -phi (y < 0 <= x), with phi = atan2(y, x) and sector
// floor((phi + pi) 64 / pi).
static std::vector<float4> make_az_table() {
    const double pi = 3.14159265358979323846264338327950288;
    double pk[33];
    for (int k = 0; k <= 32; ++k) {
        const double a = k * pi / 64.0;
        pk[k] = k == 32 ? 1.0 : std::sin(a) / (std::sin(a) + std::cos(a));
    }
    auto as_float = [](uint32_t u) {
        float f;
        std::memcpy(&f, &u, sizeof f);
        return f;
    };
    std::vector<float4> tab(AZ_TAB);
    for (int q = 0; q < 4; ++q) {
        const int sx = q >> 1, sy = q & 1;
        auto sector4 = [&](int k) {
            k = k > 31 ? 31 : k;
            return 4u * (uint32_t)((sy ? 0 : 64) + ((sx ^ sy) ? 63 - k : k));
        };
        for (int c = 0; c <= AZ_CELLS; ++c) {
            const double lo = (double)c / AZ_CELLS;
            int kb = 0;
            for (int k = 1; k <= 31; ++k)
                if (pk[k] <= lo) kb = k;
            tab[q * (AZ_CELLS + 1) + c] = make_float4((float)pk[kb], (float)pk[kb + 1], as_float(sector4(kb)),
                                                      as_float(sector4(kb + 1)));
        }
    }
    return tab;
}

// Part totals over each part's sample range [base, base + n) (base ==
// NULL: one part, range [0, n_one)): counts per axis, blind samples,
// unobstructed rays, and the concentrations as integers round(c 2^32)
// (c in [0, 1], so 2^31 samples fit in 64 bits; the mean is then within
// 2^-33 of the FP64 mean).  Every total is an integer, so PT_CHUNKS blocks
// per part add their shares with atomics in any order and the result is
// the same on every run.  `tot` starts at zero (k_zero_u32).
constexpr int PT_THREADS = 256;
constexpr int PT_CHUNKS = 32;
__global__ __launch_bounds__(PT_THREADS) void k_part_totals(const int8_t *axis, const uint32_t *cnt,
                                                            const double *conc64, const int64_t *base,
                                                            const int64_t *count, int64_t n_one, DirTotals *tot) {
    __shared__ unsigned long long si[6][PT_THREADS / 64];
    const int p = blockIdx.y, t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t b0 = base ? base[p] : 0, n = base ? count[p] : n_one;
    unsigned long long a[6] = {0ull, 0ull, 0ull, 0ull, 0ull, 0ull};
    // a block-uniform trip count, lanes past the end adding zeros (selects),
    // so the shuffles below follow no lane-dependent loop exit
    for (int64_t i0 = b0 + (int64_t)blockIdx.x * PT_THREADS; i0 < b0 + n; i0 += (int64_t)PT_CHUNKS * PT_THREADS) {
        const int64_t i = i0 + t;
        const bool ok = i < b0 + n;
        const int64_t ic = ok ? i : i0;
        const int k = axis[ic];
        const unsigned long long c = cnt[ic], fx = __double2ull_rn(conc64[ic] * 4294967296.0);
        a[0] += (ok && k == 0) ? 1ull : 0ull;
        a[1] += (ok && k == 1) ? 1ull : 0ull;
        a[2] += (ok && k == 2) ? 1ull : 0ull;
        a[3] += (ok && k < 0) ? 1ull : 0ull;
        a[4] += ok ? c : 0ull;
        a[5] += ok ? fx : 0ull;
    }
    for (int q = 0; q < 6; ++q) {
        for (int off = 32; off > 0; off >>= 1) a[q] += __shfl_down(a[q], off, 64);
        if (lane == 0) si[q][wv] = a[q];
    }
    __syncthreads();
    if (t < 6) {
        unsigned long long v = 0ull;
        for (int w = 0; w < PT_THREADS / 64; ++w) v += si[t][w];
        unsigned long long *T = reinterpret_cast<unsigned long long *>(tot + p);
        // field order of DirTotals: n_axis[3], n_blind, n_unob, conc_fx
        if (v) atomicAdd(T + t, v);
    }
}

// hist[b] += sum over a range of blocks of hist_part[block][b]: blockIdx.y
// takes blocks y, y + HR_CHUNKS, ...; the sums are integers, so the atomic
// additions give the same histogram in any order.  hist starts at zero.
constexpr int HR_CHUNKS = 32;
__global__ void k_hist_reduce(const uint32_t *hist_part, int nblocks, uint32_t *hist) {
    const int bin = blockIdx.x * blockDim.x + threadIdx.x;
    if (bin >= HIST_BINS) return;
    uint32_t acc = 0;
    for (int b = blockIdx.y; b < nblocks; b += HR_CHUNKS) acc += hist_part[(int64_t)b * HIST_BINS + bin];
    if (acc) atomicAdd(&hist[bin], acc);
}

// Reach, fixture faces, classes and the histogram of reachable-direction
// codes.  Samples of several jobs (parts) may share a launch; each block
// keeps LDS counters for the job of its first sample and sends samples of
// any other job straight to that job's global counters.
struct SetupJob {
    const PartMeta *meta;
    const float4 *tris;
    const int32_t *leaf_pos;
    int64_t sample_base;
    int64_t n;
    double tool;
};

struct SetupArgs {
    const SetupJob *jobs;   // device table, or null: job0 only
    int32_t n_jobs;
    SetupJob job0;
    int64_t n_total;
    const float *point;
    const int32_t *tri;
    const uint32_t *axes_bits;
    uint8_t *cls_out;                  // [n_total] or null
    unsigned long long *class_count;   // [n_jobs][4]
    uint32_t *code_hist;               // [n_jobs][64]
    uint32_t *err;
};

__device__ inline int setup_job_of(const SetupArgs &a, int64_t i) {
    if (!a.jobs) return 0;
    int lo = 0, hi = a.n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.jobs[mid].sample_base <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void k_setups(SetupArgs a) {
    __shared__ uint32_t hc[64];
    __shared__ unsigned long long cc[4];
    if (threadIdx.x < 64) hc[threadIdx.x] = 0;
    if (threadIdx.x < 4) cc[threadIdx.x] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x;
    const int jb = setup_job_of(a, i0 < a.n_total ? i0 : a.n_total - 1);
    const int64_t i = i0 + threadIdx.x;
    if (i < a.n_total) {
        const int jj = setup_job_of(a, i);
        const SetupJob J = a.jobs ? a.jobs[jj] : a.job0;
        const PartMeta &P = *J.meta;
        const int32_t f = a.tri[i];
        int32_t p = -1;
        if (f >= 0 && f < P.n_tris) p = J.leaf_pos[P.tri_start + f];
        if (p < 0) {
            // the null samples of a part without nonzero-area faces are no
            // error here (the build has reported the part); others are
            if (!(f == -1 && P.n_valid == 0)) atomicOr(a.err, ERR_BAD_SAMPLE_TRI);
            if (a.cls_out) a.cls_out[i] = HRA_CLASS_INACCESSIBLE;
        } else {
            double lo[3], hi[3];
            for (int c = 0; c < 3; ++c) {
                lo[c] = P.bbox[c];
                hi[c] = P.bbox[3 + c];
            }
            const double tol = 1e-6 * P.diag;
            const float4 v[3] = {J.tris[3 * (int64_t)p], J.tris[3 * (int64_t)p + 1], J.tris[3 * (int64_t)p + 2]};
            bool fixture = false;
            for (int c = 0; c < 3 && !fixture; ++c) {
                for (int side = 0; side < 2 && !fixture; ++side) {
                    const double lim = side ? hi[c] : lo[c];
                    bool all = true;
                    for (int k = 0; k < 3; ++k) {
                        const double x = c == 0 ? v[k].x : (c == 1 ? v[k].y : v[k].z);
                        all = all && fabs(x - lim) <= tol;
                    }
                    fixture = all;
                }
            }
            const double px = a.point[3 * i], py = a.point[3 * i + 1], pz = a.point[3 * i + 2];
            const double travel[6] = {hi[0] - px, px - lo[0], hi[1] - py, py - lo[1], hi[2] - pz, pz - lo[2]};
            const uint32_t acc = a.axes_bits[i] & 63u;
            uint32_t code = 0;
            for (int k = 0; k < 6; ++k)
                if (((acc >> k) & 1u) && travel[k] <= J.tool) code |= 1u << k;
            uint8_t cl;
            if (fixture) cl = HRA_CLASS_FIXTURE;
            else if (code) cl = HRA_CLASS_VIABLE;
            else if (acc) cl = HRA_CLASS_OVER;
            else cl = HRA_CLASS_INACCESSIBLE;
            if (a.cls_out) a.cls_out[i] = cl;
            if (jj == jb) {
                atomicAdd(&cc[cl], 1ull);
                if (cl == HRA_CLASS_VIABLE) atomicAdd(&hc[code], 1u);
            } else {
                atomicAdd(&a.class_count[4 * jj + cl], 1ull);
                if (cl == HRA_CLASS_VIABLE) atomicAdd(&a.code_hist[64 * jj + code], 1u);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 64 && hc[threadIdx.x]) atomicAdd(&a.code_hist[64 * jb + threadIdx.x], hc[threadIdx.x]);
    if (threadIdx.x < 4 && cc[threadIdx.x]) atomicAdd(&a.class_count[4 * jb + threadIdx.x], cc[threadIdx.x]);
}

__global__ void k_zero_u32(uint32_t *p, int n) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) p[k] = 0;
}

__global__ void k_zero_setups(unsigned long long *cc, uint32_t *hist, int n_jobs) {
    for (int k = threadIdx.x; k < 4 * n_jobs; k += blockDim.x) cc[k] = 0;
    for (int k = threadIdx.x; k < 64 * n_jobs; k += blockDim.x) hist[k] = 0;
}

// Exact minimum hitting set over the 63 nonempty direction subsets; ties go
// to the numerically smallest mask.
void solve_setups(const uint32_t *hist, int32_t *min_count, int32_t *min_mask, int32_t *g_count, int32_t *g_mask) {
    int best = -1, bestc = 7;
    bool any = false;
    for (int c = 1; c < 64; ++c) any = any || hist[c] > 0;
    if (!any) {
        *min_count = *min_mask = *g_count = *g_mask = 0;
        return;
    }
    for (int m = 1; m < 64; ++m) {
        bool ok = true;
        for (int c = 1; c < 64 && ok; ++c)
            if (hist[c] && !(c & m)) ok = false;
        if (!ok) continue;
        const int pc = __builtin_popcount(m);
        if (pc < bestc || (pc == bestc && m < best)) {
            bestc = pc;
            best = m;
        }
    }
    *min_count = bestc;
    *min_mask = best;
    // greedy set cover (the paper's strategy)
    std::vector<uint64_t> left(hist, hist + 64);
    int gm = 0, gc = 0;
    while (true) {
        uint64_t rem = 0;
        for (int c = 1; c < 64; ++c) rem += left[c];
        if (!rem) break;
        int bk = -1;
        uint64_t bg = 0;
        for (int k = 0; k < 6; ++k) {
            if (gm >> k & 1) continue;
            uint64_t g = 0;
            for (int c = 1; c < 64; ++c)
                if (c >> k & 1) g += left[c];
            if (g > bg) {
                bg = g;
                bk = k;
            }
        }
        if (bk < 0) break;
        gm |= 1 << bk;
        ++gc;
        for (int c = 1; c < 64; ++c)
            if (c >> bk & 1) left[c] = 0;
    }
    *g_count = gc;
    *g_mask = gm;
}

}  // namespace hra

using namespace hra;

// totals scratch of hra_dirstats: DirTotals, then conc64 [n], then counts [n]
extern "C" int64_t hra_dirstats_bytes(int64_t n) {
    const int64_t m = n > 0 ? n : 0;
    return (int64_t)sizeof(DirTotals) + 8 * m + 4 * m + 64;
}

namespace hra {

// Blocks of a k_dirstats launch over n samples: DS_WAVES samples per block at
// first, at most DS_BLOCKS_PER_CU blocks per compute unit (one wave of
// blocks), and at most max_blocks.
static int64_t dirstats_blocks(const hra_ctx *ctx, int64_t n, int64_t max_blocks) {
    int64_t blocks = (n + DS_WAVES - 1) / DS_WAVES;
    const int64_t cap = (int64_t)ctx->n_cu * DS_BLOCKS_PER_CU;
    if (blocks > cap) blocks = cap;
    if (blocks > max_blocks) blocks = max_blocks;
    return blocks < 1 ? 1 : blocks;
}

// Per device, once: the azimuth table uploaded to `az_table` there, and the
// array's address on that device.
static std::mutex az_mu;
static std::map<int, const float4 *> az_ptr;

hipError_t stats_setup(int device) {
    std::lock_guard<std::mutex> lk(az_mu);
    if (az_ptr.count(device)) return hipSuccess;
    const std::vector<float4> tab = make_az_table();
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(az_table), tab.data(), sizeof(float4) * tab.size());
    if (e != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(az_table));
    if (e != hipSuccess) return e;
    az_ptr[device] = (const float4 *)p;
    return hipSuccess;
}

static const float4 *az_table_ptr(int device) {
    std::lock_guard<std::mutex> lk(az_mu);
    auto it = az_ptr.find(device);
    return it == az_ptr.end() ? nullptr : it->second;
}

// hist: also form the direction histogram, from per-block slices in
// `slices` (HIST_BINS words per block; NULL: taken from the stream-ordered
// allocator for the launch and returned after it).
hipError_t launch_dirstats(hra_ctx *ctx, const float *normal, int64_t n, const float4 *table, int32_t N,
                           const uint32_t *bits, const hra_dirstats &out, double *c64, uint32_t *cnt, bool hist,
                           hipStream_t s, uint32_t *slices, int64_t max_blocks) {
    if (n <= 0) return hipSuccess;
    const float4 *az = az_table_ptr(ctx->device);
    if (hist && !az) return hipErrorNotInitialized;
    const int64_t blocks = dirstats_blocks(ctx, n, max_blocks);
    uint32_t *part = slices;
    hipError_t e = hipSuccess;
    if (hist && !slices) {
        e = hipMallocAsync((void **)&part, sizeof(uint32_t) * HIST_BINS * (size_t)blocks, s);
        if (e != hipSuccess) return e;
    }
    k_dirstats<<<(unsigned)blocks, 64 * DS_WAVES, 0, s>>>(normal, n, table, N, (N + 31) / 32, bits, out, c64, cnt,
                                                         hist ? part : nullptr, az);
    if (hist) {
        k_zero_u32<<<HIST_BINS / 256, 256, 0, s>>>(out.hist, HIST_BINS);
        k_hist_reduce<<<dim3(HIST_BINS / 256, HR_CHUNKS), 256, 0, s>>>(part, (int)blocks, out.hist);
        if (!slices) hipFreeAsync(part, s);
    }
    return hipGetLastError();
}

static_assert(sizeof(DirTotals) % sizeof(uint32_t) == 0, "totals are cleared as 32-bit words");

// Zeroes n_parts totals, then adds each part's range (base NULL: one part,
// [0, n_one)).  Kernels only, so the call can be captured in a graph.
static hipError_t part_totals(const int8_t *axis, const uint32_t *cnt, const double *c64, const int64_t *d_base,
                              const int64_t *d_count, int64_t n_one, int n_parts, DirTotals *tot, hipStream_t s) {
    const int words = (int)(sizeof(DirTotals) / sizeof(uint32_t)) * n_parts;
    k_zero_u32<<<(words + 255) / 256, 256, 0, s>>>(reinterpret_cast<uint32_t *>(tot), words);
    if (d_base || n_one > 0) k_part_totals<<<dim3(PT_CHUNKS, n_parts), PT_THREADS, 0, s>>>(axis, cnt, c64, d_base,
                                                                                         d_count, n_one, tot);
    return hipGetLastError();
}

hipError_t launch_part_totals(const int8_t *axis, const uint32_t *cnt, const double *c64, const int64_t *d_base,
                              const int64_t *d_count, int n_parts, DirTotals *tot, hipStream_t s) {
    return part_totals(axis, cnt, c64, d_base, d_count, 0, n_parts, tot, s);
}

void classify_totals(const DirTotals &t, int64_t n, int32_t n_dirs, const hra_thresholds *th, hra_class_report *out) {
    const hra_thresholds def = {0.60, 0.45, 0.40};
    const hra_thresholds &T = th ? *th : def;
    const int64_t inc = n - (int64_t)t.n_blind;
    out->n_samples = n;
    out->n_blind = (int64_t)t.n_blind;
    out->n_unobstructed = t.n_unob;
    out->access = n ? (double)t.n_unob / ((double)n * (double)n_dirs) : 0.0;
    for (int k = 0; k < 3; ++k) out->share[k] = inc ? (double)t.n_axis[k] / (double)inc : 0.0;
    out->mean_conc = inc ? std::ldexp((double)t.conc_fx, -32) / (double)inc : 0.0;
    const double smax = fmax(out->share[0], fmax(out->share[1], out->share[2]));
    int tr = 0;
    if (out->access < T.min_access) tr |= 1;
    if (smax < T.min_share) tr |= 2;
    if (out->mean_conc > T.max_conc) tr |= 4;
    out->tripped = tr;
    out->multi_axis = tr ? 1 : 0;
    out->near_tie = (fabs(out->access - T.min_access) <= 1e-9 || fabs(smax - T.min_share) <= 1e-9 ||
                     fabs(out->mean_conc - T.max_conc) <= 1e-9)
                        ? 1
                        : 0;
}

hipError_t launch_setups(const SetupJob *d_jobs, int n_jobs, const SetupJob &job0, int64_t n_total, const float *point,
                         const int32_t *tri, const uint32_t *axes_bits, uint8_t *cls_out, unsigned long long *cc,
                         uint32_t *hist, uint32_t *err, hipStream_t s) {
    k_zero_setups<<<1, 256, 0, s>>>(cc, hist, n_jobs);
    if (n_total > 0) {
        SetupArgs a;
        a.jobs = d_jobs;
        a.n_jobs = n_jobs;
        a.job0 = job0;
        a.n_total = n_total;
        a.point = point;
        a.tri = tri;
        a.axes_bits = axes_bits;
        a.cls_out = cls_out;
        a.class_count = cc;
        a.code_hist = hist;
        a.err = err;
        k_setups<<<blocks_for(n_total, 256), 256, 0, s>>>(a);
    }
    return hipGetLastError();
}

SetupJob make_setup_job(const hra_bvh *bvh, int32_t part, int64_t sample_base, int64_t n, double tool) {
    SetupJob J;
    J.meta = bvh->parts + part;
    J.tris = bvh->tris;
    J.leaf_pos = bvh->leaf_pos;
    J.sample_base = sample_base;
    J.n = n;
    J.tool = tool;
    return J;
}

}  // namespace hra

namespace hra {
// thin wrappers for the batch orchestrator (batch.hip)
size_t dir_totals_size() { return sizeof(DirTotals); }
size_t setup_job_size() { return sizeof(SetupJob); }
void fill_setup_job(void *dst, const hra_bvh *bvh, int32_t part, int64_t sample_base, int64_t n, double tool) {
    *(SetupJob *)dst = make_setup_job(bvh, part, sample_base, n, tool);
}
hipError_t launch_part_totals_raw(const int8_t *axis, const uint32_t *cnt, const double *c64, const int64_t *d_base,
                                  const int64_t *d_count, int n_parts, void *tot, hipStream_t s) {
    return launch_part_totals(axis, cnt, c64, d_base, d_count, n_parts, (DirTotals *)tot, s);
}
hipError_t launch_setups_raw(const void *d_jobs, int n_jobs, int64_t n_total, const float *point, const int32_t *tri,
                             const uint32_t *axes_bits, unsigned long long *cc, uint32_t *hist, uint32_t *err,
                             hipStream_t s) {
    SetupJob j0;
    std::memset(&j0, 0, sizeof(j0));
    return launch_setups((const SetupJob *)d_jobs, n_jobs, j0, n_total, point, tri, axes_bits, nullptr, cc, hist, err, s);
}
void classify_from_device_totals(const void *host_totals, int64_t n, int32_t n_dirs, const hra_thresholds *th,
                                 hra_class_report *out) {
    classify_totals(*(const DirTotals *)host_totals, n, n_dirs, th, out);
}
}  // namespace hra

extern "C" int32_t hra_debug_azimuth_table(float *out, int32_t capacity) {
    const std::vector<float4> tab = hra::make_az_table();
    const int32_t nf = (int32_t)(4 * tab.size());
    if (out && capacity >= nf) std::memcpy(out, tab.data(), sizeof(float) * nf);
    return nf;
}

extern "C" hra_status hra_dominant_axes(hra_ctx *ctx, const hra_samples *samples, hra_dirs dirs, const uint32_t *d_bits,
                                        const hra_dirstats *out, void *stream) {
    if (!ctx || !samples || !out) return HRA_ERR_INVALID_ARG;
    if (!out->hist || !out->totals) return ctx->fail(HRA_ERR_INVALID_ARG, "histogram and totals must be non-null");
    if (samples->n > 0 && (!d_bits || !out->mean || !out->absmean || !out->axis || !out->conc || !samples->normal))
        return ctx->fail(HRA_ERR_INVALID_ARG, "all hra_dirstats arrays must be non-null");
    if (dirs.kind != HRA_DIRS_HEMI_FIBONACCI)
        return ctx->fail(HRA_ERR_INVALID_ARG, "directional statistics need the hemisphere set");
    const float4 *table = nullptr;
    hra_status st = dir_table(ctx, dirs, &table);
    if (st != HRA_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    HRA_HIP(hipSetDevice(ctx->device));
    const int64_t n = samples->n;
    DirTotals *tot = (DirTotals *)out->totals;
    double *c64 = (double *)((char *)out->totals + sizeof(DirTotals));
    uint32_t *cnt = (uint32_t *)(c64 + (n > 0 ? n : 0));
    if (n == 0) {
        // no samples: an empty histogram and zero totals (fill kernels, so
        // the call can be captured in a graph)
        k_zero_u32<<<HIST_BINS / 256, 256, 0, s>>>(out->hist, HIST_BINS);
        HRA_HIP(part_totals(nullptr, nullptr, nullptr, nullptr, nullptr, 0, 1, tot, s));
        return HRA_OK;
    }
    HRA_HIP(launch_dirstats(ctx, samples->normal, n, table, dirs.n, d_bits, *out, c64, cnt, true, s, nullptr,
                            INT64_MAX));
    HRA_HIP(part_totals(out->axis, cnt, c64, nullptr, nullptr, n, 1, tot, s));
    return HRA_OK;
}

// ------------------------------------------------------ allocation-free form
namespace hra {
// hra_dominant_axes_noalloc keeps what hra_dominant_axes allocates (the
// canonical direction table, cached per context, and the per-block
// histogram slices, taken from the stream-ordered allocator) in this array
// instead: NA_MAX_DIRS float4 table entries (and DIR_TABLE_PAD more that
// k_dirstats may read), then NA_SLICES slices of
// HIST_BINS words (NA_SLICES is at least DS_BLOCKS_PER_CU blocks on each of
// MI355X's 256 compute units, the cap of the allocating launch, so both
// launch the same grid there).  The module holds one copy per device until the process ends.
// Host code never names the array: it uses the address that
// hipGetSymbolAddress returned for the current device (noalloc_setup).
constexpr int32_t NA_MAX_DIRS = 8192;
constexpr int64_t NA_SLICES = 1024;
static_assert(NA_SLICES >= 256 * DS_BLOCKS_PER_CU, "slices for one block wave on 256 compute units");
constexpr size_t NA_TABLE_BYTES = sizeof(float4) * (NA_MAX_DIRS + DIR_TABLE_PAD);
constexpr size_t NA_SCRATCH_BYTES = NA_TABLE_BYTES + sizeof(uint32_t) * HIST_BINS * NA_SLICES;
static __device__ __align__(256) unsigned char scratch[NA_SCRATCH_BYTES];

static std::mutex na_mu;
static std::map<int, unsigned char *> na_ptr;   // device -> address of `scratch` there

// Called by hra_ctx_create with `device` current: look up the array's
// address on this device once.
hipError_t noalloc_setup(int device) {
    std::lock_guard<std::mutex> lk(na_mu);
    if (na_ptr.count(device)) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    na_ptr[device] = (unsigned char *)p;
    return hipSuccess;
}

static unsigned char *noalloc_ptr(int device) {
    std::lock_guard<std::mutex> lk(na_mu);
    auto it = na_ptr.find(device);
    return it == na_ptr.end() ? nullptr : it->second;
}

}  // namespace hra

extern "C" hra_status hra_dominant_axes_noalloc(hra_ctx *ctx, const hra_samples *samples, hra_dirs dirs,
                                                const uint32_t *d_bits, const hra_dirstats *out, void *stream) {
    using namespace hra;
    if (!ctx || !samples || !out) return HRA_ERR_INVALID_ARG;
    if (!out->hist || !out->totals) return ctx->fail(HRA_ERR_INVALID_ARG, "histogram and totals must be non-null");
    if (samples->n < 0) return ctx->fail(HRA_ERR_INVALID_ARG, "negative sample count");
    if (samples->n > 0 && (!d_bits || !out->mean || !out->absmean || !out->axis || !out->conc || !samples->normal))
        return ctx->fail(HRA_ERR_INVALID_ARG, "all hra_dirstats arrays must be non-null");
    if (dirs.kind != HRA_DIRS_HEMI_FIBONACCI)
        return ctx->fail(HRA_ERR_INVALID_ARG, "directional statistics need the hemisphere set");
    if (dirs.n < 1 || dirs.n > NA_MAX_DIRS)
        return ctx->fail(HRA_ERR_INVALID_ARG, "hra_dominant_axes_noalloc takes 1 to 8192 directions");
    unsigned char *base = noalloc_ptr(ctx->device);
    if (!base) return ctx->fail(HRA_ERR_DEVICE, "scratch address not set up for this device");
    hipStream_t s = (hipStream_t)stream;
    HRA_HIP(hipSetDevice(ctx->device));
    float4 *table = (float4 *)base;
    uint32_t *slices = (uint32_t *)(base + NA_TABLE_BYTES);
    const int64_t n = samples->n;
    DirTotals *tot = (DirTotals *)out->totals;
    double *c64 = (double *)((char *)out->totals + sizeof(DirTotals));
    uint32_t *cnt = (uint32_t *)(c64 + (n > 0 ? n : 0));
    if (n == 0) {
        k_zero_u32<<<HIST_BINS / 256, 256, 0, s>>>(out->hist, HIST_BINS);
        HRA_HIP(part_totals(nullptr, nullptr, nullptr, nullptr, nullptr, 0, 1, tot, s));
        return HRA_OK;
    }
    // the table the cached one holds (same kernel), written on this stream
    // ahead of its readers
    HRA_HIP(launch_fibonacci(dirs.n, table, s));
    HRA_HIP(launch_dirstats(ctx, samples->normal, n, table, dirs.n, d_bits, *out, c64, cnt, true, s, slices,
                            NA_SLICES));
    HRA_HIP(part_totals(out->axis, cnt, c64, nullptr, nullptr, n, 1, tot, s));
    return HRA_OK;
}

extern "C" hra_status hra_classify(hra_ctx *ctx, const hra_dirstats *stats, int64_t n, int32_t n_dirs,
                                   const hra_thresholds *th, hra_class_report *out, void *stream) {
    if (!ctx || !stats || !stats->totals || !out || n < 0 || n_dirs < 1) return HRA_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    HRA_HIP(hipSetDevice(ctx->device));
    static_assert(sizeof(DirTotals) <= STAGE_BYTES - STAGE_USER, "totals fit the staging buffer");
    HRA_HIP(hipMemcpyAsync(stage_user(ctx), stats->totals, sizeof(DirTotals), hipMemcpyDeviceToHost, s));
    hra_status st = check_error_word(ctx, s);   // synchronises s
    if (st != HRA_OK) return st;
    DirTotals t;
    std::memcpy(&t, stage_user(ctx), sizeof(t));
    classify_totals(t, n, n_dirs, th, out);
    return HRA_OK;
}

extern "C" hra_status hra_min_setups_part(hra_ctx *ctx, const hra_bvh *bvh, int32_t part, const hra_samples *samples,
                                          const uint32_t *d_axes_bits, double tool_length, uint8_t *d_class,
                                          hra_setup_report *out, void *stream) {
    if (!ctx || !bvh || !samples || !out) return HRA_ERR_INVALID_ARG;
    if (part < 0 || part >= bvh->n_parts) return ctx->fail(HRA_ERR_INVALID_ARG, "part index out of range");
    if (samples->n < 0) return ctx->fail(HRA_ERR_INVALID_ARG, "negative sample count");
    if (samples->n > 0 && (!samples->point || !samples->tri || !d_axes_bits))
        return ctx->fail(HRA_ERR_INVALID_ARG, "sample points, faces and axis bits must be non-null");
    if (!(tool_length >= 0.0)) return ctx->fail(HRA_ERR_INVALID_ARG, "tool length must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    HRA_HIP(hipSetDevice(ctx->device));
    unsigned long long *cc = nullptr;
    HRA_HIP(hipMallocAsync((void **)&cc, 4 * sizeof(unsigned long long) + 64 * sizeof(uint32_t), s));
    uint32_t *hist = (uint32_t *)(cc + 4);
    const SetupJob J = make_setup_job(bvh, part, 0, samples->n, tool_length);
    // counters and code histogram are adjacent on the device: one copy
    unsigned long long *hcc = (unsigned long long *)stage_user(ctx);
    const uint32_t *hh = (const uint32_t *)(hcc + 4);
    hipError_t e = launch_setups(nullptr, 1, J, samples->n, samples->point, samples->tri, d_axes_bits, d_class, cc, hist,
                                 ctx->d_err, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hcc, cc, 4 * sizeof(unsigned long long) + 64 * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    const hipError_t ef = hipFreeAsync(cc, s);
    if (e == hipSuccess) e = ef;
    if (e != hipSuccess) return ctx->fail(HRA_ERR_DEVICE, "min_setups launch failed", hipGetErrorString(e));
    hra_status st = check_error_word(ctx, s);
    if (st != HRA_OK) return st;
    for (int k = 0; k < 4; ++k) out->n_class[k] = (int64_t)hcc[k];
    for (int c = 0; c < 64; ++c) out->code_hist[c] = hh[c];
    solve_setups(hh, &out->min_count, &out->min_mask, &out->greedy_count, &out->greedy_mask);
    return HRA_OK;
}

extern "C" hra_status hra_min_setups(hra_ctx *ctx, const hra_bvh *bvh, const hra_samples *samples,
                                     const uint32_t *d_axes_bits, double tool_length, uint8_t *d_class,
                                     hra_setup_report *out, void *stream) {
    return hra_min_setups_part(ctx, bvh, 0, samples, d_axes_bits, tool_length, d_class, out, stream);
}

// Bin centre of histogram bin b: z band zb = b / 128 covers z in
// [zb/32 - 1, (zb+1)/32 - 1), azimuth sector az = b % 128 covers
// [az 2pi/128 - pi, (az+1) 2pi/128 - pi).
static void bin_centre(int b, double *d) {
    const double pi = 3.14159265358979323846264338327950288;
    const int zb = b / 128, az = b % 128;
    const double z = (zb + 0.5) / 32.0 - 1.0;
    const double phi = (az + 0.5) * (2.0 * pi / 128.0) - pi;
    const double r = std::sqrt(std::fmax(0.0, 1.0 - z * z));
    d[0] = r * std::cos(phi);
    d[1] = r * std::sin(phi);
    d[2] = z;
}

extern "C" hra_status hra_histogram_peaks(const uint32_t *h, int32_t k, hra_hist_peaks *out) {
    if (!h || !out || k < 0 || k > 16) return HRA_ERR_INVALID_ARG;
    std::vector<std::pair<uint32_t, int>> peaks;
    for (int b = 0; b < HIST_BINS; ++b) {
        const uint32_t v = h[b];
        if (!v) continue;
        const int zb = b / 128, az = b % 128;
        bool is_max = true;
        for (int dz = -1; dz <= 1 && is_max; ++dz) {
            const int z2 = zb + dz;
            if (z2 < 0 || z2 > 63) continue;
            for (int da = -1; da <= 1; ++da) {
                if (!dz && !da) continue;
                const int b2 = z2 * 128 + ((az + da + 128) % 128);
                if (h[b2] > v || (h[b2] == v && b2 < b)) {
                    is_max = false;
                    break;
                }
            }
        }
        if (is_max) peaks.push_back({v, b});
    }
    std::sort(peaks.begin(), peaks.end(), [](const std::pair<uint32_t, int> &x, const std::pair<uint32_t, int> &y) {
        return x.first != y.first ? x.first > y.first : x.second < y.second;
    });
    out->n_peaks = (int32_t)std::min<size_t>(peaks.size(), (size_t)k);
    for (int i = 0; i < out->n_peaks; ++i) {
        out->bin[i] = peaks[i].second;
        out->mass[i] = peaks[i].first;
        double d[3];
        bin_centre(peaks[i].second, d);
        for (int c = 0; c < 3; ++c) out->dir[i][c] = (float)d[c];
    }
    const double c45 = std::sqrt(0.5);
    for (int a = 0; a < 6; ++a) out->axis_mass[a] = 0;
    for (int b = 0; b < HIST_BINS; ++b) {
        if (!h[b]) continue;
        double d[3];
        bin_centre(b, d);
        for (int a = 0; a < 6; ++a) {
            const double comp = (a & 1) ? -d[a >> 1] : d[a >> 1];
            if (comp > c45) out->axis_mass[a] += h[b];
        }
    }
    return HRA_OK;
}

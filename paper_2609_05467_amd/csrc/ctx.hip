// Context, error word, direction tables.
#include "common.hpp"
#include "stages.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace hra {

int blocks_for(int64_t n, int threads) {
    int64_t b = (n + threads - 1) / threads;
    return (int)(b < 1 ? 1 : b);
}

// Spherical Fibonacci points on the open upper hemisphere (a uniformly
// sampled hemisphere, Section 3.1 and Fig. 1):
//   z_j = 1 - (2j+1)/(2N), r_j = sqrt(1 - z_j^2), phi_j = 2 pi frac(j g),
//   g = (3 - sqrt 5)/2, evaluated in FP64 and rounded once to FP32.
__global__ void k_fibonacci(int32_t n, float4 *out) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double g = (3.0 - sqrt(5.0)) / 2.0;
    const double two_pi = 6.283185307179586476925286766559;
    const double z = 1.0 - (2.0 * (double)j + 1.0) / (2.0 * (double)n);
    const double zz = z * z;
    const double r = sqrt(1.0 - zz);
    const double jg = (double)j * g;
    const double f = jg - floor(jg);
    const double phi = two_pi * f;
    const double c = cos(phi), s = sin(phi);
    out[j] = make_float4((float)(r * c), (float)(r * s), (float)z, 0.0f);
}

// Section 3.2: the six principal directions of the machining frame.
__global__ void k_axes6(float4 *out) {
    const int j = threadIdx.x;
    if (j >= 6) return;
    const float s = (j & 1) ? -1.0f : 1.0f;
    const int ax = j >> 1;
    out[j] = make_float4(ax == 0 ? s : 0.0f, ax == 1 ? s : 0.0f, ax == 2 ? s : 0.0f, 0.0f);
}

// Index of cell (x, y) along the Hilbert curve over a 2^16 x 2^16 grid
// (the usual quadrant-rotation construction).
static uint64_t hilbert_index(uint32_t x, uint32_t y) {
    uint64_t d = 0;
    for (uint32_t half = 1u << 15; half > 0; half >>= 1) {
        const uint32_t rx = (x & half) ? 1u : 0u, ry = (y & half) ? 1u : 0u;
        d += (uint64_t)half * half * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = (half - 1) - (x & (half - 1));
                y = (half - 1) - (y & (half - 1));
            }
            const uint32_t tmp = x;
            x = y;
            y = tmp;
        }
        x &= half - 1;
        y &= half - 1;
    }
    return d;
}

// Traversal order of a hemisphere table: directions sorted along a Hilbert
// curve over their equal-area (Lambert azimuthal) projection, so runs of 64
// consecutive entries are compact patches of the hemisphere.  w holds the
// canonical index.  Only the order of work depends on it, never a result.
static std::vector<float4> traversal_order(const std::vector<float4> &dirs) {
    const size_t n = dirs.size();
    std::vector<std::pair<uint64_t, int32_t>> key(n);
    for (size_t j = 0; j < n; ++j) {
        const double x = dirs[j].x, y = dirs[j].y, z = dirs[j].z;
        const double k = std::sqrt(2.0 / (1.0 + (z > 0.0 ? z : 0.0)));
        const double u = (k * x / std::sqrt(2.0) + 1.0) * 0.5, v = (k * y / std::sqrt(2.0) + 1.0) * 0.5;
        auto q = [](double t) {
            const double c = std::floor(t * 65535.0 + 0.5);
            return (uint32_t)(c < 0.0 ? 0.0 : (c > 65535.0 ? 65535.0 : c));
        };
        key[j] = {hilbert_index(q(u), q(v)), (int32_t)j};
    }
    std::sort(key.begin(), key.end());
    std::vector<float4> out(n);
    for (size_t i = 0; i < n; ++i) {
        float4 d = dirs[key[i].second];
        int32_t j = key[i].second;
        std::memcpy(&d.w, &j, sizeof(j));
        out[i] = d;
    }
    return out;
}

hra_status dir_table(hra_ctx *ctx, hra_dirs dirs, const float4 **out) {
    if (dirs.kind == HRA_DIRS_AXES6) {
        if (dirs.n != 6) return ctx->fail(HRA_ERR_INVALID_ARG, "AXES6 needs n = 6");
    } else if (dirs.kind == HRA_DIRS_HEMI_FIBONACCI) {
        if (dirs.n < 1 || dirs.n > 65536) return ctx->fail(HRA_ERR_INVALID_ARG, "direction count must be in [1, 65536]");
    } else {
        return ctx->fail(HRA_ERR_INVALID_ARG, "unknown direction kind");
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto key = std::make_pair((int)dirs.kind, (int)dirs.n);
    auto it = ctx->dir_tables.find(key);
    if (it != ctx->dir_tables.end()) {
        *out = it->second;
        return HRA_OK;
    }
    // hemisphere tables hold the canonical order in [0, n) and the traversal
    // order in [n, 2n), then DIR_TABLE_PAD entries that may be read, never used
    float4 *p = nullptr;
    const bool hemi = dirs.kind == HRA_DIRS_HEMI_FIBONACCI;
    const size_t entries = hemi ? 2 * (size_t)dirs.n + DIR_TABLE_PAD : (size_t)dirs.n;
    HRA_HIP(hipMalloc(&p, sizeof(float4) * entries));
    if (!hemi)
        k_axes6<<<1, 64, 0, ctx->own>>>(p);
    else
        k_fibonacci<<<blocks_for(dirs.n, 256), 256, 0, ctx->own>>>(dirs.n, p);
    HRA_HIP(hipGetLastError());
    // tables are built once per context on its own stream; later work on any
    // stream may read them, so wait here
    HRA_HIP(hipStreamSynchronize(ctx->own));
    if (hemi) {
        std::vector<float4> h(dirs.n);
        HRA_HIP(hipMemcpyAsync(h.data(), p, sizeof(float4) * dirs.n, hipMemcpyDeviceToHost, ctx->own));
        HRA_HIP(hipStreamSynchronize(ctx->own));
        const std::vector<float4> o = traversal_order(h);
        HRA_HIP(hipMemcpyAsync(p + dirs.n, o.data(), sizeof(float4) * dirs.n, hipMemcpyHostToDevice, ctx->own));
        HRA_HIP(hipStreamSynchronize(ctx->own));
    }
    ctx->dir_tables[key] = p;
    *out = p;
    return HRA_OK;
}

hipError_t launch_fibonacci(int32_t n, float4 *out, hipStream_t s) {
    k_fibonacci<<<blocks_for(n, 256), 256, 0, s>>>(n, out);
    return hipGetLastError();
}

hra_status check_error_word(hra_ctx *ctx, hipStream_t s) {
    // the word comes through pinned memory on s itself, so the call waits
    // for s alone, not for work on other streams
    uint32_t *hw = (uint32_t *)ctx->h_stage;
    HRA_HIP(hipMemcpyAsync(hw, ctx->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HRA_HIP(hipStreamSynchronize(s));
    const uint32_t w = *hw;
    if (w == 0) return HRA_OK;
    HRA_HIP(hipMemsetAsync(ctx->d_err, 0, sizeof(uint32_t), s));
    HRA_HIP(hipStreamSynchronize(s));
    if (w & ERR_BAD_INDEX) return ctx->fail(HRA_ERR_BAD_MESH, "triangle index out of range");
    if (w & ERR_EMPTY_MESH) return ctx->fail(HRA_ERR_BAD_MESH, "mesh has no triangle with nonzero area");
    if (w & ERR_BAD_SAMPLE_TRI) return ctx->fail(HRA_ERR_INVALID_ARG, "a sample names a face outside the mesh");
    if (w & ERR_TOOL_RADIUS)
        return ctx->fail(HRA_ERR_INVALID_ARG, "tool radius below 2e-4 x the part's bounding-box diagonal");
    if (w & ERR_STACK) return ctx->fail(HRA_ERR_DEVICE, "traversal stack exhausted");
    if (w & ERR_BAD_ORDER) return ctx->fail(HRA_ERR_INVALID_ARG, "a sample order names an index outside [0, n)");
    return ctx->fail(HRA_ERR_DEVICE, "device error word set");
}

}  // namespace hra

using namespace hra;

extern "C" {

const char *hra_version(void) { return "hra 0.1 (gfx950)"; }

hra_status hra_ctx_create(int32_t device, hra_ctx **out) {
    if (!out) return HRA_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HRA_ERR_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return HRA_ERR_DEVICE;
    hra_ctx *ctx = new hra_ctx();
    ctx->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete ctx;
        return HRA_ERR_DEVICE;
    }
    ctx->n_cu = prop.multiProcessorCount;
    // stream-ordered allocations (workspaces, hierarchies) keep their memory
    // in the device's pool between calls instead of returning it to the
    // driver at each synchronisation, where the next call would map it again
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess && pool) {
        uint64_t keep = UINT64_MAX;
        if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) {
            delete ctx;
            return HRA_ERR_DEVICE;
        }
    }
    if (noalloc_setup(device) != hipSuccess || stats_setup(device) != hipSuccess) {
        delete ctx;
        return HRA_ERR_DEVICE;
    }
    if (hipMalloc(&ctx->d_err, sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&ctx->d_counter, 64 * sizeof(uint32_t)) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->own, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc(&ctx->h_stage, STAGE_BYTES, hipHostMallocDefault) != hipSuccess) {
        hra_ctx_destroy(ctx);
        return HRA_ERR_OUT_OF_MEMORY;
    }
    if (hipMemset(ctx->d_err, 0, sizeof(uint32_t)) != hipSuccess ||
        hipMemset(ctx->d_counter, 0, 64 * sizeof(uint32_t)) != hipSuccess) {
        hra_ctx_destroy(ctx);
        return HRA_ERR_DEVICE;
    }
    *out = ctx;
    return HRA_OK;
}

void hra_ctx_destroy(hra_ctx *ctx) {
    if (!ctx) return;
    hipSetDevice(ctx->device);
    if (ctx->own) hipStreamSynchronize(ctx->own);
    for (auto &kv : ctx->dir_tables) hipFree(kv.second);
    if (ctx->d_err) hipFree(ctx->d_err);
    if (ctx->d_counter) hipFree(ctx->d_counter);
    if (ctx->h_stage) hipHostFree(ctx->h_stage);
    if (ctx->own) hipStreamDestroy(ctx->own);
    delete ctx;
}

const char *hra_last_error(const hra_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

hra_status hra_dirs_table(hra_ctx *ctx, hra_dirs dirs, float *host_out) {
    if (!ctx || !host_out) return HRA_ERR_INVALID_ARG;
    const float4 *d = nullptr;
    hra_status st = dir_table(ctx, dirs, &d);
    if (st != HRA_OK) return st;
    std::vector<float4> h(dirs.n);
    HRA_HIP(hipMemcpyAsync(h.data(), d, sizeof(float4) * dirs.n, hipMemcpyDeviceToHost, ctx->own));
    HRA_HIP(hipStreamSynchronize(ctx->own));
    for (int32_t j = 0; j < dirs.n; ++j) {
        host_out[3 * j + 0] = h[j].x;
        host_out[3 * j + 1] = h[j].y;
        host_out[3 * j + 2] = h[j].z;
    }
    return HRA_OK;
}

}  // extern "C"

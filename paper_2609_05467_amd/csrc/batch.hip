// Many parts through the whole path at once: one hierarchy, then one launch
// per stage for every part together (sampling, hemisphere cast, statistics,
// part totals, six-axis cast, setups).  Work items of all parts share each
// launch, so small and large parts load the GPU together.
#include "common.hpp"

#include <vector>

namespace hra {
struct DirTotals;
struct SetupJob;
hipError_t launch_dirstats(hra_ctx *ctx, const float *normal, int64_t n, const float4 *table, int32_t N,
                           const uint32_t *bits, const hra_dirstats &out, double *c64, uint32_t *cnt, bool hist,
                           hipStream_t s);
void classify_from_device_totals(const void *host_totals, int64_t n, int32_t n_dirs, const hra_thresholds *th,
                                 hra_class_report *out);
hipError_t launch_part_totals_raw(const int8_t *axis, const uint32_t *cnt, const double *c64, const int64_t *d_base,
                                  const int64_t *d_count, int n_parts, void *tot, hipStream_t s);
size_t dir_totals_size();
hipError_t launch_setups_raw(const void *d_jobs, int n_jobs, int64_t n_total, const float *point, const int32_t *tri,
                             const uint32_t *axes_bits, unsigned long long *cc, uint32_t *hist, uint32_t *err,
                             hipStream_t s);
size_t setup_job_size();
void fill_setup_job(void *dst, const hra_bvh *bvh, int32_t part, int64_t sample_base, int64_t n, double tool);
void solve_setups(const uint32_t *hist, int32_t *min_count, int32_t *min_mask, int32_t *g_count, int32_t *g_mask);
}  // namespace hra

using namespace hra;

extern "C" hra_status hra_batch_run(hra_ctx *ctx, const hra_part_request *parts, int32_t n_parts,
                                    const hra_batch_opts *opts, hra_part_result *results, uint32_t *d_bits_out,
                                    void *stream) {
    if (!ctx || !parts || !results || !opts) return HRA_ERR_INVALID_ARG;
    if (n_parts < 1 || n_parts > MAX_PARTS) return ctx->fail(HRA_ERR_INVALID_ARG, "1..255 parts per batch");
    const int32_t N = opts->n_dirs;
    hra_dirs hemi = {HRA_DIRS_HEMI_FIBONACCI, N}, ax6 = {HRA_DIRS_AXES6, 6};
    const float4 *t_hemi = nullptr, *t_ax = nullptr;
    hra_status st = dir_table(ctx, hemi, &t_hemi);
    if (st != HRA_OK) return st;
    st = dir_table(ctx, ax6, &t_ax);
    if (st != HRA_OK) return st;
    const float frac = opts->offset_frac > 0.0f ? opts->offset_frac : 1e-4f;
    if (!(frac <= 0.01f)) return ctx->fail(HRA_ERR_INVALID_ARG, "offset_frac must be in (0, 0.01]");
    std::vector<hra_mesh> meshes(n_parts);
    std::vector<int64_t> base(n_parts), count(n_parts);
    int64_t S = 0;
    for (int p = 0; p < n_parts; ++p) {
        if (parts[p].n_samples < 1) return ctx->fail(HRA_ERR_INVALID_ARG, "every part needs at least one sample");
        if (!(parts[p].tool_length >= 0.0)) return ctx->fail(HRA_ERR_INVALID_ARG, "tool length must be >= 0");
        meshes[p] = parts[p].mesh;
        base[p] = S;
        count[p] = parts[p].n_samples;
        S += parts[p].n_samples;
    }
    hipStream_t s = (hipStream_t)stream;
    HRA_HIP(hipSetDevice(ctx->device));
    hra_bvh_opts bo = {opts->leaf_size};
    hra_bvh *bvh = nullptr;
    st = hra_build_bvh_batch(ctx, meshes.data(), n_parts, &bo, stream, &bvh);
    if (st != HRA_OK) return st;

    const int32_t W = (N + 31) / 32;
    const int rpw = ctx->cast_rpw;
    const int32_t chunks = (N + rpw - 1) / rpw;
    // host job tables
    std::vector<SampleJob> sj(n_parts);
    std::vector<CastJob> cj(n_parts), aj(n_parts);
    std::vector<char> setj(setup_job_size() * n_parts);
    // device buffers (stream ordered)
    float *pt = nullptr, *nr = nullptr, *org = nullptr, *mean = nullptr, *absm = nullptr, *conc = nullptr;
    int32_t *tri = nullptr;
    uint32_t *bits = d_bits_out, *abits = nullptr, *cnt = nullptr, *hist = nullptr, *chist = nullptr;
    int8_t *axis = nullptr;
    double *c64 = nullptr;
    void *tot = nullptr;
    unsigned long long *cc = nullptr;
    int64_t *dbase = nullptr, *dcount = nullptr;
    SampleJob *dsj = nullptr;
    CastJob *dcj = nullptr, *daj = nullptr;
    void *dsetj = nullptr;
    uint32_t *own_bits = nullptr;
    hipError_t e = hipSuccess;
#define TMP(p, n)                                                   \
    if (e == hipSuccess) e = hipMallocAsync((void **)&(p), (n), s);
    TMP(pt, sizeof(float) * 3 * S);
    TMP(nr, sizeof(float) * 3 * S);
    TMP(org, sizeof(float) * 3 * S);
    TMP(tri, sizeof(int32_t) * S);
    if (!bits) {
        TMP(own_bits, sizeof(uint32_t) * W * (size_t)S);
        bits = own_bits;
    }
    TMP(abits, sizeof(uint32_t) * S);
    TMP(mean, sizeof(float) * 3 * S);
    TMP(absm, sizeof(float) * 3 * S);
    TMP(axis, sizeof(int8_t) * S);
    TMP(conc, sizeof(float) * S);
    TMP(c64, sizeof(double) * S);
    TMP(cnt, sizeof(uint32_t) * S);
    TMP(hist, sizeof(uint32_t) * 8192);
    TMP(tot, dir_totals_size() * n_parts);
    TMP(cc, sizeof(unsigned long long) * 4 * n_parts);
    TMP(chist, sizeof(uint32_t) * 64 * n_parts);
    TMP(dbase, sizeof(int64_t) * n_parts);
    TMP(dcount, sizeof(int64_t) * n_parts);
    TMP(dsj, sizeof(SampleJob) * n_parts);
    TMP(dcj, sizeof(CastJob) * n_parts);
    TMP(daj, sizeof(CastJob) * n_parts);
    TMP(dsetj, setup_job_size() * n_parts);
#undef TMP
    int64_t items = 0, aitems = 0;
    for (int p = 0; p < n_parts && e == hipSuccess; ++p) {
        sj[p] = make_sample_job(bvh, p, HRA_SAMPLE_AREA, parts[p].seed, frac, count[p], base[p], base[p]);
        cj[p] = make_cast_job(bvh, p, org + 3 * base[p], nr + 3 * base[p], bits + (size_t)W * base[p], count[p], items);
        aj[p] = make_cast_job(bvh, p, org + 3 * base[p], nr + 3 * base[p], abits + base[p], count[p], aitems);
        fill_setup_job(setj.data() + setup_job_size() * p, bvh, p, base[p], count[p], parts[p].tool_length);
        items += count[p] * chunks;
        aitems += count[p];
    }
    if (e == hipSuccess) e = hipMemcpyAsync(dbase, base.data(), sizeof(int64_t) * n_parts, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dcount, count.data(), sizeof(int64_t) * n_parts, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dsj, sj.data(), sizeof(SampleJob) * n_parts, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dcj, cj.data(), sizeof(CastJob) * n_parts, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(daj, aj.data(), sizeof(CastJob) * n_parts, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dsetj, setj.data(), setj.size(), hipMemcpyHostToDevice, s);
    // 1. samples of every part
    if (e == hipSuccess) e = launch_sample(dsj, n_parts, sj[0], S, pt, nr, org, tri, s);
    // 2. hemisphere cast of every part, one launch
    if (e == hipSuccess) {
        CastArgs a;
        a.jobs = dcj;
        a.n_jobs = n_parts;
        a.job0 = cj[0];
        a.dirs = t_hemi;
        a.n_dirs = N;
        a.kind = 0;
        a.W = W;
        a.chunks = chunks;
        a.n_items = items;
        a.err = ctx->d_err;
        a.work = nullptr;
        e = launch_cast_any(a, rpw, ctx->cast_stack, false, s);
    }
    // 3. statistics of every sample, then per-part totals in a fixed order
    hra_dirstats ds = {mean, absm, axis, conc, hist, nullptr};
    if (e == hipSuccess) e = launch_dirstats(ctx, nr, S, t_hemi, N, bits, ds, c64, cnt, false, s);
    if (e == hipSuccess) e = launch_part_totals_raw(axis, cnt, c64, dbase, dcount, n_parts, tot, s);
    // 4. six-axis cast of every part, one launch
    if (e == hipSuccess) {
        CastArgs a;
        a.jobs = daj;
        a.n_jobs = n_parts;
        a.job0 = aj[0];
        a.dirs = t_ax;
        a.n_dirs = 6;
        a.kind = 1;
        a.W = 1;
        a.chunks = 1;
        a.n_items = aitems;
        a.err = ctx->d_err;
        a.work = nullptr;
        e = launch_cast_any(a, 64, ctx->cast_stack, false, s);
    }
    // 5. reach, classes and code histograms of every part
    if (e == hipSuccess) e = launch_setups_raw(dsetj, n_parts, S, pt, tri, abits, cc, chist, ctx->d_err, s);
    std::vector<char> htot(dir_totals_size() * n_parts);
    std::vector<unsigned long long> hcc(4 * (size_t)n_parts);
    std::vector<uint32_t> hch(64 * (size_t)n_parts);
    if (e == hipSuccess) e = hipMemcpyAsync(htot.data(), tot, htot.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hcc.data(), cc, sizeof(unsigned long long) * hcc.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hch.data(), chist, sizeof(uint32_t) * hch.size(), hipMemcpyDeviceToHost, s);
    for (void *q : {(void *)pt, (void *)nr, (void *)org, (void *)tri, (void *)own_bits, (void *)abits, (void *)mean,
                    (void *)absm, (void *)axis, (void *)conc, (void *)c64, (void *)cnt, (void *)hist, tot, (void *)cc,
                    (void *)chist, (void *)dbase, (void *)dcount, (void *)dsj, (void *)dcj, (void *)daj, dsetj})
        if (q) hipFreeAsync(q, s);
    st = check_error_word(ctx, s);   // synchronises the stream
    hra_bvh_release(bvh);
    if (e != hipSuccess) return ctx->fail(HRA_ERR_DEVICE, "batch launch failed", hipGetErrorString(e));
    if (st != HRA_OK) return st;
    for (int p = 0; p < n_parts; ++p) {
        classify_from_device_totals(htot.data() + dir_totals_size() * p, count[p], N, opts->thresholds, &results[p].cls);
        hra_setup_report &R = results[p].setups;
        for (int k = 0; k < 4; ++k) R.n_class[k] = (int64_t)hcc[4 * p + k];
        for (int c = 0; c < 64; ++c) R.code_hist[c] = hch[64 * p + c];
        solve_setups(R.code_hist, &R.min_count, &R.min_mask, &R.greedy_count, &R.greedy_mask);
    }
    return HRA_OK;
}

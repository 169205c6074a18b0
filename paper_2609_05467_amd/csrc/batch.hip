// Many parts through the whole path at once.  One launch per stage covers
// the work items of every part (sampling, hemisphere cast, statistics, part
// totals, six-axis cast, setups), so small and large parts load the GPU
// together and the launch count does not grow with the number of parts.
//
// A plan holds every buffer of one batch (hierarchy, build scratch, stage
// buffers, job tables, pinned result slots), so running it allocates
// nothing and enqueues kernels plus three small copies into pinned memory.
// That sequence can be captured once in a HIP graph and replayed.
#include "stages.hpp"
#include "prims.hpp"

#include <cstring>
#include <vector>

namespace hra {

size_t carve_stage(char *base, int64_t S, int32_t W, int32_t n_jobs, StageBufs *out) {
    size_t off = 0;
    auto take = [&](void **p, size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        if (base) *p = base + off;
        off += bytes;
    };
    StageBufs b;
    take((void **)&b.pt, sizeof(float) * 3 * S);
    take((void **)&b.nr, sizeof(float) * 3 * S);
    take((void **)&b.org, sizeof(float) * 3 * S);
    take((void **)&b.tri, sizeof(int32_t) * S);
    take((void **)&b.bits, sizeof(uint32_t) * (size_t)W * S);
    take((void **)&b.abits, sizeof(uint32_t) * S);
    take((void **)&b.mean, sizeof(float) * 3 * S);
    take((void **)&b.absm, sizeof(float) * 3 * S);
    take((void **)&b.conc, sizeof(float) * S);
    take((void **)&b.axis, sizeof(int8_t) * S);
    take((void **)&b.c64, sizeof(double) * S);
    take((void **)&b.cnt, sizeof(uint32_t) * S);
    take((void **)&b.tot, dir_totals_size() * n_jobs);
    take((void **)&b.cc, sizeof(unsigned long long) * 4 * n_jobs);
    take((void **)&b.chist, sizeof(uint32_t) * 64 * n_jobs);
    take((void **)&b.dbase, sizeof(int64_t) * n_jobs);
    take((void **)&b.dcount, sizeof(int64_t) * n_jobs);
    take((void **)&b.dsj, sizeof(SampleJob) * n_jobs);
    take((void **)&b.dcj, sizeof(CastJob) * n_jobs);
    take((void **)&b.daj, sizeof(CastJob) * n_jobs);
    take((void **)&b.dsetj, setup_job_size() * n_jobs);
    take((void **)&b.okey0, sizeof(uint64_t) * S);
    take((void **)&b.okey1, sizeof(uint64_t) * S);
    take((void **)&b.oval0, sizeof(uint32_t) * S);
    take((void **)&b.oval1, sizeof(uint32_t) * S);
    take((void **)&b.osort, sizeof(uint32_t) * (size_t)sort_pairs_ws_elems(S));
    if (out) *out = b;
    return (off + 255) & ~(size_t)255;
}

void fill_jobs(const StageBufs &B, const std::vector<const hra_bvh *> &bvh, const std::vector<int32_t> &part,
                      const std::vector<int64_t> &count, const std::vector<uint64_t> &seed,
                      const std::vector<double> &tool, float frac, StageShape *sh, HostJobs *H) {
    const int n = (int)bvh.size();
    H->base.resize(n);
    H->count = count;
    H->sj.resize(n);
    H->cj.resize(n);
    H->aj.resize(n);
    H->setj.assign(setup_job_size() * n, 0);
    int64_t S = 0, items = 0, aitems = 0;
    for (int j = 0; j < n; ++j) {
        H->base[j] = S;
        H->sj[j] = make_sample_job(bvh[j], part[j], HRA_SAMPLE_AREA, seed[j], frac, count[j], S, S);
        H->cj[j] = make_cast_job(bvh[j], part[j], B.org + 3 * S, B.nr + 3 * S, B.bits + (size_t)sh->W * S, count[j],
                                 items);
        H->aj[j] = make_cast_job(bvh[j], part[j], B.org + 3 * S, B.nr + 3 * S, B.abits + S, count[j], aitems);
        fill_setup_job(H->setj.data() + setup_job_size() * j, bvh[j], part[j], S, count[j], tool[j]);
        S += count[j];
        items += cast_items(0, count[j], sh->group);
        aitems += cast_items(1, count[j], 1);
    }
    sh->n_jobs = n;
    sh->S = S;
    sh->items = items;
    sh->aitems = aitems;
    sh->sj0 = H->sj[0];
    sh->cj0 = H->cj[0];
    sh->aj0 = H->aj[0];
}

// Job tables to the device (plain copies; not part of a captured sequence).
static hipError_t upload_jobs(const StageBufs &B, const HostJobs &H, hipStream_t s) {
    const size_t n = H.base.size();
    hipError_t e = hipMemcpyAsync(B.dbase, H.base.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(B.dcount, H.count.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(B.dsj, H.sj.data(), sizeof(SampleJob) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(B.dcj, H.cj.data(), sizeof(CastJob) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(B.daj, H.aj.data(), sizeof(CastJob) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(B.dsetj, H.setj.data(), H.setj.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // host tables may go out of scope
    return e;
}

size_t job_table_bytes(int32_t n) {
    return sizeof(int64_t) * 2 * n + sizeof(SampleJob) * n + sizeof(CastJob) * 2 * n + setup_job_size() * n;
}

void pack_jobs(const HostJobs &H, char *dst) {
    const size_t n = H.base.size();
    std::memcpy(dst, H.base.data(), sizeof(int64_t) * n);
    dst += sizeof(int64_t) * n;
    std::memcpy(dst, H.count.data(), sizeof(int64_t) * n);
    dst += sizeof(int64_t) * n;
    std::memcpy(dst, H.sj.data(), sizeof(SampleJob) * n);
    dst += sizeof(SampleJob) * n;
    std::memcpy(dst, H.cj.data(), sizeof(CastJob) * n);
    dst += sizeof(CastJob) * n;
    std::memcpy(dst, H.aj.data(), sizeof(CastJob) * n);
    dst += sizeof(CastJob) * n;
    std::memcpy(dst, H.setj.data(), H.setj.size());
}

hipError_t upload_packed_jobs(const StageBufs &B, const char *src, int32_t n, hipStream_t s) {
    // the device tables are separate pieces of the stage block; one copy each
    hipError_t e = hipMemcpyAsync(B.dbase, src, sizeof(int64_t) * n, hipMemcpyHostToDevice, s);
    src += sizeof(int64_t) * n;
    if (e == hipSuccess) e = hipMemcpyAsync(B.dcount, src, sizeof(int64_t) * n, hipMemcpyHostToDevice, s);
    src += sizeof(int64_t) * n;
    if (e == hipSuccess) e = hipMemcpyAsync(B.dsj, src, sizeof(SampleJob) * n, hipMemcpyHostToDevice, s);
    src += sizeof(SampleJob) * n;
    if (e == hipSuccess) e = hipMemcpyAsync(B.dcj, src, sizeof(CastJob) * n, hipMemcpyHostToDevice, s);
    src += sizeof(CastJob) * n;
    if (e == hipSuccess) e = hipMemcpyAsync(B.daj, src, sizeof(CastJob) * n, hipMemcpyHostToDevice, s);
    src += sizeof(CastJob) * n;
    if (e == hipSuccess) e = hipMemcpyAsync(B.dsetj, src, setup_job_size() * n, hipMemcpyHostToDevice, s);
    return e;
}

// The stage sequence after the build: kernels, then three copies of the
// per-job results into pinned host slots.  ev (optional, eager runs only)
// receives an event before each stage and one at the end: ev[0..3] on s
// (before the samples, after them, after the cast, after the statistics),
// ev[4] after the six-axis cast and ev[5] after the setups, on the side
// stream when there is one.
hipError_t enqueue_stages(hra_ctx *ctx, const StageShape &sh, const StageBufs &B, void *h_tot,
                          unsigned long long *h_cc, uint32_t *h_ch, hipStream_t s, hipEvent_t *ev, uint32_t *err,
                          hipStream_t side, hipEvent_t fork, hipEvent_t join) {
    hipError_t e = hipSuccess;
    const bool forked = side && fork && join;
    if (ev) e = hipEventRecord(ev[0], s);
    if (e == hipSuccess) e = launch_sample(B.dsj, sh.n_jobs, sh.sj0, sh.S, B.pt, B.nr, B.org, B.tri, s);
    if (ev && e == hipSuccess) e = hipEventRecord(ev[1], s);
    if (forked && e == hipSuccess) e = hipEventRecord(fork, s);
    if (forked && e == hipSuccess) e = hipStreamWaitEvent(side, fork, 0);
    const hipStream_t sa = forked ? side : s;   // the six-axis cast and the setups
    // the one-sample hemisphere cast takes the samples in a spatial order
    const int32_t *order = nullptr;
    if (e == hipSuccess && sh.group == 1 && sh.trav != HRA_TRAVERSAL_REFILL)
        e = sample_order_jobs(sh.n_jobs > 1 ? B.dcj : nullptr, sh.n_jobs, sh.cj0, sh.S, B.okey0, B.oval0, B.okey1,
                              B.oval1, B.osort, s, &order);
    if (e == hipSuccess) {
        CastArgs a;
        a.jobs = B.dcj;
        a.n_jobs = sh.n_jobs;
        a.job0 = sh.cj0;
        a.dirs = sh.t_hemi;
        a.dirs_order = sh.t_hemi + sh.N;
        a.n_dirs = sh.N;
        a.kind = 0;
        a.W = sh.W;
        a.n_items = sh.items;
        a.group = sh.group;
        a.err = err;
        a.work = nullptr;
        a.order = order;
        e = launch_cast_any(a, sh.rpw, sh.stack, sh.trav, false, s);
    }
    if (ev && e == hipSuccess) e = hipEventRecord(ev[2], s);
    hra_dirstats ds = {B.mean, B.absm, B.axis, B.conc, nullptr, nullptr};
    if (e == hipSuccess) e = launch_dirstats(ctx, B.nr, sh.S, sh.t_hemi, sh.N, B.bits, ds, B.c64, B.cnt, false, s);
    if (e == hipSuccess) e = launch_part_totals_raw(B.axis, B.cnt, B.c64, B.dbase, B.dcount, sh.n_jobs, B.tot, s);
    if (ev && e == hipSuccess) e = hipEventRecord(ev[3], s);
    if (e == hipSuccess) {
        CastArgs a;
        a.jobs = B.daj;
        a.n_jobs = sh.n_jobs;
        a.job0 = sh.aj0;
        a.dirs = sh.t_ax;
        a.dirs_order = sh.t_ax;
        a.n_dirs = 6;
        a.kind = 1;
        a.W = 1;
        a.n_items = sh.aitems;
        a.group = 1;
        a.err = err;
        a.work = nullptr;
        e = launch_cast_any(a, 64, sh.stack, sh.trav, false, sa);
    }
    if (ev && e == hipSuccess) e = hipEventRecord(ev[4], sa);
    if (e == hipSuccess) e = launch_setups_raw(B.dsetj, sh.n_jobs, sh.S, B.pt, B.tri, B.abits, B.cc, B.chist, err, sa);
    if (ev && forked && e == hipSuccess) e = hipEventRecord(ev[5], sa);
    if (forked && e == hipSuccess) e = hipEventRecord(join, side);
    if (forked && e == hipSuccess) e = hipStreamWaitEvent(s, join, 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h_tot, B.tot, dir_totals_size() * sh.n_jobs, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h_cc, B.cc, sizeof(unsigned long long) * 4 * sh.n_jobs, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h_ch, B.chist, sizeof(uint32_t) * 64 * sh.n_jobs, hipMemcpyDeviceToHost, s);
    if (ev && !forked && e == hipSuccess) e = hipEventRecord(ev[5], s);
    return e;
}

void decode_results(const StageShape &sh, const std::vector<int64_t> &count, const void *h_tot,
                           const unsigned long long *h_cc, const uint32_t *h_ch, const hra_thresholds *th,
                           hra_part_result *results) {
    for (int p = 0; p < sh.n_jobs; ++p) {
        classify_from_device_totals((const char *)h_tot + dir_totals_size() * p, count[p], sh.N, th, &results[p].cls);
        hra_setup_report &R = results[p].setups;
        for (int k = 0; k < 4; ++k) R.n_class[k] = (int64_t)h_cc[4 * p + k];
        for (int c = 0; c < 64; ++c) R.code_hist[c] = h_ch[64 * p + c];
        solve_setups(R.code_hist, &R.min_count, &R.min_mask, &R.greedy_count, &R.greedy_mask);
    }
}

}  // namespace hra

using namespace hra;

struct hra_plan {
    hra_ctx *ctx = nullptr;    // valid while the context lives (destroy does not use it)
    int32_t device = 0;        // the context's device
    hra_bvh *bvh = nullptr;
    void *ws = nullptr;        // build scratch
    void *stage = nullptr;     // stage buffers
    StageBufs B;
    StageShape sh;
    std::vector<int64_t> count;
    hra_thresholds th;
    bool has_th = false;
    void *h_tot = nullptr;     // pinned result slots
    unsigned long long *h_cc = nullptr;
    uint32_t *h_ch = nullptr;
    hipStream_t own = nullptr;
    hipStream_t side = nullptr;   // the six-axis cast and the setups, beside the cast
    hipEvent_t ev[7] = {};
    hipEvent_t fork = nullptr, join = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    float stage_ms[6] = {};
    int64_t bytes = 0;
};

extern "C" void hra_plan_destroy(hra_plan *P) {
    if (!P) return;
    hipSetDevice(P->device);
    if (P->own) hipStreamSynchronize(P->own);
    if (P->side) hipStreamSynchronize(P->side);
    if (P->exec) hipGraphExecDestroy(P->exec);
    if (P->graph) hipGraphDestroy(P->graph);
    for (hipEvent_t e : P->ev)
        if (e) hipEventDestroy(e);
    if (P->ev_in) hipEventDestroy(P->ev_in);
    if (P->ev_out) hipEventDestroy(P->ev_out);
    if (P->fork) hipEventDestroy(P->fork);
    if (P->join) hipEventDestroy(P->join);
    if (P->side) hipStreamDestroy(P->side);
    if (P->own) hipStreamDestroy(P->own);
    if (P->bvh) hra_bvh_release(P->bvh);
    hipFree(P->ws);
    hipFree(P->stage);
    hipHostFree(P->h_tot);
    hipHostFree(P->h_cc);
    hipHostFree(P->h_ch);
    delete P;
}

extern "C" hra_status hra_plan_create(hra_ctx *ctx, const hra_part_request *parts, int32_t n_parts,
                                      const hra_batch_opts *opts, hra_plan **out) {
    if (!ctx || !parts || !opts || !out) return HRA_ERR_INVALID_ARG;
    *out = nullptr;
    if (n_parts < 1 || n_parts > MAX_PARTS) return ctx->fail(HRA_ERR_INVALID_ARG, "1..255 parts per batch");
    const int32_t N = opts->n_dirs;
    const int rpw = opts->rays_per_wave ? opts->rays_per_wave : ctx->cast_rpw;
    const int stack = opts->stack_depth ? opts->stack_depth : ctx->cast_stack;
    if (rpw != 64 && rpw != 128 && rpw != 256) return ctx->fail(HRA_ERR_INVALID_ARG, "rays_per_wave: 64, 128 or 256");
    if (stack != 16 && stack != 20 && stack != 24 && stack != 32)
        return ctx->fail(HRA_ERR_INVALID_ARG, "stack_depth: 16, 20, 24 or 32");
    const int trav = opts->traversal ? opts->traversal : ctx->cast_traversal;
    if (trav != HRA_TRAVERSAL_STEP && trav != HRA_TRAVERSAL_LEAF_LOOP && trav != HRA_TRAVERSAL_REFILL)
        return ctx->fail(HRA_ERR_INVALID_ARG, "traversal: 0, HRA_TRAVERSAL_STEP, _LEAF_LOOP or _REFILL");
    const float frac = opts->offset_frac > 0.0f ? opts->offset_frac : 1e-4f;
    if (!(frac <= 0.01f)) return ctx->fail(HRA_ERR_INVALID_ARG, "offset_frac must be in (0, 0.01]");
    hra_dirs hemi = {HRA_DIRS_HEMI_FIBONACCI, N}, ax6 = {HRA_DIRS_AXES6, 6};
    const float4 *t_hemi = nullptr, *t_ax = nullptr;
    hra_status st = dir_table(ctx, hemi, &t_hemi);
    if (st != HRA_OK) return st;
    st = dir_table(ctx, ax6, &t_ax);
    if (st != HRA_OK) return st;
    std::vector<hra_mesh> meshes(n_parts);
    std::vector<int64_t> count(n_parts);
    std::vector<uint64_t> seed(n_parts);
    std::vector<double> tool(n_parts);
    int64_t S = 0;
    for (int p = 0; p < n_parts; ++p) {
        if (parts[p].n_samples < 1) return ctx->fail(HRA_ERR_INVALID_ARG, "every part needs at least one sample");
        if (!(parts[p].tool_length >= 0.0)) return ctx->fail(HRA_ERR_INVALID_ARG, "tool length must be >= 0");
        meshes[p] = parts[p].mesh;
        count[p] = parts[p].n_samples;
        seed[p] = parts[p].seed;
        tool[p] = parts[p].tool_length;
        S += count[p];
    }
    const int leaf = opts->leaf_size ? opts->leaf_size : ctx->leaf_default;
    std::vector<MeshIn> hm;
    int64_t T = 0;
    st = check_meshes(ctx, meshes.data(), n_parts, leaf, &hm, &T);
    if (st != HRA_OK) return st;
    const int32_t W = (N + 31) / 32;
    if (S >= ((int64_t)1 << 31)) return ctx->fail(HRA_ERR_INVALID_ARG, "too many samples for one batch");
    HRA_HIP(hipSetDevice(ctx->device));

    hra_plan *P = new hra_plan();
    P->ctx = ctx;
    P->device = ctx->device;
    P->count = count;
    if (opts->thresholds) {
        P->th = *opts->thresholds;
        P->has_th = true;
    }
    hra_status fail_st = HRA_OK;
    const char *what = nullptr;
    hipError_t e = hipSuccess;
    st = alloc_bvh(ctx, hm, T, leaf, &P->bvh);
    if (st != HRA_OK) {
        hra_plan_destroy(P);
        return st;
    }
    const size_t ws_bytes = build_ws_bytes(T, n_parts);
    const size_t stage_bytes = carve_stage(nullptr, S, W, n_parts, nullptr);
    if (hipMalloc(&P->ws, ws_bytes) != hipSuccess || hipMalloc(&P->stage, stage_bytes) != hipSuccess ||
        hipHostMalloc(&P->h_tot, dir_totals_size() * n_parts, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&P->h_cc, sizeof(unsigned long long) * 4 * n_parts, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void **)&P->h_ch, sizeof(uint32_t) * 64 * n_parts, hipHostMallocDefault) != hipSuccess) {
        hra_plan_destroy(P);
        return ctx->fail(HRA_ERR_OUT_OF_MEMORY, "batch plan allocation failed");
    }
    P->bytes = P->bvh->bytes + (int64_t)ws_bytes + (int64_t)stage_bytes;
    carve_stage((char *)P->stage, S, W, n_parts, &P->B);
    e = hipStreamCreateWithFlags(&P->own, hipStreamNonBlocking);
    for (int k = 0; k < 7 && e == hipSuccess; ++k) e = hipEventCreate(&P->ev[k]);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->ev_out, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->join, hipEventDisableTiming);
    StageShape &sh = P->sh;
    sh.N = N;
    sh.W = W;
    sh.rpw = rpw;
    sh.stack = stack;
    sh.trav = trav;
    sh.group = cast_group(N, ctx->cast_group);
    sh.t_hemi = t_hemi;
    sh.t_ax = t_ax;
    HostJobs H;
    std::vector<const hra_bvh *> bv(n_parts, P->bvh);
    std::vector<int32_t> pidx(n_parts);
    for (int p = 0; p < n_parts; ++p) pidx[p] = p;
    fill_jobs(P->B, bv, pidx, count, seed, tool, frac, &sh, &H);
    if (e == hipSuccess)
        e = hipMemcpyAsync(build_ws_mesh_table(P->ws, T, n_parts), hm.data(), sizeof(MeshIn) * n_parts,
                           hipMemcpyHostToDevice, P->own);
    if (e == hipSuccess) e = upload_jobs(P->B, H, P->own);
    if (e != hipSuccess) {
        what = hipGetErrorString(e);
        fail_st = HRA_ERR_DEVICE;
    }
    if (fail_st != HRA_OK) {
        hra_plan_destroy(P);
        return ctx->fail(fail_st, "batch plan set-up failed", what);
    }
    *out = P;
    return HRA_OK;
}

static hipError_t plan_enqueue(hra_plan *P, hipStream_t s, bool timed) {
    hipError_t e = hipSuccess;
    if (timed) e = hipEventRecord(P->ev[6], s);
    if (e == hipSuccess) e = enqueue_build(P->ctx, P->bvh, P->ws, s, P->ctx->d_err);
    if (e == hipSuccess)
        e = enqueue_stages(P->ctx, P->sh, P->B, P->h_tot, P->h_cc, P->h_ch, s, timed ? P->ev : nullptr, P->ctx->d_err,
                           P->side, P->fork, P->join);
    return e;
}

extern "C" hra_status hra_plan_run(hra_plan *P, int32_t use_graph, hra_part_result *results, uint32_t *d_bits_out,
                                   void *stream) {
    if (!P || !results) return HRA_ERR_INVALID_ARG;
    hra_ctx *ctx = P->ctx;
    HRA_HIP(hipSetDevice(ctx->device));
    hipStream_t caller = (hipStream_t)stream;
    hipStream_t s = P->own;
    // the plan's stream follows the caller's stream
    HRA_HIP(hipEventRecord(P->ev_in, caller));
    HRA_HIP(hipStreamWaitEvent(s, P->ev_in, 0));
    hipError_t e = hipSuccess;
    if (use_graph) {
        if (!P->exec) {
            e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t e2 = plan_enqueue(P, s, false);
                hipGraph_t g = nullptr;
                e = hipStreamEndCapture(s, &g);
                if (e2 != hipSuccess) e = e2;
                if (e == hipSuccess) {
                    P->graph = g;
                    e = hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0);
                } else if (g) {
                    hipGraphDestroy(g);
                }
            }
            if (e != hipSuccess) return ctx->fail(HRA_ERR_DEVICE, "graph capture of the batch failed", hipGetErrorString(e));
        }
        e = hipGraphLaunch(P->exec, s);
    } else {
        e = plan_enqueue(P, s, true);
    }
    if (e == hipSuccess && d_bits_out)
        e = hipMemcpyAsync(d_bits_out, P->B.bits, sizeof(uint32_t) * (size_t)P->sh.W * P->sh.S,
                           hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(P->ev_out, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(caller, P->ev_out, 0);
    if (e != hipSuccess) {
        hipStreamSynchronize(s);
        hipStreamSynchronize(P->side);
        return ctx->fail(HRA_ERR_DEVICE, "batch launch failed", hipGetErrorString(e));
    }
    hra_status st = check_error_word(ctx, s);   // synchronises the plan's stream
    if (st != HRA_OK) return st;
    if (!use_graph) {
        float t[6];
        hipEventElapsedTime(&t[0], P->ev[6], P->ev[0]);   // build
        for (int k = 0; k < 3; ++k) hipEventElapsedTime(&t[k + 1], P->ev[k], P->ev[k + 1]);
        // the six-axis cast from the samples' end (it starts there, on the
        // side stream, beside the cast), then the setups after it
        hipEventElapsedTime(&t[4], P->ev[1], P->ev[4]);
        hipEventElapsedTime(&t[5], P->ev[4], P->ev[5]);
        for (int k = 0; k < 6; ++k) P->stage_ms[k] = t[k];
    }
    decode_results(P->sh, P->count, P->h_tot, P->h_cc, P->h_ch, P->has_th ? &P->th : nullptr, results);
    return HRA_OK;
}

extern "C" hra_status hra_plan_stage_ms(const hra_plan *P, float *ms6) {
    if (!P || !ms6) return HRA_ERR_INVALID_ARG;
    for (int k = 0; k < 6; ++k) ms6[k] = P->stage_ms[k];
    return HRA_OK;
}

extern "C" int64_t hra_plan_bytes(const hra_plan *P) { return P ? P->bytes : 0; }

extern "C" const uint32_t *hra_plan_bits(const hra_plan *P) { return P ? P->B.bits : nullptr; }

extern "C" hra_status hra_batch_run(hra_ctx *ctx, const hra_part_request *parts, int32_t n_parts,
                                    const hra_batch_opts *opts, hra_part_result *results, uint32_t *d_bits_out,
                                    void *stream) {
    if (!ctx || !results) return HRA_ERR_INVALID_ARG;
    hra_plan *P = nullptr;
    hra_status st = hra_plan_create(ctx, parts, n_parts, opts, &P);
    if (st != HRA_OK) return st;
    st = hra_plan_run(P, 0, results, d_bits_out, stream);
    hra_plan_destroy(P);
    return st;
}

// Project autotuner: every (rays per wave, stack depth, leaf size) point of
// the sweep runs the same batch as a plan; the fastest whole run wins.
extern "C" hra_status hra_autotune(hra_ctx *ctx, const hra_part_request *parts, int32_t n_parts,
                                   const hra_batch_opts *opts, int32_t reps, hra_tune_report *out, void *stream) {
    if (!ctx || !parts || !opts || !out) return HRA_ERR_INVALID_ARG;
    if (reps < 1 || reps > 100) return ctx->fail(HRA_ERR_INVALID_ARG, "reps must be in 1..100");
    static const int RPW[3] = {64, 128, 256}, STACK[3] = {16, 24, 32}, LEAF[3] = {2, 4, 8};
    const int trav = opts->traversal ? opts->traversal : ctx->cast_traversal;
    if (trav != HRA_TRAVERSAL_STEP && trav != HRA_TRAVERSAL_LEAF_LOOP && trav != HRA_TRAVERSAL_REFILL)
        return ctx->fail(HRA_ERR_INVALID_ARG,
                         "traversal must be 0, HRA_TRAVERSAL_STEP, HRA_TRAVERSAL_LEAF_LOOP or HRA_TRAVERSAL_REFILL");
    std::vector<hra_part_result> ref(n_parts > 0 ? n_parts : 1), got(n_parts > 0 ? n_parts : 1);
    out->n_points = 0;
    out->best = -1;
    float best_ms = 0.0f;
    for (int li = 0; li < 3; ++li)
        for (int ri = 0; ri < 3; ++ri)
            for (int si = 0; si < 3; ++si) {
                hra_batch_opts o = *opts;
                o.leaf_size = LEAF[li];
                o.rays_per_wave = RPW[ri];
                o.stack_depth = STACK[si];
                o.traversal = trav;
                hra_plan *P = nullptr;
                hra_status st = hra_plan_create(ctx, parts, n_parts, &o, &P);
                if (st != HRA_OK) return st;
                const bool first = out->n_points == 0;
                st = hra_plan_run(P, 0, first ? ref.data() : got.data(), nullptr, stream);   // warm-up
                double sum = 0.0;
                for (int r = 0; r < reps && st == HRA_OK; ++r) {
                    st = hra_plan_run(P, 0, got.data(), nullptr, stream);
                    float ms6[6];
                    hra_plan_stage_ms(P, ms6);
                    for (int k = 0; k < 6; ++k) sum += ms6[k];
                }
                hra_plan_destroy(P);
                if (st != HRA_OK) return st;
                // the launch shape must not change any result
                if (std::memcmp(ref.data(), got.data(), sizeof(hra_part_result) * n_parts) != 0)
                    return ctx->fail(HRA_ERR_DEVICE, "autotuner: results differ between launch shapes");
                hra_tune_point &pt = out->points[out->n_points];
                pt.rays_per_wave = RPW[ri];
                pt.stack_depth = STACK[si];
                pt.leaf_size = LEAF[li];
                pt.traversal = trav;
                pt.ms = (float)(sum / reps);
                if (out->best < 0 || pt.ms < best_ms) {
                    out->best = out->n_points;
                    best_ms = pt.ms;
                }
                ++out->n_points;
            }
    const hra_tune_point &b = out->points[out->best];
    ctx->cast_rpw = b.rays_per_wave;
    ctx->cast_stack = b.stack_depth;
    ctx->leaf_default = b.leaf_size;
    ctx->cast_traversal = b.traversal;
    return HRA_OK;
}

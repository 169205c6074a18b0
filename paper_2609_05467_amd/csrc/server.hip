// Analysis server: part analyses arrive one by one (the interactive use of
// the method, Section 1) and are served with continuous batching.
//
// One worker thread owns a context and the device.  Each turn it takes the
// new submissions, notices finished builds and batches (event queries, no
// blocking), admits waiting requests in arrival order while their memory
// footprint fits the budget (evicting resident hierarchies that no request
// uses, oldest use first), starts the builds of parts that are not resident
// on a build stream, and launches the admitted requests as one batch (one
// launch per stage for all of them) on one of up to four compute streams as
// soon as a stream is free.  A request that arrives while batches run is
// admitted and built at once and goes into the next batch; builds overlap
// the running casts.  Hierarchies stay resident after their requests end
// and are reused by later requests for the same part key.
//
// The plain mode is the reference point: one request at a time in arrival
// order, built, cast and finished on one stream before the next starts,
// nothing kept resident.
#include "sched.hpp"
#include "stages.hpp"

#include <chrono>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>

namespace hra {

__global__ void k_zero_words(uint32_t *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

static int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct SrvReq {
    hra_request in;
    uint64_t ticket = 0;
    hra_request_result out;
    bool done = false;
};

struct SrvPart {
    hra_bvh *bvh = nullptr;
    hipEvent_t built = nullptr;
    uint32_t *d_err = nullptr;   // the build's error word (device)
    uint32_t *h_err = nullptr;   // its copy (pinned)
    bool known_done = false;
    bool failed_launch = false;
};

struct SrvBatch {
    int64_t id = 0;
    std::vector<uint64_t> tickets;    // every request of the batch
    std::vector<uint64_t> launched;   // those on the device, in job order
    std::vector<uint64_t> part_keys;  // part of each launched job
    std::vector<int64_t> count;
    StageShape sh;
    char *pinned = nullptr;
    size_t pinned_cap = 0;
    hipEvent_t done = nullptr;
    int stream = 0;
};

}  // namespace hra

using namespace hra;

struct hra_server {
    hra_ctx *ctx = nullptr;
    hra_server_opts opts;
    hra_thresholds th;
    bool has_th = false;
    std::unique_ptr<sched::Scheduler> S;
    const float4 *t_hemi = nullptr, *t_ax = nullptr;
    hipStream_t build_stream = nullptr;
    hipStream_t comp[4] = {};
    // shared with submitting threads
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> inbox;
    std::unordered_map<uint64_t, std::unique_ptr<SrvReq>> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    hra_server_stats st;
    // worker only
    std::unordered_map<uint64_t, SrvPart> parts;
    std::vector<std::unique_ptr<SrvBatch>> inflight;
    std::vector<std::pair<char *, size_t>> pinned_pool;
    std::vector<hipEvent_t> event_pool;
    int64_t next_batch_id = 1;
    std::thread worker;
};

namespace {

const int64_t kStageExtra = 256;   // the batch error word after the stage block

int64_t stage_bytes_of(int64_t n_samples, int32_t W) {
    return (int64_t)carve_stage(nullptr, n_samples, W, 1, nullptr);
}

char *take_pinned(hra_server *sv, size_t need, size_t *cap) {
    for (size_t i = 0; i < sv->pinned_pool.size(); ++i)
        if (sv->pinned_pool[i].second >= need) {
            auto b = sv->pinned_pool[i];
            sv->pinned_pool.erase(sv->pinned_pool.begin() + i);
            *cap = b.second;
            return b.first;
        }
    size_t c = 4096;
    while (c < need) c <<= 1;
    char *p = nullptr;
    if (hipHostMalloc((void **)&p, c, hipHostMallocDefault) != hipSuccess) return nullptr;
    *cap = c;
    return p;
}

hipEvent_t take_event(hra_server *sv) {
    if (!sv->event_pool.empty()) {
        hipEvent_t e = sv->event_pool.back();
        sv->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

void finish(hra_server *sv, uint64_t t, hra_status status, const hra_part_result *res) {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(t);
    if (it == sv->reqs.end()) return;
    SrvReq &r = *it->second;
    r.out.status = status;
    r.out.t_done_ns = now_ns();
    if (res) r.out.result = *res;
    r.done = true;
    if (status == HRA_OK) ++sv->st.completed;
    else ++sv->st.failed;
    sv->cv_done.notify_all();
}

SrvReq *req_of(hra_server *sv, uint64_t t) {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(t);
    return it == sv->reqs.end() ? nullptr : it->second.get();
}

void release_part(hra_server *sv, uint64_t key) {
    auto it = sv->parts.find(key);
    if (it == sv->parts.end()) return;
    SrvPart &p = it->second;
    hipStream_t s = p.bvh && p.bvh->alloc_stream ? p.bvh->alloc_stream : sv->build_stream;
    if (p.bvh) hra_bvh_release(p.bvh);
    if (p.d_err) hipFreeAsync(p.d_err, s);
    if (p.h_err) hipHostFree(p.h_err);
    if (p.built) sv->event_pool.push_back(p.built);
    sv->parts.erase(it);
}

// Upload the mesh and enqueue the build of part `key` from request `r`.
void start_build(hra_server *sv, uint64_t key, const hra_request &r) {
    hipStream_t s = sv->opts.mode == HRA_SERVE_PLAIN ? sv->comp[0] : sv->build_stream;
    SrvPart &p = sv->parts[key];
    hipError_t e = hipSuccess;
    float *dv = nullptr;
    int32_t *dt = nullptr;
    void *ws = nullptr;
    const int leaf = sv->opts.leaf_size ? sv->opts.leaf_size : sv->ctx->leaf_default;
    p.built = take_event(sv);
    if (!p.built) e = hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipHostMalloc((void **)&p.h_err, 64, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMallocAsync((void **)&p.d_err, 64, s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&dv, sizeof(float) * 3 * r.n_verts, s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&dt, sizeof(int32_t) * 3 * r.n_tris, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dv, r.h_verts, sizeof(float) * 3 * r.n_verts, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dt, r.h_tris, sizeof(int32_t) * 3 * r.n_tris, hipMemcpyHostToDevice, s);
    std::vector<MeshIn> hm = {MeshIn{dv, dt, r.n_verts, r.n_tris, 0, 0}};
    if (e == hipSuccess && alloc_bvh(sv->ctx, hm, r.n_tris, leaf, &p.bvh, s, BVH_POOL_KEEP) != HRA_OK) e = hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipMallocAsync(&ws, build_ws_bytes(r.n_tris, 1), s);
    if (e == hipSuccess) {
        k_zero_words<<<1, 64, 0, s>>>(p.d_err, 16);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = put_mesh_table(build_ws_mesh_table(ws, r.n_tris, 1), hm[0], s);
    if (e == hipSuccess) e = enqueue_build(sv->ctx, p.bvh, ws, s, p.d_err);
    if (e == hipSuccess) e = hipMemcpyAsync(p.h_err, p.d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    for (void *q : {(void *)dv, (void *)dt, ws})
        if (q) hipFreeAsync(q, s);
    if (e == hipSuccess) e = hipEventRecord(p.built, s);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        ++sv->st.builds;
    }
    if (e != hipSuccess) {
        hipStreamSynchronize(s);
        p.failed_launch = true;
        p.known_done = true;
        // its requests still pin it (they fail when their batch forms), so
        // nothing is released here
        sv->S->build_done(key, false);
    }
}

void fail_batch(hra_server *sv, const std::vector<uint64_t> &tickets, hra_status st) {
    for (uint64_t t : tickets) finish(sv, t, st, nullptr);
    for (uint64_t k : sv->S->batch_done(tickets)) release_part(sv, k);
}

void launch_batch(hra_server *sv, const std::vector<uint64_t> &tickets) {
    auto b = std::make_unique<SrvBatch>();
    b->id = sv->next_batch_id++;
    b->tickets = tickets;
    b->stream = sv->opts.mode == HRA_SERVE_PLAIN ? 0 : (int)(b->id % sv->opts.max_inflight);
    hipStream_t s = sv->comp[b->stream];
    std::vector<const hra_bvh *> bv;
    std::vector<int32_t> pidx;
    std::vector<uint64_t> seeds;
    std::vector<double> tools;
    std::vector<uint64_t> broken;
    const int64_t t_launch = now_ns();
    for (uint64_t t : tickets) {
        SrvReq *r = req_of(sv, t);
        if (!r) continue;
        auto pit = sv->parts.find(r->in.part_key);
        if (pit == sv->parts.end() || pit->second.failed_launch || sv->S->broken(r->in.part_key)) {
            broken.push_back(t);
            continue;
        }
        b->launched.push_back(t);
        b->part_keys.push_back(r->in.part_key);
        bv.push_back(pit->second.bvh);
        pidx.push_back(0);
        b->count.push_back(r->in.n_samples);
        seeds.push_back(r->in.seed);
        tools.push_back(r->in.tool_length);
        std::lock_guard<std::mutex> lk(sv->mu);
        r->out.t_launch_ns = t_launch;
        r->out.batch_id = b->id;
        r->out.batch_size = (int32_t)tickets.size();
    }
    for (uint64_t t : broken) finish(sv, t, HRA_ERR_BAD_MESH, nullptr);
    if (b->launched.empty()) {
        for (uint64_t k : sv->S->batch_done(tickets)) release_part(sv, k);
        return;
    }
    const int32_t n = (int32_t)b->launched.size();
    StageShape &sh = b->sh;
    sh.N = sv->opts.n_dirs;
    sh.W = (sh.N + 31) / 32;
    sh.rpw = sv->ctx->cast_rpw;
    sh.stack = sv->ctx->cast_stack;
    sh.trav = sv->ctx->cast_traversal;
    sh.group = cast_group(sh.N, sv->ctx->cast_group);
    sh.t_hemi = sv->t_hemi;
    sh.t_ax = sv->t_ax;
    int64_t S = 0;
    for (int64_t c : b->count) S += c;
    const size_t stage_bytes = carve_stage(nullptr, S, sh.W, n, nullptr);
    const size_t res_bytes = dir_totals_size() * n + sizeof(unsigned long long) * 4 * n + sizeof(uint32_t) * 64 * n;
    const size_t jt = job_table_bytes(n);
    const size_t jt_pad = (jt + 255) & ~(size_t)255;
    hipError_t e = hipSuccess;
    // a batch waits for the builds of its parts on the device, not on the host
    for (uint64_t k : b->part_keys) {
        SrvPart &p = sv->parts[k];
        if (!p.known_done && e == hipSuccess) e = hipStreamWaitEvent(s, p.built, 0);
    }
    char *stage = nullptr;
    if (e == hipSuccess) e = hipMallocAsync((void **)&stage, stage_bytes + kStageExtra, s);
    b->pinned = take_pinned(sv, jt_pad + res_bytes + 64, &b->pinned_cap);
    if (!b->pinned && e == hipSuccess) e = hipErrorOutOfMemory;
    b->done = take_event(sv);
    if (!b->done && e == hipSuccess) e = hipErrorOutOfMemory;
    if (e == hipSuccess) {
        StageBufs B;
        carve_stage(stage, S, sh.W, n, &B);
        HostJobs H;
        const float frac = sv->opts.offset_frac > 0.0f ? sv->opts.offset_frac : 1e-4f;
        fill_jobs(B, bv, pidx, b->count, seeds, tools, frac, &sh, &H);
        pack_jobs(H, b->pinned);
        uint32_t *err = (uint32_t *)(stage + stage_bytes);
        char *h_tot = b->pinned + jt_pad;
        unsigned long long *h_cc = (unsigned long long *)(h_tot + dir_totals_size() * n);
        uint32_t *h_ch = (uint32_t *)(h_cc + 4 * n);
        uint32_t *h_err = (uint32_t *)(h_ch + 64 * n);
        *h_err = 0u;
        k_zero_words<<<1, 64, 0, s>>>(err, 16);
        e = hipGetLastError();
        if (e == hipSuccess) e = upload_packed_jobs(B, b->pinned, n, s);
        if (e == hipSuccess) e = enqueue_stages(sv->ctx, sh, B, h_tot, h_cc, h_ch, s, nullptr, err);
        if (e == hipSuccess) e = hipMemcpyAsync(h_err, err, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    }
    if (stage) hipFreeAsync(stage, s);
    if (e == hipSuccess) e = hipEventRecord(b->done, s);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        ++sv->st.batches;
    }
    if (e != hipSuccess) {
        hipStreamSynchronize(s);
        if (b->pinned) sv->pinned_pool.push_back({b->pinned, b->pinned_cap});
        if (b->done) sv->event_pool.push_back(b->done);
        fail_batch(sv, b->launched, HRA_ERR_DEVICE);
        return;
    }
    sv->inflight.push_back(std::move(b));
}

void complete_batch(hra_server *sv, SrvBatch &b) {
    const int32_t n = (int32_t)b.launched.size();
    const size_t jt_pad = (job_table_bytes(n) + 255) & ~(size_t)255;
    const char *h_tot = b.pinned + jt_pad;
    const unsigned long long *h_cc = (const unsigned long long *)(h_tot + dir_totals_size() * n);
    const uint32_t *h_ch = (const uint32_t *)(h_cc + 4 * n);
    const uint32_t h_err = *(const uint32_t *)(h_ch + 64 * n);
    std::vector<hra_part_result> res(n);
    decode_results(b.sh, b.count, h_tot, h_cc, h_ch, sv->has_th ? &sv->th : nullptr, res.data());
    for (int j = 0; j < n; ++j) {
        auto pit = sv->parts.find(b.part_keys[j]);
        // the build finished before this batch did (device-side wait), so its
        // error word is in pinned memory already
        const uint32_t perr = pit != sv->parts.end() && pit->second.h_err ? *pit->second.h_err : 0u;
        hra_status st = HRA_OK;
        if (perr) st = HRA_ERR_BAD_MESH;
        else if (h_err) st = HRA_ERR_DEVICE;
        finish(sv, b.launched[j], st, st == HRA_OK ? &res[j] : nullptr);
    }
    sv->pinned_pool.push_back({b.pinned, b.pinned_cap});
    sv->event_pool.push_back(b.done);
    // a batch whose device error word is set: the hierarchies it read are
    // not trusted again (dropped when unpinned, rebuilt on next use)
    for (uint64_t k : sv->S->batch_done(b.tickets, h_err != 0u)) release_part(sv, k);
}

void worker_loop(hra_server *sv) {
    hipSetDevice(sv->ctx->device);
    for (;;) {
        bool progress = false;
        std::vector<uint64_t> fresh;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            if (sv->stop) break;
            fresh.assign(sv->inbox.begin(), sv->inbox.end());
            sv->inbox.clear();
        }
        const int32_t W = (sv->opts.n_dirs + 31) / 32;
        for (uint64_t t : fresh) {
            SrvReq *r = req_of(sv, t);
            sched::Req q;
            q.ticket = t;
            q.part_key = r->in.part_key;
            q.part_bytes = bvh_bytes(r->in.n_tris, 1);
            q.build_bytes = (int64_t)build_ws_bytes(r->in.n_tris, 1) + 12 * (r->in.n_verts + r->in.n_tris) + 1024;
            q.stage_bytes = stage_bytes_of(r->in.n_samples, W) + kStageExtra;
            sv->S->submit(q);
            progress = true;
        }
        // finished builds (a part no request holds any more is released
        // after the loop)
        std::vector<uint64_t> unheld;
        for (auto &kv : sv->parts) {
            SrvPart &p = kv.second;
            if (p.known_done || !p.built) continue;
            if (hipEventQuery(p.built) == hipSuccess) {
                p.known_done = true;
                for (uint64_t k : sv->S->build_done(kv.first, *p.h_err == 0u)) unheld.push_back(k);
                progress = true;
            }
        }
        for (uint64_t k : unheld) release_part(sv, k);
        // finished batches
        for (size_t i = 0; i < sv->inflight.size();) {
            if (hipEventQuery(sv->inflight[i]->done) == hipSuccess) {
                complete_batch(sv, *sv->inflight[i]);
                sv->inflight.erase(sv->inflight.begin() + i);
                progress = true;
            } else {
                ++i;
            }
        }
        // admission
        const sched::Admission a = sv->S->admit();
        for (uint64_t k : a.evict) release_part(sv, k);
        for (uint64_t t : a.rejected) finish(sv, t, HRA_ERR_OVER_BUDGET, nullptr);
        if (!a.admitted.empty() || !a.rejected.empty() || !a.evict.empty()) progress = true;
        {
            const int64_t t_admit = now_ns();
            std::lock_guard<std::mutex> lk(sv->mu);
            for (uint64_t t : a.admitted) sv->reqs[t]->out.t_admit_ns = t_admit;
            for (uint64_t t : a.hits) sv->reqs[t]->out.resident_hit = 1;
            sv->st.resident_hits += (int64_t)a.hits.size();
            sv->st.evictions += (int64_t)a.evict.size();
        }
        for (uint64_t k : a.build) {
            // the first admitted request naming this part supplies its mesh
            for (uint64_t t : a.admitted) {
                SrvReq *r = req_of(sv, t);
                if (r->in.part_key == k) {
                    start_build(sv, k, r->in);
                    break;
                }
            }
        }
        // launches
        for (;;) {
            std::vector<uint64_t> b = sv->S->next_batch();
            if (b.empty()) break;
            launch_batch(sv, b);
            progress = true;
        }
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->st.used_bytes = sv->S->used();
            sv->st.resident_bytes = sv->S->resident_bytes();
            if (sv->st.used_bytes > sv->st.peak_used_bytes) sv->st.peak_used_bytes = sv->st.used_bytes;
            sv->st.resident_parts = (int32_t)sv->S->resident_parts();
            sv->st.inflight = sv->S->inflight();
            sv->st.pending = (int32_t)sv->S->pending();
            if (!progress) {
                // nothing new: wait for a submission, or poll the device again
                // shortly when work is on it
                const bool busy = !sv->S->idle();
                if (busy)
                    sv->cv_work.wait_for(lk, std::chrono::microseconds(20));
                else
                    sv->cv_work.wait_for(lk, std::chrono::milliseconds(5), [&] { return sv->stop || !sv->inbox.empty(); });
            }
        }
    }
    // shut down: let the device finish, then release everything
    for (auto &b : sv->inflight) {
        hipEventSynchronize(b->done);
        complete_batch(sv, *b);
    }
    sv->inflight.clear();
    hipStreamSynchronize(sv->build_stream);
    for (hipStream_t s : sv->comp)
        if (s) hipStreamSynchronize(s);
    std::vector<uint64_t> keys;
    for (auto &kv : sv->parts) keys.push_back(kv.first);
    for (uint64_t k : keys) release_part(sv, k);
    hipStreamSynchronize(sv->build_stream);
    for (hipStream_t s : sv->comp)
        if (s) hipStreamSynchronize(s);
}

}  // namespace

extern "C" int64_t hra_now_ns(void) { return now_ns(); }

extern "C" void hra_server_destroy(hra_server *sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    if (sv->ctx) hipSetDevice(sv->ctx->device);
    for (auto &b : sv->pinned_pool) hipHostFree(b.first);
    for (hipEvent_t e : sv->event_pool) hipEventDestroy(e);
    if (sv->build_stream) hipStreamDestroy(sv->build_stream);
    for (hipStream_t s : sv->comp)
        if (s) hipStreamDestroy(s);
    if (sv->ctx) hra_ctx_destroy(sv->ctx);
    delete sv;
}

extern "C" hra_status hra_server_create(int32_t device, const hra_server_opts *opts, hra_server **out) {
    if (!opts || !out) return HRA_ERR_INVALID_ARG;
    *out = nullptr;
    hra_server_opts o = *opts;
    if (o.budget_bytes == 0) o.budget_bytes = 200ll << 30;
    if (o.max_batch == 0) o.max_batch = 64;
    if (o.max_inflight == 0) o.max_inflight = 2;
    if (o.budget_bytes < 0 || o.max_batch < 1 || o.max_batch > MAX_PARTS || o.max_inflight < 1 ||
        o.max_inflight > 4 || (o.mode != HRA_SERVE_CONTINUOUS && o.mode != HRA_SERVE_PLAIN) || o.leaf_size < 0 ||
        o.leaf_size > 16 || o.offset_frac < 0.0f || o.offset_frac > 0.01f)
        return HRA_ERR_INVALID_ARG;
    hra_server *sv = new hra_server();
    hra_status st = hra_ctx_create(device, &sv->ctx);
    if (st != HRA_OK) {
        delete sv;
        return st;
    }
    sv->opts = o;
    if (o.thresholds) {
        sv->th = *o.thresholds;
        sv->has_th = true;
    }
    sv->opts.thresholds = nullptr;
    std::memset(&sv->st, 0, sizeof(sv->st));
    hra_dirs hemi = {HRA_DIRS_HEMI_FIBONACCI, o.n_dirs}, ax6 = {HRA_DIRS_AXES6, 6};
    st = dir_table(sv->ctx, hemi, &sv->t_hemi);
    if (st == HRA_OK) st = dir_table(sv->ctx, ax6, &sv->t_ax);
    if (st != HRA_OK) {
        hra_server_destroy(sv);
        return st;
    }
    sched::Config c;
    c.budget = o.budget_bytes;
    c.max_batch = o.max_batch;
    c.max_inflight = o.max_inflight;
    c.plain = o.mode == HRA_SERVE_PLAIN;
    c.keep_resident = o.mode != HRA_SERVE_PLAIN && o.keep_resident != 0;
    sv->S = std::make_unique<sched::Scheduler>(c);
    hipError_t e = hipStreamCreateWithFlags(&sv->build_stream, hipStreamNonBlocking);
    for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&sv->comp[i], hipStreamNonBlocking);
    if (e != hipSuccess) {
        hra_server_destroy(sv);
        return HRA_ERR_DEVICE;
    }
    sv->worker = std::thread(worker_loop, sv);
    *out = sv;
    return HRA_OK;
}

extern "C" hra_status hra_server_submit(hra_server *sv, const hra_request *r, uint64_t *ticket) {
    if (!sv || !r || !ticket) return HRA_ERR_INVALID_ARG;
    if (!r->h_verts || !r->h_tris || r->n_verts < 3 || r->n_tris < 1 || r->n_verts >= ((int64_t)1 << 31) ||
        r->n_tris >= ((int64_t)1 << 27) || r->n_samples < 1 || r->n_samples >= ((int64_t)1 << 31) ||
        !(r->tool_length >= 0.0))
        return HRA_ERR_INVALID_ARG;
    auto q = std::make_unique<SrvReq>();
    q->in = *r;
    std::memset(&q->out, 0, sizeof(q->out));
    q->out.status = HRA_ERR_NOT_READY;
    q->out.t_submit_ns = now_ns();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stop) return HRA_ERR_INVALID_ARG;
        q->ticket = sv->next_ticket++;
        *ticket = q->ticket;
        sv->inbox.push_back(q->ticket);
        sv->reqs.emplace(q->ticket, std::move(q));
        ++sv->st.submitted;
    }
    sv->cv_work.notify_one();
    return HRA_OK;
}

static hra_status take_result(hra_server *sv, uint64_t ticket, hra_request_result *out) {
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return HRA_ERR_INVALID_ARG;
    if (!it->second->done) return HRA_ERR_NOT_READY;
    *out = it->second->out;
    sv->reqs.erase(it);
    return HRA_OK;
}

extern "C" hra_status hra_server_poll(hra_server *sv, uint64_t ticket, hra_request_result *out) {
    if (!sv || !out) return HRA_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    return take_result(sv, ticket, out);
}

extern "C" hra_status hra_server_wait(hra_server *sv, uint64_t ticket, int64_t timeout_ms, hra_request_result *out) {
    if (!sv || !out) return HRA_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto ready = [&] {
        auto it = sv->reqs.find(ticket);
        return it == sv->reqs.end() || it->second->done;
    };
    if (timeout_ms < 0) sv->cv_done.wait(lk, ready);
    else sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    return take_result(sv, ticket, out);
}

extern "C" hra_status hra_server_drain(hra_server *sv, int64_t timeout_ms) {
    if (!sv) return HRA_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto all = [&] { return sv->st.completed + sv->st.failed == sv->st.submitted; };
    if (timeout_ms < 0) sv->cv_done.wait(lk, all);
    else if (!sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), all)) return HRA_ERR_NOT_READY;
    return HRA_OK;
}

extern "C" hra_status hra_server_get_stats(hra_server *sv, hra_server_stats *out) {
    if (!sv || !out) return HRA_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->st;
    return HRA_OK;
}

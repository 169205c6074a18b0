// Host-only harness of the server's scheduling core for the CPU tests: a
// flat C interface over hra::sched::Scheduler (built with g++ by the tests).
#include <cstring>

#include "../paper_2609_05467_amd/csrc/sched.hpp"

using hra::sched::Scheduler;

extern "C" {

void *shim_create(long long budget, int max_batch, int max_inflight, int plain, int keep_resident) {
    hra::sched::Config c;
    c.budget = budget;
    c.max_batch = max_batch;
    c.max_inflight = max_inflight;
    c.plain = plain != 0;
    c.keep_resident = keep_resident != 0;
    return new Scheduler(c);
}

void shim_destroy(void *s) { delete (Scheduler *)s; }

void shim_submit(void *s, unsigned long long ticket, unsigned long long key, long long part_bytes,
                 long long build_bytes, long long stage_bytes) {
    hra::sched::Req r;
    r.ticket = ticket;
    r.part_key = key;
    r.part_bytes = part_bytes;
    r.build_bytes = build_bytes;
    r.stage_bytes = stage_bytes;
    ((Scheduler *)s)->submit(r);
}

static int put(const std::vector<uint64_t> &v, unsigned long long *out, int cap) {
    const int n = (int)v.size() < cap ? (int)v.size() : cap;
    for (int i = 0; i < n; ++i) out[i] = v[i];
    return (int)v.size();
}

// out: five arrays of `cap` entries (evict, build, admitted, hits, rejected);
// counts: their lengths
void shim_admit(void *s, unsigned long long *evict, unsigned long long *build, unsigned long long *admitted,
                unsigned long long *hits, unsigned long long *rejected, int cap, int *counts) {
    const hra::sched::Admission a = ((Scheduler *)s)->admit();
    counts[0] = put(a.evict, evict, cap);
    counts[1] = put(a.build, build, cap);
    counts[2] = put(a.admitted, admitted, cap);
    counts[3] = put(a.hits, hits, cap);
    counts[4] = put(a.rejected, rejected, cap);
}

int shim_build_done(void *s, unsigned long long key, int ok, unsigned long long *released, int cap) {
    return put(((Scheduler *)s)->build_done(key, ok != 0), released, cap);
}

int shim_next_batch(void *s, unsigned long long *out, int cap) { return put(((Scheduler *)s)->next_batch(), out, cap); }

int shim_batch_done(void *s, const unsigned long long *tickets, int n, unsigned long long *released, int cap) {
    std::vector<uint64_t> t(tickets, tickets + n);
    return put(((Scheduler *)s)->batch_done(t), released, cap);
}

// a batch whose device error word was set
int shim_batch_failed(void *s, const unsigned long long *tickets, int n, unsigned long long *released, int cap) {
    std::vector<uint64_t> t(tickets, tickets + n);
    return put(((Scheduler *)s)->batch_done(t, true), released, cap);
}

// 1 if cancelled (pending or admitted, not launched), 0 otherwise
int shim_cancel(void *s, unsigned long long ticket, unsigned long long *released, int cap, int *n_released) {
    std::vector<uint64_t> rel;
    const bool ok = ((Scheduler *)s)->cancel(ticket, &rel);
    *n_released = put(rel, released, cap);
    return ok ? 1 : 0;
}

int shim_broken(void *s, unsigned long long key) { return ((Scheduler *)s)->broken(key) ? 1 : 0; }

long long shim_used(void *s) { return ((Scheduler *)s)->used(); }
long long shim_resident(void *s) { return ((Scheduler *)s)->resident_bytes(); }
long long shim_evictions(void *s) { return ((Scheduler *)s)->evictions(); }
int shim_inflight(void *s) { return ((Scheduler *)s)->inflight(); }
int shim_pending(void *s) { return (int)((Scheduler *)s)->pending(); }
int shim_waiting(void *s) { return (int)((Scheduler *)s)->waiting(); }
int shim_idle(void *s) { return ((Scheduler *)s)->idle() ? 1 : 0; }
int shim_has_part(void *s, unsigned long long key) { return ((Scheduler *)s)->has_part(key) ? 1 : 0; }
int shim_pins(void *s, unsigned long long key) {
    const hra::sched::Part *p = ((Scheduler *)s)->part(key);
    return p ? p->pins : -1;
}
}

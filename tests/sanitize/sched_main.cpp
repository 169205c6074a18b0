// Host driver of the server's scheduling core for sanitizer builds: a seeded
// run of submissions, cancellations, admissions, builds (some failing) and
// batches (some failing), checking the byte accounting after every step.
// Exit 0 on success.
#include <cstdio>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "../../paper_2609_05467_amd/csrc/sched.hpp"

int main() {
    using namespace hra::sched;
    for (int mode = 0; mode < 3; ++mode) {
        Config c;
        c.budget = 6000;
        c.max_batch = 4;
        c.max_inflight = 2;
        c.plain = mode == 1;
        c.keep_resident = mode != 2;
        Scheduler s(c);
        std::mt19937_64 rng(17 + mode);
        std::set<uint64_t> building;
        std::vector<std::vector<uint64_t>> inflight;
        std::vector<uint64_t> tickets;
        uint64_t t = 0;
        for (int step = 0; step < 4000; ++step) {
            const double r = std::uniform_real_distribution<double>(0, 1)(rng);
            if (r < 0.35) {
                Req q;
                q.ticket = ++t;
                q.part_key = 100 + rng() % 15;
                q.part_bytes = 200 + (int64_t)(q.part_key % 7) * 180;
                q.build_bytes = (int64_t)(rng() % 300);
                q.stage_bytes = 10 + (int64_t)(rng() % 200);
                s.submit(q);
                tickets.push_back(q.ticket);
            } else if (r < 0.45 && !tickets.empty()) {
                std::vector<uint64_t> rel;
                s.cancel(tickets[rng() % tickets.size()], &rel);
            }
            const Admission a = s.admit();
            for (uint64_t k : a.build) building.insert(k);
            if (!building.empty() && (rng() & 1)) {
                auto it = building.begin();
                std::advance(it, (long)(rng() % building.size()));
                const uint64_t k = *it;
                building.erase(it);
                s.build_done(k, rng() % 10 != 0);
            }
            std::vector<uint64_t> b = s.next_batch();
            if (!b.empty()) inflight.push_back(b);
            if (!inflight.empty() && (rng() & 1)) {
                s.batch_done(inflight.front(), rng() % 10 == 0);
                inflight.erase(inflight.begin());
            }
            if (s.used() < s.resident_bytes() || s.used() > c.budget) {
                std::printf("accounting broken at step %d (mode %d)\n", step, mode);
                return 1;
            }
        }
        for (uint64_t k : building) s.build_done(k, true);
        for (;;) {
            for (auto &b : inflight) s.batch_done(b);
            inflight.clear();
            for (uint64_t k : s.admit().build) s.build_done(k, true);
            std::vector<uint64_t> b = s.next_batch();
            if (b.empty()) break;
            inflight.push_back(b);
        }
        if (s.used() != s.resident_bytes() || s.inflight() != 0 || s.pending() != 0 || s.waiting() != 0) {
            std::printf("end state broken (mode %d): used %lld resident %lld inflight %d pending %zu waiting %zu parts %zu\n", mode, (long long)s.used(), (long long)s.resident_bytes(), s.inflight(), s.pending(), s.waiting(), s.resident_parts());
            return 1;
        }
    }
    std::printf("sched ok\n");
    return 0;
}

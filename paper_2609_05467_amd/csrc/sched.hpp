// Scheduling core of the analysis server: admission by memory footprint,
// residency of part hierarchies with least-recently-used eviction, and the
// formation of launch batches (continuous batching).  Plain C++ with no
// device calls, so that its decisions can be exercised on the host alone;
// the server drives it and carries out what it decides (builds, evictions,
// launches).
//
// Accounting: the bytes in use are the resident hierarchies (built or being
// built), the transient scratch of builds in progress, and the working set
// of every admitted request (its samples, bitmasks and statistics) until its
// batch has finished.  A request is admitted only if that total stays within
// the budget after evicting unpinned resident hierarchies, oldest use
// first; requests are admitted in arrival order, so a request that does not
// fit holds back the ones behind it until memory frees up.
#pragma once

#include <cstdint>
#include <deque>
#include <list>
#include <unordered_map>
#include <vector>

namespace hra {
namespace sched {

enum class PartState { Building, Ready };

struct Config {
    int64_t budget = 200ll << 30;   // bytes
    int32_t max_batch = 64;         // requests per launch batch
    int32_t max_inflight = 2;       // batches on the device at once
    bool plain = false;             // one request at a time, nothing kept resident
    bool keep_resident = true;      // keep hierarchies after their requests end (LRU)
};

struct Req {
    uint64_t ticket = 0;
    uint64_t part_key = 0;
    int64_t part_bytes = 0;    // resident bytes of its hierarchy
    int64_t build_bytes = 0;   // transient bytes while building it
    int64_t stage_bytes = 0;   // working set while admitted
};

struct Part {
    uint64_t key = 0;
    int64_t bytes = 0;
    int64_t build_bytes = 0;
    int32_t pins = 0;          // admitted requests that use it
    PartState state = PartState::Building;
    std::list<uint64_t>::iterator lru;   // position in the recency list (front = oldest)
};

struct Admission {
    std::vector<uint64_t> evict;      // part keys to release (unpinned, resident)
    std::vector<uint64_t> build;      // part keys to build (first use)
    std::vector<uint64_t> admitted;   // tickets admitted now, in order
    std::vector<uint64_t> hits;       // admitted tickets whose part was already resident
    std::vector<uint64_t> rejected;   // tickets that cannot fit even alone
};

class Scheduler {
public:
    explicit Scheduler(const Config &c) : cfg_(c) {
        if (cfg_.plain) {
            cfg_.max_batch = 1;
            cfg_.max_inflight = 1;
            cfg_.keep_resident = false;
        }
        if (cfg_.max_batch < 1) cfg_.max_batch = 1;
        if (cfg_.max_inflight < 1) cfg_.max_inflight = 1;
    }

    const Config &config() const { return cfg_; }
    int64_t used() const { return used_; }
    int64_t resident_bytes() const { return resident_; }
    size_t pending() const { return pending_.size(); }
    size_t waiting() const { return waiting_.size(); }
    int32_t inflight() const { return inflight_; }
    size_t resident_parts() const { return parts_.size(); }
    int64_t evictions() const { return evictions_; }
    bool idle() const { return pending_.empty() && waiting_.empty() && inflight_ == 0 && building_ == 0; }
    bool has_part(uint64_t key) const { return parts_.count(key) != 0; }
    const Part *part(uint64_t key) const {
        auto it = parts_.find(key);
        return it == parts_.end() ? nullptr : &it->second;
    }

    void submit(const Req &r) { pending_.push_back(r); }

    // Admit pending requests in arrival order while they fit.  At most
    // max_batch requests wait admitted (not yet launched) at a time; the
    // plain mode admits one request only when nothing else is admitted.
    Admission admit() {
        Admission a;
        while (!pending_.empty()) {
            if ((int32_t)waiting_.size() >= cfg_.max_batch) break;
            if (cfg_.plain && (!waiting_.empty() || inflight_ > 0 || building_ > 0)) break;
            const Req &r = pending_.front();
            auto pit = parts_.find(r.part_key);
            const bool have = pit != parts_.end();
            const int64_t need = r.stage_bytes + (have ? 0 : r.part_bytes + r.build_bytes);
            if (used_ + need > cfg_.budget) evict_until(used_ + need - cfg_.budget, r.part_key, &a.evict);
            if (used_ + need > cfg_.budget) {
                // every unpinned hierarchy but its own is gone; if nothing
                // else is admitted, running or building, no memory will
                // free up for it later
                const bool alone = waiting_.empty() && inflight_ == 0 && building_ == 0;
                if (alone) {
                    a.rejected.push_back(r.ticket);
                    pending_.pop_front();
                    continue;
                }
                break;
            }
            used_ += need;
            if (!have) {
                Part p;
                p.key = r.part_key;
                p.bytes = r.part_bytes;
                p.build_bytes = r.build_bytes;
                p.pins = 1;
                p.state = PartState::Building;
                lru_.push_back(p.key);
                p.lru = std::prev(lru_.end());
                parts_.emplace(p.key, p);
                resident_ += p.bytes;
                ++building_;
                a.build.push_back(r.part_key);
            } else {
                Part &p = pit->second;
                ++p.pins;
                touch(p);
                if (p.state == PartState::Ready) a.hits.push_back(r.ticket);
            }
            stage_.emplace(r.ticket, r);
            waiting_.push_back(r.ticket);
            a.admitted.push_back(r.ticket);
            pending_.pop_front();
        }
        return a;
    }

    // A build finished: its scratch is released.  With `ok` false the part
    // is marked broken: the server fails its requests instead of launching
    // them, and the part is released once its last request has ended.
    // Returns the part keys to release now: the part itself when no request
    // holds it any more (all of them cancelled while it was being built) and
    // it is not to stay resident.
    std::vector<uint64_t> build_done(uint64_t key, bool ok) {
        std::vector<uint64_t> release;
        auto it = parts_.find(key);
        if (it == parts_.end() || it->second.state != PartState::Building) return release;
        Part &p = it->second;
        used_ -= p.build_bytes;
        p.build_bytes = 0;
        --building_;
        p.state = PartState::Ready;
        if (!ok) broken_.insert_or_assign(key, true);   // released when its pins drop
        if (p.pins == 0 && (!cfg_.keep_resident || broken(key))) {
            release.push_back(key);
            remove_part(it);
        }
        return release;
    }

    bool broken(uint64_t key) const { return broken_.count(key) != 0; }

    // The next launch batch: up to max_batch admitted requests in order, if
    // fewer than max_inflight batches are on the device.
    std::vector<uint64_t> next_batch() {
        std::vector<uint64_t> b;
        if (inflight_ >= cfg_.max_inflight) return b;
        while (!waiting_.empty() && (int32_t)b.size() < cfg_.max_batch) {
            b.push_back(waiting_.front());
            waiting_.pop_front();
        }
        if (!b.empty()) ++inflight_;
        return b;
    }

    // A batch returned by next_batch finished (or was failed without a
    // launch): its working sets are released and its parts unpinned.  With
    // `failed` (the batch's device error word was set) the parts it read are
    // marked broken, so they are dropped once unpinned and rebuilt on their
    // next use rather than trusted again.  Returns the part keys that must be
    // released now (parts not kept resident, broken parts).
    std::vector<uint64_t> batch_done(const std::vector<uint64_t> &tickets, bool failed = false) {
        std::vector<uint64_t> release;
        --inflight_;
        for (uint64_t t : tickets) end_request(t, failed, &release);
        return release;
    }

    // Cancel a request that has not been launched.  A pending one leaves the
    // queue; an admitted one gives back its working set and its pin (part
    // keys to release are appended to *release, as batch_done returns them;
    // a part still being built is released by build_done instead).  Returns
    // false, changing nothing, for a ticket that is unknown or already in a
    // launched batch.
    bool cancel(uint64_t ticket, std::vector<uint64_t> *release) {
        for (auto it = pending_.begin(); it != pending_.end(); ++it)
            if (it->ticket == ticket) {
                pending_.erase(it);
                return true;
            }
        for (auto it = waiting_.begin(); it != waiting_.end(); ++it)
            if (*it == ticket) {
                waiting_.erase(it);
                end_request(ticket, false, release);
                return true;
            }
        return false;
    }

    // Part key of an admitted ticket.
    uint64_t part_of(uint64_t ticket) const {
        auto it = stage_.find(ticket);
        return it == stage_.end() ? 0 : it->second.part_key;
    }

private:
    void touch(Part &p) { lru_.splice(lru_.end(), lru_, p.lru); }

    // An admitted request ended (its batch finished or failed, or it was
    // cancelled before launch): release its working set and its pin.
    void end_request(uint64_t t, bool failed, std::vector<uint64_t> *release) {
        auto sit = stage_.find(t);
        if (sit == stage_.end()) return;
        const Req r = sit->second;
        stage_.erase(sit);
        used_ -= r.stage_bytes;
        auto pit = parts_.find(r.part_key);
        if (pit == parts_.end()) return;
        Part &p = pit->second;
        if (failed) broken_.insert_or_assign(p.key, true);
        --p.pins;
        touch(p);
        if (p.pins == 0 && p.state == PartState::Ready && (!cfg_.keep_resident || broken(p.key))) {
            release->push_back(p.key);
            remove_part(pit);
        }
    }

    void remove_part(std::unordered_map<uint64_t, Part>::iterator it) {
        used_ -= it->second.bytes;
        resident_ -= it->second.bytes;
        lru_.erase(it->second.lru);
        broken_.erase(it->first);
        parts_.erase(it);
    }

    // Evict unpinned, built parts, oldest use first, until `deficit` bytes
    // are freed or none is left; never the part `keep`.
    void evict_until(int64_t deficit, uint64_t keep, std::vector<uint64_t> *out) {
        for (auto li = lru_.begin(); li != lru_.end() && deficit > 0;) {
            const uint64_t k = *li;
            ++li;
            auto it = parts_.find(k);
            if (it == parts_.end() || k == keep) continue;
            if (it->second.pins != 0 || it->second.state != PartState::Ready) continue;
            deficit -= it->second.bytes;
            out->push_back(k);
            remove_part(it);
            ++evictions_;
        }
    }

    Config cfg_;
    std::deque<Req> pending_;
    std::deque<uint64_t> waiting_;
    std::unordered_map<uint64_t, Req> stage_;   // admitted, not yet finished
    std::unordered_map<uint64_t, Part> parts_;
    std::unordered_map<uint64_t, bool> broken_;
    std::list<uint64_t> lru_;
    int64_t used_ = 0, resident_ = 0, evictions_ = 0;
    int32_t inflight_ = 0, building_ = 0;
};

}  // namespace sched
}  // namespace hra

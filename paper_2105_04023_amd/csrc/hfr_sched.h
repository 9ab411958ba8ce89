// Request scheduler of the serving engine, independent of the device: a
// shared queue of requests, a pool of reusable sketches, admission by a
// memory budget, and `slots` worker threads that each run one request at a
// time through a Backend.  The library's serving engine (hfr_server.hip)
// plugs in the HIP path; a CPU test plugs in the oracle.
//
// Scheduling rules:
//  - A free slot takes the oldest queued request it can start now: one whose
//    sketch has an idle resident copy (reuse), or whose key may get another
//    copy built (fewer than max_copies copies, resident or being built) and
//    whose build fits the budget after evicting idle sketches least recently
//    used first.  A request that cannot start is passed over, not waited on,
//    so a busy sketch never blocks requests behind it.
//  - A sketch is used by one request at a time (selection mutates it); it may
//    run on any slot (Backend::adopt moves it to the slot's stream).
//  - A build that cannot fit even with every other sketch evicted fails at
//    once with IM_ERR_OUT_OF_BUDGET and evicts nothing; one that could fit once
//    busy sketches are released waits.
//  - A queued request can be cancelled; a started one cannot.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/im.h"

namespace hfr {
namespace sched {

using Clock = std::chrono::steady_clock;

inline double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// Identity of a reusable sketch: (graph, edge model, p bits, R, hash seed, eps_c bits).
using SketchKey = std::tuple<int32_t, int32_t, uint32_t, int32_t, uint32_t, uint64_t>;

// What a slot does with a request.  Every call is made by the slot's own
// thread without the scheduler's lock, except release() during eviction and
// shutdown (made under the lock, on an idle sketch).
template <class Payload>
struct Backend {
    virtual ~Backend() = default;
    // Builds the sketch of the request on slot `slot`; on IM_OK *handle and *bytes are set.
    virtual im_status build(int slot, const Payload& p, void** handle, size_t* bytes, std::string* err) = 0;
    // Makes a resident sketch (built or last used on another slot) usable from `slot`.
    virtual void adopt(int slot, void* handle) = 0;
    // Runs the request's selection on the sketch; *rebuilds receives its rebuild count.
    virtual im_status select(int slot, void* handle, const Payload& p, int32_t* rebuilds, std::string* err) = 0;
    virtual void release(void* handle) = 0;
};

struct Outcome {
    im_response resp{};
    std::string error;
};

struct Stats {
    int64_t submitted = 0, completed = 0, failed = 0, cancelled = 0;
    int64_t sketches_built = 0, evictions = 0, resident_sketches = 0;
    size_t sketch_bytes = 0;
};

template <class Payload>
class Scheduler {
   public:
    // budget: bytes for every sketch together (0 = no bound); need_fixed: bytes already taken (graphs).
    Scheduler(int slots, size_t budget, Backend<Payload>* be, int max_copies = 2)
        : nslots_(slots), budget_(budget), be_(be), max_copies_(std::max(1, max_copies)) {}
    ~Scheduler() { stop(); }

    void set_fixed_bytes(size_t b) {
        std::lock_guard<std::mutex> lk(mu_);
        fixed_ = b;
    }

    void start() {
        std::lock_guard<std::mutex> lk(mu_);
        if (running_) return;
        running_ = true;
        for (int i = 0; i < nslots_; ++i) threads_.emplace_back([this, i] { slot_main(i); });
    }

    // Queues a request whose sketch (of key `key`) needs `need` bytes at its peak; returns its ticket.
    int64_t submit(const SketchKey& key, size_t need, const Payload& p) {
        auto r = std::make_shared<Req>();
        r->key = key;
        r->need = need;
        r->p = p;
        {
            std::lock_guard<std::mutex> lk(mu_);
            r->ticket = next_ticket_++;
            r->t_submit = Clock::now();
            queue_.push_back(r);
            reqs_[r->ticket] = r;
            stats_.submitted += 1;
        }
        cv_work_.notify_all();
        return r->ticket;
    }

    // Removes a request that has not started: IM_OK, or IM_ERR_STATE if it started, finished or is unknown.
    im_status cancel(int64_t ticket) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = reqs_.find(ticket);
            if (it == reqs_.end()) return IM_ERR_STATE;
            auto r = it->second;
            if (r->started || r->done) return IM_ERR_STATE;
            queue_.erase(std::find(queue_.begin(), queue_.end(), r));
            r->out.resp.status = IM_ERR_STATE;
            r->out.resp.slot = -1;
            r->out.error = "request cancelled before it started";
            r->t_start = r->t_end = Clock::now();
            finish_locked(*r);
            stats_.cancelled += 1;
        }
        cv_done_.notify_all();
        return IM_OK;
    }

    // Blocks until the request is done; false if the ticket is unknown.
    bool wait(int64_t ticket, Outcome* out) {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return false;
        auto r = it->second;
        cv_done_.wait(lk, [&] { return r->done; });
        reqs_.erase(ticket);
        *out = r->out;
        return true;
    }

    Stats stats() {
        std::lock_guard<std::mutex> lk(mu_);
        Stats s = stats_;
        s.resident_sketches = 0;
        for (auto& kv : cache_) s.resident_sketches += (int64_t)kv.second.size();
        s.sketch_bytes = resident_;
        return s;
    }

    // Finishes every queued request, joins the slots and releases every sketch.
    void stop() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stopping_ = true;
        }
        cv_work_.notify_all();
        for (auto& t : threads_)
            if (t.joinable()) t.join();
        threads_.clear();
        std::lock_guard<std::mutex> lk(mu_);
        for (auto& kv : cache_)
            for (auto& e : kv.second) be_->release(e.h);
        cache_.clear();
        resident_ = 0;
    }

   private:
    struct Entry {
        void* h = nullptr;
        size_t bytes = 0;
        uint64_t last_use = 0;
        bool busy = false;
    };
    struct Req {
        int64_t ticket = 0;
        SketchKey key;
        size_t need = 0;
        Payload p;
        Clock::time_point t_submit, t_start, t_end;
        Outcome out;
        bool started = false, done = false;
    };
    // A request taken by a slot: reuse of `entry` (index into cache_[key]) or a build.
    struct Pick {
        std::shared_ptr<Req> r;
        bool build = false;
        void* h = nullptr;
    };

    void finish_locked(Req& r) {
        r.done = true;
        r.out.resp.queue_ms = ms_between(r.t_submit, r.t_start);
        r.out.resp.latency_ms = ms_between(r.t_submit, r.t_end);
        stats_.completed += 1;
        if (r.out.resp.status != IM_OK) stats_.failed += 1;
    }

    bool busy_or_building() const {
        if (reserved_ > 0) return true;
        for (auto& kv : cache_)
            for (auto& e : kv.second)
                if (e.busy) return true;
        return false;
    }

    // Evicts the least recently used idle sketch; false if none is idle.
    bool evict_one() {
        auto best_k = cache_.end();
        size_t best_i = 0;
        for (auto it = cache_.begin(); it != cache_.end(); ++it)
            for (size_t i = 0; i < it->second.size(); ++i) {
                const Entry& e = it->second[i];
                if (e.busy) continue;
                if (best_k == cache_.end() || e.last_use < best_k->second[best_i].last_use) {
                    best_k = it;
                    best_i = i;
                }
            }
        if (best_k == cache_.end()) return false;
        Entry e = best_k->second[best_i];
        best_k->second.erase(best_k->second.begin() + (ptrdiff_t)best_i);
        if (best_k->second.empty()) cache_.erase(best_k);
        resident_ -= e.bytes;
        stats_.evictions += 1;
        be_->release(e.h);
        return true;
    }

    // Under the lock: the oldest queued request that can start now (see the rules above).
    bool pick(Pick* out) {
        for (auto it = queue_.begin(); it != queue_.end();) {
            auto r = *it;
            auto cit = cache_.find(r->key);
            if (cit != cache_.end()) {
                for (auto& e : cit->second)
                    if (!e.busy) {
                        e.busy = true;
                        e.last_use = ++clock_;
                        out->r = r;
                        out->build = false;
                        out->h = e.h;
                        queue_.erase(it);
                        return true;
                    }
            }
            const int copies = (cit != cache_.end() ? (int)cit->second.size() : 0) + building_[r->key];
            if (copies >= max_copies_) {
                ++it;  // wait for a copy to be released
                continue;
            }
            if (budget_) {
                if (fixed_ + r->need > budget_) {  // cannot fit even with every sketch evicted
                    r->started = true;
                    r->t_start = r->t_end = Clock::now();
                    r->out.resp.status = IM_ERR_OUT_OF_BUDGET;
                    r->out.resp.slot = -1;
                    r->out.error = "the request's sketch exceeds the memory budget";
                    finish_locked(*r);
                    it = queue_.erase(it);
                    cv_done_.notify_all();
                    continue;
                }
                while (fixed_ + resident_ + reserved_ + r->need > budget_ && evict_one()) {
                }
                if (fixed_ + resident_ + reserved_ + r->need > budget_) {
                    if (copies > 0 || busy_or_building()) {
                        ++it;  // fits once busy sketches are released
                        continue;
                    }
                    r->started = true;
                    r->t_start = r->t_end = Clock::now();
                    r->out.resp.status = IM_ERR_OUT_OF_BUDGET;
                    r->out.resp.slot = -1;
                    r->out.error = "the request's sketch does not fit the memory budget";
                    finish_locked(*r);
                    it = queue_.erase(it);
                    cv_done_.notify_all();
                    continue;
                }
            }
            reserved_ += r->need;
            building_[r->key] += 1;
            out->r = r;
            out->build = true;
            out->h = nullptr;
            queue_.erase(it);
            return true;
        }
        return false;
    }

    void slot_main(int slot) {
        while (true) {
            Pick pk;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_work_.wait(lk, [&] { return pick(&pk) || (stopping_ && queue_.empty()); });
                if (!pk.r) return;  // stopping and drained
                pk.r->started = true;
                pk.r->t_start = Clock::now();
            }
            Req& r = *pk.r;
            im_status st = IM_OK;
            void* h = pk.h;
            size_t bytes = 0;
            double build_ms = 0.0, select_ms = 0.0;
            int32_t rebuilds = 0;
            std::string err;
            if (pk.build) {
                const auto t0 = Clock::now();
                st = be_->build(slot, r.p, &h, &bytes, &err);
                build_ms = ms_between(t0, Clock::now());
            } else {
                be_->adopt(slot, h);
            }
            if (st == IM_OK) {
                const auto t0 = Clock::now();
                st = be_->select(slot, h, r.p, &rebuilds, &err);
                select_ms = ms_between(t0, Clock::now());
            }
            {
                std::lock_guard<std::mutex> lk(mu_);
                if (pk.build) {
                    reserved_ -= r.need;
                    building_[r.key] -= 1;
                    if (h) {
                        Entry e;
                        e.h = h;
                        e.bytes = bytes;
                        e.last_use = ++clock_;
                        cache_[r.key].push_back(e);
                        resident_ += bytes;
                        stats_.sketches_built += 1;
                    }
                } else {
                    for (auto& e : cache_[r.key])
                        if (e.h == h) {
                            e.busy = false;
                            e.last_use = ++clock_;
                        }
                }
                r.t_end = Clock::now();
                r.out.resp.status = st;
                r.out.resp.slot = slot;
                r.out.resp.sketch_reused = pk.build ? 0 : 1;
                r.out.resp.rebuilds = rebuilds;
                r.out.resp.build_ms = build_ms;
                r.out.resp.select_ms = select_ms;
                r.out.error = err;
                finish_locked(r);
            }
            cv_done_.notify_all();
            cv_work_.notify_all();  // a released sketch or budget may let queued requests start
        }
    }

    const int nslots_;
    const size_t budget_;
    Backend<Payload>* be_;
    const int max_copies_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::vector<std::thread> threads_;
    std::deque<std::shared_ptr<Req>> queue_;
    std::map<int64_t, std::shared_ptr<Req>> reqs_;
    std::map<SketchKey, std::vector<Entry>> cache_;
    std::map<SketchKey, int> building_;
    size_t fixed_ = 0, resident_ = 0, reserved_ = 0;
    uint64_t clock_ = 0;
    int64_t next_ticket_ = 1;
    bool running_ = false, stopping_ = false;
    Stats stats_;
};

}  // namespace sched
}  // namespace hfr

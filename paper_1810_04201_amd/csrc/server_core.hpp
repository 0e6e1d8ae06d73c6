// Host-only core of the solve server: the HBM ledger that decides admission
// and which idle gauge forms to release, and the ticket book that the client
// threads (submit, poll) share with the scheduler thread.  Nothing here calls
// HIP, so a plain C++ build runs it under the address, undefined-behaviour
// and thread sanitizers (tests/server_core_check.cpp).
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

namespace wd {

// Gauge forms a lattice may hold beside its float64 master links (18 reals,
// plus 12 where kept): the full-lattice float32 and binary16 forms and the
// even-odd halves of the three precisions.  Each is built from the master on
// first use, so it can be released and later rebuilt bit for bit.
enum DerivedForm {
    kFormF32 = 0,
    kFormF16 = 1,
    kFormEo64 = 2,
    kFormEo32 = 3,
    kFormEo16 = 4,
    kNumDerived = 5
};

// What a lattice holds now, as the ledger last saw it.
struct LedgerLat {
    size_t master = 0;                 // float64 links
    size_t derived[kNumDerived] = {};  // bytes of each derived form (0: not built)
    int running = 0;                   // admitted requests on the lattice
    uint64_t last_use = 0;             // admission stamp (least recently used first)
};

// A request's cost: its workspace, and the bytes of each derived form its
// solve reads (0: not read).
struct Need {
    size_t workspace = 0;
    size_t form_bytes[kNumDerived] = {};
};

struct Eviction {
    const void *lat;
    int form;
};

// HBM accounting of a server.  Charged: the workspace of every running
// request; every derived form resident on a lattice the ledger knows (the
// server's requests built it, and it stays allocated after they retire); the
// master links of lattices with running requests.  Admission never lets the
// charge exceed the budget: when a request would not fit, derived forms of
// lattices without running requests are released first (least recently used
// lattice first), and if it still does not fit the request waits.
class Ledger {
  public:
    explicit Ledger(size_t budget) : budget_(budget) {}

    static size_t charge(const LedgerLat &l) {
        size_t b = l.running > 0 ? l.master : 0;
        for (int f = 0; f < kNumDerived; ++f) b += l.derived[f];
        return b;
    }

    size_t budget() const { return budget_; }
    size_t peak() const { return peak_; }
    size_t used() const {
        size_t b = workspace_;
        for (const auto &kv : lats_) b += charge(kv.second);
        return b;
    }
    const LedgerLat *find(const void *lat) const {
        auto it = lats_.find(lat);
        return it == lats_.end() ? nullptr : &it->second;
    }

    // Record what a lattice holds now (read from the lattice itself).
    void observe(const void *lat, size_t master, const size_t derived[kNumDerived]) {
        LedgerLat &l = lats_[lat];
        l.master = master;
        for (int f = 0; f < kNumDerived; ++f) l.derived[f] = derived[f];
        note_peak();
    }

    // Bytes admitting `need` on `lat` adds to the charge.
    size_t extra(const void *lat, const Need &need) const {
        const LedgerLat *l = find(lat);
        const LedgerLat none{};
        if (!l) l = &none;
        size_t b = need.workspace + (l->running > 0 ? 0 : l->master);
        for (int f = 0; f < kNumDerived; ++f)
            if (need.form_bytes[f] && !l->derived[f]) b += need.form_bytes[f];
        return b;
    }

    // Whether `need` on `lat` can be admitted now.  If only after releasing
    // derived forms of lattices without running requests, *evict lists them:
    // other lattices least recently used first, then forms of lat itself that
    // the request does not read.  Never a form of a lattice with running
    // requests.  Returns false (and lists nothing) if it cannot fit yet.
    bool plan(const void *lat, const Need &need, std::vector<Eviction> *evict) const {
        evict->clear();
        const size_t cur = used(), add = extra(lat, need);
        if (add > budget_) return false;
        if (cur + add <= budget_) return true;
        std::vector<std::pair<uint64_t, const void *>> idle;
        for (const auto &kv : lats_)
            if (kv.first != lat && kv.second.running == 0) idle.push_back({kv.second.last_use, kv.first});
        std::sort(idle.begin(), idle.end());
        size_t freed = 0;
        auto take = [&](const void *k, const LedgerLat &l, bool own) {
            for (int f = 0; f < kNumDerived && cur + add - freed > budget_; ++f) {
                if (!l.derived[f] || (own && need.form_bytes[f])) continue;
                evict->push_back({k, f});
                freed += l.derived[f];
            }
        };
        for (const auto &p : idle) take(p.second, lats_.at(p.second), false);
        const LedgerLat *self = find(lat);
        if (self && self->running == 0 && cur + add - freed > budget_) take(lat, *self, true);
        if (cur + add - freed <= budget_) return true;
        evict->clear();
        return false;
    }

    // The lattices the ledger knows.
    void lattices(std::vector<const void *> *out) const {
        out->clear();
        for (const auto &kv : lats_) out->push_back(kv.first);
    }

    // The lattice is being destroyed: its forms go with it.
    void forget(const void *lat) { lats_.erase(lat); }

    // A planned release was carried out.
    void evicted(const void *lat, int form) {
        auto it = lats_.find(lat);
        if (it != lats_.end()) it->second.derived[form] = 0;
    }

    // Charge an admitted request (its forms are counted as built).
    void admit(const void *lat, const Need &need) {
        LedgerLat &l = lats_[lat];
        l.running += 1;
        l.last_use = ++stamp_;
        for (int f = 0; f < kNumDerived; ++f)
            if (need.form_bytes[f] && !l.derived[f]) l.derived[f] = need.form_bytes[f];
        workspace_ += need.workspace;
        note_peak();
    }

    // A request retired: its workspace is released; the lattice's master
    // links stop being charged when its last request goes.
    void retire(const void *lat, size_t workspace) {
        workspace_ -= workspace;
        auto it = lats_.find(lat);
        if (it != lats_.end()) it->second.running -= 1;
    }

  private:
    void note_peak() { peak_ = std::max(peak_, used()); }

    size_t budget_;
    size_t workspace_ = 0;
    size_t peak_ = 0;
    uint64_t stamp_ = 0;
    std::map<const void *, LedgerLat> lats_;
};

// Requests by ticket, shared by the client threads and the scheduler.  Rec
// must have the members `uint64_t ticket` and `bool done`, which the book
// reads and writes under its lock only.  A submitted record waits in the
// inbox until the scheduler takes it; the scheduler publishes its result
// under the lock.  The `keep` most recently finished records stay pollable;
// older ones are forgotten (polling them reports an unknown ticket), so the
// book does not grow with the number of requests served.
template <class Rec>
class TicketBook {
  public:
    explicit TicketBook(size_t keep) : keep_(keep) {}

    // Queue a record; returns its ticket, or 0 once stopping.
    uint64_t submit(const std::shared_ptr<Rec> &r) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (stopping_) return 0;
            r->ticket = next_++;
            r->done = false;
            recs_[r->ticket] = r;
            inbox_.push_back(r);
        }
        cv_.notify_one();
        return r->ticket;
    }

    // Scheduler: append the queued records to *out, waiting up to `wait` when
    // there are none and `idle` is set.  Returns false once stopping with an
    // empty inbox.
    bool take(std::vector<std::shared_ptr<Rec>> *out, bool idle, std::chrono::microseconds wait) {
        std::unique_lock<std::mutex> lk(mu_);
        // a system_clock deadline waits through pthread_cond_timedwait, which
        // the thread sanitizer follows (its clockwait form it does not)
        if (idle && inbox_.empty() && !stopping_)
            cv_.wait_until(lk, std::chrono::system_clock::now() + wait);
        while (!inbox_.empty()) {
            out->push_back(inbox_.front());
            inbox_.pop_front();
        }
        return !stopping_;
    }

    // Scheduler: fill(r) under the lock, then mark r done.
    template <class Fn>
    void publish(const std::shared_ptr<Rec> &r, Fn fill) {
        std::lock_guard<std::mutex> lk(mu_);
        fill(*r);
        r->done = true;
        finished_.push_back(r->ticket);
        while (finished_.size() > keep_) {
            recs_.erase(finished_.front());
            finished_.pop_front();
        }
    }

    // -1: unknown ticket; 0: not finished; 1: finished, read(r) called
    // under the lock.
    template <class Fn>
    int poll(uint64_t ticket, Fn read) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = recs_.find(ticket);
        if (it == recs_.end()) return -1;
        if (!it->second->done) return 0;
        read(*it->second);
        return 1;
    }

    void stop() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stopping_ = true;
        }
        cv_.notify_all();
    }

    size_t size() {
        std::lock_guard<std::mutex> lk(mu_);
        return recs_.size();
    }

  private:
    std::mutex mu_;
    std::condition_variable cv_;
    bool stopping_ = false;
    uint64_t next_ = 1;
    size_t keep_;
    std::deque<std::shared_ptr<Rec>> inbox_;
    std::map<uint64_t, std::shared_ptr<Rec>> recs_;
    std::deque<uint64_t> finished_;
};

}  // namespace wd

// Continuous-batching solve server.
//
// The problem statement of Sec. 2.3 is a stream of solves: gauge fields stay
// resident while sources change, or a new field arrives with new sources.
// wd_submit queues a request and returns a ticket at once.  A scheduler
// thread admits queued requests in arrival order while the HBM budget and a
// free slot allow it, gives each admitted request its own HIP stream, and
// then round-robins over the running requests, enqueueing their next batch
// of CG iterations and retiring those whose device status says they are done.
// Requests therefore join and leave while others iterate, and their kernels
// overlap on the GPU.  Each request owns its workspace and reductions, so its
// result is bitwise the same alone or in any mix.
//
// HBM accounting: a request is charged its solver workspace; a lattice's
// packed gauge forms are charged once while any admitted request uses them.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <map>
#include <memory>
#include <thread>

#include "runtime.hpp"

namespace wd {

struct Request {
    uint64_t ticket = 0;
    wd_lattice *lat = nullptr;
    wd_solve_params p{};
    const double *b = nullptr;
    double *x = nullptr;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int state = 0;  // 0 queued, 1 running, 2 done
    int rc = WD_PENDING;
    std::vector<wd_solve_info> info;
    std::unique_ptr<Solve> solve;
    size_t charged = 0;
    int slot = -1;
};

}  // namespace wd

struct wd_server {
    wd_server_config cfg{};
    int device = 0;
    std::thread thr;
    std::mutex mu;
    std::condition_variable cv;
    bool stopping = false;
    uint64_t next_ticket = 1;
    std::deque<uint64_t> queue;
    std::map<uint64_t, std::shared_ptr<wd::Request>> reqs;
    std::vector<std::shared_ptr<wd::Request>> active;
    std::vector<hipStream_t> streams;
    std::vector<wd::SlotRes> slots;
    std::vector<int> slot_busy;
    // per lattice: admitted requests using it and the gauge forms charged
    struct LatUse {
        int users = 0;
        size_t charged = 0;
        bool form[3] = {false, false, false};  // full-lattice forms charged
        bool eo[3] = {false, false, false};    // even-odd half forms charged
    };
    std::map<wd_lattice *, LatUse> lat_use;
    size_t used = 0, peak = 0;
    double t_start = 0, t_last = 0;
    std::vector<double> latencies;
};

namespace wd {

static size_t request_bytes(const wd_lattice *lat, const wd_solve_params &p) {
    return Solve::footprint(lat, p);
}

static bool eo_request(const wd_solve_params &p) { return (p.form & WD_SOLVE_EVEN_ODD) != 0; }

// gauge bytes a request needs on its lattice: the float64 tiles (always
// there once the gauge is set), plus the forms its solve reads
static size_t gauge_need(const wd_lattice *lat, const wd_solve_params &p, const bool form[3],
                         const bool eo[3]) {
    const int V = lat->g.V, prec = p.prec_inner;
    // the float64 forms (F64-18, and F64-12 for special unitary links)
    size_t b = form[WD_F64] ? 0
                            : gauge_bytes(WD_F64, V) +
                                  (lat->gauge12 ? gauge_bytes(kLinkF64R12, V) : 0);
    if (eo_request(p)) {
        if (!eo[WD_F64]) b += 2 * gauge_bytes(lat->gauge12 ? kLinkF64R12 : WD_F64, V / 2);
        if (prec != WD_F64 && !eo[prec]) b += 2 * gauge_bytes(prec, V / 2);
    } else if (prec != WD_F64 && !form[prec]) {
        b += gauge_bytes(prec, V);
    }
    return b;
}

static size_t lattice_gauge_charge(const wd_lattice *lat, const wd_solve_params &p) {
    const bool none[3] = {false, false, false};
    return gauge_need(lat, p, none, none);
}

// extra gauge bytes admitting request p on lat would add
static size_t gauge_extra(wd_server *s, wd_lattice *lat, const wd_solve_params &p) {
    auto it = s->lat_use.find(lat);
    if (it == s->lat_use.end()) return lattice_gauge_charge(lat, p);
    return gauge_need(lat, p, it->second.form, it->second.eo);
}

// have_info: the solve ran to completion and its device status is valid
static void finish_request(wd_server *s, const std::shared_ptr<Request> &r, int rc,
                           bool have_info) {
    r->t_done = now_seconds();
    r->rc = rc;
    r->info.assign(r->p.nrhs, wd_solve_info{});
    if (have_info) r->solve->info(r->info.data());
    for (auto &i : r->info) {
        i.seconds = r->t_done - r->t_submit;
        i.queued_seconds = r->t_admit > 0 ? r->t_admit - r->t_submit : i.seconds;
        if (!have_info) i.status = rc;
    }
    r->solve.reset();  // stream-ordered release of the workspace
    s->used -= r->charged;
    auto &lu = s->lat_use[r->lat];
    if (--lu.users == 0) {
        s->used -= lu.charged;
        s->lat_use.erase(r->lat);
    }
    r->lat->users.fetch_sub(1);
    if (r->slot >= 0) s->slot_busy[r->slot] = 0;
    r->state = 2;
    s->latencies.push_back(r->t_done - r->t_submit);
    s->t_last = r->t_done;
}

static void scheduler(wd_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // admit in arrival order while budget and slots allow
        while (!s->queue.empty() && (int)s->active.size() < s->cfg.max_active) {
            auto r = s->reqs[s->queue.front()];
            const size_t extra = gauge_extra(s, r->lat, r->p);
            const size_t need = request_bytes(r->lat, r->p) + extra;
            if (s->used + need > s->cfg.hbm_budget_bytes) break;  // head of line waits
            s->queue.pop_front();
            int slot = 0;
            while (s->slot_busy[slot]) ++slot;
            s->slot_busy[slot] = 1;
            r->slot = slot;
            r->charged = request_bytes(r->lat, r->p);
            auto &lu = s->lat_use[r->lat];
            lu.users += 1;
            lu.charged += extra;
            lu.form[WD_F64] = true;
            if (eo_request(r->p)) {
                lu.eo[WD_F64] = true;
                lu.eo[r->p.prec_inner] = true;
            } else {
                lu.form[r->p.prec_inner] = true;
            }
            s->used += r->charged + extra;
            s->peak = std::max(s->peak, s->used);
            r->t_admit = now_seconds();
            r->state = 1;
            r->solve.reset(new Solve(r->lat, r->p, r->b, r->x));
            int rc = r->solve->setup(s->streams[slot], &s->slots[slot]);
            if (rc == WD_OK && s->cfg.chunk_iters > 0) r->solve->set_chunk(s->cfg.chunk_iters);
            if (rc == WD_OK) rc = r->solve->start();
            if (rc != WD_OK) {
                finish_request(s, r, rc, false);
                continue;
            }
            s->active.push_back(r);
        }
        if (s->active.empty()) {
            if (s->stopping && s->queue.empty()) break;
            s->cv.wait_for(lk, std::chrono::milliseconds(2));
            continue;
        }
        // one non-blocking turn over the running requests
        bool progressed = false;
        for (size_t k = 0; k < s->active.size();) {
            auto r = s->active[k];
            const int a = r->solve->advance(false);
            if (a == 0) {
                ++k;
                continue;
            }
            progressed = true;
            if (a < 0)
                finish_request(s, r, a, false);
            else
                finish_request(s, r, r->solve->result(), true);
            s->active.erase(s->active.begin() + k);
        }
        if (!progressed) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(50));
            lk.lock();
        }
    }
}

}  // namespace wd

using namespace wd;

extern "C" {

int wd_server_create(const wd_server_config *cfg, wd_server **out) {
    if (!cfg || !out) return fail(WD_ERR_ARG, "null argument");
    if (cfg->hbm_budget_bytes == 0) return fail(WD_ERR_ARG, "hbm_budget_bytes must be > 0");
    wd_server *s = new (std::nothrow) wd_server();
    if (!s) return fail(WD_ERR_NOMEM, "host allocation failed");
    s->cfg = *cfg;
    if (s->cfg.max_active <= 0) s->cfg.max_active = 8;
    if (s->cfg.max_active > 64) s->cfg.max_active = 64;
    (void)hipGetDevice(&s->device);
    s->streams.assign(s->cfg.max_active, nullptr);
    s->slots.assign(s->cfg.max_active, SlotRes{});
    s->slot_busy.assign(s->cfg.max_active, 0);
    for (int i = 0; i < s->cfg.max_active; ++i) {
        if (hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) != hipSuccess) {
            for (int j = 0; j < i; ++j) {
                (void)hipStreamDestroy(s->streams[j]);
                s->slots[j].destroy();
            }
            delete s;
            return fail(WD_ERR_HIP, "hipStreamCreate failed");
        }
        int rc = s->slots[i].create();
        if (rc) {
            for (int j = 0; j <= i; ++j) {
                (void)hipStreamDestroy(s->streams[j]);
                s->slots[j].destroy();
            }
            delete s;
            return rc;
        }
    }
    s->t_start = now_seconds();
    s->thr = std::thread(scheduler, s);
    *out = s;
    return WD_OK;
}

int wd_submit(wd_server *s, wd_lattice *lat, const wd_solve_params *p, const double *b, double *x,
              uint64_t *ticket) {
    if (!s || !ticket) return fail(WD_ERR_ARG, "null argument");
    int rc = Solve::validate(lat, p);
    if (rc) return rc;
    if (!b || !x) return fail(WD_ERR_ARG, "null argument");
    if (b == x) return fail(WD_ERR_ARG, "b and x must not overlap");
    const size_t need = request_bytes(lat, *p) + lattice_gauge_charge(lat, *p);
    if (need > s->cfg.hbm_budget_bytes)
        return fail(WD_ERR_NOMEM, "request needs %zu bytes, more than the whole budget (%zu)",
                    need, s->cfg.hbm_budget_bytes);
    auto r = std::make_shared<Request>();
    r->lat = lat;
    r->p = *p;
    r->b = b;
    r->x = x;
    r->t_submit = now_seconds();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) return fail(WD_ERR_STATE, "server is shutting down");
        r->ticket = s->next_ticket++;
        lat->users.fetch_add(1);
        s->reqs[r->ticket] = r;
        s->queue.push_back(r->ticket);
        *ticket = r->ticket;
    }
    s->cv.notify_one();
    return WD_OK;
}

int wd_poll(wd_server *s, uint64_t ticket, wd_solve_info *info) {
    if (!s) return fail(WD_ERR_ARG, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(WD_ERR_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    const auto &r = it->second;
    if (r->state != 2) return WD_PENDING;
    if (info)
        for (int k = 0; k < r->p.nrhs; ++k) info[k] = r->info[k];
    if (r->rc < 0) fail(r->rc, "request %llu failed", (unsigned long long)ticket);
    return r->rc;
}

int wd_server_stats(wd_server *s, double *solves_per_s, double *p50_s, double *p99_s) {
    if (!s || !solves_per_s || !p50_s || !p99_s) return fail(WD_ERR_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> l = s->latencies;
    const size_t n = l.size();
    const double span = (s->t_last > s->t_start) ? s->t_last - s->t_start : 0.0;
    *solves_per_s = span > 0 ? (double)n / span : 0.0;
    if (n == 0) {
        *p50_s = *p99_s = 0.0;
        return WD_OK;
    }
    std::sort(l.begin(), l.end());
    // nearest rank: the ceil(q n)-th smallest
    auto rank = [&](double q) {
        size_t k = (size_t)std::ceil(q * (double)n);
        if (k < 1) k = 1;
        if (k > n) k = n;
        return l[k - 1];
    };
    *p50_s = rank(0.50);
    *p99_s = rank(0.99);
    return WD_OK;
}

int wd_server_peak_bytes(wd_server *s, size_t *bytes) {
    if (!s || !bytes) return fail(WD_ERR_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *bytes = s->peak;
    return WD_OK;
}

int wd_server_destroy(wd_server *s) {
    if (!s) return fail(WD_ERR_ARG, "null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv.notify_one();
    if (s->thr.joinable()) s->thr.join();
    for (size_t i = 0; i < s->streams.size(); ++i) {
        (void)hipStreamSynchronize(s->streams[i]);
        (void)hipStreamDestroy(s->streams[i]);
        s->slots[i].destroy();
    }
    delete s;
    return WD_OK;
}

}  // extern "C"

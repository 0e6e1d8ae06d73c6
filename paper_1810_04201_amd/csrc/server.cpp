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
// Locking: client threads (wd_submit, wd_poll) meet the scheduler only in the
// ticket book, whose lock is held for a queue push, a result copy or a map
// lookup.  Admission, kernel enqueues, graph captures and gauge-form builds
// run without it, so clients never wait behind device work.  The HBM ledger
// has a lock of its own, shared with wd_destroy_lattice (a destroyed lattice
// leaves every server's ledger before its forms are freed).
//
// HBM accounting (Ledger): running requests' workspaces, the float64 links
// of lattices with running requests, and every derived gauge form (float32,
// binary16, even-odd halves) resident on a lattice the server has used, for
// as long as it stays allocated.  A request that does not fit makes the
// server release derived forms of lattices without running requests; they
// are rebuilt on next use.
#include <algorithm>
#include <chrono>
#include <memory>
#include <set>
#include <thread>

#include "runtime.hpp"

namespace wd {

struct Request {
    // set by wd_submit before the ticket is issued, read-only afterwards
    wd_lattice *lat = nullptr;
    wd_solve_params p{};
    const double *b = nullptr;
    double *x = nullptr;
    double t_submit = 0;
    // ticket book (under its lock)
    uint64_t ticket = 0;
    bool done = false;
    int rc = WD_PENDING;
    std::vector<wd_solve_info> info;
    // scheduler thread only
    std::unique_ptr<Solve> solve;
    Need need{};
    double t_admit = 0;
    int slot = -1;
};

// finished tickets that stay pollable
constexpr size_t kKeepFinished = 4096;

}  // namespace wd

struct wd_server {
    wd_server_config cfg{};
    int device = 0;
    std::thread thr;
    wd::TicketBook<wd::Request> book{wd::kKeepFinished};
    // scheduler thread only
    std::deque<std::shared_ptr<wd::Request>> queue;
    std::vector<std::shared_ptr<wd::Request>> active;
    std::vector<hipStream_t> streams;
    bool own_streams = true;
    std::vector<wd::SlotRes> slots;
    std::vector<int> slot_busy;
    // HBM ledger (ledger_mu)
    std::mutex ledger_mu;
    wd::Ledger ledger{0};
    // statistics (stat_mu)
    std::mutex stat_mu;
    double t_start = 0, t_last = 0;
    std::vector<double> latencies;
};

namespace wd {

// every live server, so that a destroyed lattice can leave their ledgers
static std::mutex g_servers_mu;
static std::set<wd_server *> g_servers;

static Need request_need(const wd_lattice *lat, const wd_solve_params &p) {
    Need n{};
    n.workspace = Solve::footprint(lat, p);
    solve_forms(lat, p, n.form_bytes);
    return n;
}

// re-read what every lattice in the ledger holds now (ledger_mu held)
static void refresh_ledger(wd_server *s, wd_lattice *also) {
    std::vector<const void *> keys;
    s->ledger.lattices(&keys);
    if (also && std::find(keys.begin(), keys.end(), (const void *)also) == keys.end())
        keys.push_back(also);
    for (const void *k : keys) {
        size_t master = 0, derived[kNumDerived];
        lattice_forms((wd_lattice *)k, &master, derived);
        s->ledger.observe(k, master, derived);
    }
}

// have_info: the solve ran to completion and its device status is valid
static void finish_request(wd_server *s, const std::shared_ptr<Request> &r, int rc,
                           bool have_info) {
    const double t_done = now_seconds();
    std::vector<wd_solve_info> info(r->p.nrhs, wd_solve_info{});
    if (have_info) r->solve->info(info.data());
    for (auto &i : info) {
        i.seconds = t_done - r->t_submit;
        i.queued_seconds = r->t_admit > 0 ? r->t_admit - r->t_submit : i.seconds;
        if (!have_info) i.status = rc;
    }
    r->solve.reset();  // stream-ordered release of the workspace
    {
        std::lock_guard<std::mutex> lk(s->ledger_mu);
        if (r->t_admit > 0) s->ledger.retire(r->lat, r->need.workspace);
    }
    if (r->slot >= 0) s->slot_busy[r->slot] = 0;
    {
        std::lock_guard<std::mutex> lk(s->stat_mu);
        s->latencies.push_back(t_done - r->t_submit);
        s->t_last = t_done;
    }
    // the lattice is free for the caller once the result is visible (and
    // may then be destroyed: nothing below touches it)
    r->lat->users.fetch_sub(1);
    s->book.publish(r, [&](Request &q) {
        q.rc = rc;
        q.info = std::move(info);
    });
}

// admit queued requests in arrival order while the budget and the slots allow
static void admit(wd_server *s) {
    while (!s->queue.empty() && (int)s->active.size() < s->cfg.max_active) {
        auto r = s->queue.front();
        {
            std::lock_guard<std::mutex> lk(s->ledger_mu);
            refresh_ledger(s, r->lat);
            std::vector<Eviction> ev;
            if (!s->ledger.plan(r->lat, r->need, &ev)) return;  // head of line waits
            for (const Eviction &e : ev) {
                release_form((wd_lattice *)e.lat, e.form);
                s->ledger.evicted(e.lat, e.form);
            }
            s->ledger.admit(r->lat, r->need);
        }
        s->queue.pop_front();
        int slot = 0;
        while (s->slot_busy[slot]) ++slot;
        s->slot_busy[slot] = 1;
        r->slot = slot;
        r->t_admit = now_seconds();
        r->solve.reset(new Solve(r->lat, r->p, r->b, r->x));
        int rc = r->solve->setup(s->streams[slot], &s->slots[slot]);
        if (rc == WD_OK && s->cfg.chunk_iters > 0) r->solve->set_chunk(s->cfg.chunk_iters);
        if (rc == WD_OK) rc = r->solve->start();
        {
            // the forms the setup built, as the lattice holds them
            std::lock_guard<std::mutex> lk(s->ledger_mu);
            refresh_ledger(s, nullptr);
        }
        if (rc != WD_OK) {
            finish_request(s, r, rc, false);
            continue;
        }
        s->active.push_back(r);
    }
}

static void scheduler(wd_server *s) {
    (void)hipSetDevice(s->device);
    for (;;) {
        std::vector<std::shared_ptr<Request>> fresh;
        const bool idle = s->active.empty();
        const bool open = s->book.take(&fresh, idle, std::chrono::milliseconds(2));
        for (auto &r : fresh) s->queue.push_back(r);
        if (!open && s->queue.empty() && s->active.empty()) break;
        admit(s);
        if (s->active.empty()) continue;
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
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

void servers_forget(wd_lattice *lat) {
    std::lock_guard<std::mutex> g(g_servers_mu);
    for (wd_server *s : g_servers) {
        std::lock_guard<std::mutex> lk(s->ledger_mu);
        s->ledger.forget(lat);
    }
}

}  // namespace wd

using namespace wd;

extern "C" {

int wd_server_create(const wd_server_config *cfg, wd_server **out) {
    if (!cfg || !out) return fail(WD_ERR_ARG, "null argument");
    if (cfg->hbm_budget_bytes == 0) return fail(WD_ERR_ARG, "hbm_budget_bytes must be > 0");
    if (cfg->n_streams < 0 || (cfg->n_streams > 0 && !cfg->streams))
        return fail(WD_ERR_ARG, "n_streams = %d with %s stream array", (int)cfg->n_streams,
                    cfg->streams ? "a" : "no");
    if (cfg->n_streams > 64) return fail(WD_ERR_ARG, "at most 64 caller streams");
    wd_server *s = new (std::nothrow) wd_server();
    if (!s) return fail(WD_ERR_NOMEM, "host allocation failed");
    s->cfg = *cfg;
    s->ledger = Ledger(cfg->hbm_budget_bytes);
    s->own_streams = cfg->n_streams == 0;
    if (!s->own_streams) s->cfg.max_active = cfg->n_streams;
    if (s->cfg.max_active <= 0) s->cfg.max_active = 8;
    if (s->cfg.max_active > 64) s->cfg.max_active = 64;
    (void)hipGetDevice(&s->device);
    s->streams.assign(s->cfg.max_active, nullptr);
    s->slots.assign(s->cfg.max_active, SlotRes{});
    s->slot_busy.assign(s->cfg.max_active, 0);
    for (int i = 0; i < s->cfg.max_active; ++i) {
        int rc = WD_OK;
        if (!s->own_streams)
            s->streams[i] = (hipStream_t)cfg->streams[i];
        else if (hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) != hipSuccess)
            rc = fail(WD_ERR_HIP, "hipStreamCreate failed");
        if (rc == WD_OK) rc = s->slots[i].create();
        if (rc) {
            for (int j = 0; j <= i; ++j) {
                if (s->own_streams && s->streams[j]) (void)hipStreamDestroy(s->streams[j]);
                s->slots[j].destroy();
            }
            delete s;
            return rc;
        }
    }
    s->t_start = now_seconds();
    {
        std::lock_guard<std::mutex> g(g_servers_mu);
        g_servers.insert(s);
    }
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
    auto r = std::make_shared<Request>();
    r->need = request_need(lat, *p);
    // the request alone on an empty server: workspace, float64 links, forms
    size_t master = 0, derived[kNumDerived];
    lattice_forms(lat, &master, derived);
    size_t alone = r->need.workspace + master;
    for (int f = 0; f < kNumDerived; ++f) alone += r->need.form_bytes[f];
    if (alone > s->cfg.hbm_budget_bytes)
        return fail(WD_ERR_NOMEM, "request needs %zu bytes, more than the whole budget (%zu)",
                    alone, s->cfg.hbm_budget_bytes);
    r->lat = lat;
    r->p = *p;
    r->b = b;
    r->x = x;
    r->t_submit = now_seconds();
    lat->users.fetch_add(1);
    const uint64_t t = s->book.submit(r);
    if (!t) {
        lat->users.fetch_sub(1);
        return fail(WD_ERR_STATE, "server is shutting down");
    }
    *ticket = t;
    return WD_OK;
}

int wd_poll(wd_server *s, uint64_t ticket, wd_solve_info *info) {
    if (!s) return fail(WD_ERR_ARG, "null server");
    int rc = WD_PENDING;
    const int st = s->book.poll(ticket, [&](const Request &r) {
        if (info)
            for (int k = 0; k < r.p.nrhs; ++k) info[k] = r.info[k];
        rc = r.rc;
    });
    if (st < 0)
        return fail(WD_ERR_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (st == 0) return WD_PENDING;
    if (rc < 0) fail(rc, "request %llu failed", (unsigned long long)ticket);
    return rc;
}

int wd_server_stats(wd_server *s, double *solves_per_s, double *p50_s, double *p99_s) {
    if (!s || !solves_per_s || !p50_s || !p99_s) return fail(WD_ERR_ARG, "null argument");
    std::vector<double> l;
    double span = 0.0;
    {
        std::lock_guard<std::mutex> lk(s->stat_mu);
        l = s->latencies;
        span = (s->t_last > s->t_start) ? s->t_last - s->t_start : 0.0;
    }
    const size_t n = l.size();
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
    std::lock_guard<std::mutex> lk(s->ledger_mu);
    *bytes = s->ledger.peak();
    return WD_OK;
}

int wd_server_destroy(wd_server *s) {
    if (!s) return fail(WD_ERR_ARG, "null server");
    s->book.stop();
    if (s->thr.joinable()) s->thr.join();
    {
        std::lock_guard<std::mutex> g(g_servers_mu);
        g_servers.erase(s);
    }
    for (size_t i = 0; i < s->streams.size(); ++i) {
        (void)hipStreamSynchronize(s->streams[i]);
        if (s->own_streams) (void)hipStreamDestroy(s->streams[i]);
        s->slots[i].destroy();
    }
    delete s;
    return WD_OK;
}

}  // extern "C"

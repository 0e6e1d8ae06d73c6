// Host check of the solve server's core (server_core.hpp), built with the
// address / undefined-behaviour sanitizers and, separately, the thread
// sanitizer (tests/test_server_core_host.py).  Exit code 0 and a last line
// "OK" on success.
//
// 1. Ledger: a simulated scheduler admits a random stream of requests on a
//    few lattices under a tight budget, releases the forms the ledger plans
//    to release, builds the forms each admitted request reads and retires
//    requests at random.  After every step the ledger's charge must equal
//    the charge recomputed from the simulated lattices, never exceed the
//    budget, and no release may touch a lattice with running requests or a
//    form the admitted request reads; every request must run eventually.
// 2. TicketBook: client threads submit and poll while a scheduler thread
//    takes and publishes; every ticket a client got back is published, and
//    the book never holds more than the pollable finished records plus the
//    requests in flight.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "server_core.hpp"

using namespace wd;

static int fails = 0;
#define CHECK(c)                                                     \
    do {                                                             \
        if (!(c)) {                                                  \
            ++fails;                                                 \
            std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);  \
        }                                                            \
    } while (0)

struct SimLat {
    size_t master;
    size_t form_size[kNumDerived];
    size_t derived[kNumDerived];  // resident now
    int running;
};

struct SimReq {
    int lat;
    Need need;
    int remaining;  // scheduling turns until it retires
};

static size_t truth(const std::vector<SimLat> &lats, const std::vector<SimReq> &running,
                    const std::vector<bool> &known) {
    size_t b = 0;
    for (const auto &r : running) b += r.need.workspace;
    for (size_t i = 0; i < lats.size(); ++i) {
        if (!known[i]) continue;
        if (lats[i].running > 0) b += lats[i].master;
        for (int f = 0; f < kNumDerived; ++f) b += lats[i].derived[f];
    }
    return b;
}

static void ledger_run(unsigned seed) {
    std::mt19937_64 rng(seed);
    const int nl = 4;
    std::vector<SimLat> lats(nl);
    for (auto &l : lats) {
        l.master = 1000 + rng() % 1000;
        for (int f = 0; f < kNumDerived; ++f) {
            l.form_size[f] = 100 + rng() % 700;
            l.derived[f] = 0;
        }
        l.running = 0;
    }
    // the largest single request: workspace + master + every form
    size_t biggest = 0;
    std::vector<SimReq> queue;
    for (int k = 0; k < 400; ++k) {
        SimReq r{};
        r.lat = (int)(rng() % nl);
        r.need.workspace = 200 + rng() % 800;
        const int nf = (int)(rng() % 3);
        for (int j = 0; j < nf; ++j) {
            const int f = (int)(rng() % kNumDerived);
            r.need.form_bytes[f] = lats[r.lat].form_size[f];
        }
        r.remaining = 1 + (int)(rng() % 4);
        size_t alone = r.need.workspace + lats[r.lat].master;
        for (int f = 0; f < kNumDerived; ++f) alone += r.need.form_bytes[f];
        biggest = std::max(biggest, alone);
        queue.push_back(r);
    }
    const size_t budget = biggest + (rng() % 3000);
    Ledger led(budget);
    std::vector<bool> known(nl, false);
    std::vector<SimReq> running;
    size_t head = 0;
    int turns = 0;
    while ((head < queue.size() || !running.empty()) && turns < 100000) {
        ++turns;
        // admission, in arrival order
        while (head < queue.size() && running.size() < 6) {
            SimReq &r = queue[head];
            for (int i = 0; i < nl; ++i)
                if (known[i] || i == r.lat) {
                    led.observe(&lats[i], lats[i].master, lats[i].derived);
                    known[i] = true;
                }
            CHECK(led.used() == truth(lats, running, known));
            std::vector<Eviction> ev;
            if (!led.plan(&lats[r.lat], r.need, &ev)) {
                CHECK(ev.empty());
                CHECK(!running.empty());  // with nothing running it must fit
                break;
            }
            for (const Eviction &e : ev) {
                SimLat *l = (SimLat *)e.lat;
                CHECK(l->running == 0);
                CHECK(!(l == &lats[r.lat] && r.need.form_bytes[e.form]));
                CHECK(l->derived[e.form] > 0);
                l->derived[e.form] = 0;
                led.evicted(e.lat, e.form);
            }
            led.admit(&lats[r.lat], r.need);
            // the solve's setup builds the forms it reads
            lats[r.lat].running += 1;
            for (int f = 0; f < kNumDerived; ++f)
                if (r.need.form_bytes[f]) lats[r.lat].derived[f] = r.need.form_bytes[f];
            running.push_back(r);
            ++head;
            CHECK(led.used() == truth(lats, running, known));
            CHECK(led.used() <= budget);
        }
        // one turn: some requests retire
        for (size_t k = 0; k < running.size();) {
            if (--running[k].remaining <= 0) {
                led.retire(&lats[running[k].lat], running[k].need.workspace);
                lats[running[k].lat].running -= 1;
                running.erase(running.begin() + (long)k);
            } else {
                ++k;
            }
        }
        CHECK(led.used() == truth(lats, running, known));
        CHECK(led.used() <= budget);
    }
    CHECK(head == queue.size() && running.empty());
    CHECK(led.peak() <= budget);
    // a destroyed lattice leaves the ledger
    led.forget(&lats[0]);
    known[0] = false;
    CHECK(led.find(&lats[0]) == nullptr);
    CHECK(led.used() == truth(lats, running, known));
}

struct Rec {
    uint64_t ticket = 0;
    bool done = false;
    int value = 0;
    int result = 0;
};

static void book_run() {
    const size_t keep = 32;
    TicketBook<Rec> book(keep);
    const int nclients = 4, per_client = 500;
    std::atomic<int> published{0};
    std::atomic<size_t> max_size{0};
    std::thread sched([&] {
        std::vector<std::shared_ptr<Rec>> work;
        for (;;) {
            const bool open = book.take(&work, work.empty(), std::chrono::microseconds(200));
            if (!open && work.empty()) break;
            if (!work.empty()) {
                auto r = work.front();
                work.erase(work.begin());
                const int v = r->value;  // set before submit, read-only after
                book.publish(r, [&](Rec &q) { q.result = 2 * v; });
                published.fetch_add(1);
            }
            const size_t sz = book.size();
            size_t m = max_size.load();
            while (sz > m && !max_size.compare_exchange_weak(m, sz)) {
            }
        }
    });
    std::vector<std::thread> clients;
    std::atomic<int> bad{0}, seen{0};
    for (int c = 0; c < nclients; ++c) {
        clients.emplace_back([&, c] {
            std::vector<uint64_t> mine;
            for (int k = 0; k < per_client; ++k) {
                auto r = std::make_shared<Rec>();
                r->value = c * per_client + k;
                const uint64_t t = book.submit(r);
                if (t == 0) {
                    bad.fetch_add(1);
                    continue;
                }
                mine.push_back(t);
                // poll the ticket submitted a few steps back
                if (mine.size() > 3) {
                    const uint64_t q = mine[mine.size() - 4];
                    int res = -1;
                    const int st = book.poll(q, [&](const Rec &x) { res = x.result; });
                    if (st == 1) {
                        seen.fetch_add(1);
                        if (res % 2) bad.fetch_add(1);
                    }
                }
            }
        });
    }
    for (auto &t : clients) t.join();
    book.stop();
    sched.join();
    CHECK(bad.load() == 0);
    CHECK(published.load() == nclients * per_client);
    CHECK(book.size() <= keep);
    // at most the pollable records plus one client's burst in flight
    CHECK(max_size.load() <= keep + (size_t)(nclients * per_client));
    // submission after stop is refused
    CHECK(book.submit(std::make_shared<Rec>()) == 0);
    std::printf("book: %d published, %d polled done, max size %zu\n", published.load(), seen.load(),
                max_size.load());
}

int main() {
    for (unsigned seed = 1; seed <= 40; ++seed) ledger_run(seed);
    std::printf("ledger: 40 random streams\n");
    book_run();
    if (fails) {
        std::printf("%d failures\n", fails);
        return 1;
    }
    std::printf("OK\n");
    return 0;
}

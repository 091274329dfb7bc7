// The server's scheduler (paper_2503_16037_amd/csrc/sched.hpp) driven by a scripted backend
// on the CPU: no device, each "run" takes a request's scripted bytes from a budget, holds
// them for a few milliseconds (or, gated, until the scenario releases it) and gives them
// back, or fails as scripted.  A scenario that needs a request to be still running at some
// step gates it, so no outcome depends on timing.  One scenario per run (argument),
// printing "ok <name>" or "FAIL <name>: <why>"; exit status 0 when it holds.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "sched.hpp"

using namespace sg::serve;

namespace {

struct Script {
    uint64_t need = 0;         // bytes a run takes (its reservation may say less)
    int ms = 5;                // how long a run holds them
    int fail_runs = 0;         // injected allocation failures: the first runs fail
    bool gmres_nomem = false;  // the first run fails for a GMRES basis
    bool gated = false;        // hold the bytes until the scenario opens the gate
};

struct FakeBackend : public Backend {
    uint64_t budget_ = 100, gmres_ = 0, cache = 0;
    std::atomic<uint64_t> used_{0};
    std::atomic<int> running{0}, max_running{0};
    std::atomic<uint64_t> max_used{0};
    std::mutex m;
    std::map<uint64_t, Script> script;          // by ticket
    std::vector<uint64_t> started;              // tickets in the order their runs began
    std::map<uint64_t, std::vector<uint64_t>> bytes_seen;  // reservation at each run
    int released = 0;
    std::condition_variable gate_cv;
    std::map<uint64_t, bool> gate_open;  // by ticket

    void open(uint64_t ticket) {
        {
            std::lock_guard<std::mutex> lk(m);
            gate_open[ticket] = true;
        }
        gate_cv.notify_all();
    }

    uint64_t budget() const override { return budget_; }
    uint64_t used() const override { return used_.load(); }
    void release_cache() override {
        std::lock_guard<std::mutex> lk(m);
        used_ -= cache;
        cache = 0;
        ++released;
    }
    uint64_t gmres_bytes(const Request &) override { return gmres_; }
    sg_status run(Request &r, int w, bool &gmres_nomem, std::string &err) override {
        (void)w;
        Script sc;
        {
            std::lock_guard<std::mutex> lk(m);
            started.push_back(r.ticket);
            bytes_seen[r.ticket].push_back(r.bytes);
            Script &s = script[r.ticket];
            if (s.fail_runs > 0) {
                --s.fail_runs;
                err = "injected allocation failure";
                return SG_E_NOMEM;
            }
            if (s.gmres_nomem) {
                s.gmres_nomem = false;
                gmres_nomem = true;
                err = "GMRES basis out of budget";
                return SG_E_NOMEM;
            }
            sc = s;
        }
        uint64_t u = used_.load();
        do {
            if (u + sc.need > budget_) {
                err = "out of budget";
                return SG_E_NOMEM;
            }
        } while (!used_.compare_exchange_weak(u, u + sc.need));
        const uint64_t now = u + sc.need;
        uint64_t mu = max_used.load();
        while (now > mu && !max_used.compare_exchange_weak(mu, now)) {
        }
        const int rn = ++running;
        int mr = max_running.load();
        while (rn > mr && !max_running.compare_exchange_weak(mr, rn)) {
        }
        if (sc.gated) {
            std::unique_lock<std::mutex> lk(m);
            gate_cv.wait(lk, [&] { return gate_open[r.ticket]; });
        } else {
            std::this_thread::sleep_for(std::chrono::milliseconds(sc.ms));
        }
        --running;
        used_ -= sc.need;
        r.radiance.assign(1, (double)r.ticket);
        r.info.converged = 1;
        return SG_OK;
    }
};

std::unique_ptr<Request> req(uint64_t bytes) {
    std::unique_ptr<Request> r(new Request());
    r->bytes = bytes;
    r->radiance.assign(1, 0.0);
    return r;
}

struct Run {
    FakeBackend be;
    Scheduler s;
    std::vector<uint64_t> tickets;
    Run(int workers, int cap, uint64_t budget) {
        be.budget_ = budget;
        s.start(&be, workers, cap);
    }
    ~Run() { s.shutdown(); }
    sg_status submit(uint64_t bytes, Script sc) {
        uint64_t t = 0;
        std::string err;
        {
            // the ticket is known only after submit: script the next one first
            std::lock_guard<std::mutex> lk(be.m);
            be.script[s.next_ticket] = sc;
        }
        const sg_status st = s.submit(req(bytes), &t, err);
        if (st == SG_OK) tickets.push_back(t);
        return st;
    }
    sg_status wait(uint64_t t) {
        std::string err;
        double rad = 0.0;
        return s.wait(t, &rad, nullptr, err);
    }
    void wait_running(int n) {
        while (be.running.load() < n) std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    // polls cond (under the scheduler's lock) for up to 60 s
    template <class F>
    bool wait_until(F &&cond) {
        const auto t0 = std::chrono::steady_clock::now();
        while (std::chrono::steady_clock::now() - t0 < std::chrono::seconds(60)) {
            {
                std::lock_guard<std::mutex> lk(s.mu);
                if (cond()) return true;
            }
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
        return false;
    }
};

Script held(uint64_t need) {
    Script sc;
    sc.need = need;
    sc.gated = true;
    return sc;
}

bool fail(const char *name, const std::string &why) {
    std::printf("FAIL %s: %s\n", name, why.c_str());
    return false;
}

// At most what the budget holds runs at once, and every request succeeds.
bool admission() {
    Run r(3, 64, 100);
    for (int i = 0; i < 8; ++i) r.submit(40, Script{40, 10});
    for (auto t : r.tickets)
        if (r.wait(t) != SG_OK) return fail("admission", "a request failed");
    if (r.be.max_running.load() > 2) return fail("admission", "more resident than the budget holds");
    if (r.be.max_used.load() > 100) return fail("admission", "budget exceeded");
    if (r.s.latencies.size() != 8) return fail("admission", "latencies not recorded");
    return true;
}

// Only the head of the queue is admitted: a small request behind one that does not fit yet
// waits for it (no overtaking).
bool fifo() {
    Run r(3, 64, 100);
    r.submit(60, held(60));
    r.wait_running(1);
    r.submit(60, Script{60, 5});  // does not fit next to the first
    r.submit(10, Script{10, 5});  // would fit, but is behind it
    std::this_thread::sleep_for(std::chrono::milliseconds(30));  // room to overtake, if it would
    {
        std::lock_guard<std::mutex> lk(r.be.m);
        if (r.be.started.size() != 1) return fail("fifo", "a queued request started next to the held one");
    }
    r.be.open(r.tickets[0]);
    for (auto t : r.tickets)
        if (r.wait(t) != SG_OK) return fail("fifo", "a request failed");
    const auto &o = r.be.started;
    const auto p2 = std::find(o.begin(), o.end(), r.tickets[1]), p3 = std::find(o.begin(), o.end(), r.tickets[2]);
    return p2 < p3 || fail("fifo", "a later request overtook the head of the queue");
}

// A full queue refuses with SG_E_BUSY, and takes requests again once it has room.
bool backpressure() {
    Run r(1, 2, 100);
    r.submit(10, held(10));
    r.wait_running(1);
    if (r.submit(10, Script{10, 1}) != SG_OK || r.submit(10, Script{10, 1}) != SG_OK)
        return fail("backpressure", "queue refused below its capacity");
    if (r.submit(10, Script{10, 1}) != SG_E_BUSY) return fail("backpressure", "full queue accepted a request");
    r.be.open(r.tickets[0]);
    for (auto t : r.tickets)
        if (r.wait(t) != SG_OK) return fail("backpressure", "a request failed");
    if (r.submit(10, Script{10, 1}) != SG_OK) return fail("backpressure", "drained queue refused");
    return r.wait(r.tickets.back()) == SG_OK || fail("backpressure", "late request failed");
}

// A request whose reservation alone exceeds the budget is refused at submission.
bool over_budget() {
    Run r(2, 8, 100);
    if (r.submit(150, Script{150, 1}) != SG_E_NOMEM) return fail("over_budget", "accepted");
    return r.tickets.empty() || fail("over_budget", "queued");
}

// A request that runs out of budget in the mix goes back to the queue and succeeds later.
bool requeue_in_mix() {
    Run r(2, 8, 100);
    r.submit(50, held(50));       // holds its bytes while the next one starts
    r.wait_running(1);
    r.submit(50, Script{60, 5});  // needs more than reserved: 50 + 60 > 100
    if (!r.wait_until([&] { return r.s.n_requeued >= 1; })) return fail("requeue_in_mix", "nothing was requeued");
    r.be.open(r.tickets[0]);
    for (auto t : r.tickets)
        if (r.wait(t) != SG_OK) return fail("requeue_in_mix", "a request failed");
    if (r.s.n_requeued < 1) return fail("requeue_in_mix", "nothing was requeued");
    if (r.be.max_used.load() > 100) return fail("requeue_in_mix", "budget exceeded");
    return true;
}

// Alone and out of budget because of cached blocks: the cache is released and it runs again.
bool cold_retry() {
    Run r(1, 8, 100);
    r.be.cache = 30;
    r.be.used_ = 30;
    r.submit(70, Script{80, 1});
    if (r.wait(r.tickets[0]) != SG_OK) return fail("cold_retry", "failed");
    if (r.be.released != 1) return fail("cold_retry", "cache not released exactly once");
    return r.be.started.size() == 2 || fail("cold_retry", "not run twice");
}

// Alone, out of budget even with the cache released: it fails with SG_E_NOMEM.
bool alone_nomem() {
    Run r(1, 8, 100);
    r.submit(90, Script{120, 1});
    if (r.wait(r.tickets[0]) != SG_E_NOMEM) return fail("alone_nomem", "did not fail");
    return (r.be.released == 1 && r.be.started.size() == 2) || fail("alone_nomem", "not retried once");
}

// A solve out of budget for its GMRES basis: the basis joins the reservation, then it runs.
bool gmres_basis() {
    Run r(1, 8, 100);
    r.be.gmres_ = 20;
    Script sc{50, 1};
    sc.gmres_nomem = true;
    r.submit(50, sc);
    if (r.wait(r.tickets[0]) != SG_OK) return fail("gmres_basis", "failed");
    const auto &b = r.be.bytes_seen[r.tickets[0]];
    if (b.size() != 2 || b[1] != 70) return fail("gmres_basis", "basis not added to the reservation");
    return true;
}

// The basis makes the reservation exceed the budget: SG_E_NOMEM without another run.
bool gmres_over() {
    Run r(1, 8, 100);
    r.be.gmres_ = 20;
    Script sc{90, 1};
    sc.gmres_nomem = true;
    r.submit(90, sc);
    if (r.wait(r.tickets[0]) != SG_E_NOMEM) return fail("gmres_over", "did not fail");
    return r.be.started.size() == 1 || fail("gmres_over", "ran again");
}

// An injected allocation failure while others run: requeued, then completed.
bool injected() {
    Run r(2, 8, 100);
    r.submit(20, Script{20, 60});
    r.wait_running(1);
    Script sc{20, 1};
    sc.fail_runs = 1;
    r.submit(20, sc);
    r.submit(20, Script{20, 1});
    for (auto t : r.tickets)
        if (r.wait(t) != SG_OK) return fail("injected", "a request failed");
    const auto n = std::count(r.be.started.begin(), r.be.started.end(), r.tickets[1]);
    return n == 2 || fail("injected", "the failed request ran " + std::to_string(n) + " times");
}

// Cancellation: a queued request never runs and reports SG_E_CANCELLED; a running or
// finished one is not touched.
bool cancel() {
    Run r(1, 8, 100);
    r.submit(10, held(10));
    r.wait_running(1);
    r.submit(10, Script{10, 1});
    r.submit(10, Script{10, 1});
    std::string err;
    if (r.s.cancel(r.tickets[1], err) != SG_OK) return fail("cancel", "queued request not cancelled");
    if (r.s.cancel(r.tickets[0], err) != SG_E_STATE) return fail("cancel", "running request cancelled");
    r.be.open(r.tickets[0]);
    if (r.wait(r.tickets[1]) != SG_E_CANCELLED) return fail("cancel", "cancelled ticket did not say so");
    if (r.wait(r.tickets[0]) != SG_OK) return fail("cancel", "running request failed");
    for (;;) {  // the third finishes; cancelling it then changes nothing
        {
            std::lock_guard<std::mutex> lk(r.s.mu);
            if (r.s.tickets[r.tickets[2]]->done) break;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    if (r.s.cancel(r.tickets[2], err) != SG_E_STATE) return fail("cancel", "finished request cancelled");
    if (r.wait(r.tickets[2]) != SG_OK) return fail("cancel", "third request failed");
    if (r.s.cancel(r.tickets[2], err) != SG_E_INVALID) return fail("cancel", "released ticket known");
    const std::vector<uint64_t> want{r.tickets[0], r.tickets[2]};
    return r.be.started == want || fail("cancel", "the cancelled request ran");
}

// Shutdown drains what is queued.
bool drain() {
    FakeBackend be;
    be.budget_ = 100;
    Scheduler s;
    s.start(&be, 2, 16);
    for (int i = 0; i < 6; ++i) {
        {
            std::lock_guard<std::mutex> lk(be.m);
            be.script[s.next_ticket] = Script{30, 5};
        }
        uint64_t t;
        std::string err;
        s.submit(req(30), &t, err);
    }
    s.shutdown();
    if (be.started.size() != 6) return fail("drain", "queue not drained");
    for (auto &kv : s.tickets)
        if (kv.second->status != SG_OK || !kv.second->done) return fail("drain", "request not completed");
    return true;
}

}  // namespace

int main(int argc, char **argv) {
    const std::map<std::string, bool (*)()> all = {
        {"admission", admission}, {"fifo", fifo}, {"backpressure", backpressure}, {"over_budget", over_budget},
        {"requeue_in_mix", requeue_in_mix}, {"cold_retry", cold_retry}, {"alone_nomem", alone_nomem},
        {"gmres_basis", gmres_basis}, {"gmres_over", gmres_over}, {"injected", injected},
        {"cancel", cancel}, {"drain", drain}};
    if (argc < 2 || !all.count(argv[1])) {
        for (auto &kv : all) std::printf("%s\n", kv.first.c_str());
        return argc < 2 ? 0 : 2;
    }
    if (!all.at(argv[1])()) return 1;
    std::printf("ok %s\n", argv[1]);
    return 0;
}

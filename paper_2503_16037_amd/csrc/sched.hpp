// Scheduling of the server (continuous batching of scenes of uneven size on one device),
// apart from the device itself: a queue of requests, worker threads (one per resident slot)
// and admission of the head of the queue by reserved bytes against a budget.  What a worker
// does with an admitted request (create, solve and release its scene on a stream of its own)
// comes from a backend: the library's backend is the device (server.cpp); the tests drive
// the same scheduler with a scripted backend on the CPU.
//
// A request that runs out of budget in the mix (its scene, or its solve: a GMRES fallback
// allocates its basis, and the block cache may hand out blocks up to 5/4 of a request) goes
// back to the head of the queue and runs again once another request has finished, with the
// basis added to its reservation when that is what failed; alone, it runs once more after
// the backend has released its cache, then fails.  A pending request can be cancelled.
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sgrt.h"

namespace sg {
namespace serve {

inline double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// A request: its own copy of the scene description, its results and its scheduling state.
struct Request {
    uint64_t ticket = 0;
    uint64_t bytes = 0;         // reservation used for admission
    bool gmres_added = false;   // bytes include the GMRES basis (after a solve ran out of budget)
    bool retried_cold = false;  // ran again alone after the backend released its cache
    bool running = false;       // admitted and not finished
    double t_arrival = 0.0, t_done = 0.0;
    // owned copy of the description
    sg_scene_desc d{};
    std::vector<float> mu_s, mu_a, frac, albedo, abs_scale;
    std::vector<double> g, lut;
    std::vector<int32_t> kinds;
    std::vector<int32_t> pos, adj_idx, los_node;
    std::vector<int64_t> adj_ptr, los_ptr;
    std::vector<double> los_t;
    // results
    std::vector<double> radiance;
    sg_solve_info info{};
    sg_status status = SG_OK;
    std::string error;
    bool done = false;

    // deep copy of a validated description
    void copy_from(const sg_scene_desc *src) {
        d = *src;
        const size_t nvox = (size_t)src->nx * src->ny * src->nz, npx = (size_t)src->nx * src->ny;
        const size_t nvol = src->n_nodes > 0 ? (size_t)src->n_nodes : nvox;
        const size_t N = nvol + (src->surface_nodes ? npx : 0);
        const size_t E = (size_t)src->adj_ptr[N];
        mu_s.assign(src->mu_s, src->mu_s + nvox);
        mu_a.assign(src->mu_a, src->mu_a + nvox);
        if (src->phase_frac) frac.assign(src->phase_frac, src->phase_frac + (size_t)src->n_phase * nvox);
        albedo.assign(src->surf_albedo, src->surf_albedo + npx);
        if (src->abs_scale) abs_scale.assign(src->abs_scale, src->abs_scale + src->n_lambda);
        g.assign(src->hg_g, src->hg_g + src->n_phase);
        if (src->phase_kind) {
            kinds.assign(src->phase_kind, src->phase_kind + src->n_phase);
            bool table = false;
            for (int k = 0; k < src->n_phase; ++k) table = table || src->phase_kind[k] == SG_PHASE_TABLE;
            if (table) lut.assign(src->phase_lut, src->phase_lut + (size_t)src->n_phase * src->phase_lut_n);
        }
        if (src->n_nodes > 0) {  // general nodes and the lines of sight's elements
            pos.assign(src->node_pos_fx, src->node_pos_fx + 3 * nvol);
            los_ptr.assign(src->los_ptr, src->los_ptr + npx + 1);
            los_node.assign(src->los_node, src->los_node + los_ptr[npx]);
            los_t.assign(src->los_t, src->los_t + los_ptr[npx]);
        } else {
            pos.assign(src->vol_pos_fx, src->vol_pos_fx + 3 * nvox);
        }
        adj_ptr.assign(src->adj_ptr, src->adj_ptr + N + 1);
        if (E) adj_idx.assign(src->adj_idx, src->adj_idx + E);
        radiance.assign((size_t)src->n_lambda * npx, 0.0);
        relink();
    }
    void relink() {
        d.mu_s = mu_s.data();
        d.mu_a = mu_a.data();
        d.phase_frac = frac.empty() ? nullptr : frac.data();
        d.surf_albedo = albedo.data();
        d.abs_scale = abs_scale.empty() ? nullptr : abs_scale.data();
        d.hg_g = g.data();
        d.phase_kind = kinds.empty() ? nullptr : kinds.data();
        d.phase_lut = lut.empty() ? nullptr : lut.data();
        if (d.n_nodes > 0) {
            d.node_pos_fx = pos.data();
            d.los_ptr = los_ptr.data();
            d.los_node = los_node.data();
            d.los_t = los_t.data();
        } else {
            d.vol_pos_fx = pos.data();
        }
        d.adj_ptr = adj_ptr.data();
        d.adj_idx = adj_idx.empty() ? nullptr : adj_idx.data();
    }
    // the inputs are not needed once the scene has been solved
    void drop_inputs() {
        std::vector<float>().swap(mu_s);
        std::vector<float>().swap(mu_a);
        std::vector<float>().swap(frac);
        std::vector<int32_t>().swap(pos);
        std::vector<int32_t>().swap(adj_idx);
        std::vector<int64_t>().swap(adj_ptr);
        std::vector<int32_t>().swap(los_node);
        std::vector<int64_t>().swap(los_ptr);
        std::vector<double>().swap(los_t);
    }
};

// What a worker does with an admitted request, and the memory it is admitted against.
struct Backend {
    virtual ~Backend() = default;
    virtual uint64_t budget() const = 0;  // bytes the admitted requests may hold together
    virtual uint64_t used() const = 0;    // bytes held now, also by work outside the server
    virtual void release_cache() = 0;     // cached blocks returned: each block then fits its request
    virtual uint64_t gmres_bytes(const Request &r) = 0;  // what a GMRES fallback adds to r's reservation
    virtual void worker_start(int w) { (void)w; }
    // Create, solve and release r's scene on worker w (the results into r.radiance, r.info).
    // gmres_nomem: the solve ran out of budget for a GMRES basis.
    virtual sg_status run(Request &r, int w, bool &gmres_nomem, std::string &err) = 0;
};

struct Scheduler {
    Backend *be = nullptr;
    int queue_cap = 1;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> pending;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> tickets;
    std::vector<double> latencies;
    uint64_t next_ticket = 1;
    uint64_t n_finished = 0;  // requests finished so far (a requeued request waits for the next one)
    uint64_t n_requeued = 0;  // requests put back at the head of the queue after running out of budget
    int running = 0;
    uint64_t reserved = 0;  // reservations of the admitted requests
    bool stop = false;
    std::vector<std::thread> workers;

    void start(Backend *b, int n_workers, int cap) {
        be = b;
        queue_cap = cap;
        for (int w = 0; w < n_workers; ++w) workers.emplace_back(&Scheduler::worker, this, w);
    }

    // let the workers drain the queue, then join them
    void shutdown() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
            cv.notify_all();
        }
        for (auto &t : workers) t.join();
        workers.clear();
    }

    // SG_E_BUSY when the queue is full, SG_E_STATE when stopping, SG_E_NOMEM when the
    // request alone exceeds the budget
    sg_status submit(std::unique_ptr<Request> r, uint64_t *ticket, std::string &err) {
        if (r->bytes > be->budget()) {
            err = "scene alone exceeds the HBM budget";
            return SG_E_NOMEM;
        }
        r->t_arrival = now_ms();
        std::lock_guard<std::mutex> lk(mu);
        if (stop) {
            err = "server is stopping";
            return SG_E_STATE;
        }
        if ((int)pending.size() >= queue_cap) {
            err = "queue full";
            return SG_E_BUSY;
        }
        r->ticket = next_ticket++;
        *ticket = r->ticket;
        pending.push_back(r.get());
        tickets[r->ticket] = std::move(r);
        cv.notify_all();
        return SG_OK;
    }

    // A pending request leaves the queue and finishes with SG_E_CANCELLED; one that runs or
    // has finished is not touched (SG_E_STATE).
    sg_status cancel(uint64_t ticket, std::string &err) {
        std::lock_guard<std::mutex> lk(mu);
        auto it = tickets.find(ticket);
        if (it == tickets.end()) {
            err = "unknown ticket";
            return SG_E_INVALID;
        }
        Request *r = it->second.get();
        if (r->done || r->running) {
            err = r->done ? "request already finished" : "request is running";
            return SG_E_STATE;
        }
        pending.erase(std::find(pending.begin(), pending.end(), r));
        finish_locked(r, SG_E_CANCELLED, "cancelled");
        return SG_OK;
    }

    // with the lock held: the request's result, and its ticket released
    sg_status take_locked(uint64_t ticket, double *radiance, sg_solve_info *info, std::string &err) {
        auto it = tickets.find(ticket);
        Request *r = it->second.get();
        if (radiance) std::memcpy(radiance, r->radiance.data(), sizeof(double) * r->radiance.size());
        if (info) *info = r->info;
        const sg_status st = r->status;
        if (st != SG_OK) err = r->error;
        tickets.erase(it);
        return st;
    }

    sg_status poll(uint64_t ticket, double *radiance, sg_solve_info *info, int32_t *done, std::string &err) {
        std::lock_guard<std::mutex> lk(mu);
        auto it = tickets.find(ticket);
        if (it == tickets.end()) {
            err = "unknown ticket";
            return SG_E_INVALID;
        }
        if (!it->second->done) {
            *done = 0;
            return SG_OK;
        }
        *done = 1;
        return take_locked(ticket, radiance, info, err);
    }

    sg_status wait(uint64_t ticket, double *radiance, sg_solve_info *info, std::string &err) {
        std::unique_lock<std::mutex> lk(mu);
        auto it = tickets.find(ticket);
        if (it == tickets.end()) {
            err = "unknown ticket";
            return SG_E_INVALID;
        }
        Request *r = it->second.get();
        cv.wait(lk, [&] { return r->done; });
        return take_locked(ticket, radiance, info, err);
    }

    void finish_locked(Request *r, sg_status st, const std::string &err) {
        r->status = st;
        r->error = err;
        r->done = true;
        r->running = false;
        r->t_done = now_ms();
        if (st != SG_E_CANCELLED) latencies.push_back(r->t_done - r->t_arrival);
        ++n_finished;
        cv.notify_all();
    }
    void finish(Request *r, sg_status st, const std::string &err) {
        std::lock_guard<std::mutex> lk(mu);
        finish_locked(r, st, err);
    }

    void worker(int w) {
        be->worker_start(w);
        while (true) {
            Request *r = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                while (true) {
                    if (pending.empty()) {
                        if (stop) return;
                        cv.wait(lk);
                        continue;
                    }
                    Request *h = pending.front();
                    // admitted requests may not have allocated yet: admit by reservations,
                    // plus whatever the backend holds beyond them (work outside the server)
                    const uint64_t used = be->used();
                    const uint64_t outside = used > reserved ? used - reserved : 0;
                    const bool fits = reserved + h->bytes + outside <= be->budget();
                    if (fits || running == 0) {
                        pending.pop_front();
                        r = h;
                        r->running = true;
                        ++running;
                        reserved += h->bytes;
                        break;
                    }
                    cv.wait(lk);  // a finishing request releases memory
                }
            }
            bool gmres_nomem = false;
            std::string err;
            const sg_status s = be->run(*r, w, gmres_nomem, err);
            if (s == SG_E_NOMEM) {
                std::unique_lock<std::mutex> lk(mu);
                --running;
                reserved -= r->bytes;
                r->running = false;
                // the solve fell back to GMRES, whose basis the reservation left out
                if (gmres_nomem && !r->gmres_added) {
                    r->bytes += be->gmres_bytes(*r);
                    r->gmres_added = true;
                }
                if (r->bytes > be->budget()) {
                    finish_locked(r, SG_E_NOMEM, "scene does not fit the HBM budget");
                    continue;
                }
                if (running == 0) {
                    // alone and still out of budget: cached blocks may be larger than asked
                    // for (up to 5/4); with the cache released every block is exact and the
                    // reservation bounds the scene's bytes, so it runs once more
                    if (!r->retried_cold) {
                        r->retried_cold = true;
                        be->release_cache();
                        pending.push_front(r);
                        ++n_requeued;
                        cv.notify_all();
                        continue;
                    }
                    finish_locked(r, SG_E_NOMEM, err.empty() ? "scene does not fit the HBM budget" : err);
                    continue;
                }
                // again once another request has finished (others are running, so one will)
                pending.push_front(r);
                ++n_requeued;
                const uint64_t f0 = n_finished;
                cv.wait(lk, [&] { return n_finished != f0; });
                continue;
            }
            r->drop_inputs();
            {
                std::lock_guard<std::mutex> lk(mu);
                --running;
                reserved -= r->bytes;
                finish_locked(r, s, err);
            }
        }
    }
};

}  // namespace serve
}  // namespace sg

// Serving: continuous batching of scenes of uneven size on one device.
//
// sg_submit copies a scene description on the host and queues it.  Worker
// threads (one per resident slot, each with a device stream of its own: a solve
// captures its sweep chunks as HIP graphs, and a capture takes in every launch
// made on its stream, so two workers never share one) admit the head of the
// queue when a slot is free and the scene's reserved bytes (the scene's arrays
// and what a solve with the server's options allocates), added to those of the
// admitted scenes, fit the context's HBM budget, upload it, solve it (every
// scene keeps its own device state, so a result does not depend on what else
// is running) and release its memory, which admits the next request.  A request
// that runs out of budget in the mix (its scene or its solve: a GMRES fallback
// allocates its basis; the block cache may hand out blocks up to 5/4 of a
// request) goes back to the head of the queue and runs again once memory frees
// up, with the basis added to its reservation; alone, it runs once more on an
// emptied cache before it fails.  Work of different resident scenes overlaps
// on the device through their streams.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace sg {
namespace {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Resident slots a server may hold: the configurations its tests and measurements cover
// (with more workers, one run ended in a host fault inside the runtime's copy path during
// scene upload, whose cause has not been found).
constexpr int kMaxResident = 4;

struct Request {
    uint64_t ticket = 0;
    uint64_t bytes = 0;        // reservation used for admission
    bool gmres_added = false;  // bytes include the GMRES basis (after a solve ran out of budget)
    bool retried_cold = false;  // ran again alone on an emptied block cache
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

}  // namespace

struct Server {
    Ctx *ctx = nullptr;
    sg_server_opts opts{};
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> pending;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> tickets;
    std::vector<double> latencies;
    uint64_t next_ticket = 1;
    uint64_t n_finished = 0;  // requests finished so far (a requeued request waits for the next one)
    int running = 0;
    uint64_t reserved = 0;  // reservations of the admitted requests
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;

    void finish(Request *r, sg_status st, const std::string &err) {
        std::lock_guard<std::mutex> lk(mu);
        r->status = st;
        r->error = err;
        r->done = true;
        r->t_done = now_ms();
        latencies.push_back(r->t_done - r->t_arrival);
        ++n_finished;
        cv.notify_all();
    }

    void worker(int w) {
        (void)hipSetDevice(ctx->device);
        hipStream_t st = streams[w];
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
                    // plus whatever the context holds beyond them (scenes outside the server)
                    const uint64_t used = ctx->used.load();
                    const uint64_t outside = used > reserved ? used - reserved : 0;
                    const bool fits = reserved + h->bytes + outside <= ctx->budget;
                    if (fits || running == 0) {
                        pending.pop_front();
                        r = h;
                        ++running;
                        reserved += h->bytes;
                        break;
                    }
                    cv.wait(lk);  // a finishing scene releases memory
                }
            }
            Scene *sc = new Scene();
            sg_status s = create_scene(ctx, &r->d, st, *sc);
            if (s == SG_OK) s = solve_scene(*sc, opts.solve, st, r->radiance.data(), 0, &r->info);
            std::string err;
            if (s != SG_OK) err = t_last_error();
            const bool gmres_nomem = sc->gm_nomem;
            // a solve that stops early (out of budget mid-solve) may leave kernels queued on the
            // stream: its blocks go back to the pool, and to other streams, only once they ran
            (void)hipStreamSynchronize(st);
            free_scene(sc);
            delete sc;
            if (s == SG_E_NOMEM) {
                std::unique_lock<std::mutex> lk(mu);
                --running;
                reserved -= r->bytes;
                // the solve fell back to GMRES, whose basis the reservation left out
                if (gmres_nomem && !r->gmres_added) {
                    r->bytes += solve_reservation(&r->d, opts.solve, true) - solve_reservation(&r->d, opts.solve, false);
                    r->gmres_added = true;
                }
                if (r->bytes > ctx->budget) {
                    lk.unlock();
                    finish(r, SG_E_NOMEM, "scene does not fit the HBM budget");
                    continue;
                }
                if (running == 0) {
                    // alone and still out of budget: the pool may have handed out cached blocks
                    // larger than asked for (up to 5/4); with the cache released every block is
                    // exact and the reservation bounds the scene's bytes, so run once more
                    if (!r->retried_cold) {
                        r->retried_cold = true;
                        pool_trim(ctx, 0);
                        pending.push_front(r);
                        cv.notify_all();
                        continue;
                    }
                    lk.unlock();
                    finish(r, SG_E_NOMEM, err.empty() ? "scene does not fit the HBM budget" : err);
                    continue;
                }
                // retry once another request has finished (others are running, so one will)
                pending.push_front(r);
                const uint64_t f0 = n_finished;
                cv.wait(lk, [&] { return n_finished != f0; });
                continue;
            }
            r->drop_inputs();
            {
                std::lock_guard<std::mutex> lk(mu);
                --running;
                reserved -= r->bytes;
            }
            finish(r, s, err);
        }
    }
};

}  // namespace sg

using namespace sg;

struct sg_server : public sg::Server {};

extern "C" {

sg_status sg_server_create(sg_ctx *ctx_, const sg_server_opts *opts, sg_server **out) {
    Ctx *ctx = reinterpret_cast<Ctx *>(ctx_);
    if (!ctx || !opts || !out) {
        set_error("NULL argument");
        return SG_E_INVALID;
    }
    *out = nullptr;
    if (opts->abi_version != SG_ABI_VERSION) {
        set_error("server opts abi_version mismatch");
        return SG_E_ABI;
    }
    if (opts->max_resident < 1 || opts->queue_cap < 1 || opts->n_streams < 1 || opts->n_streams > 64) {
        set_error("max_resident >= 1, queue_cap >= 1, n_streams in 1..64 required");
        return SG_E_INVALID;
    }
    if (opts->max_resident > kMaxResident) {
        set_error("max_resident above " + std::to_string(kMaxResident) + " is not supported");
        return SG_E_INVALID;
    }
    if (opts->max_resident > opts->n_streams) {
        set_error("every resident slot needs a stream of its own: max_resident <= n_streams required");
        return SG_E_INVALID;
    }
    sg_solve_opts so;
    sg_status cs = check_opts(&opts->solve, so);
    if (cs != SG_OK) return cs;
    if (so.warm_start) {
        set_error("a warm start belongs to one scene: not accepted in the server's solve options");
        return SG_E_INVALID;
    }
    std::unique_ptr<sg_server> s(new sg_server());
    s->ctx = ctx;
    s->opts = *opts;
    s->opts.solve = so;
    if (hipSetDevice(ctx->device) != hipSuccess) {
        set_error("hipSetDevice failed");
        return SG_E_DEVICE;
    }
    for (int i = 0; i < opts->max_resident; ++i) {  // one stream per worker
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            set_error("hipStreamCreate failed");
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            return SG_E_DEVICE;
        }
        s->streams.push_back(st);
    }
    ctx->n_scenes.fetch_add(1);  // keeps the context alive while the server runs
    for (int w = 0; w < opts->max_resident; ++w) s->workers.emplace_back(&Server::worker, s.get(), w);
    *out = s.release();
    return SG_OK;
}

sg_status sg_submit(sg_server *srv, const sg_scene_desc *desc, uint64_t *ticket) {
    if (!srv || !desc || !ticket) {
        set_error("NULL argument");
        return SG_E_INVALID;
    }
    sg_status st;
    const uint64_t bytes = reservations(desc, &srv->opts.solve, srv->opts.solve.solver == SG_SOLVER_GMRES, &st);
    if (st != SG_OK) return st;
    if (bytes > srv->ctx->budget) {
        set_error("scene alone exceeds the HBM budget");
        return SG_E_NOMEM;
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) {
            set_error("server is stopping");
            return SG_E_STATE;
        }
        if ((int)srv->pending.size() >= srv->opts.queue_cap) {
            set_error("queue full");
            return SG_E_BUSY;
        }
    }
    std::unique_ptr<Request> r(new Request());
    r->copy_from(desc);
    r->bytes = bytes;
    r->t_arrival = now_ms();
    std::lock_guard<std::mutex> lk(srv->mu);
    r->ticket = srv->next_ticket++;
    *ticket = r->ticket;
    srv->pending.push_back(r.get());
    srv->tickets[r->ticket] = std::move(r);
    srv->cv.notify_all();
    return SG_OK;
}

static sg_status take_result(sg_server *srv, uint64_t ticket, double *radiance, sg_solve_info *info) {
    auto it = srv->tickets.find(ticket);
    Request *r = it->second.get();
    if (radiance) std::memcpy(radiance, r->radiance.data(), sizeof(double) * r->radiance.size());
    if (info) *info = r->info;
    const sg_status st = r->status;
    if (st != SG_OK) set_error(r->error);
    srv->tickets.erase(it);
    return st;
}

sg_status sg_poll(sg_server *srv, uint64_t ticket, double *radiance, sg_solve_info *info, int32_t *done) {
    if (!srv || !done) {
        set_error("NULL argument");
        return SG_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) {
        set_error("unknown ticket");
        return SG_E_INVALID;
    }
    if (!it->second->done) {
        *done = 0;
        return SG_OK;
    }
    *done = 1;
    return take_result(srv, ticket, radiance, info);
}

sg_status sg_wait(sg_server *srv, uint64_t ticket, double *radiance, sg_solve_info *info) {
    if (!srv) {
        set_error("NULL argument");
        return SG_E_INVALID;
    }
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) {
        set_error("unknown ticket");
        return SG_E_INVALID;
    }
    Request *r = it->second.get();
    srv->cv.wait(lk, [&] { return r->done; });
    return take_result(srv, ticket, radiance, info);
}

sg_status sg_server_latencies(sg_server *srv, double *ms, int32_t cap, int32_t *n) {
    if (!srv || !n) {
        set_error("NULL argument");
        return SG_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    const int32_t k = (int32_t)std::min<size_t>(srv->latencies.size(), (size_t)std::max(cap, 0));
    if (ms)
        for (int32_t i = 0; i < k; ++i) ms[i] = srv->latencies[i];
    *n = k;
    return SG_OK;
}

sg_status sg_server_destroy(sg_server *srv) {
    if (!srv) {
        set_error("NULL argument");
        return SG_E_INVALID;
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv.notify_all();
    }
    for (auto &t : srv->workers) t.join();
    (void)hipSetDevice(srv->ctx->device);
    for (auto st : srv->streams) (void)hipStreamDestroy(st);
    srv->ctx->n_scenes.fetch_sub(1);
    delete srv;
    return SG_OK;
}

}  // extern "C"

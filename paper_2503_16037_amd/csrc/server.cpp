// Serving: continuous batching of scenes of uneven size on one device.
//
// sg_submit copies a scene description on the host and queues it.  The scheduler
// (sched.hpp: queue, admission by reserved bytes against the context's HBM budget,
// requeue of a request that runs out of budget in the mix, cancellation) runs one
// worker thread per resident slot; this file is its device backend.  Each worker has
// a device stream of its own (a solve captures its sweep chunks as HIP graphs, and a
// capture takes in every launch made on its stream, so two workers never share one);
// it creates the admitted scene on that stream, solves it (every scene keeps its own
// device state, so a result does not depend on what else is running) and releases its
// memory, which admits the next request.  Work of different resident scenes overlaps
// on the device through their streams.
#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "internal.hpp"
#include "sched.hpp"

namespace sg {
namespace {

// Resident slots a server may hold: the configurations its tests and measurements cover
// (with more workers, one run ended in a host fault inside the runtime's copy path during
// scene upload, whose cause has not been found).
constexpr int kMaxResident = 4;

struct DeviceBackend : public serve::Backend {
    Ctx *ctx = nullptr;
    sg_solve_opts solve{};
    std::vector<hipStream_t> streams;  // one per worker

    uint64_t budget() const override { return ctx->budget; }
    uint64_t used() const override { return ctx->used.load(); }
    void release_cache() override { pool_trim(ctx, 0); }
    uint64_t gmres_bytes(const serve::Request &r) override {
        return solve_reservation(&r.d, solve, true) - solve_reservation(&r.d, solve, false);
    }
    void worker_start(int w) override {
        (void)w;
        (void)hipSetDevice(ctx->device);
    }
    sg_status run(serve::Request &r, int w, bool &gmres_nomem, std::string &err) override {
        hipStream_t st = streams[w];
        std::unique_ptr<Scene> sc(new Scene());
        sg_status s = create_scene(ctx, &r.d, st, *sc);
        if (s == SG_OK) s = solve_scene(*sc, solve, st, r.radiance.data(), 0, &r.info);
        if (s != SG_OK) err = t_last_error();
        gmres_nomem = sc->gm_nomem;
        // a solve that stops early (out of budget mid-solve) may leave kernels queued on the
        // stream: its blocks go back to the pool, and to other streams, only once they ran
        (void)hipStreamSynchronize(st);
        free_scene(sc.get());
        return s;
    }
};

}  // namespace

struct Server {
    Ctx *ctx = nullptr;
    sg_server_opts opts{};
    DeviceBackend backend;
    serve::Scheduler sched;
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
    s->backend.ctx = ctx;
    s->backend.solve = so;
    if (hipSetDevice(ctx->device) != hipSuccess) {
        set_error("hipSetDevice failed");
        return SG_E_DEVICE;
    }
    for (int i = 0; i < opts->max_resident; ++i) {  // one stream per worker
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            set_error("hipStreamCreate failed");
            for (auto x : s->backend.streams) (void)hipStreamDestroy(x);
            return SG_E_DEVICE;
        }
        s->backend.streams.push_back(st);
    }
    ctx->n_scenes.fetch_add(1);  // keeps the context alive while the server runs
    s->sched.start(&s->backend, opts->max_resident, opts->queue_cap);
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
    std::unique_ptr<serve::Request> r(new serve::Request());
    r->copy_from(desc);
    r->bytes = bytes;
    std::string err;
    st = srv->sched.submit(std::move(r), ticket, err);
    if (st != SG_OK) set_error(err);
    return st;
}

sg_status sg_cancel(sg_server *srv, uint64_t ticket) {
    if (!srv) {
        set_error("NULL argument");
        return SG_E_INVALID;
    }
    std::string err;
    const sg_status st = srv->sched.cancel(ticket, err);
    if (st != SG_OK) set_error(err);
    return st;
}

sg_status sg_poll(sg_server *srv, uint64_t ticket, double *radiance, sg_solve_info *info, int32_t *done) {
    if (!srv || !done) {
        set_error("NULL argument");
        return SG_E_INVALID;
    }
    std::string err;
    const sg_status st = srv->sched.poll(ticket, radiance, info, done, err);
    if (st != SG_OK) set_error(err);
    return st;
}

sg_status sg_wait(sg_server *srv, uint64_t ticket, double *radiance, sg_solve_info *info) {
    if (!srv) {
        set_error("NULL argument");
        return SG_E_INVALID;
    }
    std::string err;
    const sg_status st = srv->sched.wait(ticket, radiance, info, err);
    if (st != SG_OK) set_error(err);
    return st;
}

sg_status sg_server_latencies(sg_server *srv, double *ms, int32_t cap, int32_t *n) {
    if (!srv || !n) {
        set_error("NULL argument");
        return SG_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(srv->sched.mu);
    const auto &lat = srv->sched.latencies;
    const int32_t k = (int32_t)std::min<size_t>(lat.size(), (size_t)std::max(cap, 0));
    if (ms)
        for (int32_t i = 0; i < k; ++i) ms[i] = lat[i];
    *n = k;
    return SG_OK;
}

sg_status sg_server_destroy(sg_server *srv) {
    if (!srv) {
        set_error("NULL argument");
        return SG_E_INVALID;
    }
    srv->sched.shutdown();  // drains the queue
    (void)hipSetDevice(srv->ctx->device);
    for (auto st : srv->backend.streams) (void)hipStreamDestroy(st);
    srv->ctx->n_scenes.fetch_sub(1);
    delete srv;
    return SG_OK;
}

}  // extern "C"

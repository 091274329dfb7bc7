// Device memory of a context: allocations go through a caching pool, so scenes
// created and destroyed in a stream (serving, repeated solves of new scenes) reuse
// HBM blocks instead of calling hipMalloc / hipFree each time.
//
// Requests are rounded up (4 KiB granules below 1 MiB, 1 MiB granules above).  A
// freed block is kept and handed to a later request of at least 80% of its size.
// The context's budget bounds the memory held by live blocks plus cached ones:
// before a new hipMalloc, cached blocks are released until both fit; a failed
// hipMalloc releases the whole cache and retries once.
#include <hip/hip_runtime.h>

#include <string>

#include "internal.hpp"

namespace sg {

uint64_t pool_round(uint64_t bytes) {
    const uint64_t g = bytes >= (1ull << 20) ? (1ull << 20) : 4096ull;
    return (std::max<uint64_t>(bytes, 1) + g - 1) / g * g;
}

namespace {

// releases cached blocks, largest first, until `cached <= keep` (pool lock held)
void trim_locked(Ctx *ctx, uint64_t keep) {
    Pool &p = ctx->pool;
    while (p.cached > keep && !p.free_blocks.empty()) {
        auto it = std::prev(p.free_blocks.end());
        (void)hipFree(it->second);
        p.cached -= it->first;
        p.sizes.erase(it->second);
        p.free_blocks.erase(it);
    }
}

}  // namespace

sg_status pool_alloc(Ctx *ctx, uint64_t bytes, void **out) {
    const uint64_t r = pool_round(bytes);
    Pool &p = ctx->pool;
    std::lock_guard<std::mutex> lk(p.mu);
    auto it = p.free_blocks.lower_bound(r);
    if (it != p.free_blocks.end() && it->first <= r + r / 4) {
        const uint64_t sz = it->first;
        if (ctx->used.load() + sz > ctx->budget) {
            set_error("HBM budget exceeded");
            return SG_E_NOMEM;
        }
        *out = it->second;
        p.free_blocks.erase(it);
        p.cached -= sz;
        ctx->used.fetch_add(sz);
        return SG_OK;
    }
    if (ctx->used.load() + r > ctx->budget) {
        set_error("HBM budget exceeded");
        return SG_E_NOMEM;
    }
    const uint64_t room = ctx->budget - ctx->used.load() - r;
    if (p.cached > room) trim_locked(ctx, room);
    void *ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, r);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        trim_locked(ctx, 0);
        e = hipMalloc(&ptr, r);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
            return SG_E_NOMEM;
        }
    }
    p.sizes[ptr] = r;
    ctx->used.fetch_add(r);
    *out = ptr;
    return SG_OK;
}

void pool_free(Ctx *ctx, void *ptr) {
    if (!ptr) return;
    Pool &p = ctx->pool;
    std::lock_guard<std::mutex> lk(p.mu);
    auto it = p.sizes.find(ptr);
    if (it == p.sizes.end()) return;  // not ours
    const uint64_t sz = it->second;
    ctx->used.fetch_sub(sz);
    p.free_blocks.emplace(sz, ptr);
    p.cached += sz;
}

void pool_trim(Ctx *ctx, uint64_t keep) {
    std::lock_guard<std::mutex> lk(ctx->pool.mu);
    trim_locked(ctx, keep);
}

}  // namespace sg

// The voxel traversal export (sg_trace) without device allocation, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// sg_trace stages the ids and the traversals in device buffers it allocates per call;
// this variant stages them in a file-scope device array of kScratchBytes, one copy per
// GPU for the life of the process.  Host code never uses the array's name as a device
// address: sg_ctx_create looks up each device's address once (hipGetSymbolAddress, with
// that device current) and the entry point passes that address to the copies and the
// kernel.  Calls on one GPU share its array; the entry point serialises them with a
// per-device lock and drains its stream before releasing it, so calls from several
// threads of one process do not overlap on it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.hpp"

namespace sg {
namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
    unsigned char *ptr = nullptr;  // the device address of `scratch` on this device
    std::mutex mu;                 // held for the whole of a call that uses it
};
DeviceScratch g_scratch[kMaxDevices];
std::mutex g_setup_mu;

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

sg_status scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("device index beyond the staging table");
        return SG_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(g_setup_mu);
    if (g_scratch[device].ptr) return SG_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        return SG_E_DEVICE;
    }
    g_scratch[device].ptr = static_cast<unsigned char *>(p);
    return SG_OK;
}

uint64_t trace_noalloc_bytes(int64_t n_ids, int64_t cap) {
    const size_t n = (size_t)n_ids, c = (size_t)cap;
    return align256(sizeof(double) * n * c) + align256(sizeof(int) * n * c) + align256(sizeof(long long) * n) +
           align256(sizeof(int) * n);
}

}  // namespace sg

using namespace sg;

extern "C" {

uint64_t sg_trace_noalloc_capacity(void) { return kScratchBytes; }

sg_status sg_trace_noalloc(sg_scene *scene, int32_t kind, const int64_t *ids, int32_t n_ids, int32_t cap,
                           int32_t *voxels, double *dt, int32_t *count) {
    if (!scene || !ids || !voxels || !dt || !count) {
        set_error("NULL argument");
        return SG_E_INVALID;
    }
    if (kind < 0 || kind > 2) {
        set_error("bad trace kind");
        return SG_E_INVALID;
    }
    if (n_ids <= 0 || cap <= 0) {
        set_error("n_ids and cap must be > 0");
        return SG_E_INVALID;
    }
    const uint64_t need = trace_noalloc_bytes(n_ids, cap);
    if (need > kScratchBytes) {
        set_error("n_ids x cap needs " + std::to_string(need) + " bytes of staging, beyond the " +
                  std::to_string(kScratchBytes) + " of the allocation-free trace (about 12 bytes per slot)");
        return SG_E_INVALID;
    }
    Scene &s = *scene;
    Ctx *ctx = s.ctx;
    if (ctx->sticky.load()) {
        set_error("context is in a failed state");
        return SG_E_DEVICE;
    }
    const int64_t lim = kind == SG_TRACE_EDGE ? s.E : (kind == SG_TRACE_SUN ? s.N : s.npx);
    for (int i = 0; i < n_ids; ++i)
        if (ids[i] < 0 || ids[i] >= lim) {
            set_error("trace id out of range");
            return SG_E_INVALID;
        }
    DeviceScratch &ds = g_scratch[ctx->device];
    if (!ds.ptr) {  // sg_ctx_create sets it up; a context always has it
        set_error("staging area of the device not set up");
        return SG_E_STATE;
    }
    std::lock_guard<std::mutex> lk_scene(s.mu);
    std::lock_guard<std::mutex> lk(ds.mu);
    auto dev_fail = [&](const char *what, hipError_t e) {
        ctx->sticky.store(1);
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return SG_E_DEVICE;
    };
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return dev_fail("hipSetDevice", e);
    const size_t n = (size_t)n_ids, c = (size_t)cap;
    unsigned char *base = ds.ptr;
    double *d_dt = reinterpret_cast<double *>(base);
    int *d_vox = reinterpret_cast<int *>(base + align256(sizeof(double) * n * c));
    long long *d_ids = reinterpret_cast<long long *>(base + align256(sizeof(double) * n * c) +
                                                     align256(sizeof(int) * n * c));
    int *d_cnt = reinterpret_cast<int *>(reinterpret_cast<unsigned char *>(d_ids) + align256(sizeof(long long) * n));
    hipStream_t st = ctx->stream;
    if ((e = hipMemcpyAsync(d_ids, ids, sizeof(long long) * n, hipMemcpyHostToDevice, st)) != hipSuccess)
        return dev_fail("hipMemcpyAsync", e);
    launch_trace(s, st, kind, d_ids, n_ids, cap, d_vox, d_dt, d_cnt);  // writes every slot
    if ((e = hipGetLastError()) != hipSuccess) return dev_fail("k_trace", e);
    if ((e = hipMemcpyAsync(voxels, d_vox, sizeof(int) * n * c, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(dt, d_dt, sizeof(double) * n * c, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(count, d_cnt, sizeof(int) * n, hipMemcpyDeviceToHost, st)) != hipSuccess)
        return dev_fail("hipMemcpyAsync", e);
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return dev_fail("hipStreamSynchronize", e);
    return bounds_report();
}

}  // extern "C"

// Scattering nodes on the pixels' lines of sight (Sec. 2: the nodes of the scattering
// graph are path points of the lines of sight, taken at each layer of the medium or at
// constant distance intervals; Sec. 3, step 1 of the algorithm).
//
// One thread per pixel walks its line of sight from the surface point ((i + 1/2), (j +
// 1/2), 0) voxels along the view direction with the exact voxel walk, summing the chords'
// parameter lengths in order, and cuts the line into elements: one per layer of voxels
// crossed, or one per step.  Each element's node is the rounded middle point of the
// element, kept if it lies inside the box.  A count pass sizes the outputs, the host
// scans the counts, a fill pass writes them (the passes compute the same values).
#include "device.hpp"
#include "internal.hpp"

#include <cstring>
#include <string>

namespace sg {

namespace {

struct LosGeo {
    int nx, ny, nz, per, mode;
    long long dx, dy, dz;
    double h;                       // SG_LOS_STEP: the step in line-parameter units
    long long n_nodes = 0, n_el = 0;  // fill pass: the outputs' sizes (bounds-checked builds)
};

// The node of element [a, b] of the line from (px, py, 0): the rounded middle point (m =
// 0.5 (a + b), coordinate + floor(m D + 0.5)), wrapped on periodic axes; false when it is
// outside the box or on its outer planes.
__device__ bool element_node(const LosGeo &g, long long px, long long py, double a, double b, int q[3]) {
    const double m = 0.5 * (a + b);
    const long long P[3] = {px, py, 0}, D[3] = {g.dx, g.dy, g.dz};
    const long long W[3] = {(long long)g.nx * kFx, (long long)g.ny * kFx, (long long)g.nz * kFx};
    for (int k = 0; k < 3; ++k) {
        long long c = P[k] + (long long)floor(m * (double)D[k] + 0.5);
        if (k < 2 && (g.per >> k & 1)) {
            c %= W[k];
            if (c < 0) c += W[k];
        } else if (!(c > 0 && c < W[k])) {
            return false;
        }
        q[k] = (int)c;
    }
    return true;
}

// Count pass (fill = 0): elements and nodes per pixel.  Fill pass: node positions at
// node_off[p] ..., elements (node id or -1, end) at el_off[p] ...
__global__ __launch_bounds__(64) void k_los_place(LosGeo g, int fill, const long long *__restrict__ node_off,
                                                 const long long *__restrict__ el_off, long long *__restrict__ n_nodes,
                                                 long long *__restrict__ n_el, int *__restrict__ pos,
                                                 int *__restrict__ el_node, double *__restrict__ el_t) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= g.nx * g.ny) return;
    const long long px = (long long)(p % g.nx) * kFx + kFx / 2, py = (long long)(p / g.nx) * kFx + kFx / 2;
    long long nn = 0, ne = 0;
    const long long n0 = fill ? node_off[p] : 0, e0 = fill ? el_off[p] : 0;
    auto emit = [&](double a, double b) {
        int q[3];
        int id = -1;
        if (element_node(g, px, py, a, b, q)) {
            id = (int)(n0 + nn);
            if (fill && SG_IN(n0 + nn, g.n_nodes, 0x801)) {
                pos[3 * (n0 + nn)] = q[0];
                pos[3 * (n0 + nn) + 1] = q[1];
                pos[3 * (n0 + nn) + 2] = q[2];
            }
            ++nn;
        }
        if (fill && SG_IN(e0 + ne, g.n_el, 0x802)) {
            el_node[e0 + ne] = id;
            el_t[e0 + ne] = b;
        }
        ++ne;
    };
    double t = 0.0;
    if (g.mode == SG_LOS_LAYER) {
        int layer = -1;
        double a = 0.0;
        voxel_walk(g.nx, g.ny, g.nz, g.per, px, py, 0, g.dx, g.dy, g.dz, true,
                   [&](int, int, int z, long long num, long long den) {
                       if (z != layer) {
                           if (layer >= 0) emit(a, t);  // the previous layer's element ends here
                           layer = z;
                           a = t;
                       }
                       t = t + (double)num / (double)den;
                       return true;
                   });
        if (layer >= 0) emit(a, t);
    } else {
        voxel_walk(g.nx, g.ny, g.nz, g.per, px, py, 0, g.dx, g.dy, g.dz, true,
                   [&](int, int, int, long long num, long long den) {
                       t = t + (double)num / (double)den;
                       return true;
                   });
        const double t_exit = t;
        for (long long j = 0; (double)j * g.h < t_exit; ++j) {
            const double e = (double)(j + 1) * g.h;
            emit((double)j * g.h, e < t_exit ? e : t_exit);
        }
    }
    if (!fill) {
        n_nodes[p] = nn;
        n_el[p] = ne;
    }
}

sg_status lfail(sg_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

// device blocks from the context pool, released on scope exit
struct LosBufs {
    Ctx *ctx;
    std::vector<void *> blocks;
    explicit LosBufs(Ctx *c) : ctx(c) {}
    ~LosBufs() {
        for (void *p : blocks) pool_free(ctx, p);
    }
    template <class T>
    sg_status get(T **p, size_t n) {
        void *q = nullptr;
        const sg_status st = pool_alloc(ctx, std::max<size_t>(n, 1) * sizeof(T), &q);
        if (st != SG_OK) return st;
        blocks.push_back(q);
        *p = static_cast<T *>(q);
        return SG_OK;
    }
};

}  // namespace

}  // namespace sg

using namespace sg;

extern "C" sg_status sg_los_nodes(sg_ctx *ctx_, const sg_los_desc *d, void *hip_stream, int32_t *node_pos_fx,
                                  int64_t node_cap, int64_t *n_nodes, int64_t *los_ptr, int32_t *los_node,
                                  double *los_t, int64_t el_cap, int64_t *n_elements) {
    Ctx *ctx = reinterpret_cast<Ctx *>(ctx_);
    if (!ctx || !d || !n_nodes || !n_elements) return lfail(SG_E_INVALID, "NULL argument");
    if (d->abi_version != SG_ABI_VERSION) return lfail(SG_E_ABI, "los desc abi_version mismatch");
    if (ctx->sticky.load()) return lfail(SG_E_DEVICE, "context is in a failed state");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1 || d->nx > 1024 || d->ny > 1024 || d->nz > 1024)
        return lfail(SG_E_INVALID, "grid dimensions must be in 1..1024");
    if (!(d->voxel_m > 0.0) || !std::isfinite(d->voxel_m)) return lfail(SG_E_INVALID, "voxel_m must be > 0");
    if (d->view_dir[2] <= 0) return lfail(SG_E_INVALID, "view_dir needs a positive z component");
    for (int k = 0; k < 3; ++k)
        if (std::abs((long long)d->view_dir[k]) > (1LL << 22))
            return lfail(SG_E_INVALID, "direction components must be <= 2^22");
    if (d->periodic & ~(SG_PERIODIC_X | SG_PERIODIC_Y))
        return lfail(SG_E_INVALID, "periodic must combine SG_PERIODIC_X and SG_PERIODIC_Y");
    if (d->periodic) {
        const long long ax = std::llabs((long long)d->view_dir[0]), ay = std::llabs((long long)d->view_dir[1]),
                        az = d->view_dir[2];
        if ((long long)d->nz * (ax + ay + az) + 4 * az > 65536LL * az)
            return lfail(SG_E_INVALID, "with periodic axes the view rays must reach the top within 65536 voxels");
    }
    if (d->mode != SG_LOS_LAYER && d->mode != SG_LOS_STEP) return lfail(SG_E_INVALID, "mode must be SG_LOS_LAYER or SG_LOS_STEP");
    LosGeo g{d->nx, d->ny, d->nz, d->periodic, d->mode, d->view_dir[0], d->view_dir[1], d->view_dir[2], 0.0};
    if (d->mode == SG_LOS_STEP) {
        const double plen = std::sqrt((double)((long long)d->view_dir[0] * d->view_dir[0] +
                                               (long long)d->view_dir[1] * d->view_dir[1] +
                                               (long long)d->view_dir[2] * d->view_dir[2])) *
                            (d->voxel_m / 65536.0);
        if (!(d->step_m > 0.0) || !std::isfinite(d->step_m)) return lfail(SG_E_INVALID, "step_m must be > 0");
        g.h = d->step_m / plen;
        // elements per line: at most its length over the step; a line from the ground leaves
        // through the top at t = nz 2^16 / D_z at the latest (bounded or periodic)
        const double t_max = (double)d->nz * 65536.0 / (double)d->view_dir[2];
        if (!(t_max / g.h < 1e8)) return lfail(SG_E_INVALID, "step_m too small for the lines' length");
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return lfail(SG_E_DEVICE, "hipSetDevice failed");
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    const long long npx = (long long)d->nx * d->ny;
    LosBufs B(ctx);
    long long *cnt_n = nullptr, *cnt_e = nullptr, *off_n = nullptr, *off_e = nullptr;
    sg_status s;
    if ((s = B.get(&cnt_n, npx)) != SG_OK || (s = B.get(&cnt_e, npx)) != SG_OK) return s;
    auto dev = [&](const char *what, hipError_t err) {
        ctx->sticky.store(1);
        return lfail(SG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(err));
    };
    const int blocks = (int)((npx + 63) / 64);
    hipLaunchKernelGGL(k_los_place, dim3(blocks), dim3(64), 0, st, g, 0, (const long long *)nullptr,
                       (const long long *)nullptr, cnt_n, cnt_e, (int *)nullptr, (int *)nullptr, (double *)nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return dev("k_los_place", e);
    std::vector<long long> hn(npx), he(npx), on(npx + 1, 0), oe(npx + 1, 0);
    if ((e = hipMemcpyAsync(hn.data(), cnt_n, sizeof(long long) * npx, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(he.data(), cnt_e, sizeof(long long) * npx, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return dev("hipMemcpyAsync", e);
    for (long long p = 0; p < npx; ++p) {
        on[p + 1] = on[p] + hn[p];
        oe[p + 1] = oe[p] + he[p];
    }
    *n_nodes = on[npx];
    *n_elements = oe[npx];
    if (on[npx] >= (1LL << 31) - 1) return lfail(SG_E_INVALID, "too many nodes");
    if (los_ptr) std::memcpy(los_ptr, oe.data(), sizeof(int64_t) * (npx + 1));
    if (!node_pos_fx || !los_node || !los_t || node_cap < on[npx] || el_cap < oe[npx]) return SG_OK;  // a size query
    int *pos = nullptr, *el_node = nullptr;
    double *el_t = nullptr;
    if ((s = B.get(&off_n, npx)) != SG_OK || (s = B.get(&off_e, npx)) != SG_OK || (s = B.get(&pos, 3 * on[npx])) != SG_OK ||
        (s = B.get(&el_node, oe[npx])) != SG_OK || (s = B.get(&el_t, oe[npx])) != SG_OK)
        return s;
    if ((e = hipMemcpyAsync(off_n, on.data(), sizeof(long long) * npx, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(off_e, oe.data(), sizeof(long long) * npx, hipMemcpyHostToDevice, st)) != hipSuccess)
        return dev("hipMemcpyAsync", e);
    g.n_nodes = on[npx];
    g.n_el = oe[npx];
    hipLaunchKernelGGL(k_los_place, dim3(blocks), dim3(64), 0, st, g, 1, off_n, off_e, (long long *)nullptr,
                       (long long *)nullptr, pos, el_node, el_t);
    if ((e = hipGetLastError()) != hipSuccess) return dev("k_los_place", e);
    if ((on[npx] && (e = hipMemcpyAsync(node_pos_fx, pos, sizeof(int) * 3 * on[npx], hipMemcpyDeviceToHost, st)) != hipSuccess) ||
        (oe[npx] && (e = hipMemcpyAsync(los_node, el_node, sizeof(int) * oe[npx], hipMemcpyDeviceToHost, st)) != hipSuccess) ||
        (oe[npx] && (e = hipMemcpyAsync(los_t, el_t, sizeof(double) * oe[npx], hipMemcpyDeviceToHost, st)) != hipSuccess) ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return dev("hipMemcpyAsync", e);
    return bounds_report();
}

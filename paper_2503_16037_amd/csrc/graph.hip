// The scattering graph G(R, L) (Sec. 2, Eq. 4) of a scene's nodes, built on the
// device: which node pairs are coupled.
//
// Relative positions (Sec. 3): node positions are centred and scaled to unit
// standard deviation per axis; their projection on the principal axes that
// follows is a rotation and leaves every distance, hence every coupling,
// unchanged, so the couplings are evaluated on the scaled coordinates q.  The
// coupling C = sqrt(mu_i mu_j) / |q_i - q_j| (Eq. 4) is ranked through its square
//   k = (mu_i * mu_j) / ((u*u + v*v) + w*w),   (u, v, w) = q_i - q_j,
// in FP64 with exactly this operation order (no contraction: the selection is an
// integer decision taken from these values); surface nodes couple with
// albedo x the largest mu_s (Sec. 3) and two surface nodes never couple.
//
// Pruning.  A pair with k >= t satisfies |q_i - q_j|^2 <= mu_i mu_max / t, so for a
// threshold t every partner of node i lies in an axis-aligned box of voxels around
// it (half-width sqrt(mu_i mu_max / t) standard deviations per axis).  Box sizes
// differ by orders of magnitude (a strongly scattering node reaches far), so the
// cells of all boxes are flattened, node after node and within a box in increasing
// partner id (x fastest, then y, z, then the surface row), and evaluated one per
// thread; each thread finds its node by binary search in the prefix sum of the box
// sizes.  k is computed for the partners of higher id and the qualifying pairs are
// compacted in cell order (ballot and workgroup prefix, then the workgroups'
// prefix sum), so the candidate list is ordered by (i, j).  A stable radix sort on
// k (descending) then ranks them with equal couplings in (i, j) order.
//   threshold mode: t = c_min^2, keep k > t;
//   top-n mode: t = the lowest threshold whose boxes hold at most a fixed budget
//   of cells (bisection on the box volumes); if at least n pairs have k >= t, the
//   n best of them are the answer; otherwise every pair is streamed in node chunks
//   through a running best-n list.
// General nodes (the path points of the lines of sight, Sec. 2) are not tied to voxels:
// a volume node's partners are all nodes of higher id, and top-n requests go straight
// to the streamed ranking of every pair.
// The adjacency is assembled from the sorted directed pair codes (tail N + head).
// Scans, the evaluated-pair sum and the sorts are this file's own: a three-phase
// exclusive scan, and a stable least-significant-digit radix sort (8-bit digits, one
// wavefront per tile of 4096 keys, a key's rank among equal digits of its 64-key round
// from eight ballots).
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <memory>
#include <string>
#include <vector>

#include "device.hpp"
#include "internal.hpp"

#pragma clang fp contract(off)

namespace sg {

namespace {

// box cells a candidate pass may visit: 2^26 first, then 2^28 and 2^30 when the fitted
// threshold leaves fewer than n candidates (SG_GRAPH_CELL_BUDGET fixes a single budget,
// e.g. to exercise the streamed path on small inputs)
std::vector<unsigned long long> cell_budgets() {
    const char *v = std::getenv("SG_GRAPH_CELL_BUDGET");
    const unsigned long long b = v ? std::strtoull(v, nullptr, 10) : 0ull;
    if (b) return {b};
    return {1ull << 26, 1ull << 28, 1ull << 30};
}

struct Geo {
    int nx, ny, nz, surface;
    int general;               // 1: general volume nodes (every pair ranked), 0: one per voxel
    long long nvox, nvol, N;   // voxels, volume nodes, all nodes
    double mean[3], sd[3];  // per-axis centre and scale (sd = 0: the axis is ignored)
    double mu_max;
};

sg_status gfail(sg_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

#define GHIP(call)                                                                                   \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) {                                                                      \
            ctx->sticky.store(1);                                                                    \
            return gfail(SG_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));            \
        }                                                                                            \
    } while (0)
#define GTRY(x)                          \
    do {                                 \
        sg_status st_ = (x);             \
        if (st_ != SG_OK) return st_;    \
    } while (0)

// device blocks from the context pool, released on scope exit
struct Dev {
    Ctx *ctx;
    std::vector<void *> blocks;
    explicit Dev(Ctx *c) : ctx(c) {}
    ~Dev() {
        for (void *p : blocks) pool_free(ctx, p);
    }
    template <class T>
    sg_status get(T **p, size_t n) {
        void *q = nullptr;
        GTRY(pool_alloc(ctx, std::max<size_t>(n, 1) * sizeof(T), &q));
        blocks.push_back(q);
        *p = static_cast<T *>(q);
        return SG_OK;
    }
    void release(void *p) {  // one block back to the pool before scope exit
        for (auto it = blocks.begin(); it != blocks.end(); ++it)
            if (*it == p) {
                pool_free(ctx, p);
                blocks.erase(it);
                return;
            }
    }
};

// ---- kernels ---------------------------------------------------------------------------

// fixed-point position, coupling coefficient and scaled coordinates of every node; a
// general node couples with the mu_s of the voxel holding it
__global__ void k_graph_nodes(Geo g, const int *__restrict__ pos, const float *__restrict__ mu_s,
                              const float *__restrict__ albedo, long long *__restrict__ P, double *__restrict__ q,
                              double *__restrict__ mu) {
#pragma clang fp contract(off)
    const long long l = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (l >= g.N) return;
    long long p[3];
    if (l < g.nvol) {
        p[0] = pos[3 * l];
        p[1] = pos[3 * l + 1];
        p[2] = pos[3 * l + 2];
        const long long v =
            g.general ? p[0] / kFx + (long long)g.nx * (p[1] / kFx + (long long)g.ny * (p[2] / kFx)) : l;
        mu[l] = (double)mu_s[v];
    } else {
        const long long c = l - g.nvol;
        p[0] = (c % g.nx) * kFx + kFx / 2;
        p[1] = (c / g.nx) * kFx + kFx / 2;
        p[2] = 0;
        mu[l] = (double)albedo[c] * g.mu_max;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        P[3 * l + a] = p[a];
        q[3 * l + a] = g.sd[a] > 0.0 ? ((double)p[a] - g.mean[a]) / g.sd[a] : 0.0;
    }
}

__device__ __forceinline__ double pair_key(const double *__restrict__ q, const double *__restrict__ mu, long long i,
                                           long long j) {
#pragma clang fp contract(off)
    const double u = q[3 * i] - q[3 * j], v = q[3 * i + 1] - q[3 * j + 1], w = q[3 * i + 2] - q[3 * j + 2];
    const double d2 = (u * u + v * v) + w * w;
    return (mu[i] * mu[j]) / d2;
}

// The box of node i's possible partners at threshold t: voxel index ranges per axis
// (lo > hi: empty) and whether the surface row is inside.
struct Box {
    long long lo[3], hi[3];
    bool surf;
};

__device__ __forceinline__ Box node_box(const Geo &g, const long long *__restrict__ P, const double *__restrict__ mu,
                                        long long i, double t) {
    Box b;
    const double mi = mu[i];
    const long long n[3] = {g.nx, g.ny, g.nz};
    // k = 0 for every pair of this node, or a surface node (its pairs with volume
    // nodes are found from the volume side; two surface nodes never couple)
    if (!(mi > 0.0) || i >= g.nvol) {
        for (int a = 0; a < 3; ++a) { b.lo[a] = 1; b.hi[a] = 0; }
        b.surf = false;
        return b;
    }
    // radius in standard deviations; t = 0 (or an overflow): unbounded
    const double rho = t > 0.0 ? sqrt(mi * g.mu_max / t) * (1.0 + 1e-9) : __builtin_inf();
    bool low_z = false;
    for (int a = 0; a < 3; ++a) {
        const double r = g.sd[a] > 0.0 ? rho * g.sd[a] + 1.0 : __builtin_inf();  // fixed-point units
        const double pa = (double)P[3 * i + a];
        const double flo = floor((pa - r) / (double)kFx), fhi = floor((pa + r) / (double)kFx);
        b.lo[a] = flo < 0.0 ? 0 : (flo > (double)(n[a] - 1) ? n[a] : (long long)flo);
        b.hi[a] = fhi > (double)(n[a] - 1) ? n[a] - 1 : (fhi < 0.0 ? -1 : (long long)fhi);
        if (a == 2) low_z = pa - r <= 0.0;
    }
    b.surf = g.surface && low_z;
    return b;
}

__device__ __forceinline__ unsigned long long box_cells(const Box &b) {
    unsigned long long v = 1;
    for (int a = 0; a < 3; ++a) v *= b.hi[a] >= b.lo[a] ? (unsigned long long)(b.hi[a] - b.lo[a] + 1) : 0ull;
    if (b.surf) v += (unsigned long long)(b.hi[0] >= b.lo[0] ? b.hi[0] - b.lo[0] + 1 : 0) *
                     (unsigned long long)(b.hi[1] >= b.lo[1] ? b.hi[1] - b.lo[1] + 1 : 0);
    return v;
}

// total box cells of all nodes at threshold t (one thread per node)
__global__ void k_graph_cells(Geo g, const long long *__restrict__ P, const double *__restrict__ mu, double t,
                              unsigned long long *__restrict__ total) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    __shared__ unsigned long long wsum[4];
    unsigned long long v = 0;
    if (i < g.N) v = box_cells(node_box(g, P, mu, i, t));
    // wavefront sums, then one atomic per workgroup
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(total, wsum[0] + wsum[1] + wsum[2] + wsum[3]);
}

// Boxes of nodes n0 + r (r < n) at threshold t, stored as (lo x, lo y, lo z, extent
// x, y, z, surface row, 0), and their cell counts (volume cells + surface cells);
// cells[n] = 0 closes the array for the exclusive scan.
__global__ void k_graph_boxes(Geo g, const long long *__restrict__ P, const double *__restrict__ mu, double t,
                              long long n0, long long n, int *__restrict__ box, unsigned long long *__restrict__ cells) {
    const long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (r > n) return;
    if (r == n) {
        cells[n] = 0;
        return;
    }
    if (g.general) {  // every partner of higher id: the range n0 + r + 1 .. N - 1
        const long long i = n0 + r;
        int *o = box + 8 * r;
        for (int a = 0; a < 8; ++a) o[a] = 0;
        cells[r] = i < g.nvol && mu[i] > 0.0 ? (unsigned long long)(g.N - 1 - i) : 0ull;
        return;
    }
    const Box b = node_box(g, P, mu, n0 + r, t);
    long long e[3];
    for (int a = 0; a < 3; ++a) e[a] = b.hi[a] >= b.lo[a] ? b.hi[a] - b.lo[a] + 1 : 0;
    const unsigned long long nv = (unsigned long long)e[0] * e[1] * e[2];
    const unsigned long long ns = b.surf ? (unsigned long long)e[0] * e[1] : 0ull;
    int *o = box + 8 * r;
    o[0] = (int)b.lo[0]; o[1] = (int)b.lo[1]; o[2] = (int)b.lo[2];
    o[3] = (int)e[0]; o[4] = (int)e[1]; o[5] = (int)e[2];
    o[6] = b.surf ? 1 : 0; o[7] = 0;
    cells[r] = nv + ns;
}

constexpr int kEvalRounds = 8;  // a workgroup covers kEvalRounds x 256 consecutive cells

// last r in [a, b) with coff[r] <= c (coff ascending, coff[a] <= c)
__device__ __forceinline__ long long owner(const unsigned long long *__restrict__ coff, long long a, long long b,
                                           unsigned long long c) {
    while (b - a > 1) {
        const long long m = (a + b) >> 1;
        if (coff[m] <= c) a = m;
        else b = m;
    }
    return a;
}

// The cells of all boxes, flattened in node order (a node's cells in increasing
// partner id), one thread per cell: the partner j > i is evaluated and the pairs
// with k >= t (strict: k > t), k > 0 are counted per workgroup (kFill = false:
// bcount) or written in cell order at the workgroup's offset (kFill = true), so the
// list stays ordered by (i, j).  bev: the evaluated pairs per workgroup (count pass).
template <bool kFill>
__global__ __launch_bounds__(256) void k_graph_eval(Geo g, const double *__restrict__ q,
                                                    const double *__restrict__ mu, double t, int strict, long long n0,
                                                    long long n, const int *__restrict__ box,
                                                    const unsigned long long *__restrict__ coff, unsigned long long T,
                                                    unsigned long long *__restrict__ bcount,
                                                    const unsigned long long *__restrict__ boff,
                                                    double *__restrict__ keys, unsigned long long *__restrict__ codes,
                                                    unsigned long long *__restrict__ bev) {
    constexpr int kCells = kEvalRounds * 256;
    __shared__ unsigned int wcnt[4];
    __shared__ unsigned long long wev[4];
    __shared__ long long range[2];
    __shared__ unsigned long long scoff[kCells];  // box starts of the workgroup's nodes, when they fit
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const unsigned long long base = (unsigned long long)blockIdx.x * kCells;
    unsigned long long run = kFill ? boff[blockIdx.x] : 0ull, ev = 0ull;
    // the nodes owning this workgroup's cells: [fb, lb]
    if (threadIdx.x == 0) {
        const long long fb = owner(coff, 0, n, base);
        const unsigned long long cl = base + kCells - 1 < T ? base + kCells - 1 : T - 1;
        range[0] = fb;
        range[1] = owner(coff, fb, n, cl);
    }
    __syncthreads();
    const long long fb = range[0], lb = range[1];
    const bool staged = lb - fb + 1 <= kCells;
    if (staged)
        for (long long x = threadIdx.x; x <= lb - fb; x += blockDim.x) scoff[x] = coff[fb + x];
    __syncthreads();
    for (int rd = 0; rd < kEvalRounds; ++rd) {
        const unsigned long long c0 = base + (unsigned long long)rd * 256 + (unsigned long long)w * 64;
        const unsigned long long c = c0 + lane;
        bool ok = false, eval = false;
        double k = 0.0;
        long long i = 0, j = 0;
        if (c < T) {
            {
                long long r;
                if (staged) {  // last x with scoff[x] <= c, in LDS
                    long long a = 0, b = lb - fb + 1;
                    while (b - a > 1) {
                        const long long m2 = (a + b) >> 1;
                        if (scoff[m2] <= c) a = m2;
                        else b = m2;
                    }
                    r = fb + a;
                } else {
                    r = owner(coff, fb, lb + 1, c);
                }
                const int *o = box + 8 * r;
                // a box has at most 1024^3 + 1024^2 cells: 32-bit index arithmetic
                const unsigned bx = (unsigned)o[3], by = (unsigned)o[4], bz = (unsigned)o[5];
                const unsigned nv = bx * by * bz;
                const unsigned lc = (unsigned)(c - (staged ? scoff[r - fb] : coff[r]));
                i = n0 + r;
                if (g.general) {
                    j = i + 1 + lc;
                } else if (lc < nv) {
                    const unsigned yz = lc / bx, cx = lc - yz * bx, cz = yz / by, cy = yz - cz * by;
                    j = ((long long)o[0] + cx) + (long long)g.nx * (((long long)o[1] + cy) + (long long)g.ny * ((long long)o[2] + cz));
                } else {
                    const unsigned sl = lc - nv, sy = sl / bx, sx = sl - sy * bx;
                    j = g.nvol + ((long long)o[0] + sx) + (long long)g.nx * ((long long)o[1] + sy);
                }
                eval = j > i && SG_IN(j, g.N, 0x701);
                if (eval) {
                    k = pair_key(q, mu, i, j);
                    ok = k > 0.0 && (strict ? k > t : k >= t);
                }
            }
        }
        const unsigned long long m = __ballot(ok);
        if (!kFill) ev += __popcll(__ballot(eval));
        if (lane == 0) wcnt[w] = (unsigned int)__popcll(m);
        __syncthreads();
        unsigned long long before = 0, total = 0;
        for (int v = 0; v < 4; ++v) {
            before += v < w ? wcnt[v] : 0u;
            total += wcnt[v];
        }
        if (kFill && ok) {
            const unsigned long long at = run + before + __popcll(m & ((1ull << lane) - 1ull));
            if (SG_IN(at, boff[gridDim.x], 0x702)) {
                keys[at] = k;
                codes[at] = (unsigned long long)i * (unsigned long long)g.N + (unsigned long long)j;
            }
        }
        run += total;
        __syncthreads();  // wcnt is rewritten by the next round
    }
    if (!kFill) {
        if (lane == 0) wev[w] = ev;
        __syncthreads();
        if (threadIdx.x == 0) {
            bcount[blockIdx.x] = run;
            bev[blockIdx.x] = wev[0] + wev[1] + wev[2] + wev[3];
        }
    }
}

// directed pair codes (tail N + head) of the selected pairs, both directions
__global__ void k_graph_directed(long long n, long long N, const unsigned long long *__restrict__ pair,
                                 unsigned long long *__restrict__ dir) {
    const long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const unsigned long long c = pair[s];
    const unsigned long long i = c / (unsigned long long)N, j = c % (unsigned long long)N;
    dir[2 * s] = i * (unsigned long long)N + j;
    dir[2 * s + 1] = j * (unsigned long long)N + i;
}

__global__ void k_graph_heads(long long E, long long N, const unsigned long long *__restrict__ dir,
                              int *__restrict__ head) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e < E) head[e] = (int)(dir[e] % (unsigned long long)N);
}

// row pointers from the sorted directed codes: ptr[l] = first e with dir[e] >= l N
__global__ void k_graph_rowptr(long long N, long long E, const unsigned long long *__restrict__ dir,
                               long long *__restrict__ ptr) {
    const long long l = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (l > N) return;
    const unsigned long long key = (unsigned long long)l * (unsigned long long)N;
    long long a = 0, b = E;  // dir[0, a) < key <= dir[b, E)
    while (a < b) {
        const long long m = (a + b) >> 1;
        if (dir[m] < key) a = m + 1;
        else b = m;
    }
    ptr[l] = a;
}

// ---- scans, sums and sorts of the builder -----------------------------------------------

constexpr int kScanItems = 8;                 // consecutive items per thread
constexpr int kScanBlock = 256 * kScanItems;  // items per workgroup

// exclusive prefix of v over the workgroup's 256 threads; total = the workgroup's sum
template <class T>
__device__ __forceinline__ T block_exclusive(T v, T *lds, T &total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[w] = x;
    __syncthreads();
    T before = 0;
    total = 0;
    for (int k = 0; k < 4; ++k) {
        if (k < w) before += lds[k];
        total += lds[k];
    }
    return before + x - v;
}

// pass 1: each workgroup's items scanned (exclusive, plus init), its total to tsum
template <class T>
__global__ __launch_bounds__(256) void k_scan_local(const T *__restrict__ in, T *__restrict__ out, long long n, T init,
                                                    T *__restrict__ tsum) {
    __shared__ T lds[4];
    const long long i0 = (long long)blockIdx.x * kScanBlock + (long long)threadIdx.x * kScanItems;
    T v[kScanItems];
    T sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = i0 + j < n ? in[i0 + j] : (T)0;
        sum += v[j];
    }
    T total;
    T ex = block_exclusive(sum, lds, total) + init;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (i0 + j < n) out[i0 + j] = ex;
        ex += v[j];
    }
    if (tsum && threadIdx.x == 0) tsum[blockIdx.x] = total;
}

// pass 3: the workgroups' offsets added
template <class T>
__global__ void k_scan_add(T *__restrict__ out, long long n, const T *__restrict__ off) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) out[i] += off[i / kScanBlock];
}

// sum of n values, one atomic per workgroup (integer: the order does not matter)
__global__ __launch_bounds__(256) void k_sum_u64(const unsigned long long *__restrict__ in, long long n,
                                                 unsigned long long *__restrict__ out) {
    __shared__ unsigned long long lds[4];
    unsigned long long v = 0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        v += in[i];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, lds[0] + lds[1] + lds[2] + lds[3]);
}

constexpr int kRsItems = 16;             // keys per lane in a tile
constexpr int kRsTile = 64 * kRsItems;  // keys per tile (one wavefront; staged in LDS by the scatter)

// digit counts of each tile, digit-major: hist[digit * ntiles + tile]
__global__ __launch_bounds__(256) void k_rs_hist(const unsigned long long *__restrict__ keys, long long n, int bit,
                                                 long long ntiles, unsigned *__restrict__ hist) {
    __shared__ unsigned cnt[4][256];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long tile = (long long)blockIdx.x * 4 + w;
    for (int d = lane; d < 256; d += 64) cnt[w][d] = 0u;
    __syncthreads();
    if (tile < ntiles) {
        const long long base = tile * kRsTile;
        for (int r = 0; r < kRsItems; ++r) {
            const long long i = base + (long long)r * 64 + lane;
            if (i < n) atomicAdd(&cnt[w][(unsigned)(keys[i] >> bit) & 255u], 1u);
        }
    }
    __syncthreads();
    if (tile < ntiles)
        for (int d = lane; d < 256; d += 64) hist[(long long)d * ntiles + tile] = cnt[w][d];
}

// Stable scatter by one digit: tile t's keys with digit d go to off[d * ntiles + t] onward,
// in their order.  The tile is first sorted by digit in the wavefront's LDS (a stable
// counting sort: local digit starts from the tile's counts, then round r of the tile, keys
// base + 64 r + lane, ranked among the round's keys of its digit by the ballots of the
// digit's eight bits, after the digit's running count), then written out in that order, so
// the lanes holding one digit store to consecutive addresses.  Same order as placing every
// key straight at its global position.
__global__ __launch_bounds__(256) void k_rs_scatter(const unsigned long long *__restrict__ kin,
                                                    const unsigned long long *__restrict__ vin,
                                                    unsigned long long *__restrict__ kout,
                                                    unsigned long long *__restrict__ vout, long long n, int bit,
                                                    long long ntiles, const unsigned *__restrict__ off,
                                                    const unsigned *__restrict__ hist) {
    __shared__ unsigned gbase[4][256], lbase[4][256], run[4][256];
    __shared__ unsigned long long sk[4][kRsTile], sv[4][kRsTile];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long tile = (long long)blockIdx.x * 4 + w;
    if (tile >= ntiles) return;  // no barrier below: each wavefront works on its own LDS rows
    // the tile's digit counts, four consecutive digits per lane, and their exclusive scan
    unsigned c[4], sum = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int d = 4 * lane + j;
        c[j] = hist[(long long)d * ntiles + tile];
        gbase[w][d] = off[(long long)d * ntiles + tile];
        sum += c[j];
    }
    unsigned incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    unsigned start = incl - sum;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int d = 4 * lane + j;
        lbase[w][d] = start;
        run[w][d] = start;
        start += c[j];
    }
    __builtin_amdgcn_wave_barrier();
    const long long base = tile * kRsTile;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int r = 0; r < kRsItems; ++r) {
        const long long i = base + (long long)r * 64 + lane;
        const bool ok = i < n;
        const unsigned long long k = ok ? kin[i] : 0ull;
        const unsigned dg = (unsigned)(k >> bit) & 255u;
        unsigned long long peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const unsigned long long m = __ballot(ok && ((dg >> b) & 1u));
            peers &= ((dg >> b) & 1u) ? m : ~m;
        }
        const unsigned before = (unsigned)__popcll(peers & below);
        const unsigned p = ok ? run[w][dg] + before : 0u;
        __builtin_amdgcn_wave_barrier();
        if (ok && before == 0u) run[w][dg] = p + (unsigned)__popcll(peers);  // the digit's first lane
        if (ok && SG_IN(p, kRsTile, 0x703)) {
            sk[w][p] = k;
            if (vin) sv[w][p] = vin[i];
        }
        __builtin_amdgcn_wave_barrier();
    }
    // write-out in digit order: local position j holds the (j - lbase[digit])-th key of its
    // digit in this tile
    const int nk = (int)min((long long)kRsTile, n - base);
    for (int j = lane; j < nk; j += 64) {
        const unsigned long long k = sk[w][j];
        const unsigned dg = (unsigned)(k >> bit) & 255u;
        const unsigned g = gbase[w][dg] + ((unsigned)j - lbase[w][dg]);
        if (SG_IN(g, n, 0x704)) {
            kout[g] = k;
            if (vin) vout[g] = sv[w][j];
        }
    }
}

// descending doubles (all positive) as ascending integers, and back
__global__ void k_desc_bits(unsigned long long *__restrict__ a, long long n) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) a[i] = ~a[i];
}

unsigned blocks_for(long long n, int threads) { return (unsigned)std::max<long long>(1, (n + threads - 1) / threads); }

// ---- host driver ---------------------------------------------------------------------

struct Builder {
    Ctx *ctx;
    hipStream_t st;
    Geo g;
    Dev dev;
    long long *P = nullptr;
    double *q = nullptr, *mu = nullptr;
    unsigned long long *scal = nullptr;  // [0] cell total, [1] evaluated pairs
    // build statistics: candidate passes, summed kernel times (HIP event pairs)
    int passes = 0;
    unsigned long long evals = 0;  // pairs evaluated by the count passes
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pairs, ev_sort;
    Builder(Ctx *c, hipStream_t s) : ctx(c), st(s), dev(c) {}
    ~Builder() {
        for (auto &e : ev_pairs) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
        for (auto &e : ev_sort) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    }
    // an event pair recording around whatever the caller enqueues next
    std::pair<hipEvent_t, hipEvent_t> *mark(std::vector<std::pair<hipEvent_t, hipEvent_t>> &v) {
        hipEvent_t a = nullptr, b = nullptr;
        if (hipEventCreate(&a) != hipSuccess) return nullptr;
        if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return nullptr; }
        v.push_back({a, b});
        (void)hipEventRecord(a, st);
        return &v.back();
    }
    static double total_ms(const std::vector<std::pair<hipEvent_t, hipEvent_t>> &v) {
        double t = 0.0;
        for (auto &e : v) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) t += ms;
        }
        return t;
    }

    sg_status cells(double t, unsigned long long &out) {
        GHIP(hipMemsetAsync(scal, 0, sizeof(unsigned long long), st));
        hipLaunchKernelGGL(k_graph_cells, dim3(blocks_for(g.N, 256)), dim3(256), 0, st, g, P, mu, t, scal);
        GHIP(hipGetLastError());
        GHIP(hipMemcpyAsync(&out, scal, sizeof(out), hipMemcpyDeviceToHost, st));
        GHIP(hipStreamSynchronize(st));
        return SG_OK;
    }

    // candidates of nodes [n0, n1) at threshold t, appended after `have` entries of
    // (keys, codes), which are reallocated to fit
    sg_status pairs(double t, int strict, long long n0, long long n1, double *&keys, unsigned long long *&codes,
                    unsigned long long &have) {
        const long long n = n1 - n0;
        if (n <= 0) return SG_OK;
        Dev tmp(ctx);
        int *box = nullptr;
        unsigned long long *cells = nullptr, *coff = nullptr;
        GTRY(tmp.get(&box, 8 * n));
        GTRY(tmp.get(&cells, n + 1));
        GTRY(tmp.get(&coff, n + 1));
        hipLaunchKernelGGL(k_graph_boxes, dim3(blocks_for(n + 1, 256)), dim3(256), 0, st, g, P, mu, t, n0, n, box,
                           cells);
        GHIP(hipGetLastError());
        GTRY(scan<unsigned long long>(cells, coff, n + 1, 0ull));
        unsigned long long T = 0;
        GHIP(hipMemcpyAsync(&T, coff + n, sizeof(T), hipMemcpyDeviceToHost, st));
        GHIP(hipStreamSynchronize(st));
        if (T == 0) return SG_OK;
        const unsigned long long per = (unsigned long long)kEvalRounds * 256;
        const unsigned long long nb = (T + per - 1) / per;
        if (nb >= (1ull << 31)) return gfail(SG_E_NOMEM, "coupling boxes too large");
        unsigned long long *bcount = nullptr, *boff = nullptr, *bev = nullptr, *evsum = nullptr;
        GTRY(tmp.get(&bcount, nb + 1));
        GTRY(tmp.get(&boff, nb + 1));
        GTRY(tmp.get(&bev, nb));
        GTRY(tmp.get(&evsum, 1));
        GHIP(hipMemsetAsync(bcount + nb, 0, sizeof(unsigned long long), st));
        ++passes;
        auto *e0 = mark(ev_pairs);
        hipLaunchKernelGGL((k_graph_eval<false>), dim3((unsigned)nb), dim3(256), 0, st, g, q, mu, t, strict, n0, n,
                           box, coff, T, bcount, nullptr, nullptr, nullptr, bev);
        if (e0) (void)hipEventRecord(e0->second, st);
        GHIP(hipGetLastError());
        // boff = have + exclusive sum of the workgroup counts; boff[nb] = the new total
        GTRY(scan<unsigned long long>(bcount, boff, (long long)nb + 1, (unsigned long long)have));
        GHIP(hipMemsetAsync(evsum, 0, sizeof(unsigned long long), st));
        hipLaunchKernelGGL(k_sum_u64, dim3((unsigned)std::min<unsigned long long>((nb + 255) / 256, 1024)), dim3(256), 0,
                           st, bev, (long long)nb, evsum);
        GHIP(hipGetLastError());
        unsigned long long total = 0, ev = 0;
        GHIP(hipMemcpyAsync(&total, boff + nb, sizeof(total), hipMemcpyDeviceToHost, st));
        GHIP(hipMemcpyAsync(&ev, evsum, sizeof(ev), hipMemcpyDeviceToHost, st));
        GHIP(hipStreamSynchronize(st));
        evals += ev;
        if (total >= (1ull << 31)) return gfail(SG_E_NOMEM, "more than 2^31 coupling candidates");
        if (total > have) {
            double *nk = nullptr;
            unsigned long long *nc = nullptr;
            GTRY(dev.get(&nk, total));
            GTRY(dev.get(&nc, total));
            if (have) {
                GHIP(hipMemcpyAsync(nk, keys, sizeof(double) * have, hipMemcpyDeviceToDevice, st));
                GHIP(hipMemcpyAsync(nc, codes, sizeof(unsigned long long) * have, hipMemcpyDeviceToDevice, st));
            }
            auto *e1 = mark(ev_pairs);
            hipLaunchKernelGGL((k_graph_eval<true>), dim3((unsigned)nb), dim3(256), 0, st, g, q, mu, t, strict, n0, n,
                               box, coff, T, nullptr, boff, nk, nc, nullptr);
            if (e1) (void)hipEventRecord(e1->second, st);
            GHIP(hipGetLastError());
            GHIP(hipStreamSynchronize(st));  // the scratch above is released at return
            dev.release(keys);
            dev.release(codes);
            keys = nk;
            codes = nc;
        }
        have = total;
        return SG_OK;
    }

    // out[i] = init + in[0] + ... + in[i - 1] for i < n (in and out distinct)
    template <class T>
    sg_status scan(const T *in, T *out, long long n, T init) {
        if (n <= 0) return SG_OK;
        const long long nb = (n + kScanBlock - 1) / kScanBlock;
        if (nb == 1) {
            hipLaunchKernelGGL((k_scan_local<T>), dim3(1), dim3(256), 0, st, in, out, n, init, (T *)nullptr);
            GHIP(hipGetLastError());
            return SG_OK;
        }
        Dev tmp(ctx);
        T *tsum = nullptr, *toff = nullptr;
        GTRY(tmp.get(&tsum, nb));
        GTRY(tmp.get(&toff, nb));
        hipLaunchKernelGGL((k_scan_local<T>), dim3((unsigned)nb), dim3(256), 0, st, in, out, n, (T)0, tsum);
        GHIP(hipGetLastError());
        GTRY(scan<T>(tsum, toff, nb, init));
        hipLaunchKernelGGL((k_scan_add<T>), dim3(blocks_for(n, 256)), dim3(256), 0, st, out, n, (const T *)toff);
        GHIP(hipGetLastError());
        GHIP(hipStreamSynchronize(st));  // the scratch above is released at return
        return SG_OK;
    }

    // stable ascending sort of n 64-bit keys, with their values when vals is given, in place
    // (eight passes of 8-bit digits through a second buffer)
    sg_status sort_u64(unsigned long long *keys, unsigned long long *vals, long long n) {
        if (n < 2) return SG_OK;
        Dev tmp(ctx);
        const long long ntiles = (n + kRsTile - 1) / kRsTile;
        unsigned long long *k2 = nullptr, *v2 = nullptr;
        unsigned *hist = nullptr, *off = nullptr;
        GTRY(tmp.get(&k2, n));
        if (vals) GTRY(tmp.get(&v2, n));
        GTRY(tmp.get(&hist, 256 * ntiles));
        GTRY(tmp.get(&off, 256 * ntiles));
        const unsigned nblk = (unsigned)((ntiles + 3) / 4);
        unsigned long long *ka = keys, *va = vals, *kb = k2, *vb = v2;
        for (int bit = 0; bit < 64; bit += 8) {
            hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(256), 0, st, ka, n, bit, ntiles, hist);
            GHIP(hipGetLastError());
            GTRY(scan<unsigned>(hist, off, 256 * ntiles, 0u));
            hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(256), 0, st, ka, va, kb, vb, n, bit, ntiles,
                               (const unsigned *)off, (const unsigned *)hist);
            GHIP(hipGetLastError());
            std::swap(ka, kb);
            std::swap(va, vb);
        }
        GHIP(hipStreamSynchronize(st));  // eight passes: the result is back in keys / vals
        return SG_OK;
    }

    // stable sort by key, descending (equal keys keep their order), in place; the keys are
    // positive, so their bit patterns complemented sort ascending in the same order
    sg_status sort_desc(double *&keys, unsigned long long *&codes, unsigned long long n) {
        if (n < 2) return SG_OK;
        auto *k = reinterpret_cast<unsigned long long *>(keys);
        auto *e = mark(ev_sort);
        hipLaunchKernelGGL(k_desc_bits, dim3(blocks_for((long long)n, 256)), dim3(256), 0, st, k, (long long)n);
        GTRY(sort_u64(k, codes, (long long)n));
        hipLaunchKernelGGL(k_desc_bits, dim3(blocks_for((long long)n, 256)), dim3(256), 0, st, k, (long long)n);
        if (e) (void)hipEventRecord(e->second, st);
        GHIP(hipGetLastError());
        GHIP(hipStreamSynchronize(st));
        return SG_OK;
    }
};

}  // namespace

sg_status graph_build(Ctx *ctx, const sg_graph_desc *d, hipStream_t st, int64_t *adj_ptr, int32_t *adj_idx,
                      int64_t cap, int64_t *n_edges, sg_graph_info *info) {
    const auto t_start = std::chrono::steady_clock::now();
    if (!d) return gfail(SG_E_INVALID, "desc is NULL");
    if (d->abi_version != SG_ABI_VERSION) return gfail(SG_E_ABI, "graph desc abi_version mismatch");
    if (!n_edges) return gfail(SG_E_INVALID, "n_edges is NULL");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1 || d->nx > 1024 || d->ny > 1024 || d->nz > 1024)
        return gfail(SG_E_INVALID, "grid dimensions must be in 1..1024");
    const bool general = d->n_nodes > 0;
    if (d->n_nodes < 0) return gfail(SG_E_INVALID, "n_nodes must be >= 0");
    if (!d->mu_s || !(general ? d->node_pos_fx : d->vol_pos_fx) || (d->surface_nodes && !d->surf_albedo))
        return gfail(SG_E_INVALID, "a required array is NULL");
    if (d->n_pairs < 0) return gfail(SG_E_INVALID, "n_pairs must be >= 0");
    if (d->n_pairs == 0 && !(d->c_min >= 0.0 && std::isfinite(d->c_min)))
        return gfail(SG_E_INVALID, "c_min must be finite and >= 0");
    const long long nvox = (long long)d->nx * d->ny * d->nz;
    const long long nvol = general ? (long long)d->n_nodes : nvox;
    const long long N = nvol + (d->surface_nodes ? (long long)d->nx * d->ny : 0);
    if (N >= (1LL << 31)) return gfail(SG_E_INVALID, "too many nodes");
    float mmax = 0.0f;
    for (long long v = 0; v < nvox; ++v) {
        const float a = d->mu_s[v];
        if (!(a >= 0.0f) || !std::isfinite(a)) return gfail(SG_E_INVALID, "mu_s must be finite and >= 0");
        mmax = std::max(mmax, a);
    }
    if (d->surface_nodes)
        for (long long c = 0; c < (long long)d->nx * d->ny; ++c)
            if (!(d->surf_albedo[c] >= 0.0f) || !(d->surf_albedo[c] <= 1.0f))
                return gfail(SG_E_INVALID, "surf_albedo must be in [0, 1]");
    // exact integer moments of the positions, per axis
    __int128 s1[3] = {0, 0, 0}, s2[3] = {0, 0, 0};
    const long long W[3] = {(long long)d->nx * kFx, (long long)d->ny * kFx, (long long)d->nz * kFx};
    for (long long v = 0; v < nvol; ++v) {
        const long long c[3] = {v % d->nx, (v / d->nx) % d->ny, v / ((long long)d->nx * d->ny)};
        for (int a = 0; a < 3; ++a) {
            const long long p = general ? d->node_pos_fx[3 * v + a] : d->vol_pos_fx[3 * v + a];
            // a general node lies in the box (x = 0 and y = 0 allowed: a periodic wrap puts
            // nodes there), off the ground; a per-voxel node strictly inside its voxel
            const bool in = general ? (a < 2 ? p >= 0 && p < W[a] : p > 0 && p < W[a])
                                    : p > c[a] * kFx && p < (c[a] + 1) * kFx;
            if (!in)
                return gfail(SG_E_INVALID, std::string(general ? "node position outside the box"
                                                               : "node position not strictly inside its voxel") +
                                               " (node " + std::to_string(v) + ")");
            s1[a] += p;
            s2[a] += (__int128)p * p;
        }
    }
    if (d->surface_nodes)
        for (long long c = 0; c < (long long)d->nx * d->ny; ++c) {
            const long long p[3] = {(c % d->nx) * kFx + kFx / 2, (c / d->nx) * kFx + kFx / 2, 0};
            for (int a = 0; a < 3; ++a) {
                s1[a] += p[a];
                s2[a] += (__int128)p[a] * p[a];
            }
        }
    Builder B(ctx, st);
    Geo &g = B.g;
    g.nx = d->nx;
    g.ny = d->ny;
    g.nz = d->nz;
    g.surface = d->surface_nodes ? 1 : 0;
    g.general = general ? 1 : 0;
    g.nvox = nvox;
    g.nvol = nvol;
    g.N = N;
    g.mu_max = (double)mmax;
    for (int a = 0; a < 3; ++a) {
        g.mean[a] = (double)s1[a] / (double)N;
        const double var = (double)((__int128)N * s2[a] - s1[a] * s1[a]) / ((double)N * (double)N);
        g.sd[a] = var > 0.0 ? std::sqrt(var) : 0.0;
    }

    // node arrays
    int *pos = nullptr;
    float *mus = nullptr, *alb = nullptr;
    GTRY(B.dev.get(&pos, 3 * nvol));
    GTRY(B.dev.get(&mus, nvox));
    GTRY(B.dev.get(&alb, (long long)d->nx * d->ny));
    GTRY(B.dev.get(&B.P, 3 * N));
    GTRY(B.dev.get(&B.q, 3 * N));
    GTRY(B.dev.get(&B.mu, N));
    GTRY(B.dev.get(&B.scal, 4));
    GHIP(hipMemsetAsync(B.scal, 0, 4 * sizeof(unsigned long long), st));
    GHIP(hipMemcpyAsync(pos, general ? d->node_pos_fx : d->vol_pos_fx, sizeof(int) * 3 * nvol, hipMemcpyHostToDevice,
                        st));
    GHIP(hipMemcpyAsync(mus, d->mu_s, sizeof(float) * nvox, hipMemcpyHostToDevice, st));
    if (d->surface_nodes)
        GHIP(hipMemcpyAsync(alb, d->surf_albedo, sizeof(float) * d->nx * d->ny, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_graph_nodes, dim3(blocks_for(N, 256)), dim3(256), 0, st, g, pos, mus, alb, B.P, B.q, B.mu);
    GHIP(hipGetLastError());

    // candidates and selection
    double *keys = nullptr;
    unsigned long long *codes = nullptr, have = 0, n_sel = 0, ranked = 0;
    double t_used = 0.0;
    int streamed = 0;
    if (d->n_pairs == 0) {
        t_used = d->c_min * d->c_min;
        GTRY(B.pairs(t_used, 1, 0, N, keys, codes, have));
        n_sel = ranked = have;
    } else {
        // the lowest threshold (bisection in the exponent) whose boxes fit the cell budget;
        // a larger budget when that threshold leaves fewer than n candidates
        const std::vector<unsigned long long> budgets = cell_budgets();
        const unsigned long long budget = budgets.back();
        double t_fit = 0.0;
        unsigned long long cells = 0;
        if (!general) GTRY(B.cells(0.0, cells));
        const unsigned long long all_cells = cells;
        // general nodes have no voxel boxes: straight to the streamed ranking of every pair
        for (size_t k = 0; k < budgets.size() && !general; ++k) {
            const unsigned long long bk = budgets[k];
            t_fit = 0.0;
            if (all_cells > bk) {
                double lo = 1e-300, hi = 1e300;
                GTRY(B.cells(hi, cells));
                if (cells > bk) return gfail(SG_E_NOMEM, "coupling candidates exceed the cell budget");
                // geometric bisection to a factor of two: any threshold within the budget
                // gives the same selection, a tighter one only fewer candidates
                while (hi > 2.0 * lo) {
                    const double mid = std::sqrt(lo) * std::sqrt(hi);
                    if (!(mid > lo && mid < hi)) break;
                    GTRY(B.cells(mid, cells));
                    if (cells <= bk) hi = mid;
                    else lo = mid;
                }
                t_fit = hi;
            }
            have = 0;  // a retry replaces the candidates of a smaller budget
            GTRY(B.pairs(t_fit, 0, 0, N, keys, codes, have));
            if (have >= (unsigned long long)d->n_pairs || t_fit == 0.0) break;
        }
        t_used = t_fit;
        ranked = have;
        if (!general && (have >= (unsigned long long)d->n_pairs || t_fit == 0.0)) {
            GTRY(B.sort_desc(keys, codes, have));
            n_sel = std::min<unsigned long long>(have, (unsigned long long)d->n_pairs);
        } else {
            // every pair, streamed in node chunks through a running best-n list
            streamed = 1;
            t_used = 0.0;
            B.evals = 0;
            have = 0;
            const long long chunk = std::max<long long>(1, (long long)(budget / (unsigned long long)N));
            for (long long n0 = 0; n0 < N; n0 += chunk) {
                GTRY(B.pairs(0.0, 1, n0, std::min(N, n0 + chunk), keys, codes, have));
                ranked += have;
                GTRY(B.sort_desc(keys, codes, have));
                have = std::min<unsigned long long>(have, (unsigned long long)d->n_pairs);
            }
            n_sel = have;
        }
    }

    // adjacency: directed codes sorted ascending give the rows in order
    const long long E = 2 * (long long)n_sel;
    *n_edges = E;
    if (E >= (1LL << 31) - 1) return gfail(SG_E_INVALID, "too many edges");
    Dev tmp(ctx);
    unsigned long long *dir = nullptr;
    int *head = nullptr;
    long long *ptr = nullptr;
    GTRY(tmp.get(&dir, E));
    GTRY(tmp.get(&head, E));
    GTRY(tmp.get(&ptr, N + 1));
    if (n_sel) {
        hipLaunchKernelGGL(k_graph_directed, dim3(blocks_for((long long)n_sel, 256)), dim3(256), 0, st,
                           (long long)n_sel, N, codes, dir);
        GHIP(hipGetLastError());
        auto *e = B.mark(B.ev_sort);
        GTRY(B.sort_u64(dir, nullptr, E));
        if (e) (void)hipEventRecord(e->second, st);
        hipLaunchKernelGGL(k_graph_heads, dim3(blocks_for(E, 256)), dim3(256), 0, st, E, N, dir, head);
        GHIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_graph_rowptr, dim3(blocks_for(N + 1, 256)), dim3(256), 0, st, N, E,
                       (const unsigned long long *)dir, ptr);
    GHIP(hipGetLastError());
    if (adj_ptr) GHIP(hipMemcpyAsync(adj_ptr, ptr, sizeof(int64_t) * (N + 1), hipMemcpyDeviceToHost, st));
    if (adj_idx && cap >= E && E > 0)
        GHIP(hipMemcpyAsync(adj_idx, head, sizeof(int32_t) * E, hipMemcpyDeviceToHost, st));
    GHIP(hipStreamSynchronize(st));
    if (info) {
        info->candidates = (int64_t)ranked;
        info->pairs_evaluated = (int64_t)B.evals;
        info->threshold = t_used;
        info->streamed = streamed;
        info->passes = B.passes;
        info->ms_pairs = Builder::total_ms(B.ev_pairs);
        info->ms_sort = Builder::total_ms(B.ev_sort);
        info->ms_total =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    return SG_OK;
}

}  // namespace sg

extern "C" sg_status sg_graph_build(sg_ctx *ctx, const sg_graph_desc *desc, void *hip_stream, int64_t *adj_ptr,
                                    int32_t *adj_idx, int64_t cap, int64_t *n_edges, sg_graph_info *info) {
    if (!ctx) return sg::gfail(SG_E_INVALID, "ctx is NULL");
    if (ctx->sticky.load()) return sg::gfail(SG_E_DEVICE, "context is in a failed state");
    if (hipSetDevice(ctx->device) != hipSuccess) return sg::gfail(SG_E_DEVICE, "hipSetDevice failed");
    const sg_status r = sg::graph_build(ctx, desc, hip_stream ? (hipStream_t)hip_stream : ctx->stream, adj_ptr,
                                        adj_idx, cap, n_edges, info);
    const sg_status b = sg::bounds_report();
    return b != SG_OK ? b : r;
}

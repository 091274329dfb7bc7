// Beer-Lambert-Bouguer transmittances by exact voxel marches (Sec. 2, Eq. 3;
// the exp(-integral mu_e) factor of Eq. 6, Eq. 9 and Eq. 11).
//
// Edge march: each coupling is walked once, from the lower to the higher node id,
// and its values are written to both directed edges (the reverse edge's index from
// the structure pass), so both directions carry bit-identical values.  A workgroup
// takes a run of consecutive tail nodes and their forward edges (head id above the
// tail's: a suffix of each sorted row), spread evenly over its threads; it reduces
// the bounding box of those edges' end voxels, stages that brick of the two
// extinction channels (mu_s, mu_a) in LDS, and marches the edges from LDS; a brick
// larger than the LDS budget falls back to global (L2-resident) reads.
// Two channels are kept per path (tau_s, tau_a), so any wavelength's optical
// depth is tau_s + s * tau_a (the per-basis path arrays of Sec. 3).
#include "device.hpp"
#include "internal.hpp"

#include <type_traits>

namespace sg {

namespace {

constexpr int kMarchThreads = 256;
constexpr int kNodesPerBlock = 32;
constexpr int kBrickCap = 1024;  // voxels staged per workgroup (2 channels x 4 KB)

// Crossing-time arithmetic of the marches: FP64 on a bounded grid (exact there, and one
// multiply per product), 64-bit integers on periodic axes (walks long enough to pass 2^53)
template <bool kPer>
using WalkT = typename std::conditional<kPer, long long, double>::type;

__device__ __forceinline__ void node_voxel(const int *__restrict__ pos, int l, int &vx, int &vy, int &vz) {
    vx = pos[3 * l] >> 16;
    vy = pos[3 * l + 1] >> 16;
    vz = pos[3 * l + 2] >> 16;
}

// kPer = false: a bounded grid (per is ignored, and the periodic branches fold away)
template <class Real, bool kPer>
__global__ __launch_bounds__(kMarchThreads) void k_march_edges(
    int N, int nx, int ny, int nz, int per_arg, const long long *__restrict__ adj_ptr, const int *__restrict__ adj_idx,
    const int *__restrict__ pos, const float *__restrict__ mu_s, const float *__restrict__ mu_a, Real len_scale,
    Real scale, const int *__restrict__ rev, Real *__restrict__ tau_s, Real *__restrict__ tau_a,
    Real *__restrict__ T, int use_lds) {
    const int per = kPer ? per_arg : 0;
    __shared__ float bs[kBrickCap];
    __shared__ float ba[kBrickCap];
    __shared__ long long fbeg[kNodesPerBlock];  // first forward edge of each node
    __shared__ int fptr[kNodesPerBlock + 1];    // exclusive prefix of forward edge counts
    __shared__ int bb[6];
    const int l0 = blockIdx.x * kNodesPerBlock;
    const int l1 = min(N, l0 + kNodesPerBlock);
    const int nl = l1 - l0;
    if (threadIdx.x < nl) {  // a row is sorted by head id: its forward edges are a suffix
        const int l = l0 + threadIdx.x;
        long long lo = adj_ptr[l], hi = adj_ptr[l + 1];
        const long long end = hi;
        while (lo < hi) {
            const long long mid = (lo + hi) >> 1;
            if (adj_idx[mid] <= l) lo = mid + 1; else hi = mid;
        }
        fbeg[threadIdx.x] = lo;
        fptr[threadIdx.x + 1] = (int)(end - lo);
    }
    if (threadIdx.x < 3) bb[threadIdx.x] = 1 << 30;
    else if (threadIdx.x < 6) bb[threadIdx.x] = -(1 << 30);
    __syncthreads();
    if (threadIdx.x == 0) {
        fptr[0] = 0;
        for (int k = 0; k < nl; ++k) fptr[k + 1] += fptr[k];
    }
    __syncthreads();
    const int nf = fptr[nl];
    // bounding box of the end voxels of the block's forward edges: per-thread, then per
    // wave (butterfly), then one LDS atomic per wave and coordinate
    int mnx = 1 << 30, mny = 1 << 30, mnz = 1 << 30, mxx = -(1 << 30), mxy = -(1 << 30), mxz = -(1 << 30);
    for (int f = threadIdx.x; f < nf; f += kMarchThreads) {
        int k = 0;
        while (k + 1 < nl && fptr[k + 1] <= f) ++k;
        int vx, vy, vz;
        node_voxel(pos, adj_idx[fbeg[k] + (f - fptr[k])], vx, vy, vz);
        mnx = min(mnx, vx); mny = min(mny, vy); mnz = min(mnz, vz);
        mxx = max(mxx, vx); mxy = max(mxy, vy); mxz = max(mxz, vz);
    }
    if (threadIdx.x < nl) {
        int vx, vy, vz;
        node_voxel(pos, l0 + threadIdx.x, vx, vy, vz);
        mnx = min(mnx, vx); mny = min(mny, vy); mnz = min(mnz, vz);
        mxx = max(mxx, vx); mxy = max(mxy, vy); mxz = max(mxz, vz);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mnx = min(mnx, __shfl_xor(mnx, o, 64)); mny = min(mny, __shfl_xor(mny, o, 64));
        mnz = min(mnz, __shfl_xor(mnz, o, 64)); mxx = max(mxx, __shfl_xor(mxx, o, 64));
        mxy = max(mxy, __shfl_xor(mxy, o, 64)); mxz = max(mxz, __shfl_xor(mxz, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&bb[0], mnx); atomicMin(&bb[1], mny); atomicMin(&bb[2], mnz);
        atomicMax(&bb[3], mxx); atomicMax(&bb[4], mxy); atomicMax(&bb[5], mxz);
    }
    __syncthreads();
    if (nf == 0) return;
    const int bx0 = bb[0], by0 = bb[1], bz0 = bb[2];
    const int bw = bb[3] - bx0 + 1, bh = bb[4] - by0 + 1, bd = bb[5] - bz0 + 1;
    const bool lds = use_lds && (long long)bw * bh * bd <= kBrickCap;
    if (lds) {
        const int vol = bw * bh * bd;
        for (int t = threadIdx.x; t < vol; t += kMarchThreads) {
            const int x = t % bw, yz = t / bw;
            const int y = yz % bh, z = yz / bh;
            const long long g = (bx0 + x) + (long long)nx * ((by0 + y) + (long long)ny * (bz0 + z));
            if (SG_IN(t, kBrickCap, 0x101) && SG_IN(g, (long long)nx * ny * nz, 0x102)) {
                bs[t] = mu_s[g];
                ba[t] = mu_a[g];
            }
        }
    }
    __syncthreads();
    for (int f = threadIdx.x; f < nf; f += kMarchThreads) {
        int k = 0;
        while (k + 1 < nl && fptr[k + 1] <= f) ++k;
        const long long e = fbeg[k] + (f - fptr[k]);
        const int l = l0 + k;
        const int j = adj_idx[e];
        if (!SG_IN(j, N, 0x103)) continue;
        const int er = rev[e];  // the edge j -> l
        if (!SG_IN(er, adj_ptr[N], 0x109)) continue;
        const int a = l, b = j;  // a < b
        const long long px = pos[3 * a], py = pos[3 * a + 1], pz = pos[3 * a + 2];
        const long long dx = min_image(pos[3 * b] - px, nx * kFx, per & 1);
        const long long dy = min_image(pos[3 * b + 1] - py, ny * kFx, per & 2);
        const long long dz = pos[3 * b + 2] - pz;
        Real ss = 0, sa = 0;
        if (lds) {
            voxel_walk_t<WalkT<kPer>>(nx, ny, nz, per, px, py, pz, dx, dy, dz, false, [&](int x, int y, int z, auto num, auto den) {
                const int xo = x - bx0, yo = y - by0, zo = z - bz0;
                const Real dt = ratio<Real>(num, den);
                if ((unsigned)xo < (unsigned)bw && (unsigned)yo < (unsigned)bh && (unsigned)zo < (unsigned)bd) {
                    const int t = xo + bw * (yo + bh * zo);
                    if (SG_IN(t, kBrickCap, 0x104)) {
                        ss += (Real)bs[t] * dt;
                        sa += (Real)ba[t] * dt;
                    }
                } else {  // outside the staged brick (only a periodic segment, wrapped round the grid)
                    const long long g = x + (long long)nx * (y + (long long)ny * z);
                    if (SG_IN(g, (long long)nx * ny * nz, 0x105)) {
                        ss += (Real)mu_s[g] * dt;
                        sa += (Real)mu_a[g] * dt;
                    }
                }
                return true;
            });
        } else {
            voxel_walk_t<WalkT<kPer>>(nx, ny, nz, per, px, py, pz, dx, dy, dz, false, [&](int x, int y, int z, auto num, auto den) {
                const long long vox = x + (long long)nx * (y + (long long)ny * z);
                const Real dt = ratio<Real>(num, den);
                if (SG_IN(vox, (long long)nx * ny * nz, 0x106)) {
                    ss += (Real)mu_s[vox] * dt;
                    sa += (Real)mu_a[vox] * dt;
                }
                return true;
            });
        }
        const Real L = sqrt((Real)(dx * dx + dy * dy + dz * dz)) * len_scale;
        ss *= L;
        sa *= L;
        tau_s[e] = ss;
        tau_a[e] = sa;
        tau_s[er] = ss;
        tau_a[er] = sa;
        if (T) {
            const Real t = exp(-(ss + scale * sa));
            T[e] = t;
            T[er] = t;
        }
    }
}

// Node -> sun optical depth, both channels, to the grid exit.  A lane stops as
// soon as the smallest wavelength optical depth (tau_s + smin tau_a) passes the
// cutoff where exp(-tau) is zero in the working precision.
template <class Real, bool kPer>
__global__ __launch_bounds__(256) void k_march_sun(int N, int nx, int ny, int nz, int per_arg, const int *__restrict__ pos,
                                                  long long sdx, long long sdy, long long sdz,
                                                  const float *__restrict__ mu_s, const float *__restrict__ mu_a,
                                                  Real len_scale, Real smin, Real cutoff, Real scale,
                                                  Real *__restrict__ ts, Real *__restrict__ ta,
                                                  Real *__restrict__ Tsun) {
    const int per = kPer ? per_arg : 0;
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= N) return;
    const Real L = sqrt((Real)(sdx * sdx + sdy * sdy + sdz * sdz)) * len_scale;
    const Real lim = cutoff / L;
    Real ss = 0, sa = 0;
    voxel_walk_t<WalkT<kPer>>(nx, ny, nz, per, pos[3 * l], pos[3 * l + 1], pos[3 * l + 2], sdx, sdy, sdz, true,
               [&](int x, int y, int z, auto num, auto den) {
                   const long long vox = x + (long long)nx * (y + (long long)ny * z);
                   const Real dt = ratio<Real>(num, den);
                   if (SG_IN(vox, (long long)nx * ny * nz, 0x107)) {
                       ss += (Real)mu_s[vox] * dt;
                       sa += (Real)mu_a[vox] * dt;
                   }
                   return ss + smin * sa < lim;
               });
    ss *= L;
    sa *= L;
    ts[l] = ss;
    ta[l] = sa;
    if (Tsun) Tsun[l] = exp(-(ss + scale * sa));
}

// Node weight (reading of Eq. 7's mu_s factor): volume rho = w (1 - exp(-mu_e dx))
// computed with expm1, or mu_s dx (mode 1); surface rho = albedo.
// mu_s, mu_a: the medium at each volume node (indexed by node id)
template <class Real>
__global__ __launch_bounds__(256) void k_node_weights(int N, int nvol, const float *__restrict__ mu_s,
                                                     const float *__restrict__ mu_a,
                                                     const float *__restrict__ albedo, Real dx, Real scale,
                                                     int mode, Real *__restrict__ rho) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= N) return;
    Real r;
    if (l < nvol) {
        const Real ms = (Real)mu_s[l];
        const Real me = ms + scale * (Real)mu_a[l];
        if (mode == 1) r = ms * dx;
        else r = me > 0 ? (ms / me) * (-expm1(-me * dx)) : (Real)0;
    } else {
        r = (Real)albedo[l - nvol];
    }
    rho[l] = r;
}

__device__ int edge_tail(const long long *__restrict__ adj_ptr, int N, long long e) {
    int lo = 0, hi = N;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (adj_ptr[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(64) void k_trace(int kind, int N, int nx, int ny, int nz, int per,
                                             const long long *__restrict__ adj_ptr,
                                             const int *__restrict__ adj_idx, const int *__restrict__ pos,
                                             long long sdx, long long sdy, long long sdz, long long vdx,
                                             long long vdy, long long vdz, const long long *__restrict__ ids,
                                             int n, int cap, int *__restrict__ vox_out, double *__restrict__ dt_out,
                                             int *__restrict__ count) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const long long id = ids[t];
    long long px, py, pz, dx, dy, dz;
    bool ray = true;
    if (kind == 0) {
        const int l = edge_tail(adj_ptr, N, id);
        const int j = adj_idx[id];
        if (!SG_IN(j, N, 0x108)) return;
        const int a = min(l, j), b = max(l, j);
        px = pos[3 * a]; py = pos[3 * a + 1]; pz = pos[3 * a + 2];
        dx = min_image(pos[3 * b] - px, nx * kFx, per & 1);
        dy = min_image(pos[3 * b + 1] - py, ny * kFx, per & 2);
        dz = pos[3 * b + 2] - pz;
        ray = false;
    } else if (kind == 1) {
        px = pos[3 * id]; py = pos[3 * id + 1]; pz = pos[3 * id + 2];
        dx = sdx; dy = sdy; dz = sdz;
    } else {
        const long long ix = id % nx, iy = id / nx;
        px = ix * kFx + kFx / 2; py = iy * kFx + kFx / 2; pz = 0;
        dx = vdx; dy = vdy; dz = vdz;
    }
    int k = 0;
    const int c = voxel_walk(nx, ny, nz, per, px, py, pz, dx, dy, dz, ray, [&](int x, int y, int z, long long num, long long den) {
        if (k < cap) {
            vox_out[(long long)t * cap + k] = x + nx * (y + ny * z);
            dt_out[(long long)t * cap + k] = (double)num / (double)den;
        }
        ++k;
        return true;
    });
    count[t] = c;
    for (int j = min(c, cap); j < cap; ++j) {  // slots past the path: defined filler
        vox_out[(long long)t * cap + j] = -1;
        dt_out[(long long)t * cap + j] = 0.0;
    }
}

}  // namespace

template <class Real>
void launch_march_edges(Scene &s, hipStream_t st, float scale, int use_lds) {
    const Real len_scale = (Real)(s.voxel_m / 65536.0);
    const int nb = (s.N + kNodesPerBlock - 1) / kNodesPerBlock;
    // the bounded-grid instantiations carry no periodic branches
    const auto edges = s.periodic ? k_march_edges<Real, true> : k_march_edges<Real, false>;
    hipLaunchKernelGGL(edges, dim3(nb), dim3(kMarchThreads), 0, st, s.N, s.nx, s.ny, s.nz, s.periodic, s.adj_ptr,
                       s.adj_idx, s.pos, s.mu_s, s.mu_a, len_scale, (Real)scale, s.rev, (Real *)s.tau_s,
                       (Real *)s.tau_a, (Real *)s.T, use_lds);
}

template <class Real>
void launch_march_sun(Scene &s, hipStream_t st, float scale) {
    const Real len_scale = (Real)(s.voxel_m / 65536.0);
    float smin = scale;
    if (s.n_lambda > 1) {
        smin = s.abs_scale[0];
        for (float v : s.abs_scale) smin = v < smin ? v : smin;
    }
    const Real cutoff = sizeof(Real) == 4 ? (Real)104.0 : (Real)746.0;
    const auto sun = s.periodic ? k_march_sun<Real, true> : k_march_sun<Real, false>;
    hipLaunchKernelGGL(sun, dim3((s.N + 255) / 256), dim3(256), 0, st, s.N, s.nx, s.ny, s.nz, s.periodic, s.pos,
                       (long long)s.sun[0], (long long)s.sun[1], (long long)s.sun[2], s.mu_s, s.mu_a, len_scale,
                       (Real)smin, cutoff, (Real)scale, (Real *)s.tsun_s, (Real *)s.tsun_a, (Real *)s.Tsun);
}

template <class Real>
void launch_node_weights(Scene &s, hipStream_t st, float scale) {
    hipLaunchKernelGGL((k_node_weights<Real>), dim3((s.N + 255) / 256), dim3(256), 0, st, s.N, s.n_vol, node_mu_s(s),
                       node_mu_a(s),
                       s.albedo, (Real)s.voxel_m, (Real)scale, s.weight_mode, (Real *)s.rho);
}

void launch_trace(Scene &s, hipStream_t st, int kind, const long long *ids, int n, int cap, int *vox, double *dt,
                  int *count) {
    hipLaunchKernelGGL(k_trace, dim3((n + 63) / 64), dim3(64), 0, st, kind, s.N, s.nx, s.ny, s.nz, s.periodic,
                       s.adj_ptr, s.adj_idx, s.pos, (long long)s.sun[0], (long long)s.sun[1], (long long)s.sun[2], (long long)s.view[0],
                       (long long)s.view[1], (long long)s.view[2], ids, n, cap, vox, dt, count);
}

template void launch_march_edges<float>(Scene &, hipStream_t, float, int);
template void launch_march_edges<double>(Scene &, hipStream_t, float, int);
template void launch_march_sun<float>(Scene &, hipStream_t, float);
template void launch_march_sun<double>(Scene &, hipStream_t, float);
template void launch_node_weights<float>(Scene &, hipStream_t, float);
template void launch_node_weights<double>(Scene &, hipStream_t, float);

}  // namespace sg

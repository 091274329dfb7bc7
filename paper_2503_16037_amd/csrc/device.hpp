// Device-side building blocks shared by the HIP kernels of the library.
//
// Contents: the exact integer voxel walk used by every march (edge, sun,
// view), the Henyey-Greenstein phase function, and deterministic wave /
// block reductions.  gfx950 only: 64-lane wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace sg {

constexpr long long kFx = 65536;  // fixed-point units per voxel edge
constexpr int kWave = 64;

// Bounds-checked builds (SG_DEBUG_BOUNDS, libsgrt_debug.so): SG_IN(i, n, site) is true when
// 0 <= i < n; otherwise the first failing site of this code module is recorded and the
// caller skips the access.  Each module registers a reader of its record, which the entry
// points consult after their kernels (bounds_report).  In release builds it is the constant
// true and costs nothing.
#ifdef SG_DEBUG_BOUNDS
namespace {
__device__ unsigned g_oob_site = 0u;
__device__ __forceinline__ bool in_bounds(long long i, long long n, unsigned site) {
    if (i >= 0 && i < n) return true;
    atomicCAS(&g_oob_site, 0u, site);
    return false;
}
unsigned oob_read_and_clear() {
    unsigned v = 0u, z = 0u;
    if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_oob_site), sizeof(v)) != hipSuccess) return 0u;
    if (v) (void)hipMemcpyToSymbol(HIP_SYMBOL(g_oob_site), &z, sizeof(z));
    return v;
}
struct OobRegistrar {
    OobRegistrar() { register_bounds_reader(&oob_read_and_clear); }
} g_oob_registrar;
}  // namespace
#define SG_IN(i, n, site) (::sg::in_bounds((long long)(i), (long long)(n), (unsigned)(site)))
#else
#define SG_IN(i, n, site) true
#endif

__device__ __forceinline__ long long floor_div_fx(long long a) {
    // floor(a / kFx) for any sign (kFx is a power of two: arithmetic shift)
    return a >> 16;
}

// Exact walk of the voxels crossed with positive length by P + t D.
//
// Segment mode (ray = false): t in (0, 1]; ray mode: until the walk leaves
// the grid.  Crossing times (B - P_k) / D_k are kept as integer fractions
// n_k / d_k and compared by cross multiplication; an idle axis (D_k = 0)
// carries the fraction 1/0, which compares greater than every finite time
// and never equals one.  All axes whose crossing equals the minimum step
// together, so no zero-length voxel is produced.  A start on a voxel plane
// belongs to the voxel the path moves into (floor for D >= 0, ceil - 1 for
// D < 0).  For each voxel the visitor gets (ix, iy, iz, num, den) with the
// parameter length inside the voxel exactly num / den, and returns false to
// stop the walk early.  Each lane leaves the loop on its own; the wavefront
// retires the loop when the ballot of its live lanes is empty.  Magnitudes: grid
// <= 1024 voxels per axis and |D| <= 2^26 keep every product below 2^63.
//
// Periodic horizontal axes (bit 0 of per: x, bit 1: y; plane-parallel slabs): the
// crossing times stay on the unwrapped line, the walk never ends through such an
// axis, and the visitor gets the index wrapped into the grid.  A periodic walk
// takes at most kMaxWalk voxels; scenes whose sun or view rays could need more
// are rejected at creation, so the limit only bounds the loop.  Unwrapped crossing
// numerators then stay below kMaxWalk * kFx = 2^32, the products below 2^58.
constexpr int kMaxWalk = 65536;

__device__ __forceinline__ long long min_image(long long d, long long w, bool on) {
    // the shortest periodic image of a displacement (|d| < w on input)
    if (on) {
        if (2 * d > w) d -= w;
        else if (2 * d < -w) d += w;
    }
    return d;
}

// The walk with its crossing times held in T: long long, or double where every product
// stays below 2^53 and FP64 therefore represents it exactly (a bounded grid: crossing
// numerators below 1025 * 2^16, |D| below 2^26, so the products stay below 2^53), which
// trades the multi-instruction 64-bit integer products for one FP64 multiply each; both
// give the same voxels and the same num / den.
template <class T, class Visit>
__device__ __forceinline__ int voxel_walk_t(int nx, int ny, int nz, int per, long long px, long long py, long long pz,
                                            long long dx, long long dy, long long dz, bool ray, Visit &&visit) {
    long long ix, iy, iz;
    int sx, sy, sz;
    long long nxn0, nyn0, nzn0, dxd0, dyd0, dzd0;
    if (dx > 0) { ix = floor_div_fx(px); sx = 1; nxn0 = (ix + 1) * kFx - px; dxd0 = dx; }
    else if (dx < 0) { ix = floor_div_fx(px + kFx - 1) - 1; sx = -1; nxn0 = px - ix * kFx; dxd0 = -dx; }
    else { ix = floor_div_fx(px); sx = 0; nxn0 = 1; dxd0 = 0; }
    if (dy > 0) { iy = floor_div_fx(py); sy = 1; nyn0 = (iy + 1) * kFx - py; dyd0 = dy; }
    else if (dy < 0) { iy = floor_div_fx(py + kFx - 1) - 1; sy = -1; nyn0 = py - iy * kFx; dyd0 = -dy; }
    else { iy = floor_div_fx(py); sy = 0; nyn0 = 1; dyd0 = 0; }
    if (dz > 0) { iz = floor_div_fx(pz); sz = 1; nzn0 = (iz + 1) * kFx - pz; dzd0 = dz; }
    else if (dz < 0) { iz = floor_div_fx(pz + kFx - 1) - 1; sz = -1; nzn0 = pz - iz * kFx; dzd0 = -dz; }
    else { iz = floor_div_fx(pz); sz = 0; nzn0 = 1; dzd0 = 0; }
    T nxn = (T)nxn0, nyn = (T)nyn0, nzn = (T)nzn0;
    const T dxd = (T)dxd0, dyd = (T)dyd0, dzd = (T)dzd0, step = (T)kFx;

    const bool wx_on = per & 1, wy_on = per & 2;
    // wrapped indices (the start is at most one voxel outside on a periodic axis)
    int wx = (int)ix, wy = (int)iy;
    if (wx_on) wx = wx < 0 ? wx + nx : (wx >= nx ? wx - nx : wx);
    if (wy_on) wy = wy < 0 ? wy + ny : (wy >= ny ? wy - ny : wy);
    T cn = 0, cd = 1;  // current time
    int count = 0;
    const int max_steps = per ? kMaxWalk : nx + ny + nz + 2;
    for (int it = 0; it < max_steps; ++it) {
        if ((!wx_on && (ix < 0 || ix >= nx)) || (!wy_on && (iy < 0 || iy >= ny)) || iz < 0 || iz >= nz) break;
        T mn = nxn, md = dxd;
        if (nyn * md < mn * dyd) { mn = nyn; md = dyd; }
        if (nzn * md < mn * dzd) { mn = nzn; md = dzd; }
        bool last = false;
        if (!ray && mn >= md) { mn = 1; md = 1; last = true; }
        ++count;
        if (!visit(wx, wy, (int)iz, mn * cd - cn * md, md * cd)) break;
        if (last) break;
        const bool ex = nxn * md == mn * dxd;
        const bool ey = nyn * md == mn * dyd;
        const bool ez = nzn * md == mn * dzd;
        if (ex) {
            ix += sx; nxn += step; wx += sx;
            wx = wx == nx ? 0 : (wx < 0 ? nx - 1 : wx);  // non-periodic: the loop ends first
        }
        if (ey) {
            iy += sy; nyn += step; wy += sy;
            wy = wy == ny ? 0 : (wy < 0 ? ny - 1 : wy);
        }
        if (ez) { iz += sz; nzn += step; }
        cn = mn;
        cd = md;
    }
    return count;
}

template <class Visit>
__device__ __forceinline__ int voxel_walk(int nx, int ny, int nz, int per, long long px, long long py, long long pz,
                                          long long dx, long long dy, long long dz, bool ray, Visit &&visit) {
    return voxel_walk_t<long long>(nx, ny, nz, per, px, py, pz, dx, dy, dz, ray, visit);
}

template <class Real, class T>
__device__ __forceinline__ Real ratio(T num, T den) {
    return (Real)num / (Real)den;  // num, den exact integers (long long, or double below 2^53)
}

// Henyey-Greenstein phase function, normalised over the sphere.
__device__ __forceinline__ double hg_phase(double g, double mu) {
    const double den = 1.0 + g * g - 2.0 * g * mu;
    return (1.0 - g * g) / (4.0 * 3.14159265358979323846 * den * sqrt(den));
}

// Component c at cos(theta) = mu, normalised over the sphere.
__device__ __forceinline__ double phase_theta(const PhaseSet &ps, int c, double mu) {
    if (ps.kind[c] == 1) return (3.0 / (16.0 * 3.14159265358979323846)) * (1.0 + mu * mu);
    if (ps.kind[c] == 2) {
        const int n = ps.lut_n;
        const double x = (mu + 1.0) * (0.5 * (double)(n - 1));
        int m = (int)floor(x);
        m = m < 0 ? 0 : (m > n - 2 ? n - 2 : m);
        const double f = x - (double)m;
        const double *row = ps.lut + (long long)c * n;
        return (row[m] * (1.0 - f) + row[m + 1] * f) * ps.scale[c];
    }
    return hg_phase(ps.g[c], mu);
}

// Deterministic sum over a 64-lane wavefront (fixed butterfly order).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// Block maximum; every thread must call it; returns the result in thread 0.
template <int kThreads>
__device__ __forceinline__ double block_max(double v) {
    __shared__ double part[kThreads / kWave];
    v = wave_max(v);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) part[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < kThreads / kWave; ++i) t = fmax(t, part[i]);
    }
    __syncthreads();
    return t;
}

// Floor of the per-edge relative convergence measures |change| / (|value| + kRelFloor):
// radiances below it (in units of the solar flux) count as absolute.
constexpr double kRelFloor = 1e-30;

// A per-edge measure that is NaN (an overflowed iterate: inf - inf, inf / inf) becomes
// +inf, so that the running maxima, which take fmax and drop NaN, keep it and the host
// sees a non-finite measure instead of a zero.
__device__ __forceinline__ double keep_nan(double v) { return v == v ? v : __builtin_huge_val(); }

// Deterministic block sum; every thread must call it; returns the total in thread 0.
template <int kThreads>
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double part[kThreads / kWave];
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) part[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < kThreads / kWave; ++i) t += part[i];
    }
    __syncthreads();
    return t;
}

}  // namespace sg

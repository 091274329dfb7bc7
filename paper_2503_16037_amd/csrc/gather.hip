// Observed radiance (Sec. 2, Eq. 11; step 5 of the TURSCA algorithm): the
// light scattered toward the sensor at every node crossed by a pixel's line of
// sight, attenuated on its way out.
//
//   J_l (volume)  = Theta_l(s_sun . v) T_sun(l) + sum_{a in in(l)} Theta_l(s_a . v) T_a phi_a
//   J_s (surface) = mu0 T_sun(s) + sum_{a in in(s)} T_a phi_a
//   I_p = sum_k T_entry(k) w_k (1 - exp(-mu_e,k s_k)) J_{v_k} + T_view (A_p / pi) J_{s_p}
// with s_a the propagation direction of in-edge a, v the unit vector toward the
// sensor, s_k the chord of the line of sight in voxel v_k and T_entry(k) the
// transmittance from the chord's far end to the sensor.  With general nodes (the path
// points of the lines of sight, Sec. 2) the chords are cut at the ends of the line's
// elements and each piece takes J of its element's node instead of the voxel's.
// Everything here is accumulated in FP64 (one thread per node, then one thread per
// pixel).
#include "device.hpp"
#include "internal.hpp"

namespace sg {

namespace {

__device__ __forceinline__ double theta_mix(const PhaseSet &pm, const float *__restrict__ frac, int stride, int v,
                                            double mu) {
    double th = 0.0;
    for (int c = 0; c < pm.n; ++c) {
        const double f = frac ? (double)frac[(long long)c * stride + v] : 1.0;
        th += f * phase_theta(pm, c, mu);
    }
    return th;
}

// Two nodes per wavefront, one per 32-lane half: lane m of a half takes in-edges m, m + 32,
// ..., then a fixed-order butterfly sum within the half (degree ~24 would leave most of a
// 64-lane wavefront idle).  frac: the phase fractions at each volume node
// ([component][node]), nvol volume nodes
template <class Real, bool kPer>
__global__ __launch_bounds__(256) void k_node_J(int N, int nvol, const long long *__restrict__ adj_ptr,
                                               const int *__restrict__ adj_idx, const int *__restrict__ rev,
                                               const int *__restrict__ pos, const Real *__restrict__ T,
                                               const Real *__restrict__ Tsun, const double *__restrict__ phi,
                                               PhaseSet pm, const float *__restrict__ frac, double sx, double sy,
                                               double sz, double vx, double vy, double vz, double mu0,
                                               int multiple, int per_arg, long long wx, long long wy,
                                               double *__restrict__ J) {
    const int per = kPer ? per_arg : 0;
    const int l = blockIdx.x * 8 + (threadIdx.x >> 5);
    const int lane = threadIdx.x & 31;
    if (l >= N) return;  // a half past the last node exits; the shuffles below stay within a half
    const long long off = adj_ptr[l], end = adj_ptr[l + 1];
    const int d = (int)(end - off);
    const bool vol = l < nvol;
    // the direct-sun term is taken by the lane after the last in-edge (m == d), through the
    // same phase evaluation as the edges, so no lane finishes alone after the sum
    double acc = 0.0;
    for (int m = lane; m <= d; m += 32) {
        const bool sun = m == d;
        if (!sun && !multiple) continue;
        const long long e = off + min(m, d - 1);
        double mu = sx * vx + sy * vy + sz * vz, w;
        if (sun) {
            w = (double)Tsun[l];
        } else {
            if (!SG_IN(rev[e], adj_ptr[N], 0x501)) continue;
            w = (double)T[e] * phi[rev[e]];
            if (vol) {
                const int j = adj_idx[e];
                if (!SG_IN(j, N, 0x502)) continue;
                const long long Dx = min_image((long long)pos[3 * l] - pos[3 * j], wx, per & 1);
                const long long Dy = min_image((long long)pos[3 * l + 1] - pos[3 * j + 1], wy, per & 2);
                const long long Dz = (long long)pos[3 * l + 2] - pos[3 * j + 2];
                const double dx = (double)Dx, dy = (double)Dy, dz = (double)Dz;
                const double inv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
                mu = (dx * vx + dy * vy + dz * vz) * inv;
            }
        }
        const double th = vol ? theta_mix(pm, frac, nvol, l, mu) : (sun ? mu0 : 1.0);
        acc += th * w;
    }
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 32);
    if (lane == 0) J[l] = acc;
}

__global__ __launch_bounds__(64) void k_pixels(int nx, int ny, int nz, int per, const float *__restrict__ mu_s,
                                              const float *__restrict__ mu_a, double scale, double len_view,
                                              long long vdx, long long vdy, long long vdz, long long sdx,
                                              long long sdy, long long sdz, double len_sun,
                                              const float *__restrict__ albedo, const double *__restrict__ J,
                                              int surface, double mu0, int nvol, const long long *__restrict__ los_ptr,
                                              const int *__restrict__ los_node, const double *__restrict__ los_t,
                                              double *__restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nx * ny) return;
    const long long ix = p % nx, iy = p / nx;
    const long long px = ix * kFx + kFx / 2, py = iy * kFx + kFx / 2;
    // pass 1: optical depth of the whole line of sight
    double tau_tot = 0.0;
    voxel_walk(nx, ny, nz, per, px, py, 0, vdx, vdy, vdz, true, [&](int x, int y, int z, long long num, long long den) {
        const long long v = x + (long long)nx * (y + (long long)ny * z);
        if (!SG_IN(v, (long long)nx * ny * nz, 0x503)) return true;
        const double me = (double)mu_s[v] + scale * (double)mu_a[v];
        tau_tot += me * ((double)num / (double)den * len_view);
        return true;
    });
    // pass 2: chords, each attenuated from its far end to the sensor
    double I = 0.0, cum = 0.0;
    if (!los_ptr) {
        voxel_walk(nx, ny, nz, per, px, py, 0, vdx, vdy, vdz, true, [&](int x, int y, int z, long long num, long long den) {
            const long long v = x + (long long)nx * (y + (long long)ny * z);
            if (!SG_IN(v, (long long)nx * ny * nz, 0x504)) return true;
            const double ms = (double)mu_s[v];
            const double me = ms + scale * (double)mu_a[v];
            const double sk = (double)num / (double)den * len_view;
            const double tk = me * sk;
            const double t_entry = exp(-(tau_tot - (cum + tk)));
            const double om = me > 0.0 ? ms / me : 0.0;
            I += t_entry * (om * (-expm1(-tk))) * J[v];  // the voxel's own node
            cum += tk;
            return true;
        });
    } else {
        // general nodes: the chord [t, t + dt] cut at the ends of the line's elements; element
        // e covers (los_t[e - 1], los_t[e]], the part above the last end has no node
        const long long e1 = los_ptr[p + 1];
        long long e = los_ptr[p];
        double t = 0.0;
        voxel_walk(nx, ny, nz, per, px, py, 0, vdx, vdy, vdz, true, [&](int x, int y, int z, long long num, long long den) {
            const long long v = x + (long long)nx * (y + (long long)ny * z);
            if (!SG_IN(v, (long long)nx * ny * nz, 0x505)) return true;
            const double ms = (double)mu_s[v];
            const double me = ms + scale * (double)mu_a[v];
            const double om = me > 0.0 ? ms / me : 0.0;
            const double t1 = t + (double)num / (double)den;
            double a = t;
            while (a < t1) {
                while (e < e1 && los_t[e] <= a) ++e;
                double b = t1;
                int node = -1;
                if (e < e1) {
                    b = fmin(t1, los_t[e]);
                    node = los_node[e];
                }
                const double tk = me * ((b - a) * len_view);
                if (node >= 0 && SG_IN(node, nvol, 0x506))
                    I += exp(-(tau_tot - (cum + tk))) * (om * (-expm1(-tk))) * J[node];
                cum += tk;
                a = b;
            }
            t = t1;
            return true;
        });
    }
    const double a_pi = (double)albedo[p] / 3.14159265358979323846;
    if (surface) {
        I += exp(-tau_tot) * a_pi * J[nvol + p];
    } else {
        double ts = 0.0;
        voxel_walk(nx, ny, nz, per, px, py, 0, sdx, sdy, sdz, true, [&](int x, int y, int z, long long num, long long den) {
            const long long v = x + (long long)nx * (y + (long long)ny * z);
            if (SG_IN(v, (long long)nx * ny * nz, 0x507))
                ts += ((double)mu_s[v] + scale * (double)mu_a[v]) * ((double)num / (double)den * len_sun);
            return true;
        });
        I += exp(-tau_tot) * a_pi * mu0 * exp(-ts);
    }
    out[p] = I;
}

}  // namespace

template <class Real>
void launch_gather(Scene &s, hipStream_t st, const double *phi, int scatter_order, double *radiance) {
    const PhaseSet pm = phase_set(s);
    const auto node_J = s.periodic ? k_node_J<Real, true> : k_node_J<Real, false>;
    hipLaunchKernelGGL(node_J, dim3((s.N + 7) / 8), dim3(256), 0, st, s.N, s.n_vol, s.adj_ptr, s.adj_idx, s.rev, s.pos,
                       (const Real *)s.T, (const Real *)s.Tsun, phi, pm, node_frac(s), s.sun_in[0], s.sun_in[1], s.sun_in[2],
                       s.view_u[0], s.view_u[1], s.view_u[2], s.mu0, scatter_order == 1 ? 0 : 1, s.periodic,
                       (long long)s.nx * kFx, (long long)s.ny * kFx, s.J);
    const double fx = s.voxel_m / 65536.0;
    const double lv = sqrt((double)s.view[0] * s.view[0] + (double)s.view[1] * s.view[1] + (double)s.view[2] * s.view[2]) * fx;
    const double ls = sqrt((double)s.sun[0] * s.sun[0] + (double)s.sun[1] * s.sun[1] + (double)s.sun[2] * s.sun[2]) * fx;
    const double scale = s.abs_scale.empty() ? 1.0 : (double)s.abs_scale[0];
    hipLaunchKernelGGL(k_pixels, dim3((s.npx + 63) / 64), dim3(64), 0, st, s.nx, s.ny, s.nz, s.periodic, s.mu_s, s.mu_a, scale,
                       lv,
                       (long long)s.view[0], (long long)s.view[1], (long long)s.view[2], (long long)s.sun[0],
                       (long long)s.sun[1], (long long)s.sun[2], ls, s.albedo, s.J, s.surface, s.mu0, s.n_vol,
                       s.general ? s.los_ptr : (const long long *)nullptr, s.los_node, s.los_t, radiance);
}

template void launch_gather<float>(Scene &, hipStream_t, const double *, int, double *);
template void launch_gather<double>(Scene &, hipStream_t, const double *, int, double *);

}  // namespace sg

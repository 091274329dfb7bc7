// Phase-cell weights (Sec. 2, Eq. 7; Fibonacci lattice of Sec. 3) fused with the
// flux-matrix values (Eq. 6) and the direct-solar source (Eq. 9).
//
// One 64-lane wavefront per node l.  Lane m holds out-edge m's unit direction;
// each lane holds lattice points i = lane and lane + 64.  For every incoming
// propagation direction u (each in-edge, then the sunlight) the out-directions
// are rotated by the minimal rotation taking u to +z, each lattice point is
// owned by the out-direction with the largest dot product (ties: lowest index),
// and the owners' phase weights are summed in 2^-52 fixed point with LDS
// integer atomics (exact, so the sum is independent of the order).
// Surface nodes use the unrotated lattice with cosine weights (Lambertian).
//
// The ownership decision is an argmax over double-precision dot products; it is
// written with this exact operation sequence (also followed by the FP64 CPU
// reference):
//   s_m  = D_m / sqrt(Dx^2 + Dy^2 + Dz^2)             (exact integer sum)
//   h    = 1 / (1 + u_z);  xy = (u_x u_y) h
//   R    = [[u_z + (u_y u_y) h, -xy, -u_x], [-xy, u_z + (u_x u_x) h, -u_y], [u_x, u_y, u_z]]
//          (R = diag(1, -1, -1) when 1 + u_z < 1e-12)
//   r_mk = fma(R_k2, s_m2, fma(R_k1, s_m1, R_k0 s_m0))
//   v_im = fma(p_i2, r_m2, fma(p_i1, r_m1, p_i0 r_m0))
// with no other contraction, hence the pragma below and -ffp-contract=off.
#include "device.hpp"
#include "internal.hpp"

#pragma clang fp contract(off)

namespace sg {

namespace {

constexpr double kFix = 4503599627370496.0;  // 2^52
constexpr double kUnfix = 1.0 / 4503599627370496.0;

template <class Real, class BlkT, bool kWriteQ>
__global__ __launch_bounds__(64) void k_qbuild(
    int N, int nvox, const long long *__restrict__ adj_ptr, const int *__restrict__ adj_idx,
    const int *__restrict__ pos, const double *__restrict__ lat, const double *__restrict__ tab, int NF, int n_phase,
    const float *__restrict__ frac, double sun_x, double sun_y, double sun_z, Real mu0, const Real *__restrict__ T,
    const Real *__restrict__ rho, const Real *__restrict__ Tsun, const long long *__restrict__ nodeoff,
    BlkT *__restrict__ val, Real *__restrict__ S, float *__restrict__ qsun) {
#pragma clang fp contract(off)
    extern __shared__ double smem[];
    double *sx = smem, *sy = smem + 64, *sz = smem + 128;
    double *rx = smem + 192, *ry = smem + 256, *rz = smem + 320;
    unsigned long long *bins = reinterpret_cast<unsigned long long *>(smem + 384);

    const int l = blockIdx.x;
    const int lane = threadIdx.x;
    const long long off = adj_ptr[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    if (d == 0) return;
    const bool surf = l >= nvox;

    if (lane < d) {
        const int j = adj_idx[off + lane];
        const long long Dx = (long long)pos[3 * j] - pos[3 * l];
        const long long Dy = (long long)pos[3 * j + 1] - pos[3 * l + 1];
        const long long Dz = (long long)pos[3 * j + 2] - pos[3 * l + 2];
        const double nrm = sqrt((double)(Dx * Dx + Dy * Dy + Dz * Dz));
        sx[lane] = (double)Dx / nrm;
        sy[lane] = (double)Dy / nrm;
        sz[lane] = (double)Dz / nrm;
    }
    // lattice points and their phase weights in fixed point
    const bool has0 = lane < NF, has1 = lane + 64 < NF;
    double p0x = 0, p0y = 0, p0z = 0, p1x = 0, p1y = 0, p1z = 0;
    unsigned long long w0 = 0, w1 = 0;
    if (has0) {
        p0x = lat[3 * lane]; p0y = lat[3 * lane + 1]; p0z = lat[3 * lane + 2];
        double w;
        if (surf) {
            w = tab[n_phase * NF + lane];
        } else {
            w = 0.0;
            for (int k = 0; k < n_phase; ++k) {
                const double f = frac ? (double)frac[(long long)k * nvox + l] : 1.0;
                w = w + f * tab[k * NF + lane];
            }
        }
        w0 = (unsigned long long)llrint(w * kFix);
    }
    if (has1) {
        const int i = lane + 64;
        p1x = lat[3 * i]; p1y = lat[3 * i + 1]; p1z = lat[3 * i + 2];
        double w;
        if (surf) {
            w = tab[n_phase * NF + i];
        } else {
            w = 0.0;
            for (int k = 0; k < n_phase; ++k) {
                const double f = frac ? (double)frac[(long long)k * nvox + l] : 1.0;
                w = w + f * tab[k * NF + i];
            }
        }
        w1 = (unsigned long long)llrint(w * kFix);
    }
    __syncthreads();

    const Real rl = rho ? rho[l] : (Real)0;
    const Real tsun = Tsun ? Tsun[l] : (Real)0;
    // the node's block, column-major: element (row = out-edge n, column = in-edge m) at
    // m d + n, so each column is one coalesced store of d values
    BlkT *blk = val + nodeoff[l];
    const int n_in = surf ? 1 : d + 1;
    for (int a = 0; a < n_in; ++a) {
        if (lane < d) {
            const double s0 = sx[lane], s1 = sy[lane], s2 = sz[lane];
            if (surf) {
                rx[lane] = s0; ry[lane] = s1; rz[lane] = s2;
            } else {
                double ux, uy, uz;
                if (a < d) { ux = -sx[a]; uy = -sy[a]; uz = -sz[a]; }
                else { ux = sun_x; uy = sun_y; uz = sun_z; }
                double R0, R1, R2, R3, R4, R5, R6, R7, R8;
                if (1.0 + uz < 1e-12) {
                    R0 = 1.0; R1 = 0.0; R2 = 0.0; R3 = 0.0; R4 = -1.0; R5 = 0.0; R6 = 0.0; R7 = 0.0; R8 = -1.0;
                } else {
                    const double h = 1.0 / (1.0 + uz);
                    const double xy = (ux * uy) * h;
                    R0 = uz + (uy * uy) * h; R1 = -xy; R2 = -ux;
                    R3 = -xy; R4 = uz + (ux * ux) * h; R5 = -uy;
                    R6 = ux; R7 = uy; R8 = uz;
                }
                rx[lane] = fma(R2, s2, fma(R1, s1, R0 * s0));
                ry[lane] = fma(R5, s2, fma(R4, s1, R3 * s0));
                rz[lane] = fma(R8, s2, fma(R7, s1, R6 * s0));
            }
            bins[lane] = 0ull;
        }
        __syncthreads();
        // argmax with ties to the lowest index: the index moves only on a strict
        // increase, and the running maximum (fmax) equals the kept value on ties
        int o0 = 0, o1 = 0;
        double b0 = -__builtin_inf(), b1 = -__builtin_inf();
        for (int m = 0; m < d; ++m) {
            const double qx = rx[m], qy = ry[m], qz = rz[m];
            const double v0 = fma(p0z, qz, fma(p0y, qy, p0x * qx));
            const double v1 = fma(p1z, qz, fma(p1y, qy, p1x * qx));
            o0 = v0 > b0 ? m : o0;
            o1 = v1 > b1 ? m : o1;
            b0 = fmax(b0, v0);
            b1 = fmax(b1, v1);
        }
        if (has0) atomicAdd(&bins[o0], w0);
        if (has1) atomicAdd(&bins[o1], w1);
        __syncthreads();
        if (lane < d) {
            const double Q = (double)(long long)bins[lane] * kUnfix;
            const long long b = off + lane;
            if (surf) {
                for (int m = 0; m < d; ++m) {
                    if (kWriteQ) blk[m * d + lane] = (BlkT)Q;
                    else blk[m * d + lane] = (BlkT)(T[off + m] * rl * (Real)Q);
                }
                if (!kWriteQ) S[b] = rl * mu0 * tsun * (Real)Q;
                qsun[b] = (float)Q;
            } else if (a < d) {
                if (kWriteQ) blk[a * d + lane] = (BlkT)Q;
                else blk[a * d + lane] = (BlkT)(T[off + a] * rl * (Real)Q);
            } else {
                if (!kWriteQ) S[b] = tsun * rl * (Real)Q;
                qsun[b] = (float)Q;
            }
        }
        __syncthreads();
    }
}

}  // namespace

template <class Real>
void launch_qbuild(Scene &s, hipStream_t st, int write_q) {
    const size_t shm = 448 * sizeof(double);
    if (write_q) {
        hipLaunchKernelGGL((k_qbuild<Real, float, true>), dim3(s.N), dim3(64), shm, st, s.N, s.nvox, s.adj_ptr,
                           s.adj_idx, s.pos, s.lat, s.tab, s.n_fib, s.n_phase, s.frac, s.sun_in[0], s.sun_in[1],
                           s.sun_in[2], (Real)s.mu0, (const Real *)nullptr, (const Real *)nullptr,
                           (const Real *)nullptr, s.nodeoff, s.q, (Real *)nullptr, s.qsun);
    } else {
        hipLaunchKernelGGL((k_qbuild<Real, Real, false>), dim3(s.N), dim3(64), shm, st, s.N, s.nvox, s.adj_ptr,
                           s.adj_idx, s.pos, s.lat, s.tab, s.n_fib, s.n_phase, s.frac, s.sun_in[0], s.sun_in[1],
                           s.sun_in[2], (Real)s.mu0, (const Real *)s.T, (const Real *)s.rho, (const Real *)s.Tsun,
                           s.nodeoff, (Real *)s.val, (Real *)s.S, s.qsun);
    }
}

template void launch_qbuild<float>(Scene &, hipStream_t, int);
template void launch_qbuild<double>(Scene &, hipStream_t, int);

}  // namespace sg

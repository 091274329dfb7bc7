// Many wavelengths over one scattering graph (Sec. 3: when only absorption
// changes between wavelengths, the geometry, the graph and the phase cells are
// computed once and reused; path integrals are kept per medium component).
//
// Per wavelength lambda with absorption multiplier s:
//   tau_e(s) = tau_s,e + s tau_a,e            (exact by linearity of the path integral)
//   T_e      = exp(-tau_e(s)),  rho_l(s) = w(s) (1 - exp(-mu_e(s) dx))  (albedo on the surface)
//   S_b      = rho_l T_sun,l (mu0 on the surface) Qsun_b
//   y_b      = S_b + rho_l sum_m Q_l[n][m] T_{a_m} x_{a_m}
// The SpMM keeps the wavelengths in the lanes of a wavefront (lambda fastest in
// every [E][n_lambda] array), so each node's phase-cell block Q (shared by all
// wavelengths, column-major within the block) is read once per sweep for all
// of them.  The grid is persistent: a fixed set of workgroups strides over node
// groups.
#include "device.hpp"
#include "internal.hpp"

namespace sg {

namespace {

// rho_l(lambda) and the solar factor T_sun,l(lambda) (x mu0 on the surface); mu_s, mu_a:
// the medium at each of the nvol volume nodes.
__global__ __launch_bounds__(256) void k_bnode_coef(int N, int nvol, int nl, const float *__restrict__ mu_s,
                                                   const float *__restrict__ mu_a, const float *__restrict__ albedo,
                                                   const float *__restrict__ tsun_s, const float *__restrict__ tsun_a,
                                                   const float *__restrict__ abs_scale, float dx, float mu0,
                                                   int mode, float *__restrict__ brho, float *__restrict__ bsrc) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= (long long)N * nl) return;
    const int l = (int)(i / nl), lam = (int)(i % nl);
    const float s = abs_scale[lam];
    float r;
    if (l < nvol) {
        const float ms = mu_s[l];
        const float me = ms + s * mu_a[l];
        if (mode == 1) r = ms * dx;
        else r = me > 0.f ? (ms / me) * (-expm1f(-me * dx)) : 0.f;
    } else {
        r = albedo[l - nvol];
    }
    const float ts = expf(-(tsun_s[l] + s * tsun_a[l]));
    brho[i] = r;
    bsrc[i] = l < nvol ? ts : mu0 * ts;
}

// One node per wavefront, lanes = wavelengths (tiles of 64).  The node's phase-cell
// block Q is staged, coalesced, in the wavefront's LDS slice and its entries are read
// as broadcasts (measured: reading the columns through scalar loads instead exposes
// their latency, 1.4x slower at 64 wavelengths); the in-edge list and optical depths
// are loaded once, coalesced, and broadcast with readlane; eight input gathers are in
// flight at a time; the node's rows are accumulated in registers, the row count
// rounded up to a multiple of 8 (DB) so the column reads are unguarded (the LDS slice
// is padded past the block by 64 floats).
// kResidual: FP64 residual r = S - x + K x of an FP64 iterate instead of a sweep.
// exp(-(tau_s + s tau_a)) as one hardware exp2; its relative error (~|tau| 1e-7) is
// below that of the FP32 path integral itself.  The sweep and the FP64 residual use
// the same function, so iterative refinement sees one matrix.
__device__ __forceinline__ float edge_T(float ts, float ta, float s) {
    return __builtin_amdgcn_exp2f(-(ts + s * ta) * 1.4426950408889634f);
}

// n passes of 64 consecutive block elements from t0 into the wavefront's LDS slice
template <int n>
__device__ __forceinline__ void stage_q(const float *__restrict__ qg, float *__restrict__ qs, int t0, int nq,
                                        int lane) {
    float v[n];
#pragma unroll
    for (int j = 0; j < n; ++j) v[j] = qg[min(t0 + j * 64 + lane, nq - 1)];
#pragma unroll
    for (int j = 0; j < n; ++j) qs[min(t0 + j * 64 + lane, nq - 1)] = v[j];
}

template <int DB, class XT, class YT, class AccT, bool kResidual>
__device__ __forceinline__ float2 wide_node(int l, int lane, int lam, bool lv, float s, int nl, int monitor,
                                            float *__restrict__ qs, const long long *__restrict__ adj_ptr,
                                            const long long *__restrict__ nodeoff, const int *__restrict__ rev,
                                            const float *__restrict__ q, const float *__restrict__ qsun,
                                            const float *__restrict__ tau_s, const float *__restrict__ tau_a,
                                            const float *__restrict__ brho, const float *__restrict__ bsrc,
                                            const float *__restrict__ rhs, const XT *__restrict__ x,
                                            YT *__restrict__ y) {
    constexpr int kU = 8;
    const long long off = adj_ptr[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    const long long base = nodeoff[l];
    // per in-edge data in lane m (lanes past d repeat the last in-edge), then the node's
    // phase-cell block into this wavefront's LDS slice: as many 64-element passes as the
    // block needs, at most 16 at a time (a wave-uniform switch into straight-line copies,
    // so the loads are issued back to back; out-of-range lanes reload and rewrite the last
    // element)
    const long long em = off + min(lane, d - 1);
    const int rv = rev[em];
    const float ts = tau_s[em], ta = tau_a[em];
    {
        const int nq = d * d;
        for (int t0 = 0; t0 < nq; t0 += 64 * 16) {
            switch (min(16, (nq - t0 + 63) >> 6)) {
#define SG_STAGE_CASE(n) \
    case n: stage_q<n>(q + base, qs, t0, nq, lane); break;
                SG_STAGE_CASE(1) SG_STAGE_CASE(2) SG_STAGE_CASE(3) SG_STAGE_CASE(4) SG_STAGE_CASE(5)
                SG_STAGE_CASE(6) SG_STAGE_CASE(7) SG_STAGE_CASE(8) SG_STAGE_CASE(9) SG_STAGE_CASE(10)
                SG_STAGE_CASE(11) SG_STAGE_CASE(12) SG_STAGE_CASE(13) SG_STAGE_CASE(14) SG_STAGE_CASE(15)
                default: stage_q<16>(q + base, qs, t0, nq, lane);
#undef SG_STAGE_CASE
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    AccT acc[DB];
#pragma unroll
    for (int n = 0; n < DB; ++n) acc[n] = (AccT)0;
    for (int m0 = 0; m0 < d; m0 += kU) {
        XT xv[kU];
#pragma unroll
        for (int j = 0; j < kU; ++j) {
            const int m = min(m0 + j, 63);
            const int r = __builtin_amdgcn_readlane(rv, m);
            xv[j] = (m0 + j < d && lv) ? x[(long long)r * nl + lam] : (XT)0;
        }
#pragma unroll
        for (int j = 0; j < kU; ++j) {
            const int m = m0 + j;
            if (m < d) {
                const float tsm = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ts), m));
                const float tam = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ta), m));
                const AccT xm = (AccT)edge_T(tsm, tam, s) * (AccT)xv[j];
                const float *qm = qs + m * d;  // column m: Q[n][m], n contiguous (LDS, uniform address)
#pragma unroll
                for (int n = 0; n < DB; ++n) acc[n] += (AccT)qm[n] * xm;
            }
        }
    }
    double sum = 0.0, mrel = 0.0;  // convergence measures of this node's rows
    if (lv) {
        const float rl = brho[(long long)l * nl + lam];
        const float sl = bsrc[(long long)l * nl + lam];
#pragma unroll
        for (int n = 0; n < DB; ++n) {
            if (n < d) {
                const long long b = off + n;
                const long long bi = b * nl + lam;
                if (kResidual) {
                    const double Sb = (double)(rl * sl * qsun[b]);
                    const double rb = (Sb - (double)x[bi]) + (double)rl * (double)acc[n];
                    y[bi] = (YT)rb;
                    sum += fabs(rb);
                    mrel = fmax(mrel, keep_nan(fabs(rb) / (fabs((double)x[bi]) + kRelFloor)));
                } else {
                    const float src = rhs ? rhs[bi] : rl * sl * qsun[b];
                    const float yv = src + rl * (float)acc[n];
                    y[bi] = (YT)yv;
                    if (monitor) {
                        const double du = fabs((double)yv - (double)x[bi]);
                        sum += du;
                        mrel = fmax(mrel, keep_nan(du / (fabs((double)yv) + kRelFloor)));
                    }
                }
            }
        }
    }
    return make_float2((float)sum, (float)mrel);
}

// Occupancy hints: at the requested waves per SIMD the compiler fits each instantiation
// without spilling (the FP32 sweep: 72 VGPRs at D = 40 instead of 98; the FP64 residual up
// to D = 40: 122 instead of 144, four waves per SIMD instead of three, where five would
// spill its accumulators; the larger FP64 residuals keep their natural allocation, since
// their accumulators alone fill four waves' registers).
template <int D, bool kResidual>
constexpr int wide_waves_per_eu() { return kResidual ? (D <= 40 ? 4 : 1) : (D <= 40 ? 7 : 5); }

template <int D, class XT, class YT, class AccT, bool kResidual>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(wide_waves_per_eu<D, kResidual>()))) void k_spmm_wide(
    int N, int nl, int groups, const long long *__restrict__ adj_ptr, const long long *__restrict__ nodeoff,
    const int *__restrict__ rev, const float *__restrict__ q, const float *__restrict__ qsun,
    const float *__restrict__ tau_s, const float *__restrict__ tau_a, const float *__restrict__ abs_scale,
    const float *__restrict__ brho, const float *__restrict__ bsrc, const float *__restrict__ rhs,
    const XT *__restrict__ x, YT *__restrict__ y, float2 *__restrict__ meas, int monitor, int dmax) {
    extern __shared__ float qs_all[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lam = blockIdx.y * 64 + lane;
    const bool lv = lam < nl;
    const float s = lv ? abs_scale[lam] : 0.f;
    float *qs = qs_all + (size_t)w * (dmax * dmax + 64);  // + padding: whole-column reads past d
    const int waves = blockDim.x >> 6;
    for (int g = blockIdx.x; g < groups; g += gridDim.x) {
        const int l = __builtin_amdgcn_readfirstlane(g * waves + w);
        if (l >= N) break;
        const int d = (int)(adj_ptr[l + 1] - adj_ptr[l]);
        if (d == 0) {  // an isolated node: no rows
            if (monitor && lv) meas[(long long)l * nl + lam] = make_float2(0.f, 0.f);
            continue;
        }
#ifdef SG_DEBUG_BOUNDS
        {  // the node's Q block and its in-edges' reverse ids
            bool ok = SG_IN(nodeoff[l] + (long long)d * d - 1, nodeoff[N], 0x401);
            if (lane < d) ok = SG_IN(rev[adj_ptr[l] + lane], adj_ptr[N], 0x402) && ok;
            if (!__all(ok)) continue;
        }
#endif
        const int bucket = (d + 7) >> 3;
        float2 part = make_float2(0.f, 0.f);
#define SG_NODE(DB)                                                                                              \
    part = wide_node<DB, XT, YT, AccT, kResidual>(l, lane, lam, lv, s, nl, monitor, qs, adj_ptr, nodeoff, rev, q, \
                                              qsun, tau_s, tau_a, brho, bsrc, rhs, x, y)
        if (bucket <= 1) { SG_NODE(8); }
        else if (bucket == 2) { if constexpr (D >= 16) SG_NODE(16); }
        else if (bucket == 3) { if constexpr (D >= 24) SG_NODE(24); }
        else if (bucket == 4) { if constexpr (D >= 32) SG_NODE(32); }
        else if (bucket == 5) { if constexpr (D >= 40) SG_NODE(40); }
        else if (bucket == 6) { if constexpr (D >= 48) SG_NODE(48); }
        else if (bucket == 7) { if constexpr (D >= 56) SG_NODE(56); }
        else { if constexpr (D >= 64) SG_NODE(64); }
#undef SG_NODE
        if (monitor && lv) meas[(long long)l * nl + lam] = part;  // per node and wavelength
    }
}

// The first batched Neumann iterate from x = 0: x = rhs, or the solar source
// rho_l s_l Qsun_b, computed as the sweep computes it (plus rho_l times a zero sum), so
// it has the sweep's bits; measures per (node, wavelength).
__global__ __launch_bounds__(256) void k_bfirst(int N, int nl, const long long *__restrict__ adj_ptr,
                                                const float *__restrict__ qsun, const float *__restrict__ brho,
                                                const float *__restrict__ bsrc, const float *__restrict__ rhs,
                                                float *__restrict__ x, float2 *__restrict__ meas) {
    const int lane = threadIdx.x & 63;
    const int l = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const int lam = blockIdx.y * 64 + lane;
    if (l >= N || lam >= nl) return;
    const long long off = adj_ptr[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    const float rl = brho[(long long)l * nl + lam], sl = bsrc[(long long)l * nl + lam];
    double sum = 0.0, mrel = 0.0;
    for (int n = 0; n < d; ++n) {
        const long long bi = (off + n) * nl + lam;
        const float src = rhs ? rhs[bi] : rl * sl * qsun[off + n];
        const float yv = src + rl * 0.0f;
        x[bi] = yv;
        const double du = fabs((double)yv);
        sum += du;
        mrel = fmax(mrel, keep_nan(du / (du + kRelFloor)));
    }
    meas[(long long)l * nl + lam] = make_float2((float)sum, (float)mrel);
}

// ---- wavelength tiles narrower than a wavefront -------------------------------------
// For n_lambda <= 32 a wavefront holds 64 / W node slots of W wavelength lanes each, so
// a small wavelength count does not leave lanes idle.  Each slot's in-edge data (rev,
// tau_s, tau_a) goes to a small LDS slice; the phase-cell columns are read straight
// from memory with 16-byte loads (the lanes of a slot share the addresses, so each
// load costs one request per slot).  Per lane the arithmetic is exactly that of the
// full-wavefront kernel (same expressions, columns in the same order), so the two give
// the same bits.
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));

template <int DB, class XT, class YT, class AccT, bool kResidual>
__device__ __forceinline__ float2 pack_node(int l, int lam, bool lv, float s, int nl, int monitor, long long off,
                                            int d, long long base, int dw, const int *__restrict__ srv,
                                            const float *__restrict__ sts, const float *__restrict__ sta,
                                            const float *__restrict__ q, const float *__restrict__ qsun,
                                            const float *__restrict__ brho, const float *__restrict__ bsrc,
                                            const float *__restrict__ rhs, const XT *__restrict__ x,
                                            YT *__restrict__ y) {
    AccT acc[DB];
#pragma unroll
    for (int n = 0; n < DB; ++n) acc[n] = (AccT)0;
    for (int m = 0; m < dw; ++m) {
        // slots with fewer in-edges repeat their last column with a zero input: adding
        // Q * 0 leaves every valid row's sum unchanged
        const bool mv = m < d;
        const int mc = min(m, d - 1);
        const XT xin = (mv && lv) ? x[(long long)srv[mc] * nl + lam] : (XT)0;
        const AccT xm = (AccT)edge_T(sts[mc], sta[mc], s) * (AccT)xin;
        const f4u *qm = reinterpret_cast<const f4u *>(q + base + (long long)mc * d);
#pragma unroll
        for (int c = 0; c < DB / 4; ++c) {
            const f4u v = qm[c];
            acc[4 * c] += (AccT)v.x * xm;
            acc[4 * c + 1] += (AccT)v.y * xm;
            acc[4 * c + 2] += (AccT)v.z * xm;
            acc[4 * c + 3] += (AccT)v.w * xm;
        }
    }
    double sum = 0.0, mrel = 0.0;
    if (lv) {
        const float rl = brho[(long long)l * nl + lam];
        const float sl = bsrc[(long long)l * nl + lam];
#pragma unroll
        for (int n = 0; n < DB; ++n) {
            if (n < d) {
                const long long b = off + n;
                const long long bi = b * nl + lam;
                if (kResidual) {
                    const double Sb = (double)(rl * sl * qsun[b]);
                    const double rb = (Sb - (double)x[bi]) + (double)rl * (double)acc[n];
                    y[bi] = (YT)rb;
                    sum += fabs(rb);
                    mrel = fmax(mrel, keep_nan(fabs(rb) / (fabs((double)x[bi]) + kRelFloor)));
                } else {
                    const float src = rhs ? rhs[bi] : rl * sl * qsun[b];
                    const float yv = src + rl * (float)acc[n];
                    y[bi] = (YT)yv;
                    if (monitor) {
                        const double du = fabs((double)yv - (double)x[bi]);
                        sum += du;
                        mrel = fmax(mrel, keep_nan(du / (fabs((double)yv) + kRelFloor)));
                    }
                }
            }
        }
    }
    return make_float2((float)sum, (float)mrel);
}

template <int W, int D, class XT, class YT, class AccT, bool kResidual>
__global__ __launch_bounds__(256) void k_spmm_pack(
    int N, int nl, int groups, const long long *__restrict__ adj_ptr, const long long *__restrict__ nodeoff,
    const int *__restrict__ rev, const float *__restrict__ q, const float *__restrict__ qsun,
    const float *__restrict__ tau_s, const float *__restrict__ tau_a, const float *__restrict__ abs_scale,
    const float *__restrict__ brho, const float *__restrict__ bsrc, const float *__restrict__ rhs,
    const XT *__restrict__ x, YT *__restrict__ y, float2 *__restrict__ meas, int monitor) {
    constexpr int P = 64 / W;  // node slots per wavefront
    __shared__ int srv_all[4][P][64];
    __shared__ float sts_all[4][P][64], sta_all[4][P][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int k = lane / W, lam = lane - k * W;
    const bool lam_ok = lam < nl;
    const float s = lam_ok ? abs_scale[lam] : 0.f;
    int *srv = srv_all[w][k];
    float *sts = sts_all[w][k], *sta = sta_all[w][k];
    for (int g = blockIdx.x; g < groups; g += gridDim.x) {
        const int l0 = __builtin_amdgcn_readfirstlane((g * 4 + w) * P);
        if (l0 >= N) break;
        const int l = l0 + k;
        const bool node_ok = l < N;
        long long off = 0, base = 0;
        int d = 0;
        if (node_ok) {
            off = adj_ptr[l];
            d = (int)(adj_ptr[l + 1] - off);
            base = nodeoff[l];
        }
        for (int m = lam; m < d; m += W) {
            const long long e = off + m;
            srv[m] = SG_IN(rev[e], adj_ptr[N], 0x403) ? rev[e] : (int)e;
            sts[m] = tau_s[e];
            sta[m] = tau_a[e];
        }
        __builtin_amdgcn_wave_barrier();
        int dw = d;  // the wavefront's largest degree (uniform loop bound)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) dw = max(dw, __shfl_xor(dw, o, 64));
        dw = __builtin_amdgcn_readfirstlane(dw);
        const bool lv = node_ok && lam_ok && d > 0;
        float2 part = make_float2(0.f, 0.f);
        if (dw > 0) {
            const int bucket = (dw + 7) >> 3;
#define SG_PACK(DB)                                                                                        \
    part = pack_node<DB, XT, YT, AccT, kResidual>(l, lam, lv, s, nl, monitor, off, max(d, 1), base, dw, srv, sts, \
                                              sta, q, qsun, brho, bsrc, rhs, x, y)
            if (bucket <= 1) { SG_PACK(8); }
            else if (bucket == 2) { if constexpr (D >= 16) SG_PACK(16); }
            else if (bucket == 3) { if constexpr (D >= 24) SG_PACK(24); }
            else if (bucket == 4) { if constexpr (D >= 32) SG_PACK(32); }
            else if (bucket == 5) { if constexpr (D >= 40) SG_PACK(40); }
            else if (bucket == 6) { if constexpr (D >= 48) SG_PACK(48); }
            else if (bucket == 7) { if constexpr (D >= 56) SG_PACK(56); }
            else { if constexpr (D >= 64) SG_PACK(64); }
#undef SG_PACK
        }
        if (monitor && node_ok && lam_ok) meas[(long long)l * nl + lam] = part;
        __builtin_amdgcn_wave_barrier();  // the slices are rewritten by the next group
    }
}

// One wavelength of a batched scene in FP64, for its GMRES fallback: one wavefront per node,
// lane n = the node's row n (degree <= 64), columns summed in increasing order.  The matrix
// is the batched sweep's at wavelength lam, K[b, a] = rho_l Q[b, a] T_a with T_a from the
// same exp2 (so the fallback solves the system the batched residual measures).
//   kResidual: r = S - v + K v with the node's measures (sum |r|, max |r| / (|v| + floor));
//   otherwise: w = v - K v.
template <bool kResidual>
__global__ __launch_bounds__(256) void k_blam64(int N, int nl, int lam, float s, const long long *__restrict__ adj_ptr,
                                               const long long *__restrict__ nodeoff, const int *__restrict__ rev,
                                               const float *__restrict__ q, const float *__restrict__ qsun,
                                               const float *__restrict__ tau_s, const float *__restrict__ tau_a,
                                               const float *__restrict__ brho, const float *__restrict__ bsrc,
                                               const double *__restrict__ v, double *__restrict__ w,
                                               float2 *__restrict__ meas) {
    const int l = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (l >= N) return;
    const long long off = adj_ptr[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    if (d == 0) {
        if (kResidual && lane == 0) meas[l] = make_float2(0.f, 0.f);
        return;
    }
    const long long base = nodeoff[l];
    const long long em = off + min(lane, d - 1);  // lane m: in-edge m's input
    const int rv0 = rev[em];
    const double xin = (double)edge_T(tau_s[em], tau_a[em], s) * v[SG_IN(rv0, adj_ptr[N], 0x405) ? rv0 : (int)em];
    const bool act = lane < d;
    double acc = 0.0;
    for (int m = 0; m < d; ++m) {
        const double xm = __shfl(xin, m, 64);
        if (act) acc += (double)q[base + (long long)m * d + lane] * xm;
    }
    double a = 0.0, u = 0.0;
    if (act) {
        const long long b = off + lane;
        const float rlf = brho[(long long)l * nl + lam];
        if (kResidual) {
            const double Sb = (double)(rlf * bsrc[(long long)l * nl + lam] * qsun[b]);
            const double rb = (Sb - v[b]) + (double)rlf * acc;
            w[b] = rb;
            a = fabs(rb);
            u = keep_nan(a / (fabs(v[b]) + kRelFloor));
        } else {
            w[b] = v[b] - (double)rlf * acc;
        }
    }
    if (kResidual) {
        a = wave_sum(a);
        u = wave_max(u);
        if (lane == 0) meas[l] = make_float2((float)a, (float)u);
    }
}

// one wavelength's slice of an edge-major [E][nl] vector, and back
__global__ void k_lam_take64(const double *__restrict__ x, int nl, int lam, long long E, double *__restrict__ out) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e < E) out[e] = x[e * nl + lam];
}
__global__ void k_lam_put64(const double *__restrict__ in, int nl, int lam, long long E, double *__restrict__ x) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e < E) x[e * nl + lam] = in[e];
}

__global__ void k_lam_scale_f32(float *__restrict__ b, const double *__restrict__ sc, int nl, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = (float)((double)b[i] * sc[i % nl]);
}

__global__ void k_lam_axpy(double *__restrict__ x, const float *__restrict__ d, const double *__restrict__ sc, int nl,
                           long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        x[i] += (double)d[i] / sc[i % nl];
}

// [nl][E] -> [E][nl] (edge-major, wavelength fastest): coalesced writes
__global__ __launch_bounds__(256) void k_lam_to_edge_major(const double *__restrict__ src, double *__restrict__ dst,
                                                          int nl, long long E) {
    const long long n = E * nl;
    for (long long t = blockIdx.x * 256LL + threadIdx.x; t < n; t += (long long)gridDim.x * 256) {
        const long long e = t / nl, k = t - e * nl;
        dst[t] = src[k * E + e];
    }
}

__global__ void k_f32_to_64(const float *__restrict__ a, double *__restrict__ b, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = (double)a[i];
}

__global__ void k_fill_f32(float *__restrict__ a, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        a[i] = 0.f;
}

__device__ __forceinline__ double theta_mix_b(const PhaseSet &pm, const float *__restrict__ frac, int stride, int v,
                                              double mu) {
    double th = 0.0;
    for (int c = 0; c < pm.n; ++c) {
        const double f = frac ? (double)frac[(long long)c * stride + v] : 1.0;
        th += f * phase_theta(pm, c, mu);
    }
    return th;
}

// J[l][lambda]: one wavefront per node; lane m evaluates in-edge m's phase function
// once, then the lanes (wavelengths) accumulate in FP64.
template <class PhiT>
__global__ __launch_bounds__(64) void k_bnode_J(int N, int nvol, int nl, const long long *__restrict__ adj_ptr,
                                               const int *__restrict__ adj_idx, const int *__restrict__ rev,
                                               const int *__restrict__ pos, const float *__restrict__ tau_s,
                                               const float *__restrict__ tau_a, const float *__restrict__ abs_scale,
                                               const float *__restrict__ bsrc, const PhiT *__restrict__ phi,
                                               PhaseSet pm, const float *__restrict__ frac, double sx, double sy,
                                               double sz, double vx, double vy, double vz, int multiple,
                                               int per, long long wx, long long wy, double *__restrict__ J) {
    __shared__ double th[64];
    const int l = blockIdx.x;
    const int lane = threadIdx.x;
    const long long off = adj_ptr[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    const bool vol = l < nvol;
    if (lane < d) {
        double t = 1.0;
        if (vol) {
            const int j0 = adj_idx[off + lane];
            const int j = SG_IN(j0, N, 0x404) ? j0 : l;
            const long long Dx = min_image((long long)pos[3 * l] - pos[3 * j], wx, per & 1);
            const long long Dy = min_image((long long)pos[3 * l + 1] - pos[3 * j + 1], wy, per & 2);
            const long long Dz = (long long)pos[3 * l + 2] - pos[3 * j + 2];
            const double nrm = sqrt((double)(Dx * Dx + Dy * Dy + Dz * Dz));
            const double mu = ((double)Dx / nrm) * vx + ((double)Dy / nrm) * vy + ((double)Dz / nrm) * vz;
            t = theta_mix_b(pm, frac, nvol, l, mu);
        }
        th[lane] = t;
    }
    const double th_sun = vol ? theta_mix_b(pm, frac, nvol, l, sx * vx + sy * vy + sz * vz) : 1.0;
    __syncthreads();
    for (int l0 = 0; l0 < nl; l0 += 64) {
        const int lam = l0 + lane;
        if (lam >= nl) continue;
        const float s = abs_scale[lam];
        double acc = th_sun * (double)bsrc[(long long)l * nl + lam];  // T_sun (x mu0 on the surface)
        if (multiple) {
            for (int m = 0; m < d; ++m) {
                const long long e = off + m;
                const double T = (double)edge_T(tau_s[e], tau_a[e], s);
                acc += th[m] * T * (double)phi[(long long)rev[e] * nl + lam];
            }
        }
        J[(long long)l * nl + lam] = acc;
    }
}

// One wavefront per pixel, lanes = wavelengths: the voxel walk is the same for all
// lanes, each accumulates its own wavelength in FP64.
__global__ __launch_bounds__(64) void k_bpixels(int nx, int ny, int nz, int per, int nl, const float *__restrict__ mu_s,
                                               const float *__restrict__ mu_a, const float *__restrict__ abs_scale,
                                               double len_view, long long vdx, long long vdy, long long vdz,
                                               long long sdx, long long sdy, long long sdz, double len_sun,
                                               const float *__restrict__ albedo, const double *__restrict__ J,
                                               int surface, double mu0, int nvol,
                                               const long long *__restrict__ los_ptr, const int *__restrict__ los_node,
                                               const double *__restrict__ los_t, double *__restrict__ out) {
    const int p = blockIdx.x;
    const int lane = threadIdx.x;
    const long long ix = p % nx, iy = p / nx;
    const long long px = ix * kFx + kFx / 2, py = iy * kFx + kFx / 2;
    const double a_pi = (double)albedo[p] / 3.14159265358979323846;
    for (int l0 = 0; l0 < nl; l0 += 64) {
        const int lam = min(l0 + lane, nl - 1);
        const double s = (double)abs_scale[lam];
        double tau_tot = 0.0;
        voxel_walk(nx, ny, nz, per, px, py, 0, vdx, vdy, vdz, true, [&](int x, int y, int z, long long num, long long den) {
            const long long v = x + (long long)nx * (y + (long long)ny * z);
            if (SG_IN(v, (long long)nx * ny * nz, 0x406))
                tau_tot += ((double)mu_s[v] + s * (double)mu_a[v]) * ((double)num / (double)den * len_view);
            return true;
        });
        double I = 0.0, cum = 0.0;
        if (!los_ptr) {
            voxel_walk(nx, ny, nz, per, px, py, 0, vdx, vdy, vdz, true, [&](int x, int y, int z, long long num, long long den) {
                const long long v = x + (long long)nx * (y + (long long)ny * z);
                if (!SG_IN(v, (long long)nx * ny * nz, 0x407)) return true;
                const double ms = (double)mu_s[v];
                const double me = ms + s * (double)mu_a[v];
                const double tk = me * ((double)num / (double)den * len_view);
                const double om = me > 0.0 ? ms / me : 0.0;
                I += exp(-(tau_tot - (cum + tk))) * (om * (-expm1(-tk))) * J[v * nl + lam];
                cum += tk;
                return true;
            });
        } else {
            // general nodes: chords cut at the ends of the line's elements (see k_pixels)
            const long long e1 = los_ptr[p + 1];
            long long e = los_ptr[p];
            double t = 0.0;
            voxel_walk(nx, ny, nz, per, px, py, 0, vdx, vdy, vdz, true, [&](int x, int y, int z, long long num, long long den) {
                const long long v = x + (long long)nx * (y + (long long)ny * z);
                if (!SG_IN(v, (long long)nx * ny * nz, 0x408)) return true;
                const double ms = (double)mu_s[v];
                const double me = ms + s * (double)mu_a[v];
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
                    if (node >= 0 && SG_IN(node, nvol, 0x409))
                        I += exp(-(tau_tot - (cum + tk))) * (om * (-expm1(-tk))) * J[(long long)node * nl + lam];
                    cum += tk;
                    a = b;
                }
                t = t1;
                return true;
            });
        }
        if (surface) {
            I += exp(-tau_tot) * a_pi * J[((long long)nvol + p) * nl + lam];
        } else {
            double ts = 0.0;
            voxel_walk(nx, ny, nz, per, px, py, 0, sdx, sdy, sdz, true, [&](int x, int y, int z, long long num, long long den) {
                const long long v = x + (long long)nx * (y + (long long)ny * z);
                if (SG_IN(v, (long long)nx * ny * nz, 0x40a))
                    ts += ((double)mu_s[v] + s * (double)mu_a[v]) * ((double)num / (double)den * len_sun);
                return true;
            });
            I += exp(-tau_tot) * a_pi * mu0 * exp(-ts);
        }
        if (l0 + lane < nl) out[(long long)(l0 + lane) * nx * ny + p] = I;
    }
}

inline int grid_for(long long n) {
    long long g = (n + 255) / 256;
    return (int)(g > 4096 ? 4096 : (g < 1 ? 1 : g));
}

}  // namespace

void launch_bnode_coef(Scene &s, hipStream_t st) {
    const long long n = (long long)s.N * s.n_lambda;
    hipLaunchKernelGGL(k_bnode_coef, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s.N, s.n_vol, s.n_lambda,
                       node_mu_s(s), node_mu_a(s), s.albedo, (const float *)s.tsun_s, (const float *)s.tsun_a, s.abs_scale_d,
                       (float)s.voxel_m, (float)s.mu0, s.weight_mode, s.brho, s.bsrc);
}

// wavefronts per workgroup: four unless the LDS slices of the phase-cell blocks would pass 60 KB
int wide_waves(const Scene &s) { return (size_t)4 * (s.dmax * s.dmax + 64) * sizeof(float) <= 60 * 1024 ? 4 : 2; }

// Wavelength lanes per node: 8, 16, 32 or 64 (counts above 64 use several 64-lane
// columns of the full-wavefront kernel).  The narrow tiles read the phase-cell columns
// through the vector cache, once per node slot; the full-wavefront kernel stages them
// in LDS.  Measured on MI355X, 8 and 16 lanes beat the full wavefront by up to 2x while
// 32 lanes lose to it by about 1.5x, so 32 is left to the autotuner.
int smallest_tile(int n_lambda) { return n_lambda <= 8 ? 8 : n_lambda <= 16 ? 16 : n_lambda <= 32 ? 32 : 64; }
int default_tile(int n_lambda) { return smallest_tile(n_lambda) <= 16 ? smallest_tile(n_lambda) : 64; }

static int lambda_tile(const Scene &s) { return s.tile >= smallest_tile(s.n_lambda) ? s.tile : 64; }

int batched_groups(const Scene &s) {
    const int W = lambda_tile(s);
    if (W < 64) return (s.N + 4 * (64 / W) - 1) / (4 * (64 / W));
    return (s.N + wide_waves(s) - 1) / wide_waves(s);
}

template <int W, class XT, class YT, class AccT, bool kRes>
static void launch_pack(Scene &s, hipStream_t st, int grid, const float *rhs, const XT *x, YT *y, int monitor) {
    const int groups = batched_groups(s);
#define SG_PK(DD)                                                                                                  \
    hipLaunchKernelGGL((k_spmm_pack<W, DD, XT, YT, AccT, kRes>), dim3(grid), dim3(256), 0, st, s.N, s.n_lambda, groups, \
                       s.adj_ptr, s.nodeoff, s.rev, s.q, s.qsun, (const float *)s.tau_s, (const float *)s.tau_a,      \
                       s.abs_scale_d, s.brho, s.bsrc, rhs, x, y, s.meas, monitor)
    if (s.dmax <= 16) SG_PK(16);
    else if (s.dmax <= 24) SG_PK(24);
    else if (s.dmax <= 32) SG_PK(32);
    else if (s.dmax <= 40) SG_PK(40);
    else if (s.dmax <= 48) SG_PK(48);
    else if (s.dmax <= 56) SG_PK(56);
    else SG_PK(64);
#undef SG_PK
}

template <class XT, class YT, class AccT, bool kRes>
static void launch_wide(Scene &s, hipStream_t st, int grid, const float *rhs, const XT *x, YT *y, int monitor) {
    const int W = lambda_tile(s);
    grid = std::max(1, std::min(grid, batched_groups(s)));
    if (W == 8) return launch_pack<8, XT, YT, AccT, kRes>(s, st, grid, rhs, x, y, monitor);
    if (W == 16) return launch_pack<16, XT, YT, AccT, kRes>(s, st, grid, rhs, x, y, monitor);
    if (W == 32) return launch_pack<32, XT, YT, AccT, kRes>(s, st, grid, rhs, x, y, monitor);
    const int waves = wide_waves(s);
    const int groups = batched_groups(s);
    dim3 gr(grid, (s.n_lambda + 63) / 64);
    const size_t shm = (size_t)waves * (s.dmax * s.dmax + 64) * sizeof(float);
#define SG_WIDE(DD)                                                                                                 \
    hipLaunchKernelGGL((k_spmm_wide<DD, XT, YT, AccT, kRes>), gr, dim3(64 * waves), shm, st, s.N, s.n_lambda, groups, \
                       s.adj_ptr, s.nodeoff, s.rev, s.q, s.qsun, (const float *)s.tau_s, (const float *)s.tau_a,      \
                       s.abs_scale_d, s.brho, s.bsrc, rhs, x, y, s.meas, monitor, s.dmax)
    if (s.dmax <= 16) SG_WIDE(16);
    else if (s.dmax <= 24) SG_WIDE(24);
    else if (s.dmax <= 32) SG_WIDE(32);
    else if (s.dmax <= 40) SG_WIDE(40);
    else if (s.dmax <= 48) SG_WIDE(48);
    else if (s.dmax <= 56) SG_WIDE(56);
    else SG_WIDE(64);
#undef SG_WIDE
}

void launch_spmm(Scene &s, hipStream_t st, int grid, const float *rhs, const float *x, float *y, int monitor) {
    launch_wide<float, float, float, false>(s, st, grid, rhs, x, y, monitor);
}

void launch_bresidual64(Scene &s, hipStream_t st, int grid, const double *x64, float *r32) {
    launch_wide<double, float, double, true>(s, st, grid, nullptr, x64, r32, 1);
}

void launch_bresidual32(Scene &s, hipStream_t st, int grid, const float *x, float *r32) {
    launch_wide<float, float, double, true>(s, st, grid, nullptr, x, r32, 1);
}

void launch_bfirst(Scene &s, hipStream_t st, const float *rhs, float *x) {
    dim3 gr((s.N + 3) / 4, (s.n_lambda + 63) / 64);
    hipLaunchKernelGGL(k_bfirst, gr, dim3(256), 0, st, s.N, s.n_lambda, s.adj_ptr, s.qsun, s.brho, s.bsrc, rhs, x,
                       s.meas);
}

void launch_blam_residual64(Scene &s, hipStream_t st, int lam, const double *x, double *r) {
    hipLaunchKernelGGL(k_blam64<true>, dim3((s.N + 3) / 4), dim3(256), 0, st, s.N, s.n_lambda, lam, s.abs_scale[lam],
                       s.adj_ptr, s.nodeoff, s.rev, s.q, s.qsun, (const float *)s.tau_s, (const float *)s.tau_a, s.brho,
                       s.bsrc, x, r, s.meas);
    launch_measures(s, 1, s.scal, st);
}

void launch_blam_apply64(Scene &s, hipStream_t st, int lam, const double *v, double *w) {
    hipLaunchKernelGGL(k_blam64<false>, dim3((s.N + 3) / 4), dim3(256), 0, st, s.N, s.n_lambda, lam, s.abs_scale[lam],
                       s.adj_ptr, s.nodeoff, s.rev, s.q, s.qsun, (const float *)s.tau_s, (const float *)s.tau_a, s.brho,
                       s.bsrc, v, w, (float2 *)nullptr);
}

void launch_lam_take64(const double *x, int nl, int lam, long long E, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_lam_take64, dim3(grid_for(E)), dim3(256), 0, st, x, nl, lam, E, out);
}

void launch_lam_put64(const double *in, int nl, int lam, long long E, double *x, hipStream_t st) {
    hipLaunchKernelGGL(k_lam_put64, dim3(grid_for(E)), dim3(256), 0, st, in, nl, lam, E, x);
}

void launch_lam_scale_f32(float *b, const double *sc, int nl, long long n, hipStream_t st) {
    hipLaunchKernelGGL(k_lam_scale_f32, dim3(grid_for(n)), dim3(256), 0, st, b, sc, nl, n);
}

void launch_lam_axpy(double *x, const float *d, const double *sc, int nl, long long n, hipStream_t st) {
    hipLaunchKernelGGL(k_lam_axpy, dim3(grid_for(n)), dim3(256), 0, st, x, d, sc, nl, n);
}

void launch_lam_to_edge_major(const double *src, double *dst, int nl, long long E, hipStream_t st) {
    hipLaunchKernelGGL(k_lam_to_edge_major, dim3(grid_for(E * nl)), dim3(256), 0, st, src, dst, nl, E);
}

void launch_f32_to_64(const float *a, double *b, long long n, hipStream_t st) {
    hipLaunchKernelGGL(k_f32_to_64, dim3(grid_for(n)), dim3(256), 0, st, a, b, n);
}

void launch_fill_f32(float *a, long long n, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n)), dim3(256), 0, st, a, n);
}

template <class PhiT>
static void batched_gather(Scene &s, hipStream_t st, const PhiT *phi, int scatter_order, double *radiance) {
    const PhaseSet pm = phase_set(s);
    hipLaunchKernelGGL(k_bnode_J<PhiT>, dim3(s.N), dim3(64), 0, st, s.N, s.n_vol, s.n_lambda, s.adj_ptr, s.adj_idx, s.rev,
                       s.pos, (const float *)s.tau_s, (const float *)s.tau_a, s.abs_scale_d, s.bsrc, phi, pm, node_frac(s),
                       s.sun_in[0], s.sun_in[1], s.sun_in[2], s.view_u[0], s.view_u[1], s.view_u[2],
                       scatter_order == 1 ? 0 : 1, s.periodic, (long long)s.nx * kFx, (long long)s.ny * kFx, s.J);
    const double fx = s.voxel_m / 65536.0;
    const double lv = sqrt((double)s.view[0] * s.view[0] + (double)s.view[1] * s.view[1] + (double)s.view[2] * s.view[2]) * fx;
    const double ls = sqrt((double)s.sun[0] * s.sun[0] + (double)s.sun[1] * s.sun[1] + (double)s.sun[2] * s.sun[2]) * fx;
    hipLaunchKernelGGL(k_bpixels, dim3(s.npx), dim3(64), 0, st, s.nx, s.ny, s.nz, s.periodic, s.n_lambda, s.mu_s,
                       s.mu_a, s.abs_scale_d, lv, (long long)s.view[0], (long long)s.view[1], (long long)s.view[2],
                       (long long)s.sun[0], (long long)s.sun[1], (long long)s.sun[2], ls, s.albedo, s.J, s.surface,
                       s.mu0, s.n_vol, s.general ? s.los_ptr : (const long long *)nullptr, s.los_node, s.los_t,
                       radiance);
}

void launch_batched_gather(Scene &s, hipStream_t st, const double *phi, int scatter_order, double *radiance) {
    batched_gather(s, st, phi, scatter_order, radiance);
}
void launch_batched_gather(Scene &s, hipStream_t st, const float *phi, int scatter_order, double *radiance) {
    batched_gather(s, st, phi, scatter_order, radiance);
}

}  // namespace sg

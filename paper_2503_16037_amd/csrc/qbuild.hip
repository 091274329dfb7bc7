// Phase-cell weights (Sec. 2, Eq. 7; Fibonacci lattice of Sec. 3) fused with the
// flux-matrix values (Eq. 6) and the direct-solar source (Eq. 9).
//
// One 64-lane wavefront per node l.  For every incoming propagation direction u
// (each in-edge, then the sunlight) the lattice is rotated so that its pole is u,
// each lattice point is owned by the out-edge direction s_m with the largest dot
// product (ties: lowest index), and the owners' phase weights are summed in 2^-52
// fixed point with LDS integer atomics (exact, so the sum is independent of the
// order).  Surface nodes use the unrotated lattice with cosine weights (Lambertian).
//
// The incoming directions are processed in groups of G; the G x N_fib (direction,
// lattice point) pairs are spread over the lanes, up to eight per lane, so every
// out-edge direction read from LDS serves eight dot products per lane: the kernel is
// bound by FP64 issue, not by LDS broadcasts.  Each direction's column of the node
// block (column-major) is one coalesced store.
//
// The ownership decision is an argmax over double-precision dot products; it is
// written with this exact operation sequence (also followed by the FP64 CPU
// reference):
//   s_m  = D_m / sqrt(Dx^2 + Dy^2 + Dz^2)             (exact integer sum)
//   h    = 1 / (1 + u_z);  xy = (u_x u_y) h
//   R    = [[u_z + (u_y u_y) h, -xy, -u_x], [-xy, u_z + (u_x u_x) h, -u_y], [u_x, u_y, u_z]]
//          (R = diag(1, -1, -1) when 1 + u_z < 1e-12; the identity on the surface)
//   q_ik = fma(R_2k, p_i2, fma(R_1k, p_i1, R_0k p_i0))      (q_i = R^T p_i)
//   v_im = fma(q_i2, s_m2, fma(q_i1, s_m1, q_i0 s_m0))      (= p_i . R s_m)
// with no other contraction, hence the pragma below and -ffp-contract=off.
//
// The regular kernel finds that argmax through an FP32 screen with a proven error bound
// (FP64 compares and maxima issue at about half the rate of FP32 and 32-bit integer
// operations): every decision the screen cannot certify is taken by the FP64 sequence above,
// so each owner is the one the FP64 sequence gives (see screen_owners).
#include "device.hpp"
#include "internal.hpp"

#pragma clang fp contract(off)

namespace sg {

namespace {

constexpr double kFix = 4503599627370496.0;  // 2^52
constexpr double kUnfix = 1.0 / 4503599627370496.0;
constexpr int kQSlots = 8;     // (direction, lattice point) pairs per lane in a group
constexpr int kQMaxGroup = 8;  // incoming directions per group

// Dynamic LDS layout of a node in k_qbuild (in doubles), sized by the lattice and the group so
// that four workgroups fit per SIMD: sites [3][64]; in FP32 as float4 (16-byte aligned): the
// sites [64], the lattice [N_fib], the rotations' columns [group][3]; then lattice weights
// [N_fib] (fixed point), rotations [group][9] (FP64), bins [group][64] (fixed point)
__host__ __device__ constexpr int qbuild_lds_doubles(int NF, int group) { return 320 + 3 * NF + 79 * group; }

// p / n for 0 <= p < 1024 and 1 <= n <= 128 with one FP32 multiply: (p + 1/2) / n is at
// least 1/(2n) >= 2^-8 away from an integer, far above the rounding error of the
// product (below 2^-12 here, also with a reciprocal a few ulp off)
__device__ __forceinline__ int small_div(int p, float inv_n) { return (int)(((float)p + 0.5f) * inv_n); }

// q = R^T p for lattice point (x, y, z) (R row-major, 9 doubles)
__device__ __forceinline__ void rotate_point(const double *R, double x, double y, double z, double &q0, double &q1,
                                             double &q2) {
#pragma clang fp contract(off)
    q0 = fma(R[6], z, fma(R[3], y, R[0] * x));
    q1 = fma(R[7], z, fma(R[4], y, R[1] * x));
    q2 = fma(R[8], z, fma(R[5], y, R[2] * x));
}

// The FP32 screen.  For a slot with rotated point q and every out-edge m it forms
//   t_m = fma(q2', s_m2', fma(q1', s_m1', fma(q0', s_m0', c))),  c = 1 + 2^-10,
// where s' is s_m rounded to FP32 and q' = R'^T p' is the rotation done in FP32 (one multiply,
// two FMAs per component) from the FP32 roundings R' and p'; it replaces the low six bits of
// t_m's bit pattern by 63 - m (t_m is positive, so the patterns order like the values and the
// packed maximum names its index) and keeps the largest packed value P_b and the second
// largest P_2.  Error bound: with |p|, |s_m| and R's columns of norm <= 1 + 2^-49, every
// component of q' is within 5 * 2^-24 of q (two input roundings and three operation roundings,
// each at most 2^-24 times a magnitude <= 1), so q'.s' is within 5 sqrt(3) 2^-24 + 2^-23 <
// 2^-20.5 of q.s; the three FMAs (results in [2^-11, 2.01]) round by at most 2^-23 each; and the
// packing moves a value by less than 64 ulp <= 2^-17 P.  So every packed P_m lies within E_m =
// 2^-17 P_m + 2^-19 of c + q.s_m, while the FP64 sequence lies within 2^-51 of q.s_m.  If
// P_b - P_2 > 2^-16 P_b + 2^-17 (>= E_b + E_2 + 2^-50) then for every m != b the FP64 value of
// m is strictly below that of b: b is the FP64 argmax, with no tie.  Other slots (near-ties:
// a few pairs in 10,000 on jittered grids) rerun the FP64 sequence.
constexpr float kScreenOff = 1.0f + 0x1p-10f;

// one bitfield insert, (63 & k) | (~63 & t), under the inline constant 63 (written out: the
// compiler splits the plain expression into an AND with a literal and an OR)
__device__ __forceinline__ float screen_pack(float t, int k) {
    float r;
    asm("v_bfi_b32 %0, 63, %1, %2" : "=v"(r) : "s"(k), "v"(t));
    return r;
}

// Owners of the lane's first S slots of (direction, lattice point) pairs (S covers the
// group's pairs; slots past its last pair within them hold repeats and are scanned too).
template <int S>
__device__ __forceinline__ void screen_owners(int d, const float4 *s4, const double *sx, const double *sy,
                                              const double *sz, const double *Rg, const double *__restrict__ lat,
                                              int lane, int ng, int NF, float inv_nf, const float (&f0)[kQSlots],
                                              const float (&f1)[kQSlots], const float (&f2)[kQSlots], bool screen,
                                              int (&own)[kQSlots]) {
#pragma clang fp contract(off)
    float best[S], second[S];
#pragma unroll
    for (int j = 0; j < S; ++j) {
        best[j] = 0.0f;
        second[j] = 0.0f;
    }
    // two out-edges per step: the top two of (best, second, p, w) are max3(best, p, w) and
    // max(second, med3(best, p, w)) since second <= best
    int m = 0;
    for (; m + 1 < d; m += 2) {
        const float4 t = s4[m], u = s4[m + 1];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const float pv = screen_pack(fmaf(f2[j], t.z, fmaf(f1[j], t.y, fmaf(f0[j], t.x, kScreenOff))), 63 - m);
            const float pw = screen_pack(fmaf(f2[j], u.z, fmaf(f1[j], u.y, fmaf(f0[j], u.x, kScreenOff))), 62 - m);
            second[j] = fmaxf(second[j], __builtin_amdgcn_fmed3f(best[j], pv, pw));
            best[j] = fmaxf(fmaxf(best[j], pv), pw);
        }
    }
    if (m < d) {
        const float4 t = s4[m];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const float pv = screen_pack(fmaf(f2[j], t.z, fmaf(f1[j], t.y, fmaf(f0[j], t.x, kScreenOff))), 63 - m);
            second[j] = __builtin_amdgcn_fmed3f(best[j], second[j], pv);
            best[j] = fmaxf(best[j], pv);
        }
    }
    unsigned pending = 0;  // slots the screen does not certify
#pragma unroll
    for (int j = 0; j < S; ++j) {
        own[j] = 63 - (int)(__float_as_uint(best[j]) & 63u);
        if (!(screen && best[j] - second[j] > fmaf(best[j], 0x1p-16f, 0x1p-17f))) pending |= 1u << j;
    }
    // each lane decides its pending slots with the FP64 sequence (one slot per pass: lanes
    // with different pending slots share the passes); ties go to the lowest index, the index
    // moving only on a strict increase.  A slot past the group's last pair takes any valid
    // direction (its owner is not used).
    while (pending) {
        const int j = __builtin_ctz(pending);
        pending &= pending - 1;
        const int p = j * 64 + lane;
        const int al0 = small_div(p, inv_nf), i = p - al0 * NF, al = min(al0, ng - 1);
        double q0, q1, q2;
        rotate_point(Rg + 9 * al, lat[3 * i], lat[3 * i + 1], lat[3 * i + 2], q0, q1, q2);
        double bb = -__builtin_inf();
        int o = 0;
        for (int k = 0; k < d; ++k) {
            const double v = fma(q2, sz[k], fma(q1, sy[k], q0 * sx[k]));
            o = v > bb ? k : o;
            bb = fmax(bb, v);
        }
#pragma unroll
        for (int jj = 0; jj < S; ++jj) own[jj] = jj == j ? o : own[jj];
    }
}

// Five wavefronts per SIMD (96 VGPRs; its LDS allows about 4.75): the per-node setup
// spills a few values that each group reloads, which costs less than the fifth wavefront
// gains in hiding the loads and atomics around the screen
template <class Real, class BlkT, bool kWriteQ>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) void k_qbuild(
    int N, int nvol, const long long *__restrict__ adj_ptr, const int *__restrict__ adj_idx,
    const int *__restrict__ pos, const double *__restrict__ lat, const double *__restrict__ tab, int NF, int n_phase,
    const float *__restrict__ frac, double sun_x, double sun_y, double sun_z, Real mu0, const Real *__restrict__ T,
    const Real *__restrict__ rho, const Real *__restrict__ Tsun, const long long *__restrict__ nodeoff,
    BlkT *__restrict__ val, Real *__restrict__ S, float *__restrict__ qsun, int group, int per, long long wx,
    long long wy, int screen) {
#pragma clang fp contract(off)
    extern __shared__ double qb_lds[];
    double *sx = qb_lds, *sy = qb_lds + 64, *sz = qb_lds + 128;
    float4 *s4 = reinterpret_cast<float4 *>(qb_lds + 192);
    float4 *lt4 = reinterpret_cast<float4 *>(qb_lds + 320);
    float4 *Rc4 = reinterpret_cast<float4 *>(qb_lds + 320 + 2 * NF);
    unsigned long long *wq = reinterpret_cast<unsigned long long *>(qb_lds + 320 + 2 * NF + 6 * group);
    double *Rg = qb_lds + 320 + 3 * NF + 6 * group;
    unsigned long long *bins = reinterpret_cast<unsigned long long *>(Rg + 9 * group);

    const int l = blockIdx.x;
    const int lane = threadIdx.x;
    const long long off = adj_ptr[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    if (d == 0 || d > kWave) return;  // higher degree: k_qbuild_big
    const bool surf = l >= nvol;
    if (!SG_IN(nodeoff[l] + (long long)d * d - 1, nodeoff[N], 0x201)) return;

    if (lane < d) {
        const int j0 = adj_idx[off + lane];
        const int j = SG_IN(j0, N, 0x202) ? j0 : l;
        const long long Dx = min_image((long long)pos[3 * j] - pos[3 * l], wx, per & 1);
        const long long Dy = min_image((long long)pos[3 * j + 1] - pos[3 * l + 1], wy, per & 2);
        const long long Dz = (long long)pos[3 * j + 2] - pos[3 * l + 2];
        const double nrm = sqrt((double)(Dx * Dx + Dy * Dy + Dz * Dz));
        const double ex = (double)Dx / nrm, ey = (double)Dy / nrm, ez = (double)Dz / nrm;
        sx[lane] = ex;
        sy[lane] = ey;
        sz[lane] = ez;
        s4[lane] = make_float4((float)ex, (float)ey, (float)ez, 0.0f);
    }
    for (int i = lane; i < NF; i += 64)
        lt4[i] = make_float4((float)lat[3 * i], (float)lat[3 * i + 1], (float)lat[3 * i + 2], 0.0f);
    const float inv_nf = 1.0f / (float)NF, inv_d = 1.0f / (float)d;
    // the lane's slots: slot j holds pair p = 64 j + lane of a group, direction p / N_fib of
    // the group and lattice point p mod N_fib, kept as direction * 128 + point
    int sai[kQSlots];
#pragma unroll
    for (int j = 0; j < kQSlots; ++j) {
        const int p = j * 64 + lane;
        const int al = small_div(p, inv_nf);
        sai[j] = al * 128 + (p - al * NF);
    }
    // phase weights of the lattice points in fixed point
    for (int i = lane; i < NF; i += 64) {
        double w;
        if (surf) {
            w = tab[n_phase * NF + i];
        } else {
            w = 0.0;
            for (int k = 0; k < n_phase; ++k) {
                const double f = frac ? (double)frac[(long long)k * nvol + l] : 1.0;
                w = w + f * tab[k * NF + i];
            }
        }
        wq[i] = (unsigned long long)llrint(w * kFix);
    }

    const Real rl = rho ? rho[l] : (Real)0;
    const Real tsun = Tsun ? Tsun[l] : (Real)0;
    BlkT *blk = val + nodeoff[l];  // column-major: element (row n, column m) at m d + n
    const int n_in = surf ? 1 : d + 1;
    for (int a0 = 0; a0 < n_in; a0 += group) {
        const int ng = min(group, n_in - a0);
        // rotations of this group's incoming directions (FP64, and their columns in FP32), and
        // empty bins
        if (lane < ng) {
            const int a = a0 + lane;
            double *R = Rg + 9 * lane;
            if (surf) {
                R[0] = 1.0; R[1] = 0.0; R[2] = 0.0; R[3] = 0.0; R[4] = 1.0; R[5] = 0.0; R[6] = 0.0; R[7] = 0.0;
                R[8] = 1.0;
            } else {
                double ux, uy, uz;
                if (a < d) { ux = -sx[a]; uy = -sy[a]; uz = -sz[a]; }
                else { ux = sun_x; uy = sun_y; uz = sun_z; }
                if (1.0 + uz < 1e-12) {
                    R[0] = 1.0; R[1] = 0.0; R[2] = 0.0; R[3] = 0.0; R[4] = -1.0; R[5] = 0.0; R[6] = 0.0;
                    R[7] = 0.0; R[8] = -1.0;
                } else {
                    const double h = 1.0 / (1.0 + uz);
                    const double xy = (ux * uy) * h;
                    R[0] = uz + (uy * uy) * h; R[1] = -xy; R[2] = -ux;
                    R[3] = -xy; R[4] = uz + (ux * ux) * h; R[5] = -uy;
                    R[6] = ux; R[7] = uy; R[8] = uz;
                }
            }
#pragma unroll
            for (int k = 0; k < 3; ++k)
                Rc4[3 * lane + k] = make_float4((float)R[k], (float)R[3 + k], (float)R[6 + k], 0.0f);
        }
        for (int t = lane; t < ng * 64; t += 64) bins[t] = 0ull;
        __syncthreads();
        // this lane's pairs: q' = R'^T p' in FP32 for each (a slot past the group's last pair
        // takes the group's last direction: scanned, not counted), then the owners
        const int np = ng * NF;  // pairs of this group
        float f0[kQSlots], f1[kQSlots], f2[kQSlots];
        int own[kQSlots];
#pragma unroll
        for (int j = 0; j < kQSlots; ++j) {
            const int al = min(sai[j] >> 7, ng - 1);
            const float4 pt = lt4[sai[j] & 127], c0 = Rc4[3 * al], c1 = Rc4[3 * al + 1], c2 = Rc4[3 * al + 2];
            f0[j] = fmaf(c0.z, pt.z, fmaf(c0.y, pt.y, c0.x * pt.x));
            f1[j] = fmaf(c1.z, pt.z, fmaf(c1.y, pt.y, c1.x * pt.x));
            f2[j] = fmaf(c2.z, pt.z, fmaf(c2.y, pt.y, c2.x * pt.x));
            own[j] = 0;
        }
        // slots per lane that this group's pairs need (a node's last group is often short)
        const bool scr = screen != 0;
        if (np <= 2 * 64) screen_owners<2>(d, s4, sx, sy, sz, Rg, lat, lane, ng, NF, inv_nf, f0, f1, f2, scr, own);
        else if (np <= 4 * 64) screen_owners<4>(d, s4, sx, sy, sz, Rg, lat, lane, ng, NF, inv_nf, f0, f1, f2, scr, own);
        else if (np <= 6 * 64) screen_owners<6>(d, s4, sx, sy, sz, Rg, lat, lane, ng, NF, inv_nf, f0, f1, f2, scr, own);
        else screen_owners<kQSlots>(d, s4, sx, sy, sz, Rg, lat, lane, ng, NF, inv_nf, f0, f1, f2, scr, own);
#pragma unroll
        for (int j = 0; j < kQSlots; ++j) {
            const int al = sai[j] >> 7;  // below ng exactly for the group's pairs
            if (al < ng && SG_IN(al * 64 + own[j], group * 64, 0x203))
                atomicAdd(&bins[al * 64 + own[j]], wq[sai[j] & 127]);
        }
        __syncthreads();
        // this group's columns: pair t = (a - a0) d + m is column a, row m
        for (int t = lane; t < ng * d; t += 64) {
            const int al = small_div(t, inv_d), m = t - al * d, a = a0 + al;
            const double Q = (double)(long long)bins[al * 64 + m] * kUnfix;
            const long long b = off + m;
            if (surf) {
                for (int c = 0; c < d; ++c) {
                    if (kWriteQ) blk[c * d + m] = (BlkT)Q;
                    else blk[c * d + m] = (BlkT)(T[off + c] * rl * (Real)Q);
                }
                if (!kWriteQ) S[b] = rl * mu0 * tsun * (Real)Q;
                qsun[b] = (float)Q;
            } else if (a < d) {
                if (kWriteQ) blk[a * d + m] = (BlkT)Q;
                else blk[a * d + m] = (BlkT)(T[off + a] * rl * (Real)Q);
            } else {
                if (!kWriteQ) S[b] = tsun * rl * (Real)Q;
                qsun[b] = (float)Q;
            }
        }
        __syncthreads();
    }
}

// Nodes of degree above 64 (graphs whose strongest couplings gather on the dense nodes):
// one 64-lane workgroup per (node, group of `group` incoming directions), wg = bigdir[b] +
// g.  The (direction, lattice point) pairs fill the lanes' eight slots as in k_qbuild, and
// the node's out-edge directions are formed in LDS 64 at a time and scanned in ascending
// order with k_qbuild's operation sequence and tie rule, so each direction read from LDS
// serves eight dot products.  No FP32 screen here: with hundreds to thousands of out-edges
// the top two of a pair are within the screen's bound far more often (percents of the
// pairs), and deciding those again cost more than the screen saved.  A direction's lattice points have at most N_fib distinct
// owners among the d out-edges, so its cell sums go to a 256-slot open-addressing table in
// LDS (owner -> fixed-point sum, exact integer atomics) rather than d words; the column is
// then written by looking every row up (absent: 0).
constexpr int kCellHash = 256;  // above the most owners a direction can have (N_fib <= 128)
constexpr int kBigGroup = 5;    // directions per workgroup (the tables' LDS)

constexpr unsigned short kNoOwner = 0xffff;  // owners are below 4096

__device__ __forceinline__ int cell_find(const unsigned short *keys, int m) {
    int h = m & (kCellHash - 1);
    while (keys[h] != m && keys[h] != kNoOwner) h = (h + 1) & (kCellHash - 1);
    return keys[h] == m ? h : -1;
}

template <class Real, class BlkT, bool kWriteQ>
__global__ __launch_bounds__(64) void k_qbuild_big(
    int nbig, const int *__restrict__ big, const long long *__restrict__ bigdir, int nvol,
    const long long *__restrict__ adj_ptr, const int *__restrict__ adj_idx, const int *__restrict__ pos,
    const double *__restrict__ lat, const double *__restrict__ tab, int NF, int n_phase,
    const float *__restrict__ frac, double sun_x, double sun_y, double sun_z, Real mu0, const Real *__restrict__ T,
    const Real *__restrict__ rho, const Real *__restrict__ Tsun, const long long *__restrict__ nodeoff,
    BlkT *__restrict__ val, Real *__restrict__ S, float *__restrict__ qsun, int group, int per, long long wx,
    long long wy) {
#pragma clang fp contract(off)
    __shared__ double cx[64], cy[64], cz[64], Rg[kBigGroup * 9], lt[384];
    __shared__ unsigned long long wq[128], hval[kBigGroup][kCellHash];
    __shared__ unsigned short hkey[kBigGroup][kCellHash];
    const long long wg = blockIdx.x;
    int lo = 0, hi = nbig;  // the node b with bigdir[b] <= wg < bigdir[b + 1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (bigdir[mid] <= wg) lo = mid; else hi = mid;
    }
    const int l = big[lo];
    const int lane = threadIdx.x;
    const long long off = adj_ptr[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    const bool surf = l >= nvol;
    const int n_in = surf ? 1 : d + 1;
    const int a0 = (int)(wg - bigdir[lo]) * group;
    const int ng = min(group, n_in - a0);
    // the unit direction of out-edge m (the operation sequence of k_qbuild)
    auto edge_dir = [&](int m, double &ex, double &ey, double &ez) {
        const int j = adj_idx[off + m];
        const long long Dx = min_image((long long)pos[3 * j] - pos[3 * l], wx, per & 1);
        const long long Dy = min_image((long long)pos[3 * j + 1] - pos[3 * l + 1], wy, per & 2);
        const long long Dz = (long long)pos[3 * j + 2] - pos[3 * l + 2];
        const double nrm = sqrt((double)(Dx * Dx + Dy * Dy + Dz * Dz));
        ex = (double)Dx / nrm;
        ey = (double)Dy / nrm;
        ez = (double)Dz / nrm;
    };
    for (int i = lane; i < NF; i += 64) {
        lt[i] = lat[3 * i];
        lt[128 + i] = lat[3 * i + 1];
        lt[256 + i] = lat[3 * i + 2];
        double w;
        if (surf) {
            w = tab[n_phase * NF + i];
        } else {
            w = 0.0;
            for (int k = 0; k < n_phase; ++k) {
                const double f = frac ? (double)frac[(long long)k * nvol + l] : 1.0;
                w = w + f * tab[k * NF + i];
            }
        }
        wq[i] = (unsigned long long)llrint(w * kFix);
    }
    for (int t = lane; t < ng * kCellHash; t += 64) {
        hkey[t / kCellHash][t % kCellHash] = kNoOwner;
        hval[t / kCellHash][t % kCellHash] = 0ull;
    }
    // rotations of this group's incoming directions
    if (lane < ng) {
        const int a = a0 + lane;
        double *R = Rg + 9 * lane;
        if (surf) {
            R[0] = 1.0; R[1] = 0.0; R[2] = 0.0; R[3] = 0.0; R[4] = 1.0; R[5] = 0.0; R[6] = 0.0; R[7] = 0.0; R[8] = 1.0;
        } else {
            double ux, uy, uz;
            if (a < d) {
                edge_dir(a, ux, uy, uz);
                ux = -ux; uy = -uy; uz = -uz;
            } else {
                ux = sun_x; uy = sun_y; uz = sun_z;
            }
            if (1.0 + uz < 1e-12) {
                R[0] = 1.0; R[1] = 0.0; R[2] = 0.0; R[3] = 0.0; R[4] = -1.0; R[5] = 0.0; R[6] = 0.0; R[7] = 0.0;
                R[8] = -1.0;
            } else {
                const double h = 1.0 / (1.0 + uz);
                const double xy = (ux * uy) * h;
                R[0] = uz + (uy * uy) * h; R[1] = -xy; R[2] = -ux;
                R[3] = -xy; R[4] = uz + (ux * ux) * h; R[5] = -uy;
                R[6] = ux; R[7] = uy; R[8] = uz;
            }
        }
    }
    __syncthreads();
    // this lane's pairs: q = R^T p
    const int np = ng * NF;
    const float inv_nf = 1.0f / (float)NF;
    double q0[kQSlots], q1[kQSlots], q2[kQSlots], best[kQSlots];
    int own[kQSlots];
#pragma unroll
    for (int j = 0; j < kQSlots; ++j) {
        const int p = min(j * 64 + lane, np - 1);  // past the last pair: a repeat, not counted
        const int al = small_div(p, inv_nf), i = p - al * NF;
        const double *R = Rg + 9 * al;
        const double x = lt[i], y = lt[128 + i], z = lt[256 + i];
        q0[j] = fma(R[6], z, fma(R[3], y, R[0] * x));
        q1[j] = fma(R[7], z, fma(R[4], y, R[1] * x));
        q2[j] = fma(R[8], z, fma(R[5], y, R[2] * x));
        best[j] = -__builtin_inf();
        own[j] = 0;
    }
    for (int m0 = 0; m0 < d; m0 += 64) {
        const int nm = min(64, d - m0);
        if (lane < nm) edge_dir(m0 + lane, cx[lane], cy[lane], cz[lane]);
        __syncthreads();
        for (int mm = 0; mm < nm; ++mm) {
            const double tx = cx[mm], ty = cy[mm], tz = cz[mm];
#pragma unroll
            for (int j = 0; j < kQSlots; ++j) {
                const double v = fma(q2[j], tz, fma(q1[j], ty, q0[j] * tx));
                own[j] = v > best[j] ? m0 + mm : own[j];
                best[j] = fmax(best[j], v);
            }
        }
        __syncthreads();  // the next chunk rewrites the directions
    }
    // cell sums: owner -> fixed-point sum in the direction's table
#pragma unroll
    for (int j = 0; j < kQSlots; ++j) {
        const int p = j * 64 + lane;
        if (p < np) {
            const int al = small_div(p, inv_nf);
            unsigned short *keys = hkey[al];
            const unsigned short key = (unsigned short)own[j];
            int h = own[j] & (kCellHash - 1);
            while (true) {
                const unsigned short old = atomicCAS(&keys[h], kNoOwner, key);
                if (old == kNoOwner || old == key) break;
                h = (h + 1) & (kCellHash - 1);
            }
            atomicAdd(&hval[al][h], wq[p - al * NF]);
        }
    }
    __syncthreads();
    const Real rl = rho ? rho[l] : (Real)0;
    const Real tsun = Tsun ? Tsun[l] : (Real)0;
    BlkT *blk = val + nodeoff[l];  // column-major: element (row n, column m) at m d + n
    for (int al = 0; al < ng; ++al) {
        const int a = a0 + al;
        for (int m = lane; m < d; m += 64) {
            const int h = cell_find(hkey[al], m);
            const double Q = h < 0 ? 0.0 : (double)(long long)hval[al][h] * kUnfix;
            const long long b = off + m;
            if (surf) {
                for (int c = 0; c < d; ++c) {
                    if (kWriteQ) blk[(long long)c * d + m] = (BlkT)Q;
                    else blk[(long long)c * d + m] = (BlkT)(T[off + c] * rl * (Real)Q);
                }
                if (!kWriteQ) S[b] = rl * mu0 * tsun * (Real)Q;
                qsun[b] = (float)Q;
            } else if (a < d) {
                if (kWriteQ) blk[(long long)a * d + m] = (BlkT)Q;
                else blk[(long long)a * d + m] = (BlkT)(T[off + a] * rl * (Real)Q);
            } else {
                if (!kWriteQ) S[b] = tsun * rl * (Real)Q;
                qsun[b] = (float)Q;
            }
        }
    }
}


// The paper's discretisation of Sigma (Sec. 3), for scenes that ask for it: per
// incoming direction, every out-edge direction colours its closest lattice point and
// the colours spread over the lattice by flood fill along the edges of its convex
// hull.  One 64-lane wavefront per node, lattice points i and i + 64 in lane i.
//   seeds: for m = 0, 1, ...: the lattice point of largest v_im (the Voronoi
//   ownership's dot products, same operation sequence; ties to the lowest i) takes
//   colour m unless it was claimed with a value >= v_im by an earlier direction;
//   fill: in rounds, every uncoloured point takes the colour its lowest-index
//   coloured neighbour had at the start of the round, until all are coloured (the
//   hull graph is connected and there is at least one seed).
// Q(u -> m) is the fixed-point sum of the phase weights of colour m, as in k_qbuild.
// order-preserving 64-bit keys of doubles (for integer atomic max in LDS)
__device__ __forceinline__ unsigned long long order_key(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double order_value(unsigned long long k) {
    const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

template <class Real, class BlkT, bool kWriteQ>
__global__ __launch_bounds__(64) void k_qcolour(
    int N, int nvol, const long long *__restrict__ adj_ptr, const int *__restrict__ adj_idx,
    const int *__restrict__ pos, const double *__restrict__ lat, const double *__restrict__ tab, int NF, int n_phase,
    const float *__restrict__ frac, double sun_x, double sun_y, double sun_z, Real mu0, const Real *__restrict__ T,
    const Real *__restrict__ rho, const Real *__restrict__ Tsun, const long long *__restrict__ nodeoff,
    BlkT *__restrict__ val, Real *__restrict__ S, float *__restrict__ qsun, const int *__restrict__ hull, int per,
    long long wx, long long wy) {
#pragma clang fp contract(off)
    __shared__ double sx[64], sy[64], sz[64], lq[3][128];  // sites; this direction's rotated lattice
    __shared__ unsigned long long wq[128], bins[64], bkey[128], mkey[64];
    __shared__ int col[128], snap[128], mi[64];

    const int l = blockIdx.x;
    const int lane = threadIdx.x;
    const long long off = adj_ptr[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    if (d == 0 || d > kWave) return;  // higher degree: k_qcolour_big
    const bool surf = l >= nvol;
    if (!SG_IN(nodeoff[l] + (long long)d * d - 1, nodeoff[N], 0x204)) return;
    if (lane < d) {
        const int j0 = adj_idx[off + lane];
        const int j = SG_IN(j0, N, 0x205) ? j0 : l;
        const long long Dx = min_image((long long)pos[3 * j] - pos[3 * l], wx, per & 1);
        const long long Dy = min_image((long long)pos[3 * j + 1] - pos[3 * l + 1], wy, per & 2);
        const long long Dz = (long long)pos[3 * j + 2] - pos[3 * l + 2];
        const double nrm = sqrt((double)(Dx * Dx + Dy * Dy + Dz * Dz));
        sx[lane] = (double)Dx / nrm;
        sy[lane] = (double)Dy / nrm;
        sz[lane] = (double)Dz / nrm;
    }
    for (int i = lane; i < NF; i += 64) {
        double w;
        if (surf) {
            w = tab[n_phase * NF + i];
        } else {
            w = 0.0;
            for (int k = 0; k < n_phase; ++k) {
                const double f = frac ? (double)frac[(long long)k * nvol + l] : 1.0;
                w = w + f * tab[k * NF + i];
            }
        }
        wq[i] = (unsigned long long)llrint(w * kFix);
    }
    __syncthreads();

    const Real rl = rho ? rho[l] : (Real)0;
    const Real tsun = Tsun ? Tsun[l] : (Real)0;
    BlkT *blk = val + nodeoff[l];  // column-major: element (row n, column m) at m d + n
    const int n_in = surf ? 1 : d + 1;
    const int i0 = lane, i1 = lane + 64;
    const bool ok0 = i0 < NF, ok1 = i1 < NF;
    const int P = min(4, kWave / d);             // lanes per out-direction in the seed scan
    const int blk_pts = (NF + P - 1) / P;        // lattice points per lane
    double px[2], py[2], pz[2];  // this lane's lattice points i0, i1
    int nn[2];                    // and their hull neighbours, four indices (< 128) a word
    unsigned nbw[2][kHullNb / 4];
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
        const int i = min(h2 ? i1 : i0, NF - 1);
        px[h2] = lat[3 * i];
        py[h2] = lat[3 * i + 1];
        pz[h2] = lat[3 * i + 2];
        nn[h2] = hull[NF * kHullNb + i];
#pragma unroll
        for (int w = 0; w < kHullNb / 4; ++w) {
            unsigned v = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) v |= ((unsigned)hull[i * kHullNb + 4 * w + b] & 0xffu) << (8 * b);
            nbw[h2][w] = v;
        }
    }
    for (int a = 0; a < n_in; ++a) {
        // rotation of this incoming direction (every lane, the same values)
        double R[9];
        if (surf) {
            R[0] = 1.0; R[1] = 0.0; R[2] = 0.0; R[3] = 0.0; R[4] = 1.0; R[5] = 0.0; R[6] = 0.0; R[7] = 0.0; R[8] = 1.0;
        } else {
            double ux, uy, uz;
            if (a < d) { ux = -sx[a]; uy = -sy[a]; uz = -sz[a]; }
            else { ux = sun_x; uy = sun_y; uz = sun_z; }
            if (1.0 + uz < 1e-12) {
                R[0] = 1.0; R[1] = 0.0; R[2] = 0.0; R[3] = 0.0; R[4] = -1.0; R[5] = 0.0; R[6] = 0.0; R[7] = 0.0;
                R[8] = -1.0;
            } else {
                const double h = 1.0 / (1.0 + uz);
                const double xy = (ux * uy) * h;
                R[0] = uz + (uy * uy) * h; R[1] = -xy; R[2] = -ux;
                R[3] = -xy; R[4] = uz + (ux * ux) * h; R[5] = -uy;
                R[6] = ux; R[7] = uy; R[8] = uz;
            }
        }
        // the rotated lattice (q_i = R^T p_i), and cleared claims
        for (int h2 = 0; h2 < 2; ++h2) {
            const int i = h2 ? i1 : i0;
            if (i >= NF) continue;
            const double x = px[h2], y = py[h2], z = pz[h2];
            lq[0][i] = fma(R[6], z, fma(R[3], y, R[0] * x));
            lq[1][i] = fma(R[7], z, fma(R[4], y, R[1] * x));
            lq[2][i] = fma(R[8], z, fma(R[5], y, R[2] * x));
            bkey[i] = 0ull;
            col[i] = 0x7fffffff;
        }
        if (lane < d) {
            mkey[lane] = 0ull;
            mi[lane] = 0x7fffffff;
        }
        __syncthreads();
        // seeds: lane m scans the lattice points in ascending order (strict >) for the
        // largest v_im, and raises that point's best value; then every m whose seed value
        // equals its point's best offers its index: a point seeded by several directions
        // goes to the largest value, ties to the lowest m (claiming in order of m)
        // (with P = 64 / d > 1 lanes per direction, lane m + part d scans the part-th block
        // of points and the blocks combine by value, ties to the lower point)
        double bv = 0.0;
        int bi = 0;
        const int part = lane / d;
        const bool scans = part < P && part * blk_pts < NF;  // a block can be empty for tiny N_fib
        if (scans) {
            const int m = lane - part * d;
            const int ib = part * blk_pts, ie = min(NF, ib + blk_pts);
            const double tx = sx[m], ty = sy[m], tz = sz[m];
            bv = fma(lq[2][ib], tz, fma(lq[1][ib], ty, lq[0][ib] * tx));
            bi = ib;
#pragma unroll 4
            for (int i = ib + 1; i < ie; ++i) {
                const double v = fma(lq[2][i], tz, fma(lq[1][i], ty, lq[0][i] * tx));
                bi = v > bv ? i : bi;
                bv = fmax(bv, v);
            }
            if (P > 1) atomicMax(&mkey[m], order_key(bv));
        }
        if (P > 1) {
            __syncthreads();
            if (scans && bv == order_value(mkey[lane - part * d])) atomicMin(&mi[lane - part * d], bi);
            __syncthreads();
            if (lane < d) {
                bi = mi[lane];
                bv = order_value(mkey[lane]);
            }
        }
        if (lane < d) atomicMax(&bkey[bi], order_key(bv));
        __syncthreads();
        if (lane < d && bv == order_value(bkey[bi])) atomicMin(&col[bi], lane);
        __syncthreads();
        if (ok0 && col[i0] == 0x7fffffff) col[i0] = -1;  // each lane its own points
        if (ok1 && col[i1] == 0x7fffffff) col[i1] = -1;
        // flood fill in rounds: an uncoloured point takes the colour of its lowest-index
        // coloured neighbour (the lists ascend) in the snapshot of the round's start; the
        // list's reads are independent, so they are issued together
        for (int round = 0; round < NF; ++round) {
            if (ok0) snap[i0] = col[i0];
            if (ok1) snap[i1] = col[i1];
            __syncthreads();
            bool missing = false;
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {
                const int i = h2 ? i1 : i0;
                if (i >= NF || snap[i] >= 0) continue;
                int c = -1;
#pragma unroll
                for (int t = kHullNb - 1; t >= 0; --t) {
                    if (t < nn[h2]) {
                        const int ct = snap[(nbw[h2][t >> 2] >> (8 * (t & 3))) & 0xffu];
                        c = ct >= 0 ? ct : c;
                    }
                }
                col[i] = c;
                missing = missing || c < 0;
            }
            const bool any = __ballot(missing) != 0ull;
            __syncthreads();
            if (!any) break;
        }
        // cells: fixed-point sums per colour, then this direction's column
        if (lane < d) bins[lane] = 0ull;
        __syncthreads();
        if (ok0 && col[i0] >= 0 && SG_IN(col[i0], d, 0x206)) atomicAdd(&bins[col[i0]], wq[i0]);
        if (ok1 && col[i1] >= 0 && SG_IN(col[i1], d, 0x207)) atomicAdd(&bins[col[i1]], wq[i1]);
        __syncthreads();
        if (lane < d) {
            const int m = lane;
            const double Q = (double)(long long)bins[m] * kUnfix;
            const long long b = off + m;
            if (surf) {
                for (int c = 0; c < d; ++c) {
                    if (kWriteQ) blk[c * d + m] = (BlkT)Q;
                    else blk[c * d + m] = (BlkT)(T[off + c] * rl * (Real)Q);
                }
                if (!kWriteQ) S[b] = rl * mu0 * tsun * (Real)Q;
                qsun[b] = (float)Q;
            } else if (a < d) {
                if (kWriteQ) blk[a * d + m] = (BlkT)Q;
                else blk[a * d + m] = (BlkT)(T[off + a] * rl * (Real)Q);
            } else {
                if (!kWriteQ) S[b] = tsun * rl * (Real)Q;
                qsun[b] = (float)Q;
            }
        }
        __syncthreads();
    }
}

// The colouring for nodes of degree above 64: one 64-lane workgroup per (node, incoming
// direction), lattice points i and i + 64 in lane i, their rotated coordinates in LDS.
//   seeds: lanes run over the out-directions m; each scans the lattice points in
//   ascending order (strict >) for its seed and raises the point's best value (an
//   order-preserving 64-bit key, atomic max); then every m whose seed value equals its
//   point's best offers its index (atomic min): a point claimed several times goes to
//   the largest value, ties to the lowest m, as claiming in order of m gives.
//   fill and cells as in k_qcolour, the colours' sums in a hash table (at most N_fib
//   colours among the d out-edges), the column written by looking up every row.

// unit vector of node l's out-edge m (the shortest periodic image)
__device__ __forceinline__ void edge_unit(const long long *__restrict__ adj_ptr, const int *__restrict__ adj_idx,
                                          const int *__restrict__ pos, int l, int m, int per, long long wx,
                                          long long wy, double &ex, double &ey, double &ez) {
    const int j = adj_idx[adj_ptr[l] + m];
    const long long Dx = min_image((long long)pos[3 * j] - pos[3 * l], wx, per & 1);
    const long long Dy = min_image((long long)pos[3 * j + 1] - pos[3 * l + 1], wy, per & 2);
    const long long Dz = (long long)pos[3 * j + 2] - pos[3 * l + 2];
    const double nrm = sqrt((double)(Dx * Dx + Dy * Dy + Dz * Dz));
    ex = (double)Dx / nrm;
    ey = (double)Dy / nrm;
    ez = (double)Dz / nrm;
}

// seeds of S out-directions per lane (m0 + 64 s + lane, s < S): each scans the lattice
// points in ascending order (strict >), so every point read from LDS serves S dot products;
// then the point's best value is raised (order-preserving key, atomic max)
template <int S>
__device__ __forceinline__ void colour_seeds(int m0, int d, int NF, const double (*lq)[128],
                                             const long long *__restrict__ adj_ptr,
                                             const int *__restrict__ adj_idx, const int *__restrict__ pos, int l,
                                             int per, long long wx, long long wy, unsigned char *seed_pt,
                                             unsigned long long *bkey) {
#pragma clang fp contract(off)
    double tx[S], ty[S], tz[S], bv[S];
    int bi[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int m = min(m0 + 64 * s + (int)threadIdx.x, d - 1);
        edge_unit(adj_ptr, adj_idx, pos, l, m, per, wx, wy, tx[s], ty[s], tz[s]);
        bv[s] = fma(lq[2][0], tz[s], fma(lq[1][0], ty[s], lq[0][0] * tx[s]));
        bi[s] = 0;
    }
    for (int i = 1; i < NF; ++i) {
        const double x = lq[0][i], y = lq[1][i], z = lq[2][i];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const double v = fma(z, tz[s], fma(y, ty[s], x * tx[s]));
            bi[s] = v > bv[s] ? i : bi[s];  // moves only on a strict increase
            bv[s] = fmax(bv[s], v);
        }
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int m = m0 + 64 * s + (int)threadIdx.x;
        if (m < d) {
            seed_pt[m] = (unsigned char)bi[s];
            atomicMax(&bkey[bi[s]], order_key(bv[s]));
        }
    }
}

template <class Real, class BlkT, bool kWriteQ>
__global__ __launch_bounds__(64) void k_qcolour_big(
    int nbig, const int *__restrict__ big, const long long *__restrict__ bigdir, int nvol,
    const long long *__restrict__ adj_ptr, const int *__restrict__ adj_idx, const int *__restrict__ pos,
    const double *__restrict__ lat, const double *__restrict__ tab, int NF, int n_phase,
    const float *__restrict__ frac, double sun_x, double sun_y, double sun_z, Real mu0, const Real *__restrict__ T,
    const Real *__restrict__ rho, const Real *__restrict__ Tsun, const long long *__restrict__ nodeoff,
    BlkT *__restrict__ val, Real *__restrict__ S, float *__restrict__ qsun, const int *__restrict__ hull, int per,
    long long wx, long long wy) {
#pragma clang fp contract(off)
    __shared__ double lq[3][128];  // the rotated lattice; after the claims, the cells' hash table
    __shared__ unsigned long long bkey[128], wq[128];
    __shared__ int col[128], snap[128];
    __shared__ unsigned char seed_pt[kMaxDegree];
    static_assert(kCellHash * (sizeof(unsigned long long) + sizeof(unsigned short)) <= sizeof(lq), "hash in lq");
    unsigned long long *hval = reinterpret_cast<unsigned long long *>(&lq[0][0]);
    unsigned short *hkey = reinterpret_cast<unsigned short *>(hval + kCellHash);
    const long long wg = blockIdx.x;
    int lo = 0, hi = nbig;  // the node b with bigdir[b] <= wg < bigdir[b + 1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (bigdir[mid] <= wg) lo = mid; else hi = mid;
    }
    const int l = big[lo];
    const int a = (int)(wg - bigdir[lo]);
    const int lane = threadIdx.x;
    const long long off = adj_ptr[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    const bool surf = l >= nvol;
    auto edge_dir = [&](int m, double &ex, double &ey, double &ez) {
        const int j = adj_idx[off + m];
        const long long Dx = min_image((long long)pos[3 * j] - pos[3 * l], wx, per & 1);
        const long long Dy = min_image((long long)pos[3 * j + 1] - pos[3 * l + 1], wy, per & 2);
        const long long Dz = (long long)pos[3 * j + 2] - pos[3 * l + 2];
        const double nrm = sqrt((double)(Dx * Dx + Dy * Dy + Dz * Dz));
        ex = (double)Dx / nrm;
        ey = (double)Dy / nrm;
        ez = (double)Dz / nrm;
    };
    double R[9];
    if (surf) {
        R[0] = 1.0; R[1] = 0.0; R[2] = 0.0; R[3] = 0.0; R[4] = 1.0; R[5] = 0.0; R[6] = 0.0; R[7] = 0.0; R[8] = 1.0;
    } else {
        double ux, uy, uz;
        if (a < d) {
            edge_dir(a, ux, uy, uz);
            ux = -ux; uy = -uy; uz = -uz;
        } else {
            ux = sun_x; uy = sun_y; uz = sun_z;
        }
        if (1.0 + uz < 1e-12) {
            R[0] = 1.0; R[1] = 0.0; R[2] = 0.0; R[3] = 0.0; R[4] = -1.0; R[5] = 0.0; R[6] = 0.0; R[7] = 0.0;
            R[8] = -1.0;
        } else {
            const double h = 1.0 / (1.0 + uz);
            const double xy = (ux * uy) * h;
            R[0] = uz + (uy * uy) * h; R[1] = -xy; R[2] = -ux;
            R[3] = -xy; R[4] = uz + (ux * ux) * h; R[5] = -uy;
            R[6] = ux; R[7] = uy; R[8] = uz;
        }
    }
    for (int i = lane; i < NF; i += 64) {
        const double x = lat[3 * i], y = lat[3 * i + 1], z = lat[3 * i + 2];
        lq[0][i] = fma(R[6], z, fma(R[3], y, R[0] * x));
        lq[1][i] = fma(R[7], z, fma(R[4], y, R[1] * x));
        lq[2][i] = fma(R[8], z, fma(R[5], y, R[2] * x));
        double w;
        if (surf) {
            w = tab[n_phase * NF + i];
        } else {
            w = 0.0;
            for (int k = 0; k < n_phase; ++k) {
                const double f = frac ? (double)frac[(long long)k * nvol + l] : 1.0;
                w = w + f * tab[k * NF + i];
            }
        }
        wq[i] = (unsigned long long)llrint(w * kFix);
        bkey[i] = 0ull;
        col[i] = 0x7fffffff;
    }
    int nn[2];  // this lane's lattice points' hull neighbours, four indices (< 128) a word
    unsigned nbw[2][kHullNb / 4];
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
        const int i = min(h2 ? lane + 64 : lane, NF - 1);
        nn[h2] = hull[NF * kHullNb + i];
#pragma unroll
        for (int w = 0; w < kHullNb / 4; ++w) {
            unsigned v = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) v |= ((unsigned)hull[i * kHullNb + 4 * w + b] & 0xffu) << (8 * b);
            nbw[h2][w] = v;
        }
    }
    __syncthreads();
    // seeds: each out-direction's closest lattice point, and the points' best values
    for (int m0 = 0; m0 < d; m0 += 4 * 64) {
        const int left = d - m0;
        if (left > 3 * 64) colour_seeds<4>(m0, d, NF, lq, adj_ptr, adj_idx, pos, l, per, wx, wy, seed_pt, bkey);
        else if (left > 2 * 64) colour_seeds<3>(m0, d, NF, lq, adj_ptr, adj_idx, pos, l, per, wx, wy, seed_pt, bkey);
        else if (left > 64) colour_seeds<2>(m0, d, NF, lq, adj_ptr, adj_idx, pos, l, per, wx, wy, seed_pt, bkey);
        else colour_seeds<1>(m0, d, NF, lq, adj_ptr, adj_idx, pos, l, per, wx, wy, seed_pt, bkey);
    }
    __syncthreads();
    for (int m = lane; m < d; m += 64) {
        double tx, ty, tz;
        edge_dir(m, tx, ty, tz);
        const int bi = seed_pt[m];
        const double v = fma(lq[2][bi], tz, fma(lq[1][bi], ty, lq[0][bi] * tx));
        if (v == order_value(bkey[bi])) atomicMin(&col[bi], m);
    }
    __syncthreads();
    for (int t = lane; t < kCellHash; t += 64) {  // lq is free now (the fill's barriers publish this)
        hkey[t] = kNoOwner;
        hval[t] = 0ull;
    }
    const int i0 = lane, i1 = lane + 64;
    const bool ok0 = i0 < NF, ok1 = i1 < NF;
    if (ok0 && col[i0] == 0x7fffffff) col[i0] = -1;  // each lane its own points
    if (ok1 && col[i1] == 0x7fffffff) col[i1] = -1;
    for (int round = 0; round < NF; ++round) {
        if (ok0) snap[i0] = col[i0];
        if (ok1) snap[i1] = col[i1];
        __syncthreads();
        bool missing = false;
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) {
            const int i = h2 ? i1 : i0;
            if (i >= NF || snap[i] >= 0) continue;
            int c = -1;
#pragma unroll
            for (int t = kHullNb - 1; t >= 0; --t) {
                if (t < nn[h2]) {
                    const int ct = snap[(nbw[h2][t >> 2] >> (8 * (t & 3))) & 0xffu];
                    c = ct >= 0 ? ct : c;
                }
            }
            col[i] = c;
            missing = missing || c < 0;
        }
        const bool any = __ballot(missing) != 0ull;
        __syncthreads();
        if (!any) break;
    }
    // cells: colour -> fixed-point sum
    for (int h2 = 0; h2 < 2; ++h2) {
        const int i = h2 ? i1 : i0;
        if (i >= NF || col[i] < 0) continue;
        const unsigned short key = (unsigned short)col[i];
        int h = col[i] & (kCellHash - 1);
        while (true) {
            const unsigned short old = atomicCAS(&hkey[h], kNoOwner, key);
            if (old == kNoOwner || old == key) break;
            h = (h + 1) & (kCellHash - 1);
        }
        atomicAdd(&hval[h], wq[i]);
    }
    __syncthreads();
    const Real rl = rho ? rho[l] : (Real)0;
    const Real tsun = Tsun ? Tsun[l] : (Real)0;
    BlkT *blk = val + nodeoff[l];  // column-major: element (row n, column m) at m d + n
    for (int m = lane; m < d; m += 64) {
        const int h = cell_find(hkey, m);
        const double Q = h < 0 ? 0.0 : (double)(long long)hval[h] * kUnfix;
        const long long b = off + m;
        if (surf) {
            for (int c = 0; c < d; ++c) {
                if (kWriteQ) blk[(long long)c * d + m] = (BlkT)Q;
                else blk[(long long)c * d + m] = (BlkT)(T[off + c] * rl * (Real)Q);
            }
            if (!kWriteQ) S[b] = rl * mu0 * tsun * (Real)Q;
            qsun[b] = (float)Q;
        } else if (a < d) {
            if (kWriteQ) blk[(long long)a * d + m] = (BlkT)Q;
            else blk[(long long)a * d + m] = (BlkT)(T[off + a] * rl * (Real)Q);
        } else {
            if (!kWriteQ) S[b] = tsun * rl * (Real)Q;
            qsun[b] = (float)Q;
        }
    }
}


}  // namespace

// directions per group: as many as fill the lanes' pair slots
int qbuild_group(int NF) { return std::max(1, std::min(kQMaxGroup, kQSlots * 64 / NF)); }
int qbuild_group_big(int NF) { return std::min(qbuild_group(NF), kBigGroup); }

template <class Real>
void launch_qbuild(Scene &s, hipStream_t st, int write_q) {
    const size_t shm = 0;
    const int group = qbuild_group(s.n_fib);
    const size_t qshm = sizeof(double) * (size_t)qbuild_lds_doubles(s.n_fib, group);
    if (s.sigma_mode == SG_SIGMA_COLOUR) {
        if (write_q) {
            hipLaunchKernelGGL((k_qcolour<Real, float, true>), dim3(s.N), dim3(64), shm, st, s.N, s.n_vol, s.adj_ptr,
                               s.adj_idx, s.pos, s.lat, s.tab, s.n_fib, s.n_phase, node_frac(s), s.sun_in[0], s.sun_in[1],
                               s.sun_in[2], (Real)s.mu0, (const Real *)nullptr, (const Real *)nullptr,
                               (const Real *)nullptr, s.nodeoff, s.q, (Real *)nullptr, s.qsun, s.hull, s.periodic,
                               (long long)s.nx * kFx, (long long)s.ny * kFx);
        } else {
            hipLaunchKernelGGL((k_qcolour<Real, Real, false>), dim3(s.N), dim3(64), shm, st, s.N, s.n_vol, s.adj_ptr,
                               s.adj_idx, s.pos, s.lat, s.tab, s.n_fib, s.n_phase, node_frac(s), s.sun_in[0], s.sun_in[1],
                               s.sun_in[2], (Real)s.mu0, (const Real *)s.T, (const Real *)s.rho,
                               (const Real *)s.Tsun, s.nodeoff, (Real *)s.val, (Real *)s.S, s.qsun, s.hull, s.periodic,
                               (long long)s.nx * kFx, (long long)s.ny * kFx);
        }
        if (s.n_big) {  // nodes of degree above 64: one workgroup per (node, incoming direction)
            if (write_q)
                hipLaunchKernelGGL((k_qcolour_big<Real, float, true>), dim3(s.n_bigdir), dim3(64), 0, st, s.n_big,
                                   s.big, s.bigdir, s.n_vol, s.adj_ptr, s.adj_idx, s.pos, s.lat, s.tab, s.n_fib,
                                   s.n_phase, node_frac(s), s.sun_in[0], s.sun_in[1], s.sun_in[2], (Real)s.mu0,
                                   (const Real *)nullptr, (const Real *)nullptr, (const Real *)nullptr, s.nodeoff, s.q,
                                   (Real *)nullptr, s.qsun, s.hull, s.periodic, (long long)s.nx * kFx,
                                   (long long)s.ny * kFx);
            else
                hipLaunchKernelGGL((k_qcolour_big<Real, Real, false>), dim3(s.n_bigdir), dim3(64), 0, st, s.n_big,
                                   s.big, s.bigdir, s.n_vol, s.adj_ptr, s.adj_idx, s.pos, s.lat, s.tab, s.n_fib,
                                   s.n_phase, node_frac(s), s.sun_in[0], s.sun_in[1], s.sun_in[2], (Real)s.mu0,
                                   (const Real *)s.T, (const Real *)s.rho, (const Real *)s.Tsun, s.nodeoff,
                                   (Real *)s.val, (Real *)s.S, s.qsun, s.hull, s.periodic, (long long)s.nx * kFx,
                                   (long long)s.ny * kFx);
        }
        return;
    }
    if (s.n_big) {  // nodes of degree above 64
        if (write_q)
            hipLaunchKernelGGL((k_qbuild_big<Real, float, true>), dim3(s.n_bigdir), dim3(64), 0, st, s.n_big, s.big,
                               s.bigdir, s.n_vol, s.adj_ptr, s.adj_idx, s.pos, s.lat, s.tab, s.n_fib, s.n_phase, node_frac(s),
                               s.sun_in[0], s.sun_in[1], s.sun_in[2], (Real)s.mu0, (const Real *)nullptr,
                               (const Real *)nullptr, (const Real *)nullptr, s.nodeoff, s.q, (Real *)nullptr, s.qsun,
                               qbuild_group_big(s.n_fib), s.periodic, (long long)s.nx * kFx,
                               (long long)s.ny * kFx);
        else
            hipLaunchKernelGGL((k_qbuild_big<Real, Real, false>), dim3(s.n_bigdir), dim3(64), 0, st, s.n_big, s.big,
                               s.bigdir, s.n_vol, s.adj_ptr, s.adj_idx, s.pos, s.lat, s.tab, s.n_fib, s.n_phase, node_frac(s),
                               s.sun_in[0], s.sun_in[1], s.sun_in[2], (Real)s.mu0, (const Real *)s.T,
                               (const Real *)s.rho, (const Real *)s.Tsun, s.nodeoff, (Real *)s.val, (Real *)s.S, s.qsun,
                               qbuild_group_big(s.n_fib), s.periodic, (long long)s.nx * kFx,
                               (long long)s.ny * kFx);
    }
    if (write_q) {
        hipLaunchKernelGGL((k_qbuild<Real, float, true>), dim3(s.N), dim3(64), qshm, st, s.N, s.n_vol, s.adj_ptr,
                           s.adj_idx, s.pos, s.lat, s.tab, s.n_fib, s.n_phase, node_frac(s), s.sun_in[0], s.sun_in[1],
                           s.sun_in[2], (Real)s.mu0, (const Real *)nullptr, (const Real *)nullptr,
                           (const Real *)nullptr, s.nodeoff, s.q, (Real *)nullptr, s.qsun, group, s.periodic, (long long)s.nx * kFx,
                           (long long)s.ny * kFx, s.qscreen);
    } else {
        hipLaunchKernelGGL((k_qbuild<Real, Real, false>), dim3(s.N), dim3(64), qshm, st, s.N, s.n_vol, s.adj_ptr,
                           s.adj_idx, s.pos, s.lat, s.tab, s.n_fib, s.n_phase, node_frac(s), s.sun_in[0], s.sun_in[1],
                           s.sun_in[2], (Real)s.mu0, (const Real *)s.T, (const Real *)s.rho, (const Real *)s.Tsun,
                           s.nodeoff, (Real *)s.val, (Real *)s.S, s.qsun, group, s.periodic, (long long)s.nx * kFx,
                           (long long)s.ny * kFx, s.qscreen);
    }
}

template void launch_qbuild<float>(Scene &, hipStream_t, int);
template void launch_qbuild<double>(Scene &, hipStream_t, int);

}  // namespace sg

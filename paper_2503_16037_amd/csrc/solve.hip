// Solve of (I - K) phi = S (Sec. 2, Eq. 8) by the Neumann series phi = S + K S
// + K^2 S + ... (Eq. 5), i.e. Jacobi sweeps x <- S + K x (diag K = 0), with
// FP64 residuals for iterative refinement and the pieces of a GMRES fallback.
//
// The sweep is node-blocked: node l owns a dense d_l x d_l block of K (rows
// = its out-edges, columns = its in-edges), stored column-major, so a
// wavefront (lane = row) reads each column with one coalesced load, gathers
// the d_l inputs x[rev(out(l))] once and never reads a column index.  Every reduction has a fixed order (wave
// butterfly, then block, then one final block), so results are bit-identical
// from run to run.
#include <algorithm>

#include "device.hpp"
#include "internal.hpp"

namespace sg {

namespace {

constexpr int kSpmvThreads = 256;
constexpr int kNodesPerSpmvBlock = kSpmvThreads / 64;
constexpr int kVecThreads = 256;

// Convergence measures of a sweep.  Every node writes meas[node][lambda] = (sum over
// its rows of |change|, max over its rows of |change| / (|value| + kRelFloor)); two
// fixed-shape kernels reduce them over nodes in FP64: chunk c of node_chunk(N, nl)
// consecutive nodes -> part[c][lambda][2], then over the chunks in a fixed order, so the
// result does not depend on how the sweep kernel was launched.  With several wavelengths
// the lanes run over wavelengths (coalesced rows) and the wavefronts over nodes.
__global__ __launch_bounds__(kSpmvThreads) void k_measure_chunks(const float2 *__restrict__ meas, int N, int nl,
                                                                int cn, double *__restrict__ part) {
    const int c = blockIdx.x, n0 = c * cn, n1 = min(N, n0 + cn);
    if (nl == 1) {
        double t = 0.0, u = 0.0;
        for (int i = n0 + (int)threadIdx.x; i < n1; i += kSpmvThreads) {
            const float2 m = meas[i];
            t += (double)m.x;
            u = fmax(u, (double)m.y);
        }
        t = block_sum<kSpmvThreads>(t);
        u = block_max<kSpmvThreads>(u);
        if (threadIdx.x == 0) {
            part[2 * c] = t;
            part[2 * c + 1] = u;
        }
        return;
    }
    constexpr int kW = kSpmvThreads / 64;
    __shared__ double red[kW][64][2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lam = blockIdx.y * 64 + lane;
    double t = 0.0, u = 0.0;
    if (lam < nl)
#pragma unroll 8
        for (int i = n0 + w; i < n1; i += kW) {
            const float2 m = meas[(long long)i * nl + lam];
            t += (double)m.x;
            u = fmax(u, (double)m.y);
        }
    red[w][lane][0] = t;
    red[w][lane][1] = u;
    __syncthreads();
    if (w == 0 && lam < nl) {
        double tt = 0.0, uu = 0.0;
#pragma unroll
        for (int k = 0; k < kW; ++k) {
            tt += red[k][lane][0];
            uu = fmax(uu, red[k][lane][1]);
        }
        part[((long long)c * nl + lam) * 2] = tt;
        part[((long long)c * nl + lam) * 2 + 1] = uu;
    }
}

// out[2 lambda] = sum, out[2 lambda + 1] = max over the nc chunks
__global__ __launch_bounds__(kSpmvThreads) void k_measure_nodes(const double *__restrict__ part, int nc, int nl,
                                                               double *__restrict__ out) {
    if (nl == 1) {
        double t = 0.0, u = 0.0;
        for (int i = threadIdx.x; i < nc; i += kSpmvThreads) {
            t += part[2 * i];
            u = fmax(u, part[2 * i + 1]);
        }
        t = block_sum<kSpmvThreads>(t);
        u = block_max<kSpmvThreads>(u);
        if (threadIdx.x == 0) {
            out[0] = t;
            out[1] = u;
        }
        return;
    }
    constexpr int kW = kSpmvThreads / 64;
    __shared__ double red[kW][64][2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lam = blockIdx.x * 64 + lane;
    double t = 0.0, u = 0.0;
    if (lam < nl)
#pragma unroll 8
        for (int i = w; i < nc; i += kW) {
            t += part[((long long)i * nl + lam) * 2];
            u = fmax(u, part[((long long)i * nl + lam) * 2 + 1]);
        }
    red[w][lane][0] = t;
    red[w][lane][1] = u;
    __syncthreads();
    if (w == 0 && lam < nl) {
        double tt = 0.0, uu = 0.0;
#pragma unroll
        for (int k = 0; k < kW; ++k) {
            tt += red[k][lane][0];
            uu = fmax(uu, red[k][lane][1]);
        }
        out[2 * lam] = tt;
        out[2 * lam + 1] = uu;
    }
}

// Broadcast lane m's value to the whole wavefront (m wave-uniform).
__device__ __forceinline__ float bcast(float v, int m) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), m));
}
__device__ __forceinline__ double bcast(double v, int m) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), m);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), m);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

constexpr int kStage = 16;  // block loads in flight per lane

// n passes of 64 consecutive block elements from t0 into the wavefront's LDS slice
template <int n, class Real>
__device__ __forceinline__ void stage_passes(const Real *__restrict__ blk_g, Real *__restrict__ blk, int t0, int nq,
                                             int lane) {
    Real v[n];
#pragma unroll
    for (int j = 0; j < n; ++j) v[j] = blk_g[min(t0 + j * 64 + lane, nq - 1)];
#pragma unroll
    for (int j = 0; j < n; ++j) blk[min(t0 + j * 64 + lane, nq - 1)] = v[j];
}

// Row lane of node block K_l times the gathered inputs: sum over m < d of K[lane][m] xg_m,
// in increasing m.  The block (d^2 values at blk_g, column-major: element (row n,
// column m) at m d + n) is copied to this wavefront's LDS slice with flat coalesced
// loads, kStage per lane in flight; rows are then read from LDS without bank conflicts
// (consecutive lanes, consecutive addresses).  The caller issues its other loads around
// this call; xl holds the input of in-edge `lane` (lane m's value is broadcast).
// blk == NULL: no LDS slice, every lane reads its row from memory.
template <class Acc, class Real, class XT>
__device__ __forceinline__ Acc node_row(const Real *__restrict__ blk_g, Real *__restrict__ blk, int d, int lane,
                                        XT xl) {
    if (!blk) {  // no LDS slice (FP64 blocks of large degree): columns straight from memory
        Acc acc = (Acc)0;
        if (lane < d)
            for (int m = 0; m < d; ++m) acc += (Acc)blk_g[(long long)m * d + lane] * (Acc)bcast(xl, m);
        return acc;
    }
    // as many 64-element passes as the block needs, at most kStage at a time (a wave-uniform
    // switch into straight-line copies, so the loads are issued back to back and waited for
    // once); lanes past the block's end reload and rewrite its last element
    const int nq = d * d;
    for (int t0 = 0; t0 < nq; t0 += 64 * kStage) {
        switch (min(kStage, (nq - t0 + 63) >> 6)) {
#define SG_STAGE_CASE(n) \
    case n: stage_passes<n>(blk_g, blk, t0, nq, lane); break;
            SG_STAGE_CASE(1) SG_STAGE_CASE(2) SG_STAGE_CASE(3) SG_STAGE_CASE(4) SG_STAGE_CASE(5) SG_STAGE_CASE(6)
            SG_STAGE_CASE(7) SG_STAGE_CASE(8) SG_STAGE_CASE(9) SG_STAGE_CASE(10) SG_STAGE_CASE(11) SG_STAGE_CASE(12)
            SG_STAGE_CASE(13) SG_STAGE_CASE(14) SG_STAGE_CASE(15) default: stage_passes<kStage>(blk_g, blk, t0, nq, lane);
#undef SG_STAGE_CASE
        }
    }
    __builtin_amdgcn_wave_barrier();
    Acc acc = (Acc)0;
    const int n = min(lane, d - 1);
    // eight LDS reads in flight at a time (the products still accumulate in increasing m)
    int m = 0;
    for (; m + 8 <= d; m += 8) {
        Real k[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) k[j] = blk[(m + j) * d + n];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc += (Acc)k[j] * (Acc)bcast(xl, m + j);
    }
    for (; m < d; ++m) acc += (Acc)blk[m * d + n] * (Acc)bcast(xl, m);
    __builtin_amdgcn_wave_barrier();  // the slice is rewritten by the next node
    return acc;
}

// A node's edge range and block offset (off, d, base); zeros past the last node.
struct NodeMeta {
    long long off, base;
    int d;
};
__device__ __forceinline__ NodeMeta load_meta(const long long *__restrict__ adj_ptr,
                                              const long long *__restrict__ nodeoff, int l, int N) {
    NodeMeta m{0, 0, 0};
    if (l < N) {
        m.off = adj_ptr[l];
        m.d = (int)(adj_ptr[l + 1] - m.off);
        m.base = nodeoff[l];
    }
    return m;
}

// y = S + K x, persistent over groups of four nodes, one wavefront per node.  With
// monitor != 0, meas[node] = (sum, max relative) of the node's updates y - x.
template <class Real>
__global__ __launch_bounds__(kSpmvThreads) void k_spmv(int N, int groups, const long long *__restrict__ adj_ptr,
                                                      const long long *__restrict__ nodeoff,
                                                      const int *__restrict__ rev, const Real *__restrict__ val,
                                                      const Real *__restrict__ S, const Real *__restrict__ x,
                                                      Real *__restrict__ y, float2 *__restrict__ meas, int monitor,
                                                      int dmax) {
    extern __shared__ unsigned char smem_raw[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    Real *blk = dmax ? reinterpret_cast<Real *>(smem_raw) + (size_t)w * dmax * dmax : nullptr;
    // node metadata is loaded one node ahead, so its latency overlaps the current node
    const int step = gridDim.x * kNodesPerSpmvBlock;
    int l = __builtin_amdgcn_readfirstlane(blockIdx.x * kNodesPerSpmvBlock + w);
    NodeMeta nm = load_meta(adj_ptr, nodeoff, l, N);
    for (; l < N; l += step) {
        const NodeMeta cur = nm;
        nm = load_meta(adj_ptr, nodeoff, l + step, N);
        const long long off = cur.off, base = cur.base;
        const int d = cur.d;
        if (d > kWave) continue;  // a node of higher degree: k_spmv_big
        if (d == 0) {
            if (monitor && lane == 0) meas[l] = make_float2(0.f, 0.f);
            continue;
        }
        if (!SG_IN(base + (long long)d * d - 1, nodeoff[N], 0x301)) continue;
        const bool act = lane < d;
        const long long b = off + min(lane, d - 1);  // lanes past d repeat the last row
        // the index load first, so that the gather waits for it alone
        const int rv0 = rev[b];
        const int rv = SG_IN(rv0, adj_ptr[N], 0x302) ? rv0 : (int)b;
        const Real sb = S[b];
        const Real xb = monitor ? x[b] : (Real)0;  // the previous value only for the measures
        const Real xl = x[rv];
        const Real acc = node_row<Real>(val + base, d <= dmax ? blk : nullptr, d, lane, xl);
        double r = 0.0, u = 0.0;
        if (act) {
            const Real yn = sb + acc;
            y[b] = yn;
            r = fabs((double)yn - (double)xb);
            // a NaN here is dropped by the max below, but it also makes this sweep's L1 sum
            // non-finite, which the solve policy checks first (guarding u as well would cost
            // this kernel two registers and a wave per SIMD)
            u = r / (fabs((double)yn) + kRelFloor);
        }
        if (monitor) {
            r = wave_sum(r);
            u = wave_max(u);
            if (lane == 0) meas[l] = make_float2((float)r, (float)u);
        }
    }
}

// The first Neumann iterate from x = 0 is the right-hand side itself: x = rhs, with the
// node measures of that update (a sweep would add K 0 = 0 and give the same bits).
template <class Real>
__global__ __launch_bounds__(kSpmvThreads) void k_first(int N, const long long *__restrict__ adj_ptr,
                                                       const Real *__restrict__ rhs, Real *__restrict__ x,
                                                       float2 *__restrict__ meas) {
    // two nodes per wavefront, one per 32-lane half (a node has ~24 rows)
    const int l = blockIdx.x * (2 * kNodesPerSpmvBlock) + (threadIdx.x >> 5), lane = threadIdx.x & 31;
    if (l >= N) return;  // a half past the last node exits; the shuffles below stay within a half
    const long long off = adj_ptr[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    double r = 0.0, u = 0.0;
    for (int n = lane; n < d; n += 32) {
        const Real v = rhs[off + n];
        x[off + n] = v;
        const double a = fabs((double)v);
        r += a;
        u = fmax(u, keep_nan(a / (a + kRelFloor)));
    }
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) {
        r += __shfl_xor(r, o, 32);
        u = fmax(u, __shfl_xor(u, o, 32));
    }
    if (lane == 0) meas[l] = make_float2((float)r, (float)u);
}

// r = S - x + K x in FP64 (K values promoted), persistent; meas[node] = (sum |r|,
// max |r| / (|x| + kRelFloor)) over the node's rows.
template <class Real>
__global__ __launch_bounds__(kSpmvThreads) void k_residual64(int N, int groups, const long long *__restrict__ adj_ptr,
                                                            const long long *__restrict__ nodeoff,
                                                            const int *__restrict__ rev, const Real *__restrict__ val,
                                                            const Real *__restrict__ S, const double *__restrict__ x,
                                                            double *__restrict__ r, float2 *__restrict__ meas,
                                                            int dmax) {
    extern __shared__ unsigned char smem_raw[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    Real *blk = dmax ? reinterpret_cast<Real *>(smem_raw) + (size_t)w * dmax * dmax : nullptr;
    const int step = gridDim.x * kNodesPerSpmvBlock;
    int l = __builtin_amdgcn_readfirstlane(blockIdx.x * kNodesPerSpmvBlock + w);
    NodeMeta nm = load_meta(adj_ptr, nodeoff, l, N);
    for (; l < N; l += step) {
        const NodeMeta cur = nm;
        nm = load_meta(adj_ptr, nodeoff, l + step, N);
        const long long off = cur.off, base = cur.base;
        const int d = cur.d;
        if (d > kWave) continue;  // a node of higher degree: k_residual64_big
        if (d == 0) {
            if (lane == 0) meas[l] = make_float2(0.f, 0.f);
            continue;
        }
        if (!SG_IN(base + (long long)d * d - 1, nodeoff[N], 0x303)) continue;
        const bool act = lane < d;
        const long long b = off + min(lane, d - 1);
        const int rv0 = rev[b];
        const int rv = SG_IN(rv0, adj_ptr[N], 0x304) ? rv0 : (int)b;
        const double sb = (double)S[b], xb = x[b];
        const double xl = x[rv];
        const double acc = node_row<double>(val + base, d <= dmax ? blk : nullptr, d, lane, xl);
        double a = 0.0, u = 0.0;
        if (act) {
            const double rb = (sb - xb) + acc;
            r[b] = rb;
            a = fabs(rb);
            u = keep_nan(a / (fabs(xb) + kRelFloor));
        }
        a = wave_sum(a);
        u = wave_max(u);
        if (lane == 0) meas[l] = make_float2((float)a, (float)u);
    }
}

// w = v - K v in FP64.
template <class Real>
__global__ __launch_bounds__(kSpmvThreads) void k_apply_imk64(int N, const long long *__restrict__ adj_ptr,
                                                             const long long *__restrict__ nodeoff,
                                                             const int *__restrict__ rev, const Real *__restrict__ val,
                                                             const double *__restrict__ v, double *__restrict__ wv,
                                                             int dmax) {
    extern __shared__ unsigned char smem_raw[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    Real *blk = dmax ? reinterpret_cast<Real *>(smem_raw) + (size_t)w * dmax * dmax : nullptr;
    const int l = __builtin_amdgcn_readfirstlane(blockIdx.x * kNodesPerSpmvBlock + w);
    if (l >= N) return;
    const long long off = adj_ptr[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    if (d == 0 || d > kWave) return;  // higher degree: k_apply_imk64_big
    const long long base = nodeoff[l];
    if (!SG_IN(base + (long long)d * d - 1, nodeoff[N], 0x305)) return;
    const bool act = lane < d;
    const long long b = off + min(lane, d - 1);
    const int rv0 = rev[b];
    const double xl = v[SG_IN(rv0, adj_ptr[N], 0x306) ? rv0 : (int)b];
    const double acc = node_row<double>(val + base, d <= dmax ? blk : nullptr, d, lane, xl);
    if (act) wv[b] = v[b] - acc;
}

// Row n of a node block of degree d times the staged inputs xin, summed in increasing
// column order (as node_row); eight columns' values are loaded before their products so
// that the loads overlap (32 measured slower).
template <class Acc, class Real, class XT>
__device__ __forceinline__ Acc big_row(const Real *__restrict__ blk, const XT *__restrict__ xin, int d, int n) {
    constexpr int kB = 8;
    Acc acc = (Acc)0;
    int m = 0;
    for (; m + kB <= d; m += kB) {
        Real v[kB];
#pragma unroll
        for (int j = 0; j < kB; ++j) v[j] = blk[(long long)(m + j) * d + n];
#pragma unroll
        for (int j = 0; j < kB; ++j) acc += (Acc)v[j] * (Acc)xin[m + j];
    }
    for (; m < d; ++m) acc += (Acc)blk[(long long)m * d + n] * (Acc)xin[m];
    return acc;
}

// Nodes of degree above 64 (graphs whose strongest couplings gather on the dense
// nodes): one 256-thread workgroup per (node, chunk of 256 rows), wg = bigrow[b] + c, so
// that a node of thousands of couplings is spread over many CUs; each workgroup stages
// the node's gathered inputs in LDS and each thread computes one row with the columns in
// increasing order.  Measures: each chunk writes its (sum, max) in FP64 to part[wg], and
// k_big_measures folds a node's chunks in order into meas[node].
__device__ __forceinline__ int big_locate(int nbig, const long long *__restrict__ bigrow, long long wg) {
    int lo = 0, hi = nbig;  // the node b with bigrow[b] <= wg < bigrow[b + 1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (bigrow[mid] <= wg) lo = mid; else hi = mid;
    }
    return lo;
}

template <class Real>
__global__ __launch_bounds__(256) void k_spmv_big(int nbig, const int *__restrict__ big,
                                                 const long long *__restrict__ bigrow,
                                                 const long long *__restrict__ adj_ptr,
                                                 const long long *__restrict__ nodeoff, const int *__restrict__ rev,
                                                 const Real *__restrict__ val, const Real *__restrict__ S,
                                                 const Real *__restrict__ x, Real *__restrict__ y,
                                                 double2 *__restrict__ part, int monitor) {
    extern __shared__ unsigned char smem_raw[];
    Real *xin = reinterpret_cast<Real *>(smem_raw);
    const long long wg = blockIdx.x;
    const int b = big_locate(nbig, bigrow, wg);
    const int l = big[b];
    const long long off = adj_ptr[l], base = nodeoff[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    for (int m = threadIdx.x; m < d; m += 256) xin[m] = x[rev[off + m]];
    __syncthreads();
    const int n = (int)(wg - bigrow[b]) * 256 + threadIdx.x;
    double r = 0.0, u = 0.0;
    if (n < d) {
        const Real acc = big_row<Real>(val + base, xin, d, n);
        const Real yn = S[off + n] + acc;
        y[off + n] = yn;
        if (monitor) {
            r = fabs((double)yn - (double)x[off + n]);
            u = keep_nan(r / (fabs((double)yn) + kRelFloor));
        }
    }
    if (monitor) {
        r = block_sum<256>(r);
        u = block_max<256>(u);
        if (threadIdx.x == 0) part[wg] = make_double2(r, u);
    }
}

// r = S - x + K x in FP64 for the nodes of degree above 64 (see k_spmv_big).
template <class Real>
__global__ __launch_bounds__(256) void k_residual64_big(int nbig, const int *__restrict__ big,
                                                       const long long *__restrict__ bigrow,
                                                       const long long *__restrict__ adj_ptr,
                                                       const long long *__restrict__ nodeoff,
                                                       const int *__restrict__ rev, const Real *__restrict__ val,
                                                       const Real *__restrict__ S, const double *__restrict__ x,
                                                       double *__restrict__ res, double2 *__restrict__ part) {
    extern __shared__ unsigned char smem_raw[];
    double *xin = reinterpret_cast<double *>(smem_raw);
    const long long wg = blockIdx.x;
    const int b = big_locate(nbig, bigrow, wg);
    const int l = big[b];
    const long long off = adj_ptr[l], base = nodeoff[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    for (int m = threadIdx.x; m < d; m += 256) xin[m] = x[rev[off + m]];
    __syncthreads();
    const int n = (int)(wg - bigrow[b]) * 256 + threadIdx.x;
    double a = 0.0, u = 0.0;
    if (n < d) {
        const double acc = big_row<double>(val + base, xin, d, n);
        const double xb = x[off + n];
        const double rb = ((double)S[off + n] - xb) + acc;
        res[off + n] = rb;
        a = fabs(rb);
        u = keep_nan(a / (fabs(xb) + kRelFloor));
    }
    a = block_sum<256>(a);
    u = block_max<256>(u);
    if (threadIdx.x == 0) part[wg] = make_double2(a, u);
}

// w = v - K v in FP64 for the nodes of degree above 64.
template <class Real>
__global__ __launch_bounds__(256) void k_apply_imk64_big(int nbig, const int *__restrict__ big,
                                                        const long long *__restrict__ bigrow,
                                                        const long long *__restrict__ adj_ptr,
                                                        const long long *__restrict__ nodeoff,
                                                        const int *__restrict__ rev, const Real *__restrict__ val,
                                                        const double *__restrict__ v, double *__restrict__ wv) {
    extern __shared__ unsigned char smem_raw[];
    double *xin = reinterpret_cast<double *>(smem_raw);
    const long long wg = blockIdx.x;
    const int b = big_locate(nbig, bigrow, wg);
    const int l = big[b];
    const long long off = adj_ptr[l], base = nodeoff[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    for (int m = threadIdx.x; m < d; m += 256) xin[m] = v[rev[off + m]];
    __syncthreads();
    const int n = (int)(wg - bigrow[b]) * 256 + threadIdx.x;
    if (n < d) wv[off + n] = v[off + n] - big_row<double>(val + base, xin, d, n);
}

// meas[node] of the nodes of degree above 64: their chunks' (sum, max) folded in order.
__global__ __launch_bounds__(256) void k_big_measures(int nbig, const int *__restrict__ big,
                                                     const long long *__restrict__ bigrow,
                                                     const double2 *__restrict__ part, float2 *__restrict__ meas) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nbig) return;
    double r = 0.0, u = 0.0;
    for (long long c = bigrow[b]; c < bigrow[b + 1]; ++c) {
        r += part[c].x;
        u = fmax(u, part[c].y);
    }
    meas[big[b]] = make_float2((float)r, (float)u);
}

// partial[j * nblk + block] = sum_i V[j][i] w[i], j < k (one pass over w).
__global__ __launch_bounds__(kVecThreads) void k_dot_multi(const double *__restrict__ V, long long ld, int k,
                                                          const double *__restrict__ w, long long n,
                                                          double *__restrict__ partial) {
    double acc[8];
    for (int j0 = 0; j0 < k; j0 += 8) {
        const int kk = min(8, k - j0);
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = 0.0;
        for (long long i = blockIdx.x * (long long)kVecThreads + threadIdx.x; i < n;
             i += (long long)gridDim.x * kVecThreads) {
            const double wi = w[i];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (j < kk) acc[j] += V[(long long)(j0 + j) * ld + i] * wi;
        }
        for (int j = 0; j < kk; ++j) {
            const double t = block_sum<kVecThreads>(acc[j]);
            if (threadIdx.x == 0) partial[(long long)(j0 + j) * gridDim.x + blockIdx.x] = t;
        }
    }
}

__global__ __launch_bounds__(1024) void k_reduce_multi(const double *__restrict__ partial, int nblk, int k,
                                                      double *__restrict__ out) {
    for (int j = 0; j < k; ++j) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nblk; i += 1024) s += partial[(long long)j * nblk + i];
        const double t = block_sum<1024>(s);
        if (threadIdx.x == 0) out[j] = t;
    }
}

// w -= sum_j h[j] V[j]
__global__ __launch_bounds__(kVecThreads) void k_axpy_multi(double *__restrict__ w, const double *__restrict__ V,
                                                           long long ld, int k, const double *__restrict__ h,
                                                           long long n) {
    for (long long i = blockIdx.x * (long long)kVecThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kVecThreads) {
        double s = w[i];
        for (int j = 0; j < k; ++j) s -= h[j] * V[(long long)j * ld + i];
        w[i] = s;
    }
}

template <class Real>
__global__ void k_to64(const Real *__restrict__ a, double *__restrict__ b, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = (double)a[i];
}

template <class Real>
__global__ void k_scaled_to_real(const double *__restrict__ a, double scale, Real *__restrict__ b, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = (Real)(a[i] * scale);
}

template <class Real>
__global__ void k_axpy_real_to64(double *__restrict__ x, const Real *__restrict__ d, double alpha, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        x[i] += alpha * (double)d[i];
}

__global__ void k_scale64(double *__restrict__ x, double alpha, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        x[i] *= alpha;
}

template <class Real>
__global__ void k_fill(Real *__restrict__ a, Real v, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        a[i] = v;
}

inline int grid_for(long long n) {
    long long g = (n + kVecThreads - 1) / kVecThreads;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

int spmv_blocks(const Scene &s) { return (s.N + kNodesPerSpmvBlock - 1) / kNodesPerSpmvBlock; }

// LDS of a sweep workgroup: one node block per wavefront, sized for degree up to 32 (a
// 4 KB FP32 slice, so eight wavefronts per SIMD fit; a radius graph's nodes above it are a
// few in a million) and at most 64 KiB; the rows of larger nodes are read from memory (the
// same products in the same order)
constexpr int kLdsDegree = 32;
template <class Real>
static size_t block_lds(const Scene &s) {
    const int dm = std::min(s.dmax, kLdsDegree);
    const size_t b = (size_t)kNodesPerSpmvBlock * dm * dm * sizeof(Real);
    return b <= 64 * 1024 ? b : 0;
}
template <class Real>
static int lds_dmax(const Scene &s) { return block_lds<Real>(s) ? std::min(s.dmax, kLdsDegree) : 0; }

// default launch shape of the sweeps: one group of four nodes per workgroup (the kernels
// also run persistent over fewer workgroups; the tuner measures both)
static int default_grid(const Scene &s) { return spmv_blocks(s); }

template <class Real>
void launch_spmv(Scene &s, hipStream_t st, const Real *S, const Real *x, Real *y, double *out, int grid,
                 hipEvent_t after, bool with_big) {
    if (grid <= 0) grid = default_grid(s);
    grid = std::min(grid, spmv_blocks(s));
    hipLaunchKernelGGL((k_spmv<Real>), dim3(grid), dim3(kSpmvThreads), block_lds<Real>(s), st, s.N, spmv_blocks(s),
                       s.adj_ptr, s.nodeoff, s.rev, (const Real *)s.val, S, x, y, s.meas, out ? 1 : 0, lds_dmax<Real>(s));
    if (s.n_big && with_big) {
        hipLaunchKernelGGL((k_spmv_big<Real>), dim3(s.n_bigrow), dim3(256), sizeof(Real) * s.dmax, st, s.n_big, s.big,
                           s.bigrow, s.adj_ptr, s.nodeoff, s.rev, (const Real *)s.val, S, x, y, s.big_part,
                           out ? 1 : 0);
        if (out)
            hipLaunchKernelGGL(k_big_measures, dim3((s.n_big + 255) / 256), dim3(256), 0, st, s.n_big, s.big, s.bigrow,
                               s.big_part, s.meas);
    }
    if (after) (void)hipEventRecord(after, st);
    if (out) launch_measures(s, 1, out, st);
}

template <class Real>
void launch_first(Scene &s, hipStream_t st, const Real *rhs, Real *x, double *out) {
    hipLaunchKernelGGL((k_first<Real>), dim3((s.N + 2 * kNodesPerSpmvBlock - 1) / (2 * kNodesPerSpmvBlock)),
                       dim3(kSpmvThreads), 0, st, s.N, s.adj_ptr, rhs, x, s.meas);
    launch_measures(s, 1, out, st);
}

template <class Real>
void launch_residual64(Scene &s, hipStream_t st, const Real *S, const double *x64, double *r64, double *out) {
    hipLaunchKernelGGL((k_residual64<Real>), dim3(default_grid(s)), dim3(kSpmvThreads), block_lds<Real>(s), st,
                       s.N, spmv_blocks(s), s.adj_ptr, s.nodeoff, s.rev, (const Real *)s.val, S, x64, r64, s.meas,
                       lds_dmax<Real>(s));
    if (s.n_big) {
        hipLaunchKernelGGL((k_residual64_big<Real>), dim3(s.n_bigrow), dim3(256), sizeof(double) * s.dmax, st, s.n_big,
                           s.big, s.bigrow, s.adj_ptr, s.nodeoff, s.rev, (const Real *)s.val, S, x64, r64, s.big_part);
        hipLaunchKernelGGL(k_big_measures, dim3((s.n_big + 255) / 256), dim3(256), 0, st, s.n_big, s.big, s.bigrow,
                           s.big_part, s.meas);
    }
    launch_measures(s, 1, out, st);
}

template <class Real>
void launch_apply_imk64(Scene &s, hipStream_t st, const double *v, double *w) {
    hipLaunchKernelGGL((k_apply_imk64<Real>), dim3(spmv_blocks(s)), dim3(kSpmvThreads), block_lds<Real>(s), st, s.N,
                       s.adj_ptr, s.nodeoff, s.rev, (const Real *)s.val, v, w, lds_dmax<Real>(s));
    if (s.n_big)
        hipLaunchKernelGGL((k_apply_imk64_big<Real>), dim3(s.n_bigrow), dim3(256), sizeof(double) * s.dmax, st,
                           s.n_big, s.big, s.bigrow, s.adj_ptr, s.nodeoff, s.rev, (const Real *)s.val, v, w);
}

void launch_measures(Scene &s, int nl, double *out, hipStream_t st) {
    const int cn = node_chunk(s.N, nl), nc = (s.N + cn - 1) / cn;
    const int lt = (nl + 63) / 64;
    hipLaunchKernelGGL(k_measure_chunks, dim3(nc, nl == 1 ? 1 : lt), dim3(kSpmvThreads), 0, st,
                       (const float2 *)s.meas, s.N, nl, cn, s.meas_part);
    hipLaunchKernelGGL(k_measure_nodes, dim3(nl == 1 ? 1 : lt), dim3(kSpmvThreads), 0, st,
                       (const double *)s.meas_part, nc, nl, out);
}

void launch_dot_multi(const double *V, int64_t ld, int k, const double *w, int64_t n, double *partial, int nblk,
                      double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_dot_multi, dim3(nblk), dim3(kVecThreads), 0, st, V, (long long)ld, k, w, (long long)n, partial);
    hipLaunchKernelGGL(k_reduce_multi, dim3(1), dim3(1024), 0, st, partial, nblk, k, out);
}

void launch_axpy_multi(double *w, const double *V, int64_t ld, int k, const double *h, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_axpy_multi, dim3(grid_for(n)), dim3(kVecThreads), 0, st, w, V, (long long)ld, k, h, (long long)n);
}

template <class Real>
void launch_to64(const Real *a, double *b, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL((k_to64<Real>), dim3(grid_for(n)), dim3(kVecThreads), 0, st, a, b, (long long)n);
}

template <class Real>
void launch_scaled_to_real(const double *a, double scale, Real *b, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL((k_scaled_to_real<Real>), dim3(grid_for(n)), dim3(kVecThreads), 0, st, a, scale, b, (long long)n);
}

template <class Real>
void launch_axpy_real_to64(double *x64, const Real *d, double alpha, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL((k_axpy_real_to64<Real>), dim3(grid_for(n)), dim3(kVecThreads), 0, st, x64, d, alpha, (long long)n);
}

void launch_scale64(double *x, double alpha, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_scale64, dim3(grid_for(n)), dim3(kVecThreads), 0, st, x, alpha, (long long)n);
}

template <class Real>
void launch_fill(Real *a, Real v, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL((k_fill<Real>), dim3(grid_for(n)), dim3(kVecThreads), 0, st, a, v, (long long)n);
}

#define SG_INST(R)                                                                                           \
    template void launch_spmv<R>(Scene &, hipStream_t, const R *, const R *, R *, double *, int, hipEvent_t, bool);               \
    template void launch_residual64<R>(Scene &, hipStream_t, const R *, const double *, double *, double *); \
    template void launch_first<R>(Scene &, hipStream_t, const R *, R *, double *);                          \
    template void launch_apply_imk64<R>(Scene &, hipStream_t, const double *, double *);                  \
    template void launch_to64<R>(const R *, double *, int64_t, hipStream_t);                               \
    template void launch_scaled_to_real<R>(const double *, double, R *, int64_t, hipStream_t);             \
    template void launch_axpy_real_to64<R>(double *, const R *, double, int64_t, hipStream_t);             \
    template void launch_fill<R>(R *, R, int64_t, hipStream_t);                                            \

SG_INST(float)
SG_INST(double)
#undef SG_INST

}  // namespace sg

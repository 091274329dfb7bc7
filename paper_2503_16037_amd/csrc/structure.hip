// CSR structure of the flux matrix K from the node adjacency.
//
// K is the adjacency matrix of the line graph of G(R, L) (Sec. 2, after
// Eq. 5): row b (an edge l -> n) has one column per in-edge a = (j -> l) of
// its tail l, so all d_l rows of node l share the same d_l columns and the
// node owns a dense d_l x d_l block stored row-major at nodeoff[l].
//   nodeoff   = exclusive scan over nodes of d_l^2
//   row_ptr[b] = nodeoff[l] + (b - adj_ptr[l]) * d_l
//   col_idx    = in(l) ascending = rev(adj_ptr[l] + m), m = 0..d_l-1
// (in(l) is ascending because heads are ascending within a row and edge ids
// are sorted by tail.)
#include "device.hpp"
#include "internal.hpp"

namespace sg {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;  // elements per thread
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ __launch_bounds__(256) void k_degree_sq(int N, const long long *__restrict__ adj_ptr,
                                                  long long *__restrict__ out) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < N) {
        const long long d = adj_ptr[l + 1] - adj_ptr[l];
        out[l] = d * d;
    }
}

// Exclusive scan, pass 1: each tile scanned locally in place, tile total to tsum.
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(long long *__restrict__ a, int n,
                                                            long long *__restrict__ tsum) {
    __shared__ long long sh[kScanThreads];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    long long v[kScanItems];
    long long run = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const long long x = (base + i < n) ? a[base + i] : 0;
        v[i] = run;
        run += x;
    }
    sh[threadIdx.x] = run;
    __syncthreads();
    // Hillis-Steele inclusive scan of the per-thread totals
    for (int o = 1; o < kScanThreads; o <<= 1) {
        const long long t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    const long long excl = threadIdx.x ? sh[threadIdx.x - 1] : 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) a[base + i] = v[i] + excl;
    if (threadIdx.x == kScanThreads - 1) tsum[blockIdx.x] = sh[kScanThreads - 1];
}

// Pass 2: exclusive scan of the tile totals by one block (serial over chunks).
__global__ __launch_bounds__(kScanThreads) void k_scan_totals(long long *__restrict__ tsum, int nt,
                                                             long long *__restrict__ grand) {
    __shared__ long long sh[kScanThreads];
    long long carry = 0;
    for (int c0 = 0; c0 < nt; c0 += kScanThreads) {
        const int i = c0 + threadIdx.x;
        const long long x = i < nt ? tsum[i] : 0;
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int o = 1; o < kScanThreads; o <<= 1) {
            const long long t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nt) tsum[i] = carry + sh[threadIdx.x] - x;
        const long long tot = sh[kScanThreads - 1];
        __syncthreads();
        carry += tot;
    }
    if (threadIdx.x == 0) *grand = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(long long *__restrict__ a, int n,
                                                          const long long *__restrict__ tsum) {
    const int base = blockIdx.x * kScanTile;
    const long long off = tsum[blockIdx.x];
    for (int i = threadIdx.x; i < kScanTile; i += kScanThreads)
        if (base + i < n) a[base + i] += off;
}

// rev(e) for every edge: position of (head, tail) in the head's row.  Two nodes per
// wavefront, one per 32-lane half (a node has ~24 edges, each a chain of dependent loads
// through the binary search, so a resident wavefront advances two chains per node slot).
__global__ __launch_bounds__(256) void k_rev(int N, const long long *__restrict__ adj_ptr,
                                            const int *__restrict__ adj_idx, int *__restrict__ rev) {
    const int l = blockIdx.x * 8 + (threadIdx.x >> 5);
    const int lane = threadIdx.x & 31;
    if (l >= N) return;
    const long long off = adj_ptr[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    for (int m = lane; m < d; m += 32) {
        const int j = adj_idx[off + m];
        if (!SG_IN(j, N, 0x601)) continue;
        long long lo = adj_ptr[j], hi = adj_ptr[j + 1];
        while (lo < hi) {
            const long long mid = (lo + hi) >> 1;
            if (adj_idx[mid] < l) lo = mid + 1; else hi = mid;
        }
        rev[off + m] = (int)lo;
    }
}

// Symmetry of the adjacency (every edge l -> j has its reverse j -> l): counts the
// edges whose reverse is missing (one wave per node, the search of k_rev).
__global__ __launch_bounds__(256) void k_check_symmetric(int N, const long long *__restrict__ adj_ptr,
                                                        const int *__restrict__ adj_idx, unsigned *__restrict__ bad) {
    const int l = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (l >= N) return;
    const long long off = adj_ptr[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    for (int m = lane; m < d; m += 64) {
        const int j = adj_idx[off + m];
        if (!SG_IN(j, N, 0x602)) continue;
        const long long end = adj_ptr[j + 1];
        long long lo = adj_ptr[j], hi = end;
        while (lo < hi) {
            const long long mid = (lo + hi) >> 1;
            if (adj_idx[mid] < l) lo = mid + 1; else hi = mid;
        }
        if (lo == end || adj_idx[lo] != l) atomicAdd(bad, 1u);
    }
}

__global__ __launch_bounds__(256) void k_row_ptr(int N, long long E, const long long *__restrict__ adj_ptr,
                                                const long long *__restrict__ nodeoff,
                                                long long *__restrict__ row_ptr) {
    const int l = blockIdx.x * 8 + (threadIdx.x >> 5);  // two nodes per wavefront
    const int lane = threadIdx.x & 31;
    if (l >= N) return;
    const long long off = adj_ptr[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    const long long b0 = nodeoff[l];
    for (int m = lane; m < d; m += 32) row_ptr[off + m] = b0 + (long long)m * d;
    if (l == N - 1 && lane == 0) row_ptr[E] = nodeoff[N];
}

__global__ __launch_bounds__(256) void k_col_idx(int N, const long long *__restrict__ adj_ptr,
                                                const long long *__restrict__ nodeoff, const int *__restrict__ rev,
                                                int *__restrict__ col) {
    const int l = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (l >= N) return;
    const long long off = adj_ptr[l];
    const int d = (int)(adj_ptr[l + 1] - off);
    const long long b0 = nodeoff[l];
    if (!SG_IN(b0 + (long long)d * d - 1, nodeoff[N], 0x603)) return;
    for (int t = lane; t < d * d; t += 64) col[b0 + t] = rev[off + (t % d)];
}

}  // namespace

void launch_structure(Scene &s, hipStream_t st) {
    const int N = s.N;
    hipLaunchKernelGGL(k_degree_sq, dim3((N + 255) / 256), dim3(256), 0, st, N, s.adj_ptr, s.nodeoff);
    const int nt = (N + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(kScanThreads), 0, st, s.nodeoff, N, s.scan_tmp);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanThreads), 0, st, s.scan_tmp, nt, s.nodeoff + N);
    hipLaunchKernelGGL(k_scan_add, dim3(nt), dim3(kScanThreads), 0, st, s.nodeoff, N, s.scan_tmp);
    const int nb = (N + 7) / 8;  // two nodes per wavefront, eight per workgroup
    hipLaunchKernelGGL(k_rev, dim3(nb), dim3(256), 0, st, N, s.adj_ptr, s.adj_idx, s.rev);
    hipLaunchKernelGGL(k_row_ptr, dim3(nb), dim3(256), 0, st, N, (long long)s.E, s.adj_ptr, s.nodeoff, s.row_ptr);
}

void launch_check_symmetric(Scene &s, unsigned *bad, hipStream_t st) {
    const int nb = (s.N + 3) / 4;
    hipLaunchKernelGGL(k_check_symmetric, dim3(nb), dim3(256), 0, st, s.N, s.adj_ptr, s.adj_idx, bad);
}

// The bounds checker's self-test: one check that fails by construction (the index equals
// the extent); the array behind it is never read.
__global__ void k_bounds_selftest(int n) {
    if (threadIdx.x == 0 && !SG_IN(n, n, 0xffffu)) return;
}

void launch_bounds_selftest(hipStream_t st) { hipLaunchKernelGGL(k_bounds_selftest, dim3(1), dim3(64), 0, st, 7); }

void launch_col_idx(Scene &s, hipStream_t st) {
    const int nb = (s.N + 3) / 4;
    hipLaunchKernelGGL(k_col_idx, dim3(nb), dim3(256), 0, st, s.N, s.adj_ptr, s.nodeoff, s.rev, s.col_idx);
}

}  // namespace sg

// Internal host-side definitions of the library: context, scene state and the
// launchers of the HIP kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <functional>
#include <map>
#include <unordered_map>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sgrt.h"

namespace sg {

constexpr int kHullNb = 16;  // neighbour slots per lattice point (hull adjacency)
// Largest node degree of a one-wavelength scene with Voronoi cells; wavelength batches and
// the colouring of the phase cells keep every node's couplings within one wavefront (64).
constexpr int kMaxDegree = 4096;
constexpr int kMaxWaveDegree = 64;

void set_error(const std::string &msg);
// Bounds-checked builds: each code module registers a reader of its first failed check
// (0: none), and bounds_report returns SG_E_DEVICE naming it (SG_OK in release builds).
void register_bounds_reader(unsigned (*reader)());
sg_status bounds_report();
void launch_bounds_selftest(hipStream_t st);  // one failing check on purpose (never dereferenced)
std::string t_last_error();

// a captured chunk of sweeps: key = (kind, chunk length, buffers and flags it was recorded with)
using GraphKey = std::array<uintptr_t, 8>;
struct SceneGraph {
    int seen = 0;                   // times the chunk ran; captured on the second
    hipGraphExec_t exec = nullptr;
};

// Caching pool of device blocks (pool.cpp): size -> free block, and every block's size.
struct Pool {
    std::mutex mu;
    std::multimap<uint64_t, void *> free_blocks;
    std::unordered_map<void *, uint64_t> sizes;
    uint64_t cached = 0;  // bytes in free_blocks
};

struct Ctx {
    int device = 0;
    uint64_t budget = 0;
    std::atomic<uint64_t> used{0};
    std::atomic<int> sticky{0};
    std::atomic<int> n_scenes{0};
    hipStream_t stream = nullptr;
    Pool pool;
};

// ---- pool.cpp ----
uint64_t pool_round(uint64_t bytes);  // the size the pool allocates for a request
// a block of at least `bytes`, counted in ctx->used; SG_E_NOMEM beyond the budget
sg_status pool_alloc(Ctx *ctx, uint64_t bytes, void **out);
void pool_free(Ctx *ctx, void *ptr);  // back to the cache (NULL and foreign pointers ignored)
void pool_trim(Ctx *ctx, uint64_t keep);  // release cached blocks down to `keep` bytes

// Device arrays of one scene.  "Real" arrays hold float in FP32 solves and
// double in FP64 solves; they are allocated for the precision of the first
// solve that needs them.
struct Scene {
    Ctx *ctx = nullptr;
    // sizes
    int nx = 0, ny = 0, nz = 0;
    double voxel_m = 0.0;
    int nvox = 0, N = 0, npx = 0;
    // volume nodes: nvox (one per voxel, node id = voxel id) or a general node set (the path
    // points of the lines of sight), each node with the medium of its voxel
    int n_vol = 0;
    bool general = false;
    int64_t E = 0, nnz = 0;
    int dmax = 0;
    // nodes of degree above 64 (handled by their own kernels: one workgroup per node in the
    // sweeps, one per (node, incoming direction) in the phase cells)
    int n_big = 0;
    int *big = nullptr;           // [n_big] node ids, ascending
    long long *bigdir = nullptr;  // [n_big + 1] prefix of their groups of incoming directions
    long long n_bigdir = 0;
    long long *bigrow = nullptr;  // [n_big + 1] prefix of their chunks of 256 rows
    long long n_bigrow = 0;
    double2 *big_part = nullptr;  // [n_bigrow] per-chunk measures of the sweeps
    int n_phase = 1;
    double hg_g[4] = {0, 0, 0, 0};
    int phase_kind[4] = {0, 0, 0, 0};  // SG_PHASE_HG, SG_PHASE_RAYLEIGH, SG_PHASE_TABLE
    int lut_n = 0;                     // samples per phase table row (0: no table)
    double lut_scale[4] = {1, 1, 1, 1};  // 1 / integral over the sphere of each table row
    double *lut = nullptr;             // [n_phase][lut_n] phase tables (device)
    int sigma_mode = 0;                // SG_SIGMA_VORONOI or SG_SIGMA_COLOUR
    float *phi32 = nullptr;  // a batched solve's solution while it is the FP32 iterate itself (bx or by),
                             // before any FP64 copy was needed
    int qscreen = 1;                   // phase-cell owners through the FP32 screen (0: FP64 scan only)
    int periodic = 0;                  // bit 0: x, bit 1: y repeat with the grid's period
    int *hull = nullptr;               // colouring: [n_fib][kHullNb] hull neighbours, then [n_fib] counts
    int n_fib = 100;
    int surface = 1;
    int weight_mode = 0;
    int n_lambda = 1;
    std::vector<float> abs_scale;
    int sun[3] = {0, 0, 0}, view[3] = {0, 0, 0};
    double sun_in[3] = {0, 0, 0};  // propagation direction of sunlight (unit)
    double view_u[3] = {0, 0, 0};  // unit vector toward the sensor
    double mu0 = 0.0;
    uint64_t bytes = 0;

    // inputs
    float *mu_s = nullptr, *mu_a = nullptr, *frac = nullptr, *albedo = nullptr, *abs_scale_d = nullptr;
    // general nodes: the medium of each node's voxel ([n_vol], fractions [n_phase][n_vol]) and
    // the lines of sight's elements (pixel p's at los_ptr[p] ...: node and upper end)
    float *gmu_s = nullptr, *gmu_a = nullptr, *gfrac = nullptr;
    long long *los_ptr = nullptr;
    int *los_node = nullptr;
    double *los_t = nullptr;
    int *pos = nullptr;  // [N][3]
    long long *adj_ptr = nullptr;
    int *adj_idx = nullptr;
    double *lat = nullptr;  // [n_fib][3]
    double *tab = nullptr;  // [n_phase + 1][n_fib]: HG tables, then the Lambertian cosine weights

    // structure
    int *rev = nullptr;
    long long *nodeoff = nullptr;  // [N + 1] exclusive scan of degree^2
    long long *row_ptr = nullptr;  // [E + 1]
    int *col_idx = nullptr;        // [nnz], on demand
    long long *scan_tmp = nullptr;
    bool col_built = false;

    // single-wavelength arrays (Real)
    int real_bytes = 0;  // 4 or 8, 0 = not allocated
    void *tau_s = nullptr, *tau_a = nullptr, *tsun_s = nullptr, *tsun_a = nullptr;
    void *T = nullptr, *Tsun = nullptr, *rho = nullptr, *val = nullptr, *S = nullptr, *x = nullptr, *y = nullptr;
    void *c_rhs = nullptr, *c_a = nullptr, *c_b = nullptr;  // refinement correction: RHS and two iterates
    float *qsun = nullptr;  // [E]

    // batched arrays (n_lambda > 1, FP32)
    float *q = nullptr;                   // [nnz] phase-cell weights in K layout
    float *bS = nullptr, *bx = nullptr, *by = nullptr;  // [E][n_lambda]
    float *brho = nullptr;                // [N][n_lambda] node weights
    float *bsrc = nullptr;                // [N][n_lambda] T_sun (x mu0 on the surface)
    double *lam_buf = nullptr;            // [68 * n_lambda] per-wavelength scales and measures

    // FP64 solve state
    double *x64 = nullptr, *r64 = nullptr;  // [E * n_lambda]
    double *gm_V = nullptr;                 // GMRES basis [(m+1) * E] (+ [2 * E] in a batched scene)
    int gm_m = 0;
    bool gm_nomem = false;                  // the last solve ran out of budget allocating the basis
    double *partial = nullptr;  // block partial sums (GMRES dot products)
    float2 *meas = nullptr;      // [N][n_lambda] per-node (sum, max relative) of the last sweep's changes
    double *meas_part = nullptr;  // [node_chunks(N, n_lambda)][n_lambda][2] chunk reductions of meas
    int n_partial = 0;
    double *scal = nullptr;  // device scalars
    double *J = nullptr;     // [N * n_lambda] node radiance toward the sensor
    double *pix = nullptr;   // [n_lambda * npx] radiance staging for host outputs

    std::map<GraphKey, SceneGraph> graphs;  // captured sweep chunks
    // a second stream for the sun march, which runs beside the structure pass and the edge
    // march (fork from the solve's stream at its start, join before the first reader of the
    // sun's optical depths); created with the scene, default priority
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int spmv_grid = 0, spmm_grid = 0;       // tuned launch shapes (0 = not tuned yet)
    int spmm_tile = 0;                      // tuned wavelength tile of the batched sweeps
    int tile = 64;                          // wavelength tile of the current batched solve
    int spmv_grid_bytes = 0;                // element size spmv_grid was tuned for

    int solves = 0;  // solves started on this scene
    bool solved = false;
    int last_precision = 0;
    int last_scatter_order = 0;
    std::mutex mu;
};

// The medium at each volume node (indexed by node id; stride n_vol for the fractions): the
// voxel arrays themselves when nodes and voxels coincide.
inline const float *node_mu_s(const Scene &s) { return s.general ? s.gmu_s : s.mu_s; }
inline const float *node_mu_a(const Scene &s) { return s.general ? s.gmu_a : s.mu_a; }
inline const float *node_frac(const Scene &s) { return s.general ? s.gfrac : s.frac; }

// The phase-function components of a scene (Sec. 3): kind 0 Henyey-Greenstein (g),
// 1 Rayleigh, 2 a table in cos(theta) (row c of lut, lut_n samples at -1 + 2 m /
// (lut_n - 1), linear between them, times scale[c] = 1 / its integral over the
// sphere).  Passed to kernels by value; lut in device memory.
struct PhaseSet {
    double g[4], scale[4];
    int kind[4];
    int n, lut_n;
    const double *lut;
};

inline PhaseSet phase_set(const Scene &s) {
    PhaseSet p;
    for (int c = 0; c < 4; ++c) {
        p.g[c] = s.hg_g[c];
        p.scale[c] = s.lut_scale[c];
        p.kind[c] = s.phase_kind[c];
    }
    p.n = s.n_phase;
    p.lut_n = s.lut_n;
    p.lut = s.lut;
    return p;
}

// ---- scene lifecycle (api.cpp) ----
sg_status create_scene(Ctx *ctx, const sg_scene_desc *d, hipStream_t st, Scene &s);
void free_scene(Scene *s);
sg_status solve_scene(Scene &s, const sg_solve_opts &o, hipStream_t st, double *radiance, int on_dev,
                      sg_solve_info *info);
sg_status check_opts(const sg_solve_opts *opts, sg_solve_opts &o);
// device bytes a scene reserves (validates the description; *st = its status)
uint64_t scene_reservation(const sg_scene_desc *d, sg_status *st);
// device bytes a solve with options o may allocate beyond the scene's reservation: the FP64
// working arrays, the CSR column index, and (with_gmres) the GMRES basis (0 if d is invalid)
uint64_t solve_reservation(const sg_scene_desc *d, const sg_solve_opts &o, bool with_gmres);
// both in one validation: the scene's reservation plus, with o, its solve's (*st = status)
uint64_t reservations(const sg_scene_desc *d, const sg_solve_opts *o, bool with_gmres, sg_status *st);

// ---- noalloc.hip ----
// looks up, once per device and with that device current, the device address of the
// allocation-free trace's staging array (called by sg_ctx_create)
sg_status scratch_setup(int device);
// staging bytes of an allocation-free trace of n_ids paths of cap slots
uint64_t trace_noalloc_bytes(int64_t n_ids, int64_t cap);

// ---- runtime.cpp ----
// persistent grid of the single-wavelength sweep (0 = default shape when autotune is off);
// x and y are scratch vectors that tuning may overwrite
template <class Real>
int spmv_grid(Scene &s, hipStream_t st, const Real *S, Real *x, Real *y, bool autotune);
// persistent grid of the batched sweep (x, y: scratch as above)
// launch shape of the batched sweeps: sets s.tile (force_tile > 0: that tile, default
// grid) and returns the grid
int spmm_grid(Scene &s, hipStream_t st, float *x, float *y, bool autotune, int force_tile);
// runs body() (kernel launches only) directly, or as a captured graph replay
sg_status run_chunk(Scene &s, hipStream_t st, const GraphKey &key, bool use_graphs, const std::function<void()> &body);
void clear_graphs(Scene &s);

// ---- launchers (defined in the .hip files) ----
void launch_structure(Scene &s, hipStream_t st);
void launch_col_idx(Scene &s, hipStream_t st);
// *bad += number of edges whose reverse edge is missing (*bad zeroed by the caller)
void launch_check_symmetric(Scene &s, unsigned *bad, hipStream_t st);

template <class Real>
void launch_march_edges(Scene &s, hipStream_t st, float scale, int use_lds);
template <class Real>
void launch_march_sun(Scene &s, hipStream_t st, float scale);
template <class Real>
void launch_node_weights(Scene &s, hipStream_t st, float scale);
template <class Real>
void launch_qbuild(Scene &s, hipStream_t st, int write_q);
// incoming directions the phase-cell kernels take per group (a lattice of NF points), and
// per workgroup of the kernel for nodes of degree above 64
int qbuild_group(int NF);
int qbuild_group_big(int NF);

template <class Real>
// one sweep y = S + K x; out[0..1] = measures of y - x (see launch_measures);
// after: an event recorded right after the sweep kernel; with_big = false leaves out the
// nodes of degree above 64 (the launch-shape tuner times the regular kernel alone)
void launch_spmv(Scene &s, hipStream_t st, const Real *S, const Real *x, Real *y, double *out, int grid = 0,
                 hipEvent_t after = nullptr, bool with_big = true);
// the first Neumann iterate from x = 0: x = rhs; out[0..1] = measures of that update
template <class Real>
void launch_first(Scene &s, hipStream_t st, const Real *rhs, Real *x, double *out);
template <class Real>
void launch_residual64(Scene &s, hipStream_t st, const Real *S, const double *x64, double *r64, double *norm_out);
template <class Real>
void launch_apply_imk64(Scene &s, hipStream_t st, const double *v, double *w);
int spmv_blocks(const Scene &s);
// Convergence measures of the last sweep or residual, reduced over nodes:
// out[2 lambda] = sum over edges of |change|, out[2 lambda + 1] = max over edges of
// |change| / (|value| + 1e-30), for lambda < nl.
// nodes per reduction chunk: 2048 for one wavelength; about sqrt(N) for several, which
// balances the chunk pass (chunk length) against the final pass (number of chunks)
inline int node_chunk(int N, int nl) {
    if (nl == 1) return 2048;
    int c = 32;
    while ((long long)c * c < N) c *= 2;
    return c;
}
inline int node_chunks(int N, int nl) { return (N + node_chunk(N, nl) - 1) / node_chunk(N, nl); }
void launch_measures(Scene &s, int nl, double *out, hipStream_t st);
void launch_dot_multi(const double *V, int64_t ld, int k, const double *w, int64_t n, double *partial, int nblk,
                      double *out, hipStream_t st);
void launch_axpy_multi(double *w, const double *V, int64_t ld, int k, const double *h, int64_t n, hipStream_t st);

template <class Real>
void launch_to64(const Real *a, double *b, int64_t n, hipStream_t st);
template <class Real>
void launch_scaled_to_real(const double *a, double scale, Real *b, int64_t n, hipStream_t st);
template <class Real>
void launch_axpy_real_to64(double *x64, const Real *d, double alpha, int64_t n, hipStream_t st);
void launch_scale64(double *x, double alpha, int64_t n, hipStream_t st);
template <class Real>
void launch_fill(Real *a, Real v, int64_t n, hipStream_t st);

template <class Real>
void launch_gather(Scene &s, hipStream_t st, const double *phi, int scatter_order, double *radiance);

void launch_trace(Scene &s, hipStream_t st, int kind, const long long *ids, int n, int cap, int *vox, double *dt,
                  int *count);

// batched wavelengths
int smallest_tile(int n_lambda);  // the narrowest of 8, 16, 32, 64 lanes that holds n_lambda
int default_tile(int n_lambda);   // the untuned choice
int batched_groups(const Scene &s);  // node groups of the batched sweep at tile s.tile
void launch_bnode_coef(Scene &s, hipStream_t st);
// the first batched Neumann iterate from x = 0: x = rhs (NULL: the solar source), with
// per-node measures to s.meas
void launch_bfirst(Scene &s, hipStream_t st, const float *rhs, float *x);
// one batched sweep y = rhs + K x for all wavelengths (rhs = NULL: the solar source);
// monitor != 0: per-node measures of y - x to s.meas
void launch_spmm(Scene &s, hipStream_t st, int grid, const float *rhs, const float *x, float *y, int monitor);
// r = S + K x64 - x64 evaluated in FP64 for all wavelengths and stored in FP32 (the correction
// solve takes it in FP32); per-node measures of r relative to x (from the FP64 values) to s.meas
void launch_bresidual64(Scene &s, hipStream_t st, int grid, const double *x64, float *r32);
// the same residual of the FP32 iterate itself (its values promoted: the bits of x64 = x)
void launch_bresidual32(Scene &s, hipStream_t st, int grid, const float *x, float *r32);
// b[e][lambda] *= sc[lambda] (FP32 values, FP64 scales)
void launch_lam_scale_f32(float *b, const double *sc, int nl, long long n, hipStream_t st);
// one wavelength of a batched scene in FP64 (its GMRES fallback): the residual r = S - (I - K) x
// with its two measures in scal[0..1], w = (I - K) v, and one wavelength's slice of [E][nl]
void launch_blam_residual64(Scene &s, hipStream_t st, int lam, const double *x, double *r);
void launch_blam_apply64(Scene &s, hipStream_t st, int lam, const double *v, double *w);
void launch_lam_take64(const double *x, int nl, int lam, long long E, double *out, hipStream_t st);
void launch_lam_put64(const double *in, int nl, int lam, long long E, double *x, hipStream_t st);
void launch_lam_axpy(double *x, const float *d, const double *sc, int nl, long long n, hipStream_t st);
void launch_f32_to_64(const float *a, double *b, long long n, hipStream_t st);
void launch_lam_to_edge_major(const double *src, double *dst, int nl, long long E, hipStream_t st);
void launch_fill_f32(float *a, long long n, hipStream_t st);
void launch_batched_gather(Scene &s, hipStream_t st, const double *phi, int scatter_order, double *radiance);
void launch_batched_gather(Scene &s, hipStream_t st, const float *phi, int scatter_order, double *radiance);

}  // namespace sg

// the public handles of a context and a scene
struct sg_ctx : public sg::Ctx {};
struct sg_scene : public sg::Scene {};

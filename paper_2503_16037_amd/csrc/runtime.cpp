// Host runtime around the sweep kernels: a launch-shape autotuner and the
// replay of fixed chunks of sweeps as HIP graphs.
//
// Autotuner.  The persistent sweep kernels take any grid size, and their
// results do not depend on it (every output element and every per-node norm
// contribution is produced by one wavefront in a fixed order; the norms are
// reduced by fixed-shape kernels).  From a scene's second solve on, the tuner
// times a short list of grid sizes with HIP events on the scene's own data and
// keeps the fastest, per problem shape, for the life of the process (a scene
// solved once, as in serving, never pays for tuning); SG_AUTOTUNE_CACHE names
// an optional text file that keeps the choices across processes.
//
// Graphs.  A chunk of sweeps is a fixed sequence of kernel launches on fixed
// buffers.  The second time a scene runs the same chunk it is captured on the
// scene's stream and from then on replayed with one hipGraphLaunch, which
// removes the per-launch host cost that dominates small scenes.  Captured
// graphs hold only kernel nodes (no memset or copy nodes).
#include <hip/hip_runtime.h>

#include <array>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace sg {

namespace {

using TuneKey = std::array<long long, 7>;  // kind, N, E, nnz, dmax, n_lambda, element bytes

std::mutex g_tune_mu;
std::map<TuneKey, int> g_tuned;
bool g_cache_loaded = false;

const char *cache_path() {
    const char *p = std::getenv("SG_AUTOTUNE_CACHE");
    return (p && p[0]) ? p : nullptr;
}

void load_cache_locked() {
    if (g_cache_loaded) return;
    g_cache_loaded = true;
    const char *p = cache_path();
    if (!p) return;
    FILE *f = std::fopen(p, "r");
    if (!f) return;
    TuneKey k;
    int grid;
    while (std::fscanf(f, "%lld %lld %lld %lld %lld %lld %lld %d", &k[0], &k[1], &k[2], &k[3], &k[4], &k[5], &k[6],
                       &grid) == 8)
        if (grid > 0) g_tuned[k] = grid;
    std::fclose(f);
}

void store_cache_locked(const TuneKey &k, int grid) {
    g_tuned[k] = grid;
    const char *p = cache_path();
    if (!p) return;
    FILE *f = std::fopen(p, "a");
    if (!f) return;
    std::fprintf(f, "%lld %lld %lld %lld %lld %lld %lld %d\n", k[0], k[1], k[2], k[3], k[4], k[5], k[6], grid);
    std::fclose(f);
}

// Times launch(grid) for every candidate (one warm-up launch, then three timed
// launches each) and returns the fastest; 0 if the device reports an error.
template <class F>
int time_candidates(hipStream_t st, const std::vector<int> &cands, F &&launch) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return 0;
    int best = 0;
    float best_ms = 0.0f;
    for (int g : cands) {
        launch(g);
        (void)hipEventRecord(a, st);
        for (int r = 0; r < 3; ++r) launch(g);
        (void)hipEventRecord(b, st);
        if (hipEventSynchronize(b) != hipSuccess) { best = 0; break; }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, a, b);
        if (!best || ms < best_ms) { best = g; best_ms = ms; }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (hipGetLastError() != hipSuccess) return 0;
    return best;
}

std::vector<int> grid_candidates(int groups) {
    std::vector<int> c;
    for (int g : {256, 512, 768, 1024, 1536, 2048, 3072, 4096})
        if (g < groups) c.push_back(g);
    c.push_back(groups);  // one node group per workgroup
    return c;
}

}  // namespace

template <class Real>
int spmv_grid(Scene &s, hipStream_t st, const Real *S, Real *x, Real *y, bool autotune) {
    if (!autotune) return 0;
    if (s.spmv_grid > 0 && s.spmv_grid_bytes == (int)sizeof(Real)) return s.spmv_grid;
    const TuneKey k{0, s.N, s.E, s.nnz, s.dmax, 1, (long long)sizeof(Real)};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    auto it = g_tuned.find(k);
    int grid = it != g_tuned.end() ? it->second : 0;
    if (!grid && s.solves < 2) return 0;  // a scene's first solve does not tune
    if (!grid) {
        double *scratch = s.scal + 200;  // two measures (the tuned sweeps are monitored ones)
        launch_fill<Real>(x, (Real)0, s.E, st);  // x and y are scratch vectors here
        grid = time_candidates(st, grid_candidates(spmv_blocks(s)),
                               [&](int g) { launch_spmv<Real>(s, st, S, x, y, scratch, g); });
        if (grid) store_cache_locked(k, grid);
    }
    s.spmv_grid = grid;
    s.spmv_grid_bytes = (int)sizeof(Real);
    return grid;
}

int spmm_grid(Scene &s, hipStream_t st, float *x, float *y, bool autotune) {
    const int groups = batched_groups(s);
    const int fallback = groups;  // one node group per workgroup
    if (!autotune) return fallback;
    if (s.spmm_grid > 0) return s.spmm_grid;
    const TuneKey k{1, s.N, s.E, s.nnz, s.dmax, s.n_lambda, 4};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    auto it = g_tuned.find(k);
    int grid = it != g_tuned.end() ? it->second : 0;
    if (!grid && s.solves < 2) return fallback;  // a scene's first solve does not tune
    if (!grid) {
        launch_fill_f32(x, (long long)s.E * s.n_lambda, st);  // x and y are scratch vectors here
        grid = time_candidates(st, grid_candidates(groups), [&](int g) { launch_spmm(s, st, g, nullptr, x, y, 1); });
        if (grid) store_cache_locked(k, grid);
    }
    s.spmm_grid = grid ? grid : fallback;
    return s.spmm_grid;
}

template int spmv_grid<float>(Scene &, hipStream_t, const float *, float *, float *, bool);
template int spmv_grid<double>(Scene &, hipStream_t, const double *, double *, double *, bool);

sg_status run_chunk(Scene &s, hipStream_t st, const GraphKey &key, bool use_graphs, const std::function<void()> &body) {
    if (!use_graphs) {
        body();
        return hipGetLastError() == hipSuccess ? SG_OK : SG_E_DEVICE;
    }
    SceneGraph &g = s.graphs[key];
    if (!g.exec && ++g.seen >= 2) {
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            body();
            const hipError_t e = hipStreamEndCapture(st, &graph);
            if (e != hipSuccess || !graph) {
                if (graph) (void)hipGraphDestroy(graph);
                set_error(std::string("graph capture failed: ") + hipGetErrorString(e));
                return SG_E_DEVICE;
            }
            hipGraphExec_t ex = nullptr;
            const hipError_t ei = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ei != hipSuccess) {
                set_error(std::string("graph instantiate failed: ") + hipGetErrorString(ei));
                return SG_E_DEVICE;
            }
            g.exec = ex;
        } else {
            (void)hipGetLastError();  // stream cannot be captured: launch directly from now on
            g.seen = -1000000;
        }
    }
    if (g.exec) {
        const hipError_t e = hipGraphLaunch(g.exec, st);
        if (e != hipSuccess) {
            set_error(std::string("hipGraphLaunch failed: ") + hipGetErrorString(e));
            return SG_E_DEVICE;
        }
        return SG_OK;
    }
    body();
    return hipGetLastError() == hipSuccess ? SG_OK : SG_E_DEVICE;
}

void clear_graphs(Scene &s) {
    for (auto &kv : s.graphs)
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    s.graphs.clear();
}

}  // namespace sg

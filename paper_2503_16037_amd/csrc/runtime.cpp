// Host runtime around the sweep kernels: a launch-shape autotuner and the
// replay of fixed chunks of sweeps as HIP graphs.
//
// Autotuner.  The persistent sweep kernels take any grid size, and the batched
// sweep any wavelength tile that holds the scene's wavelengths; their results do
// not depend on either (every output element and every per-node norm contribution
// is produced by one lane in a fixed order; the norms are reduced by fixed-shape
// kernels).  From a scene's second solve on, the tuner times a short list of
// launch shapes with HIP events on the scene's own data and keeps the fastest, per
// problem shape, for the life of the process (a scene solved once, as in serving,
// never pays for tuning); SG_AUTOTUNE_CACHE names an optional file that keeps the
// choices across processes, one JSON object per line (appended as choices are made):
//   {"kind": k, "N": n, "E": e, "nnz": z, "dmax": d, "n_lambda": l, "bytes": b, "grid": g, "tile": t}
// Lines of any other shape are ignored.
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
struct Shape {
    int grid = 0, tile = 0;  // tile: batched sweeps only
};

std::mutex g_tune_mu;
std::map<TuneKey, Shape> g_tuned;
bool g_cache_loaded = false;

// one cache entry (printf and scanf format alike: the keys in this order)
constexpr const char *kCacheLine =
    "{\"kind\": %lld, \"N\": %lld, \"E\": %lld, \"nnz\": %lld, \"dmax\": %lld, \"n_lambda\": %lld, "
    "\"bytes\": %lld, \"grid\": %d, \"tile\": %d}";

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
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        TuneKey k;
        Shape v;
        if (std::sscanf(line, kCacheLine, &k[0], &k[1], &k[2], &k[3], &k[4], &k[5], &k[6], &v.grid, &v.tile) == 9 &&
            v.grid > 0)
            g_tuned[k] = v;
    }
    std::fclose(f);
}

void store_cache_locked(const TuneKey &k, Shape v) {
    g_tuned[k] = v;
    const char *p = cache_path();
    if (!p) return;
    FILE *f = std::fopen(p, "a");
    if (!f) return;
    std::fprintf(f, kCacheLine, k[0], k[1], k[2], k[3], k[4], k[5], k[6], v.grid, v.tile);
    std::fputc('\n', f);
    std::fclose(f);
}

// Times every candidate shape (one warm-up launch, then three timed launches each)
// and returns the fastest; {0, 0} if the device reports an error.
template <class F>
Shape time_candidates(hipStream_t st, const std::vector<Shape> &cands, F &&launch) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return Shape{};
    Shape best;
    float best_ms = 0.0f;
    for (const Shape &c : cands) {
        launch(c);
        (void)hipEventRecord(a, st);
        for (int r = 0; r < 3; ++r) launch(c);
        (void)hipEventRecord(b, st);
        if (hipEventSynchronize(b) != hipSuccess) { best = Shape{}; break; }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, a, b);
        if (!best.grid || ms < best_ms) { best = c; best_ms = ms; }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (hipGetLastError() != hipSuccess) return Shape{};
    return best;
}

std::vector<Shape> grid_candidates(int groups, int tile = 0) {
    std::vector<Shape> c;
    for (int g : {256, 512, 768, 1024, 1536, 2048, 3072, 4096, 6144, 8192, 12288, 16384})
        if (g < groups) c.push_back({g, tile});
    c.push_back({groups, tile});  // one node group per workgroup
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
    int grid = it != g_tuned.end() ? it->second.grid : 0;
    if (!grid && s.solves < 2) return 0;  // a scene's first solve does not tune
    if (!grid) {
        double *scratch = s.scal + 200;  // two measures (the tuned sweeps are monitored ones)
        launch_fill<Real>(x, (Real)0, s.E, st);  // x and y are scratch vectors here
        grid = time_candidates(st, grid_candidates(spmv_blocks(s)),
                               [&](const Shape &c) { launch_spmv<Real>(s, st, S, x, y, scratch, c.grid, nullptr, false); })
                   .grid;
        if (grid) store_cache_locked(k, Shape{grid, 0});
    }
    s.spmv_grid = grid;
    s.spmv_grid_bytes = (int)sizeof(Real);
    return grid;
}

int spmm_grid(Scene &s, hipStream_t st, float *x, float *y, bool autotune, int force_tile) {
    if (force_tile > 0) {
        s.tile = force_tile;
        return batched_groups(s);
    }
    s.tile = default_tile(s.n_lambda);
    const int fallback = batched_groups(s);  // one node group per workgroup
    if (!autotune) return fallback;
    if (s.spmm_grid > 0) {
        s.tile = s.spmm_tile;
        return s.spmm_grid;
    }
    const TuneKey k{1, s.N, s.E, s.nnz, s.dmax, s.n_lambda, 4};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    auto it = g_tuned.find(k);
    Shape best = it != g_tuned.end() ? it->second : Shape{};
    if (!best.grid && s.solves < 2) return fallback;  // a scene's first solve does not tune
    if (!best.grid) {
        launch_fill_f32(x, (long long)s.E * s.n_lambda, st);  // x and y are scratch vectors here
        // the narrowest tile that holds the wavelengths, and the full wavefront
        std::vector<Shape> cands;
        for (int W : {smallest_tile(s.n_lambda), 64}) {
            if (!cands.empty() && cands.back().tile == W) break;
            s.tile = W;
            for (const Shape &c : grid_candidates(batched_groups(s), W)) cands.push_back(c);
        }
        best = time_candidates(st, cands, [&](const Shape &c) {
            s.tile = c.tile;
            launch_spmm(s, st, c.grid, nullptr, x, y, 1);
        });
        if (best.grid) store_cache_locked(k, best);
    }
    if (!best.grid || best.tile < smallest_tile(s.n_lambda)) best = Shape{fallback, default_tile(s.n_lambda)};
    s.spmm_grid = best.grid;
    s.spmm_tile = best.tile;
    s.tile = best.tile;
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

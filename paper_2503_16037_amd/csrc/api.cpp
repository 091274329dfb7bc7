// Host runtime of the library: the C ABI of sgrt.h, scene validation and
// device memory, and the solve orchestration (sweeps, FP64 residuals and
// iterative refinement, GMRES fallback, timing).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "internal.hpp"

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

namespace sg {

namespace {
thread_local std::string t_err;
}

void set_error(const std::string &msg) { t_err = msg; }
std::string t_last_error() { return t_err; }

namespace {
std::vector<unsigned (*)()> &bounds_readers() {
    static std::vector<unsigned (*)()> v;  // filled while the library loads
    return v;
}
}  // namespace

void register_bounds_reader(unsigned (*reader)()) { bounds_readers().push_back(reader); }

sg_status bounds_report() {
#ifdef SG_DEBUG_BOUNDS
    unsigned site = 0u;
    for (auto r : bounds_readers()) {
        const unsigned v = r();
        if (v && !site) site = v;
    }
    if (site) {
        char buf[96];
        std::snprintf(buf, sizeof(buf), "bounds check failed at site 0x%04x (the access was skipped)", site);
        set_error(buf);
        return SG_E_DEVICE;
    }
#endif
    return SG_OK;
}

namespace {

bool sg_log() {
    static const bool on = [] {
        const char *v = std::getenv("SG_LOG");
        return v && v[0] && v[0] != '0';
    }();
    return on;
}

sg_status fail(sg_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

sg_status device_fail(Ctx *ctx, const char *what, hipError_t e) {
    if (ctx) ctx->sticky.store(1);
    return fail(SG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define SG_HIP(call)                                                   \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) return device_fail(ctx, #call, e_);      \
    } while (0)


// Device allocation tracked against the context budget.
template <class T>
sg_status dalloc(Scene &s, T **p, size_t count) {
    Ctx *ctx = s.ctx;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    void *q = nullptr;
    const sg_status st = pool_alloc(ctx, bytes, &q);
    if (st != SG_OK) return st;
    *p = static_cast<T *>(q);
    s.bytes += pool_round(bytes);
    return SG_OK;
}

#define SG_TRY(x)                          \
    do {                                   \
        sg_status st_ = (x);               \
        if (st_ != SG_OK) return st_;      \
    } while (0)

// Fibonacci lattice, as the exact operation sequence z_i = 1 - (2i + 1) / N,
// phi_i = (i * pi (3 - sqrt 5)) mod 2 pi, p_i = (r cos phi_i, r sin phi_i, z_i),
// r = sqrt(1 - z_i z_i) (this file is compiled without FP contraction).
void host_lattice(int N, std::vector<double> &p) {
    p.resize(3 * (size_t)N);
    const double ga = M_PI * (3.0 - std::sqrt(5.0));
    const double two_pi = 2.0 * M_PI;
    for (int i = 0; i < N; ++i) {
        const double z = 1.0 - (2.0 * (double)i + 1.0) / (double)N;
        const double ph = std::fmod((double)i * ga, two_pi);
        const double r = std::sqrt(1.0 - z * z);
        p[3 * i] = r * std::cos(ph);
        p[3 * i + 1] = r * std::sin(ph);
        p[3 * i + 2] = z;
    }
}

// Per-component Henyey-Greenstein table normalised over the lattice, then the
// Lambertian cosine weights max(0, z_i) / sum_j max(0, z_j).
// Neighbour lists of the lattice along the edges of its convex hull (the adjacency the
// flood fill of the colouring mode walks): (i, j) is an edge when some k makes (i, j, k)
// a face, i.e. no lattice point lies strictly on both sides of the plane through the
// three (coplanar points do not count against it), tested as s_l = (n_x e_x + n_y e_y)
// + n_z e_z with n = (p_j - p_i) x (p_k - p_i), e = p_l - p_i; below 4 points every pair.
// nb [N][kHullNb] ascending and nnb [N]; false when a point has more neighbours.
bool host_hull(int N, const std::vector<double> &p, std::vector<int> &nb, std::vector<int> &nnb) {
    std::vector<unsigned char> adj((size_t)N * N, 0);
    if (N < 4) {
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) adj[(size_t)i * N + j] = i != j;
    } else {
        for (int i = 0; i < N; ++i)
            for (int j = i + 1; j < N; ++j)
                for (int k = j + 1; k < N; ++k) {
                    const double ax = p[3 * j] - p[3 * i], ay = p[3 * j + 1] - p[3 * i + 1], az = p[3 * j + 2] - p[3 * i + 2];
                    const double bx = p[3 * k] - p[3 * i], by = p[3 * k + 1] - p[3 * i + 1], bz = p[3 * k + 2] - p[3 * i + 2];
                    const double nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
                    bool above = false, below = false;
                    for (int l = 0; l < N && !(above && below); ++l) {
                        if (l == i || l == j || l == k) continue;
                        const double sl = (nx * (p[3 * l] - p[3 * i]) + ny * (p[3 * l + 1] - p[3 * i + 1])) +
                                          nz * (p[3 * l + 2] - p[3 * i + 2]);
                        above = above || sl > 0.0;
                        below = below || sl < 0.0;
                    }
                    if (above && below) continue;
                    for (auto e : {std::make_pair(i, j), std::make_pair(i, k), std::make_pair(j, k)}) {
                        adj[(size_t)e.first * N + e.second] = 1;
                        adj[(size_t)e.second * N + e.first] = 1;
                    }
                }
    }
    nb.assign((size_t)N * kHullNb, 0);
    nnb.assign(N, 0);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            if (adj[(size_t)i * N + j]) {
                if (nnb[i] == kHullNb) return false;
                nb[(size_t)i * kHullNb + nnb[i]++] = j;
            }
    return true;
}

// A phase table row at cos(theta) = mu: linear between the samples at -1 + 2 m / (n - 1)
// (unscaled).
double table_value(const double *row, int n, double mu) {
    const double x = (mu + 1.0) * (0.5 * (double)(n - 1));
    int m = (int)std::floor(x);
    m = m < 0 ? 0 : (m > n - 2 ? n - 2 : m);
    const double f = x - (double)m;
    return row[m] * (1.0 - f) + row[m + 1] * f;
}

// Integral over the sphere of a table row's interpolant: 2 pi x the trapezoid rule in mu
// (exact for the piecewise-linear interpolant).
double table_integral(const double *row, int n) {
    double sum = 0.0;
    for (int m = 0; m < n; ++m) sum += row[m];
    const double trap = sum - 0.5 * (row[0] + row[n - 1]);
    return (2.0 * M_PI) * ((2.0 / (double)(n - 1)) * trap);
}

// Lattice weights of every phase component (the value toward lattice point i, whose
// angle to the pole has cosine p_i,z, normalised to sum 1), then the Lambertian
// cosine weights.
void host_tables(int N, const std::vector<double> &p, int n_phase, const int *kind, const double *g,
                 const double *lut, int lut_n, std::vector<double> &t) {
    t.assign((size_t)(n_phase + 1) * N, 0.0);
    for (int k = 0; k < n_phase; ++k) {
        double s = 0.0;
        for (int i = 0; i < N; ++i) {
            const double mu = p[3 * i + 2];
            double v;
            if (kind[k] == SG_PHASE_RAYLEIGH) {
                v = 1.0 + mu * mu;
            } else if (kind[k] == SG_PHASE_TABLE) {
                v = table_value(lut + (size_t)k * lut_n, lut_n, mu);
            } else {
                const double den = 1.0 + g[k] * g[k] - 2.0 * g[k] * mu;
                v = (1.0 - g[k] * g[k]) / (4.0 * M_PI * den * std::sqrt(den));
            }
            t[(size_t)k * N + i] = v;
            s += v;
        }
        for (int i = 0; i < N; ++i) t[(size_t)k * N + i] = t[(size_t)k * N + i] / s;
    }
    double tot = 0.0;
    for (int i = 0; i < N; ++i) tot += std::max(0.0, p[3 * i + 2]);
    for (int i = 0; i < N; ++i) t[(size_t)n_phase * N + i] = std::max(0.0, p[3 * i + 2]) / tot;
}

void unit3(const int v[3], double u[3], double sign) {
    const long long x = v[0], y = v[1], z = v[2];
    const double n = std::sqrt((double)(x * x + y * y + z * z));
    u[0] = (double)(long long)(sign * x) / n;
    u[1] = (double)(long long)(sign * y) / n;
    u[2] = (double)(long long)(sign * z) / n;
}

// Host validation of large arrays: check(i) over [0, n) on up to 16 host threads, contiguous
// ranges; returns the smallest failing index and its message (nullptr: all hold), so the
// reported failure does not depend on the thread count.
struct FirstFailure {
    int64_t index;
    const char *why;
};
template <class F>
FirstFailure first_failure(int64_t n, F &&check) {
    const int64_t hw = std::max(1u, std::thread::hardware_concurrency());
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>({16, hw, n / 65536}));
    std::vector<FirstFailure> first(T, FirstFailure{n, nullptr});
    auto run = [&](int t) {
        const int64_t a = n * t / T, b = n * (t + 1) / T;
        for (int64_t i = a; i < b; ++i)
            if (const char *why = check(i)) {
                first[t] = FirstFailure{i, why};
                return;
            }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < T; ++t) th.emplace_back(run, t);
    run(0);
    for (auto &x : th) x.join();
    for (const auto &f : first)
        if (f.why) return f;  // ranges are in index order
    return FirstFailure{n, nullptr};
}

sg_status validate(const sg_scene_desc *d, int64_t &N, int64_t &E, int64_t &nnz, int &dmax) {
    if (!d) return fail(SG_E_INVALID, "desc is NULL");
    if (d->abi_version != SG_ABI_VERSION) return fail(SG_E_ABI, "scene desc abi_version mismatch");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1 || d->nx > 1024 || d->ny > 1024 || d->nz > 1024)
        return fail(SG_E_INVALID, "grid dimensions must be in 1..1024");
    if (!(d->voxel_m > 0.0) || !std::isfinite(d->voxel_m)) return fail(SG_E_INVALID, "voxel_m must be > 0");
    if (d->n_nodes < 0) return fail(SG_E_INVALID, "n_nodes must be >= 0");
    const bool general = d->n_nodes > 0;
    if (!d->mu_s || !d->mu_a || !(general ? d->node_pos_fx : d->vol_pos_fx) || !d->adj_ptr || !d->surf_albedo ||
        !d->hg_g)
        return fail(SG_E_INVALID, "a required array is NULL");
    if (general && !d->los_ptr) return fail(SG_E_INVALID, "general nodes need los_ptr");
    if (general && d->los_ptr[(int64_t)d->nx * d->ny] > 0 && (!d->los_node || !d->los_t))
        return fail(SG_E_INVALID, "general nodes need los_node and los_t");
    if (d->n_phase < 1 || d->n_phase > 4) return fail(SG_E_INVALID, "n_phase must be 1..4");
    if ((d->n_phase > 1) != (d->phase_frac != nullptr))
        return fail(SG_E_INVALID, "phase_frac must be given iff n_phase > 1");
    bool any_table = false;
    for (int k = 0; k < d->n_phase; ++k) {
        const int kind = d->phase_kind ? d->phase_kind[k] : SG_PHASE_HG;
        if (kind != SG_PHASE_HG && kind != SG_PHASE_RAYLEIGH && kind != SG_PHASE_TABLE)
            return fail(SG_E_INVALID, "phase_kind must be SG_PHASE_HG, SG_PHASE_RAYLEIGH or SG_PHASE_TABLE");
        if (kind == SG_PHASE_HG && !(std::fabs(d->hg_g[k]) < 1.0)) return fail(SG_E_INVALID, "|g| must be < 1");
        any_table = any_table || kind == SG_PHASE_TABLE;
    }
    if (any_table) {
        if (!d->phase_lut || d->phase_lut_n < 2 || d->phase_lut_n > 4096)
            return fail(SG_E_INVALID, "a table phase function needs phase_lut and phase_lut_n in 2..4096");
        for (int k = 0; k < d->n_phase; ++k) {
            if (d->phase_kind[k] != SG_PHASE_TABLE) continue;
            const double *row = d->phase_lut + (size_t)k * d->phase_lut_n;
            for (int m = 0; m < d->phase_lut_n; ++m)
                if (!(row[m] >= 0.0) || !std::isfinite(row[m]))
                    return fail(SG_E_INVALID, "phase_lut values must be finite and >= 0");
            if (!(table_integral(row, d->phase_lut_n) > 0.0)) return fail(SG_E_INVALID, "a phase_lut row is all zero");
        }
    }
    if (d->n_fib < 2 || d->n_fib > 128) return fail(SG_E_INVALID, "n_fib must be 2..128");
    if (d->sigma_mode != SG_SIGMA_VORONOI && d->sigma_mode != SG_SIGMA_COLOUR)
        return fail(SG_E_INVALID, "sigma_mode must be SG_SIGMA_VORONOI or SG_SIGMA_COLOUR");
    if (d->node_weight_mode != 0 && d->node_weight_mode != 1) return fail(SG_E_INVALID, "node_weight_mode must be 0 or 1");
    if (d->n_lambda < 1 || d->n_lambda > 256) return fail(SG_E_INVALID, "n_lambda must be 1..256");
    if (d->n_lambda > 1 && !d->abs_scale) return fail(SG_E_INVALID, "abs_scale required when n_lambda > 1");
    if (d->abs_scale)
        for (int k = 0; k < d->n_lambda; ++k)
            if (!(d->abs_scale[k] > 0.0f) || !std::isfinite(d->abs_scale[k]))
                return fail(SG_E_INVALID, "abs_scale must be finite and > 0");
    for (const int32_t *v : {d->sun_dir, d->view_dir}) {
        if (v[2] <= 0) return fail(SG_E_INVALID, "sun_dir and view_dir need a positive z component");
        for (int k = 0; k < 3; ++k)
            if (std::abs((long long)v[k]) > (1LL << 22)) return fail(SG_E_INVALID, "direction components must be <= 2^22");
    }
    const int64_t nvox = (int64_t)d->nx * d->ny * d->nz;
    const int64_t nvol = general ? (int64_t)d->n_nodes : nvox;
    N = nvol + (d->surface_nodes ? (int64_t)d->nx * d->ny : 0);
    {
        const FirstFailure f = first_failure(nvox, [&](int64_t v) -> const char * {
            const float a = d->mu_s[v], b = d->mu_a[v];
            return (!(a >= 0.0f) || !(b >= 0.0f) || !std::isfinite(a) || !std::isfinite(b))
                       ? "mu_s and mu_a must be finite and >= 0"
                       : nullptr;
        });
        if (f.why) return fail(SG_E_INVALID, f.why);
    }
    if (d->phase_frac) {
        const FirstFailure f = first_failure(nvox * d->n_phase, [&](int64_t v) -> const char * {
            return (!(d->phase_frac[v] >= 0.0f) || !(d->phase_frac[v] <= 1.0f)) ? "phase_frac must be in [0, 1]"
                                                                                  : nullptr;
        });
        if (f.why) return fail(SG_E_INVALID, f.why);
    }
    for (int64_t v = 0; v < (int64_t)d->nx * d->ny; ++v)
        if (!(d->surf_albedo[v] >= 0.0f) || !(d->surf_albedo[v] <= 1.0f))
            return fail(SG_E_INVALID, "surf_albedo must be in [0, 1]");
    if (!general) {
        const FirstFailure f = first_failure(nvox, [&](int64_t v) -> const char * {
            const int64_t ix = v % d->nx, iy = (v / d->nx) % d->ny, iz = v / ((int64_t)d->nx * d->ny);
            const int64_t p[3] = {d->vol_pos_fx[3 * v], d->vol_pos_fx[3 * v + 1], d->vol_pos_fx[3 * v + 2]};
            const int64_t c[3] = {ix, iy, iz};
            for (int k = 0; k < 3; ++k)
                if (!(p[k] > c[k] * 65536 && p[k] < (c[k] + 1) * 65536)) return "node position not strictly inside its voxel";
            return nullptr;
        });
        if (f.why) return fail(SG_E_INVALID, std::string(f.why) + " (node " + std::to_string(f.index) + ")");
    } else {
        const int64_t W[3] = {(int64_t)d->nx * 65536, (int64_t)d->ny * 65536, (int64_t)d->nz * 65536};
        const FirstFailure f = first_failure(nvol, [&](int64_t l) -> const char * {
            for (int k = 0; k < 3; ++k) {
                const int64_t c = d->node_pos_fx[3 * l + k];
                const bool per = k < 2 && (d->periodic >> k & 1);
                if (per ? !(c >= 0 && c < W[k]) : !(c > 0 && c < W[k])) return "general node outside the box";
            }
            return nullptr;
        });
        if (f.why) return fail(SG_E_INVALID, std::string(f.why) + " (node " + std::to_string(f.index) + ")");
        const int64_t npx = (int64_t)d->nx * d->ny;
        if (d->los_ptr[0] != 0) return fail(SG_E_INVALID, "los_ptr[0] must be 0");
        for (int64_t p = 0; p < npx; ++p) {
            if (d->los_ptr[p + 1] < d->los_ptr[p]) return fail(SG_E_INVALID, "los_ptr must be non-decreasing");
            double prev = 0.0;
            for (int64_t e = d->los_ptr[p]; e < d->los_ptr[p + 1]; ++e) {
                if (!(d->los_t[e] > prev) || !std::isfinite(d->los_t[e]))
                    return fail(SG_E_INVALID, "los_t must be finite and strictly increasing from 0 (pixel " +
                                                  std::to_string(p) + ")");
                if (d->los_node[e] < -1 || d->los_node[e] >= nvol)
                    return fail(SG_E_INVALID, "los_node out of range (pixel " + std::to_string(p) + ")");
                prev = d->los_t[e];
            }
        }
    }
    const int64_t *ap = d->adj_ptr;
    if (ap[0] != 0) return fail(SG_E_INVALID, "adj_ptr[0] must be 0");
    for (int64_t l = 0; l < N; ++l)
        if (ap[l + 1] < ap[l]) return fail(SG_E_INVALID, "adj_ptr must be non-decreasing");
    E = ap[N];
    if (E >= (1LL << 31) - 1) return fail(SG_E_INVALID, "too many edges");
    if (E > 0 && !d->adj_idx) return fail(SG_E_INVALID, "adj_idx is NULL");
    nnz = 0;
    dmax = 0;
    const bool wave_only = d->n_lambda > 1;
    const int64_t deg_cap = wave_only ? kMaxWaveDegree : kMaxDegree;
    for (int64_t l = 0; l < N; ++l) {
        const int64_t deg = ap[l + 1] - ap[l];
        if (deg > deg_cap)
            return fail(SG_E_INVALID, "node degree above " + std::to_string(deg_cap) + " (node " + std::to_string(l) +
                                          (wave_only ? "; several wavelengths allow 64)" : ")"));
        dmax = std::max<int>(dmax, (int)deg);
        nnz += deg * deg;
    }
    {  // symmetry is checked on the device once the adjacency is uploaded
        const FirstFailure f = first_failure(N, [&](int64_t l) -> const char * {
            for (int64_t e = ap[l]; e < ap[l + 1]; ++e) {
                const int64_t j = d->adj_idx[e];
                if (j < 0 || j >= N) return "adjacency head out of range";
                if (j == l) return "self loop";
                if (e > ap[l] && d->adj_idx[e - 1] >= j) return "adjacency rows must be strictly ascending";
                if (l >= nvol && j >= nvol) return "surface-surface pair";
            }
            return nullptr;
        });
        if (f.why) return fail(SG_E_INVALID, f.why);
    }
    if (d->periodic & ~(SG_PERIODIC_X | SG_PERIODIC_Y))
        return fail(SG_E_INVALID, "periodic must combine SG_PERIODIC_X and SG_PERIODIC_Y");
    if (d->periodic) {
        // a ray from height z crosses at most nz z-planes and nz |d_x| / d_z + 1 x-planes
        // (y alike): this bound keeps every sun and view walk within the walk's limit
        for (const int32_t *v : {d->sun_dir, d->view_dir}) {
            const long long ax = std::llabs((long long)v[0]), ay = std::llabs((long long)v[1]), az = v[2];
            if ((long long)d->nz * (ax + ay + az) + 4 * az > 65536LL * az)
                return fail(SG_E_INVALID, "with periodic axes the sun and view rays must reach the top within 65536 voxels");
        }
        const auto coord = [&](int64_t l, int k) -> long long {
            if (l < nvol) return general ? d->node_pos_fx[3 * l + k] : d->vol_pos_fx[3 * l + k];
            const int64_t c = l - nvol;  // surface node: the column's centre
            return (k == 0 ? c % d->nx : c / d->nx) * 65536LL + 32768;
        };
        const long long W[2] = {(long long)d->nx * 65536, (long long)d->ny * 65536};
        const FirstFailure f = first_failure(N, [&](int64_t l) -> const char * {
            for (int64_t e = ap[l]; e < ap[l + 1]; ++e)
                for (int k = 0; k < 2; ++k)
                    if ((d->periodic >> k & 1) && 2 * std::llabs(coord(d->adj_idx[e], k) - coord(l, k)) == W[k])
                        return "a coupled pair is exactly half a period apart";
            return nullptr;
        });
        if (f.why) return fail(SG_E_INVALID, std::string(f.why) + " (node " + std::to_string(f.index) + ")");
    }
    return SG_OK;
}

void fill_default_opts(sg_solve_opts &o) {
    std::memset(&o, 0, sizeof(o));
    o.abi_version = SG_ABI_VERSION;
}

// Launch policy and HIP-event timing of one solve.  With timing on, sweeps are
// launched one by one with an event pair around each sweep kernel; otherwise
// chunks of sweeps replay captured graphs (unless disabled).
struct Exec {
    bool on = false;
    bool graphs = true, autotune = true;
    hipStream_t st = nullptr;
    std::vector<hipEvent_t> ev;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> spmv;
    int monitored = 0;  // timed sweeps that computed the convergence measures
    hipEvent_t fresh() {  // an event for a launcher to record
        hipEvent_t e = nullptr;
        if (!on) return e;
        (void)hipEventCreate(&e);
        ev.push_back(e);
        return e;
    }
    hipEvent_t mark() {
        hipEvent_t e = fresh();
        if (e) (void)hipEventRecord(e, st);
        return e;
    }
    ~Exec() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    double between(hipEvent_t a, hipEvent_t b) {
        if (!a || !b) return 0.0;
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, a, b);
        return (double)ms;
    }
};

template <class Real>
sg_status ensure_real(Scene &s) {
    const int rb = (int)sizeof(Real);
    if (s.real_bytes == rb) return SG_OK;
    Ctx *ctx = s.ctx;
    auto drop = [&](void *&p, size_t n) {
        if (p) {
            pool_free(ctx, p);
            s.bytes -= pool_round(n);
            p = nullptr;
        }
    };
    if (s.real_bytes) {
        clear_graphs(s);  // captured chunks hold the old buffers
        const size_t ob = (size_t)s.real_bytes;
        drop(s.tau_s, s.E * ob); drop(s.tau_a, s.E * ob); drop(s.T, s.E * ob);
        drop(s.tsun_s, s.N * ob); drop(s.tsun_a, s.N * ob); drop(s.Tsun, s.N * ob); drop(s.rho, s.N * ob);
        drop(s.val, s.nnz * ob); drop(s.S, s.E * ob); drop(s.x, s.E * ob); drop(s.y, s.E * ob);
        drop(s.c_rhs, s.E * ob); drop(s.c_a, s.E * ob); drop(s.c_b, s.E * ob);
        s.real_bytes = 0;
    }
    Real *p;
    SG_TRY(dalloc(s, &p, s.E)); s.tau_s = p;
    SG_TRY(dalloc(s, &p, s.E)); s.tau_a = p;
    SG_TRY(dalloc(s, &p, s.E)); s.T = p;
    SG_TRY(dalloc(s, &p, s.N)); s.tsun_s = p;
    SG_TRY(dalloc(s, &p, s.N)); s.tsun_a = p;
    SG_TRY(dalloc(s, &p, s.N)); s.Tsun = p;
    SG_TRY(dalloc(s, &p, s.N)); s.rho = p;
    SG_TRY(dalloc(s, &p, (size_t)s.nnz)); s.val = p;
    SG_TRY(dalloc(s, &p, s.E)); s.S = p;
    SG_TRY(dalloc(s, &p, s.E)); s.x = p;
    SG_TRY(dalloc(s, &p, s.E)); s.y = p;
    SG_TRY(dalloc(s, &p, s.E)); s.c_rhs = p;
    SG_TRY(dalloc(s, &p, s.E)); s.c_a = p;
    SG_TRY(dalloc(s, &p, s.E)); s.c_b = p;
    s.real_bytes = rb;
    return SG_OK;
}

// Read n doubles of device scalars after the stream drains.
// Pinned host staging for the convergence scalars, one buffer per host thread (a thread runs
// one solve at a time): a copy into pageable memory would go through a bounce buffer and
// lengthen every host round trip of the solve policy.
struct PinnedScalars {
    double *p = nullptr;
    size_t n = 0;
    ~PinnedScalars() {
        if (p) (void)hipHostFree(p);
    }
};

sg_status read_scalars(Scene &s, hipStream_t st, const double *dev, double *host, int n) {
    Ctx *ctx = s.ctx;
    thread_local PinnedScalars buf;
    if (buf.n < (size_t)n) {
        if (buf.p) (void)hipHostFree(buf.p);
        buf.p = nullptr;
        buf.n = 0;
        const size_t want = std::max<size_t>((size_t)n, 1024);
        SG_HIP(hipHostMalloc((void **)&buf.p, sizeof(double) * want, hipHostMallocDefault));
        buf.n = want;
    }
    SG_HIP(hipMemcpyAsync(buf.p, dev, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    SG_HIP(hipStreamSynchronize(st));
    std::memcpy(host, buf.p, sizeof(double) * n);
    return SG_OK;
}

// The warm start [n_lambda][E] into x64 ([E] for one wavelength, [E][n_lambda] for
// several; staged through r64, which the first residual overwrites).
sg_status load_warm_start(Scene &s, const sg_solve_opts &o, hipStream_t st) {
    Ctx *ctx = s.ctx;
    const size_t n = (size_t)s.E * s.n_lambda;
    if (!o.warm_start_on_device)
        for (size_t k = 0; k < n; ++k)
            if (!std::isfinite(o.warm_start[k])) return fail(SG_E_INVALID, "warm_start values must be finite");
    const hipMemcpyKind kind = o.warm_start_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    double *dst = s.n_lambda > 1 ? s.r64 : s.x64;
    SG_HIP(hipMemcpyAsync(dst, o.warm_start, sizeof(double) * n, kind, st));
    if (s.n_lambda > 1) launch_lam_to_edge_major(s.r64, s.x64, s.n_lambda, s.E, st);
    return SG_OK;
}

// Stop of a correction solve (I - K) d = r, as the L1 update relative to the first one.
// 1e-5 in general; the first two corrections of a warm start, whose residual rel may be
// far below 1, only need d to about 0.1 rtol / rel (never coarser than 1e-2): the per-edge
// FP64 residual that follows decides convergence either way.
inline double correction_stop(bool warm, int it, double rel, double rtol) {
    if (!warm || it >= 2 || !(rel > 0)) return 1e-5;
    return std::min(1e-2, std::max(1e-5, 0.1 * rtol / rel));
}

// A warm start is kept only if it is better than phi = 0: its per-edge relative residual
// max |r_e| / |phi_e| must be at most 1/2 (and finite), else the solve starts cold.  The
// correction right-hand side r / rel is then at most |phi| per edge, inside the FP32 range.
constexpr double kWarmKeep = 0.5;

struct SolveStats {
    int sweeps = 0, refinements = 0, gmres_used = 0, converged = 0;
    double rel = 0.0;
};

// FP32/FP64 Neumann sweeps x <- rhs + K x from x = 0.  Every sweep yields two measures
// of its update dx: the L1 norm, which shrinks at least by the factor max_a T_a rho < 1
// per sweep and so gives the sweep ratio q, and the largest per-edge relative update
// max |dx_e| / |x_e|, which bounds the error of every edge, bright or deep in shadow.
// relative != 0: stop once the relative measure is (predicted) below stop; otherwise
// once the L1 update is below stop times the first one (sum |rhs|).  A ratio q >= 0.95
// or growth after three sweeps, with the relative measure not falling either, is a
// stall (stalled = 1); a measure that is not finite (the iterate overflowed) sets
// stalled = 2.  The solution ends in xa.
template <class Real>
sg_status neumann(Scene &s, hipStream_t st, Exec &tm, const Real *rhs, Real *&xa, Real *&xb, int relative,
                  double stop, int max_sweeps, SolveStats &ss, int &stalled) {
    Ctx *ctx = s.ctx;
    const int grid = spmv_grid<Real>(s, st, rhs, xa, xb, tm.autotune);
    std::vector<double> l1, rel;  // measures of consecutive monitored sweeps
    int chunk = 2, first = 1;
    stalled = 0;
    double host[64];
    double *meas = s.scal + 128;  // [32][2] measures of the chunk's sweeps
    while (true) {
        chunk = std::max(1, std::min(chunk, 32));
        // only the sweeps whose measures are read (the first one, and the last two of
        // each chunk) compute them
        const int c_mon = std::max(0, chunk - 2);
        auto out = [&](int c) { return (first && c == 0) || c >= c_mon ? meas + 2 * c : nullptr; };
        // the first iterate from x = 0 is rhs itself: a copy instead of a sweep
        const int n_copy = first ? 1 : 0;
        if (tm.on) {
            for (int c = 0; c < chunk; ++c) {
                if (c < n_copy) {
                    launch_first<Real>(s, st, rhs, xb, out(c));
                } else {
                    hipEvent_t e0 = tm.mark(), e1 = tm.fresh();
                    launch_spmv<Real>(s, st, rhs, xa, xb, out(c), grid, e1);
                    tm.spmv.push_back({e0, e1});
                    tm.monitored += out(c) != nullptr;
                }
                std::swap(xa, xb);
            }
        } else {
            const GraphKey key{1, (uintptr_t)chunk, (uintptr_t)rhs, (uintptr_t)xa, (uintptr_t)xb, (uintptr_t)grid,
                               sizeof(Real), (uintptr_t)first};
            Real *a0 = xa, *b0 = xb;
            SG_TRY(run_chunk(s, st, key, tm.graphs, [&]() {
                Real *a = a0, *b = b0;
                for (int c = 0; c < chunk; ++c) {
                    if (c < n_copy) launch_first<Real>(s, st, rhs, b, out(c));
                    else launch_spmv<Real>(s, st, rhs, a, b, out(c), grid, nullptr);
                    std::swap(a, b);
                }
            }));
            if (chunk & 1) std::swap(xa, xb);
        }
        ss.sweeps += chunk - n_copy;
        SG_HIP(hipGetLastError());
        SG_TRY(read_scalars(s, st, meas, host, 2 * chunk));
        // the first chunk (two sweeps) is monitored whole; later ones in their last two
        for (int c = first ? 0 : c_mon; c < chunk; ++c) {
            l1.push_back(host[2 * c]);
            rel.push_back(host[2 * c + 1]);
        }
        if (first && !relative) stop *= host[0];  // first sweep from 0: sum |rhs|
        first = 0;
        const size_t k = l1.size();
        const double r = relative ? rel.back() : l1.back();
        if (sg_log())
            fprintf(stderr, "[sgrt] sweeps %d chunk %d: L1 update %.3e, max relative %.3e (stop %.3e)\n", ss.sweeps,
                    chunk, l1.back(), rel.back(), stop);
        if (!std::isfinite(l1.back()) || !std::isfinite(rel.back())) { stalled = 2; break; }
        const double q = k >= 2 && l1[k - 2] > 0 ? l1.back() / l1[k - 2] : 0.5;
        // the measured update belongs to the previous iterate; the current one's is about q r
        const double qr = relative && k >= 2 && rel[k - 2] > 0 ? std::max(q, rel.back() / rel[k - 2]) : q;
        if (r <= stop || (k >= 2 && qr < 0.9 && qr * r <= 0.5 * stop)) break;
        if (ss.sweeps >= max_sweeps) break;
        // a stall: neither measure still falls (the L1 update alone flattens once it
        // reaches rounding while dark edges still converge)
        const double q2 = k >= 2 && rel[k - 2] > 0 ? rel.back() / rel[k - 2] : 0.0;
        if (k >= 3 && q >= 0.95 && (!relative || q2 >= 0.95)) { stalled = 1; break; }
        // sweeps still needed at the asymptotic rate: the smaller ratio (the relative one is
        // near 1 until light has reached the dark edges, the L1 one once it hits rounding)
        const double qa = relative && q2 > 0 ? std::min(q, q2) : q;
        const double qc = std::min(std::max(qa, 1e-12), 0.95);
        chunk = (int)std::ceil(std::max(1.0, std::log(stop / r) / std::log(qc)));
    }
    return SG_OK;
}

// GMRES basis of a scene: m + 1 Krylov vectors of E doubles; a batched scene also holds one
// wavelength's iterate and residual there (two more)
size_t gmres_len(const Scene &s, int m) { return (size_t)(m + 1 + (s.n_lambda > 1 ? 2 : 0)) * (size_t)s.E; }

sg_status gmres_basis(Scene &s, int m) {
    Ctx *ctx = s.ctx;
    if (s.gm_V && s.gm_m >= m) return SG_OK;
    if (s.gm_V) {
        pool_free(ctx, s.gm_V);
        s.bytes -= pool_round(gmres_len(s, s.gm_m) * sizeof(double));
        s.gm_V = nullptr;
    }
    const sg_status st_v = dalloc(s, &s.gm_V, gmres_len(s, m));
    s.gm_nomem = st_v == SG_E_NOMEM;
    if (st_v != SG_OK) return st_v;
    s.gm_m = m;
    return SG_OK;
}

// Restarted GMRES(m) in FP64 on (I - K) x = S for one right-hand side of length E: x is the
// iterate (updated in place), r its residual, V the m + 1 basis vectors.  residual(m2)
// computes r = S - (I - K) x and reads its measures (sum |r|, max |r| / (|x| + floor));
// apply(v, w) computes w = (I - K) v.  Stops at max |r| / |x| <= rtol or after max_sweeps.
template <class Residual, class Apply>
sg_status gmres_core(Scene &s, hipStream_t st, double rtol, int m, int max_sweeps, int64_t E, double *x, double *r,
                     double *V, Residual residual, Apply apply, SolveStats &ss) {
    Ctx *ctx = s.ctx;
    ss.gmres_used = 1;
    const int nbv = 1024;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), yv(m), h(m + 1), h2(m + 1);
    while (true) {
        double m2[2];
        SG_TRY(residual(m2));
        ++ss.sweeps;
        ++ss.refinements;
        ss.rel = std::isfinite(m2[0]) ? m2[1] : HUGE_VAL;  // max over edges of |r| / |x|
        if (ss.rel <= rtol || ss.sweeps >= max_sweeps) break;
        launch_dot_multi(r, E, 1, r, E, s.partial, nbv, s.scal, st);
        double beta2;
        SG_TRY(read_scalars(s, st, s.scal, &beta2, 1));
        const double beta = std::sqrt(beta2);
        if (!std::isfinite(beta)) break;  // a non-finite iterate: reported as not converged
        SG_HIP(hipMemcpyAsync(V, r, sizeof(double) * E, hipMemcpyDeviceToDevice, st));
        launch_scale64(V, 1.0 / beta, E, st);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        bool bad = false;  // a non-finite Krylov vector (e.g. K holds infinities): stop after this cycle
        for (; k < m && ss.sweeps < max_sweeps; ++k) {
            double *vk = V + (size_t)k * E, *w = V + (size_t)(k + 1) * E;
            apply(vk, w);
            ++ss.sweeps;
            // classical Gram-Schmidt, twice
            launch_dot_multi(V, E, k + 1, w, E, s.partial, nbv, s.scal, st);
            SG_TRY(read_scalars(s, st, s.scal, h.data(), k + 1));
            SG_HIP(hipMemcpyAsync(s.scal + 64, h.data(), sizeof(double) * (k + 1), hipMemcpyHostToDevice, st));
            launch_axpy_multi(w, V, E, k + 1, s.scal + 64, E, st);
            launch_dot_multi(V, E, k + 1, w, E, s.partial, nbv, s.scal, st);
            SG_TRY(read_scalars(s, st, s.scal, h2.data(), k + 1));
            SG_HIP(hipMemcpyAsync(s.scal + 64, h2.data(), sizeof(double) * (k + 1), hipMemcpyHostToDevice, st));
            launch_axpy_multi(w, V, E, k + 1, s.scal + 64, E, st);
            for (int j = 0; j <= k; ++j) h[j] += h2[j];
            launch_dot_multi(w, E, 1, w, E, s.partial, nbv, s.scal, st);
            double hn2;
            SG_TRY(read_scalars(s, st, s.scal, &hn2, 1));
            const double hn = std::sqrt(std::max(hn2, 0.0));
            if (!std::isfinite(hn)) { bad = true; break; }
            if (hn > 0) launch_scale64(w, 1.0 / hn, E, st);
            for (int j = 0; j <= k; ++j) H[(size_t)j * m + k] = h[j];
            H[(size_t)(k + 1) * m + k] = hn;
            for (int j = 0; j < k; ++j) {
                const double a = H[(size_t)j * m + k], b = H[(size_t)(j + 1) * m + k];
                H[(size_t)j * m + k] = cs[j] * a + sn[j] * b;
                H[(size_t)(j + 1) * m + k] = -sn[j] * a + cs[j] * b;
            }
            const double a = H[(size_t)k * m + k], b = H[(size_t)(k + 1) * m + k];
            const double den = std::sqrt(a * a + b * b);
            cs[k] = den > 0 ? a / den : 1.0;
            sn[k] = den > 0 ? b / den : 0.0;
            H[(size_t)k * m + k] = den;
            H[(size_t)(k + 1) * m + k] = 0.0;
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            if (std::fabs(g[k + 1]) <= 1e-3 * rtol * beta || hn == 0.0) { ++k; break; }
        }
        for (int j = k - 1; j >= 0; --j) {
            double acc = g[j];
            for (int q = j + 1; q < k; ++q) acc -= H[(size_t)j * m + q] * yv[q];
            yv[j] = acc / H[(size_t)j * m + j];
        }
        // x += V y  (axpy_multi subtracts, so pass -y)
        std::vector<double> ny(k);
        for (int j = 0; j < k; ++j) ny[j] = -yv[j];
        SG_HIP(hipMemcpyAsync(s.scal + 64, ny.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
        launch_axpy_multi(x, V, E, k, s.scal + 64, E, st);
        SG_HIP(hipStreamSynchronize(st));
        if (bad) break;
    }
    ss.converged = ss.rel <= rtol;
    return SG_OK;
}

template <class Real>
sg_status gmres64(Scene &s, hipStream_t st, Exec &tm, const Real *S, double rtol, int m, int max_sweeps,
                  SolveStats &ss) {
    (void)tm;
    SG_TRY(gmres_basis(s, m));
    return gmres_core(
        s, st, rtol, m, max_sweeps, s.E, s.x64, s.r64, s.gm_V,
        [&](double *m2) {
            launch_residual64<Real>(s, st, S, s.x64, s.r64, s.scal);
            return read_scalars(s, st, s.scal, m2, 2);
        },
        [&](const double *v, double *w) { launch_apply_imk64<Real>(s, st, v, w); }, ss);
}

// GMRES fallback of a batched scene: each wavelength whose relative residual rel[k] is above
// rtol is solved on its own, in FP64 with the batched matrix at that wavelength, from its
// current iterate (from zero when that iterate is not finite); rel[k] is updated.  Each
// wavelength gets its own budget of max_sweeps.
sg_status gmres_batched(Scene &s, hipStream_t st, double rtol, int m, int max_sweeps, std::vector<double> &rel,
                        SolveStats &ss) {
    const int nl = s.n_lambda;
    const int64_t E = s.E;
    SG_TRY(gmres_basis(s, m));
    double *V = s.gm_V, *xl = s.gm_V + (size_t)(m + 1) * E, *rl = xl + E;
    bool all = true;
    for (int k = 0; k < nl; ++k) {
        if (rel[k] <= rtol) continue;
        if (std::isfinite(rel[k])) launch_lam_take64(s.x64, nl, k, E, xl, st);
        else launch_fill<double>(xl, 0.0, E, st);
        SolveStats ls;
        SG_TRY(gmres_core(
            s, st, rtol, m, max_sweeps, E, xl, rl, V,
            [&](double *m2) {
                launch_blam_residual64(s, st, k, xl, rl);
                return read_scalars(s, st, s.scal, m2, 2);
            },
            [&](const double *v, double *w) { launch_blam_apply64(s, st, k, v, w); }, ls));
        launch_lam_put64(xl, nl, k, E, s.x64, st);
        rel[k] = ls.rel;
        ss.sweeps += ls.sweeps;
        ss.refinements += ls.refinements;
        all = all && ls.converged;
        if (sg_log())
            fprintf(stderr, "[sgrt] batched GMRES, wavelength %d: relative residual %.3e after %d sweeps\n", k, ls.rel,
                    ls.sweeps);
    }
    ss.gmres_used = 1;
    ss.converged = all;
    return SG_OK;
}

template <class Real>
sg_status solve_linear(Scene &s, const sg_solve_opts &o, hipStream_t st, Exec &tm, SolveStats &ss) {
    Ctx *ctx = s.ctx;
    const int64_t E = s.E;
    const double rtol = o.rtol > 0 ? o.rtol : (sizeof(Real) == 4 ? 1e-6 : 1e-12);
    const int max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : 2000;
    const int m = o.gmres_restart > 0 ? std::min(std::max(o.gmres_restart, 2), 64) : 32;
    Real *S = (Real *)s.S;
    // a zero source needs no special case: every measure is zero from the first sweep
    launch_fill<double>(s.x64, 0.0, E, st);
    int use_gmres = o.solver == SG_SOLVER_GMRES;
    bool warm = false, have_r = false;
    if (o.warm_start) {
        SG_TRY(load_warm_start(s, o, st));
        launch_residual64<Real>(s, st, S, s.x64, s.r64, s.scal);
        ++ss.sweeps;
        ++ss.refinements;
        double m2[2];
        SG_TRY(read_scalars(s, st, s.scal, m2, 2));
        ss.rel = m2[1];
        warm = have_r = ss.rel <= kWarmKeep;
        if (!warm) launch_fill<double>(s.x64, 0.0, E, st);
    }
    // an iterate that overflowed (a Neumann series that diverges fast, e.g. with the literal
    // node weight) leaves x64 non-finite: GMRES then starts from x = 0
    bool nonfinite = false;
    if (!use_gmres) {
        Real *xa = (Real *)s.x, *xb = (Real *)s.y;
        int stalled = 0;
        // per-edge relative updates settle at a few units of rounding: never ask for less
        const double floor_rel = sizeof(Real) == 4 ? 4e-6 : 1e-14;
        if (!warm) {  // a kept warm start goes straight to the refinement below
            SG_TRY(neumann<Real>(s, st, tm, S, xa, xb, 1, std::max(0.3 * rtol, floor_rel), max_sweeps, ss, stalled));
            launch_to64<Real>(xa, s.x64, E, st);
            nonfinite = stalled == 2;
        }
        if (stalled && o.solver == SG_SOLVER_AUTO) use_gmres = 1;
        // FP64 residual and iterative refinement
        for (int it = 0; !use_gmres && it < 12; ++it) {
            if (!have_r) {
                launch_residual64<Real>(s, st, S, s.x64, s.r64, s.scal);
                ++ss.sweeps;
                ++ss.refinements;
                double m2[2];
                SG_TRY(read_scalars(s, st, s.scal, m2, 2));
                ss.rel = std::isfinite(m2[0]) ? m2[1] : HUGE_VAL;  // max over edges of |r| / |x|
            }
            have_r = false;
            if (sg_log()) fprintf(stderr, "[sgrt] FP64 residual after %d sweeps: %.3e\n", ss.sweeps, ss.rel);
            if (ss.rel <= rtol) { ss.converged = 1; break; }
            if (!std::isfinite(ss.rel)) {
                nonfinite = true;
                if (o.solver == SG_SOLVER_AUTO) use_gmres = 1;
                break;
            }
            if (ss.sweeps >= max_sweeps) break;
            // correction (I - K) d = r by sweeps in the working precision; r / rel is at most
            // |x| per edge, which keeps it well inside the FP32 range
            const double sc = 1.0 / ss.rel;
            Real *crhs = (Real *)s.c_rhs, *c0 = (Real *)s.c_a, *c1 = (Real *)s.c_b;
            launch_scaled_to_real<Real>(s.r64, sc, crhs, E, st);
            int stalled2 = 0;
            SG_TRY(neumann<Real>(s, st, tm, crhs, c0, c1, 0, std::max(correction_stop(warm, it, ss.rel, rtol), floor_rel),
                                 max_sweeps, ss, stalled2));
            // a correction that overflowed is dropped (x64 stays the last finite iterate)
            if (stalled2 != 2) launch_axpy_real_to64<Real>(s.x64, c0, 1.0 / sc, E, st);
            if (stalled2 && o.solver == SG_SOLVER_AUTO) use_gmres = 1;
        }
    }
    if (use_gmres && nonfinite) launch_fill<double>(s.x64, 0.0, E, st);
    if (use_gmres) SG_TRY(gmres64<Real>(s, st, tm, S, rtol, m, max_sweeps, ss));
    SG_HIP(hipGetLastError());
    return SG_OK;
}

// The sun march (scale: the absorption multiplier) on the scene's second stream, ordered
// after everything already queued on st (the previous solve's readers of the sun's optical
// depths included); st waits for ev_join before this solve's first reader.  It needs only
// the positions and the extinction grids, so it runs beside the structure pass and the edge
// march.
template <class Real>
sg_status fork_sun_march(Scene &s, hipStream_t st, float scale) {
    Ctx *ctx = s.ctx;
    SG_HIP(hipEventRecord(s.ev_fork, st));
    SG_HIP(hipStreamWaitEvent(s.aux, s.ev_fork, 0));
    launch_march_sun<Real>(s, s.aux, scale);
    SG_HIP(hipEventRecord(s.ev_join, s.aux));
    return SG_OK;
}

template <class Real>
sg_status solve_single(Scene &s, const sg_solve_opts &o, hipStream_t st, double *radiance, int on_dev,
                       sg_solve_info *info) {
    Ctx *ctx = s.ctx;
    SG_TRY(ensure_real<Real>(s));
    Exec tm;
    tm.on = o.timing != 0;
    tm.graphs = !(o.flags & SG_NO_GRAPHS) && !tm.on;
    tm.autotune = !(o.flags & SG_NO_AUTOTUNE);
    s.qscreen = (o.flags & SG_EXACT_CELLS) ? 0 : 1;
    s.phi32 = nullptr;
    tm.st = st;
    const float scale = s.abs_scale.empty() ? 1.0f : s.abs_scale[0];
    if (o.build_col_idx && !s.col_idx) SG_TRY(dalloc(s, &s.col_idx, (size_t)s.nnz));
    SG_TRY(fork_sun_march<Real>(s, st, scale));
    hipEvent_t e0 = tm.mark();
    launch_structure(s, st);
    if (o.build_col_idx) {
        launch_col_idx(s, st);
        s.col_built = true;
    } else {
        s.col_built = false;
    }
    hipEvent_t e1 = tm.mark();
    launch_march_edges<Real>(s, st, scale, 1);
    launch_node_weights<Real>(s, st, scale);
    hipEvent_t e2 = tm.mark();
    SG_HIP(hipStreamWaitEvent(st, s.ev_join, 0));  // the sun march
    launch_qbuild<Real>(s, st, 0);
    hipEvent_t e3 = tm.mark();
    SG_HIP(hipGetLastError());
    SolveStats ss;
    if (o.scatter_order == 1) {
        launch_fill<double>(s.x64, 0.0, s.E, st);
        ss.converged = 1;
    } else {
        SG_TRY(solve_linear<Real>(s, o, st, tm, ss));
    }
    hipEvent_t e4 = tm.mark();
    double *dst = on_dev ? radiance : s.pix;
    launch_gather<Real>(s, st, s.x64, o.scatter_order, dst);
    hipEvent_t e5 = tm.mark();
    SG_HIP(hipGetLastError());
    if (!on_dev) {
        SG_HIP(hipMemcpyAsync(radiance, dst, sizeof(double) * s.npx, hipMemcpyDeviceToHost, st));
    }
    SG_HIP(hipStreamSynchronize(st));
    s.solved = true;
    s.last_precision = sizeof(Real) == 4 ? SG_FP32 : SG_FP64;
    s.last_scatter_order = o.scatter_order;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->converged = ss.converged;
        info->sweeps = ss.sweeps;
        info->gmres_used = ss.gmres_used;
        info->refinements = ss.refinements;
        info->rel_residual = ss.rel;
        info->n_nodes = s.N;
        info->n_edges = s.E;
        info->nnz = s.nnz;
        if (tm.on) {
            info->ms_structure = tm.between(e0, e1);
            info->ms_march = tm.between(e1, e2);
            info->ms_qbuild = tm.between(e2, e3);
            info->ms_solve = tm.between(e3, e4);
            info->ms_gather = tm.between(e4, e5);
            info->ms_total = tm.between(e0, e5);
            double sum = 0.0;
            for (auto &p : tm.spmv) sum += tm.between(p.first, p.second);
            info->ms_spmv_sum = sum;
            info->spmv_launches = (int)tm.spmv.size();
            info->spmv_monitored = tm.monitored;
        }
    }
    if (!ss.converged) return fail(SG_E_NOCONV, "solve stopped at relative residual " + std::to_string(ss.rel));
    return SG_OK;
}


// Neumann sweeps for all wavelengths at once: x <- rhs + K x (rhs = NULL: the solar
// source built on the fly), with the two measures of the single-wavelength sweeps per
// wavelength (L1 update for the ratio and the stall test, largest per-edge relative
// update for the stop when relative != 0, else L1 below stop times the first sweep's).
// Only the last sweep of each chunk computes the measures (and the first iterate, a copy
// that reads no previous iterate): a measured sweep reads the previous iterate of every
// edge and wavelength, half again the bytes of a plain sweep at 64 wavelengths.  The
// convergence ratio per sweep is the ratio of two measures taken k sweeps apart, to the
// power 1/k.  A wavelength is done once its stop is met or predicted; stall = a
// wavelength not done whose L1 ratio (and relative ratio, when that decides the stop)
// reaches 0.95; a measure that is not finite (an overflowed iterate) sets stalled = 2.
sg_status neumann_batched(Scene &s, hipStream_t st, Exec &tm, int grid, const float *rhs, float *&xa, float *&xb,
                          int relative, double stop, int max_sweeps, SolveStats &ss, int &stalled) {
    Ctx *ctx = s.ctx;
    const int nl = s.n_lambda;
    std::vector<double> host((size_t)4 * nl);
    std::vector<double> l1p(nl, -1.0), l1(nl, 0.0), relp(nl, -1.0), rel(nl, 0.0), l1first(nl, 0.0);
    std::vector<int> done(nl, 0);
    int chunk = 3, first = 1;  // the first iterate and the third: a ratio over two sweeps
    int at = 0, at_prev = 0;   // sweep index of the last measure and of the one before
    stalled = 0;
    double *hist = s.lam_buf + 4 * nl;  // [2][nl][2]: the first iterate's and the chunk's last sweep's
    while (true) {
        chunk = std::max(1, std::min(chunk, 32));
        // the first iterate from x = 0 is rhs itself: a copy instead of a sweep
        const int n_copy = first ? 1 : 0;
        auto sweep = [&](int c, const float *a, float *b, hipEvent_t after) {
            const int mon = (first && c == 0) || c == chunk - 1;
            if (c < n_copy) launch_bfirst(s, st, rhs, b);
            else launch_spmm(s, st, grid, rhs, a, b, mon);
            if (after) (void)hipEventRecord(after, st);
            if (mon) launch_measures(s, nl, hist + (size_t)(c == chunk - 1 ? 1 : 0) * nl * 2, st);
        };
        if (tm.on) {
            for (int c = 0; c < chunk; ++c) {
                if (c < n_copy) {
                    sweep(c, xa, xb, nullptr);
                } else {
                    hipEvent_t e0 = tm.mark(), e1 = tm.fresh();
                    sweep(c, xa, xb, e1);
                    tm.spmv.push_back({e0, e1});
                    tm.monitored += c == chunk - 1;
                }
                std::swap(xa, xb);
            }
        } else {
            const GraphKey key{2, (uintptr_t)chunk, (uintptr_t)rhs, (uintptr_t)xa, (uintptr_t)xb, (uintptr_t)grid,
                               (uintptr_t)first, (uintptr_t)s.tile};
            float *a0 = xa, *b0 = xb;
            SG_TRY(run_chunk(s, st, key, tm.graphs, [&]() {
                float *a = a0, *b = b0;
                for (int c = 0; c < chunk; ++c) {
                    sweep(c, a, b, nullptr);
                    std::swap(a, b);
                }
            }));
            if (chunk & 1) std::swap(xa, xb);
        }
        ss.sweeps += chunk - n_copy;
        SG_HIP(hipGetLastError());
        SG_TRY(read_scalars(s, st, hist, host.data(), 4 * nl));
        const double *last = host.data() + 2 * nl;  // [nl][2] of the chunk's last sweep
        if (first) {  // the first iterate's measures: the starting point of the ratios
            for (int k = 0; k < nl; ++k) {
                l1first[k] = host[2 * k];
                l1[k] = host[2 * k];
                rel[k] = host[2 * k + 1];
            }
            at = 1;
        }
        at_prev = at;
        at += first ? chunk - 1 : chunk;
        first = 0;
        const double gap = (double)(at - at_prev);  // sweeps between the two measures
        bool all = true;
        double need = 1.0;
        for (int k = 0; k < nl; ++k) {
            if (done[k]) continue;
            l1p[k] = l1[k];
            relp[k] = rel[k];
            l1[k] = last[2 * k];
            rel[k] = last[2 * k + 1];
            if (!std::isfinite(l1[k]) || !std::isfinite(rel[k])) { stalled = 2; continue; }
            const double stop_k = relative ? stop : stop * l1first[k];
            const double r = relative ? rel[k] : l1[k];
            const double q = l1p[k] > 0 ? std::pow(l1[k] / l1p[k], 1.0 / gap) : 0.5;
            const double q2 = relp[k] > 0 ? std::pow(rel[k] / relp[k], 1.0 / gap) : 0.0;
            const double qr = relative && relp[k] > 0 ? std::max(q, q2) : q;
            // the measured update belongs to the previous iterate; the current one's is about q r
            if (r <= stop_k || (l1p[k] > 0 && qr < 0.9 && qr * r <= 0.5 * stop_k)) { done[k] = 1; continue; }
            all = false;
            if (l1p[k] > 0 && ss.sweeps >= 4 && q >= 0.95 && (!relative || q2 >= 0.95)) stalled = 1;
            const double qa = relative && q2 > 0 ? std::min(q, q2) : q;
            const double qc = std::min(std::max(qa, 1e-12), 0.95);
            need = std::max(need, std::log(stop_k / r) / std::log(qc));
        }
        if (sg_log()) {
            double worst = 0.0;
            int nd = 0;
            for (int k = 0; k < nl; ++k) {
                nd += done[k];
                worst = std::max(worst, relative ? rel[k] : (l1first[k] > 0 ? l1[k] / l1first[k] : 0.0));
            }
            fprintf(stderr, "[sgrt] batched sweeps %d chunk %d: %d/%d wavelengths done, worst measure %.3e\n",
                    ss.sweeps, chunk, nd, nl, worst);
        }
        if (all || stalled || ss.sweeps >= max_sweeps) break;
        chunk = (int)std::ceil(need);
    }
    return SG_OK;
}

sg_status solve_batched_linear(Scene &s, const sg_solve_opts &o, hipStream_t st, Exec &tm, SolveStats &ss) {
    Ctx *ctx = s.ctx;
    const int nl = s.n_lambda;
    const long long n = (long long)s.E * nl;
    const double rtol = o.rtol > 0 ? o.rtol : 1e-6;
    const int max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : 2000;
    const int m = o.gmres_restart > 0 ? std::min(std::max(o.gmres_restart, 2), 64) : 32;
    if (o.lambda_tile > 0 && o.lambda_tile < 64 && o.lambda_tile < smallest_tile(nl))
        return fail(SG_E_INVALID, "lambda_tile " + std::to_string(o.lambda_tile) + " is narrower than the " +
                                      std::to_string(nl) + " wavelengths");
    float *xa = s.bx, *xb = s.by;
    const int grid = spmm_grid(s, st, xa, xb, tm.autotune, o.lambda_tile);  // sets s.tile
    const int rgrid = batched_groups(s);  // FP64 pass: the tile's default grid
    int stalled = 0;
    std::vector<double> m2((size_t)2 * nl), sc(nl);
    double *d_sc = s.lam_buf;  // [nl]
    // the solution as an FP64 copy (made only when a correction, GMRES or an export needs it;
    // until then it is the FP32 iterate, whose promoted values the residual reads)
    auto materialize = [&]() {
        if (s.phi32) launch_f32_to_64(s.phi32, s.x64, n, st);
        s.phi32 = nullptr;
    };
    // FP64 residual of the solution for every wavelength: the worst per-edge relative
    // residual, and the scales r / rel (at most |x| per edge: well inside the FP32 range)
    auto residual = [&](double &worst) -> sg_status {
        // r in FP32: the correction's right-hand side
        if (s.phi32) launch_bresidual32(s, st, rgrid, s.phi32, s.bS);
        else launch_bresidual64(s, st, rgrid, s.x64, s.bS);
        launch_measures(s, nl, s.lam_buf + nl, st);  // [nl][2]
        ++ss.sweeps;
        ++ss.refinements;
        SG_TRY(read_scalars(s, st, s.lam_buf + nl, m2.data(), 2 * nl));
        worst = 0.0;
        for (int k = 0; k < nl; ++k) {
            const double rel = m2[2 * k + 1];  // max over edges of |r| / |x|
            worst = std::max(worst, std::isfinite(rel) && std::isfinite(m2[2 * k]) ? rel : HUGE_VAL);
            sc[k] = rel > 0 ? 1.0 / rel : 1.0;
        }
        return SG_OK;
    };
    if (o.solver == SG_SOLVER_GMRES) {  // every wavelength by GMRES from zero
        launch_fill<double>(s.x64, 0.0, n, st);
        std::vector<double> rel(nl, HUGE_VAL);
        SG_TRY(gmres_batched(s, st, rtol, m, max_sweeps, rel, ss));
        ss.rel = *std::max_element(rel.begin(), rel.end());
        SG_HIP(hipGetLastError());
        return SG_OK;
    }
    bool warm = false, have_r = false;
    double worst = 0.0;
    if (o.warm_start) {  // kept if better than zero for every wavelength
        SG_TRY(load_warm_start(s, o, st));
        SG_TRY(residual(worst));
        warm = have_r = worst <= kWarmKeep;
    }
    if (!warm) {
        // per-edge relative updates settle at a few FP32 rounding units: never ask for less
        SG_TRY(neumann_batched(s, st, tm, grid, nullptr, xa, xb, 1, std::max(0.3 * rtol, 4e-6), max_sweeps, ss,
                               stalled));
        s.phi32 = xa;  // the solution, until a step below needs it in FP64
    }
    for (int it = 0; it < 10; ++it) {
        if (!have_r) SG_TRY(residual(worst));
        have_r = false;
        ss.rel = worst;
        if (sg_log()) fprintf(stderr, "[sgrt] FP64 residual after %d sweeps: worst relative %.3e\n", ss.sweeps, worst);
        if (worst <= rtol) { ss.converged = 1; break; }
        if (stalled || ss.sweeps >= max_sweeps || !std::isfinite(worst)) break;
        materialize();  // the correction's sweeps reuse the FP32 iterate's buffers
        SG_HIP(hipMemcpyAsync(d_sc, sc.data(), sizeof(double) * nl, hipMemcpyHostToDevice, st));
        launch_lam_scale_f32(s.bS, d_sc, nl, n, st);  // r / rel per wavelength
        float *ca = s.bx, *cb = s.by;
        int st2 = 0;
        SG_TRY(neumann_batched(s, st, tm, grid, s.bS, ca, cb, 0, correction_stop(warm, it, worst, rtol), max_sweeps,
                               ss, st2));
        launch_lam_axpy(s.x64, ca, d_sc, nl, n, st);
        if (st2) stalled = 1;
    }
    // a stall, an overflow or refinements that did not get there: the wavelengths still above
    // rtol go to GMRES (each with the sweeps left of the budget)
    const int left = max_sweeps - ss.sweeps;
    if (!ss.converged && o.solver == SG_SOLVER_AUTO && left > 1) {
        materialize();
        SG_TRY(residual(worst));
        std::vector<double> rel(nl);
        for (int k = 0; k < nl; ++k)
            rel[k] = std::isfinite(m2[2 * k]) && std::isfinite(m2[2 * k + 1]) ? m2[2 * k + 1] : HUGE_VAL;
        if (worst <= rtol) {
            ss.converged = 1;
        } else {
            SG_TRY(gmres_batched(s, st, rtol, m, left, rel, ss));
        }
        ss.rel = *std::max_element(rel.begin(), rel.end());
    }
    SG_HIP(hipGetLastError());
    return SG_OK;
}

sg_status solve_batched(Scene &s, const sg_solve_opts &o, hipStream_t st, double *radiance, int on_dev,
                        sg_solve_info *info) {
    Ctx *ctx = s.ctx;
    Exec tm;
    tm.on = o.timing != 0;
    tm.graphs = !(o.flags & SG_NO_GRAPHS) && !tm.on;
    tm.autotune = !(o.flags & SG_NO_AUTOTUNE);
    s.qscreen = (o.flags & SG_EXACT_CELLS) ? 0 : 1;
    s.phi32 = nullptr;
    tm.st = st;
    if (o.build_col_idx && !s.col_idx) SG_TRY(dalloc(s, &s.col_idx, (size_t)s.nnz));
    SG_TRY(fork_sun_march<float>(s, st, 1.0f));
    hipEvent_t e0 = tm.mark();
    launch_structure(s, st);
    if (o.build_col_idx) {
        launch_col_idx(s, st);
        s.col_built = true;
    } else {
        s.col_built = false;
    }
    hipEvent_t e1 = tm.mark();
    launch_march_edges<float>(s, st, 1.0f, 1);
    SG_HIP(hipStreamWaitEvent(st, s.ev_join, 0));  // the sun march, read by the node coefficients
    launch_bnode_coef(s, st);
    hipEvent_t e2 = tm.mark();
    launch_qbuild<float>(s, st, 1);
    hipEvent_t e3 = tm.mark();
    SG_HIP(hipGetLastError());
    SolveStats ss;
    const long long n = (long long)s.E * s.n_lambda;
    if (o.scatter_order == 1) {
        launch_fill<double>(s.x64, 0.0, n, st);
        ss.converged = 1;
    } else {
        SG_TRY(solve_batched_linear(s, o, st, tm, ss));
    }
    hipEvent_t e4 = tm.mark();
    double *dst = on_dev ? radiance : s.pix;
    if (s.phi32) launch_batched_gather(s, st, (const float *)s.phi32, o.scatter_order, dst);
    else launch_batched_gather(s, st, (const double *)s.x64, o.scatter_order, dst);
    hipEvent_t e5 = tm.mark();
    SG_HIP(hipGetLastError());
    if (!on_dev)
        SG_HIP(hipMemcpyAsync(radiance, dst, sizeof(double) * s.npx * s.n_lambda, hipMemcpyDeviceToHost, st));
    SG_HIP(hipStreamSynchronize(st));
    s.solved = true;
    s.last_precision = SG_FP32;
    s.last_scatter_order = o.scatter_order;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->converged = ss.converged;
        info->sweeps = ss.sweeps;
        info->refinements = ss.refinements;
        info->gmres_used = ss.gmres_used;
        info->rel_residual = ss.rel;
        info->n_nodes = s.N;
        info->n_edges = s.E;
        info->nnz = s.nnz;
        if (tm.on) {
            info->ms_structure = tm.between(e0, e1);
            info->ms_march = tm.between(e1, e2);
            info->ms_qbuild = tm.between(e2, e3);
            info->ms_solve = tm.between(e3, e4);
            info->ms_gather = tm.between(e4, e5);
            info->ms_total = tm.between(e0, e5);
            double sum = 0.0;
            for (auto &p : tm.spmv) sum += tm.between(p.first, p.second);
            info->ms_spmv_sum = sum;
            info->spmv_launches = (int)tm.spmv.size();
            info->spmv_monitored = tm.monitored;
        }
    }
    if (!ss.converged) return fail(SG_E_NOCONV, "solve stopped at relative residual " + std::to_string(ss.rel));
    return SG_OK;
}

}  // namespace
}  // namespace sg

using namespace sg;


extern "C" {

const char *sg_last_error(void) { return t_err.c_str(); }

uint32_t sg_abi_version(void) { return SG_ABI_VERSION; }

sg_status sg_ctx_create(int32_t hip_device, uint64_t hbm_budget_bytes, sg_ctx **out) {
    if (!out) return fail(SG_E_INVALID, "out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return fail(SG_E_DEVICE, "no HIP device");
    if (hip_device < 0 || hip_device >= n) return fail(SG_E_INVALID, "bad device index");
    Ctx *ctx = nullptr;
    SG_HIP(hipSetDevice(hip_device));
    size_t fr = 0, tot = 0;
    SG_HIP(hipMemGetInfo(&fr, &tot));
    std::unique_ptr<sg_ctx> c(new sg_ctx());
    c->device = hip_device;
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)fr);
    ctx = c.get();
    SG_TRY(scratch_setup(hip_device));  // the allocation-free trace's staging on this device
    SG_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    *out = c.release();
    return SG_OK;
}

sg_status sg_ctx_destroy(sg_ctx *ctx) {
    if (!ctx) return fail(SG_E_INVALID, "ctx is NULL");
    if (ctx->n_scenes.load() != 0) return fail(SG_E_STATE, "context still has scenes");
    (void)hipSetDevice(ctx->device);
    pool_trim(ctx, 0);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return SG_OK;
}

}  // extern "C"

namespace sg {
namespace {
sg_status create_scene_impl(Ctx *ctx, const sg_scene_desc *d, hipStream_t st, Scene &s);
void free_scene_impl(Scene *s);
}  // namespace

void free_scene(Scene *s) { free_scene_impl(s); }
sg_status create_scene(Ctx *ctx, const sg_scene_desc *d, hipStream_t st, Scene &s) {
    const sg_status r = create_scene_impl(ctx, d, st, s);
    return r == SG_OK ? bounds_report() : r;
}

namespace {

void free_scene_impl(Scene *s) {
    clear_graphs(*s);
    // the sun march of a solve that stopped before joining may still run on the second
    // stream: it ends before any block goes back to the pool
    if (s->aux) {
        (void)hipStreamSynchronize(s->aux);
        (void)hipStreamDestroy(s->aux);
        s->aux = nullptr;
    }
    if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
    if (s->ev_join) (void)hipEventDestroy(s->ev_join);
    s->ev_fork = s->ev_join = nullptr;
    void *ptrs[] = {s->big, s->bigdir, s->bigrow, s->big_part, s->mu_s, s->mu_a, s->frac, s->albedo, s->abs_scale_d, s->pos, s->adj_ptr, s->adj_idx, s->lat,
                    s->tab, s->lut, s->hull, s->rev, s->nodeoff, s->row_ptr, s->col_idx, s->scan_tmp, s->tau_s, s->tau_a, s->tsun_s,
                    s->tsun_a, s->T, s->Tsun, s->rho, s->val, s->S, s->x, s->y, s->c_rhs, s->c_a, s->c_b, s->qsun,
                    s->q, s->bS, s->bx, s->by, s->brho, s->bsrc, s->lam_buf, s->x64, s->r64, s->gm_V, s->partial, s->meas, s->meas_part, s->scal, s->J, s->pix,
                    s->gmu_s, s->gmu_a, s->gfrac, s->los_ptr, s->los_node, s->los_t};
    if (s->ctx)
        for (void *p : ptrs) pool_free(s->ctx, p);
    s->bytes = 0;
}

sg_status upload(Scene &s, void *dst, const void *src, size_t bytes, hipStream_t st) {
    Ctx *ctx = s.ctx;
    SG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    return SG_OK;
}

double host_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

sg_status create_scene_impl(Ctx *ctx, const sg_scene_desc *d, hipStream_t st, Scene &s) {
    int64_t N, E, nnz;
    int dmax;
    const double t0 = host_ms();
    SG_TRY(validate(d, N, E, nnz, dmax));
    const double t1 = host_ms();
    s.ctx = ctx;
    s.nx = d->nx; s.ny = d->ny; s.nz = d->nz;
    s.voxel_m = d->voxel_m;
    s.nvox = d->nx * d->ny * d->nz;
    s.general = d->n_nodes > 0;
    s.n_vol = s.general ? d->n_nodes : s.nvox;
    s.N = (int)N;
    s.npx = d->nx * d->ny;
    s.E = E;
    s.nnz = nnz;
    s.dmax = std::max(dmax, 1);
    s.n_phase = d->n_phase;
    for (int k = 0; k < d->n_phase; ++k) {
        s.hg_g[k] = d->hg_g[k];
        s.phase_kind[k] = d->phase_kind ? d->phase_kind[k] : SG_PHASE_HG;
        if (s.phase_kind[k] == SG_PHASE_TABLE) {
            s.lut_n = d->phase_lut_n;
            s.lut_scale[k] = 1.0 / table_integral(d->phase_lut + (size_t)k * d->phase_lut_n, d->phase_lut_n);
        }
    }
    s.n_fib = d->n_fib;
    s.sigma_mode = d->sigma_mode;
    s.periodic = d->periodic;
    s.surface = d->surface_nodes ? 1 : 0;
    s.weight_mode = d->node_weight_mode;
    s.n_lambda = d->n_lambda;
    s.abs_scale.assign(d->n_lambda, 1.0f);
    if (d->abs_scale) for (int k = 0; k < d->n_lambda; ++k) s.abs_scale[k] = d->abs_scale[k];
    for (int k = 0; k < 3; ++k) { s.sun[k] = d->sun_dir[k]; s.view[k] = d->view_dir[k]; }
    double su[3];
    unit3(s.sun, su, 1.0);
    unit3(s.sun, s.sun_in, -1.0);
    unit3(s.view, s.view_u, 1.0);
    s.mu0 = su[2];

    const int nl = s.n_lambda;
    // inputs
    SG_TRY(dalloc(s, &s.mu_s, s.nvox));
    SG_TRY(dalloc(s, &s.mu_a, s.nvox));
    if (s.n_phase > 1) SG_TRY(dalloc(s, &s.frac, (size_t)s.n_phase * s.nvox));
    SG_TRY(dalloc(s, &s.albedo, s.npx));
    SG_TRY(dalloc(s, &s.pos, (size_t)3 * s.N));
    SG_TRY(dalloc(s, &s.adj_ptr, (size_t)s.N + 1));
    SG_TRY(dalloc(s, &s.adj_idx, (size_t)s.E));
    // nodes of degree above one wavefront, and the prefix of their groups of incoming
    // directions (in-edges and the sun; one for a surface node; qbuild_group_big per group)
    // and of their chunks of 256 rows (the sweeps' workgroups)
    std::vector<int> bigv;
    std::vector<long long> bigdir(1, 0), bigrow(1, 0);
    for (int64_t l = 0; l < s.N; ++l) {
        const int64_t deg = d->adj_ptr[l + 1] - d->adj_ptr[l];
        if (deg > kMaxWaveDegree) {
            bigv.push_back((int)l);
            // one direction per workgroup for the colouring, groups for the Voronoi cells
            const int64_t n_in = l < s.n_vol ? deg + 1 : 1;
            const int64_t G = s.sigma_mode == SG_SIGMA_COLOUR ? 1 : qbuild_group_big(s.n_fib);
            bigdir.push_back(bigdir.back() + (n_in + G - 1) / G);
            bigrow.push_back(bigrow.back() + (deg + 255) / 256);
        }
    }
    s.n_big = (int)bigv.size();
    s.n_bigdir = bigdir.back();
    s.n_bigrow = bigrow.back();
    if (s.n_big) {
        SG_TRY(dalloc(s, &s.big, bigv.size()));
        SG_TRY(dalloc(s, &s.bigdir, bigdir.size()));
        SG_TRY(dalloc(s, &s.bigrow, bigrow.size()));
        SG_TRY(dalloc(s, &s.big_part, (size_t)s.n_bigrow));
    }
    int64_t n_el = 0;
    if (s.general) {
        n_el = d->los_ptr[s.npx];
        SG_TRY(dalloc(s, &s.gmu_s, (size_t)s.n_vol));
        SG_TRY(dalloc(s, &s.gmu_a, (size_t)s.n_vol));
        if (s.n_phase > 1) SG_TRY(dalloc(s, &s.gfrac, (size_t)s.n_phase * s.n_vol));
        SG_TRY(dalloc(s, &s.los_ptr, (size_t)s.npx + 1));
        SG_TRY(dalloc(s, &s.los_node, (size_t)n_el));
        SG_TRY(dalloc(s, &s.los_t, (size_t)n_el));
    }
    SG_TRY(dalloc(s, &s.lat, (size_t)3 * s.n_fib));
    SG_TRY(dalloc(s, &s.tab, (size_t)(s.n_phase + 1) * s.n_fib));
    if (s.lut_n) SG_TRY(dalloc(s, &s.lut, (size_t)s.n_phase * s.lut_n));
    if (s.sigma_mode == SG_SIGMA_COLOUR) SG_TRY(dalloc(s, &s.hull, (size_t)s.n_fib * (kHullNb + 1)));
    // structure
    SG_TRY(dalloc(s, &s.rev, (size_t)s.E));
    SG_TRY(dalloc(s, &s.nodeoff, (size_t)s.N + 1));
    SG_TRY(dalloc(s, &s.row_ptr, (size_t)s.E + 1));
    SG_TRY(dalloc(s, &s.scan_tmp, (size_t)s.N / 2048 + 2));
    SG_TRY(dalloc(s, &s.qsun, (size_t)s.E));
    // solve state
    SG_TRY(dalloc(s, &s.x64, (size_t)s.E * nl));
    SG_TRY(dalloc(s, &s.r64, (size_t)s.E * nl));
    s.n_partial = std::max(spmv_blocks(s), 65 * 1024);
    SG_TRY(dalloc(s, &s.partial, (size_t)s.n_partial));
    SG_TRY(dalloc(s, &s.meas, (size_t)s.N * nl));
    SG_TRY(dalloc(s, &s.meas_part, (size_t)node_chunks(s.N, nl) * nl * 2));
    SG_TRY(dalloc(s, &s.scal, 256));
    SG_TRY(dalloc(s, &s.J, (size_t)s.N * nl));
    SG_TRY(dalloc(s, &s.pix, (size_t)s.npx * nl));
    if (nl == 1) {
        SG_TRY(ensure_real<float>(s));
    } else {
        float *p;
        SG_TRY(dalloc(s, &p, s.E)); s.tau_s = p;
        SG_TRY(dalloc(s, &p, s.E)); s.tau_a = p;
        SG_TRY(dalloc(s, &p, s.N)); s.tsun_s = p;
        SG_TRY(dalloc(s, &p, s.N)); s.tsun_a = p;
        SG_TRY(dalloc(s, &s.q, (size_t)s.nnz + 64));  // padded: whole-column reads past the last block
        SG_TRY(dalloc(s, &s.bS, (size_t)s.E * nl));
        SG_TRY(dalloc(s, &s.bx, (size_t)s.E * nl));
        SG_TRY(dalloc(s, &s.by, (size_t)s.E * nl));
        SG_TRY(dalloc(s, &s.brho, (size_t)s.N * nl));
        SG_TRY(dalloc(s, &s.bsrc, (size_t)s.N * nl));
        SG_TRY(dalloc(s, &s.lam_buf, (size_t)68 * nl));
        SG_TRY(dalloc(s, &s.abs_scale_d, (size_t)nl));
        SG_TRY(upload(s, s.abs_scale_d, s.abs_scale.data(), sizeof(float) * nl, st));
    }

    const double t2 = host_ms();
    // host-side staging of the inputs
    std::vector<int32_t> pos((size_t)3 * s.N);
    std::memcpy(pos.data(), s.general ? d->node_pos_fx : d->vol_pos_fx, sizeof(int32_t) * 3 * (size_t)s.n_vol);
    if (s.surface) {
        for (int iy = 0; iy < s.ny; ++iy)
            for (int ix = 0; ix < s.nx; ++ix) {
                const size_t l = (size_t)s.n_vol + ix + (size_t)s.nx * iy;
                pos[3 * l] = ix * 65536 + 32768;
                pos[3 * l + 1] = iy * 65536 + 32768;
                pos[3 * l + 2] = 0;
            }
    }
    std::vector<double> lat, tab;
    host_lattice(s.n_fib, lat);
    host_tables(s.n_fib, lat, s.n_phase, s.phase_kind, s.hg_g, d->phase_lut, s.lut_n, tab);
    if (s.lut) SG_TRY(upload(s, s.lut, d->phase_lut, sizeof(double) * s.n_phase * (size_t)s.lut_n, st));
    std::vector<int> hull;  // [n_fib][kHullNb] neighbours, then [n_fib] counts
    if (s.hull) {
        static std::mutex mu;
        static std::map<int, std::vector<int>> cache;  // per lattice size (the lattice is fixed by it)
        {
            std::lock_guard<std::mutex> lk(mu);
            auto it = cache.find(s.n_fib);
            if (it != cache.end()) hull = it->second;
        }
        if (hull.empty()) {
            std::vector<int> nb, nnb;
            if (!host_hull(s.n_fib, lat, nb, nnb))
                return fail(SG_E_INVALID, "a lattice point has more than 16 hull neighbours");
            hull = nb;
            hull.insert(hull.end(), nnb.begin(), nnb.end());
            std::lock_guard<std::mutex> lk(mu);
            cache[s.n_fib] = hull;
        }
        SG_TRY(upload(s, s.hull, hull.data(), sizeof(int) * hull.size(), st));
    }
    SG_TRY(upload(s, s.mu_s, d->mu_s, sizeof(float) * s.nvox, st));
    SG_TRY(upload(s, s.mu_a, d->mu_a, sizeof(float) * s.nvox, st));
    if (s.frac) SG_TRY(upload(s, s.frac, d->phase_frac, sizeof(float) * s.n_phase * (size_t)s.nvox, st));
    std::vector<float> gms, gma, gfr;  // staged until the stream drains
    if (s.general) {
        // the medium of each general node: that of the voxel containing it
        gms.resize(s.n_vol);
        gma.resize(s.n_vol);
        gfr.resize(s.frac ? (size_t)s.n_phase * s.n_vol : 0);
        for (int l = 0; l < s.n_vol; ++l) {
            const int64_t v = (int64_t)(pos[3 * l] >> 16) +
                              (int64_t)s.nx * ((int64_t)(pos[3 * l + 1] >> 16) + (int64_t)s.ny * (pos[3 * l + 2] >> 16));
            gms[l] = d->mu_s[v];
            gma[l] = d->mu_a[v];
            for (int k = 0; s.frac && k < s.n_phase; ++k)
                gfr[(size_t)k * s.n_vol + l] = d->phase_frac[(size_t)k * s.nvox + v];
        }
        SG_TRY(upload(s, s.gmu_s, gms.data(), sizeof(float) * s.n_vol, st));
        SG_TRY(upload(s, s.gmu_a, gma.data(), sizeof(float) * s.n_vol, st));
        if (s.gfrac) SG_TRY(upload(s, s.gfrac, gfr.data(), sizeof(float) * gfr.size(), st));
        SG_TRY(upload(s, s.los_ptr, d->los_ptr, sizeof(int64_t) * ((size_t)s.npx + 1), st));
        if (n_el) {
            SG_TRY(upload(s, s.los_node, d->los_node, sizeof(int32_t) * (size_t)n_el, st));
            SG_TRY(upload(s, s.los_t, d->los_t, sizeof(double) * (size_t)n_el, st));
        }
    }
    SG_TRY(upload(s, s.albedo, d->surf_albedo, sizeof(float) * s.npx, st));
    SG_TRY(upload(s, s.pos, pos.data(), sizeof(int32_t) * pos.size(), st));
    SG_TRY(upload(s, s.adj_ptr, d->adj_ptr, sizeof(int64_t) * ((size_t)s.N + 1), st));
    if (s.E) SG_TRY(upload(s, s.adj_idx, d->adj_idx, sizeof(int32_t) * (size_t)s.E, st));
    if (s.n_big) {
        SG_TRY(upload(s, s.big, bigv.data(), sizeof(int) * bigv.size(), st));
        SG_TRY(upload(s, s.bigdir, bigdir.data(), sizeof(long long) * bigdir.size(), st));
        SG_TRY(upload(s, s.bigrow, bigrow.data(), sizeof(long long) * bigrow.size(), st));
    }
    SG_TRY(upload(s, s.lat, lat.data(), sizeof(double) * lat.size(), st));
    SG_TRY(upload(s, s.tab, tab.data(), sizeof(double) * tab.size(), st));
    if (s.E) {
        unsigned *bad = reinterpret_cast<unsigned *>(s.scal);
        SG_HIP(hipMemsetAsync(bad, 0, sizeof(unsigned), st));
        launch_check_symmetric(s, bad, st);
        unsigned nbad = 0;
        SG_HIP(hipMemcpyAsync(&nbad, bad, sizeof(unsigned), hipMemcpyDeviceToHost, st));
        SG_HIP(hipStreamSynchronize(st));
        if (nbad) return fail(SG_E_INVALID, "adjacency is not symmetric (" + std::to_string(nbad) + " edges)");
    }
    SG_HIP(hipStreamCreateWithFlags(&s.aux, hipStreamNonBlocking));
    SG_HIP(hipEventCreateWithFlags(&s.ev_fork, hipEventDisableTiming));
    SG_HIP(hipEventCreateWithFlags(&s.ev_join, hipEventDisableTiming));
    SG_HIP(hipStreamSynchronize(st));
    if (sg_log())
        fprintf(stderr, "[sgrt] scene create: validate %.2f ms, allocate %.2f ms, upload %.2f ms (%zu MB reserved)\n",
                t1 - t0, t2 - t1, host_ms() - t2, (size_t)(s.bytes >> 20));
    return SG_OK;
}

hipStream_t pick_stream(Ctx *ctx, void *st) { return st ? (hipStream_t)st : ctx->stream; }

}  // namespace
}  // namespace sg

extern "C" {

sg_status sg_scene_create(sg_ctx *ctx, const sg_scene_desc *desc, void *hip_stream, sg_scene **out) {
    if (!ctx || !out) return fail(SG_E_INVALID, "ctx or out is NULL");
    *out = nullptr;
    if (ctx->sticky.load()) return fail(SG_E_DEVICE, "context is in a failed state");
    SG_HIP(hipSetDevice(ctx->device));
    std::unique_ptr<sg_scene> s(new sg_scene());
    sg_status st = create_scene(ctx, desc, pick_stream(ctx, hip_stream), *s);
    if (st != SG_OK) {
        std::string msg = t_err;
        (void)hipStreamSynchronize(pick_stream(ctx, hip_stream));  // uploads queued before the failure
        free_scene(s.get());
        set_error(msg);
        return st;
    }
    ctx->n_scenes.fetch_add(1);
    *out = s.release();
    return SG_OK;
}

sg_status sg_scene_destroy(sg_scene *scene) {
    if (!scene) return fail(SG_E_INVALID, "scene is NULL");
    Ctx *ctx = scene->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    free_scene(scene);
    ctx->n_scenes.fetch_sub(1);
    delete scene;
    return SG_OK;
}

sg_status sg_scene_sizes(const sg_scene *scene, int64_t *n_nodes, int64_t *n_edges, int64_t *nnz, int32_t *max_degree,
                         int32_t *n_lambda, uint64_t *device_bytes) {
    if (!scene) return fail(SG_E_INVALID, "scene is NULL");
    if (n_nodes) *n_nodes = scene->N;
    if (n_edges) *n_edges = scene->E;
    if (nnz) *nnz = scene->nnz;
    if (max_degree) *max_degree = scene->dmax;
    if (n_lambda) *n_lambda = scene->n_lambda;
    if (device_bytes) *device_bytes = scene->bytes;
    return SG_OK;
}

}  // extern "C"

namespace sg {
sg_status solve_scene(Scene &s, const sg_solve_opts &o, hipStream_t st, double *radiance, int on_dev,
                      sg_solve_info *info) {
    Ctx *ctx = s.ctx;
    std::lock_guard<std::mutex> lk(s.mu);
    SG_HIP(hipSetDevice(ctx->device));
    ++s.solves;
    sg_status r;
    if (s.n_lambda > 1) {
        if (o.precision != SG_FP32) return fail(SG_E_INVALID, "several wavelengths are solved in FP32 only");
        r = solve_batched(s, o, st, radiance, on_dev, info);
    } else if (o.precision == SG_FP64) {
        r = solve_single<double>(s, o, st, radiance, on_dev, info);
    } else {
        r = solve_single<float>(s, o, st, radiance, on_dev, info);
    }
    const sg_status b = bounds_report();
    return b != SG_OK ? b : r;
}

sg_status check_opts(const sg_solve_opts *opts, sg_solve_opts &o) {
    if (opts) {
        if (opts->abi_version != SG_ABI_VERSION) return fail(SG_E_ABI, "solve opts abi_version mismatch");
        o = *opts;
    } else {
        fill_default_opts(o);
    }
    if (o.precision != SG_FP32 && o.precision != SG_FP64) return fail(SG_E_INVALID, "precision must be SG_FP32 or SG_FP64");
    if (o.solver < 0 || o.solver > 2) return fail(SG_E_INVALID, "bad solver");
    if (o.scatter_order != 0 && o.scatter_order != 1) return fail(SG_E_INVALID, "scatter_order must be 0 or 1");
    if (o.lambda_tile != 0 && o.lambda_tile != 8 && o.lambda_tile != 16 && o.lambda_tile != 32 && o.lambda_tile != 64)
        return fail(SG_E_INVALID, "lambda_tile must be 0, 8, 16, 32 or 64");
    if (o.warm_start_on_device != 0 && o.warm_start_on_device != 1)
        return fail(SG_E_INVALID, "warm_start_on_device must be 0 or 1");
    return SG_OK;
}


uint64_t scene_reservation(const sg_scene_desc *d, sg_status *st) {
    return reservations(d, nullptr, false, st);
}

uint64_t solve_reservation(const sg_scene_desc *d, const sg_solve_opts &o, bool with_gmres) {
    sg_status st;
    const uint64_t all = reservations(d, &o, with_gmres, &st);
    return st == SG_OK ? all - reservations(d, nullptr, false, &st) : 0;
}

uint64_t reservations(const sg_scene_desc *d, const sg_solve_opts *o, bool with_gmres, sg_status *st) {
    int64_t N, E, nnz;
    int dmax;
    *st = validate(d, N, E, nnz, dmax);
    if (*st != SG_OK) return 0;
    // mirrors the allocations of create_scene (each at least one element, rounded as
    // the pool rounds)
    auto a = [](uint64_t count, uint64_t size) { return pool_round(std::max<uint64_t>(count, 1) * size); };
    const uint64_t nvox = (uint64_t)d->nx * d->ny * d->nz, npx = (uint64_t)d->nx * d->ny;
    const uint64_t nl = (uint64_t)d->n_lambda, nf = (uint64_t)d->n_fib, np = (uint64_t)d->n_phase;
    const uint64_t n = (uint64_t)N, e = (uint64_t)E, z = (uint64_t)nnz;
    const uint64_t n_vol = d->n_nodes > 0 ? (uint64_t)d->n_nodes : nvox;
    const uint64_t n_el = d->n_nodes > 0 ? (uint64_t)d->los_ptr[npx] : 0;
    bool table = false;
    for (int k = 0; k < d->n_phase; ++k) table = table || (d->phase_kind && d->phase_kind[k] == SG_PHASE_TABLE);
    uint64_t b = a(nvox, 4) * 2 + (np > 1 ? a(np * nvox, 4) : 0) + a(npx, 4) + a(3 * n, 4) + a(n + 1, 8) +
                 a(e, 4) + a(3 * nf, 8) + a((np + 1) * nf, 8) + (table ? a(np * (uint64_t)d->phase_lut_n, 8) : 0) +
                 (d->sigma_mode == SG_SIGMA_COLOUR ? a(nf * (kHullNb + 1), 4) : 0);
    if (d->n_nodes > 0)  // general nodes: their medium and the lines of sight's elements
        b += a(n_vol, 4) * 2 + (np > 1 ? a(np * n_vol, 4) : 0) + a(npx + 1, 8) + a(n_el, 4) + a(n_el, 8);
    b += a(e, 4) + a(n + 1, 8) + a(e + 1, 8) + a(n / 2048 + 2, 8) + a(e, 4);
    uint64_t n_big = 0, n_rows = 0;
    for (int64_t l = 0; l < N; ++l) {
        const int64_t deg = d->adj_ptr[l + 1] - d->adj_ptr[l];
        if (deg > kMaxWaveDegree) {
            ++n_big;
            n_rows += (uint64_t)(deg + 255) / 256;
        }
    }
    if (n_big) b += a(n_big, 4) + a(n_big + 1, 8) * 2 + a(n_rows, 16);
    b += a(e * nl, 8) * 2 + a(std::max<uint64_t>((n + 3) / 4, 65 * 1024), 8) +
         a(n * nl, 8) + a((uint64_t)node_chunks((int)n, (int)nl) * nl * 2, 8) + a(256, 8) +
         a(n * nl, 8) + a(npx * nl, 8);
    if (nl == 1) {
        b += a(e, 4) * 9 + a(n, 4) * 4 + a(z, 4);
    } else {
        b += a(e, 4) * 2 + a(n, 4) * 2 + a(z + 64, 4) + a(e * nl, 4) * 3 + a(n * nl, 4) * 2 + a(68 * nl, 8) +
             a(nl, 4);
    }
    if (o) {  // what a solve with these options allocates beyond the scene's arrays
        if (o->build_col_idx) b += a(z, 4);
        // FP64 solves trade the FP32 working arrays (released first) for FP64 ones
        if (nl == 1 && o->precision == SG_FP64)
            b += (a(e, 8) * 9 + a(n, 8) * 4 + a(z, 8)) - (a(e, 4) * 9 + a(n, 4) * 4 + a(z, 4));
        if (with_gmres) {  // the basis; a batched scene adds one wavelength's iterate and residual
            const uint64_t m = o->gmres_restart > 0 ? (uint64_t)std::min(std::max(o->gmres_restart, 2), 64) : 32;
            b += a((m + 1 + (nl > 1 ? 2 : 0)) * e, 8);
        }
    }
    return b;
}

}  // namespace sg

extern "C" {

sg_status sg_solve(sg_scene *scene, const sg_solve_opts *opts, void *hip_stream, double *radiance,
                   int32_t radiance_on_device, sg_solve_info *info) {
    if (!scene || !radiance) return fail(SG_E_INVALID, "scene or radiance is NULL");
    Ctx *ctx = scene->ctx;
    if (ctx->sticky.load()) return fail(SG_E_DEVICE, "context is in a failed state");
    sg_solve_opts o;
    SG_TRY(check_opts(opts, o));
    return solve_scene(*scene, o, pick_stream(ctx, hip_stream), radiance, radiance_on_device, info);
}

sg_status sg_scene_reservation(const sg_scene_desc *desc, uint64_t *bytes) {
    if (!bytes) return fail(SG_E_INVALID, "bytes is NULL");
    sg_status st;
    *bytes = scene_reservation(desc, &st);
    return st;
}

sg_status sg_export_csr(sg_scene *scene, int32_t lambda, int64_t *row_ptr, int32_t *col_idx, double *val) {
    if (!scene) return fail(SG_E_INVALID, "scene is NULL");
    Scene &s = *scene;
    Ctx *ctx = s.ctx;
    if (!s.solved) return fail(SG_E_STATE, "no solve yet");
    if (lambda < 0 || lambda >= s.n_lambda) return fail(SG_E_INVALID, "bad wavelength index");
    std::lock_guard<std::mutex> lk(s.mu);
    SG_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    if (row_ptr) SG_HIP(hipMemcpyAsync(row_ptr, s.row_ptr, sizeof(int64_t) * (s.E + 1), hipMemcpyDeviceToHost, st));
    if (col_idx) {
        if (!s.col_built) {
            if (!s.col_idx) SG_TRY(dalloc(s, &s.col_idx, (size_t)s.nnz));
            launch_col_idx(s, st);
            s.col_built = true;
        }
        SG_HIP(hipMemcpyAsync(col_idx, s.col_idx, sizeof(int32_t) * s.nnz, hipMemcpyDeviceToHost, st));
    }
    if (val) {
        if (s.n_lambda > 1) {
            // K(lambda)[b][a] = T_a(lambda) rho_l(lambda) Q_l(a -> b), rebuilt on the host from device arrays
            std::vector<float> q(s.nnz), ts(s.E), ta(s.E), rho((size_t)s.N * s.n_lambda);
            std::vector<int64_t> ap(s.N + 1), no(s.N + 1);
            SG_HIP(hipMemcpyAsync(q.data(), s.q, sizeof(float) * s.nnz, hipMemcpyDeviceToHost, st));
            SG_HIP(hipMemcpyAsync(ts.data(), s.tau_s, sizeof(float) * s.E, hipMemcpyDeviceToHost, st));
            SG_HIP(hipMemcpyAsync(ta.data(), s.tau_a, sizeof(float) * s.E, hipMemcpyDeviceToHost, st));
            SG_HIP(hipMemcpyAsync(rho.data(), s.brho, sizeof(float) * rho.size(), hipMemcpyDeviceToHost, st));
            SG_HIP(hipMemcpyAsync(ap.data(), s.adj_ptr, sizeof(int64_t) * (s.N + 1), hipMemcpyDeviceToHost, st));
            SG_HIP(hipMemcpyAsync(no.data(), s.nodeoff, sizeof(int64_t) * (s.N + 1), hipMemcpyDeviceToHost, st));
            SG_HIP(hipStreamSynchronize(st));
            const float sl = s.abs_scale[lambda];
            for (int64_t l = 0; l < s.N; ++l) {
                const int64_t d = ap[l + 1] - ap[l];
                const float r = rho[(size_t)l * s.n_lambda + lambda];
                for (int64_t n = 0; n < d; ++n)
                    for (int64_t m = 0; m < d; ++m) {
                        const int64_t e = ap[l] + m;
                        const float T = expf(-(ts[e] + sl * ta[e]));
                        val[no[l] + n * d + m] = (double)(T * r * q[no[l] + m * d + n]);
                    }
            }
        } else {
            // the device blocks are column-major; CSR rows are row-major within each block
            std::vector<double> tmp(s.nnz);
            std::vector<int64_t> ap(s.N + 1), no(s.N + 1);
            if (s.real_bytes == 4) {
                std::vector<float> t32(s.nnz);
                SG_HIP(hipMemcpyAsync(t32.data(), s.val, sizeof(float) * s.nnz, hipMemcpyDeviceToHost, st));
                SG_HIP(hipStreamSynchronize(st));
                for (int64_t i = 0; i < s.nnz; ++i) tmp[i] = t32[i];
            } else {
                SG_HIP(hipMemcpyAsync(tmp.data(), s.val, sizeof(double) * s.nnz, hipMemcpyDeviceToHost, st));
            }
            SG_HIP(hipMemcpyAsync(ap.data(), s.adj_ptr, sizeof(int64_t) * (s.N + 1), hipMemcpyDeviceToHost, st));
            SG_HIP(hipMemcpyAsync(no.data(), s.nodeoff, sizeof(int64_t) * (s.N + 1), hipMemcpyDeviceToHost, st));
            SG_HIP(hipStreamSynchronize(st));
            for (int64_t l = 0; l < s.N; ++l) {
                const int64_t d = ap[l + 1] - ap[l];
                for (int64_t n = 0; n < d; ++n)
                    for (int64_t m = 0; m < d; ++m) val[no[l] + n * d + m] = tmp[no[l] + m * d + n];
            }
        }
    }
    SG_HIP(hipStreamSynchronize(st));
    return bounds_report();
}

sg_status sg_export_vector(sg_scene *scene, int32_t which, double *out) {
    if (!scene || !out) return fail(SG_E_INVALID, "scene or out is NULL");
    Scene &s = *scene;
    Ctx *ctx = s.ctx;
    if (!s.solved) return fail(SG_E_STATE, "no solve yet");
    std::lock_guard<std::mutex> lk(s.mu);
    SG_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const bool batched = s.n_lambda > 1;
    const int rb = batched ? 4 : s.real_bytes;
    const void *src = nullptr;
    size_t n = 0;
    int esz = rb;
    switch (which) {
        case SG_VEC_TAU_S: src = s.tau_s; n = s.E; break;
        case SG_VEC_TAU_A: src = s.tau_a; n = s.E; break;
        case SG_VEC_TAU_SUN_S: src = s.tsun_s; n = s.N; break;
        case SG_VEC_TAU_SUN_A: src = s.tsun_a; n = s.N; break;
        case SG_VEC_RHO: src = batched ? (const void *)s.brho : s.rho; n = (size_t)s.N * s.n_lambda; break;
        case SG_VEC_SOURCE:
            if (batched) {
                const int nl = s.n_lambda;
                std::vector<float> br((size_t)s.N * nl), bs((size_t)s.N * nl), qs(s.E);
                std::vector<int64_t> ap(s.N + 1);
                SG_HIP(hipMemcpyAsync(br.data(), s.brho, sizeof(float) * br.size(), hipMemcpyDeviceToHost, st));
                SG_HIP(hipMemcpyAsync(bs.data(), s.bsrc, sizeof(float) * bs.size(), hipMemcpyDeviceToHost, st));
                SG_HIP(hipMemcpyAsync(qs.data(), s.qsun, sizeof(float) * s.E, hipMemcpyDeviceToHost, st));
                SG_HIP(hipMemcpyAsync(ap.data(), s.adj_ptr, sizeof(int64_t) * (s.N + 1), hipMemcpyDeviceToHost, st));
                SG_HIP(hipStreamSynchronize(st));
                for (int64_t l = 0; l < s.N; ++l)
                    for (int64_t e = ap[l]; e < ap[l + 1]; ++e)
                        for (int k = 0; k < nl; ++k)
                            out[(size_t)k * s.E + e] = (double)(br[l * nl + k] * bs[l * nl + k] * qs[e]);
                return SG_OK;
            }
            src = s.S; n = (size_t)s.E; break;
        case SG_VEC_PHI:  // a batched solution may still be the FP32 iterate (promoted here)
            src = s.phi32 ? (const void *)s.phi32 : (const void *)s.x64;
            n = (size_t)s.E * s.n_lambda;
            esz = s.phi32 ? 4 : 8;
            break;
        case SG_VEC_QSUN: src = s.qsun; n = s.E; esz = 4; break;
        default: return fail(SG_E_INVALID, "unknown vector");
    }
    if (esz == 8) {
        SG_HIP(hipMemcpyAsync(out, src, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        SG_HIP(hipStreamSynchronize(st));
    } else {
        std::vector<float> tmp(n);
        SG_HIP(hipMemcpyAsync(tmp.data(), src, sizeof(float) * n, hipMemcpyDeviceToHost, st));
        SG_HIP(hipStreamSynchronize(st));
        for (size_t i = 0; i < n; ++i) out[i] = tmp[i];
    }
    // batched layouts are [E][n_lambda] on the device; the export is [n_lambda][E]
    if (batched && (which == SG_VEC_RHO || which == SG_VEC_SOURCE || which == SG_VEC_PHI)) {
        const size_t rows = which == SG_VEC_RHO ? (size_t)s.N : (size_t)s.E;
        std::vector<double> t(out, out + n);
        for (size_t r = 0; r < rows; ++r)
            for (int k = 0; k < s.n_lambda; ++k) out[(size_t)k * rows + r] = t[r * s.n_lambda + k];
    }
    return bounds_report();
}

sg_status sg_trace(sg_scene *scene, int32_t kind, const int64_t *ids, int32_t n_ids, int32_t cap, int32_t *voxels,
                   double *dt, int32_t *count) {
    if (!scene || !ids || !voxels || !dt || !count) return fail(SG_E_INVALID, "NULL argument");
    if (kind < 0 || kind > 2) return fail(SG_E_INVALID, "bad trace kind");
    if (n_ids <= 0 || cap <= 0) return fail(SG_E_INVALID, "n_ids and cap must be > 0");
    Scene &s = *scene;
    Ctx *ctx = s.ctx;
    const int64_t lim = kind == SG_TRACE_EDGE ? s.E : (kind == SG_TRACE_SUN ? s.N : s.npx);
    for (int i = 0; i < n_ids; ++i)
        if (ids[i] < 0 || ids[i] >= lim) return fail(SG_E_INVALID, "trace id out of range");
    std::lock_guard<std::mutex> lk(s.mu);
    SG_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    long long *d_ids = nullptr;
    int *d_vox = nullptr, *d_cnt = nullptr;
    double *d_dt = nullptr;
    SG_HIP(hipMalloc((void **)&d_ids, sizeof(long long) * n_ids));
    SG_HIP(hipMalloc((void **)&d_vox, sizeof(int) * (size_t)n_ids * cap));
    SG_HIP(hipMalloc((void **)&d_dt, sizeof(double) * (size_t)n_ids * cap));
    SG_HIP(hipMalloc((void **)&d_cnt, sizeof(int) * n_ids));
    SG_HIP(hipMemcpyAsync(d_ids, ids, sizeof(long long) * n_ids, hipMemcpyHostToDevice, st));
    launch_trace(s, st, kind, d_ids, n_ids, cap, d_vox, d_dt, d_cnt);
    SG_HIP(hipGetLastError());
    SG_HIP(hipMemcpyAsync(voxels, d_vox, sizeof(int) * (size_t)n_ids * cap, hipMemcpyDeviceToHost, st));
    SG_HIP(hipMemcpyAsync(dt, d_dt, sizeof(double) * (size_t)n_ids * cap, hipMemcpyDeviceToHost, st));
    SG_HIP(hipMemcpyAsync(count, d_cnt, sizeof(int) * n_ids, hipMemcpyDeviceToHost, st));
    SG_HIP(hipStreamSynchronize(st));
    (void)hipFree(d_ids);
    (void)hipFree(d_vox);
    (void)hipFree(d_dt);
    (void)hipFree(d_cnt);
    return bounds_report();
}


sg_status sg_debug_bounds(sg_ctx *ctx_, int32_t selftest, int32_t *enabled, uint32_t *site) {
    Ctx *ctx = reinterpret_cast<Ctx *>(ctx_);
    if (!ctx || !enabled || !site) return fail(SG_E_INVALID, "NULL argument");
    *site = 0u;
#ifdef SG_DEBUG_BOUNDS
    *enabled = 1;
    SG_HIP(hipSetDevice(ctx->device));
    if (selftest) {
        launch_bounds_selftest(ctx->stream);
        SG_HIP(hipStreamSynchronize(ctx->stream));
    }
    const sg_status r = bounds_report();
    if (r != SG_OK) {
        const std::string m = t_last_error();
        *site = (uint32_t)std::strtoul(m.substr(m.find("0x")).c_str(), nullptr, 16);
        return SG_OK;
    }
#else
    (void)selftest;
    *enabled = 0;
#endif
    return SG_OK;
}

}  // extern "C"

/*
 * sgoracle.c -- FP64 CPU reference ("oracle") of the scattering-graph hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the GPU
 * path.  It is deliberately plain and slow: straightforward loops in double
 * precision that follow the method's definitions in the paper's order.
 * OpenMP only splits independent items (edges, nodes, rows, pixels) across
 * threads; no sum is reordered by it.
 *
 * Method (Mikkonen et al., "Scattering graph method for 3D radiative
 * transfer"):
 *   - Sec. 2, Eq. 3 (Beer-Lambert-Bouguer): transmittance exp(-int mu_e) of
 *     every graph edge, integrated by an exact voxel traversal (O2 below);
 *   - Sec. 2, Eq. 6 / Eq. 7: flux-matrix element = edge transmittance x the
 *     node's scattering weight x the phase function integrated over the
 *     spherical cell Sigma of the outgoing edge (discretised on a Fibonacci
 *     lattice, Sec. 3);
 *   - Sec. 2, Eq. 9: the direct-solar source; Eq. 8 / Eq. 5: (I - F) phi = S
 *     solved by the Neumann series; Eq. 11: the observed radiance gather.
 * The readings taken where the paper is silent or garbled are listed in the
 * repository's design notes; the ones that change arithmetic are restated at
 * the function that takes them.
 *
 * Notation: a directed edge id is its position in the adjacency CSR (edges
 * sorted by (tail, head)); K is the transpose of the paper's F (row = the
 * destination edge b, column = the source edge a), so that phi = S + K phi.
 *
 * Operation-order contract: the lattice, the unit edge directions, the
 * rotation and the dot products that decide lattice ownership are written
 * with the exact sequence of IEEE operations stated at each function (fma()
 * where named, no contraction elsewhere; compile with -ffp-contract=off).
 * Ownership is an argmax, so both implementations must take it with the same
 * double-precision operations to agree bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FXS 65536LL /* fixed-point units per voxel edge */

#include <time.h>
static double wall_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ==================================================================== */
/* O2: exact voxel traversal of a segment or ray (Sec. 2, Eq. 3 / Eq. 6) */
/* ==================================================================== */

typedef struct {
    int64_t n, d; /* non-negative rational n / d, d > 0 */
} rat;

static int rat_lt(rat a, rat b) { return a.n * b.d < b.n * a.d; }
static int rat_eq(rat a, rat b) { return a.n * b.d == b.n * a.d; }

static int64_t floor_div(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
    return q;
}

/*
 * Walk the voxels that P + t D crosses with positive length, for t in
 * (0, 1] (a node-to-node segment, is_ray = 0) or until the ray leaves the
 * grid (is_ray = 1).  P is fixed point, D integer.  A start point lying on a
 * voxel plane belongs to the voxel the path moves into.  Crossing times
 * (B - P_k) / D_k are compared exactly by cross multiplication; when several
 * axes cross at the same time all of them step together, so no voxel of zero
 * length is reported.  For each voxel the callback receives its linear id
 * (ix + nx (iy + ny iz)) and dt, the parameter length inside it, computed as
 * one correctly rounded division of exact integers.
 * Returns the number of voxels, or -1 when a segment leaves the grid.
 */
typedef void (*visit_fn)(void *ctx, int64_t vox, double dt);

/*
 * Periodic horizontal boundaries (plane-parallel slabs, Sec. 3): with bit 0 (x) or
 * bit 1 (y) of `periodic` set, the medium repeats along that axis with the grid's
 * period.  The walk then keeps its exact crossing times on the unwrapped line, never
 * leaves through that axis, and visits the voxel whose index is wrapped into the grid
 * (ix mod nx); a ray ends only through z.  A walk takes at most MAX_WALK_STEPS voxels
 * (a ray close to horizontal in a clear periodic medium would otherwise run on).
 */
#define MAX_WALK_STEPS 65536

static int64_t wrap_index(int64_t i, int64_t n) {
    const int64_t r = i % n;
    return r < 0 ? r + n : r;
}

static int dda_walk_p(int nx, int ny, int nz, int periodic, const int64_t P[3], const int64_t D[3], int is_ray,
                      visit_fn visit, void *ctx) {
    int64_t n[3] = {nx, ny, nz};
    int64_t idx[3], step[3];
    rat tn[3];
    int active[3];
    for (int k = 0; k < 3; ++k) {
        if (D[k] > 0) {
            idx[k] = floor_div(P[k], FXS);
            step[k] = 1;
            tn[k].n = (idx[k] + 1) * FXS - P[k];
            tn[k].d = D[k];
            active[k] = 1;
        } else if (D[k] < 0) {
            idx[k] = floor_div(P[k] + FXS - 1, FXS) - 1; /* ceil(P / FXS) - 1 */
            step[k] = -1;
            tn[k].n = P[k] - idx[k] * FXS;
            tn[k].d = -D[k];
            active[k] = 1;
        } else {
            idx[k] = floor_div(P[k], FXS);
            step[k] = 0;
            tn[k].n = 0;
            tn[k].d = 1;
            active[k] = 0;
        }
    }
    if (!active[0] && !active[1] && !active[2]) return -1;
    rat tcur = {0, 1};
    const rat tend = {1, 1};
    int count = 0;
    for (;;) {
        int inside = ((periodic & 1) || (idx[0] >= 0 && idx[0] < n[0])) &&
                     ((periodic & 2) || (idx[1] >= 0 && idx[1] < n[1])) && idx[2] >= 0 && idx[2] < n[2];
        if (!inside) {
            if (is_ray) break;
            return -1;
        }
        if (count >= MAX_WALK_STEPS) break;
        rat tmin = {1, 0}; /* +infinity */
        int have = 0;
        for (int k = 0; k < 3; ++k) {
            if (!active[k]) continue;
            if (!have || rat_lt(tn[k], tmin)) {
                tmin = tn[k];
                have = 1;
            }
        }
        int last = 0;
        if (!is_ray && !rat_lt(tmin, tend)) {
            tmin = tend;
            last = 1;
        }
        int64_t num = tmin.n * tcur.d - tcur.n * tmin.d;
        int64_t den = tmin.d * tcur.d;
        double dt = (double)num / (double)den;
        const int64_t wx = (periodic & 1) ? wrap_index(idx[0], nx) : idx[0];
        const int64_t wy = (periodic & 2) ? wrap_index(idx[1], ny) : idx[1];
        visit(ctx, wx + (int64_t)nx * (wy + (int64_t)ny * idx[2]), dt);
        ++count;
        if (last) break;
        for (int k = 0; k < 3; ++k) {
            if (active[k] && rat_eq(tn[k], tmin)) {
                idx[k] += step[k];
                tn[k].n += FXS;
            }
        }
        tcur = tmin;
    }
    return count;
}

static int dda_walk(int nx, int ny, int nz, const int64_t P[3], const int64_t D[3], int is_ray, visit_fn visit,
                    void *ctx) {
    return dda_walk_p(nx, ny, nz, 0, P, D, is_ray, visit, ctx);
}

/* The displacement from node a to node b: b - a, on a periodic axis the shortest of its
   images (the scene guarantees it is shorter than half the period). */
static void node_disp(const int64_t *pos, int64_t a, int64_t b, int nx, int ny, int periodic, int64_t D[3]) {
    for (int k = 0; k < 3; ++k) D[k] = pos[3 * b + k] - pos[3 * a + k];
    const int64_t W[2] = {(int64_t)nx * FXS, (int64_t)ny * FXS};
    for (int k = 0; k < 2; ++k) {
        if (!(periodic & (1 << k))) continue;
        if (2 * D[k] > W[k]) D[k] -= W[k];
        else if (2 * D[k] < -W[k]) D[k] += W[k];
    }
}

typedef struct {
    int64_t *vox;
    double *dt;
    int cap, n;
} trace_buf;

static void trace_visit(void *c, int64_t vox, double dt) {
    trace_buf *b = (trace_buf *)c;
    if (b->n < b->cap) {
        b->vox[b->n] = vox;
        b->dt[b->n] = dt;
    }
    b->n++;
}

/* Exported for the traversal pins: voxel ids and parameter lengths of one walk. */
int or_trace(int nx, int ny, int nz, const int64_t *P, const int64_t *D, int is_ray, int64_t *vox,
             double *dt, int cap) {
    trace_buf b = {vox, dt, cap, 0};
    int r = dda_walk(nx, ny, nz, P, D, is_ray, trace_visit, &b);
    return r < 0 ? r : b.n;
}

/* The same with periodic horizontal axes (bit 0: x, bit 1: y). */
int or_trace_p(int nx, int ny, int nz, int periodic, const int64_t *P, const int64_t *D, int is_ray, int64_t *vox,
               double *dt, int cap) {
    trace_buf b = {vox, dt, cap, 0};
    int r = dda_walk_p(nx, ny, nz, periodic, P, D, is_ray, trace_visit, &b);
    return r < 0 ? r : b.n;
}

/* Many walks at once (for checks of whole scenes): path k starts at P[k] along D[k];
   its voxels and parameter lengths go to vox[k][cap], dt[k][cap] (slots past the path:
   -1 and 0), its voxel count (which may exceed cap) to count[k], or a negative code. */
void or_trace_many(int nx, int ny, int nz, int periodic, int64_t n, const int64_t *P, const int64_t *D,
                   int is_ray, int cap, int64_t *vox, double *dt, int64_t *count) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < n; ++k) {
        trace_buf b = {vox + k * cap, dt + k * cap, cap, 0};
        int r = dda_walk_p(nx, ny, nz, periodic, P + 3 * k, D + 3 * k, is_ray, trace_visit, &b);
        count[k] = r < 0 ? r : b.n;
        for (int j = b.n < cap ? b.n : cap; j < cap; ++j) {
            vox[k * cap + j] = -1;
            dt[k * cap + j] = 0.0;
        }
    }
}

/* The voxel containing a volume node (floor of its fixed-point position; periodic axes
   wrap); -1 outside the box or on its outer planes (z = 0 included: the ground). */
static int64_t node_voxel(const int64_t p[3], int nx, int ny, int nz, int periodic) {
    const int64_t n[3] = {nx, ny, nz};
    int64_t v[3];
    for (int k = 0; k < 3; ++k) {
        int64_t c = p[k];
        if (k < 2 && (periodic & (1 << k))) {
            if (c < 0 || c >= n[k] * FXS) return -1;
        } else if (c <= 0 || c >= n[k] * FXS) {
            return -1;
        }
        v[k] = c / FXS;
    }
    return v[0] + (int64_t)nx * (v[1] + (int64_t)ny * v[2]);
}

/*
 * Path points of the lines of sight (Sec. 2: the points of a line of sight are taken at
 * constant distance intervals or at each layer of the medium; Sec. 3, step 1 of the
 * algorithm).  Pixel p = i + nx j looks from its surface point P = ((i + 1/2), (j + 1/2),
 * 0) voxels along the view direction D until the line leaves the grid; the exact walk
 * splits it into voxel chords k of parameter length dt_k (t = 1 is one D), starting at
 * t_k = dt_0 + ... + dt_(k-1) (summed in this order) and ending at t_exit.  The line is cut
 * into elements [a, b]:
 *   mode 0 (layers): one per layer of voxels it crosses, from the start of the layer's
 *     first chord to the end of its last (D_z > 0: a layer's chords are consecutive);
 *   mode 1 (constant step): [j h, min((j + 1) h, t_exit)] for j = 0, 1, ... while
 *     j h < t_exit, h = step_m / (|D| voxel_m / 2^16) (the step in parameter units).
 * Element [a, b] has a node at the rounded middle point: m = 0.5 (a + b), pos_c = P_c +
 * floor(m D_c + 0.5) on each axis, wrapped into the period on periodic axes; a node outside
 * the box or on its outer planes is not made (the element then carries -1).  Node ids follow
 * the pixels, then the elements in order.  Outputs: pos [cap][3]; los_ptr [nx ny + 1]: pixel
 * p's elements at los_ptr[p] ...; per element its node los_node and its end b in los_t
 * [el_cap]; counts[0] = nodes, counts[1] = elements.  Returns 0, 1 when a capacity is too
 * small (the counts are still written), or -1 for a bad argument.
 */
typedef struct {
    int64_t *vox;
    double *dt;
    int64_t n, cap;
} chord_buf;

static void chord_visit(void *c, int64_t vox, double dt) {
    chord_buf *b = (chord_buf *)c;
    if (b->n < b->cap) {
        b->vox[b->n] = vox;
        b->dt[b->n] = dt;
    }
    b->n++;
}

int or_los_nodes(int nx, int ny, int nz, int periodic, const int64_t *view_dir, double voxel_m, int mode,
                 double step_m, int64_t *pos, int64_t cap, int64_t *los_ptr, int32_t *los_node, double *los_t,
                 int64_t el_cap, int64_t *counts) {
    if (view_dir[2] <= 0 || (mode != 0 && mode != 1) || (mode == 1 && !(step_m > 0.0))) return -1;
    const int64_t npx = (int64_t)nx * ny;
    const int wcap = periodic ? MAX_WALK_STEPS : nx + ny + nz + 2;
    int64_t *vox = (int64_t *)malloc(sizeof(int64_t) * wcap);
    double *dt = (double *)malloc(sizeof(double) * wcap);
    int64_t icap = wcap + 1; /* element arrays, grown for short steps */
    double *ia = (double *)malloc(sizeof(double) * icap), *ib = (double *)malloc(sizeof(double) * icap);
    const double plen = sqrt((double)(view_dir[0] * view_dir[0] + view_dir[1] * view_dir[1] + view_dir[2] * view_dir[2])) *
                        (voxel_m / (double)FXS);
    const double h = mode == 1 ? step_m / plen : 0.0;
    int64_t nn = 0, ne = 0;
    los_ptr[0] = 0;
    for (int64_t p = 0; p < npx; ++p) {
        const int64_t P[3] = {(p % nx) * FXS + FXS / 2, (p / nx) * FXS + FXS / 2, 0};
        chord_buf cb = {vox, dt, 0, wcap};
        dda_walk_p(nx, ny, nz, periodic, P, view_dir, 1, chord_visit, &cb);
        const int64_t nk = cb.n;
        int64_t ni = 0;
        if (mode == 0) {
            int64_t layer = -1;
            double t = 0.0;
            for (int64_t k = 0; k < nk; ++k) {
                const int64_t z = vox[k] / npx;
                if (z != layer) {
                    layer = z;
                    ia[ni] = t;
                    ++ni;
                }
                t = t + dt[k];
                ib[ni - 1] = t;
            }
        } else {
            double t_exit = 0.0;
            for (int64_t k = 0; k < nk; ++k) t_exit = t_exit + dt[k];
            while ((double)ni * h < t_exit) {
                if (ni == icap) {
                    icap *= 2;
                    ia = (double *)realloc(ia, sizeof(double) * icap);
                    ib = (double *)realloc(ib, sizeof(double) * icap);
                }
                ia[ni] = (double)ni * h;
                const double e = (double)(ni + 1) * h;
                ib[ni] = e < t_exit ? e : t_exit;
                ++ni;
            }
        }
        for (int64_t j = 0; j < ni; ++j) {
            const double m = 0.5 * (ia[j] + ib[j]);
            int64_t q[3];
            for (int c = 0; c < 3; ++c) {
                q[c] = P[c] + (int64_t)floor(m * (double)view_dir[c] + 0.5);
                if (c < 2 && (periodic & (1 << c))) {
                    const int64_t W = (c ? ny : nx) * (int64_t)FXS;
                    q[c] = ((q[c] % W) + W) % W;
                }
            }
            int32_t id = -1;
            if (node_voxel(q, nx, ny, nz, periodic) >= 0) {
                id = (int32_t)nn;
                if (nn < cap)
                    for (int c = 0; c < 3; ++c) pos[3 * nn + c] = q[c];
                ++nn;
            }
            if (ne + j < el_cap) {
                los_node[ne + j] = id;
                los_t[ne + j] = ib[j];
            }
        }
        ne += ni;
        los_ptr[p + 1] = ne;
    }
    free(vox); free(dt); free(ia); free(ib);
    counts[0] = nn;
    counts[1] = ne;
    return nn > cap || ne > el_cap ? 1 : 0;
}

typedef struct {
    const double *mu_e;
    double tau; /* accumulated sum of mu_e * dt (dt in parameter units) */
} tau_acc;

static void tau_visit(void *c, int64_t vox, double dt) {
    tau_acc *a = (tau_acc *)c;
    a->tau += a->mu_e[vox] * dt;
}

/* Length in metres of the whole parameter interval t in [0, 1] of direction D. */
static double param_length_m(const int64_t D[3], double voxel_m) {
    int64_t s = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
    return sqrt((double)s) * (voxel_m / (double)FXS);
}

/* Optical depth along a segment (is_ray = 0) or a ray to the grid exit. */
static double optical_depth(int nx, int ny, int nz, int periodic, const double *mu_e, double voxel_m,
                            const int64_t P[3], const int64_t D[3], int is_ray) {
    tau_acc a = {mu_e, 0.0};
    dda_walk_p(nx, ny, nz, periodic, P, D, is_ray, tau_visit, &a);
    return a.tau * param_length_m(D, voxel_m);
}

/* ==================================================================== */
/* O3-O5: directions, phase function, Fibonacci lattice, ownership       */
/* ==================================================================== */

/* Henyey-Greenstein phase function, normalised to 1 over the sphere. */
static double hg(double g, double mu) {
    double den = 1.0 + g * g - 2.0 * g * mu;
    return (1.0 - g * g) / (4.0 * M_PI * den * sqrt(den));
}

/*
 * Fibonacci lattice (Sec. 3, phase integration; spherical Fibonacci point set
 * with the golden angle): z_i = 1 - (2i + 1) / N, phi_i = (i * ga) mod 2 pi
 * with ga = pi (3 - sqrt 5), p_i = (r cos phi_i, r sin phi_i, z_i),
 * r = sqrt(1 - z_i * z_i).  Written as that exact operation sequence.
 */
void or_lattice(int N, double *p /* [N][3] */) {
    const double ga = M_PI * (3.0 - sqrt(5.0));
    const double two_pi = 2.0 * M_PI;
    for (int i = 0; i < N; ++i) {
        double z = 1.0 - (2.0 * (double)i + 1.0) / (double)N;
        double phi = fmod((double)i * ga, two_pi);
        double r = sqrt(1.0 - z * z);
        p[3 * i + 0] = r * cos(phi);
        p[3 * i + 1] = r * sin(phi);
        p[3 * i + 2] = z;
    }
}

/* Normalised lattice table of one HG component: Theta(z_i) / sum_j Theta(z_j). */
void or_hg_table(double g, int N, const double *p, double *t) {
    double s = 0.0;
    for (int i = 0; i < N; ++i) {
        t[i] = hg(g, p[3 * i + 2]);
        s += t[i];
    }
    for (int i = 0; i < N; ++i) t[i] = t[i] / s;
}

/* Unit vector of an integer direction: D / sqrt(Dx^2 + Dy^2 + Dz^2). */
static void unit_of(const int64_t D[3], double u[3]) {
    double nrm = sqrt((double)(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]));
    u[0] = (double)D[0] / nrm;
    u[1] = (double)D[1] / nrm;
    u[2] = (double)D[2] / nrm;
}

/*
 * Rotation taking the unit vector u to +z (the forward direction onto the
 * table's theta = 0 axis, Sec. 3): the minimal rotation about u x z,
 *   R = c I + [w]x + w w^T / (1 + c),  c = u_z,  w = (u_y, -u_x, 0),
 * entry by entry with h = 1 / (1 + c); for 1 + c < 1e-12, R = diag(1, -1, -1).
 */
void or_rotation(const double u[3], double R[9]) {
    double c = u[2];
    if (1.0 + c < 1e-12) {
        R[0] = 1.0; R[1] = 0.0;  R[2] = 0.0;
        R[3] = 0.0; R[4] = -1.0; R[5] = 0.0;
        R[6] = 0.0; R[7] = 0.0;  R[8] = -1.0;
        return;
    }
    double h = 1.0 / (1.0 + c);
    double ux = u[0], uy = u[1];
    double xy = (ux * uy) * h;
    R[0] = c + (uy * uy) * h; R[1] = -xy;               R[2] = -ux;
    R[3] = -xy;               R[4] = c + (ux * ux) * h; R[5] = -uy;
    R[6] = ux;                R[7] = uy;                R[8] = c;
}

/* q = R^T p, each component as fma(R2k, p2, fma(R1k, p1, R0k * p0)). */
static void rot_apply_t(const double R[9], const double p[3], double q[3]) {
    for (int k = 0; k < 3; ++k) q[k] = fma(R[6 + k], p[2], fma(R[3 + k], p[1], R[k] * p[0]));
}

/* q . s as fma(q2, s2, fma(q1, s1, q0 * s0)). */
static double dot3(const double q[3], const double s[3]) {
    return fma(q[2], s[2], fma(q[1], s[1], q[0] * s[0]));
}

/*
 * Lattice ownership (Eq. 7 and the definition of Sigma after it): with the
 * lattice rotated so that its pole is the incoming propagation direction u,
 * lattice point i belongs to the outgoing direction m with the largest
 * p_i . (R(u) s_m), evaluated as q_i . s_m with q_i = R(u)^T p_i (the same
 * dot product; u == NULL: no rotation, the Lambertian surface case).  Ties
 * go to the smallest m, which also drops a second coupling in exactly the
 * same direction.
 */
void or_ownership(const double *u, int d, const double *s /* [d][3] */, int N, const double *p,
                  int32_t *own) {
    double R[9];
    if (u) or_rotation(u, R);
    for (int i = 0; i < N; ++i) {
        double q[3];
        if (u) rot_apply_t(R, p + 3 * i, q);
        else memcpy(q, p + 3 * i, sizeof q);
        int best = -1;
        double bv = 0.0;
        for (int m = 0; m < d; ++m) {
            double v = dot3(q, s + 3 * m);
            if (best < 0 || v > bv) {
                best = m;
                bv = v;
            }
        }
        own[i] = best;
    }
}

/* ==================================================================== */
/* The scene and the full pipeline                                       */
/* ==================================================================== */

typedef struct {
    int nx, ny, nz;
    double voxel_m;
    const double *mu_s, *mu_a; /* [nvox] in 1/m (mu_a already multiplied by the wavelength scale) */
    int n_phase;
    const double *hg_g;       /* [n_phase] */
    const double *phase_frac; /* [n_phase][nvox] or NULL */
    const int64_t *pos;       /* [N][3] every node, volume then surface */
    int surface;
    const int64_t *adj_ptr; /* [N+1] */
    const int32_t *adj_idx; /* [E] */
    const double *albedo;   /* [ny][nx] */
    const int64_t *sun_dir; /* [3] toward the sun */
    const int64_t *view_dir;/* [3] toward the sensor */
    int n_fib;
    int node_weight_mode;
    int scatter_order; /* 0 = multiple scattering, 1 = single scattering only */
    double tol;        /* target of the solve: L1 update / ||S||_1, and 10 tol per edge (relative) */
    const int *phase_kind; /* [n_phase] 0 Henyey-Greenstein, 1 Rayleigh, 2 table; NULL: all 0 */
    int lut_n;             /* samples per table row */
    const double *lut;     /* [n_phase][lut_n] tables in mu = cos(theta) on [-1, 1] */
    int sigma_mode;        /* 0: Voronoi ownership of the lattice; 1: nearest-point colouring + flood fill */
    int periodic;          /* bit 0: periodic in x, bit 1: periodic in y (plane-parallel slabs) */
    /* Volume nodes.  n_vol = 0: one per voxel, node id = voxel id (pos [nvox] first).
       n_vol > 0: n_vol nodes anywhere in the box (pos [n_vol] first; Sec. 2: the path points
       of the lines of sight), each with the medium of the voxel that contains it; pixel p's
       line of sight is then cut into elements e = los_ptr[p] ... los_ptr[p+1]-1, consecutive
       from its surface point up to the parameters los_t[e] (t = 1 is one view_dir), element e
       scattering toward the sensor the radiance of volume node los_node[e] (-1: none). */
    int64_t n_vol;
    const int64_t *los_ptr; /* [nx*ny + 1] */
    const int32_t *los_node;
    const double *los_t;
} or_scene;

/*
 * Phase-function components (Sec. 3: Rayleigh scattering, or a particle phase
 * function given as a look-up table), each normalised over the sphere.  A table
 * holds samples at mu_m = -1 + 2 m / (n - 1), linear in mu between them; its
 * interpolant integrates over the sphere to 2 pi x the trapezoid rule in mu.
 */
double or_table_integral(const double *row, int n) {
    double sum = 0.0;
    for (int m = 0; m < n; ++m) sum += row[m];
    return (2.0 * M_PI) * ((2.0 / (double)(n - 1)) * (sum - 0.5 * (row[0] + row[n - 1])));
}

double or_phase_value(int kind, double g, const double *row, int n, double mu) {
    if (kind == 1) return (3.0 / (16.0 * M_PI)) * (1.0 + mu * mu);
    if (kind == 2) {
        const double x = (mu + 1.0) * (0.5 * (double)(n - 1));
        int m = (int)floor(x);
        if (m < 0) m = 0;
        if (m > n - 2) m = n - 2;
        const double f = x - (double)m;
        return (row[m] * (1.0 - f) + row[m + 1] * f) / or_table_integral(row, n);
    }
    return hg(g, mu);
}

static double phase_of(const or_scene *sc, int c, double mu) {
    const int kind = sc->phase_kind ? sc->phase_kind[c] : 0;
    return or_phase_value(kind, sc->hg_g[c], sc->lut ? sc->lut + (size_t)c * sc->lut_n : NULL, sc->lut_n, mu);
}

typedef struct {
    double *tau;      /* [E]   optical depth of the edge's pair (lower id -> higher id) */
    double *tau_sun;  /* [N]   node -> sun, to the grid exit */
    double *rho;      /* [N]   node weight */
    int64_t *row_ptr; /* [E+1] */
    int32_t *col;     /* [nnz] */
    double *val;      /* [nnz] */
    double *S;        /* [E] */
    double *phi;      /* [E] */
    double *pix;      /* [ny*nx] radiance / F0 */
    double *stats;    /* [8]: sweeps, relative residual, used GMRES, GMRES iterations, then the
                         seconds of the marches, the matrix, the solve and the gather */
} or_out;

static int64_t edge_rev(const or_scene *sc, int64_t e, int64_t tail) {
    int64_t head = sc->adj_idx[e];
    int64_t lo = sc->adj_ptr[head], hi = sc->adj_ptr[head + 1];
    while (lo < hi) { /* first position with adj_idx >= tail */
        int64_t mid = (lo + hi) / 2;
        if (sc->adj_idx[mid] < tail) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static int64_t tail_of(const int64_t *adj_ptr, int64_t N, int64_t e) {
    int64_t lo = 0, hi = N; /* last node with adj_ptr[node] <= e */
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) / 2;
        if (adj_ptr[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

/* ---- O8 solve helpers ---- */

/* y = S + K x (one Jacobi / Neumann sweep, Eq. 5). */
static void sweep(int64_t E, const int64_t *rp, const int32_t *col, const double *val, const double *S,
                  const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < E; ++b) {
        double acc = 0.0;
        for (int64_t q = rp[b]; q < rp[b + 1]; ++q) acc += val[q] * x[col[q]];
        y[b] = S[b] + acc;
    }
}

static double norm1(int64_t n, const double *v) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += fabs(v[i]);
    return s;
}

static double norm2(int64_t n, const double *v) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += v[i] * v[i];
    return sqrt(s);
}

/* r = S - (I - K) x */
static void residual(int64_t E, const int64_t *rp, const int32_t *col, const double *val, const double *S,
                     const double *x, double *r) {
    sweep(E, rp, col, val, S, x, r);
    for (int64_t b = 0; b < E; ++b) r[b] -= x[b];
}

/* Restarted GMRES(m) with modified Gram-Schmidt and Givens rotations on (I - K) x = S. */
static int gmres(int64_t E, const int64_t *rp, const int32_t *col, const double *val, const double *S,
                 double *x, int m, double tol, int max_iter, double *relres) {
    double *V = (double *)malloc(sizeof(double) * (size_t)E * (m + 1));
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = (double *)malloc(sizeof(double) * m), *sn = (double *)malloc(sizeof(double) * m);
    double *g = (double *)malloc(sizeof(double) * (m + 1)), *yv = (double *)malloc(sizeof(double) * m);
    double *w = (double *)malloc(sizeof(double) * E), *zero = (double *)calloc(E, sizeof(double));
    double nS1 = norm1(E, S);
    int it = 0;
    for (;;) {
        residual(E, rp, col, val, S, x, w);
        double r1 = norm1(E, w);
        *relres = nS1 > 0 ? r1 / nS1 : 0.0;
        if (*relres <= tol || it >= max_iter) break;
        double beta = norm2(E, w);
        for (int64_t i = 0; i < E; ++i) V[i] = w[i] / beta;
        memset(g, 0, sizeof(double) * (m + 1));
        g[0] = beta;
        int k;
        for (k = 0; k < m && it < max_iter; ++k, ++it) {
            double *vk = V + (size_t)k * E, *vn = V + (size_t)(k + 1) * E;
            /* vn = (I - K) vk = vk - K vk */
            sweep(E, rp, col, val, zero, vk, vn);
            for (int64_t i = 0; i < E; ++i) vn[i] = vk[i] - vn[i];
            for (int j = 0; j <= k; ++j) {
                double *vj = V + (size_t)j * E;
                double h = 0.0;
                for (int64_t i = 0; i < E; ++i) h += vn[i] * vj[i];
                H[j * m + k] = h;
                for (int64_t i = 0; i < E; ++i) vn[i] -= h * vj[i];
            }
            double hn = norm2(E, vn);
            H[(k + 1) * m + k] = hn;
            if (hn > 0) for (int64_t i = 0; i < E; ++i) vn[i] /= hn;
            for (int j = 0; j < k; ++j) {
                double a = H[j * m + k], b = H[(j + 1) * m + k];
                H[j * m + k] = cs[j] * a + sn[j] * b;
                H[(j + 1) * m + k] = -sn[j] * a + cs[j] * b;
            }
            double a = H[k * m + k], b = H[(k + 1) * m + k];
            double den = sqrt(a * a + b * b);
            cs[k] = den > 0 ? a / den : 1.0;
            sn[k] = den > 0 ? b / den : 0.0;
            H[k * m + k] = den;
            H[(k + 1) * m + k] = 0.0;
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            if (fabs(g[k + 1]) <= 1e-3 * tol * beta) { ++k; ++it; break; }
        }
        for (int j = k - 1; j >= 0; --j) {
            double s = g[j];
            for (int q = j + 1; q < k; ++q) s -= H[j * m + q] * yv[q];
            yv[j] = s / H[j * m + j];
        }
        for (int j = 0; j < k; ++j) {
            double *vj = V + (size_t)j * E;
            for (int64_t i = 0; i < E; ++i) x[i] += yv[j] * vj[i];
        }
    }
    free(V); free(H); free(cs); free(sn); free(g); free(yv); free(w); free(zero);
    return it;
}

/*
 * O8: phi = (I - K)^-1 S (Eq. 8), by the Neumann series x <- S + K x (Eq. 5);
 * y - x is the residual S - (I - K) x of the previous iterate.  Stops when its
 * L1 norm is below tol ||S||_1 and no edge changes by more than 10 tol of its
 * value.  Falls back to GMRES(50) when the L1 sweep ratio reaches 0.99, the
 * residual grows, or 5000 sweeps pass.  stats: sweeps, final relative 1-norm residual, GMRES used,
 * GMRES iterations.
 */
int or_solve(int64_t E, const int64_t *rp, const int32_t *col, const double *val, const double *S,
             double tol, double *phi, double *stats) {
    double *x = (double *)calloc(E > 0 ? E : 1, sizeof(double));
    double *y = (double *)malloc(sizeof(double) * (E > 0 ? E : 1));
    double nS = norm1(E, S);
    int sweeps = 0, use_gmres = 0;
    double prev = -1.0, rel = 0.0;
    if (nS == 0.0) {
        memset(phi, 0, sizeof(double) * E);
        stats[0] = 0; stats[1] = 0; stats[2] = 0; stats[3] = 0;
        free(x); free(y);
        return 0;
    }
    for (;;) {
        sweep(E, rp, col, val, S, x, y);
        ++sweeps;
        /* two measures of the update: L1 relative to ||S||_1, and the largest relative
           update of a single edge, which also resolves edges far darker than the mean */
        double r = 0.0, mr = 0.0;
        for (int64_t i = 0; i < E; ++i) {
            double d = fabs(y[i] - x[i]);
            r += d;
            mr = fmax(mr, d / (fabs(y[i]) + 1e-200));
        }
        rel = r / nS;
        memcpy(x, y, sizeof(double) * E);
        if (rel <= tol && mr <= 10.0 * tol) break;
        /* stall test on the L1 measure, which contracts monotonically */
        if (rel > tol && prev > 0 && (rel / prev >= 0.99 || rel > prev)) { use_gmres = 1; break; }
        if (sweeps >= 5000) { use_gmres = 1; break; }
        prev = rel;
    }
    int git = 0;
    if (use_gmres) git = gmres(E, rp, col, val, S, x, 50, tol, 20000, &rel);
    else {
        /* rel above is the residual of the iterate before the last sweep; report the final one */
        residual(E, rp, col, val, S, x, y);
        rel = norm1(E, y) / nS;
    }
    memcpy(phi, x, sizeof(double) * E);
    stats[0] = sweeps; stats[1] = rel; stats[2] = use_gmres; stats[3] = git;
    free(x); free(y);
    return 0;
}

/* Number of structural nonzeros sum_l d_l^2 of K. */
int64_t or_nnz(int64_t N, const int64_t *adj_ptr) {
    int64_t s = 0;
    for (int64_t l = 0; l < N; ++l) {
        int64_t d = adj_ptr[l + 1] - adj_ptr[l];
        s += d * d;
    }
    return s;
}

/*
 * Phase-cell weights of one node for one incoming direction (Eq. 7):
 * Q[m] = sum_k f_k sum_{i : own(i) = m} Theta~_k(i)   (volume node, rotation by u)
 * Q[m] = sum_{i : own(i) = m} max(0, z_i) / sum_j max(0, z_j)   (surface node, u ignored)
 */
static void node_q(int is_surface, const double *u, int d, const double *s, int N, const double *lat,
                   const double *w /* [N] mixed table, volume only */, double *Q, int32_t *own) {
    or_ownership(is_surface ? NULL : u, d, s, N, lat, own);
    for (int m = 0; m < d; ++m) Q[m] = 0.0;
    if (is_surface) {
        double tot = 0.0;
        for (int i = 0; i < N; ++i) tot += fmax(0.0, lat[3 * i + 2]);
        for (int i = 0; i < N; ++i) Q[own[i]] += fmax(0.0, lat[3 * i + 2]) / tot;
    } else {
        for (int i = 0; i < N; ++i) Q[own[i]] += w[i];
    }
}

/* Exported for the phase-cell pins. */
/*
 * The paper's own discretisation of Sigma (Sec. 3): each out-edge direction,
 * rotated with the lattice, colours its closest lattice point, and the colours
 * are spread over the rest of the lattice by flood fill along the edges of the
 * lattice's convex hull.
 *
 * Hull edges: (i, j) is an edge when some k makes (i, j, k) a face, i.e. no lattice
 * point lies strictly on each side of the plane through p_i, p_j, p_k:
 *   d1 = p_j - p_i, d2 = p_k - p_i, n = d1 x d2 (components (d1y d2z - d1z d2y,
 *   d1z d2x - d1x d2z, d1x d2y - d1y d2x)), s_l = (n_x e_x + n_y e_y) + n_z e_z with
 *   e = p_l - p_i (no contraction); coplanar points do not count against a face,
 *   so both diagonals of a coplanar quadrilateral are edges.  Below 4 points every
 *   pair is an edge.  Lists ascending; returns the largest degree (-1 above maxnb).
 */
int or_hull_adjacency(int N, const double *p, int maxnb, int32_t *nb /* [N][maxnb] */, int32_t *nnb /* [N] */) {
    unsigned char *adj = (unsigned char *)calloc((size_t)N * N, 1);
    if (N < 4) {
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) adj[(size_t)i * N + j] = i != j;
    } else {
        for (int i = 0; i < N; ++i)
            for (int j = i + 1; j < N; ++j)
                for (int k = j + 1; k < N; ++k) {
                    double d1[3], d2[3], n[3];
                    for (int a = 0; a < 3; ++a) {
                        d1[a] = p[3 * j + a] - p[3 * i + a];
                        d2[a] = p[3 * k + a] - p[3 * i + a];
                    }
                    n[0] = d1[1] * d2[2] - d1[2] * d2[1];
                    n[1] = d1[2] * d2[0] - d1[0] * d2[2];
                    n[2] = d1[0] * d2[1] - d1[1] * d2[0];
                    int pos = 0, neg = 0;
                    for (int l = 0; l < N && !(pos && neg); ++l) {
                        if (l == i || l == j || l == k) continue;
                        const double e0 = p[3 * l] - p[3 * i], e1 = p[3 * l + 1] - p[3 * i + 1],
                                     e2 = p[3 * l + 2] - p[3 * i + 2];
                        const double sl = (n[0] * e0 + n[1] * e1) + n[2] * e2;
                        if (sl > 0.0) pos = 1;
                        else if (sl < 0.0) neg = 1;
                    }
                    if (pos && neg) continue;
                    adj[(size_t)i * N + j] = adj[(size_t)j * N + i] = 1;
                    adj[(size_t)i * N + k] = adj[(size_t)k * N + i] = 1;
                    adj[(size_t)j * N + k] = adj[(size_t)k * N + j] = 1;
                }
    }
    int dmax = 0;
    for (int i = 0; i < N; ++i) {
        int c = 0;
        for (int j = 0; j < N; ++j)
            if (adj[(size_t)i * N + j]) {
                if (c < maxnb) nb[(size_t)i * maxnb + c] = j;
                ++c;
            }
        nnb[i] = c < maxnb ? c : maxnb;
        if (c > dmax) dmax = c;
    }
    free(adj);
    return dmax <= maxnb ? dmax : -1;
}

/*
 * Colours of one node and incoming direction: seeds, then flood fill.
 *   seeds: for m = 0, 1, ...: the closest lattice point i*(m) = argmax_i v_im (the
 *   same v_im = q_i . s_m as the Voronoi ownership; ties to the lowest i) takes
 *   colour m, unless an earlier direction claimed it with a value >= v (a point
 *   claimed twice goes to the closer direction, ties to the lower index; the other
 *   direction then owns no lattice point);
 *   fill: in synchronous rounds, every uncoloured point takes the colour of its
 *   coloured neighbour of lowest index (colours of the previous round), until every
 *   point is coloured.
 * The paper gives no rule for conflicts or for several coloured neighbours; these
 * are the readings taken.
 */
static void colour_points(const double *u, int d, const double *s, int N, const double *p, const int32_t *nb,
                          const int32_t *nnb, int maxnb, int32_t *col) {
    double R[9];
    if (u) or_rotation(u, R);
    double *q = (double *)malloc(sizeof(double) * 3 * N), *cv = (double *)malloc(sizeof(double) * N);
    int32_t *snap = (int32_t *)malloc(sizeof(int32_t) * N);
    for (int i = 0; i < N; ++i) {
        if (u) rot_apply_t(R, p + 3 * i, q + 3 * i);
        else memcpy(q + 3 * i, p + 3 * i, sizeof(double) * 3);
        col[i] = -1;
        cv[i] = 0.0;
    }
    for (int m = 0; m < d; ++m) {
        int bi = 0;
        double bv = dot3(q, s + 3 * m);
        for (int i = 1; i < N; ++i) {
            const double v = dot3(q + 3 * i, s + 3 * m);
            if (v > bv) {
                bv = v;
                bi = i;
            }
        }
        if (col[bi] < 0 || bv > cv[bi]) {
            col[bi] = m;
            cv[bi] = bv;
        }
    }
    for (int round = 0; round < N; ++round) {
        int missing = 0;
        memcpy(snap, col, sizeof(int32_t) * N);
        for (int i = 0; i < N; ++i) {
            if (snap[i] >= 0) continue;
            for (int t = 0; t < nnb[i]; ++t) {
                const int j = nb[(size_t)i * maxnb + t];
                if (snap[j] >= 0) {
                    col[i] = snap[j];
                    break;
                }
            }
            missing += col[i] < 0;
        }
        if (!missing) break;
    }
    free(q);
    free(cv);
    free(snap);
}

static void colour_q(int is_surface, const double *u, int d, const double *s, int N, const double *lat,
                     const int32_t *nb, const int32_t *nnb, int maxnb, const double *w, double *Q, int32_t *col) {
    colour_points(is_surface ? NULL : u, d, s, N, lat, nb, nnb, maxnb, col);
    for (int m = 0; m < d; ++m) Q[m] = 0.0;
    double tot = 0.0;
    if (is_surface)
        for (int i = 0; i < N; ++i) tot += fmax(0.0, lat[3 * i + 2]);
    for (int i = 0; i < N; ++i) {
        if (col[i] < 0) continue;
        Q[col[i]] += is_surface ? fmax(0.0, lat[3 * i + 2]) / tot : w[i];
    }
}

/* Colours of one incoming direction, for the pins (u == NULL: no rotation). */
int or_colours(const double *u, int d, const double *s, int N, int maxnb, int32_t *col) {
    double *lat = (double *)malloc(sizeof(double) * 3 * N);
    int32_t *nb = (int32_t *)malloc(sizeof(int32_t) * (size_t)N * maxnb), *nnb = (int32_t *)malloc(sizeof(int32_t) * N);
    or_lattice(N, lat);
    const int dm = or_hull_adjacency(N, lat, maxnb, nb, nnb);
    if (dm >= 0) colour_points(u, d, s, N, lat, nb, nnb, maxnb, col);
    free(lat);
    free(nb);
    free(nnb);
    return dm;
}

void or_node_q(int is_surface, const double *u, int d, const double *s, int N, const double *w, double *Q) {
    double *lat = (double *)malloc(sizeof(double) * 3 * N);
    int32_t *own = (int32_t *)malloc(sizeof(int32_t) * N);
    or_lattice(N, lat);
    node_q(is_surface, u, d, s, N, lat, w, Q, own);
    free(lat);
    free(own);
}

/*
 * The whole pipeline: O2 transmittances, O5 cells, O6 weights, O7 matrix and
 * source, O8 solve, O9 gather.  Returns 0, or a negative value on an invalid
 * scene (a segment leaving the grid).
 */
int or_run(const or_scene *sc, or_out *out) {
    const int nx = sc->nx, ny = sc->ny, nz = sc->nz;
    const int64_t nvox = (int64_t)nx * ny * nz;
    const int64_t nvol = sc->n_vol > 0 ? sc->n_vol : nvox;
    const int64_t N = nvol + (sc->surface ? (int64_t)nx * ny : 0);
    const int64_t E = sc->adj_ptr[N];
    const double dx = sc->voxel_m;
    const int NF = sc->n_fib;
    /* the Lambertian cells need a lattice point above the surface: with one point,
       z_0 = 1 - 1/N = 0 lies on the horizon and the cosine weights are 0 / 0 */
    if (NF < 2) return 8;
    /* periodic axes: only x and y; every node-to-node displacement must have a unique
       shortest image (|D_k| != half the period), and the sun and view rays must reach the
       top within the walk's step limit: a ray from height z crosses at most nz z-planes
       and nz |D_x| / D_z + 1 x-planes (y alike), so the bound below covers every start */
    if (sc->periodic & ~3) return 9;
    if (sc->periodic) {
        const int64_t W[2] = {(int64_t)nx * FXS, (int64_t)ny * FXS};
        for (int64_t l = 0; l < N; ++l)
            for (int64_t e = sc->adj_ptr[l]; e < sc->adj_ptr[l + 1]; ++e) {
                int64_t D[3];
                node_disp(sc->pos, l, sc->adj_idx[e], nx, ny, sc->periodic, D);
                for (int k = 0; k < 2; ++k)
                    if ((sc->periodic & (1 << k)) && 2 * (D[k] < 0 ? -D[k] : D[k]) == W[k]) return 9;
            }
        for (int r = 0; r < 2; ++r) {
            const int64_t *d = r ? sc->view_dir : sc->sun_dir;
            const int64_t ax = d[0] < 0 ? -d[0] : d[0], ay = d[1] < 0 ? -d[1] : d[1];
            if (d[2] <= 0 || (int64_t)nz * (ax + ay + d[2]) + 4 * d[2] > (int64_t)MAX_WALK_STEPS * d[2]) return 9;
        }
    }

    /* the voxel of every volume node; general nodes come with their lines of sight */
    int64_t *nv = (int64_t *)malloc(sizeof(int64_t) * (nvol > 0 ? nvol : 1));
    for (int64_t l = 0; l < nvol; ++l) {
        nv[l] = sc->n_vol > 0 ? node_voxel(sc->pos + 3 * l, nx, ny, nz, sc->periodic) : l;
        if (nv[l] < 0) { free(nv); return 10; }
    }
    if (sc->n_vol > 0) {
        if (!sc->los_ptr || !sc->los_node || !sc->los_t || sc->los_ptr[0] != 0) { free(nv); return 11; }
        for (int64_t p = 0; p < (int64_t)nx * ny; ++p) {
            if (sc->los_ptr[p + 1] < sc->los_ptr[p]) { free(nv); return 11; }
            double prev = 0.0;
            for (int64_t e = sc->los_ptr[p]; e < sc->los_ptr[p + 1]; ++e) {
                if (!(sc->los_t[e] > prev) || !isfinite(sc->los_t[e])) { free(nv); return 11; }
                if (sc->los_node[e] < -1 || sc->los_node[e] >= nvol) { free(nv); return 11; }
                prev = sc->los_t[e];
            }
        }
    }

    /* wall time of the stages, for the benchmark's CPU baseline (stats[4..7]) */
    const double t_start = wall_s();

    /* O0: extinction and single-scattering albedo of each voxel */
    double *mu_e = (double *)malloc(sizeof(double) * nvox);
    double *omega = (double *)malloc(sizeof(double) * nvox);
    for (int64_t v = 0; v < nvox; ++v) {
        mu_e[v] = sc->mu_s[v] + sc->mu_a[v];
        omega[v] = mu_e[v] > 0.0 ? sc->mu_s[v] / mu_e[v] : 0.0;
    }

    /* O2: edge optical depth, from the lower to the higher node id (shared by both directions) */
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t l = 0; l < N; ++l) {
        for (int64_t e = sc->adj_ptr[l]; e < sc->adj_ptr[l + 1]; ++e) {
            int64_t j = sc->adj_idx[e];
            int64_t a = l < j ? l : j, b = l < j ? j : l;
            int64_t P[3], D[3];
            for (int k = 0; k < 3; ++k) P[k] = sc->pos[3 * a + k];
            node_disp(sc->pos, a, b, nx, ny, sc->periodic, D);
            tau_acc acc = {mu_e, 0.0};
            if (dda_walk_p(nx, ny, nz, sc->periodic, P, D, 0, tau_visit, &acc) < 0) bad = 1;
            out->tau[e] = acc.tau * param_length_m(D, dx);
        }
    }
    if (bad) { free(mu_e); free(omega); free(nv); return -2; }

    /* O2: node -> sun optical depth to the grid exit */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t l = 0; l < N; ++l) {
        out->tau_sun[l] = optical_depth(nx, ny, nz, sc->periodic, mu_e, dx, sc->pos + 3 * l, sc->sun_dir, 1);
    }

    /* O6: node weights (bounded scattering probability over one voxel edge; mode 1: mu_s * edge) */
    for (int64_t l = 0; l < N; ++l) {
        if (l < nvol) {
            const int64_t v = nv[l];
            if (sc->node_weight_mode == 1) out->rho[l] = sc->mu_s[v] * dx;
            else out->rho[l] = omega[v] * (-expm1(-mu_e[v] * dx));
        } else {
            out->rho[l] = sc->albedo[l - nvol];
        }
    }

    const double t_march = wall_s();

    /* O5: lattice and per-component tables */
    double *lat = (double *)malloc(sizeof(double) * 3 * NF);
    or_lattice(NF, lat);
    double *tab = (double *)malloc(sizeof(double) * NF * sc->n_phase);
    for (int k = 0; k < sc->n_phase; ++k) {
        /* the component toward each lattice point (cosine p_i,z to the pole), normalised */
        double *t = tab + (size_t)k * NF, s = 0.0;
        for (int i = 0; i < NF; ++i) {
            t[i] = phase_of(sc, k, lat[3 * i + 2]);
            s += t[i];
        }
        for (int i = 0; i < NF; ++i) t[i] = t[i] / s;
    }
    /* hull adjacency of the lattice, for the colouring of Sigma */
    enum { MAXNB = 16 };
    int32_t *hnb = NULL, *hnnb = NULL;
    if (sc->sigma_mode == 1) {
        hnb = (int32_t *)malloc(sizeof(int32_t) * NF * MAXNB);
        hnnb = (int32_t *)malloc(sizeof(int32_t) * NF);
        if (or_hull_adjacency(NF, lat, MAXNB, hnb, hnnb) < 0) {
            free(hnb); free(hnnb); free(lat); free(tab); free(mu_e); free(omega); free(nv);
            return 7;
        }
    }

    double sun_u[3], sun_in[3];
    unit_of(sc->sun_dir, sun_u);
    {
        int64_t nsd[3] = {-sc->sun_dir[0], -sc->sun_dir[1], -sc->sun_dir[2]};
        unit_of(nsd, sun_in); /* propagation direction of sunlight */
    }
    const double mu0 = sun_u[2];

    /* O7: K (CSR, rows = destination edges, columns = in(tail) ascending) and S */
    out->row_ptr[0] = 0;
    for (int64_t l = 0; l < N; ++l) {
        int64_t d = sc->adj_ptr[l + 1] - sc->adj_ptr[l];
        for (int64_t e = sc->adj_ptr[l]; e < sc->adj_ptr[l + 1]; ++e) out->row_ptr[e + 1] = out->row_ptr[e] + d;
    }
#pragma omp parallel
    {
        int dmax = 1;
        for (int64_t l = 0; l < N; ++l) {
            int d = (int)(sc->adj_ptr[l + 1] - sc->adj_ptr[l]);
            if (d > dmax) dmax = d;
        }
        double *s = (double *)malloc(sizeof(double) * 3 * dmax);
        int64_t *rev = (int64_t *)malloc(sizeof(int64_t) * dmax);
        double *Q = (double *)malloc(sizeof(double) * dmax);
        double *w = (double *)malloc(sizeof(double) * NF);
        int32_t *own = (int32_t *)malloc(sizeof(int32_t) * NF);
#pragma omp for schedule(dynamic, 64)
        for (int64_t l = 0; l < N; ++l) {
            int64_t off = sc->adj_ptr[l];
            int d = (int)(sc->adj_ptr[l + 1] - off);
            if (d == 0) continue;
            int is_surf = l >= nvol;
            for (int m = 0; m < d; ++m) {
                int64_t e = off + m, j = sc->adj_idx[e];
                int64_t D[3];
                node_disp(sc->pos, l, j, nx, ny, sc->periodic, D);
                unit_of(D, s + 3 * m); /* out-direction of edge (l -> j) */
                rev[m] = edge_rev(sc, e, l); /* in-edge (j -> l) */
            }
            if (!is_surf) {
                for (int i = 0; i < NF; ++i) {
                    double acc = 0.0;
                    for (int k = 0; k < sc->n_phase; ++k) {
                        double f = sc->phase_frac ? sc->phase_frac[(size_t)k * nvox + nv[l]] : 1.0;
                        acc += f * tab[(size_t)k * NF + i];
                    }
                    w[i] = acc;
                }
            }
            /* columns: in-edges a_m = rev[m] (ascending, since heads are ascending) */
            for (int m = 0; m < d; ++m) {
                double u[3] = {-s[3 * m], -s[3 * m + 1], -s[3 * m + 2]}; /* propagation of (j -> l) */
                if (sc->sigma_mode == 1) colour_q(is_surf, u, d, s, NF, lat, hnb, hnnb, MAXNB, w, Q, own);
                else node_q(is_surf, u, d, s, NF, lat, w, Q, own);
                double Ta = exp(-out->tau[off + m]); /* same pair as rev[m] */
                for (int n = 0; n < d; ++n) {
                    int64_t b = off + n;
                    int64_t q = out->row_ptr[b] + m;
                    out->col[q] = (int32_t)rev[m];
                    out->val[q] = Ta * out->rho[l] * Q[n];
                }
            }
            /* source (Eq. 9): sunlight arriving at l along sun_in */
            if (sc->sigma_mode == 1) colour_q(is_surf, sun_in, d, s, NF, lat, hnb, hnnb, MAXNB, w, Q, own);
            else node_q(is_surf, sun_in, d, s, NF, lat, w, Q, own);
            double Ts = exp(-out->tau_sun[l]);
            for (int n = 0; n < d; ++n) {
                if (is_surf) out->S[off + n] = out->rho[l] * mu0 * Ts * Q[n];
                else out->S[off + n] = Ts * out->rho[l] * Q[n];
            }
        }
        free(s); free(rev); free(Q); free(w); free(own);
    }

    const double t_matrix = wall_s();

    /* O8 */
    if (sc->scatter_order == 1) {
        memset(out->phi, 0, sizeof(double) * E);
        out->stats[0] = out->stats[1] = out->stats[2] = out->stats[3] = 0.0;
    } else {
        or_solve(E, out->row_ptr, out->col, out->val, out->S, sc->tol, out->phi, out->stats);
    }

    const double t_solve = wall_s();

    /* O9: gather (Eq. 11).  First every node's radiance toward the sensor: for a volume node
       the sun's beam and the in-edges' fluxes weighted by the node's phase function toward
       the sensor, for a surface node the Lambertian sum mu0 T_sun + sum T_a phi_a. */
    double vu[3];
    unit_of(sc->view_dir, vu);
    const double Lview = param_length_m(sc->view_dir, dx);
    double *Jn = (double *)malloc(sizeof(double) * (N > 0 ? N : 1));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t l = 0; l < N; ++l) {
        if (l < nvol) {
            const int64_t v = nv[l];
            double th_sun = 0.0;
            for (int c = 0; c < sc->n_phase; ++c) {
                double f = sc->phase_frac ? sc->phase_frac[(size_t)c * nvox + v] : 1.0;
                th_sun += f * phase_of(sc, c, sun_in[0] * vu[0] + sun_in[1] * vu[1] + sun_in[2] * vu[2]);
            }
            double J = th_sun * exp(-out->tau_sun[l]);
            if (sc->scatter_order != 1) {
                for (int64_t e = sc->adj_ptr[l]; e < sc->adj_ptr[l + 1]; ++e) {
                    int64_t j = sc->adj_idx[e];
                    int64_t D[3];
                    node_disp(sc->pos, j, l, nx, ny, sc->periodic, D);
                    double sa[3];
                    unit_of(D, sa); /* propagation direction of in-edge (j -> l) */
                    double mu = sa[0] * vu[0] + sa[1] * vu[1] + sa[2] * vu[2];
                    double th = 0.0;
                    for (int c = 0; c < sc->n_phase; ++c) {
                        double f = sc->phase_frac ? sc->phase_frac[(size_t)c * nvox + v] : 1.0;
                        th += f * phase_of(sc, c, mu);
                    }
                    int64_t a = edge_rev(sc, e, l);
                    J += th * exp(-out->tau[e]) * out->phi[a];
                }
            }
            Jn[l] = J;
        } else {
            double Js = mu0 * exp(-out->tau_sun[l]);
            if (sc->scatter_order != 1) {
                for (int64_t e = sc->adj_ptr[l]; e < sc->adj_ptr[l + 1]; ++e) {
                    int64_t a = edge_rev(sc, e, l);
                    Js += exp(-out->tau[e]) * out->phi[a];
                }
            }
            Jn[l] = Js;
        }
    }
    /* then along every pixel's line of sight: each voxel chord scatters toward the sensor
       the radiance of its node (the voxel's own node, or the line-of-sight node it is
       assigned to), weighted by the chord's scattering w (1 - exp(-mu_e s)) and the
       transmittance above it; the ground adds its Lambertian term */
#pragma omp parallel
    {
        int cap = sc->periodic ? MAX_WALK_STEPS : 4 * (nx + ny + nz) + 8;
        int64_t *vox = (int64_t *)malloc(sizeof(int64_t) * cap);
        double *dtv = (double *)malloc(sizeof(double) * cap);
        double *tcum = (double *)malloc(sizeof(double) * (cap + 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < (int64_t)nx * ny; ++p) {
            int64_t ix = p % nx, iy = p / nx;
            int64_t P[3] = {ix * FXS + FXS / 2, iy * FXS + FXS / 2, 0};
            trace_buf tb = {vox, dtv, cap, 0};
            dda_walk_p(nx, ny, nz, sc->periodic, P, sc->view_dir, 1, trace_visit, &tb);
            int nseg = tb.n;
            double Iv = 0.0;
            double tau_after = 0.0; /* optical depth between the segment's far end and the sensor */
            if (sc->n_vol == 0) {
                for (int k = nseg - 1; k >= 0; --k) {
                    int64_t v = vox[k];
                    double sk = dtv[k] * Lview;
                    double Tent = exp(-tau_after);
                    double wch = omega[v] * (-expm1(-mu_e[v] * sk));
                    Iv += Tent * wch * Jn[v]; /* the voxel's own node */
                    tau_after += mu_e[v] * sk;
                }
            } else {
                /* the chords cut at the elements' ends: each piece scatters the radiance of
                   its element's node; from the top down, as above.  Chord k spans [tcum[k],
                   tcum[k+1]] of the line parameter (prefix sums of the walk's lengths). */
                const int64_t e0 = sc->los_ptr[p], e1 = sc->los_ptr[p + 1];
                tcum[0] = 0.0;
                for (int k = 0; k < nseg; ++k) tcum[k + 1] = tcum[k] + dtv[k];
                int64_t e = e1 - 1; /* the element holding the point just below `top` */
                for (int k = nseg - 1; k >= 0; --k) {
                    const int64_t v = vox[k];
                    double top = tcum[k + 1];
                    while (top > tcum[k]) {
                        /* step e down to the element with start < top <= end (or, above the
                           last end, keep e1 - 1) */
                        while (e >= e0 && (e == e0 ? 0.0 : sc->los_t[e - 1]) >= top) --e;
                        double bot = tcum[k];
                        int64_t node = -1;
                        if (e >= e0) {
                            if (top <= sc->los_t[e]) {
                                const double start = e == e0 ? 0.0 : sc->los_t[e - 1];
                                if (start > bot) bot = start;
                                node = sc->los_node[e];
                            } else if (sc->los_t[e] > bot) {
                                bot = sc->los_t[e]; /* the part above the last end: no node */
                            }
                        }
                        const double sk = (top - bot) * Lview;
                        const double wch = omega[v] * (-expm1(-mu_e[v] * sk));
                        if (node >= 0) Iv += exp(-tau_after) * wch * Jn[node];
                        tau_after += mu_e[v] * sk;
                        top = bot;
                    }
                }
            }
            double Tsurf = exp(-tau_after);
            if (sc->surface) {
                Iv += Tsurf * (sc->albedo[p] / M_PI) * Jn[nvol + p];
            } else {
                Iv += Tsurf * (sc->albedo[p] / M_PI) * mu0 * exp(-optical_depth(nx, ny, nz, sc->periodic, mu_e, dx, P, sc->sun_dir, 1));
            }
            out->pix[p] = Iv;
        }
        free(vox);
        free(dtv);
        free(tcum);
    }
    free(Jn);
    free(nv);
    free(lat); free(tab); free(mu_e); free(omega); free(hnb); free(hnnb);
    const double t_end = wall_s();
    out->stats[4] = t_march - t_start;   /* node properties, edge and sun marches, node weights */
    out->stats[5] = t_matrix - t_march;  /* phase cells, K and S */
    out->stats[6] = t_solve - t_matrix;  /* the solve */
    out->stats[7] = t_end - t_solve;     /* the gather */
    return 0;
}

void or_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* tail of every edge, exported for tests */
void or_tails(int64_t N, const int64_t *adj_ptr, int64_t E, int64_t *tail) {
    for (int64_t e = 0; e < E; ++e) tail[e] = tail_of(adj_ptr, N, e);
}

/* ==================================================================== */
/* O9: the scattering graph (Sec. 2, Eq. 4; relative positions and the  */
/* coupling of Lambertian surface nodes, Sec. 3)                        */
/* ==================================================================== */
/*
 * Nodes: the node of every voxel (id = voxel index, position vol_pos_fx) and,
 * with surface nodes on, one node per column at (i + 1/2, j + 1/2, 0) voxels
 * (id nvox + i + nx j), as in the scene.
 *
 * The scattering coefficient of the coupling is that of the node's voxel; a
 * surface node takes A times the largest mu_s of the medium (Sec. 3).
 *
 * Relative positions (Sec. 3): the node positions are centred, scaled to unit
 * standard deviation per axis and expressed on the principal axes of the
 * scaled set.  The last step is a rotation and changes no distance, so the
 * coupling is evaluated on the centred, scaled coordinates:
 *   mean_a = S1_a / N                        S1, S2: exact integer sums
 *   var_a  = (N S2_a - S1_a^2) / (N N)       exact numerator, one rounding, divide
 *   q_ia   = (p_ia - mean_a) / sqrt(var_a)   (0 on an axis of zero variance)
 * Coupling (Eq. 4): C = sqrt(mu_i mu_j) / |q_i - q_j|.  Ranking and the
 * threshold use its square, evaluated as
 *   k = (mu_i * mu_j) / ((u*u + v*v) + w*w),   (u, v, w) = q_i - q_j,
 * which orders pairs as C does (the square root is monotone).
 * Candidates: pairs i < j with k > 0 that are not both surface nodes (two
 * points of the ground are joined along the ground, not through the medium).
 * Selection: n_pairs > 0: the n_pairs candidates of largest k, ties to the
 * lexicographically smaller (i, j) (the paper's experiments fix the number of
 * couplings); otherwise every candidate with k > c_min * c_min (the threshold
 * of Sec. 2).  Output: the symmetric adjacency in CSR, rows ascending.
 */
typedef struct {
    double k;
    int64_t i, j;
} or_pair;

/* a ranks before b */
static int pair_before(const or_pair *a, const or_pair *b) {
    if (a->k != b->k) return a->k > b->k;
    if (a->i != b->i) return a->i < b->i;
    return a->j < b->j;
}

/* min-heap on rank: h[0] is the candidate ranked last among those kept */
static void heap_down(or_pair *h, int64_t n, int64_t p) {
    for (;;) {
        int64_t c = 2 * p + 1, w = p;
        if (c < n && pair_before(&h[w], &h[c])) w = c;
        if (c + 1 < n && pair_before(&h[w], &h[c + 1])) w = c + 1;
        if (w == p) return;
        or_pair t = h[p];
        h[p] = h[w];
        h[w] = t;
        p = w;
    }
}
static void heap_up(or_pair *h, int64_t p) {
    while (p > 0) {
        int64_t a = (p - 1) / 2;
        if (!pair_before(&h[a], &h[p])) return;
        or_pair t = h[p];
        h[p] = h[a];
        h[a] = t;
        p = a;
    }
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Node positions (fixed point), coupling coefficients and the scaled coordinates
   q [N][3]; returns N. */
int64_t or_coupling_nodes(int nx, int ny, int nz, int64_t n_vol, const int32_t *vol_pos_fx, const float *mu_s,
                          int surface, const float *albedo, int64_t *pos /* [N][3] */, double *mu /* [N] */,
                          double *q) {
    const int64_t nvox = (int64_t)nx * ny * nz, nsurf = surface ? (int64_t)nx * ny : 0;
    const int64_t nv = n_vol > 0 ? n_vol : nvox, N = nv + nsurf;  /* general nodes: n_vol of them */
    double mmax = 0.0;
    for (int64_t v = 0; v < nvox; ++v) mmax = fmax(mmax, (double)mu_s[v]);
    for (int64_t l = 0; l < N; ++l) {
        if (l < nv) {
            for (int a = 0; a < 3; ++a) pos[3 * l + a] = vol_pos_fx[3 * l + a];
            /* the coupling coefficient of the node's voxel (node id = voxel id for one per voxel);
               a general node on the x = 0 or y = 0 plane (a periodic wrap puts it there) is in
               the first column, as for the scene's medium */
            const int64_t v = n_vol > 0 ? node_voxel(pos + 3 * l, nx, ny, nz, 3) : l;
            mu[l] = v >= 0 ? (double)mu_s[v] : 0.0;
        } else {
            const int64_t c = l - nv, i = c % nx, j = c / nx;
            pos[3 * l] = i * FXS + FXS / 2;
            pos[3 * l + 1] = j * FXS + FXS / 2;
            pos[3 * l + 2] = 0;
            mu[l] = (double)albedo[c] * mmax;
        }
    }
    for (int a = 0; a < 3; ++a) {
        __int128 s1 = 0, s2 = 0;
        for (int64_t l = 0; l < N; ++l) {
            s1 += pos[3 * l + a];
            s2 += (__int128)pos[3 * l + a] * pos[3 * l + a];
        }
        const double mean = (double)s1 / (double)N;
        const double var = (double)((__int128)N * s2 - s1 * s1) / ((double)N * (double)N);
        const double sd = sqrt(var);
        for (int64_t l = 0; l < N; ++l) q[3 * l + a] = var > 0.0 ? ((double)pos[3 * l + a] - mean) / sd : 0.0;
    }
    return N;
}

static double coupling_key(const double *q, const double *mu, int64_t i, int64_t j) {
    const double u = q[3 * i] - q[3 * j], v = q[3 * i + 1] - q[3 * j + 1], w = q[3 * i + 2] - q[3 * j + 2];
    const double d2 = (u * u + v * v) + w * w;
    return (mu[i] * mu[j]) / d2;
}

/* The selected pairs as a symmetric CSR adjacency over the N nodes; returns the
   number of directed edges (twice the pairs), or -1 when it exceeds cap (then
   adj_idx is not written). */
int64_t or_coupling_graph(int nx, int ny, int nz, int64_t n_vol, const int32_t *vol_pos_fx, const float *mu_s,
                          int surface, const float *albedo, int64_t n_pairs, double c_min,
                          int64_t *adj_ptr /* [N+1] */, int32_t *adj_idx, int64_t cap) {
    const int64_t nvox = n_vol > 0 ? n_vol : (int64_t)nx * ny * nz, N = nvox + (surface ? (int64_t)nx * ny : 0);
    int64_t *pos = malloc(sizeof(int64_t) * 3 * N);
    double *mu = malloc(sizeof(double) * N), *q = malloc(sizeof(double) * 3 * N);
    or_coupling_nodes(nx, ny, nz, n_vol, vol_pos_fx, mu_s, surface, albedo, pos, mu, q);
    or_pair *sel = NULL;
    int64_t ns = 0, scap = 0;
    if (n_pairs > 0) {
        sel = malloc(sizeof(or_pair) * n_pairs);
        for (int64_t i = 0; i < N; ++i)
            for (int64_t j = i + 1; j < N; ++j) {
                if (i >= nvox && j >= nvox) continue;
                or_pair c = {coupling_key(q, mu, i, j), i, j};
                if (!(c.k > 0.0)) continue;
                if (ns < n_pairs) {
                    sel[ns] = c;
                    heap_up(sel, ns++);
                } else if (pair_before(&c, &sel[0])) {
                    sel[0] = c;
                    heap_down(sel, ns, 0);
                }
            }
    } else {
        const double t = c_min * c_min;
        for (int64_t i = 0; i < N; ++i)
            for (int64_t j = i + 1; j < N; ++j) {
                if (i >= nvox && j >= nvox) continue;
                const double k = coupling_key(q, mu, i, j);
                if (!(k > t)) continue;
                if (ns == scap) {
                    scap = scap ? 2 * scap : 1024;
                    sel = realloc(sel, sizeof(or_pair) * scap);
                }
                sel[ns].k = k;
                sel[ns].i = i;
                sel[ns++].j = j;
            }
    }
    for (int64_t l = 0; l <= N; ++l) adj_ptr[l] = 0;
    for (int64_t s = 0; s < ns; ++s) {
        ++adj_ptr[sel[s].i + 1];
        ++adj_ptr[sel[s].j + 1];
    }
    for (int64_t l = 0; l < N; ++l) adj_ptr[l + 1] += adj_ptr[l];
    const int64_t E = adj_ptr[N];
    if (E <= cap) {
        int64_t *fill = malloc(sizeof(int64_t) * (N + 1));
        memcpy(fill, adj_ptr, sizeof(int64_t) * (N + 1));
        for (int64_t s = 0; s < ns; ++s) {
            adj_idx[fill[sel[s].i]++] = (int32_t)sel[s].j;
            adj_idx[fill[sel[s].j]++] = (int32_t)sel[s].i;
        }
        for (int64_t l = 0; l < N; ++l)
            qsort(adj_idx + adj_ptr[l], (size_t)(adj_ptr[l + 1] - adj_ptr[l]), sizeof(int32_t), cmp_i32);
        free(fill);
    }
    free(sel);
    free(pos);
    free(mu);
    free(q);
    return E <= cap ? E : -1;
}

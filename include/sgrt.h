/*
 * sgrt.h -- C ABI of the scattering-graph radiative-transfer hot path on
 * AMD Instinct MI355X (gfx950).
 *
 * The library implements, on one GPU, the hot path of the scattering graph
 * method (Mikkonen et al., "Scattering graph method for 3D radiative
 * transfer"): Beer-Lambert-Bouguer transmittance of every graph edge by an
 * exact voxel march (Sec. 2, Eq. 3 and Eq. 6), the phase-cell weights of
 * Eq. 7 on a Fibonacci lattice (Sec. 3), assembly of the flux matrix and
 * the direct-solar source (Eq. 6, Eq. 9), the solve of (I - F) phi = S
 * (Eq. 8, by the series of Eq. 5 with FP64 iterative refinement and a
 * GMRES fallback) and the gather of the observed pixel radiances (Eq. 11).
 *
 * Conventions used throughout:
 *  - fixed-point positions, 65536 units per voxel edge, absolute in the box
 *    [0, nx] x [0, ny] x [0, nz] voxels; the surface is the plane z = 0 and
 *    the medium outside the box is vacuum, unless the scene repeats along x
 *    and/or y (sg_scene_desc.periodic: a plane-parallel slab);
 *  - node ids: volume node of voxel (ix, iy, iz) = ix + nx*(iy + ny*iz),
 *    exactly one per voxel; surface node of column (ix, iy) =
 *    nx*ny*nz + ix + nx*iy at the column centre on z = 0;
 *  - directed edge id = its position in the adjacency CSR, so edges are
 *    sorted by (tail, head); the matrix K that the library builds is the
 *    transpose of the paper's F: row = destination edge b, column = source
 *    edge a, K[b][a] = T_a * rho_l * Q_l(a -> b) with l = head(a) = tail(b);
 *  - radiances are in units of the solar flux F0 per steradian (F0 = 1 on a
 *    plane normal to the beam).
 *
 * Every entry point returns an sg_status and never throws or aborts across
 * the ABI.  On a non-OK status, sg_last_error() returns a message for the
 * calling thread.  A device failure (SG_E_DEVICE) is sticky for the context:
 * every later call on that context returns it.
 *
 * Thread safety: distinct scenes may be solved concurrently from different
 * threads; one scene must not be used by two threads at once.  The server
 * owns its worker threads.
 */
#ifndef SGRT_H
#define SGRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SG_ABI_VERSION 7u

typedef int32_t sg_status;
enum {
    SG_OK = 0,
    SG_E_INVALID = -1, /* malformed argument or scene */
    SG_E_NOMEM = -2,   /* device allocation failed or the context's HBM budget is exceeded */
    SG_E_DEVICE = -3,  /* a HIP call or kernel failed; sticky for the context */
    SG_E_NOCONV = -4,  /* the solve stopped above its tolerance; outputs hold the best iterate */
    SG_E_BUSY = -5,    /* server queue full, try again */
    SG_E_ABI = -6,     /* abi_version mismatch */
    SG_E_STATE = -7,   /* operation needs a prior solve (exports) or a finished ticket */
    SG_E_CANCELLED = -8 /* the request was cancelled before it ran (sg_cancel) */
};

/* Thread-local text of the last non-OK status on the calling thread ("" if none). */
const char *sg_last_error(void);

/* SG_ABI_VERSION of the loaded library. */
uint32_t sg_abi_version(void);

typedef struct sg_ctx sg_ctx;
typedef struct sg_scene sg_scene;
typedef struct sg_server sg_server;

/*
 * Create a context on HIP device `hip_device`.  hbm_budget_bytes caps the
 * device memory the context holds (0 = 90% of the device's free memory at
 * creation): the blocks of its live scenes plus the freed blocks it keeps
 * for reuse by later scenes (a caching pool; kept blocks are released when
 * a new allocation needs the room, and by sg_ctx_destroy).  The context
 * owns one default-priority HIP stream, used when a call passes
 * hip_stream = NULL.
 * Errors: SG_E_INVALID (bad device), SG_E_DEVICE.
 */
sg_status sg_ctx_create(int32_t hip_device, uint64_t hbm_budget_bytes, sg_ctx **out);

/* Destroy a context and release its device memory.  All its scenes must have
   been destroyed first (else SG_E_STATE). */
sg_status sg_ctx_destroy(sg_ctx *ctx);

/*
 * A scene: voxel medium, scattering graph G(R, L) (Sec. 2, after Eq. 4),
 * surface, illumination and view.  All pointers are host memory, borrowed
 * for the duration of sg_scene_create only (the library copies them).
 */
typedef struct sg_scene_desc {
    uint32_t abi_version;      /* SG_ABI_VERSION */
    int32_t nx, ny, nz;        /* grid, 1..1024 each */
    double voxel_m;            /* voxel edge in metres, > 0 */
    const float *mu_s;         /* [nz][ny][nx] scattering coefficient, 1/m, finite, >= 0 */
    const float *mu_a;         /* [nz][ny][nx] absorption coefficient, 1/m, finite, >= 0 */
    int32_t n_phase;           /* 1..4 phase-function components (kinds below) */
    const double *hg_g;        /* [n_phase] Henyey-Greenstein asymmetry parameters, |g| < 1
                                  (read for Henyey-Greenstein components) */
    const float *phase_frac;   /* [n_phase][nz][ny][nx] mixing fractions (by scattering
                                  coefficient); NULL iff n_phase == 1 */
    const int32_t *vol_pos_fx; /* [nz*ny*nx][3] node positions (x, y, z), fixed point,
                                  strictly inside the node's own voxel */
    int32_t surface_nodes;     /* 1: one Lambertian node per column at z = 0; 0: none */
    const int64_t *adj_ptr;    /* [N + 1] symmetric adjacency CSR over node ids */
    const int32_t *adj_idx;    /* [E] heads, ascending within a row, no self loops,
                                  no surface-surface pairs; node degree <= 4096 for one
                                  wavelength (nodes above 64 have their own kernels: the
                                  strongest couplings of Eq. 4 gather on dense nodes),
                                  <= 64 with several wavelengths */
    const float *surf_albedo;  /* [ny][nx] Lambertian albedo in [0, 1] */
    int32_t sun_dir[3];        /* integer vector toward the sun (z > 0), |components| <= 2^22 */
    int32_t view_dir[3];       /* integer vector toward the sensor (z > 0), |components| <= 2^22 */
    int32_t n_fib;             /* Fibonacci lattice size, 2..128 (the paper uses 100; one point
                                  would lie on the horizon, leaving a surface node no cell) */
    int32_t node_weight_mode;  /* 0: rho = w (1 - exp(-mu_e * voxel_m)) (bounded scattering
                                  probability); 1: rho = mu_s * voxel_m (literal) */
    int32_t n_lambda;          /* wavelengths solved together, 1..256 */
    const float *abs_scale;    /* [n_lambda] multipliers of mu_a per wavelength (> 0);
                                  NULL means one wavelength with multiplier 1 */
    /* Phase-function kinds (Sec. 3: Rayleigh scattering, or a particle phase function
       given as a look-up table), per component; NULL: all Henyey-Greenstein.  Every
       component is normalised to integrate to 1 over the sphere. */
    const int32_t *phase_kind; /* [n_phase]: SG_PHASE_HG (hg_g[k]), SG_PHASE_RAYLEIGH
                                  ((3 / 16 pi)(1 + cos^2)), SG_PHASE_TABLE (row k of phase_lut) */
    int32_t phase_lut_n;       /* samples per table row, 2..4096 (when a component is a table) */
    const double *phase_lut;   /* [n_phase][phase_lut_n]: the phase function at cos(theta) =
                                  -1 + 2 m / (phase_lut_n - 1), finite, >= 0, not all zero in a
                                  table row; linear in cos(theta) between samples, scaled by the
                                  exact integral of that interpolant (rows of other kinds are
                                  not read) */
    int32_t sigma_mode;        /* the cells Sigma of Eq. 7 on the lattice: SG_SIGMA_VORONOI (0)
                                  each lattice point to the out-direction of largest dot
                                  product; SG_SIGMA_COLOUR (1) the paper's procedure (Sec. 3):
                                  each out-direction colours its closest lattice point (a point
                                  claimed twice goes to the closer direction, ties to the lower
                                  index) and the colours spread by flood fill along the edges
                                  of the lattice's convex hull, in rounds, an uncoloured point
                                  taking the colour of its lowest-index coloured neighbour */
    int32_t periodic;          /* flat slabs of infinite horizontal extent (Sec. 3: media
                                  bounded by parallel planes): bit 0 (SG_PERIODIC_X) and bit 1
                                  (SG_PERIODIC_Y) make the grid repeat along that axis with
                                  its period.  Every march then wraps voxel indices round the
                                  period and ends only through z; node-to-node directions and
                                  couplings use the shortest periodic image of the
                                  displacement, which must be unique (no pair exactly half a
                                  period apart).  The sun and view rays must reach the top
                                  within 65536 voxels: nz (|d_x| + |d_y| + d_z) + 4 d_z <=
                                  65536 d_z on both directions.  0: bounded grid */
    /* General volume nodes (Sec. 2: the nodes of the scattering graph are path points of the
       lines of sight, e.g. those of sg_los_nodes).  n_nodes = 0: one node per voxel at
       vol_pos_fx, node id = voxel id.  n_nodes > 0: n_nodes volume nodes at node_pos_fx
       (vol_pos_fx is not read), each with the medium (mu_s, mu_a, phase fractions) of the voxel
       that contains it, strictly inside the box (0 <= coordinate < period on periodic axes, the
       ground z = 0 excluded); surface nodes follow with ids n_nodes + column.  The radiance of
       pixel p then comes from its line of sight's elements e = los_ptr[p] .. los_ptr[p+1]-1,
       consecutive from the pixel's surface point up to the line parameters los_t[e] (t = 1 is
       one view_dir; strictly increasing, positive): element e scatters toward the sensor the
       radiance of volume node los_node[e] (-1: none) with the exact chord weights of the voxels
       it crosses (Eq. 11); the part of a line above its last element scatters nothing. */
    int32_t n_nodes;
    const int32_t *node_pos_fx; /* [n_nodes][3] */
    const int64_t *los_ptr;     /* [nx*ny + 1], los_ptr[0] = 0 */
    const int32_t *los_node;    /* [los_ptr[nx*ny]] */
    const double *los_t;        /* [los_ptr[nx*ny]] */
} sg_scene_desc;
enum { SG_SIGMA_VORONOI = 0, SG_SIGMA_COLOUR = 1 };
enum { SG_PERIODIC_X = 1, SG_PERIODIC_Y = 2 };
enum { SG_PHASE_HG = 0, SG_PHASE_RAYLEIGH = 1, SG_PHASE_TABLE = 2 };

/*
 * Validate a scene (sizes, finite and bounded values, node positions strictly
 * inside their voxels, strictly ascending adjacency rows without self loops
 * or surface-surface pairs on the host; symmetry of the adjacency on the
 * device after the upload), copy it to the device and reserve the device
 * memory of its FP32 solves (sg_solve allocates nothing for them).  FP64
 * solves, the optional CSR column index and the GMRES basis allocate their
 * arrays on first use and keep them until sg_scene_destroy.  The copies are
 * enqueued on hip_stream (NULL: the context stream) and are complete when the
 * call returns.
 * Errors: SG_E_ABI, SG_E_INVALID (with the reason), SG_E_NOMEM (budget or
 * allocation), SG_E_DEVICE.
 */
sg_status sg_scene_create(sg_ctx *ctx, const sg_scene_desc *desc, void *hip_stream, sg_scene **out);

/* Release a scene's device memory (waits for its work to finish). */
sg_status sg_scene_destroy(sg_scene *scene);

/*
 * Sizes of a scene: nodes N, directed edges E (= couplings, rows of K),
 * structural nonzeros of K (sum over nodes of degree^2), the largest
 * degree, wavelengths, and the device bytes reserved.  Any pointer may be NULL.
 */
sg_status sg_scene_sizes(const sg_scene *scene, int64_t *n_nodes, int64_t *n_edges, int64_t *nnz,
                         int32_t *max_degree, int32_t *n_lambda, uint64_t *device_bytes);

/*
 * Device bytes sg_scene_create would reserve for this description (validated
 * on the host, except the adjacency's symmetry, which sg_scene_create checks
 * on the device; no device work).  Used for admission against an HBM budget.
 * Errors: those of host validation (SG_E_ABI, SG_E_INVALID).
 */
sg_status sg_scene_reservation(const sg_scene_desc *desc, uint64_t *bytes);

enum { SG_FP32 = 0, SG_FP64 = 1 };
enum { SG_SOLVER_AUTO = 0, SG_SOLVER_NEUMANN = 1, SG_SOLVER_GMRES = 2 };

typedef struct sg_solve_opts {
    uint32_t abi_version;  /* SG_ABI_VERSION */
    int32_t precision;     /* SG_FP32: march, matrix and sweeps in FP32, residual and pixel
                              accumulation in FP64; SG_FP64: everything in FP64 */
    int32_t solver;        /* SG_SOLVER_AUTO: Neumann sweeps, GMRES if they stall, overflow or do
                              not reach rtol (in a batched scene each wavelength still above
                              rtol gets its own FP64 GMRES with the sweeps left of max_sweeps);
                              SG_SOLVER_GMRES: GMRES from zero (per wavelength when batched) */
    double rtol;           /* target of the per-edge relative residual max_e |r_e| / (|phi_e| + 1e-30),
                              r = S - (I - K) phi in FP64; it bounds the error of every edge,
                              including edges many orders of magnitude darker than the mean
                              (<= 0: 1e-6 FP32, 1e-12 FP64) */
    int32_t max_sweeps;    /* cap on matrix sweeps of all kinds (<= 0: 2000) */
    int32_t gmres_restart; /* GMRES(m) restart length, 2..64 (<= 0: 32) */
    int32_t scatter_order; /* 0: multiple scattering; 1: single scattering only (no solve) */
    int32_t build_col_idx; /* 1: also materialise the CSR column index array */
    int32_t timing;        /* 1: per-stage HIP-event timings into sg_solve_info */
    int32_t flags;         /* SG_NO_GRAPHS: launch sweep chunks one by one instead of replaying
                              captured HIP graphs; SG_NO_AUTOTUNE: default launch shapes;
                              SG_EXACT_CELLS: every phase-cell ownership decision (Eq. 7) by the
                              FP64 scan alone, without the FP32 screen that certifies most of
                              them first (the same owners and result bits, slower) */
    int32_t lambda_tile;   /* scenes of several wavelengths: wavelength lanes per node in the
                              sweep kernels, 8, 16, 32 or 64 (a wavefront then holds 64 /
                              lambda_tile nodes); at least n_lambda unless 64 (more than 64
                              wavelengths take several 64-lane tiles).  0: the library's choice
                              (8 or 16 when they hold n_lambda, else 64; from a scene's second
                              solve on, the autotuner's).  A set tile uses the default grid.
                              The tile does not change any result bit.  Ignored for one
                              wavelength. */
    /* Warm start of the solve of Eq. 8: an initial phi, e.g. a previous solve's (the layout
       of sg_export_vector's SG_VEC_PHI: [n_lambda][E] doubles in the scene's edge order),
       in host memory or, with warm_start_on_device = 1, device memory on the scene's
       device; borrowed for the call.  The solve starts its FP64 iterative refinement from
       it (residual r = S - (I - K) phi, correction sweeps, repeat) instead of from the
       Neumann series of phi = 0, so a good start saves sweeps; the stopping rule and the
       bar are unchanged.  Host values must be finite (SG_E_INVALID otherwise).  NULL: a
       cold start.  Not accepted in sg_server_opts.solve (SG_E_INVALID). */
    const double *warm_start;
    int32_t warm_start_on_device;
} sg_solve_opts;
enum { SG_NO_GRAPHS = 1, SG_NO_AUTOTUNE = 2, SG_EXACT_CELLS = 4 };

typedef struct sg_solve_info {
    int32_t converged;      /* 1 if every wavelength reached rtol */
    int32_t sweeps;         /* matrix sweeps (FP32 + FP64 residual + GMRES products) */
    int32_t gmres_used;     /* 1 if GMRES ran for any wavelength */
    int32_t refinements;    /* FP64 residual evaluations */
    double rel_residual;    /* max over wavelengths of the final per-edge relative residual (see rtol) */
    double ms_structure;    /* timings (timing = 1): CSR structure from the adjacency */
    double ms_march;        /* edge and sun transmittances */
    double ms_qbuild;       /* phase cells, matrix values and source */
    double ms_solve;        /* all sweeps and residuals */
    double ms_gather;       /* pixel radiances */
    double ms_total;
    double ms_spmv_sum;     /* summed duration of the FP32/FP64 sweep kernel launches */
    int32_t spmv_launches;  /* their number */
    int32_t spmv_monitored; /* how many of them also computed the convergence measures (these
                               read the previous iterate too: 4 more bytes per edge and
                               wavelength in FP32) */
    int64_t n_nodes, n_edges, nnz;
} sg_solve_info;

/*
 * Solve the scene for all its wavelengths: transmittances (Eq. 3, Eq. 6),
 * phase cells (Eq. 7), K and S (Eq. 6, Eq. 9), phi = (I - K)^-1 S (Eq. 5,
 * Eq. 8) and the pixel radiances (Eq. 11).  radiance: [n_lambda][ny][nx]
 * doubles, caller-allocated, host memory (radiance_on_device = 0) or device
 * memory on the context's device (1).  Kernels run on hip_stream (NULL: the
 * context stream); the call returns when the radiances are written.
 * opts may be NULL (defaults); info may be NULL.
 * Errors: SG_E_INVALID, SG_E_NOCONV (radiances of the best iterate are
 * still written), SG_E_DEVICE.
 */
sg_status sg_solve(sg_scene *scene, const sg_solve_opts *opts, void *hip_stream, double *radiance,
                   int32_t radiance_on_device, sg_solve_info *info);

/*
 * Verification exports of the last sg_solve (host buffers, NULL to skip).
 * sg_export_csr: K of wavelength `lambda` as CSR: row_ptr [E + 1], col_idx
 * [nnz] (ascending in-edges of the row's tail node, Sec. 2 line-graph
 * structure), val [nnz] as double; the column index is built on the device
 * if the solve did not build it.
 */
sg_status sg_export_csr(sg_scene *scene, int32_t lambda, int64_t *row_ptr, int32_t *col_idx, double *val);

enum {
    SG_VEC_TAU_S = 0,   /* [E] optical depth of mu_s along each edge's pair (Eq. 3 path integral) */
    SG_VEC_TAU_A = 1,   /* [E] same for mu_a */
    SG_VEC_TAU_SUN_S = 2, /* [N] node -> sun, mu_s channel (marched until it alone exceeds the cutoff) */
    SG_VEC_TAU_SUN_A = 3, /* [N] node -> sun, mu_a channel */
    SG_VEC_RHO = 4,     /* [n_lambda][N] node weights */
    SG_VEC_SOURCE = 5,  /* [n_lambda][E] source S (Eq. 9) */
    SG_VEC_PHI = 6,     /* [n_lambda][E] solution phi (Eq. 10) */
    SG_VEC_QSUN = 7     /* [E] phase-cell weight of the sun direction per out-edge (Eq. 7) */
};
/* Copy one vector of the last solve, as double, into out (host). */
sg_status sg_export_vector(sg_scene *scene, int32_t which, double *out);

enum { SG_TRACE_EDGE = 0, SG_TRACE_SUN = 1, SG_TRACE_VIEW = 2 };
/*
 * Voxel traversal used by the march kernels (the exact integer walk of the
 * Beer-Lambert-Bouguer path integral), for n_ids paths in one launch:
 * SG_TRACE_EDGE id = directed edge (walked from the lower to the higher node
 * id), SG_TRACE_SUN id = node (to the grid exit along sun_dir),
 * SG_TRACE_VIEW id = pixel ix + nx*iy (from its surface point along
 * view_dir).  Host buffers: voxels [n_ids][cap] (int32 voxel ids), dt
 * [n_ids][cap] (parameter length inside the voxel, as double), count
 * [n_ids] (voxels of the path; a value > cap means truncated output); slots
 * past a path's count hold voxel -1 and dt 0.
 * With periodic axes the edge walk follows the shortest periodic image and
 * every voxel id is wrapped into the grid.
 * Errors: SG_E_INVALID (NULL buffers, bad kind, sizes <= 0, an id out of
 * range), SG_E_DEVICE.
 */
sg_status sg_trace(sg_scene *scene, int32_t kind, const int64_t *ids, int32_t n_ids, int32_t cap,
                   int32_t *voxels, double *dt, int32_t *count);

/*
 * sg_trace for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, outputs and errors, the same kernel, but no device
 * allocation and no free.  The ids and the traversals are staged in a
 * staging area the library holds on each GPU for the life of the process
 * (sg_trace_noalloc_capacity() bytes, 16 MiB): a call needs about
 * 12 n_ids cap + 12 n_ids bytes of it (each of its four arrays rounded up to
 * 256 bytes) and larger calls are refused with SG_E_INVALID.  Calls on one
 * GPU share that area: the library serialises them within the process (a
 * per-device lock held until the call's stream has drained), so concurrent
 * calls wait rather than race.  Host buffers, as for sg_trace.
 */
sg_status sg_trace_noalloc(sg_scene *scene, int32_t kind, const int64_t *ids, int32_t n_ids, int32_t cap,
                           int32_t *voxels, double *dt, int32_t *count);
/* Bytes of the staging area of sg_trace_noalloc on each GPU. */
uint64_t sg_trace_noalloc_capacity(void);

/* ------------------------------------------------------------------------------------ */
/* Scattering nodes on the lines of sight (Sec. 2; Sec. 3, step 1 of the algorithm)      */
/* ------------------------------------------------------------------------------------ */

typedef struct sg_los_desc {
    uint32_t abi_version;   /* SG_ABI_VERSION */
    int32_t nx, ny, nz;     /* grid, 1..1024 each */
    double voxel_m;         /* voxel edge in metres, > 0 */
    int32_t view_dir[3];    /* toward the sensor (z > 0), |components| <= 2^22 */
    int32_t periodic;       /* as in sg_scene_desc */
    int32_t mode;           /* SG_LOS_LAYER or SG_LOS_STEP */
    double step_m;          /* SG_LOS_STEP: the distance between nodes along a line, metres (> 0;
                               fewer than 1e8 steps per line, else SG_E_INVALID) */
} sg_los_desc;
enum { SG_LOS_LAYER = 0, SG_LOS_STEP = 1 };

/*
 * Path points of the pixels' lines of sight (Sec. 2: a line of sight's points are taken at
 * each layer of the medium or at constant distance intervals).  Pixel p = i + nx j looks from
 * its surface point ((i + 1/2), (j + 1/2), 0) voxels along view_dir until the line leaves the
 * grid; the exact voxel walk splits it into chords of parameter length dt_k (t = 1 is one
 * view_dir), starting at t_k = dt_0 + ... + dt_(k-1) (summed in this order).  The line is cut
 * into elements [a, b]: SG_LOS_LAYER, one per layer of voxels it crosses (from the start of
 * the layer's first chord to the end of its last); SG_LOS_STEP, [j h, min((j + 1) h, t_exit)]
 * for j = 0, 1, ... while j h < t_exit, with h = step_m / (|view_dir| voxel_m / 65536).  Each
 * element gets a node at the rounded middle point: m = 0.5 (a + b), coordinate c = surface
 * point_c + floor(m view_dir_c + 0.5) (FP64, that operation order), wrapped into the period
 * on periodic axes; a node outside the box or on its outer planes is not made (the element
 * then carries -1).  Node ids follow the pixels, then the elements in order.
 * Outputs (host, caller-owned): node_pos_fx [n_nodes][3], los_ptr [nx*ny + 1], and per
 * element los_node and los_t (its end b): the fields of the same names in sg_scene_desc.
 * When a capacity is too small (or a buffer NULL) only the counts and los_ptr (if given) are
 * written.  Errors: SG_E_ABI, SG_E_INVALID, SG_E_NOMEM, SG_E_DEVICE.
 */
sg_status sg_los_nodes(sg_ctx *ctx, const sg_los_desc *desc, void *hip_stream, int32_t *node_pos_fx,
                       int64_t node_cap, int64_t *n_nodes, int64_t *los_ptr, int32_t *los_node, double *los_t,
                       int64_t el_cap, int64_t *n_elements);

/*
 * Bounds-checked builds.  libsgrt_debug.so is the same library compiled with
 * SG_DEBUG_BOUNDS: the kernels check their indexed global and LDS accesses against the
 * arrays' extents; a failed check skips the access (no fault) and records the first failing
 * site of its code module, and the entry point that ran the kernel (scene creation, solve,
 * export, trace, graph build, placement) returns SG_E_DEVICE naming the site.  A debugging
 * aid for callers that suspect their inputs or the library; results of a build without the
 * checks are identical when no check fails.
 * *enabled: 1 in a checked build, 0 otherwise.  selftest = 1 (checked builds): one check that
 * fails by construction runs first (its index is never used), so *site returns 0xffff -- the
 * checker's own test.  *site: the first failed check since the last report, or 0.
 */
sg_status sg_debug_bounds(sg_ctx *ctx, int32_t selftest, int32_t *enabled, uint32_t *site);

/* ------------------------------------------------------------------------------------ */
/* The scattering graph itself (Sec. 2, Eq. 4; Sec. 3)                                   */
/* ------------------------------------------------------------------------------------ */

/*
 * Nodes as in sg_scene_desc: one per voxel (id = voxel index, position vol_pos_fx),
 * or the n_nodes general nodes at node_pos_fx, and, with surface_nodes, one per column
 * at (i + 1/2, j + 1/2, 0) voxels (ids after the volume nodes).  A node's coupling
 * coefficient is its voxel's mu_s; a surface node's is surf_albedo times the largest mu_s
 * of the medium (Sec. 3).  General node sets have no voxel boxes to prune with: every pair
 * is ranked (the lines of sight of a scene hold few nodes next to a voxel grid).
 */
typedef struct sg_graph_desc {
    uint32_t abi_version;       /* SG_ABI_VERSION */
    int32_t nx, ny, nz;         /* grid, 1..1024 each */
    const float *mu_s;          /* [nz][ny][nx], finite, >= 0 */
    const int32_t *vol_pos_fx;  /* [nz*ny*nx][3], 2^16 units per voxel, strictly inside the node's voxel */
    int32_t surface_nodes;      /* 1: one surface node per column */
    const float *surf_albedo;   /* [ny][nx] in [0, 1] (read when surface_nodes) */
    int64_t n_pairs;            /* > 0: keep the n_pairs strongest couplings */
    double c_min;               /* n_pairs == 0: keep every coupling above c_min (>= 0) */
    int32_t n_nodes;            /* > 0: general volume nodes at node_pos_fx (as in sg_scene_desc;
                                   a node couples with its voxel's mu_s), 0: one per voxel */
    const int32_t *node_pos_fx; /* [n_nodes][3] */
} sg_graph_desc;

/*
 * Build the scattering graph G(R, L) of Sec. 2 on the device.  Positions are
 * taken relative (Sec. 3): centred and scaled to unit standard deviation per
 * axis (their projection on the principal axes, a rotation, changes no
 * distance).  The coupling of nodes i, j is Eq. 4, C = sqrt(mu_i mu_j) / |q_i -
 * q_j| on those coordinates, ranked through C^2 = mu_i mu_j / |q_i - q_j|^2
 * evaluated in FP64 with the fixed operation order
 *   (mu_i * mu_j) / ((u*u + v*v) + w*w),  (u, v, w) = q_i - q_j,
 *   q_a = (p_a - mean_a) / sqrt(var_a),  mean and variance from exact integer sums.
 * Candidate pairs: i != j, C > 0, not both surface nodes.  Selected: the n_pairs
 * candidates with the largest C (equal couplings: the lexicographically smaller
 * pair (min(i,j), max(i,j)) first; all candidates if fewer), or, with n_pairs =
 * 0, every candidate with C^2 > c_min^2.
 * Output (host buffers, caller-owned): the symmetric adjacency in the form
 * sg_scene_desc takes, adj_ptr [N+1] and adj_idx [n_edges] with each row
 * ascending; n_edges = twice the selected pairs.  When adj_idx is NULL or
 * cap < n_edges, only adj_ptr (if not NULL) and *n_edges are written (a size
 * query; the work is redone by the next call).  Node degrees are not capped:
 * sg_scene_create accepts degrees up to 4096 for one wavelength and 64 for
 * several.  info (optional) receives counts
 * and timings of the build.
 * Errors: SG_E_ABI, SG_E_INVALID (with the reason), SG_E_NOMEM, SG_E_DEVICE.
 */
typedef struct sg_graph_info {
    int64_t candidates;      /* pairs ranked (C^2 >= threshold; in threshold mode, selected) */
    int64_t pairs_evaluated; /* couplings computed to find the ranked candidates (pairs j > i in
                                the boxes, counted once; the fill kernel recomputes those it keeps) */
    double threshold;        /* C^2 bound of the last candidate pass (0: every pair) */
    int32_t streamed;        /* 1: every pair went through the streamed best-n list */
    int32_t passes;          /* candidate passes, each a count and a fill kernel over the boxes */
    double ms_total;         /* wall time of the call */
    double ms_pairs;         /* summed kernel time of the candidate passes (HIP events) */
    double ms_sort;          /* summed time of the ranking and adjacency sorts (HIP events) */
} sg_graph_info;

sg_status sg_graph_build(sg_ctx *ctx, const sg_graph_desc *desc, void *hip_stream, int64_t *adj_ptr,
                         int32_t *adj_idx, int64_t cap, int64_t *n_edges, sg_graph_info *info /* or NULL */);

/* ------------------------------------------------------------------------------------ */
/* Serving: continuous batching of many scenes on one device                             */
/* ------------------------------------------------------------------------------------ */

typedef struct sg_server_opts {
    uint32_t abi_version;     /* SG_ABI_VERSION */
    int32_t max_resident;     /* scenes held on the device at once (1..4; more are refused: a run
                                 with eight worker threads ended in a host fault inside the
                                 runtime's copy path, cause not found) */
    int32_t queue_cap;        /* pending requests before sg_submit returns SG_E_BUSY (>= 1) */
    int32_t n_streams;        /* device streams of the scheduler (1..64), at least max_resident:
                                 each resident slot runs on a stream of its own (a solve captures
                                 its sweep chunks as HIP graphs, and a capture would take in the
                                 launches of another slot on the same stream) */
    sg_solve_opts solve;      /* options applied to every request */
} sg_server_opts;

/*
 * Start a server on a context.  It admits queued scenes when a resident
 * slot is free and their reserved bytes (sg_scene_reservation plus what a
 * solve with opts->solve allocates: the FP64 arrays, the column index, the
 * GMRES basis when GMRES is forced), added to those of the admitted scenes,
 * fit the context's HBM budget, overlaps the resident scenes' work on their
 * streams, and completes each ticket independently.  A request that runs out
 * of budget in the mix (e.g. a solve falling back to GMRES, whose basis is
 * not reserved in advance) is put back at the head of the queue with the
 * basis added to its reservation and runs again once another request has
 * finished; it ends with SG_E_NOMEM only if it does not fit alone.  Results
 * are the same bits as the scene solved alone.  A scene whose adjacency is
 * not symmetric is refused when it is admitted: its ticket completes with
 * SG_E_INVALID.
 * Errors: SG_E_ABI, SG_E_INVALID (max_resident > n_streams among others),
 * SG_E_DEVICE.
 */
sg_status sg_server_create(sg_ctx *ctx, const sg_server_opts *opts, sg_server **out);

/*
 * Queue a scene (copied on the host before return; desc arrays are
 * borrowed for the call only).  Non-blocking.  Errors: SG_E_BUSY (queue
 * full), SG_E_INVALID (scene rejected), SG_E_NOMEM (the scene alone exceeds
 * the budget).
 */
sg_status sg_submit(sg_server *srv, const sg_scene_desc *desc, uint64_t *ticket);

/*
 * Poll a ticket: *done = 1 when finished, then radiance ([n_lambda][ny][nx],
 * host, may be NULL) and info are written and the ticket is released;
 * returns the request's own status (e.g. SG_E_NOCONV).  *done = 0: still
 * queued or running.
 */
sg_status sg_poll(sg_server *srv, uint64_t ticket, double *radiance, sg_solve_info *info, int32_t *done);

/*
 * Cancel a request that is still queued: it leaves the queue and its ticket finishes with
 * SG_E_CANCELLED (sg_poll / sg_wait then return that status and release the ticket).
 * Errors: SG_E_STATE (the request is running or has finished: it is not touched),
 * SG_E_INVALID (unknown ticket).
 */
sg_status sg_cancel(sg_server *srv, uint64_t ticket);

/* Block until the ticket finishes; same outputs as sg_poll. */
sg_status sg_wait(sg_server *srv, uint64_t ticket, double *radiance, sg_solve_info *info);

/* Per-request wall times: arrival (sg_submit) to completion, in ms; writes up to cap values. */
sg_status sg_server_latencies(sg_server *srv, double *ms, int32_t cap, int32_t *n);

/* Drain in-flight work and stop the server. */
sg_status sg_server_destroy(sg_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* SGRT_H */

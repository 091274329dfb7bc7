"""FP64 CPU reference ("oracle") of the scattering-graph hot path -- TEST INFRASTRUCTURE.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
this package imports nothing from the product: it takes a scene as any object
with the scene-format attributes (``nx, ny, nz, voxel_m, mu_s, mu_a, hg_g,
phase_frac, vol_pos_fx, surface_nodes, adj_ptr, adj_idx, surf_albedo,
sun_dir, view_dir, n_fib, node_weight_mode``) and returns numpy arrays.

The arithmetic lives in ``sgoracle.c`` (plain C, double precision); this
module marshals arrays and builds the shared object on first use.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sgoracle.c")
_LIB = os.path.join(_HERE, "libsgoracle.so")
# a prebuilt library to load instead (e.g. a sanitizer build of sgoracle.c)
_LIB_OVERRIDE = os.environ.get("SGORACLE_LIB")
_lock = threading.Lock()
_lib = None

FX = 1 << 16


def build(force: bool = True) -> str:
    """Compile sgoracle.c with gcc (FP contraction off, OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-std=c11", "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if _LIB_OVERRIDE:
                L = C.CDLL(_LIB_OVERRIDE)
            else:
                if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                    build(force=True)
                L = C.CDLL(_LIB)
            P = C.c_void_p
            L.or_trace_p.restype = C.c_int
            L.or_trace_p.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, P, P, C.c_int, P, P, C.c_int]
            L.or_trace_many.restype = None
            L.or_trace_many.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64, P, P, C.c_int, C.c_int, P, P,
                                        P]
            L.or_los_nodes.restype = C.c_int
            L.or_los_nodes.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, P, C.c_double, C.c_int, C.c_double, P,
                                       C.c_int64, P, P, P, C.c_int64, P]
            L.or_trace.restype = C.c_int
            L.or_trace.argtypes = [C.c_int, C.c_int, C.c_int, P, P, C.c_int, P, P, C.c_int]
            L.or_lattice.restype = None
            L.or_lattice.argtypes = [C.c_int, P]
            L.or_hg_table.restype = None
            L.or_hg_table.argtypes = [C.c_double, C.c_int, P, P]
            L.or_rotation.restype = None
            L.or_rotation.argtypes = [P, P]
            L.or_ownership.restype = None
            L.or_ownership.argtypes = [P, C.c_int, P, C.c_int, P, P]
            L.or_node_q.restype = None
            L.or_node_q.argtypes = [C.c_int, P, C.c_int, P, C.c_int, P, P]
            L.or_solve.restype = C.c_int
            L.or_solve.argtypes = [C.c_int64, P, P, P, P, C.c_double, P, P]
            L.or_nnz.restype = C.c_int64
            L.or_nnz.argtypes = [C.c_int64, P]
            L.or_run.restype = C.c_int
            L.or_run.argtypes = [P, P]
            L.or_set_threads.restype = None
            L.or_set_threads.argtypes = [C.c_int]
            L.or_num_threads.restype = C.c_int
            L.or_num_threads.argtypes = []
            L.or_phase_value.restype = C.c_double
            L.or_phase_value.argtypes = [C.c_int, C.c_double, P, C.c_int, C.c_double]
            L.or_table_integral.restype = C.c_double
            L.or_table_integral.argtypes = [P, C.c_int]
            L.or_hull_adjacency.restype = C.c_int
            L.or_hull_adjacency.argtypes = [C.c_int, P, C.c_int, P, P]
            L.or_colours.restype = C.c_int
            L.or_colours.argtypes = [P, C.c_int, P, C.c_int, C.c_int, P]
            L.or_tails.restype = None
            L.or_tails.argtypes = [C.c_int64, P, C.c_int64, P]
            L.or_coupling_nodes.restype = C.c_int64
            L.or_coupling_nodes.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int64, P, P, C.c_int, P, P, P, P]
            L.or_coupling_graph.restype = C.c_int64
            L.or_coupling_graph.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int64, P, P, C.c_int, P, C.c_int64,
                                            C.c_double, P, P, C.c_int64]
            _lib = L
        return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of the later calls (the pipeline's parallel loops)."""
    lib().or_set_threads(int(n))


# ------------------------------------------------------------------------------------------
# stage functions (pins)
# ------------------------------------------------------------------------------------------

def trace(nx, ny, nz, P, D, is_ray, cap=None, periodic=0):
    """Voxel ids and parameter lengths dt of the exact traversal of P + t D (periodic:
    bit 0 x, bit 1 y repeat with the grid's period)."""
    P = np.ascontiguousarray(P, dtype=np.int64)
    D = np.ascontiguousarray(D, dtype=np.int64)
    cap = cap or (65536 if periodic else 4 * (nx + ny + nz) + 8)
    vox = np.zeros(cap, np.int64)
    dt = np.zeros(cap, np.float64)
    n = lib().or_trace_p(nx, ny, nz, int(periodic), _p(P), _p(D), int(is_ray), _p(vox), _p(dt), cap)
    if n < 0:
        raise ValueError("segment leaves the grid")
    return vox[:n].copy(), dt[:n].copy()


def trace_many(nx, ny, nz, P, D, is_ray, cap, periodic=0):
    """trace() of many paths: P, D [n][3]; returns vox [n][cap] (int64), dt [n][cap] and the
    voxel count of each path (which may exceed cap; slots past the path hold -1 and 0)."""
    P = np.ascontiguousarray(np.broadcast_to(np.asarray(P, np.int64), (len(P), 3)))
    D = np.ascontiguousarray(np.broadcast_to(np.asarray(D, np.int64), P.shape))
    n = P.shape[0]
    vox = np.zeros((n, cap), np.int64)
    dt = np.zeros((n, cap), np.float64)
    cnt = np.zeros(n, np.int64)
    lib().or_trace_many(nx, ny, nz, int(periodic), n, _p(P), _p(D), int(is_ray), int(cap), _p(vox), _p(dt), _p(cnt))
    if (cnt < 0).any():
        raise ValueError("a segment leaves the grid")
    return vox, dt, cnt


def los_nodes(nx, ny, nz, view_dir, voxel_m, mode="layer", step_m=0.0, periodic=0):
    """Path points of the pixels' lines of sight (Sec. 2): node positions int64 [n][3],
    los_ptr int64 [nx ny + 1] over the lines' elements, and per element its node los_node
    int32 (-1: none) and its upper end los_t float64 along the line.  mode "layer": one
    element per layer crossed; "step": one per step_m metres along the line."""
    m = {"layer": 0, "step": 1}[mode]
    D = np.ascontiguousarray(view_dir, np.int64)
    npx = nx * ny
    los_ptr = np.zeros(npx + 1, np.int64)
    counts = np.zeros(2, np.int64)
    cap = ecap = 0
    while True:
        pos = np.zeros((max(cap, 1), 3), np.int64)
        los_node = np.zeros(max(ecap, 1), np.int32)
        los_t = np.zeros(max(ecap, 1), np.float64)
        rc = lib().or_los_nodes(nx, ny, nz, int(periodic), _p(D), float(voxel_m), m, float(step_m), _p(pos), cap,
                                _p(los_ptr), _p(los_node), _p(los_t), ecap, _p(counts))
        if rc < 0:
            raise ValueError("los_nodes: bad arguments")
        if rc == 0:
            return pos[:counts[0]].copy(), los_ptr.copy(), los_node[:counts[1]].copy(), los_t[:counts[1]].copy()
        cap, ecap = int(counts[0]), int(counts[1])


def lattice(N: int) -> np.ndarray:
    p = np.zeros((N, 3), np.float64)
    lib().or_lattice(N, _p(p))
    return p


def hg_table(g: float, N: int) -> np.ndarray:
    p = lattice(N)
    t = np.zeros(N, np.float64)
    lib().or_hg_table(float(g), N, _p(p), _p(t))
    return t


def rotation(u) -> np.ndarray:
    u = np.ascontiguousarray(u, np.float64)
    R = np.zeros(9, np.float64)
    lib().or_rotation(_p(u), _p(R))
    return R.reshape(3, 3)


def ownership(u, dirs, N: int) -> np.ndarray:
    """Lattice owner index per lattice point; u None = no rotation (surface)."""
    dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    p = lattice(N)
    own = np.zeros(N, np.int32)
    uu = None if u is None else np.ascontiguousarray(u, np.float64)
    lib().or_ownership(_p(uu), dirs.shape[0], _p(dirs), N, _p(p), _p(own))
    return own


def node_q(u, dirs, N: int, w=None, surface=False) -> np.ndarray:
    dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    d = dirs.shape[0]
    Q = np.zeros(d, np.float64)
    uu = None if u is None else np.ascontiguousarray(u, np.float64)
    ww = None if w is None else np.ascontiguousarray(w, np.float64)
    lib().or_node_q(1 if surface else 0, _p(uu), d, _p(dirs), N, _p(ww), _p(Q))
    return Q


def solve(row_ptr, col, val, S, tol=1e-13):
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    val = np.ascontiguousarray(val, np.float64)
    S = np.ascontiguousarray(S, np.float64)
    E = S.shape[0]
    phi = np.zeros(E, np.float64)
    st = np.zeros(4, np.float64)
    lib().or_solve(E, _p(row_ptr), _p(col), _p(val), _p(S), float(tol), _p(phi), _p(st))
    return phi, dict(sweeps=int(st[0]), rel_residual=float(st[1]), gmres=bool(st[2]), gmres_iters=int(st[3]))


def tails(adj_ptr) -> np.ndarray:
    adj_ptr = np.ascontiguousarray(adj_ptr, np.int64)
    N = adj_ptr.shape[0] - 1
    E = int(adj_ptr[-1])
    t = np.zeros(E, np.int64)
    lib().or_tails(N, _p(adj_ptr), E, _p(t))
    return t


# ------------------------------------------------------------------------------------------
# full pipeline
# ------------------------------------------------------------------------------------------

class _Scene(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("voxel_m", C.c_double),
                ("mu_s", C.c_void_p), ("mu_a", C.c_void_p), ("n_phase", C.c_int), ("hg_g", C.c_void_p),
                ("phase_frac", C.c_void_p), ("pos", C.c_void_p), ("surface", C.c_int),
                ("adj_ptr", C.c_void_p), ("adj_idx", C.c_void_p), ("albedo", C.c_void_p),
                ("sun_dir", C.c_void_p), ("view_dir", C.c_void_p), ("n_fib", C.c_int),
                ("node_weight_mode", C.c_int), ("scatter_order", C.c_int), ("tol", C.c_double),
                ("phase_kind", C.c_void_p), ("lut_n", C.c_int), ("lut", C.c_void_p), ("sigma_mode", C.c_int),
                ("periodic", C.c_int), ("n_vol", C.c_int64), ("los_ptr", C.c_void_p), ("los_node", C.c_void_p),
                ("los_t", C.c_void_p)]


class _Out(C.Structure):
    _fields_ = [("tau", C.c_void_p), ("tau_sun", C.c_void_p), ("rho", C.c_void_p),
                ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p), ("S", C.c_void_p),
                ("phi", C.c_void_p), ("pix", C.c_void_p), ("stats", C.c_void_p)]


def node_positions(scene) -> np.ndarray:
    """int64 [N, 3]: the scene's volume positions (one per voxel, or the general nodes of a
    scene that has node_pos_fx) then the surface node positions."""
    general = getattr(scene, "node_pos_fx", None)
    pos = np.asarray(scene.vol_pos_fx if general is None else general, np.int64).reshape(-1, 3)
    if scene.surface_nodes:
        iy, ix = np.meshgrid(np.arange(scene.ny), np.arange(scene.nx), indexing="ij")
        sp = np.zeros((scene.nx * scene.ny, 3), np.int64)
        sp[:, 0] = ix.reshape(-1) * FX + FX // 2
        sp[:, 1] = iy.reshape(-1) * FX + FX // 2
        pos = np.concatenate([pos, sp], axis=0)
    return np.ascontiguousarray(pos)


def run(scene, abs_scale: float = 1.0, scatter_order: int = 0, tol: float = 1e-13,
        want_matrix: bool = True):
    """Run the whole FP64 pipeline on one wavelength (mu_a multiplied by abs_scale).

    Returns a dict with tau [E], tau_sun [N], rho [N], row_ptr/col/val (K in CSR),
    S [E], phi [E], radiance [ny, nx] and solve stats.
    """
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a

    nvox = scene.nx * scene.ny * scene.nz
    mu_s = arr(np.asarray(scene.mu_s, np.float64).reshape(-1), np.float64)
    mu_a = arr(np.asarray(scene.mu_a, np.float64).reshape(-1) * float(abs_scale), np.float64)
    hg_g = arr(scene.hg_g, np.float64)
    pf = None
    if scene.phase_frac is not None:
        pf = arr(np.asarray(scene.phase_frac, np.float64).reshape(len(scene.hg_g), nvox), np.float64)
    pos = arr(node_positions(scene), np.int64)
    adj_ptr = arr(scene.adj_ptr, np.int64)
    adj_idx = arr(scene.adj_idx, np.int32)
    alb = arr(np.asarray(scene.surf_albedo, np.float64).reshape(-1), np.float64)
    sun = arr(np.asarray(scene.sun_dir, np.int64), np.int64)
    view = arr(np.asarray(scene.view_dir, np.int64), np.int64)
    N = pos.shape[0]
    E = int(adj_ptr[-1])
    nnz = int(lib().or_nnz(N, _p(adj_ptr)))

    kind = getattr(scene, "phase_kind", None)
    lut = getattr(scene, "phase_lut", None)
    kind = None if kind is None else arr(kind, np.int32)
    lut = None if lut is None else arr(lut, np.float64)
    general = getattr(scene, "node_pos_fx", None)
    n_vol = 0 if general is None else int(np.asarray(general).reshape(-1, 3).shape[0])
    los_ptr = None if general is None else arr(scene.los_ptr, np.int64)
    los_node = None if general is None else arr(scene.los_node, np.int32)
    los_t = None if general is None else arr(scene.los_t, np.float64)
    sc = _Scene(scene.nx, scene.ny, scene.nz, float(scene.voxel_m), _p(mu_s), _p(mu_a), len(hg_g), _p(hg_g),
                _p(pf), _p(pos), int(scene.surface_nodes), _p(adj_ptr), _p(adj_idx), _p(alb), _p(sun),
                _p(view), int(scene.n_fib), int(scene.node_weight_mode), int(scatter_order), float(tol),
                _p(kind), 0 if lut is None else int(lut.shape[-1]), _p(lut), int(getattr(scene, "sigma_mode", 0)),
                int(getattr(scene, "periodic", 0)), n_vol, _p(los_ptr), _p(los_node), _p(los_t))
    res = dict(tau=np.zeros(E), tau_sun=np.zeros(N), rho=np.zeros(N), row_ptr=np.zeros(E + 1, np.int64),
               col=np.zeros(nnz, np.int32), val=np.zeros(nnz), S=np.zeros(E), phi=np.zeros(E),
               radiance=np.zeros(scene.nx * scene.ny), stats=np.zeros(8))
    out = _Out(*[_p(res[k]) for k in ("tau", "tau_sun", "rho", "row_ptr", "col", "val", "S", "phi",
                                       "radiance", "stats")])
    rc = lib().or_run(C.byref(sc), C.byref(out))
    if rc != 0:
        raise ValueError("oracle: invalid scene (code %d)" % rc)
    st = res.pop("stats")
    res["solve"] = dict(sweeps=int(st[0]), rel_residual=float(st[1]), gmres=bool(st[2]), gmres_iters=int(st[3]))
    res["stage_s"] = dict(march=float(st[4]), matrix=float(st[5]), solve=float(st[6]), gather=float(st[7]))
    res["radiance"] = res["radiance"].reshape(scene.ny, scene.nx)
    res["nnz"] = nnz
    if not want_matrix:
        for k in ("col", "val"):
            res.pop(k)
    return res


# ------------------------------------------------------------------------------------------
# the scattering graph (Sec. 2, Eq. 4; Sec. 3)
# ------------------------------------------------------------------------------------------

def _graph_inputs(scene):
    general = getattr(scene, "node_pos_fx", None)
    pos = np.ascontiguousarray(scene.vol_pos_fx if general is None else general, np.int32)
    n_vol = 0 if general is None else int(pos.reshape(-1, 3).shape[0])
    mus = np.ascontiguousarray(scene.mu_s, np.float32)
    alb = np.ascontiguousarray(scene.surf_albedo, np.float32)
    return pos, mus, alb, n_vol


def coupling_nodes(scene):
    """Node positions (fixed point, [N][3]), coupling coefficients mu [N] (a volume node:
    the mu_s of its voxel; surface: albedo x the largest mu_s) and the centred, per-axis
    scaled coordinates q [N][3]."""
    pos, mus, alb, n_vol = _graph_inputs(scene)
    nv = n_vol if n_vol else scene.nx * scene.ny * scene.nz
    N = nv + (scene.nx * scene.ny if scene.surface_nodes else 0)
    P = np.zeros((N, 3), np.int64)
    mu = np.zeros(N, np.float64)
    q = np.zeros((N, 3), np.float64)
    lib().or_coupling_nodes(scene.nx, scene.ny, scene.nz, n_vol, _p(pos), _p(mus), int(bool(scene.surface_nodes)),
                            _p(alb), _p(P), _p(mu), _p(q))
    return P, mu, q


def coupling_graph(scene, n_pairs: int = 0, c_min: float = 0.0):
    """The scattering graph of the scene's nodes: the n_pairs strongest couplings
    (Eq. 4), or every coupling above c_min when n_pairs is 0.  Returns the symmetric
    adjacency (adj_ptr int64 [N+1], adj_idx int32 [2 * pairs]), rows ascending."""
    pos, mus, alb, n_vol = _graph_inputs(scene)
    nv = n_vol if n_vol else scene.nx * scene.ny * scene.nz
    N = nv + (scene.nx * scene.ny if scene.surface_nodes else 0)
    adj_ptr = np.zeros(N + 1, np.int64)
    cap = 2 * n_pairs if n_pairs > 0 else 0
    while True:
        adj_idx = np.zeros(max(cap, 1), np.int32)
        E = lib().or_coupling_graph(scene.nx, scene.ny, scene.nz, n_vol, _p(pos), _p(mus),
                                    int(bool(scene.surface_nodes)), _p(alb), int(n_pairs), float(c_min), _p(adj_ptr),
                                    _p(adj_idx), cap)
        if E >= 0:
            return adj_ptr, adj_idx[:E].copy()
        cap = int(adj_ptr[-1])


def phase_value(kind: int, mu: float, g: float = 0.0, row=None) -> float:
    """A phase-function component at cos(theta) = mu, normalised over the sphere
    (0 Henyey-Greenstein g, 1 Rayleigh, 2 the table row)."""
    r = None if row is None else np.ascontiguousarray(row, np.float64)
    return float(lib().or_phase_value(int(kind), float(g), _p(r), 0 if r is None else len(r), float(mu)))


def hull_adjacency(N: int, maxnb: int = 16):
    """Neighbour lists of the N-point lattice along its convex hull's edges."""
    p = lattice(N)
    nb = np.zeros((N, maxnb), np.int32)
    nnb = np.zeros(N, np.int32)
    dm = lib().or_hull_adjacency(N, _p(p), maxnb, _p(nb), _p(nnb))
    if dm < 0:
        raise ValueError("a lattice point has more hull neighbours than maxnb")
    return [nb[i, :nnb[i]].tolist() for i in range(N)]


def colours(u, dirs, N: int) -> np.ndarray:
    """Colour of every lattice point for incoming direction u (None: no rotation) and
    unit out-directions dirs [d][3]: nearest-point seeds, then flood fill (Sec. 3)."""
    s = np.ascontiguousarray(dirs, np.float64)
    uu = None if u is None else np.ascontiguousarray(u, np.float64)
    col = np.zeros(N, np.int32)
    if lib().or_colours(_p(uu), int(s.shape[0]), _p(s), N, 16, _p(col)) < 0:
        raise ValueError("hull degree above 16")
    return col

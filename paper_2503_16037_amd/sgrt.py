"""Python binding of libsgrt.so (include/sgrt.h): argument marshalling only.

Every step of the hot path runs in the library's HIP kernels.  PyTorch is
used for nothing but device output buffers and the current HIP stream.  The
binding refuses to run without the built library: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SGRT_LIB=debug selects the bounds-checked build (libsgrt_debug.so); another value is a path
LIB_PATH = {"": os.path.join(HERE, "libsgrt.so"), "debug": os.path.join(HERE, "libsgrt_debug.so")}.get(
    os.environ.get("SGRT_LIB", ""), os.environ.get("SGRT_LIB", ""))
ABI_VERSION = 7

SG_OK, SG_E_INVALID, SG_E_NOMEM, SG_E_DEVICE, SG_E_NOCONV, SG_E_BUSY, SG_E_ABI, SG_E_STATE = 0, -1, -2, -3, -4, -5, -6, -7
SG_E_CANCELLED = -8
SG_FP32, SG_FP64 = 0, 1
SOLVERS = {"auto": 0, "neumann": 1, "gmres": 2}
VEC = {"tau_s": 0, "tau_a": 1, "tau_sun_s": 2, "tau_sun_a": 3, "rho": 4, "source": 5, "phi": 6, "qsun": 7}
TRACE = {"edge": 0, "sun": 1, "view": 2}


class SgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"sgrt status {status}: {msg}")
        self.status = status


class SceneDesc(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("voxel_m", C.c_double), ("mu_s", C.c_void_p), ("mu_a", C.c_void_p), ("n_phase", C.c_int32),
                ("hg_g", C.c_void_p), ("phase_frac", C.c_void_p), ("vol_pos_fx", C.c_void_p),
                ("surface_nodes", C.c_int32), ("adj_ptr", C.c_void_p), ("adj_idx", C.c_void_p),
                ("surf_albedo", C.c_void_p), ("sun_dir", C.c_int32 * 3), ("view_dir", C.c_int32 * 3),
                ("n_fib", C.c_int32), ("node_weight_mode", C.c_int32), ("n_lambda", C.c_int32),
                ("abs_scale", C.c_void_p), ("phase_kind", C.c_void_p), ("phase_lut_n", C.c_int32),
                ("phase_lut", C.c_void_p), ("sigma_mode", C.c_int32),
                ("periodic", C.c_int32), ("n_nodes", C.c_int32), ("node_pos_fx", C.c_void_p),
                ("los_ptr", C.c_void_p), ("los_node", C.c_void_p), ("los_t", C.c_void_p)]


class GraphDesc(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("mu_s", C.c_void_p), ("vol_pos_fx", C.c_void_p), ("surface_nodes", C.c_int32),
                ("surf_albedo", C.c_void_p), ("n_pairs", C.c_int64), ("c_min", C.c_double),
                ("n_nodes", C.c_int32), ("node_pos_fx", C.c_void_p)]


class LosDesc(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("voxel_m", C.c_double), ("view_dir", C.c_int32 * 3), ("periodic", C.c_int32),
                ("mode", C.c_int32), ("step_m", C.c_double)]


class GraphInfo(C.Structure):
    _fields_ = [("candidates", C.c_int64), ("pairs_evaluated", C.c_int64), ("threshold", C.c_double),
                ("streamed", C.c_int32), ("passes", C.c_int32), ("ms_total", C.c_double),
                ("ms_pairs", C.c_double), ("ms_sort", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolveOpts(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("precision", C.c_int32), ("solver", C.c_int32), ("rtol", C.c_double),
                ("max_sweeps", C.c_int32), ("gmres_restart", C.c_int32), ("scatter_order", C.c_int32),
                ("build_col_idx", C.c_int32), ("timing", C.c_int32), ("flags", C.c_int32),
                ("lambda_tile", C.c_int32), ("warm_start", C.c_void_p), ("warm_start_on_device", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("converged", C.c_int32), ("sweeps", C.c_int32), ("gmres_used", C.c_int32),
                ("refinements", C.c_int32), ("rel_residual", C.c_double), ("ms_structure", C.c_double),
                ("ms_march", C.c_double), ("ms_qbuild", C.c_double), ("ms_solve", C.c_double),
                ("ms_gather", C.c_double), ("ms_total", C.c_double), ("ms_spmv_sum", C.c_double),
                ("spmv_launches", C.c_int32), ("spmv_monitored", C.c_int32), ("n_nodes", C.c_int64),
                ("n_edges", C.c_int64), ("nnz", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerOpts(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("max_resident", C.c_int32), ("queue_cap", C.c_int32),
                ("n_streams", C.c_int32), ("solve", SolveOpts)]


_lib = None
_lock = threading.Lock()


def lib():
    """Load libsgrt.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2503_16037_amd/build.py")
            # torch ships its own HIP runtime (SONAME libamdhip64.so.7, requested by torch as
            # libamdhip64.so).  Loading torch first makes libsgrt bind to that same runtime; the
            # other order leaves two HIP/HSA runtimes in the process and torch then sees no GPU.
            try:
                import torch  # noqa: F401
            except ImportError:
                pass
            L = C.CDLL(LIB_PATH)
            P, I32, I64, U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
            sigs = {
                "sg_last_error": (C.c_char_p, []),
                "sg_abi_version": (C.c_uint32, []),
                "sg_ctx_create": (I32, [I32, U64, P]),
                "sg_ctx_destroy": (I32, [P]),
                "sg_scene_create": (I32, [P, P, P, P]),
                "sg_scene_destroy": (I32, [P]),
                "sg_scene_sizes": (I32, [P, P, P, P, P, P, P]),
                "sg_scene_reservation": (I32, [P, P]),
                "sg_solve": (I32, [P, P, P, P, I32, P]),
                "sg_export_csr": (I32, [P, I32, P, P, P]),
                "sg_export_vector": (I32, [P, I32, P]),
                "sg_trace": (I32, [P, I32, P, I32, I32, P, P, P]),
                "sg_trace_noalloc": (I32, [P, I32, P, I32, I32, P, P, P]),
                "sg_trace_noalloc_capacity": (C.c_uint64, []),
                "sg_server_create": (I32, [P, P, P]),
                "sg_submit": (I32, [P, P, P]),
                "sg_poll": (I32, [P, U64, P, P, P]),
                "sg_wait": (I32, [P, U64, P, P]),
                "sg_cancel": (I32, [P, U64]),
                "sg_debug_bounds": (I32, [P, I32, P, P]),
                "sg_server_latencies": (I32, [P, P, I32, P]),
                "sg_server_destroy": (I32, [P]),
                "sg_graph_build": (I32, [P, P, P, P, P, I64, P, P]),
                "sg_los_nodes": (I32, [P, P, P, P, I64, P, P, P, P, I64, P]),
            }
            for name, (res, args) in sigs.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            if L.sg_abi_version() != ABI_VERSION:
                raise RuntimeError("libsgrt ABI version mismatch")
            _lib = L
        return _lib


def _check(status: int, allow=()):
    if status != SG_OK and status not in allow:
        raise SgError(status, lib().sg_last_error().decode())
    return status


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_desc(scene, keep: list) -> SceneDesc:
    """Fill an sg_scene_desc from a scene-format object; arrays kept alive in `keep`."""

    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a

    d = SceneDesc()
    d.abi_version = ABI_VERSION
    d.nx, d.ny, d.nz = int(scene.nx), int(scene.ny), int(scene.nz)
    d.voxel_m = float(scene.voxel_m)
    d.mu_s = _ptr(arr(scene.mu_s, np.float32))
    d.mu_a = _ptr(arr(scene.mu_a, np.float32))
    g = arr(scene.hg_g, np.float64)
    d.n_phase = int(g.shape[0])
    d.hg_g = _ptr(g)
    d.phase_frac = None if scene.phase_frac is None else _ptr(arr(scene.phase_frac, np.float32))
    general = getattr(scene, "node_pos_fx", None)
    if general is None:
        d.vol_pos_fx = _ptr(arr(scene.vol_pos_fx, np.int32))
        d.n_nodes = 0
    else:
        g_pos = arr(general, np.int32)
        d.n_nodes = int(g_pos.reshape(-1, 3).shape[0])
        d.node_pos_fx = _ptr(g_pos)
        d.los_ptr = _ptr(arr(scene.los_ptr, np.int64))
        d.los_node = _ptr(arr(scene.los_node, np.int32))
        d.los_t = _ptr(arr(scene.los_t, np.float64))
    d.surface_nodes = int(scene.surface_nodes)
    d.adj_ptr = _ptr(arr(scene.adj_ptr, np.int64))
    d.adj_idx = _ptr(arr(scene.adj_idx, np.int32))
    d.surf_albedo = _ptr(arr(scene.surf_albedo, np.float32))
    for k in range(3):
        d.sun_dir[k] = int(scene.sun_dir[k])
        d.view_dir[k] = int(scene.view_dir[k])
    d.n_fib = int(scene.n_fib)
    d.node_weight_mode = int(scene.node_weight_mode)
    kind = getattr(scene, "phase_kind", None)
    lut = getattr(scene, "phase_lut", None)
    d.phase_kind = None if kind is None else _ptr(arr(kind, np.int32))
    d.phase_lut = None if lut is None else _ptr(arr(lut, np.float64))
    d.phase_lut_n = 0 if lut is None else int(np.asarray(lut).shape[-1])
    d.sigma_mode = int(getattr(scene, "sigma_mode", 0))
    d.periodic = int(getattr(scene, "periodic", 0))
    abs_scale = getattr(scene, "abs_scale", None)
    if abs_scale is None:
        d.n_lambda = 1
        d.abs_scale = None
    else:
        a = arr(abs_scale, np.float32)
        d.n_lambda = int(a.shape[0])
        d.abs_scale = _ptr(a)
    return d


SG_NO_GRAPHS, SG_NO_AUTOTUNE, SG_EXACT_CELLS = 1, 2, 4


def make_opts(precision="fp32", solver="auto", rtol=0.0, max_sweeps=0, gmres_restart=0, scatter_order=0,
              build_col_idx=False, timing=False, graphs=True, autotune=True, lambda_tile=0,
              screen=True) -> SolveOpts:
    o = SolveOpts()
    o.abi_version = ABI_VERSION
    o.precision = SG_FP64 if precision in ("fp64", SG_FP64) else SG_FP32
    o.solver = SOLVERS[solver] if isinstance(solver, str) else int(solver)
    o.rtol = float(rtol)
    o.max_sweeps = int(max_sweeps)
    o.gmres_restart = int(gmres_restart)
    o.scatter_order = int(scatter_order)
    o.build_col_idx = 1 if build_col_idx else 0
    o.timing = 1 if timing else 0
    o.flags = ((0 if graphs else SG_NO_GRAPHS) | (0 if autotune else SG_NO_AUTOTUNE)
               | (0 if screen else SG_EXACT_CELLS))
    o.lambda_tile = int(lambda_tile)
    return o


class Context:
    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = C.c_void_p()
        _check(lib().sg_ctx_create(device, hbm_budget_bytes, C.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            _check(lib().sg_ctx_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)  # torch.cuda.Stream (a HIP stream on ROCm)


class Scene:
    """A scene resident on the device (sg_scene_create)."""

    def __init__(self, ctx: Context, scene, stream=None):
        keep: list = []
        desc = make_desc(scene, keep)
        h = C.c_void_p()
        _check(lib().sg_scene_create(ctx.handle, C.byref(desc), _stream_ptr(stream), C.byref(h)))
        self.handle = h
        self.ctx = ctx
        self.nx, self.ny, self.nz = scene.nx, scene.ny, scene.nz
        self.n_lambda = desc.n_lambda
        self.sizes = self._sizes()

    def _sizes(self):
        n, e, z = C.c_int64(), C.c_int64(), C.c_int64()
        dm, nl = C.c_int32(), C.c_int32()
        b = C.c_uint64()
        _check(lib().sg_scene_sizes(self.handle, C.byref(n), C.byref(e), C.byref(z), C.byref(dm), C.byref(nl),
                                    C.byref(b)))
        return dict(n_nodes=n.value, n_edges=e.value, nnz=z.value, max_degree=dm.value, n_lambda=nl.value,
                    device_bytes=b.value)

    def close(self):
        if self.handle:
            _check(lib().sg_scene_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def solve(self, out=None, stream=None, allow_noconv=False, warm_start=None, **opts):
        """Solve; returns (radiance, info).  out: None (host numpy result) or a device
        tensor of n_lambda * ny * nx float64 (radiance written in place).  warm_start: an
        initial phi of n_lambda * E float64 values ([n_lambda][E], as export_vector("phi")),
        a host array or a device tensor."""
        o = make_opts(**opts)
        if warm_start is not None:
            n = self.n_lambda * self.sizes["n_edges"]
            if hasattr(warm_start, "data_ptr"):
                if warm_start.numel() != n or str(warm_start.dtype) != "torch.float64" or not warm_start.is_contiguous():
                    raise ValueError("warm_start must be a contiguous float64 tensor of n_lambda * E values")
                o.warm_start, o.warm_start_on_device = warm_start.data_ptr(), 1
            else:
                warm_start = np.ascontiguousarray(warm_start, np.float64).reshape(-1)
                if warm_start.size != n:
                    raise ValueError("warm_start must hold n_lambda * E values")
                o.warm_start, o.warm_start_on_device = warm_start.ctypes.data, 0
        info = SolveInfo()
        npx = self.n_lambda * self.ny * self.nx
        if out is None:
            rad = np.zeros(npx, np.float64)
            ptr, on_dev = _ptr(rad), 0
        else:
            if out.numel() != npx or str(out.dtype) != "torch.float64":
                raise ValueError("out must hold n_lambda * ny * nx float64 values")
            rad = out
            ptr, on_dev = C.c_void_p(out.data_ptr()), 1
        st = lib().sg_solve(self.handle, C.byref(o), _stream_ptr(stream), ptr, on_dev, C.byref(info))
        _check(st, allow=(SG_E_NOCONV,) if allow_noconv else ())
        if out is None:
            rad = rad.reshape(self.n_lambda, self.ny, self.nx)
            if self.n_lambda == 1:
                rad = rad[0]
        d = info.as_dict()
        d["status"] = st
        return rad, d

    def export_csr(self, lam: int = 0, values=True, cols=True):
        E, nnz = self.sizes["n_edges"], self.sizes["nnz"]
        rp = np.zeros(E + 1, np.int64)
        col = np.zeros(nnz, np.int32) if cols else None
        val = np.zeros(nnz, np.float64) if values else None
        _check(lib().sg_export_csr(self.handle, lam, _ptr(rp), _ptr(col), _ptr(val)))
        return rp, col, val

    def export_vector(self, which: str) -> np.ndarray:
        E, N, nl = self.sizes["n_edges"], self.sizes["n_nodes"], self.n_lambda
        n = {"tau_s": E, "tau_a": E, "tau_sun_s": N, "tau_sun_a": N, "rho": N * nl, "source": E * nl,
             "phi": E * nl, "qsun": E}[which]
        out = np.zeros(n, np.float64)
        _check(lib().sg_export_vector(self.handle, VEC[which], _ptr(out)))
        if which in ("rho", "source", "phi") and nl > 1:
            out = out.reshape(nl, -1)
        return out

    def trace(self, kind: str, ids, cap: int = 512):
        ids = np.ascontiguousarray(ids, np.int64)
        n = ids.shape[0]
        vox = np.zeros((n, cap), np.int32)
        dt = np.zeros((n, cap), np.float64)
        cnt = np.zeros(n, np.int32)
        _check(lib().sg_trace(self.handle, TRACE[kind], _ptr(ids), n, cap, _ptr(vox), _ptr(dt), _ptr(cnt)))
        return vox, dt, cnt

    def trace_noalloc(self, kind: str, ids, cap: int = 512):
        """trace() through the allocation-free entry point (staging in the library's
        per-device area instead of per-call device buffers)."""
        ids = np.ascontiguousarray(ids, np.int64)
        n = ids.shape[0]
        vox = np.zeros((n, cap), np.int32)
        dt = np.zeros((n, cap), np.float64)
        cnt = np.zeros(n, np.int32)
        _check(lib().sg_trace_noalloc(self.handle, TRACE[kind], _ptr(ids), n, cap, _ptr(vox), _ptr(dt), _ptr(cnt)))
        return vox, dt, cnt


def scene_reservation(scene) -> int:
    """Device bytes a scene would reserve (host-side validation only)."""
    keep: list = []
    desc = make_desc(scene, keep)
    b = C.c_uint64()
    _check(lib().sg_scene_reservation(C.byref(desc), C.byref(b)))
    return b.value


class Server:
    """Continuous-batching server (sg_server_*)."""

    def __init__(self, ctx: Context, max_resident=4, queue_cap=64, n_streams=4, **solve_opts):
        o = ServerOpts()
        o.abi_version = ABI_VERSION
        o.max_resident = max_resident
        o.queue_cap = queue_cap
        o.n_streams = n_streams
        o.solve = make_opts(**solve_opts)
        h = C.c_void_p()
        _check(lib().sg_server_create(ctx.handle, C.byref(o), C.byref(h)))
        self.handle = h
        self.shapes = {}

    def submit(self, scene) -> Optional[int]:
        keep: list = []
        desc = make_desc(scene, keep)
        t = C.c_uint64()
        st = lib().sg_submit(self.handle, C.byref(desc), C.byref(t))
        if st == SG_E_BUSY:
            return None
        _check(st)
        self.shapes[t.value] = (desc.n_lambda, scene.ny, scene.nx)
        return t.value

    def _out(self, ticket):
        nl, ny, nx = self.shapes[ticket]
        return np.zeros(nl * ny * nx, np.float64), (nl, ny, nx)

    def poll(self, ticket: int):
        rad, shp = self._out(ticket)
        info = SolveInfo()
        done = C.c_int32()
        st = lib().sg_poll(self.handle, ticket, _ptr(rad), C.byref(info), C.byref(done))
        if not done.value:
            return None
        self.shapes.pop(ticket)
        d = info.as_dict()
        d["status"] = st
        return rad.reshape(shp), d

    def wait(self, ticket: int):
        rad, shp = self._out(ticket)
        info = SolveInfo()
        st = lib().sg_wait(self.handle, ticket, _ptr(rad), C.byref(info))
        self.shapes.pop(ticket)
        d = info.as_dict()
        d["status"] = st
        return rad.reshape(shp), d

    def cancel(self, ticket: int) -> int:
        """sg_cancel: SG_OK when the queued request was cancelled (its wait then reports
        SG_E_CANCELLED), SG_E_STATE when it is running or finished."""
        st = lib().sg_cancel(self.handle, ticket)
        if st not in (SG_OK, SG_E_STATE):
            _check(st)
        return st

    @staticmethod
    def reservation(scene) -> int:
        return scene_reservation(scene)

    def latencies(self, cap=100000):
        ms = np.zeros(cap, np.float64)
        n = C.c_int32()
        _check(lib().sg_server_latencies(self.handle, _ptr(ms), cap, C.byref(n)))
        return ms[:n.value].copy()

    def close(self):
        if self.handle:
            _check(lib().sg_server_destroy(self.handle))
            self.handle = None


def graph_build(ctx: Context, scene, n_pairs: int = 0, c_min: float = 0.0, stream=None, info: bool = False):
    """sg_graph_build: the scattering graph of the scene's nodes (the n_pairs strongest
    couplings, or those above c_min when n_pairs is 0).  Returns (adj_ptr int64 [N+1],
    adj_idx int32 [n_edges]), the form a scene's adjacency takes, and with info=True
    also the build statistics (sg_graph_info) as a dict."""
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a

    d = GraphDesc()
    d.abi_version = ABI_VERSION
    d.nx, d.ny, d.nz = int(scene.nx), int(scene.ny), int(scene.nz)
    d.mu_s = _ptr(arr(scene.mu_s, np.float32))
    general = getattr(scene, "node_pos_fx", None)
    n_vol = d.nx * d.ny * d.nz
    if general is None:
        d.vol_pos_fx = _ptr(arr(scene.vol_pos_fx, np.int32))
    else:
        g_pos = arr(general, np.int32)
        n_vol = d.n_nodes = int(g_pos.reshape(-1, 3).shape[0])
        d.node_pos_fx = _ptr(g_pos)
    d.surface_nodes = 1 if scene.surface_nodes else 0
    d.surf_albedo = _ptr(arr(scene.surf_albedo, np.float32))
    d.n_pairs = int(n_pairs)
    d.c_min = float(c_min)
    N = n_vol + (d.nx * d.ny if d.surface_nodes else 0)
    adj_ptr = np.zeros(N + 1, np.int64)
    ne = C.c_int64(0)
    cap = 2 * int(n_pairs)
    adj_idx = np.zeros(max(cap, 1), np.int32)
    gi = GraphInfo()
    _check(lib().sg_graph_build(ctx.handle, C.byref(d), _stream_ptr(stream), _ptr(adj_ptr),
                                _ptr(adj_idx) if cap else None, cap, C.byref(ne), C.byref(gi)))
    if ne.value > cap:  # threshold mode: the size is known now
        adj_idx = np.zeros(ne.value, np.int32)
        _check(lib().sg_graph_build(ctx.handle, C.byref(d), _stream_ptr(stream), _ptr(adj_ptr), _ptr(adj_idx),
                                    ne.value, C.byref(ne), C.byref(gi)))
    out = (adj_ptr, adj_idx[:ne.value].copy())
    return out + (gi.as_dict(),) if info else out


def debug_bounds(ctx: Context, selftest: bool = False):
    """sg_debug_bounds: (enabled, site) -- whether this library checks its kernels' indexed
    accesses, and the first failed check since the last report (0: none); selftest runs one
    check that fails by construction first (site 0xffff)."""
    en, site = C.c_int32(), C.c_uint32()
    _check(lib().sg_debug_bounds(ctx.handle, 1 if selftest else 0, C.byref(en), C.byref(site)))
    return bool(en.value), int(site.value)


def los_nodes(ctx: Context, nx, ny, nz, view_dir, voxel_m, mode="layer", step_m=0.0, periodic=0, stream=None):
    """sg_los_nodes: the path points of the pixels' lines of sight (one per layer crossed, or
    every step_m metres).  Returns (node_pos_fx int32 [n][3], los_ptr int64 [nx ny + 1],
    los_node int32 [elements], los_t float64 [elements]), the general-node fields of a scene."""
    d = LosDesc()
    d.abi_version = ABI_VERSION
    d.nx, d.ny, d.nz = int(nx), int(ny), int(nz)
    d.voxel_m = float(voxel_m)
    for k in range(3):
        d.view_dir[k] = int(view_dir[k])
    d.periodic = int(periodic)
    d.mode = {"layer": 0, "step": 1}[mode]
    d.step_m = float(step_m)
    los_ptr = np.zeros(nx * ny + 1, np.int64)
    nn, ne = C.c_int64(0), C.c_int64(0)
    _check(lib().sg_los_nodes(ctx.handle, C.byref(d), _stream_ptr(stream), None, 0, C.byref(nn), None, None, None, 0,
                              C.byref(ne)))
    pos = np.zeros((max(nn.value, 1), 3), np.int32)
    node = np.zeros(max(ne.value, 1), np.int32)
    t = np.zeros(max(ne.value, 1), np.float64)
    _check(lib().sg_los_nodes(ctx.handle, C.byref(d), _stream_ptr(stream), _ptr(pos), nn.value, C.byref(nn),
                              _ptr(los_ptr), _ptr(node), _ptr(t), ne.value, C.byref(ne)))
    return pos[:nn.value].copy(), los_ptr, node[:ne.value].copy(), t[:ne.value].copy()

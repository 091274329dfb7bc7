"""Seeded synthetic scene generators (inputs only).

This module produces the *inputs* of the scattering-graph hot path: a voxel
grid of scattering / absorption coefficients, one scattering node per voxel
(jittered inside it) plus optional Lambertian surface nodes, the symmetric
node adjacency (the scattering graph G(R, L), Sec. 2, Eq. 4 and the
paragraph after it), surface albedo and the integer sun / sensor directions.

It holds none of the method's arithmetic (no transmittance, phase-cell,
flux-matrix, solve or gather code) and is shared by the HIP path, the tests
and the benchmark.  The FP64 reference lives elsewhere and never imports this
module; it takes the arrays produced here.

Conventions fixed here (the scene format):
  * positions are fixed point, FX = 2**16 units per voxel edge, absolute in the
    box [0, nx*FX] x [0, ny*FX] x [0, nz*FX]; the surface is the plane z = 0;
  * volume node id = ix + nx*(iy + ny*iz) (one node per voxel, x fastest);
    surface node id = nx*ny*nz + ix + nx*iy, at ((ix+1/2)FX, (iy+1/2)FX, 0);
  * the adjacency is CSR over node ids, rows ascending, symmetric, no self
    loops, no surface-surface pairs; a directed edge's id is its CSR position,
    so edges are sorted by (tail, head);
  * sun_dir / view_dir are round(2**20 * s) for the unit vector s pointing
    from the scene toward the sun / the sensor (azimuth measured from +x
    toward +y).
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import Optional

import numpy as np

FX = 1 << 16          # fixed-point units per voxel edge
DIR_SCALE = 1 << 20   # fixed-point scale of the sun / sensor direction vectors


@dataclasses.dataclass
class Scene:
    name: str
    seed: int
    nx: int
    ny: int
    nz: int
    voxel_m: float
    mu_s: np.ndarray            # float32 [nz, ny, nx], 1/m
    mu_a: np.ndarray            # float32 [nz, ny, nx], 1/m
    hg_g: np.ndarray            # float64 [n_phase]
    phase_frac: Optional[np.ndarray]  # float32 [n_phase, nz, ny, nx] or None (n_phase == 1)
    vol_pos_fx: np.ndarray      # int32 [nvox, 3]
    surface_nodes: int          # 1 = one Lambertian node per column at z = 0
    adj_ptr: np.ndarray         # int64 [N + 1]
    adj_idx: np.ndarray         # int32 [E]
    surf_albedo: np.ndarray     # float32 [ny, nx]
    sun_dir: np.ndarray         # int32 [3]
    view_dir: np.ndarray        # int32 [3]
    n_fib: int = 100
    node_weight_mode: int = 0   # 0 = bounded scattering probability, 1 = literal mu_s * voxel edge
    abs_scale: Optional[np.ndarray] = None  # float32 [n_lambda] multipliers of mu_a (batched wavelengths)
    angles: tuple = (0.0, 0.0, 0.0, 0.0)    # (sza, saa, vza, vaa) in degrees, informational
    phase_kind: Optional[np.ndarray] = None  # int32 [n_phase]: 0 Henyey-Greenstein, 1 Rayleigh, 2 table
    phase_lut: Optional[np.ndarray] = None   # float64 [n_phase, n] tables in cos(theta) on [-1, 1]
    sigma_mode: int = 0         # 0 = Voronoi ownership of the lattice, 1 = nearest-point colouring + flood fill
    periodic: int = 0           # bit 0: x, bit 1: y repeat with the grid's period (plane-parallel slabs)
    # general volume nodes (path points of the lines of sight) instead of one per voxel:
    node_pos_fx: Optional[np.ndarray] = None  # int32 [n_vol, 3], anywhere inside the box
    los_ptr: Optional[np.ndarray] = None      # int64 [nx*ny + 1]: pixel p's line-of-sight elements at los_ptr[p] ...
    los_node: Optional[np.ndarray] = None     # int32 [elements]: each element's node (-1: none)
    los_t: Optional[np.ndarray] = None        # float64 [elements]: each element's upper end along the line (t = 1: one view_dir)

    # ---- derived sizes (no method arithmetic) ----
    @property
    def nvox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_vol(self) -> int:
        """Volume nodes: one per voxel, or the general node set."""
        return self.nvox if self.node_pos_fx is None else int(self.node_pos_fx.shape[0])

    @property
    def n_nodes(self) -> int:
        return self.n_vol + (self.nx * self.ny if self.surface_nodes else 0)

    @property
    def n_edges(self) -> int:
        return int(self.adj_idx.shape[0])

    @property
    def n_phase(self) -> int:
        return int(self.hg_g.shape[0])

    @property
    def n_lambda(self) -> int:
        return 1 if self.abs_scale is None else int(self.abs_scale.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.adj_ptr)

    def nnz(self) -> int:
        d = self.degrees().astype(np.int64)
        return int((d * d).sum())

    def nbytes(self) -> int:
        """Bytes of the input arrays handed to the library."""
        arrs = [self.mu_s, self.mu_a, self.hg_g, self.vol_pos_fx, self.adj_ptr, self.adj_idx, self.surf_albedo]
        if self.phase_frac is not None:
            arrs.append(self.phase_frac)
        for a in (self.abs_scale, self.phase_kind, self.phase_lut, self.node_pos_fx, self.los_ptr, self.los_node,
                  self.los_t):
            if a is not None:
                arrs.append(a)
        return int(sum(a.nbytes for a in arrs))

    def all_positions(self) -> np.ndarray:
        """int64 [N, 3] positions of every node (volume then surface)."""
        pos = (self.vol_pos_fx if self.node_pos_fx is None else self.node_pos_fx).astype(np.int64)
        if self.surface_nodes:
            pos = np.concatenate([pos, surface_positions(self.nx, self.ny)], axis=0)
        return pos

    def fingerprint(self) -> str:
        h = hashlib.sha256()
        for a in (self.mu_s, self.mu_a, self.hg_g, self.vol_pos_fx, self.adj_ptr, self.adj_idx,
                  self.surf_albedo, self.sun_dir, self.view_dir):
            h.update(np.ascontiguousarray(a).tobytes())
        if self.phase_frac is not None:
            h.update(np.ascontiguousarray(self.phase_frac).tobytes())
        for a in (self.abs_scale, self.phase_kind, self.phase_lut, self.node_pos_fx, self.los_ptr, self.los_node,
                  self.los_t):
            if a is not None:
                h.update(np.ascontiguousarray(a).tobytes())
        h.update(repr((self.nx, self.ny, self.nz, self.voxel_m, self.surface_nodes, self.n_fib,
                       self.node_weight_mode, self.sigma_mode, self.periodic)).encode())
        return h.hexdigest()[:16]

    def with_(self, **kw) -> "Scene":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------------------
# geometry helpers
# --------------------------------------------------------------------------------------

def surface_positions(nx: int, ny: int) -> np.ndarray:
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.zeros((ny * nx, 3), dtype=np.int64)
    pos[:, 0] = ix.reshape(-1) * FX + FX // 2
    pos[:, 1] = iy.reshape(-1) * FX + FX // 2
    return pos


def direction_fx(zenith_deg: float, azimuth_deg: float) -> np.ndarray:
    """round(2**20 * (sin t cos p, sin t sin p, cos t)) as int32."""
    t = math.radians(zenith_deg)
    p = math.radians(azimuth_deg)
    v = np.array([math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t)])
    return np.rint(v * DIR_SCALE).astype(np.int32)


def jittered_positions(rng: np.random.Generator, nx: int, ny: int, nz: int,
                       jitter: float = 0.25) -> np.ndarray:
    """Voxel centre + U(-jitter, jitter) voxel per axis, quantised to FX (int32 [nvox, 3])."""
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    base = np.stack([ix, iy, iz], axis=-1).reshape(-1, 3).astype(np.float64)
    u = rng.uniform(-jitter, jitter, size=base.shape)
    pos = np.rint((base + 0.5 + u) * FX).astype(np.int64)
    return pos.astype(np.int32)


def _pairs_for_offset(vol: np.ndarray, vid: np.ndarray, off, r2: int):
    """Pairs (a, b) of volume nodes whose voxels differ by off, within squared radius r2."""
    nz, ny, nx, _ = vol.shape
    dx, dy, dz = off
    xs_a = slice(max(0, -dx), nx - max(0, dx))
    ys_a = slice(max(0, -dy), ny - max(0, dy))
    zs_a = slice(max(0, -dz), nz - max(0, dz))
    xs_b = slice(max(0, dx), nx - max(0, -dx))
    ys_b = slice(max(0, dy), ny - max(0, -dy))
    zs_b = slice(max(0, dz), nz - max(0, -dz))
    a = vol[zs_a, ys_a, xs_a]
    b = vol[zs_b, ys_b, xs_b]
    if a.size == 0:
        return None
    d = b - a
    d2 = (d * d).sum(axis=-1)
    m = d2 <= r2
    return vid[zs_a, ys_a, xs_a][m], vid[zs_b, ys_b, xs_b][m]


def radius_graph(vol_pos_fx: np.ndarray, nx: int, ny: int, nz: int, radius_vox: float,
                 surface: bool = True, jitter: float = 0.25):
    """Symmetric adjacency of all node pairs within radius_vox voxel edges.

    Distances are compared exactly in integers on the fixed-point positions:
    pair iff |P_a - P_b|^2 <= floor((radius_vox * FX)^2).  Surface nodes couple
    only to volume nodes.  Returns (adj_ptr int64 [N+1], adj_idx int32 [E]).
    """
    r2 = int(math.floor((radius_vox * FX) ** 2))
    K = int(math.floor(radius_vox + 2 * jitter))
    vol = vol_pos_fx.astype(np.int64).reshape(nz, ny, nx, 3)
    nvox = nx * ny * nz
    vid = np.arange(nvox, dtype=np.int64).reshape(nz, ny, nx)
    tails, heads = [], []
    for dz in range(-K, K + 1):
        for dy in range(-K, K + 1):
            for dx in range(-K, K + 1):
                if (dz, dy, dx) <= (0, 0, 0):
                    continue  # each unordered offset once
                lo = sum(max(0.0, abs(o) - 2 * jitter) ** 2 for o in (dx, dy, dz))
                if lo > radius_vox ** 2:
                    continue
                res = _pairs_for_offset(vol, vid, (dx, dy, dz), r2)
                if res is None:
                    continue
                a, b = res
                tails.append(a)
                heads.append(b)
    n_nodes = nvox
    if surface:
        n_nodes = nvox + nx * ny
        spos = surface_positions(nx, ny).reshape(ny, nx, 3)
        sid = nvox + np.arange(nx * ny, dtype=np.int64).reshape(ny, nx)
        for dz in range(0, K + 1):
            for dy in range(-K, K + 1):
                for dx in range(-K, K + 1):
                    xs_s = slice(max(0, -dx), nx - max(0, dx))
                    ys_s = slice(max(0, -dy), ny - max(0, dy))
                    xs_v = slice(max(0, dx), nx - max(0, -dx))
                    ys_v = slice(max(0, dy), ny - max(0, -dy))
                    if dz >= nz:
                        continue
                    s = spos[ys_s, xs_s]
                    v = vol[dz, ys_v, xs_v]
                    if s.size == 0:
                        continue
                    d = v - s
                    m = (d * d).sum(axis=-1) <= r2
                    tails.append(sid[ys_s, xs_s][m])
                    heads.append(vid[dz, ys_v, xs_v][m])
    if tails:
        t = np.concatenate(tails)
        h = np.concatenate(heads)
    else:
        t = np.zeros(0, np.int64)
        h = np.zeros(0, np.int64)
    return adjacency_from_pairs(n_nodes, t, h)


def periodic_radius_graph(vol_pos_fx: np.ndarray, nx: int, ny: int, nz: int, radius_vox: float,
                          periodic: int, surface: bool = True, jitter: float = 0.25):
    """radius_graph with x (bit 0 of periodic) and/or y (bit 1) repeating with the grid's
    period: distances use the shortest image along those axes.  Needs the grid wider
    than twice the search reach along each periodic axis, so that every pair is found
    once and its shortest image is unique."""
    r2 = int(math.floor((radius_vox * FX) ** 2))
    K = int(math.floor(radius_vox + 2 * jitter))
    if (periodic & 1 and nx <= 2 * K + 1) or (periodic & 2 and ny <= 2 * K + 1):
        raise ValueError("a periodic axis must be wider than twice the search reach")
    W = np.array([nx * FX, ny * FX, 0], np.int64)
    per = np.array([bool(periodic & 1), bool(periodic & 2), False])
    vol = vol_pos_fx.astype(np.int64).reshape(nz, ny, nx, 3)
    nvox = nx * ny * nz
    vid = np.arange(nvox, dtype=np.int64).reshape(nz, ny, nx)

    def shortest(d):
        for k in (0, 1):
            if per[k]:
                d[..., k] -= W[k] * np.round(d[..., k] / W[k]).astype(np.int64)
        return d

    def shifted(a, dy, dx):  # a[y + dy, x + dx] with wrapping on the periodic axes
        return np.roll(np.roll(a, -dy, axis=-2), -dx, axis=-1)

    tails, heads = [], []
    for dz in range(0, min(K, nz - 1) + 1):
        for dy in range(-K, K + 1):
            for dx in range(-K, K + 1):
                if (dz, dy, dx) <= (0, 0, 0):
                    continue
                a_pos, a_id = vol[:nz - dz], vid[:nz - dz]
                b_pos = shifted(vol[dz:].transpose(3, 0, 1, 2), dy, dx).transpose(1, 2, 3, 0)
                b_id = shifted(vid[dz:], dy, dx)
                # pairs whose offset leaves the grid on a non-periodic axis do not exist
                ok = np.ones(a_id.shape, bool)
                yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
                if not per[1]:
                    ok &= ((yy + dy >= 0) & (yy + dy < ny))[None]
                if not per[0]:
                    ok &= ((xx + dx >= 0) & (xx + dx < nx))[None]
                d = shortest(b_pos - a_pos)
                m = ok & ((d * d).sum(axis=-1) <= r2)
                tails.append(a_id[m])
                heads.append(b_id[m])
    n_nodes = nvox
    if surface:
        n_nodes = nvox + nx * ny
        spos = surface_positions(nx, ny).reshape(ny, nx, 3).astype(np.int64)
        sid = nvox + np.arange(nx * ny, dtype=np.int64).reshape(ny, nx)
        yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        for dz in range(0, min(K, nz - 1) + 1):
            for dy in range(-K, K + 1):
                for dx in range(-K, K + 1):
                    v_pos = shifted(vol[dz].transpose(2, 0, 1), dy, dx).transpose(1, 2, 0)
                    v_id = shifted(vid[dz], dy, dx)
                    ok = np.ones((ny, nx), bool)
                    if not per[1]:
                        ok &= (yy + dy >= 0) & (yy + dy < ny)
                    if not per[0]:
                        ok &= (xx + dx >= 0) & (xx + dx < nx)
                    d = shortest(v_pos - spos)
                    m = ok & ((d * d).sum(axis=-1) <= r2)
                    tails.append(sid[m])
                    heads.append(v_id[m])
    t = np.concatenate(tails) if tails else np.zeros(0, np.int64)
    h = np.concatenate(heads) if heads else np.zeros(0, np.int64)
    return adjacency_from_pairs(n_nodes, t, h)


def general_radius_graph(node_pos_fx: np.ndarray, nx: int, ny: int, radius_vox: float, surface: bool = True):
    """Symmetric adjacency of a general node set (positions int [n, 3], then one surface
    node per column when surface): every pair within radius_vox voxel edges, compared exactly
    in integers, |P_a - P_b|^2 <= floor((radius_vox * FX)^2); no surface-surface pairs."""
    from scipy.spatial import cKDTree
    pos = np.asarray(node_pos_fx, np.int64).reshape(-1, 3)
    n_vol = pos.shape[0]
    if surface:
        pos = np.concatenate([pos, surface_positions(nx, ny)], axis=0)
    r2 = int(math.floor((radius_vox * FX) ** 2))
    tree = cKDTree(pos.astype(np.float64))
    pairs = tree.query_pairs(math.sqrt(r2) + 2.0, output_type="ndarray").astype(np.int64)
    if len(pairs):
        d = pos[pairs[:, 0]] - pos[pairs[:, 1]]
        keep = ((d * d).sum(axis=1) <= r2) & ~((pairs[:, 0] >= n_vol) & (pairs[:, 1] >= n_vol))
        pairs = pairs[keep]
    return adjacency_from_pairs(pos.shape[0], pairs[:, 0], pairs[:, 1])


def with_los_nodes(sc: "Scene", node_pos_fx, los_ptr, los_node, los_t, radius_vox=None, name=None) -> "Scene":
    """The scene with general volume nodes on the pixels' lines of sight (positions, the
    per-pixel elements with their nodes and ends) and, with radius_vox, the radius graph over
    them (else an empty graph, to be replaced by the caller's)."""
    pos = np.ascontiguousarray(np.asarray(node_pos_fx).reshape(-1, 3), dtype=np.int32)
    n = pos.shape[0] + (sc.nx * sc.ny if sc.surface_nodes else 0)
    if radius_vox is not None:
        adj_ptr, adj_idx = general_radius_graph(pos, sc.nx, sc.ny, radius_vox, surface=bool(sc.surface_nodes))
    else:
        adj_ptr, adj_idx = np.zeros(n + 1, np.int64), np.zeros(0, np.int32)
    return dataclasses.replace(sc, name=name or sc.name + "-los", node_pos_fx=pos,
                               los_ptr=np.ascontiguousarray(los_ptr, dtype=np.int64),
                               los_node=np.ascontiguousarray(los_node, dtype=np.int32),
                               los_t=np.ascontiguousarray(los_t, dtype=np.float64), adj_ptr=adj_ptr, adj_idx=adj_idx)


def adjacency_from_pairs(n_nodes: int, a: np.ndarray, b: np.ndarray):
    """CSR (adj_ptr, adj_idx) of the symmetric graph with the unordered pairs (a, b)."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    tail = np.concatenate([a, b])
    head = np.concatenate([b, a])
    key = np.unique(tail * n_nodes + head)
    tail = key // n_nodes
    head = key % n_nodes
    counts = np.bincount(tail, minlength=n_nodes)
    adj_ptr = np.zeros(n_nodes + 1, dtype=np.int64)
    np.cumsum(counts, out=adj_ptr[1:])
    return adj_ptr, head.astype(np.int32)


def voxel_centres_m(nx: int, ny: int, nz: int, dx: float):
    z = (np.arange(nz) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dx
    x = (np.arange(nx) + 0.5) * dx
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


# --------------------------------------------------------------------------------------
# extinction fields
# --------------------------------------------------------------------------------------

def rayleigh_background(nx, ny, nz, dx, k0=1.2e-5, scale_height=8000.0):
    _, _, Z = voxel_centres_m(nx, ny, nz, dx)
    return k0 * np.exp(-Z / scale_height)


def plume_field(rng, nx, ny, nz, dx, peak=5e-3, sigma=300.0, n_puffs=30):
    """Bent Gaussian-puff plume: source in the central half of the domain at
    150 m, random wind azimuth, centreline bending with radius U[2, 6] km to a
    random side, rising as 300 m (1 - exp(-s / 500 m)), length 0.6 x domain
    width, rescaled so that the voxel maximum equals peak."""
    X, Y, Z = voxel_centres_m(nx, ny, nz, dx)
    W = nx * dx
    sx = rng.uniform(0.25, 0.75) * nx * dx
    sy = rng.uniform(0.25, 0.75) * ny * dx
    psi = rng.uniform(0.0, 2.0 * math.pi)
    rc = rng.uniform(2000.0, 6000.0)
    side = 1.0 if rng.uniform() < 0.5 else -1.0
    L = 0.6 * W
    s = np.linspace(0.0, L, n_puffs)
    heading = psi + side * s / rc
    cx = sx + side * rc * (np.sin(heading) - math.sin(psi))
    cy = sy - side * rc * (np.cos(heading) - math.cos(psi))
    cz = 150.0 + 300.0 * (1.0 - np.exp(-s / 500.0))
    f = np.zeros_like(X)
    inv = 1.0 / (2.0 * sigma * sigma)
    for k in range(n_puffs):
        f += np.exp(-((X - cx[k]) ** 2 + (Y - cy[k]) ** 2 + (Z - cz[k]) ** 2) * inv)
    f *= peak / f.max()
    return f


def cloud_field(rng, nx, ny, nz, dx, kmax=0.05):
    """6-12 ellipsoidal blobs with parabolic profile k_peak (1 - r^2), summed and clipped at kmax."""
    X, Y, Z = voxel_centres_m(nx, ny, nz, dx)
    Xw, Yw, Hz = nx * dx, ny * dx, nz * dx
    nb = int(rng.integers(6, 13))
    f = np.zeros_like(X)
    for _ in range(nb):
        cx = rng.uniform(0.1, 0.9) * Xw
        cy = rng.uniform(0.1, 0.9) * Yw
        cz = rng.uniform(0.25, 0.75) * Hz
        a = rng.uniform(300.0, 1000.0)
        b = rng.uniform(300.0, 1000.0)
        c = rng.uniform(150.0, 400.0)
        yaw = rng.uniform(0.0, math.pi)
        kp = rng.uniform(0.02, 0.05)
        ddx, ddy = X - cx, Y - cy
        u = math.cos(yaw) * ddx + math.sin(yaw) * ddy
        v = -math.sin(yaw) * ddx + math.cos(yaw) * ddy
        r2 = (u / a) ** 2 + (v / b) ** 2 + ((Z - cz) / c) ** 2
        f += np.where(r2 < 1.0, kp * (1.0 - r2), 0.0)
    return np.minimum(f, kmax)


# --------------------------------------------------------------------------------------
# the benchmark configurations
# --------------------------------------------------------------------------------------

def _finish(name, seed, nx, ny, nz, dx, mu_s, mu_a, hg_g, phase_frac, pos, R, albedo,
            sza, saa, vza, vaa, surface=True, n_fib=100, abs_scale=None, periodic=0):
    if periodic:
        adj_ptr, adj_idx = periodic_radius_graph(pos, nx, ny, nz, R, periodic, surface=surface)
    else:
        adj_ptr, adj_idx = radius_graph(pos, nx, ny, nz, R, surface=surface)
    return Scene(
        name=name, seed=seed, nx=nx, ny=ny, nz=nz, voxel_m=float(dx),
        mu_s=np.ascontiguousarray(mu_s, dtype=np.float32),
        mu_a=np.ascontiguousarray(mu_a, dtype=np.float32),
        hg_g=np.asarray(hg_g, dtype=np.float64),
        phase_frac=None if phase_frac is None else np.ascontiguousarray(phase_frac, dtype=np.float32),
        vol_pos_fx=pos, surface_nodes=1 if surface else 0,
        adj_ptr=adj_ptr, adj_idx=adj_idx,
        surf_albedo=np.ascontiguousarray(albedo, dtype=np.float32),
        sun_dir=direction_fx(sza, saa), view_dir=direction_fx(vza, vaa),
        n_fib=n_fib, abs_scale=None if abs_scale is None else np.asarray(abs_scale, np.float32),
        angles=(sza, saa, vza, vaa), periodic=periodic)


def make_plain(seed=1, nx=8, ny=8, nz=8, dx=100.0, R=2.0):
    """Plain case: lognormal extinction exp(-3 + 0.5 Z), albedo 0.9, HG g 0.7, surface 0.2,
    SZA 30 / SAA 30, nadir view."""
    rng = np.random.default_rng(seed)
    pos = jittered_positions(rng, nx, ny, nz)
    mu_e = np.exp(-3.0 + 0.5 * rng.standard_normal((nz, ny, nx)))
    mu_s = 0.9 * mu_e
    mu_a = 0.1 * mu_e
    alb = np.full((ny, nx), 0.2)
    return _finish("plain-8x8x8", seed, nx, ny, nz, dx, mu_s, mu_a, [0.7], None, pos, R, alb,
                   30.0, 30.0, 0.0, 0.0)


def make_plume(seed=2, nx=64, ny=64, nz=32, dx=50.0, R=1.8, name=None, n_lambda=0, periodic=0):
    """Emission plume over a Rayleigh-like background; albedo 0.95, g 0.75,
    surface albedo U[0.1, 0.3], SZA 50 / SAA 30, VZA 20 / VAA 120.  periodic: the grid
    repeats along x (bit 0) and/or y (bit 1), the graph searches across the period."""
    rng = np.random.default_rng(seed)
    pos = jittered_positions(rng, nx, ny, nz)
    mu_e = rayleigh_background(nx, ny, nz, dx) + plume_field(rng, nx, ny, nz, dx)
    alb = rng.uniform(0.1, 0.3, size=(ny, nx))
    abs_scale = None
    if n_lambda > 0:
        abs_scale = 10.0 ** rng.uniform(-1.0, 1.0, size=n_lambda)
    return _finish(name or f"plume-{nx}x{ny}x{nz}" + (f"-p{periodic}" if periodic else ""), seed, nx, ny, nz, dx,
                   0.95 * mu_e, 0.05 * mu_e, [0.75], None, pos, R, alb, 50.0, 30.0, 20.0, 120.0,
                   abs_scale=abs_scale, periodic=periodic)


def make_cloud(seed=3, nx=128, ny=128, nz=48, dx=50.0, R=1.8, name=None, n_lambda=0):
    """Ellipsoidal clouds (albedo 0.999, g 0.85) over a conservative Rayleigh-like background
    (g 0), mixed by scattering coefficient; surface albedo 0.2; SZA 70 / SAA 30, VZA 40 / VAA 120."""
    rng = np.random.default_rng(seed)
    pos = jittered_positions(rng, nx, ny, nz)
    bg = rayleigh_background(nx, ny, nz, dx)
    cl = cloud_field(rng, nx, ny, nz, dx)
    mu_s = bg + 0.999 * cl
    mu_a = 0.001 * cl
    frac = np.stack([0.999 * cl / mu_s, bg / mu_s])
    alb = np.full((ny, nx), 0.2)
    abs_scale = None
    if n_lambda > 0:
        abs_scale = 10.0 ** rng.uniform(-1.0, 1.0, size=n_lambda)
    return _finish(name or f"cloud-{nx}x{ny}x{nz}", seed, nx, ny, nz, dx, mu_s, mu_a,
                   [0.85, 0.0], frac, pos, R, alb, 70.0, 30.0, 40.0, 120.0, abs_scale=abs_scale)


def make_batched(seed=4, nx=96, ny=96, nz=32, dx=50.0, n_lambda=64):
    """Plume generator on 96x96x32 with n_lambda absorption multipliers 10**U[-1, 1]."""
    return make_plume(seed=seed, nx=nx, ny=ny, nz=nz, dx=dx, name=f"batched-{nx}x{ny}x{nz}x{n_lambda}",
                      n_lambda=n_lambda)


def served_stream_params(i: int):
    """(generator, nx, ny, nz, n_lambda, seed) of request i of the served stream."""
    seed = 5000 + i
    rng = np.random.default_rng(seed)
    nx = int(rng.integers(16, 129))
    ny = int(rng.integers(16, 129))
    nz = int(rng.integers(16, 49))
    nl = int(rng.integers(1, 33))
    gen = "plume" if seed % 2 == 0 else "cloud"
    return gen, nx, ny, nz, nl, seed


def make_served(i: int, max_voxels: Optional[int] = None):
    gen, nx, ny, nz, nl, seed = served_stream_params(i)
    if max_voxels is not None:
        while nx * ny * nz > max_voxels:
            nx, ny, nz = max(4, nx // 2), max(4, ny // 2), max(4, nz // 2)
    f = make_plume if gen == "plume" else make_cloud
    return f(seed=seed, nx=nx, ny=ny, nz=nz, name=f"served-{i}-{gen}-{nx}x{ny}x{nz}x{nl}", n_lambda=nl)


CONFIGS = {
    "plain": make_plain,
    "plume": make_plume,
    "cloud": make_cloud,
    "batched": make_batched,
}


# --------------------------------------------------------------------------------------
# small scenes for tests
# --------------------------------------------------------------------------------------

def make_homogeneous(nx=6, ny=6, nz=4, dx=100.0, mu_e=0.004, omega=0.9, g=0.7, albedo=0.2,
                     R=1.8, sza=30.0, saa=30.0, vza=0.0, vaa=0.0, seed=7, surface=True,
                     graph=True, layers=None):
    """Homogeneous (or horizontally homogeneous layered, via layers[nz]) medium."""
    rng = np.random.default_rng(seed)
    pos = jittered_positions(rng, nx, ny, nz)
    k = np.full((nz, ny, nx), mu_e, dtype=np.float64)
    if layers is not None:
        k = np.broadcast_to(np.asarray(layers, np.float64)[:, None, None], (nz, ny, nx)).copy()
    alb = np.full((ny, nx), albedo)
    sc = _finish(f"homog-{nx}x{ny}x{nz}", seed, nx, ny, nz, dx, omega * k, (1.0 - omega) * k,
                 [g], None, pos, R, alb, sza, saa, vza, vaa, surface=surface)
    if not graph:
        n = sc.n_nodes
        sc = sc.with_(adj_ptr=np.zeros(n + 1, np.int64), adj_idx=np.zeros(0, np.int32))
    return sc


def make_random_small(seed, nx=3, ny=3, nz=3, dx=100.0, R=1.8, two_phase=False, surface=True,
                      sza=40.0, saa=30.0, vza=25.0, vaa=120.0, kscale=1.0):
    """Small random scene with lognormal extinction, random albedo per voxel."""
    rng = np.random.default_rng(seed)
    pos = jittered_positions(rng, nx, ny, nz)
    mu_e = kscale * np.exp(-5.0 + 1.0 * rng.standard_normal((nz, ny, nx)))
    om = rng.uniform(0.5, 1.0, size=(nz, ny, nx))
    mu_s = om * mu_e
    mu_a = (1.0 - om) * mu_e
    alb = rng.uniform(0.0, 0.5, size=(ny, nx))
    if two_phase:
        fr = rng.uniform(0.0, 1.0, size=(nz, ny, nx))
        frac = np.stack([fr, 1.0 - fr])
        gg = [0.8, -0.3]
    else:
        frac = None
        gg = [0.6]
    return _finish(f"rand-{nx}x{ny}x{nz}-s{seed}", seed, nx, ny, nz, dx, mu_s, mu_a, gg, frac, pos,
                   R, alb, sza, saa, vza, vaa, surface=surface)


def make_slab(nx=12, ny=10, nz=6, dx=100.0, layers=(0.02, 0.01, 0.004, 0.002, 0.001, 0.0005), omega=0.9,
              g=0.7, albedo=0.2, R=1.8, periodic=3, jitter=None, seed=13, sza=40.0, saa=30.0, vza=25.0,
              vaa=120.0, n_lambda=0):
    """Horizontally homogeneous layers (extinction layers[iz] in 1/m), periodic in x and y
    (plane-parallel slab): with nodes at the voxel centres (jitter None) every column
    sees the same medium, so every pixel has the same radiance."""
    rng = np.random.default_rng(seed)
    pos = (jittered_positions(rng, nx, ny, nz) if jitter is not None else
           jittered_positions(rng, nx, ny, nz, jitter=0.0))
    ke = np.broadcast_to(np.asarray(layers[:nz], np.float64)[:, None, None], (nz, ny, nx))
    alb = np.full((ny, nx), albedo)
    adj_ptr, adj_idx = periodic_radius_graph(pos, nx, ny, nz, R, periodic,
                                             jitter=0.25 if jitter is None else jitter)
    abs_scale = None
    if n_lambda > 0:
        abs_scale = np.geomspace(0.3, 3.0, n_lambda).astype(np.float32)
    return Scene(name=f"slab-{nx}x{ny}x{nz}-p{periodic}", seed=seed, nx=nx, ny=ny, nz=nz, voxel_m=float(dx),
                 mu_s=np.ascontiguousarray(omega * ke, dtype=np.float32),
                 mu_a=np.ascontiguousarray((1 - omega) * ke, dtype=np.float32),
                 hg_g=np.array([g]), phase_frac=None, vol_pos_fx=pos, surface_nodes=1, adj_ptr=adj_ptr,
                 adj_idx=adj_idx, surf_albedo=np.ascontiguousarray(alb, dtype=np.float32),
                 sun_dir=direction_fx(sza, saa), view_dir=direction_fx(vza, vaa), abs_scale=abs_scale,
                 angles=(sza, saa, vza, vaa), periodic=periodic)


def make_worked_example(dx=100.0, mu_e=0.002, omega=0.9, g=0.7, seed=11):
    """Four nodes, r3 coupled to r1, r2 and r4 (the paper's Sec. 2.1 example, Fig. 1).

    Nodes 0..3 stand for r1..r4 in a 2 x 2 x 1 grid; no surface nodes."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = 2, 2, 1
    pos = jittered_positions(rng, nx, ny, nz)
    k = np.full((nz, ny, nx), mu_e)
    adj_ptr, adj_idx = adjacency_from_pairs(4, np.array([0, 1, 3]), np.array([2, 2, 2]))
    return Scene(name="worked-example", seed=seed, nx=nx, ny=ny, nz=nz, voxel_m=dx,
                 mu_s=(omega * k).astype(np.float32), mu_a=((1 - omega) * k).astype(np.float32),
                 hg_g=np.array([g]), phase_frac=None, vol_pos_fx=pos, surface_nodes=0,
                 adj_ptr=adj_ptr, adj_idx=adj_idx, surf_albedo=np.zeros((ny, nx), np.float32),
                 sun_dir=direction_fx(30.0, 30.0), view_dir=direction_fx(0.0, 0.0))

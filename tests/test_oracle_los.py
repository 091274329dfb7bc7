"""Pins of the oracle's scattering nodes on the lines of sight (Sec. 2: the nodes of the
scattering graph are path points of the lines of sight, taken at each layer of the medium or
at constant distance intervals; Sec. 3, step 1 of the algorithm).

Independent checks:
  * geometry of the placement against the pinned voxel walk: every node lies on its pixel's
    line of sight (within the rounding to fixed point); a layer node sits at the middle height
    of its layer wherever the line crosses the layer whole; constant-step nodes are the step
    apart; the elements of a line are its layers or its steps, in order;
  * with a nadir view the layer nodes are the voxel centres, and the scene on them
    reproduces the one-node-per-voxel scene with nodes at the centres (K, S, pixels);
  * the single-scattering image of a horizontally homogeneous periodic slab with layer nodes
    on slant lines of sight is the plane-parallel closed form at every pixel; with nodes at a
    constant step it is the same integral with the source of each step element taken at its
    node, evaluated here from the analytic intersections of the layers and the elements;
  * the coupling graph (Eq. 4) over general nodes is the set of strongest couplings of an
    independent numpy evaluation (standardisation, principal axes, the voxel's mu_s).
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_2503_16037_amd import scenes

FX = scenes.FX


def walk(sc, p):
    """Voxels and parameter lengths of pixel p's line of sight (the pinned walk)."""
    P = np.array([(p % sc.nx) * FX + FX // 2, (p // sc.nx) * FX + FX // 2, 0])
    return P, oracle.trace(sc.nx, sc.ny, sc.nz, P, sc.view_dir, 1, periodic=sc.periodic)


def dist_to_line(q, P, D):
    d = np.asarray(D, np.float64)
    v = np.asarray(q, np.float64) - np.asarray(P, np.float64)
    return np.linalg.norm(v - (v @ d) / (d @ d) * d)


@pytest.mark.parametrize("vza,vaa,periodic", [(0.0, 0.0, 0), (25.0, 120.0, 0), (40.0, 300.0, 0), (35.0, 70.0, 3)])
def test_layer_nodes_geometry(vza, vaa, periodic):
    sc = scenes.make_random_small(3, nx=7, ny=6, nz=5, vza=vza, vaa=vaa)
    sc = dataclasses.replace(sc, periodic=periodic)
    pos, lp, ln, lt = oracle.los_nodes(sc.nx, sc.ny, sc.nz, sc.view_dir, sc.voxel_m, "layer", periodic=periodic)
    nxy = sc.nx * sc.ny
    W = np.array([sc.nx * FX, sc.ny * FX, 1 << 62])
    D = np.asarray(sc.view_dir, np.float64)
    used = []
    for p in range(nxy):
        P, (vox, dt) = walk(sc, p)
        t = np.concatenate([[0.0], np.cumsum(dt)])
        z = vox // nxy
        layers = list(dict.fromkeys(z.tolist()))
        els = range(lp[p], lp[p + 1])
        assert len(els) == len(layers)  # one element per layer crossed, in order
        start = 0.0
        for e, zl in zip(els, layers):
            ks = np.flatnonzero(z == zl)
            # the element ends where the layer's last chord ends
            assert lt[e] == pytest.approx(t[ks[-1] + 1], rel=1e-14)
            assert t[ks[0]] == pytest.approx(start, abs=1e-14)
            start = lt[e]
            if ln[e] < 0:
                continue
            used.append(int(ln[e]))
            q = pos[ln[e]].astype(np.int64)
            ref = P + 0.5 * (t[ks[0]] + t[ks[-1] + 1]) * D
            for a in (0, 1):
                if periodic & (1 << a):
                    q[a] += int(round((ref[a] - q[a]) / W[a])) * W[a]
            assert np.abs(q - ref).max() <= 0.5 + 1e-6
            assert dist_to_line(q, P, D) <= 1.0
            assert q[2] // FX == zl
            # a layer crossed whole has its node at the middle height
            whole = abs(t[ks[-1] + 1] * D[2] - (zl + 1) * FX) < 1e-6 * FX and abs(t[ks[0]] * D[2] - zl * FX) < 1e-6 * FX
            if whole:
                assert q[2] == zl * FX + FX // 2
    # every node belongs to exactly one element, in id order
    assert used == list(range(len(pos)))


@pytest.mark.parametrize("step_m", [37.0, 100.0, 260.0])
def test_step_nodes_geometry(step_m):
    sc = scenes.make_random_small(4, nx=6, ny=6, nz=4, vza=30.0, vaa=40.0)
    pos, lp, ln, lt = oracle.los_nodes(sc.nx, sc.ny, sc.nz, sc.view_dir, sc.voxel_m, "step", step_m=step_m)
    D = np.asarray(sc.view_dir, np.float64)
    plen = np.linalg.norm(D) * sc.voxel_m / FX  # metres per unit of the line parameter
    used = []
    for p in range(sc.nx * sc.ny):
        P, (vox, dt) = walk(sc, p)
        t_exit = np.sum(dt)
        ends = lt[lp[p]:lp[p + 1]]
        # elements one step long, the last clipped at the line's exit
        assert len(ends) == int(math.ceil(t_exit * plen / step_m - 1e-12))
        assert np.allclose(np.diff(np.concatenate([[0.0], ends[:-1]])) * plen, step_m, rtol=1e-12)
        assert ends[-1] == pytest.approx(t_exit, rel=1e-14)
        starts = np.concatenate([[0.0], ends[:-1]])
        for e in range(lp[p], lp[p + 1]):
            if ln[e] < 0:
                continue
            used.append(int(ln[e]))
            q = pos[ln[e]]
            mid = 0.5 * (starts[e - lp[p]] + ends[e - lp[p]])
            assert np.abs(q - (P + mid * D)).max() <= 0.5 + 1e-6
            assert dist_to_line(q, P, D) <= 1.0
    assert used == list(range(len(pos)))


def centred(sc):
    """The scene with its nodes at the voxel centres and the radius graph on them."""
    pos = scenes.jittered_positions(np.random.default_rng(0), sc.nx, sc.ny, sc.nz, jitter=0.0)
    adj_ptr, adj_idx = scenes.radius_graph(pos, sc.nx, sc.ny, sc.nz, 1.8, surface=bool(sc.surface_nodes), jitter=0.0)
    return dataclasses.replace(sc, vol_pos_fx=pos, adj_ptr=adj_ptr, adj_idx=adj_idx)


@pytest.mark.parametrize("two_phase", [False, True])
def test_nadir_layer_nodes_reproduce_the_per_voxel_scene(two_phase):
    sc = centred(scenes.make_random_small(6, nx=5, ny=4, nz=4, vza=0.0, vaa=0.0, two_phase=two_phase, kscale=3.0))
    pos, lp, ln, lt = oracle.los_nodes(sc.nx, sc.ny, sc.nz, sc.view_dir, sc.voxel_m, "layer")
    # the layer nodes of a nadir view are the voxel centres, column by column
    assert len(pos) == sc.nvox and np.all(ln >= 0)
    vid = (pos[:, 0] // FX) + sc.nx * ((pos[:, 1] // FX) + sc.ny * (pos[:, 2] // FX))
    assert np.array_equal(np.sort(vid), np.arange(sc.nvox))
    assert np.array_equal(pos, np.asarray(sc.vol_pos_fx, np.int64)[vid])
    los = scenes.with_los_nodes(sc, pos, lp, ln, lt, radius_vox=1.8)
    a, b = oracle.run(sc), oracle.run(los)
    assert np.allclose(b["radiance"], a["radiance"], rtol=1e-12, atol=0)
    # the same matrix up to the renumbering of the nodes (and with it of the edges)
    assert b["nnz"] == a["nnz"] and np.isclose(np.sort(b["val"]), np.sort(a["val"]), rtol=1e-12).all()
    assert np.allclose(np.sort(b["S"]), np.sort(a["S"]), rtol=1e-12)


def test_layer_nodes_single_scatter_is_the_plane_parallel_closed_form():
    from test_oracle_periodic import LAYERS, closed_single_scatter
    sc = scenes.make_slab(layers=LAYERS, omega=0.9, g=0.7, albedo=0.2, vza=35.0, vaa=70.0)
    pos, lp, ln, lt = oracle.los_nodes(sc.nx, sc.ny, sc.nz, sc.view_dir, sc.voxel_m, "layer", periodic=sc.periodic)
    assert np.all(ln >= 0) and len(pos) == sc.nx * sc.ny * sc.nz  # slant lines never leave a periodic slab
    los = scenes.with_los_nodes(sc, pos, lp, ln, lt)  # no couplings: single scattering needs none
    ref = closed_single_scatter(sc, 0.7)
    pix = oracle.run(los, scatter_order=1)["radiance"]
    assert np.abs(pix - ref).max() <= 1e-12 * ref
    # nodes at a constant step along the line are another discretisation of the same
    # integral: close, not equal
    pos2, lp2, ln2, lt2 = oracle.los_nodes(sc.nx, sc.ny, sc.nz, sc.view_dir, sc.voxel_m, "step", step_m=30.0,
                                           periodic=sc.periodic)
    pix2 = oracle.run(scenes.with_los_nodes(sc, pos2, lp2, ln2, lt2), scatter_order=1)["radiance"]
    err = np.abs(pix2 - ref).max() / ref
    assert 1e-9 < err < 2e-2


def numpy_couplings_general(sc):
    """C of every candidate pair of a general node set: numpy standardisation and
    principal axes, a volume node's mu_s read from the voxel that contains it."""
    pos = np.asarray(sc.node_pos_fx, np.float64)
    ip = np.asarray(sc.node_pos_fx, np.int64) // FX
    mus = np.asarray(sc.mu_s, np.float64)
    mu = mus[ip[:, 2], ip[:, 1], ip[:, 0]]
    n_vol = len(mu)
    if sc.surface_nodes:
        jj, ii = np.meshgrid(np.arange(sc.ny), np.arange(sc.nx), indexing="ij")
        sp = np.stack([ii.reshape(-1) * FX + FX // 2, jj.reshape(-1) * FX + FX // 2, np.zeros(sc.nx * sc.ny)], -1)
        pos = np.concatenate([pos, sp])
        mu = np.concatenate([mu, np.asarray(sc.surf_albedo, np.float64).reshape(-1) * mus.max()])
    z = (pos - pos.mean(0)) / pos.std(0)
    _, V = np.linalg.eigh(np.cov(z.T, bias=True))
    r = z @ V
    i, j = np.triu_indices(len(mu), 1)
    keep = ~((i >= n_vol) & (j >= n_vol))
    i, j = i[keep], j[keep]
    return i, j, np.sqrt(mu[i] * mu[j]) / np.linalg.norm(r[i] - r[j], axis=1)


@pytest.mark.parametrize("mode", ["layer", "step"])
def test_coupling_graph_of_line_of_sight_nodes(mode):
    sc = scenes.make_random_small(8, nx=6, ny=5, nz=4, vza=30.0, vaa=200.0, kscale=2.0)
    pos, lp, ln, lt = oracle.los_nodes(sc.nx, sc.ny, sc.nz, sc.view_dir, sc.voxel_m, mode, step_m=70.0)
    los = scenes.with_los_nodes(sc, pos, lp, ln, lt)
    i, j, C = numpy_couplings_general(los)
    order = np.argsort(-C, kind="stable")
    n = 4 * len(pos)
    got = set()
    ap, ai = oracle.coupling_graph(los, n_pairs=n)
    for r in range(len(ap) - 1):
        got |= {(r, int(c)) for c in ai[ap[r]:ap[r + 1]] if r < c}
    want = {(int(i[o]), int(j[o])) for o in order[:n]}
    cut = C[order[n - 1]]
    sel = dict(zip(zip(i.tolist(), j.tolist()), C.tolist()))
    assert len(got) == n and all(abs(sel[p] - cut) <= 1e-12 * cut for p in got ^ want)
    # and the scene on that graph solves (every pixel finite and positive)
    pix = oracle.run(dataclasses.replace(los, adj_ptr=ap, adj_idx=ai))["radiance"]
    assert np.all(np.isfinite(pix)) and pix.min() > 0


@pytest.mark.parametrize("step_m", [23.0, 61.0, 140.0])
def test_step_nodes_single_scatter_is_the_plane_parallel_sum(step_m):
    """Single scattering in a periodic layered slab with nodes every step_m metres along the
    slant lines of sight: each element [a, b] of a line scatters, toward the sensor, its
    node's sun beam Theta T_sun(z_node) with the exact chord weight of every layer piece it
    contains, attenuated above it; computed here from the layer and element intervals
    (vertical optical depths divided by the cosines), not by a walk."""
    from test_oracle_periodic import LAYERS
    g = 0.7
    sc = scenes.make_slab(layers=LAYERS, omega=0.9, g=g, albedo=0.2, vza=35.0, vaa=70.0)
    pos, lp, ln, lt = oracle.los_nodes(sc.nx, sc.ny, sc.nz, sc.view_dir, sc.voxel_m, "step", step_m=step_m,
                                       periodic=sc.periodic)
    pix = oracle.run(scenes.with_los_nodes(sc, pos, lp, ln, lt), scatter_order=1)["radiance"]
    dz = sc.voxel_m
    D = np.asarray(sc.view_dir, np.float64)
    su = np.asarray(sc.sun_dir, np.float64)
    su, vu = su / np.linalg.norm(su), D / np.linalg.norm(D)
    mu0, muv = su[2], vu[2]
    mu = float(np.dot(-su, vu))
    theta = (1 - g * g) / (4 * np.pi * (1 + g * g - 2 * g * mu) ** 1.5)
    ms = np.asarray(sc.mu_s, np.float64)[:, 0, 0]
    me = ms + np.asarray(sc.mu_a, np.float64)[:, 0, 0]
    bounds = np.arange(sc.nz + 1) * dz  # layer boundaries, metres

    def tau_above(z):  # vertical optical depth from height z (metres) to the top
        return sum(me[k] * max(0.0, bounds[k + 1] - max(z, bounds[k])) for k in range(sc.nz))

    zt = lambda t: t * D[2] * dz / FX  # height of line parameter t
    tot = tau_above(0.0)
    albedo = float(np.asarray(sc.surf_albedo, np.float64)[0, 0])  # as stored (float32)
    worst = 0.0
    for p in range(sc.nx * sc.ny):
        I = 0.0
        a = 0.0
        for e in range(lp[p], lp[p + 1]):
            b = lt[e]
            zn = pos[ln[e]][2] * dz / FX  # the node's height (rounded position)
            J = theta * math.exp(-tau_above(zn) / mu0)
            for k in range(sc.nz):  # the element's piece in layer k
                lo, hi = max(zt(a), bounds[k]), min(zt(b), bounds[k + 1])
                if hi > lo:
                    w = (ms[k] / me[k]) * (-math.expm1(-me[k] * (hi - lo) / muv))
                    I += math.exp(-tau_above(hi) / muv) * w * J
            a = b
        I += math.exp(-tot / muv) * (albedo / np.pi) * mu0 * math.exp(-tot / mu0)
        worst = max(worst, abs(pix.reshape(-1)[p] - I) / I)
    assert worst <= 1e-12

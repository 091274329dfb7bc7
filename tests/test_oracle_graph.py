"""Pins of the oracle's scattering graph (Sec. 2, Eq. 4; relative positions and the
Lambertian coupling of Sec. 3), each against something other than the oracle's own
arithmetic: a lattice whose ranking follows in closed form from the per-axis scaling,
an independent numpy evaluation of C on principal-axis coordinates, exact counts.
"""
import types

import numpy as np
import pytest

import oracle
from paper_2503_16037_amd import scenes

FX = 1 << 16


def lattice_scene(nx, ny, nz, mu=0.01, surface=False, albedo=0.3, jitter_seed=None):
    """Nodes at voxel centres (or jittered), uniform mu_s."""
    idx = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1)
    idx = idx.transpose(2, 1, 0, 3).reshape(-1, 3)  # canonical order: x fastest, then y, then z
    pos = idx * FX + FX // 2
    if jitter_seed is not None:
        rng = np.random.default_rng(jitter_seed)
        pos = pos + rng.integers(-FX // 4, FX // 4, size=pos.shape)
    return types.SimpleNamespace(nx=nx, ny=ny, nz=nz, vol_pos_fx=pos.astype(np.int32),
                                 mu_s=np.full((nz, ny, nx), mu, np.float32), surface_nodes=surface,
                                 surf_albedo=np.full((ny, nx), albedo, np.float32))


def pairs_of(adj_ptr, adj_idx):
    out = set()
    for i in range(len(adj_ptr) - 1):
        for j in adj_idx[adj_ptr[i]:adj_ptr[i + 1]]:
            if i < j:
                out.add((i, int(j)))
    return out


def numpy_couplings(sc):
    """C for every candidate pair, from numpy's own standardisation and principal-axis
    projection (eigh of the covariance), with the square-root form of Eq. 4."""
    nvox = sc.nx * sc.ny * sc.nz
    pos = np.asarray(sc.vol_pos_fx, np.float64)
    mu = np.asarray(sc.mu_s, np.float64).reshape(-1)
    if sc.surface_nodes:
        jj, ii = np.meshgrid(np.arange(sc.ny), np.arange(sc.nx), indexing="ij")
        sp = np.stack([ii.reshape(-1) * FX + FX // 2, jj.reshape(-1) * FX + FX // 2, np.zeros(sc.nx * sc.ny)], -1)
        pos = np.concatenate([pos, sp])
        mu = np.concatenate([mu, np.asarray(sc.surf_albedo, np.float64).reshape(-1) * mu.max()])
    z = (pos - pos.mean(0)) / pos.std(0)
    w, V = np.linalg.eigh(np.cov(z.T, bias=True))
    r = z @ V  # coordinates on the principal axes
    N = len(mu)
    i, j = np.triu_indices(N, 1)
    keep = ~((i >= nvox) & (j >= nvox))
    i, j = i[keep], j[keep]
    C = np.sqrt(mu[i] * mu[j]) / np.linalg.norm(r[i] - r[j], axis=1)
    return i, j, C, z


def test_scaled_coordinates_match_numpy_standardisation():
    sc = scenes.make_plain()
    P, mu, q = oracle.coupling_nodes(sc)
    _, _, _, z = numpy_couplings(sc)
    assert np.abs(q - z).max() < 1e-12
    nvox = sc.nx * sc.ny * sc.nz
    # Lambertian surface nodes couple with albedo x the largest mu_s of the medium
    assert np.array_equal(mu[nvox:], sc.surf_albedo.reshape(-1).astype(np.float64) * sc.mu_s.max())


def test_lattice_ranking_follows_the_axis_scaling():
    # 8 x 4 x 2 voxel centres: per-axis standard deviations 2.29, 1.12, 0.5 voxels, so in
    # scaled coordinates x-neighbours (0.436) are strictly closest, then pairs two steps
    # apart in x (0.873), then y-neighbours (0.894); unscaled distances would tie all
    # axis neighbours
    sc = lattice_scene(8, 4, 2)
    xn = {(a, a + 1) for a in range(64) if a % 8 != 7}
    x2 = {(a, a + 2) for a in range(64) if a % 8 < 6}
    assert len(xn) == 56 and len(x2) == 48
    assert pairs_of(*oracle.coupling_graph(sc, n_pairs=56)) == xn
    assert pairs_of(*oracle.coupling_graph(sc, n_pairs=104)) == xn | x2


def test_equal_couplings_go_to_the_smallest_pairs():
    # 2 x 2 x 2 voxel centres: every axis has mean 2^16 and standard deviation 2^15
    # fixed-point units, so the scaled coordinates are exactly +-1 and the 12 axis
    # neighbour pairs tie exactly (k = mu^2 / 4), ahead of face (8) and body (12)
    # diagonals
    sc = lattice_scene(2, 2, 2)
    P, mu, q = oracle.coupling_nodes(sc)
    assert set(np.unique(q).tolist()) == {-1.0, 1.0}
    axis = sorted((a, b) for a in range(8) for b in range(a + 1, 8) if bin(a ^ b).count("1") == 1)
    assert len(axis) == 12
    assert pairs_of(*oracle.coupling_graph(sc, n_pairs=5)) == set(axis[:5])
    assert pairs_of(*oracle.coupling_graph(sc, n_pairs=12)) == set(axis)


@pytest.mark.parametrize("surface", [False, True])
def test_top_n_is_the_n_strongest_couplings(surface):
    sc = scenes.make_plain() if surface else lattice_scene(9, 7, 5, jitter_seed=3)
    if not surface:
        sc.mu_s = np.random.default_rng(4).lognormal(-3, 0.5, size=sc.mu_s.shape).astype(np.float32)
    i, j, C, _ = numpy_couplings(sc)
    order = np.argsort(-C, kind="stable")
    n = 2500
    got = pairs_of(*oracle.coupling_graph(sc, n_pairs=n))
    assert len(got) == n
    want = {(int(i[o]), int(j[o])) for o in order[:n]}
    # identical unless a tie within rounding straddles the cut
    cut = C[order[n - 1]]
    diff = got ^ want
    sel = dict(zip(zip(i.tolist(), j.tolist()), C.tolist()))
    assert all(abs(sel[p] - cut) <= 1e-12 * cut for p in diff)
    nvox = sc.nx * sc.ny * sc.nz
    assert not any(a >= nvox and b >= nvox for a, b in got)


def test_threshold_keeps_the_couplings_above_c_min():
    sc = scenes.make_plain()
    i, j, C, _ = numpy_couplings(sc)
    c_min = float(np.quantile(C, 0.97))
    c_min *= 1.0 + 1e-9  # off any pair's value
    ap, ai = oracle.coupling_graph(sc, c_min=c_min)
    assert pairs_of(ap, ai) == {(int(a), int(b)) for a, b in zip(i[C > c_min], j[C > c_min])}
    # the adjacency is symmetric with ascending rows
    for r in range(len(ap) - 1):
        row = ai[ap[r]:ap[r + 1]]
        assert np.all(np.diff(row) > 0)
        for c in row:
            assert r in ai[ap[c]:ap[c + 1]]

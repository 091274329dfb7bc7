"""Degenerate inputs of the method on the device, against the FP64 oracle: a graph with
no couplings, a single voxel, a one-row slab, the smallest lattices (both phase-cell
definitions), no scattering at all, and a node of the largest accepted degree (64)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2503_16037_amd import scenes

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2503_16037_amd import sgrt
    c = sgrt.Context(0)
    yield c
    c.close()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return (np.abs(a - b) / np.maximum(np.abs(b), 1e-300)).max()


def check(ctx, sc, precision="fp32", bar=1e-4):
    from paper_2503_16037_amd import sgrt
    say("edge case", sc.name, precision)
    ref = oracle.run(sc)["radiance"]
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve(precision=precision)
    assert info["converged"] == 1, info
    err = rel(rad, ref)
    say("  max rel err", err)
    assert err < bar


def empty_graph(sc):
    return sc.with_(adj_ptr=np.zeros(sc.n_nodes + 1, np.int64), adj_idx=np.zeros(0, np.int32),
                    name=sc.name + "-no-edges")


@pytest.mark.parametrize("precision,bar", [("fp32", 1e-4), ("fp64", 1e-10)])
def test_graph_without_couplings(ctx, precision, bar):
    # single scattering of the sunlight and the directly lit surface only
    check(ctx, empty_graph(scenes.make_random_small(7, nx=4, ny=3, nz=3)), precision, bar)


@pytest.mark.parametrize("surface", [True, False])
def test_single_voxel(ctx, surface):
    check(ctx, scenes.make_random_small(8, nx=1, ny=1, nz=1, surface=surface))


def test_one_row_slab(ctx):
    check(ctx, scenes.make_random_small(9, nx=7, ny=1, nz=5, two_phase=True))


@pytest.mark.parametrize("n_fib,mode", [(2, 0), (4, 0), (2, 1), (4, 1), (7, 1)])
def test_smallest_lattices(ctx, n_fib, mode):
    check(ctx, scenes.make_plain().with_(n_fib=n_fib, sigma_mode=mode, name=f"plain-fib{n_fib}-mode{mode}"))


def test_one_point_lattice_is_refused(ctx):
    # its only point lies on the horizon: a surface node would own no cell
    from paper_2503_16037_amd import sgrt
    with pytest.raises(sgrt.SgError) as e:
        sgrt.Scene(ctx, scenes.make_plain().with_(n_fib=1))
    assert e.value.status == sgrt.SG_E_INVALID


def test_no_scattering(ctx):
    sc = scenes.make_plain()
    check(ctx, sc.with_(mu_s=np.zeros_like(sc.mu_s), name="plain-no-scattering"))


def degree_64_scene():
    sc = scenes.make_random_small(5, nx=6, ny=6, nz=5, R=2.3)
    deg = np.diff(sc.adj_ptr)
    hub = int(np.argmax(deg[:sc.nvox]))
    have = set(sc.adj_idx[sc.adj_ptr[hub]:sc.adj_ptr[hub + 1]].tolist()) | {hub}
    extra = [v for v in range(sc.nvox) if v not in have][:64 - int(deg[hub])]
    a = np.repeat(np.arange(sc.n_nodes), deg)
    b = sc.adj_idx.astype(np.int64)
    ap, ai = scenes.adjacency_from_pairs(sc.n_nodes, np.concatenate([a, [hub] * len(extra)]),
                                         np.concatenate([b, extra]))
    assert np.diff(ap).max() == 64
    return sc.with_(adj_ptr=ap, adj_idx=ai, name="rand-6x6x5-degree64")


def test_largest_degree(ctx):
    check(ctx, degree_64_scene())


def test_largest_degree_batched(ctx):
    from paper_2503_16037_amd import sgrt
    base = degree_64_scene()
    for nl in (5, 40):  # an 8-lane tile and the full-wavefront kernel
        sc = base.with_(abs_scale=np.geomspace(0.3, 3.0, nl).astype(np.float32))
        with sgrt.Scene(ctx, sc) as g:
            rad, info = g.solve()
        assert info["converged"] == 1
        for k in (0, nl - 1):
            err = rel(rad[k], oracle.run(sc, abs_scale=float(sc.abs_scale[k]))["radiance"])
            say("degree 64 batched", nl, k, err)
            assert err < 1e-4


def top_cluster(mu_s_dx, seed=0):
    """Four nodes of a 2 x 2 x 1 grid within 14 / 2^16 voxel of the midpoint of the top
    face's shared corner line, fully coupled, with the literal node weight mu_s * voxel edge:
    edges and sun paths are so short that K's spectral radius is about mu_s_dx / 2 and the
    source about mu_s_dx (the FP64 oracle solves it by GMRES)."""
    S = scenes.FX
    rng = np.random.default_rng(seed)
    sc = scenes.make_random_small(seed, nx=2, ny=2, nz=1, surface=False)
    pos = []
    for iy in range(2):
        for ix in range(2):
            p = np.array([S, S, S])
            p[:2] += np.array([ix * 2 - 1, iy * 2 - 1]) * rng.integers(2, 14, 2)
            p[2] -= rng.integers(2, 14)
            pos.append(p)
    a, b = np.triu_indices(4, 1)
    adj_ptr, adj_idx = scenes.adjacency_from_pairs(4, a, b)
    dx = sc.voxel_m
    return sc.with_(vol_pos_fx=np.array(pos, np.int32), adj_ptr=adj_ptr, adj_idx=adj_idx,
                    mu_s=np.full((1, 2, 2), mu_s_dx / dx, np.float32),
                    mu_a=np.full((1, 2, 2), 0.1 * mu_s_dx / dx, np.float32), node_weight_mode=1)


@pytest.mark.parametrize("n_lambda", [1, 3])
def test_overflowing_neumann_series_ends_finite_or_unconverged(ctx, n_lambda):
    """The literal node weight (mu_s times the voxel edge, 2000 here) on a tight cluster
    makes the FP32 Neumann iterate grow about 1000-fold per sweep, so it overflows inside one
    chunk of sweeps (inf - inf = NaN in the convergence measures).  The solve must not
    report convergence on such an iterate: GMRES restarted from zero (per wavelength when
    batched) ends it converged with finite radiances that match the oracle's GMRES solve."""
    from paper_2503_16037_amd import sgrt
    sc = top_cluster(2000.0)
    if n_lambda > 1:
        sc = sc.with_(abs_scale=np.array([0.5, 1.0, 2.0][:n_lambda], np.float32))
    say("overflowing Neumann series", sc.name, n_lambda)
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve(allow_noconv=True)
    assert info["status"] in (0, sgrt.SG_E_NOCONV), info
    if info["status"] == 0:
        assert info["converged"] == 1 and np.all(np.isfinite(rad)), info
        assert info["rel_residual"] <= 1e-6
    else:
        assert info["converged"] == 0 and not info["rel_residual"] <= 1e-6, info
    # GMRES from zero solves it, as the oracle does (each wavelength on its own when batched)
    assert info["status"] == 0 and info["gmres_used"] == 1
    rad = np.asarray(rad).reshape(n_lambda, sc.ny, sc.nx)
    for k in range(n_lambda):
        ora = oracle.run(sc, abs_scale=float(sc.abs_scale[k]) if n_lambda > 1 else 1.0)
        assert ora["solve"]["gmres"]
        scale = np.abs(ora["radiance"]).max()
        assert np.abs(rad[k] - ora["radiance"]).max() <= 1e-4 * scale, k

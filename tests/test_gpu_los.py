"""Scattering nodes on the lines of sight (Sec. 2: path points of the lines of sight, one per
layer of the medium or at constant distance intervals; Sec. 3, step 1) through the C ABI,
against the FP64 oracle.

  * Placement (sg_los_nodes): node positions, the lines' elements and their ends, bit for
    bit: layer and step modes, nadir and slant views, periodic axes, ragged grids, a step
    longer than every line, and the 64 x 64 x 32 plume's grid.
  * Scenes on these nodes (the gather splits each chord at the ends of the line's elements):
    every pixel within 1e-4 (FP32) and 1e-10 (FP64), the CSR structure exact, on a radius
    graph and on the graph that sg_graph_build ranks over the same nodes.
  * sg_graph_build over general nodes equals the oracle's graph (top-n, threshold, with and
    without surface nodes).
  * A multi-wavelength scene on line-of-sight nodes, per wavelength against the oracle.
  * Served: line-of-sight scenes through the server equal their solo solves bit for bit, and
    the admission estimate equals what the scene reserves.
"""
import dataclasses
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


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


PLACEMENTS = [
    # nx, ny, nz, view zenith, view azimuth, periodic, mode, step_m (voxel edge 100 m)
    (7, 6, 5, 0.0, 0.0, 0, "layer", 0.0),
    (7, 6, 5, 25.0, 120.0, 0, "layer", 0.0),
    (13, 9, 6, 40.0, 300.0, 0, "step", 37.0),
    (13, 9, 6, 35.0, 70.0, 3, "layer", 0.0),
    (13, 9, 6, 35.0, 70.0, 3, "step", 61.0),
    (11, 5, 7, 55.0, 200.0, 1, "step", 140.0),
    (5, 4, 3, 30.0, 10.0, 0, "step", 1e4),  # one element per line
    (1, 1, 9, 20.0, 45.0, 0, "layer", 0.0),
    (64, 64, 32, 30.0, 45.0, 0, "layer", 0.0),
    (64, 64, 32, 30.0, 45.0, 0, "step", 50.0),
]


@pytest.mark.parametrize("nx,ny,nz,vza,vaa,per,mode,step", PLACEMENTS)
def test_placement_bit_exact(ctx, nx, ny, nz, vza, vaa, per, mode, step):
    from paper_2503_16037_amd import sgrt
    D = scenes.direction_fx(vza, vaa)
    say("placement", nx, ny, nz, vza, vaa, per, mode, step)
    got = sgrt.los_nodes(ctx, nx, ny, nz, D, 100.0, mode=mode, step_m=step, periodic=per)
    want = oracle.los_nodes(nx, ny, nz, D, 100.0, mode, step_m=step, periodic=per)
    assert np.array_equal(got[0].astype(np.int64), want[0])
    for k in (1, 2, 3):
        assert np.array_equal(got[k], want[k]), k
    assert len(got[0]) > 0


def test_placement_rejects_invalid_descriptions(ctx):
    from paper_2503_16037_amd import sgrt
    D = scenes.direction_fx(20.0, 10.0)
    for kw in (dict(view_dir=(1, 0, 0)), dict(mode="step", step_m=0.0), dict(mode="step", step_m=-3.0),
               dict(periodic=4), dict(voxel_m=0.0)):
        a = dict(view_dir=D, voxel_m=100.0)
        a.update(kw)
        with pytest.raises(sgrt.SgError):
            sgrt.los_nodes(ctx, 4, 4, 3, **a)


def los_scene(seed, nx, ny, nz, mode, step_m=0.0, vza=30.0, vaa=200.0, periodic=0, **kw):
    sc = scenes.make_random_small(seed, nx=nx, ny=ny, nz=nz, vza=vza, vaa=vaa, kscale=2.0, **kw)
    sc = dataclasses.replace(sc, periodic=periodic)
    pos, lp, ln, lt = oracle.los_nodes(sc.nx, sc.ny, sc.nz, sc.view_dir, sc.voxel_m, mode, step_m=step_m,
                                       periodic=periodic)
    return scenes.with_los_nodes(sc, pos, lp, ln, lt, radius_vox=1.8, name=f"{sc.name}-{mode}")


LOS_SCENES = [
    (0, 6, 5, 4, "layer", 0.0, {}),
    (1, 6, 5, 4, "step", 45.0, dict(two_phase=True)),
    (2, 7, 6, 5, "step", 80.0, dict(surface=False)),
    (3, 7, 6, 5, "layer", 0.0, dict(two_phase=True)),
]


@pytest.mark.parametrize("seed,nx,ny,nz,mode,step,kw", LOS_SCENES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_los_scene_matches_oracle(ctx, seed, nx, ny, nz, mode, step, kw, precision):
    from paper_2503_16037_amd import sgrt
    sc = los_scene(seed, nx, ny, nz, mode, step, **kw)
    say("los scene", sc.name, precision, sc.n_vol, "nodes", sc.n_edges, "edges")
    ora = oracle.run(sc, want_matrix=True)
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve(precision=precision)
        assert info["converged"] == 1
        rp, col, _ = g.export_csr(values=False)
        assert np.array_equal(rp, ora["row_ptr"]) and np.array_equal(col, ora["col"])
        err = rel_err(rad, ora["radiance"])
        say("  max pixel rel err", err.max())
        assert err.max() < (1e-10 if precision == "fp64" else 1e-4)
        S = g.export_vector("source")
        m = ora["S"] > (1e-300 if precision == "fp64" else 1e-30)
        assert rel_err(S[m], ora["S"][m]).max() < (1e-12 if precision == "fp64" else 2e-5)


def test_periodic_los_scene_matches_oracle(ctx):
    from paper_2503_16037_amd import sgrt
    # odd periods: nodes of pixels half a period apart would otherwise be exactly half a
    # period apart, with no unique shortest image
    sc0 = scenes.make_random_small(6, nx=7, ny=5, nz=4, vza=35.0, vaa=70.0, kscale=2.0)
    sc0 = dataclasses.replace(sc0, periodic=3)
    pos, lp, ln, lt = oracle.los_nodes(sc0.nx, sc0.ny, sc0.nz, sc0.view_dir, sc0.voxel_m, "step", step_m=55.0,
                                       periodic=3)
    # no radius graph for wrapped nodes here: couple them with the ranked graph
    sc = scenes.with_los_nodes(sc0, pos, lp, ln, lt, name="periodic-los")
    ap, ai = oracle.coupling_graph(sc, n_pairs=5 * len(pos))
    sc = dataclasses.replace(sc, adj_ptr=ap, adj_idx=ai)
    say("periodic los scene", sc.n_vol, "nodes", sc.n_edges, "edges")
    ora = oracle.run(sc)
    with sgrt.Scene(ctx, sc) as g:
        for precision, bar in (("fp64", 1e-10), ("fp32", 1e-4)):
            rad, info = g.solve(precision=precision)
            assert info["converged"] == 1
            assert rel_err(rad, ora["radiance"]).max() < bar, precision


def test_single_scatter_los_scene(ctx):
    from paper_2503_16037_amd import sgrt
    sc = los_scene(4, 6, 6, 4, "step", 70.0)
    ora = oracle.run(sc, scatter_order=1)
    with sgrt.Scene(ctx, sc) as g:
        rad, _ = g.solve(precision="fp64", scatter_order=1)
    assert rel_err(rad, ora["radiance"]).max() < 1e-12


@pytest.mark.parametrize("surface", [True, False])
@pytest.mark.parametrize("mode", ["layer", "step"])
def test_graph_build_over_los_nodes(ctx, surface, mode):
    from paper_2503_16037_amd import sgrt
    sc = los_scene(8, 6, 5, 4, mode, 70.0, surface=surface)
    n = len(sc.node_pos_fx)
    # a threshold inside the couplings' range: the median C of the volume pairs
    _, mu, q = oracle.coupling_nodes(sc)
    i, j = np.triu_indices(n, 1)
    c = np.sqrt(mu[i] * mu[j]) / np.linalg.norm(q[i] - q[j], axis=1)
    c_mid = float(np.median(c[c > 0]))
    for kw in (dict(n_pairs=1), dict(n_pairs=4 * n), dict(n_pairs=10 ** 7), dict(c_min=0.0), dict(c_min=c_mid)):
        say("general graph", sc.name, surface, kw)
        got = sgrt.graph_build(ctx, sc, **kw)
        want = oracle.coupling_graph(sc, **kw)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), kw


def test_scene_on_a_ranked_graph_of_los_nodes(ctx):
    from paper_2503_16037_amd import sgrt
    sc = los_scene(9, 8, 7, 5, "step", 60.0, two_phase=True)
    n = len(sc.node_pos_fx)
    ap, ai = sgrt.graph_build(ctx, sc, n_pairs=6 * n)
    oap, oai = oracle.coupling_graph(sc, n_pairs=6 * n)
    assert np.array_equal(ap, oap) and np.array_equal(ai, oai)
    sc = dataclasses.replace(sc, adj_ptr=ap, adj_idx=ai)
    ora = oracle.run(sc)
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve(precision="fp32")
    assert info["converged"] == 1
    assert rel_err(rad, ora["radiance"]).max() < 1e-4


def test_batched_los_scene_per_wavelength(ctx):
    from paper_2503_16037_amd import sgrt
    sc0 = scenes.make_batched(nx=10, ny=9, nz=6, n_lambda=7)
    pos, lp, ln, lt = oracle.los_nodes(sc0.nx, sc0.ny, sc0.nz, sc0.view_dir, sc0.voxel_m, "step", step_m=40.0)
    sc = scenes.with_los_nodes(sc0, pos, lp, ln, lt, radius_vox=1.8)
    say("batched los", sc.name, sc.n_vol, "nodes", sc.n_lambda, "wavelengths")
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve()
        assert info["converged"] == 1
    for k in sorted({0, sc.n_lambda - 1, int(np.argmax(sc.abs_scale))}):
        ora = oracle.run(sc, abs_scale=float(sc.abs_scale[k]))
        err = rel_err(rad[k], ora["radiance"])
        say("  lambda", k, "max rel err", err.max())
        assert err.max() < 1e-4


def test_served_los_scenes_equal_solo_solves(ctx):
    from paper_2503_16037_amd import sgrt
    stream = [los_scene(10, 6, 5, 4, "layer"), los_scene(11, 7, 6, 4, "step", 50.0),
              scenes.make_random_small(12, nx=5, ny=5, nz=4, kscale=2.0)]
    solo = []
    for sc in stream:
        with sgrt.Scene(ctx, sc) as g:
            r, _ = g.solve()
            solo.append(np.asarray(r).reshape(sc.n_lambda, sc.ny, sc.nx))
    srv = sgrt.Server(ctx, max_resident=2, queue_cap=8, n_streams=2)
    try:
        for sc in stream[:2]:
            with sgrt.Scene(ctx, sc) as g:
                assert srv.reservation(sc) == g.sizes["device_bytes"], sc.name
        tickets = [srv.submit(sc) for sc in stream]
        out = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for sc, (rad, info), ref in zip(stream, out, solo):
        assert info["status"] == 0 and info["converged"] == 1, sc.name
        assert np.array_equal(rad, ref), sc.name


def test_invalid_los_scenes_are_rejected(ctx):
    from paper_2503_16037_amd import sgrt
    sc = los_scene(13, 5, 4, 3, "layer")
    W = sc.nx * scenes.FX
    bad = []
    p = sc.node_pos_fx.copy()
    p[0, 0] = W
    bad.append(("outside the box", dataclasses.replace(sc, node_pos_fx=p)))
    p = sc.node_pos_fx.copy()
    p[0, 2] = 0
    bad.append(("on the ground", dataclasses.replace(sc, node_pos_fx=p)))
    ln = sc.los_node.copy()
    ln[0] = len(sc.node_pos_fx)
    bad.append(("no such node", dataclasses.replace(sc, los_node=ln)))
    # two equal ends inside one line (the ends restart from 0 at every pixel)
    e = int(sc.los_ptr[np.flatnonzero(np.diff(sc.los_ptr) >= 2)[0]])
    lt = sc.los_t.copy()
    lt[e + 1] = lt[e]
    bad.append(("ends not increasing", dataclasses.replace(sc, los_t=lt)))
    with sgrt.Scene(ctx, sc):
        pass
    for what, b in bad:
        say("invalid los scene:", what)
        with pytest.raises(sgrt.SgError):
            with sgrt.Scene(ctx, b):
                pass


@pytest.mark.parametrize("sigma_mode", [0, 1])
def test_high_degree_los_nodes_fp64(ctx, sigma_mode):
    """Line-of-sight nodes on their ranked graph (Eq. 4, 12 couplings per node: degrees up to
    250, above 64 on 25 nodes): the high-degree kernels on general nodes, both phase-cell
    rules, every pixel within 1e-10 of the oracle in FP64."""
    from paper_2503_16037_amd import sgrt
    sc0 = scenes.make_random_small(2, nx=10, ny=9, nz=6, vza=30.0, vaa=200.0, kscale=2.0)
    pos, lp, ln, lt = oracle.los_nodes(sc0.nx, sc0.ny, sc0.nz, sc0.view_dir, sc0.voxel_m, "layer")
    sc = scenes.with_los_nodes(sc0, pos, lp, ln, lt, name="los-ranked")
    ap, ai = oracle.coupling_graph(sc, n_pairs=12 * len(pos))
    sc = dataclasses.replace(sc, adj_ptr=ap, adj_idx=ai, sigma_mode=sigma_mode)
    assert np.diff(ap).max() > 64
    say("high-degree los", sc.n_vol, "nodes, max degree", int(np.diff(ap).max()), "sigma", sigma_mode)
    ora = oracle.run(sc)
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve(precision="fp64")
    assert info["converged"] == 1
    assert rel_err(rad, ora["radiance"]).max() < 1e-10

"""The FP32 screen of the phase-cell ownership argmax (Eq. 7) changes no owner.

The regular phase-cell kernel certifies most owners with an FP32 screen whose error bound
is proven in its source, and takes every other decision with the FP64 operation sequence;
SG_EXACT_CELLS takes all of them with the FP64 sequence.  Both must give the same owners,
hence the same matrix values, sources and radiances bit for bit.  The scenes cover jittered
grids (few near-ties), nodes at the voxel centres (exact ties everywhere: the fallback
decides them), two phase components, surfaces, a periodic slab, line-of-sight nodes, nodes of
degree above 64 (the chunked screen of the high-degree kernel), both precisions and a batch of
wavelengths (the Q-only build).
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


def centred_cloud():
    """A small cloud with every node at its voxel centre (symmetric stencils: exact ties)."""
    sc = scenes.make_cloud(nx=16, ny=14, nz=8)
    pos = scenes.jittered_positions(np.random.default_rng(0), sc.nx, sc.ny, sc.nz, jitter=0.0)
    ap, ai = scenes.radius_graph(pos, sc.nx, sc.ny, sc.nz, 1.8)
    return dataclasses.replace(sc, vol_pos_fx=pos, adj_ptr=ap, adj_idx=ai, name="cloud-centred")


def los():
    sc = scenes.make_random_small(1, nx=6, ny=5, nz=4, vza=30.0, vaa=200.0, kscale=2.0, two_phase=True)
    pos, lp, ln, lt = oracle.los_nodes(sc.nx, sc.ny, sc.nz, sc.view_dir, sc.voxel_m, "step", step_m=45.0)
    return scenes.with_los_nodes(sc, pos, lp, ln, lt, radius_vox=1.8, name="los-step")


def coupled():
    """Strongest couplings (Eq. 4), 20 per voxel: nodes of degree above 64 (the high-degree
    kernel, with its chunked screen and second pass)."""
    sc = scenes.make_random_small(4, nx=8, ny=8, nz=6, kscale=2.0)
    ap, ai = oracle.coupling_graph(sc, n_pairs=20 * sc.nvox)
    assert np.diff(ap).max() > 64
    return dataclasses.replace(sc, adj_ptr=ap, adj_idx=ai, name="coupled-20")


def star():
    """One node coupled to 2000 others on a 17x16x16 grid: 32 chunks of out-edge directions."""
    sc = scenes.make_random_small(8, nx=17, ny=16, nz=16, kscale=0.5)
    c = sc.nvox // 2
    leaves = [v for v in range(sc.nvox) if v != c][:2000]
    rows = [[] for _ in range(sc.n_nodes)]
    rows[c] = leaves
    for v in leaves:
        rows[v] = [c]
    ap = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    ai = np.concatenate([np.asarray(r, np.int32) for r in rows if r]).astype(np.int32)
    return dataclasses.replace(sc, adj_ptr=ap, adj_idx=ai, name="star-2000")


SCENES = {
    "plume": lambda: scenes.make_plume(nx=32, ny=32, nz=16),
    "cloud": lambda: scenes.make_cloud(nx=32, ny=32, nz=12),
    "cloud-centred": centred_cloud,
    "slab-centred": lambda: scenes.make_slab(),
    "random-two-phase": lambda: scenes.make_random_small(5, nx=5, ny=4, nz=4, two_phase=True),
    "los": los,
    "coupled-20": coupled,
    "star-2000": star,
}


def _outputs(g, nl, **opts):
    rad, _ = g.solve(**opts)
    vals = [g.export_csr(lam=k, cols=False)[2] for k in range(nl)]
    return rad, vals, g.export_vector("source"), g.export_vector("qsun")


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name", list(SCENES))
def test_screen_gives_the_fp64_owners(ctx, name, precision):
    from paper_2503_16037_amd import sgrt
    sc = SCENES[name]()
    say("screen vs FP64 scan", name, precision, sc.nx, sc.ny, sc.nz)
    with sgrt.Scene(ctx, sc) as g:
        a = _outputs(g, 1, precision=precision)
        b = _outputs(g, 1, precision=precision, screen=False)
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1][0], b[1][0])
    assert np.array_equal(a[2], b[2])
    assert np.array_equal(a[3], b[3])


def test_screen_in_a_wavelength_batch(ctx):
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_plume(nx=24, ny=24, nz=12, n_lambda=5)
    say("screen vs FP64 scan, batch of", sc.abs_scale.shape[0], "wavelengths")
    with sgrt.Scene(ctx, sc) as g:
        a = _outputs(g, 5)
        b = _outputs(g, 5, screen=False)
    assert np.array_equal(a[0], b[0])
    for k in range(5):
        assert np.array_equal(a[1][k], b[1][k])
    assert np.array_equal(a[2], b[2])
    assert np.array_equal(a[3], b[3])

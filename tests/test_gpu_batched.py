"""Batched wavelengths (one graph, one set of phase cells, many absorption multipliers).

Every wavelength must match the FP64 oracle run with mu_a scaled by its multiplier
(1e-4 relative per pixel) and the same wavelength solved alone through the
single-wavelength path.  Wavelength counts cover every lane-tile shape of the SpMM
(several nodes per wavefront, one node per wavefront, more than 64 wavelengths).
"""
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
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(np.asarray(b)), 1e-300)


@pytest.mark.parametrize("n_lambda", [3, 17, 64, 70])
def test_batched_matches_oracle_per_wavelength(ctx, n_lambda):
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_batched(nx=14, ny=12, nz=8, n_lambda=n_lambda)
    say("batched scene", sc.name)
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve(timing=True)
        assert rad.shape == (n_lambda, sc.ny, sc.nx)
        assert info["converged"] == 1
        lams = sorted(set([0, n_lambda - 1, int(np.argmin(sc.abs_scale)), int(np.argmax(sc.abs_scale))]))
        for k in lams:
            ora = oracle.run(sc, abs_scale=float(sc.abs_scale[k]))
            err = rel_err(rad[k], ora["radiance"])
            say("  lambda", k, "scale", float(sc.abs_scale[k]), "max rel err", err.max())
            assert err.max() < 1e-4
        phi = g.export_vector("phi")
        S = g.export_vector("source")
        ora = oracle.run(sc, abs_scale=float(sc.abs_scale[lams[-1]]))
        k = lams[-1]
        m = ora["S"] > 1e-30
        assert rel_err(S[k][m], ora["S"][m]).max() < 3e-5
        assert np.abs(phi[k] - ora["phi"]).max() < 1e-5 * ora["phi"].max()
        _, _, val = g.export_csr(lam=k, cols=False)
        big = ora["val"] > 1e-9 * ora["val"].max()
        assert rel_err(val[big], ora["val"][big]).max() < 5e-5


def test_batched_equals_single_wavelength_solves(ctx):
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_batched(nx=16, ny=16, nz=8, n_lambda=6)
    say("batched vs single", sc.name)
    with sgrt.Scene(ctx, sc) as g:
        rad, _ = g.solve()
    for k in range(sc.n_lambda):
        one = sc.with_(abs_scale=sc.abs_scale[k:k + 1].copy())
        with sgrt.Scene(ctx, one) as g1:
            r1, _ = g1.solve()
        assert rel_err(rad[k], r1).max() < 2e-5


def test_batched_single_scatter(ctx):
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_batched(nx=10, ny=10, nz=6, n_lambda=5)
    say("batched single scatter", sc.name)
    with sgrt.Scene(ctx, sc) as g:
        rad, _ = g.solve(scatter_order=1)
    for k in (0, 4):
        ora = oracle.run(sc, abs_scale=float(sc.abs_scale[k]), scatter_order=1)
        assert rel_err(rad[k], ora["radiance"]).max() < 1e-4


def test_batched_full_size_sampled_wavelengths(ctx):
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_batched()
    say("batched full size", sc.name, sc.n_edges, sc.nnz())
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve(timing=True)
        say("  info", info)
        assert info["converged"] == 1
    for k in (int(np.argmin(sc.abs_scale)), int(np.argmax(sc.abs_scale)), 17):
        ora = oracle.run(sc, abs_scale=float(sc.abs_scale[k]), want_matrix=False)
        err = rel_err(rad[k], ora["radiance"])
        say("  lambda", k, "max / p99 rel err", err.max(), np.percentile(err, 99))
        assert err.max() < 1e-4


def test_batched_deep_shadow_pixels(ctx):
    """Every wavelength of a thick cloud at a 70 deg sun (pixels down to 1e-7 of the
    median) meets the per-pixel bar."""
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_served(3, max_voxels=6000)
    say("batched deep shadow", sc.name)
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve()
    assert info["converged"] == 1
    for k in range(sc.n_lambda):
        o = oracle.run(sc, abs_scale=float(sc.abs_scale[k]))["radiance"]
        assert rel_err(rad[k], o).max() <= 1e-4, k


@pytest.mark.parametrize("n_lambda", [3, 12, 22])
def test_lambda_tiles_give_identical_bits(ctx, n_lambda):
    """Every wavelength tile that holds the wavelengths (several nodes per wavefront
    down to one) computes the same bits: same sweeps, same radiance."""
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_batched(nx=15, ny=13, nz=9, n_lambda=n_lambda, seed=11)
    tiles = [t for t in (8, 16, 32, 64) if t >= n_lambda]
    with sgrt.Scene(ctx, sc) as g:
        runs = {}
        for t in tiles:
            say("tile", t, "scene", sc.name)
            runs[t] = g.solve(lambda_tile=t)
        auto = g.solve()
    rad64, info64 = runs[64]
    assert info64["converged"] == 1
    for t in tiles + ["auto"]:
        rad, info = auto if t == "auto" else runs[t]
        assert info["sweeps"] == info64["sweeps"], t
        assert np.array_equal(rad, rad64), t
    ora = oracle.run(sc, abs_scale=float(sc.abs_scale[n_lambda - 1]))
    assert rel_err(rad64[n_lambda - 1], ora["radiance"]).max() < 1e-4


def test_lambda_tile_rejected_when_invalid(ctx):
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_batched(nx=8, ny=8, nz=6, n_lambda=12)
    with sgrt.Scene(ctx, sc) as g:
        for bad in (8, 7, 128):
            with pytest.raises(sgrt.SgError) as e:
                g.solve(lambda_tile=bad)
            assert e.value.status == sgrt.SG_E_INVALID
        rad, info = g.solve(lambda_tile=16)
        assert info["converged"] == 1


def test_batched_gmres_forced(ctx):
    """solver = GMRES on a batched scene: every wavelength by its own FP64 GMRES with the
    batched matrix at that wavelength, from zero; each against the oracle and against the
    batched Neumann solve."""
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_batched(nx=10, ny=9, nz=6, n_lambda=5)
    say("batched forced GMRES", sc.name)
    with sgrt.Scene(ctx, sc) as g:
        rad_n, _ = g.solve()
        rad, info = g.solve(solver="gmres", gmres_restart=16)
    assert info["converged"] == 1 and info["gmres_used"] == 1
    assert info["rel_residual"] <= 1e-6
    assert rel_err(rad, rad_n).max() < 2e-5
    for k in range(sc.n_lambda):
        ora = oracle.run(sc, abs_scale=float(sc.abs_scale[k]))
        assert rel_err(rad[k], ora["radiance"]).max() < 1e-4, k


def test_batched_gmres_fallback_on_divergent_series(ctx):
    """The literal node weight on a tight cluster makes the batched Neumann series diverge at
    every wavelength; the solve falls back to GMRES per wavelength and matches the oracle
    (which solves the same systems by GMRES)."""
    from paper_2503_16037_amd import sgrt
    from test_oracle_matrix_solve import clustered_scene
    sc = clustered_scene()
    sc = sc.with_(abs_scale=np.array([0.3, 1.0, 3.0, 10.0], np.float32))
    say("batched GMRES fallback", sc.name)
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve()
    assert info["converged"] == 1 and info["gmres_used"] == 1
    for k in range(sc.n_lambda):
        ora = oracle.run(sc, abs_scale=float(sc.abs_scale[k]))
        assert ora["solve"]["gmres"]
        scale = np.abs(ora["radiance"]).max()
        assert np.abs(rad[k] - ora["radiance"]).max() <= 1e-4 * scale, k

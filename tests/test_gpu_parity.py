"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: voxel traversals and CSR structure bit-exact; FP64 mode within 1e-10
relative per pixel; FP32 mode within 1e-4 relative per pixel (the bar of the
FP32 path), intermediate arrays within tolerances derived in the design
notes from FP32 rounding.
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


def _scene(ctx, sc):
    from paper_2503_16037_amd import sgrt
    return sgrt.Scene(ctx, sc)


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def check_csr_structure(g, ora):
    rp, col, _ = g.export_csr(values=False)
    assert np.array_equal(rp, ora["row_ptr"])
    assert np.array_equal(col, ora["col"])


def test_traversals_bit_exact(ctx):
    for sc in (scenes.make_plain(), scenes.make_random_small(3, nx=5, ny=4, nz=3, sza=63.0, saa=200.0, vza=41.0,
                                                             vaa=300.0)):
        say("traversal case", sc.name)
        with _scene(ctx, sc) as g:
            pos = oracle.node_positions(sc)
            tails = oracle.tails(sc.adj_ptr)
            heads = sc.adj_idx.astype(np.int64)
            E = sc.n_edges
            ids = np.arange(E) if E <= 20000 else np.random.default_rng(0).choice(E, 20000, replace=False)
            vox, dt, cnt = g.trace("edge", ids, cap=64)
            for k, e in enumerate(ids):
                a, b = min(tails[e], heads[e]), max(tails[e], heads[e])
                v2, d2 = oracle.trace(sc.nx, sc.ny, sc.nz, pos[a], pos[b] - pos[a], 0)
                assert cnt[k] == len(v2)
                assert np.array_equal(vox[k, :cnt[k]], v2)
                assert np.array_equal(dt[k, :cnt[k]], d2)
            ids = np.arange(sc.n_nodes)
            vox, dt, cnt = g.trace("sun", ids, cap=256)
            for l in ids:
                v2, d2 = oracle.trace(sc.nx, sc.ny, sc.nz, pos[l], sc.sun_dir, 1)
                assert np.array_equal(vox[l, :cnt[l]], v2) and np.array_equal(dt[l, :cnt[l]], d2)
            ids = np.arange(sc.nx * sc.ny)
            vox, dt, cnt = g.trace("view", ids, cap=256)
            for p in ids:
                P = np.array([(p % sc.nx) * 65536 + 32768, (p // sc.nx) * 65536 + 32768, 0])
                v2, d2 = oracle.trace(sc.nx, sc.ny, sc.nz, P, sc.view_dir, 1)
                assert np.array_equal(vox[p, :cnt[p]], v2) and np.array_equal(dt[p, :cnt[p]], d2)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_plain_config(ctx, precision):
    sc = scenes.make_plain()
    say("plain config", precision)
    ora = oracle.run(sc)
    with _scene(ctx, sc) as g:
        rad, info = g.solve(precision=precision, timing=True)
        assert info["converged"] == 1
        check_csr_structure(g, ora)
        tau = g.export_vector("tau_s") + g.export_vector("tau_a")
        _, _, val = g.export_csr(cols=False)
        S = g.export_vector("source")
        phi = g.export_vector("phi")
        if precision == "fp64":
            assert rel_err(tau, ora["tau"]).max() < 1e-13
            assert rel_err(val, ora["val"]).max() < 1e-12
            assert rel_err(S[ora["S"] > 0], ora["S"][ora["S"] > 0]).max() < 1e-12
            assert rel_err(phi, ora["phi"]).max() < 1e-10
            assert rel_err(rad, ora["radiance"]).max() < 1e-10
        else:
            assert rel_err(tau, ora["tau"]).max() < 1e-5
            big = ora["val"] > 1e-12 * ora["val"].max()
            assert rel_err(val[big], ora["val"][big]).max() < 5e-5
            # phi: relative to its largest element (the solve's stopping rule is a norm-wise
            # residual); elements above 1e-3 of the maximum also element-wise
            assert np.abs(phi - ora["phi"]).max() < 1e-5 * ora["phi"].max()
            hi = ora["phi"] > 1e-3 * ora["phi"].max()
            assert rel_err(phi[hi], ora["phi"][hi]).max() < 1e-4
            assert rel_err(rad, ora["radiance"]).max() < 1e-4
        say("  max pixel rel err", rel_err(rad, ora["radiance"]).max(), info["sweeps"], info["ms_total"])


@pytest.mark.parametrize("seed,two_phase,surface", [(0, False, True), (1, True, True), (2, True, False),
                                                    (5, False, True)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_small_random_scenes(ctx, seed, two_phase, surface, precision):
    # lognormal extinction with a median optical depth of ~1.3 per voxel (tail ~10)
    sc = scenes.make_random_small(seed, nx=5, ny=4, nz=4, two_phase=two_phase, surface=surface, kscale=2.0)
    say("random scene", sc.name, precision)
    ora = oracle.run(sc)
    with _scene(ctx, sc) as g:
        rad, info = g.solve(precision=precision)
        check_csr_structure(g, ora)
        tol = 1e-10 if precision == "fp64" else 1e-4
        assert rel_err(rad, ora["radiance"]).max() < tol
        qsun = g.export_vector("qsun")
        # the sun's cell weights are S / (T_sun rho) (x mu0 on the surface); compare through S
        S = g.export_vector("source")
        # FP32 holds values down to ~1e-38 (normal range); compare above that floor
        m = ora["S"] > (1e-300 if precision == "fp64" else 1e-30)
        assert rel_err(S[m], ora["S"][m]).max() < (1e-12 if precision == "fp64" else 2e-5)
        assert np.all(qsun >= 0) and np.all(qsun <= 1.0 + 1e-6)


def test_thick_stress_scene(ctx):
    """Optical depth ~20 per voxel: most pixels are dark (down to 1e-50), far below what the
    global residual target resolves.  Bright pixels (within 1e-6 of the brightest) must still
    meet the per-pixel bar; every pixel must meet it up to 10 x rtol of the image maximum."""
    sc = scenes.make_random_small(0, nx=5, ny=4, nz=4, kscale=30.0)
    say("thick stress scene", sc.name)
    ora = oracle.run(sc)
    o = ora["radiance"]
    with _scene(ctx, sc) as g:
        for precision, rtol in (("fp64", 1e-12), ("fp32", 1e-6)):
            rad, _ = g.solve(precision=precision)
            bright = o > 1e-6 * o.max()
            assert rel_err(rad[bright], o[bright]).max() < (1e-10 if precision == "fp64" else 1e-4)
            assert np.all(np.abs(rad - o) <= 1e-4 * o + 10 * rtol * o.max())


def test_single_scatter_mode(ctx):
    sc = scenes.make_random_small(4, nx=6, ny=5, nz=4, two_phase=True, kscale=2.0)
    say("single scatter", sc.name)
    ora = oracle.run(sc, scatter_order=1)
    with _scene(ctx, sc) as g:
        rad, _ = g.solve(precision="fp64", scatter_order=1)
        assert rel_err(rad, ora["radiance"]).max() < 1e-10
        rad32, _ = g.solve(scatter_order=1)
        assert rel_err(rad32, ora["radiance"]).max() < 1e-4


def test_gmres_forced_and_fallback(ctx):
    sc = scenes.make_plain()
    say("gmres forced on plain config")
    ora = oracle.run(sc)
    with _scene(ctx, sc) as g:
        rad, info = g.solve(precision="fp64", solver="gmres")
        assert info["gmres_used"] == 1 and info["converged"] == 1
        assert rel_err(rad, ora["radiance"]).max() < 1e-9
        rad, info = g.solve(precision="fp32", solver="gmres")
        assert rel_err(rad, ora["radiance"]).max() < 1e-4
    # divergent Neumann series (literal node weight on clustered nodes): automatic fallback
    from test_oracle_matrix_solve import clustered_scene
    sc = clustered_scene()
    say("gmres fallback on clustered scene")
    ora = oracle.run(sc)
    assert ora["solve"]["gmres"]
    with _scene(ctx, sc) as g:
        rad, info = g.solve(precision="fp64")
        assert info["gmres_used"] == 1 and info["converged"] == 1
        assert rel_err(rad, ora["radiance"]).max() < 1e-8


def test_nonconvergence_is_reported(ctx):
    sc = scenes.make_plain()
    say("non-convergence report")
    from paper_2503_16037_amd import sgrt
    with _scene(ctx, sc) as g:
        rad, info = g.solve(precision="fp64", max_sweeps=2, allow_noconv=True)
        assert info["status"] == sgrt.SG_E_NOCONV and info["converged"] == 0
        assert np.all(np.isfinite(rad))
        with pytest.raises(sgrt.SgError):
            g.solve(precision="fp64", max_sweeps=2)


def test_run_to_run_determinism(ctx):
    sc = scenes.make_plume(nx=24, ny=24, nz=12)
    say("determinism", sc.name)
    with _scene(ctx, sc) as g:
        a, _ = g.solve()
        b, _ = g.solve()
        assert np.array_equal(a, b)
        va = g.export_csr(cols=False)[2]
        g.solve()
        vb = g.export_csr(cols=False)[2]
        assert np.array_equal(va, vb)


def test_device_output_and_stream(ctx):
    import torch
    sc = scenes.make_plain()
    say("device output")
    with _scene(ctx, sc) as g:
        host, _ = g.solve()
        out = torch.zeros(sc.ny * sc.nx, dtype=torch.float64, device="cuda:0")
        s = torch.cuda.Stream(device=0)
        with torch.cuda.stream(s):
            g.solve(out=out, stream=s)
        s.synchronize()
        assert np.array_equal(out.cpu().numpy().reshape(sc.ny, sc.nx), host)


def test_plume_full_size(ctx):
    sc = scenes.make_plume()
    say("plume full size", sc.name, sc.n_edges, sc.nnz())
    ora = oracle.run(sc, want_matrix=True)
    say("  oracle done", ora["solve"])
    with _scene(ctx, sc) as g:
        rad, info = g.solve(timing=True)
        say("  gpu info", info)
        assert info["converged"] == 1
        err = rel_err(rad, ora["radiance"])
        say("  max / p99 pixel rel err", err.max(), np.percentile(err, 99))
        assert err.max() < 1e-4
        rp, col, val = g.export_csr()
        assert np.array_equal(rp, ora["row_ptr"])
        assert np.array_equal(col, ora["col"])
        big = ora["val"] > 1e-9 * ora["val"].max()
        assert rel_err(val[big], ora["val"][big]).max() < 5e-5
        tau = g.export_vector("tau_s") + g.export_vector("tau_a")
        assert rel_err(tau, ora["tau"]).max() < 1e-5


def test_cloud_full_size(ctx):
    """The 128 x 128 x 48 cloud (18.3 M couplings, 424 M nonzeros; single-scattering
    albedo 0.999, sun at 70 deg): every pixel against the oracle, the structure (row
    pointers and column indices) bit-exact, the K values, and the transmittances of all
    edges."""
    sc = scenes.make_cloud()
    say("cloud full size", sc.name, sc.n_edges)
    ora = oracle.run(sc, want_matrix=True)
    say("  oracle done", ora["solve"])
    with _scene(ctx, sc) as g:
        rad, info = g.solve(timing=True)
        say("  gpu info", info)
        assert info["converged"] == 1
        err = rel_err(rad, ora["radiance"])
        say("  max / p99 pixel rel err", err.max(), np.percentile(err, 99))
        assert err.max() < 1e-4
        rp, col, val = g.export_csr()
        assert np.array_equal(rp, ora["row_ptr"])
        assert np.array_equal(col, ora["col"])
        big = ora["val"] > 1e-9 * ora["val"].max()
        assert rel_err(val[big], ora["val"][big]).max() < 5e-5
        del col, val
        tau = g.export_vector("tau_s") + g.export_vector("tau_a")
        assert rel_err(tau, ora["tau"]).max() < 1e-5


@pytest.mark.parametrize("precision,bar", [("fp32", 1e-4), ("fp64", 1e-10)])
def test_deep_shadow_pixels(ctx, precision, bar):
    """A thick conservative-scattering cloud at a 70 deg sun: some pixels carry 1e-7 of
    the median radiance and get their light through many scattering orders.  Every
    pixel must meet the bar, so the solve must converge edge by edge, not in norm."""
    import dataclasses
    sc0 = scenes.make_served(3, max_voxels=6000)
    sc = dataclasses.replace(sc0, abs_scale=np.array([sc0.abs_scale[0]], np.float32))
    say("deep shadow", sc.name, precision)
    ora = oracle.run(sc, abs_scale=float(sc.abs_scale[0]))
    o = ora["radiance"]
    assert o.min() / np.median(o) < 1e-5
    with _scene(ctx, sc) as g:
        rad, info = g.solve(precision=precision)
    assert info["converged"] == 1 and info["gmres_used"] == 0
    assert rel_err(rad, o).max() <= bar

"""The paper's colouring of Sigma (nearest lattice point + flood fill over the convex
hull, Sec. 3; sigma_mode = 1) on the device against the FP64 oracle."""
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
    return (np.abs(np.asarray(a) - np.asarray(b)) / np.abs(np.asarray(b))).max()


@pytest.mark.parametrize("surface", [True, False])
def test_colouring_matches_oracle(ctx, surface):
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_plain().with_(sigma_mode=1)
    if not surface:
        sc = scenes.make_random_small(3, nx=7, ny=6, nz=5, two_phase=True, surface=False).with_(sigma_mode=1)
    ora = oracle.run(sc)
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve()
        assert info["converged"] == 1
        _, _, val = g.export_csr(lam=0, cols=False)
    big = ora["val"] > 1e-9 * ora["val"].max()
    say(sc.name, "radiance", rel(rad, ora["radiance"]), "K", rel(val[big], ora["val"][big]))
    assert rel(rad, ora["radiance"]) < 1e-4
    assert rel(val[big], ora["val"][big]) < 5e-5


def test_colouring_fp64(ctx):
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_plain().with_(sigma_mode=1)
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve(precision="fp64")
    assert rel(rad, oracle.run(sc)["radiance"]) < 1e-10


def test_colouring_batched(ctx):
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_batched(nx=12, ny=10, nz=8, n_lambda=3).with_(sigma_mode=1)
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve()
    for k in range(3):
        assert rel(rad[k], oracle.run(sc, abs_scale=float(sc.abs_scale[k]))["radiance"]) < 1e-4


def test_colouring_reservation_and_validation(ctx):
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_plain().with_(sigma_mode=1)
    with sgrt.Scene(ctx, sc) as g:
        created = g.sizes["device_bytes"]
    srv = sgrt.Server(ctx, max_resident=1, queue_cap=2, n_streams=1)
    try:
        assert srv.reservation(sc) == created
    finally:
        srv.close()
    with pytest.raises(sgrt.SgError) as e:
        sgrt.Scene(ctx, sc.with_(sigma_mode=2))
    assert e.value.status == sgrt.SG_E_INVALID


@pytest.mark.parametrize("n_fib", [4, 7, 13, 61, 128])
def test_colouring_lattice_sizes(ctx, n_fib):
    """Small and large lattices (with few points a direction's seed scan can leave blocks of
    its lanes empty; 128 is the largest lattice): FP64 phase weights and pixels against the
    oracle, the surface node's cosine cells included."""
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_random_small(5, nx=6, ny=5, nz=4, two_phase=True).with_(sigma_mode=1, n_fib=n_fib)
    ora = oracle.run(sc)
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve(precision="fp64")
        assert info["converged"] == 1
        _, _, val = g.export_csr(lam=0, cols=False)
    big = ora["val"] > 1e-12 * ora["val"].max()
    say("n_fib", n_fib, "radiance", rel(rad, ora["radiance"]), "K", rel(val[big], ora["val"][big]))
    assert rel(val[big], ora["val"][big]) < 1e-12
    assert rel(rad, ora["radiance"]) < 1e-10

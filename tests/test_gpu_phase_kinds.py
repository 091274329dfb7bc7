"""Rayleigh and tabulated phase functions (Sec. 3) on the device against the FP64 oracle:
one wavelength, a two-component mixture, batched wavelengths, the server's copy of a
request, validation, and the reservation of a scene that carries tables."""
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


def cloud_table(n=181):
    """Forward and backward lobes, as a tabulated particle phase function."""
    mu = np.linspace(-1.0, 1.0, n)
    hg = lambda g: (1 - g * g) / (1 + g * g - 2 * g * mu) ** 1.5
    return 0.9 * hg(0.85) + 0.1 * hg(-0.4)


def test_rayleigh_single_wavelength(ctx):
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_plain().with_(phase_kind=np.array([1], np.int32))
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve()
    assert info["converged"] == 1
    err = rel(rad, oracle.run(sc)["radiance"])
    say("rayleigh plain max rel err", err)
    assert err < 1e-4


def test_table_and_rayleigh_mixture(ctx):
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_cloud(nx=20, ny=18, nz=10, seed=5)
    lut = np.stack([cloud_table(), np.zeros(181)])  # row 1 (Rayleigh) is not read
    sc = sc.with_(phase_kind=np.array([2, 1], np.int32), phase_lut=lut)
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve()
    assert info["converged"] == 1
    err = rel(rad, oracle.run(sc)["radiance"])
    say("cloud table + rayleigh max rel err", err)
    assert err < 1e-4


def test_table_batched_wavelengths(ctx):
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_batched(nx=14, ny=12, nz=8, n_lambda=5)
    sc = sc.with_(phase_kind=np.array([2], np.int32), phase_lut=cloud_table(33)[None, :])
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve()
    assert info["converged"] == 1
    for k in (0, 4):
        err = rel(rad[k], oracle.run(sc, abs_scale=float(sc.abs_scale[k]))["radiance"])
        say("batched table lambda", k, err)
        assert err < 1e-4


def test_served_table_scene_equals_solo(ctx):
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_plain().with_(phase_kind=np.array([2], np.int32), phase_lut=cloud_table(65)[None, :])
    with sgrt.Scene(ctx, sc) as g:
        solo, _ = g.solve()
    srv = sgrt.Server(ctx, max_resident=1, queue_cap=4, n_streams=1)
    try:
        t = srv.submit(sc)
        rad, info = srv.wait(t)
        est = srv.reservation(sc)
    finally:
        srv.close()
    assert info["status"] == 0
    assert np.array_equal(np.asarray(rad).reshape(solo.shape), solo)
    with sgrt.Scene(ctx, sc) as g:
        assert est == g.sizes["device_bytes"]


def test_invalid_phase_descriptions(ctx):
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_plain()
    bad = [dict(phase_kind=np.array([3], np.int32)),
           dict(phase_kind=np.array([2], np.int32)),  # no table
           dict(phase_kind=np.array([2], np.int32), phase_lut=np.array([[1.0]])),  # one sample
           dict(phase_kind=np.array([2], np.int32), phase_lut=np.array([[1.0, -0.5, 1.0]])),
           dict(phase_kind=np.array([2], np.int32), phase_lut=np.zeros((1, 4)))]
    for kw in bad:
        with pytest.raises(sgrt.SgError) as e:
            sgrt.Scene(ctx, sc.with_(**kw))
        assert e.value.status == sgrt.SG_E_INVALID, kw

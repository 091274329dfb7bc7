"""Pins of the oracle's Rayleigh and tabulated phase functions (Sec. 3): normalisation
by independent quadrature, exact linear interpolation, and whole-pipeline agreement
between independent routes to the same phase function (a table of the analytic form,
the isotropic special case)."""
import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_2503_16037_amd import scenes


def sphere_integral(f):
    return 2.0 * np.pi * integrate.quad(f, -1.0, 1.0, epsabs=1e-13, epsrel=1e-12, limit=400)[0]


@pytest.mark.parametrize("kind,g,row", [(0, 0.7, None), (0, -0.3, None), (1, 0.0, None),
                                        (2, 0.0, np.random.default_rng(1).uniform(0.1, 3.0, 37))])
def test_components_integrate_to_one(kind, g, row):
    pts = None if row is None else np.linspace(-1, 1, len(row))[1:-1]
    val = 2.0 * np.pi * integrate.quad(lambda m: oracle.phase_value(kind, m, g, row), -1, 1, points=pts,
                                       epsabs=1e-13, epsrel=1e-12, limit=400)[0]
    assert abs(val - 1.0) < 1e-9


def test_table_interpolates_linear_functions_exactly():
    a, b = 2.0, 0.75
    row = a + b * np.linspace(-1.0, 1.0, 9)
    for mu in np.linspace(-1.0, 1.0, 41):
        # a + b mu integrates over the sphere to 4 pi a
        assert abs(oracle.phase_value(2, mu, 0.0, row) - (a + b * mu) / (4 * np.pi * a)) < 1e-15


def scene_with(kind, lut=None, g=0.7):
    sc = scenes.make_plain()
    return sc.with_(hg_g=np.array([g]), phase_kind=np.array([kind], np.int32),
                    phase_lut=None if lut is None else np.asarray(lut, np.float64)[None, :])


def test_constant_table_is_isotropic():
    iso = oracle.run(scenes.make_plain().with_(hg_g=np.array([0.0])))["radiance"]
    tab = oracle.run(scene_with(2, np.full(5, 3.0)))["radiance"]
    assert np.abs(tab - iso).max() <= 1e-12 * np.abs(iso).max()


def test_dense_tables_reproduce_the_analytic_forms():
    mu = np.linspace(-1.0, 1.0, 4097)
    g = 0.5
    hg = (1 - g * g) / (1 + g * g - 2 * g * mu) ** 1.5  # shape only: the table is rescaled
    ref = oracle.run(scenes.make_plain().with_(hg_g=np.array([g])))["radiance"]
    got = oracle.run(scene_with(2, hg, g=0.0))["radiance"]
    assert (np.abs(got - ref) / ref).max() < 1e-5
    ray = oracle.run(scene_with(1))["radiance"]
    ray_tab = oracle.run(scene_with(2, 1.0 + mu * mu, g=0.0))["radiance"]
    assert (np.abs(ray_tab - ray) / ray).max() < 1e-6
    # and Rayleigh differs from the forward-peaked default, so the kind is read
    assert (np.abs(ray - oracle.run(scenes.make_plain())["radiance"]) / ray).max() > 1e-2

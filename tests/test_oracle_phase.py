"""Pins of the oracle's phase-cell weights (Sec. 2, Eq. 7; Sec. 3, Fibonacci lattice).

Independent checks: the rotation is compared with one built by scipy from
the rotation vector (axis u x z, angle acos u_z); lattice ownership with a
numpy argmax in that independently rotated frame; the lattice sums against
closed forms of the Henyey-Greenstein function (normalisation, mean cosine
g, and the forward-hemisphere fraction (1+g)/(2g) - (1-g^2)/(2g sqrt(1+g^2))).
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def test_lattice_geometry(oracle_mod):
    for N in (1, 2, 7, 100, 1001):
        p = oracle_mod.lattice(N)
        assert np.allclose(np.linalg.norm(p, axis=1), 1.0, atol=1e-15)
        i = np.arange(N)
        assert np.allclose(p[:, 2], 1.0 - (2 * i + 1) / N, atol=1e-15)
        # successive azimuths advance by the golden angle
        if N > 2:
            az = np.arctan2(p[:, 1], p[:, 0])
            step = np.mod(np.diff(az), 2 * np.pi)
            assert np.allclose(step, np.pi * (3 - np.sqrt(5)), atol=1e-9)
    # equal-area bands: the mean of z over the lattice is 0, and of z^2 is ~1/3
    p = oracle_mod.lattice(100000)
    assert abs(p[:, 2].mean()) < 1e-12
    assert p[:, 2] @ p[:, 2] / len(p) == pytest.approx(1 / 3, abs=1e-6)


def test_rotation_matches_scipy_rotvec(oracle_mod):
    rng = np.random.default_rng(0)
    for _ in range(500):
        u = _unit(rng.standard_normal(3))
        R = oracle_mod.rotation(u)
        axis = np.cross(u, [0.0, 0.0, 1.0])
        ang = math.acos(max(-1.0, min(1.0, u[2])))
        Rs = Rotation.from_rotvec(axis / np.linalg.norm(axis) * ang).as_matrix()
        assert np.allclose(R, Rs, atol=1e-12)
        assert np.allclose(R @ u, [0, 0, 1], atol=1e-14)
        assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-13)
    # the antipodal case: u = -z maps to +z
    R = oracle_mod.rotation([0.0, 0.0, -1.0])
    assert np.allclose(R @ np.array([0, 0, -1.0]), [0, 0, 1])
    assert np.allclose(R @ R.T, np.eye(3))


def test_ownership_matches_independent_argmax(oracle_mod):
    rng = np.random.default_rng(1)
    N = 100
    p = oracle_mod.lattice(N)
    skipped = 0
    for _ in range(300):
        d = int(rng.integers(1, 31))
        dirs = np.array([_unit(rng.standard_normal(3)) for _ in range(d)])
        u = _unit(rng.standard_normal(3))
        own = oracle_mod.ownership(u, dirs, N)
        axis = np.cross(u, [0.0, 0.0, 1.0])
        Rs = Rotation.from_rotvec(axis / np.linalg.norm(axis) * math.acos(u[2])).as_matrix()
        dots = p @ (dirs @ Rs.T).T  # [N, d]
        ref = np.argmax(dots, axis=1)
        srt = np.sort(dots, axis=1)
        margin = srt[:, -1] - (srt[:, -2] if d > 1 else -np.inf)
        ok = margin > 1e-12
        skipped += int((~ok).sum())
        assert np.array_equal(own[ok], ref[ok])
    assert skipped < 5
    # surface (no rotation)
    for _ in range(100):
        d = int(rng.integers(1, 20))
        dirs = np.array([_unit(rng.standard_normal(3)) for _ in range(d)])
        own = oracle_mod.ownership(None, dirs, N)
        assert np.array_equal(own, np.argmax(p @ dirs.T, axis=1))


def test_ties_go_to_the_smallest_index(oracle_mod):
    dirs = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 1.0], [0.0, 0.0, -1.0]])
    own = oracle_mod.ownership(None, dirs, 100)
    assert set(own.tolist()) == {0, 2}


@pytest.mark.parametrize("g", [0.0, 0.3, 0.7, 0.85])
def test_table_normalisation_and_mean_cosine(oracle_mod, g):
    N = 200001
    t = oracle_mod.hg_table(g, N)
    p = oracle_mod.lattice(N)
    assert t.sum() == pytest.approx(1.0, abs=N * 1e-16)
    # the lattice table is a quadrature of Theta over the sphere: its mean cosine is g
    assert t @ p[:, 2] == pytest.approx(g, abs=2e-4)


@pytest.mark.parametrize("g,expect", [(0.7, 0.915851), (0.75, 14.0 / 15.0), (0.85, 0.963860)])
def test_forward_hemisphere_fraction(oracle_mod, g, expect):
    """Two antipodal out-edges along +-u split the lattice into hemispheres; the
    forward one carries the HG forward-hemisphere fraction as N grows."""
    closed = (1 + g) / (2 * g) - (1 - g * g) / (2 * g * math.sqrt(1 + g * g))
    assert closed == pytest.approx(expect, abs=1e-6)
    rng = np.random.default_rng(3)
    u = _unit(rng.standard_normal(3))
    for N, tol in ((20001, 3e-3), (200001, 1e-3)):
        w = oracle_mod.hg_table(g, N)
        Q = oracle_mod.node_q(u, np.array([u, -u]), N, w=w)
        assert Q.sum() == pytest.approx(1.0, abs=1e-12)
        assert Q[0] == pytest.approx(closed, abs=tol)


def test_cell_weights_partition_and_special_cases(oracle_mod):
    rng = np.random.default_rng(4)
    N = 100
    w = oracle_mod.hg_table(0.8, N)
    for _ in range(100):
        d = int(rng.integers(1, 30))
        dirs = np.array([_unit(rng.standard_normal(3)) for _ in range(d)])
        u = _unit(rng.standard_normal(3))
        Q = oracle_mod.node_q(u, dirs, N, w=w)
        assert Q.sum() == pytest.approx(1.0, abs=1e-13)
        assert np.all(Q >= 0)
    # a single out-edge takes everything
    Q = oracle_mod.node_q(_unit([1, 2, 3]), np.array([_unit([-1, 0, 2])]), N, w=w)
    assert Q[0] == pytest.approx(1.0, abs=1e-14)
    # isotropic scattering: each out-edge gets its owned lattice count / N
    w0 = oracle_mod.hg_table(0.0, N)
    assert np.allclose(w0, 1.0 / N, atol=1e-16)
    dirs = np.array([_unit(rng.standard_normal(3)) for _ in range(9)])
    u = _unit(rng.standard_normal(3))
    Q = oracle_mod.node_q(u, dirs, N, w=w0)
    own = oracle_mod.ownership(u, dirs, N)
    assert np.allclose(Q, np.bincount(own, minlength=9) / N, atol=1e-15)


def test_lambertian_cells(oracle_mod):
    N = 100
    p = oracle_mod.lattice(N)
    # one upward edge takes the whole cosine-weighted upper hemisphere
    Q = oracle_mod.node_q(None, np.array([_unit([0.2, 0.1, 1.0])]), N, surface=True)
    assert Q[0] == pytest.approx(1.0, abs=1e-14)
    # two mirror-image edges split the lattice's cosine weight by the owned points
    dirs = np.array([_unit([1.0, 0.0, 1.0]), _unit([-1.0, 0.0, 1.0])])
    Q = oracle_mod.node_q(None, dirs, N, surface=True)
    zc = np.maximum(p[:, 2], 0.0)
    own = np.argmax(p @ dirs.T, axis=1)
    assert Q == pytest.approx([zc[own == 0].sum() / zc.sum(), zc[own == 1].sum() / zc.sum()], abs=1e-14)
    assert Q.sum() == pytest.approx(1.0, abs=1e-14)
    assert abs(Q[0] - 0.5) < 0.05

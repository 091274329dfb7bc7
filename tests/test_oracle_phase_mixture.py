"""Pins of the oracle's phase-function mixture (Sec. 3: one phase table per medium
component, mixed at a node by the components' shares of the scattering coefficient).

The mixture enters twice: in the lattice weights of the phase cells (Eq. 7), where each
component's table is normalised over the lattice and the normalised tables are mixed,
w_l(i) = sum_k f_lk Theta_k(z_i) / sum_j Theta_k(z_j); and in the gather (Eq. 11), where the
mixed phase function sum_k f_k Theta_k(mu) weighs the radiance scattered toward the sensor.

Independent checks:
  * two components with the same asymmetry reproduce the one-component scene whatever the
    fractions, and the fractions (1, 0) and (0, 1) reproduce each pure component;
  * every K value and source term of a two-component scene equals T_a rho_l sum_{i owned by b}
    w_l(i) with the cells and the weights computed here in numpy (lattice, Henyey-Greenstein
    function, a scipy rotation and an argmax); mixing the raw values and normalising the
    mixture instead differs by percents at g = 0.85, which the check would see;
  * the single-scattering image of a horizontally homogeneous periodic slab whose layers mix
    a g = 0.85 and a g = 0 component in different proportions is the plane-parallel closed
    form with the mixed phase function, at every pixel.
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from paper_2503_16037_amd import scenes


def two_component(sc, g, frac0):
    """The scene with two Henyey-Greenstein components g[0], g[1] and per-voxel fractions
    (frac0, 1 - frac0)."""
    f0 = np.broadcast_to(np.asarray(frac0, np.float64), (sc.nz, sc.ny, sc.nx))
    frac = np.ascontiguousarray(np.stack([f0, 1.0 - f0]), dtype=np.float32)
    return dataclasses.replace(sc, hg_g=np.asarray(g, np.float64), phase_frac=frac)


def hg(g, mu):
    return (1 - g * g) / (4 * np.pi * (1 + g * g - 2 * g * mu) ** 1.5)


def np_lattice(N):
    i = np.arange(N, dtype=np.float64)
    z = 1.0 - (2 * i + 1) / N
    ph = np.mod(i * np.pi * (3 - np.sqrt(5.0)), 2 * np.pi)
    r = np.sqrt(1 - z * z)
    return np.stack([r * np.cos(ph), r * np.sin(ph), z], axis=1)


def to_pole(u):
    """Rotation taking the unit vector u to +z about the axis u x z (scipy)."""
    axis = np.cross(u, [0.0, 0.0, 1.0])
    n = np.linalg.norm(axis)
    if n < 1e-15:
        return np.eye(3) if u[2] > 0 else np.diag([1.0, -1.0, -1.0])
    return Rotation.from_rotvec(axis / n * math.acos(max(-1.0, min(1.0, u[2])))).as_matrix()


def cells(u, s, lat):
    """Owner of each lattice point (argmax of p_i . R s_m, lowest m on ties) and the gap to
    the runner-up (an ownership decided by less than rounding is not compared)."""
    v = lat @ (to_pole(u) @ s.T)  # [N][d]
    own = np.argmax(v, axis=1)
    if s.shape[0] == 1:
        return own, np.full(len(lat), np.inf)
    top2 = np.sort(v, axis=1)[:, -2:]
    return own, top2[:, 1] - top2[:, 0]


def test_equal_asymmetry_reproduces_one_component():
    base = scenes.make_random_small(21, nx=4, ny=3, nz=3, kscale=3.0)
    g = float(base.hg_g[0])
    rng = np.random.default_rng(4)
    # fractions on a 1/256 grid: f and 1 - f are exact in float32 and sum to 1 exactly
    mixed = two_component(base, [g, g], rng.integers(0, 257, (base.nz, base.ny, base.nx)) / 256.0)
    a, b = oracle.run(base), oracle.run(mixed)
    for k in ("val", "S", "phi"):
        assert np.allclose(b[k], a[k], rtol=1e-14, atol=1e-300), k
    assert np.abs(b["radiance"] - a["radiance"]).max() <= 1e-14 * a["radiance"].max()


@pytest.mark.parametrize("which", [0, 1])
def test_pure_fractions_reproduce_each_component(which):
    base = scenes.make_random_small(22, nx=4, ny=3, nz=3, kscale=3.0)
    g = [0.85, 0.0]
    pure = dataclasses.replace(base, hg_g=np.array([g[which]]), phase_frac=None)
    mixed = two_component(base, g, 1.0 if which == 0 else 0.0)
    a, b = oracle.run(pure), oracle.run(mixed)
    for k in ("val", "S", "phi"):
        assert np.allclose(b[k], a[k], rtol=1e-14, atol=1e-300), k
    assert np.abs(b["radiance"] - a["radiance"]).max() <= 1e-14 * a["radiance"].max()
    # and the two components do give different matrices (the check above can fail)
    other = oracle.run(dataclasses.replace(base, hg_g=np.array([g[1 - which]]), phase_frac=None))
    assert np.abs(other["val"] - a["val"]).max() > 1e-3 * a["val"].max()


def test_mixed_cell_weights_equal_an_independent_evaluation():
    sc = scenes.make_random_small(23, nx=4, ny=4, nz=3, kscale=3.0)
    rng = np.random.default_rng(9)
    g = np.array([0.85, 0.0])
    sc = two_component(sc, g, rng.integers(0, 257, (sc.nz, sc.ny, sc.nx)) / 256.0)
    out = oracle.run(sc)
    N = sc.n_fib
    lat = np_lattice(N)
    tables = np.stack([hg(gk, lat[:, 2]) for gk in g])
    tables_norm = tables / tables.sum(axis=1, keepdims=True)
    frac = np.asarray(sc.phase_frac, np.float64).reshape(2, -1)
    pos = oracle.node_positions(sc).astype(np.float64)
    T = np.exp(-out["tau"])
    rho, val, S, row_ptr = out["rho"], out["val"], out["S"], out["row_ptr"]
    tsun = np.exp(-out["tau_sun"])
    sun = np.asarray(sc.sun_dir, np.float64)
    sun_in = -sun / np.linalg.norm(sun)
    compared = wrong_seen = 0
    worst = 0.0
    for l in range(sc.nvox):
        off, end = sc.adj_ptr[l], sc.adj_ptr[l + 1]
        d = int(end - off)
        if d == 0:
            continue
        heads = sc.adj_idx[off:end]
        s = pos[heads] - pos[l]
        s /= np.linalg.norm(s, axis=1, keepdims=True)
        w = frac[:, l] @ tables_norm                            # the reading: mix normalised tables
        w_wrong = frac[:, l] @ tables
        w_wrong /= w_wrong.sum()                                # mixing raw values, then normalising
        incoming = [(-s[m], m) for m in range(d)] + [(sun_in, -1)]
        for u, m in incoming:
            own, gap = cells(u, s, lat)
            if gap.min() < 1e-9:
                continue
            Q = np.bincount(own, weights=w, minlength=d)
            Qw = np.bincount(own, weights=w_wrong, minlength=d)
            for n in range(d):
                b = off + n
                if m >= 0:
                    got = val[row_ptr[b] + m]
                    fac = T[off + m] * rho[l]
                else:
                    got = S[b]
                    fac = tsun[l] * rho[l]
                want = fac * Q[n]
                assert got == pytest.approx(want, rel=1e-12, abs=1e-300), (l, m, n)
                worst = max(worst, abs(got - want) / max(abs(want), 1e-300))
                wrong_seen += abs(fac * Qw[n] - got) > 1e-3 * abs(got)
                compared += 1
    assert compared > 3000
    # the other reading of the mixture would have failed on many entries
    assert wrong_seen > compared // 10


def closed_single_scatter_mixed(sc, g):
    """Single-scattering radiance of a homogeneous layered periodic slab (nodes at the voxel
    centres) whose layer iz scatters with f[0][iz] HG(g[0]) + f[1][iz] HG(g[1]) (the stored
    fractions of the scene's first column): per layer,
    the scattered sun at mid-layer times the chance of scattering inside the layer along the
    line of sight and the view transmittance above it, plus the ground's reflected beam."""
    dz = sc.voxel_m
    su = np.asarray(sc.sun_dir, np.float64)
    vu = np.asarray(sc.view_dir, np.float64)
    su, vu = su / np.linalg.norm(su), vu / np.linalg.norm(vu)
    mu0, muv = su[2], vu[2]
    mu = float(np.dot(-su, vu))
    ms = np.asarray(sc.mu_s, np.float64)[:, 0, 0]
    mu_e = ms + np.asarray(sc.mu_a, np.float64)[:, 0, 0]
    f = np.asarray(sc.phase_frac, np.float64)[:, :, 0, 0]
    I = 0.0
    for iz in range(sc.nz):
        phase = f[0, iz] * hg(g[0], mu) + f[1, iz] * hg(g[1], mu)
        above = mu_e[iz + 1:].sum() * dz
        tau_sun = (0.5 * mu_e[iz] * dz + above) / mu0
        I += (ms[iz] / mu_e[iz]) * phase * math.exp(-tau_sun) * math.exp(-above / muv) * \
            (-math.expm1(-mu_e[iz] * dz / muv))
    tot = mu_e.sum() * dz
    albedo = float(np.asarray(sc.surf_albedo, np.float64)[0, 0])
    return I + math.exp(-tot / muv) * (albedo / np.pi) * mu0 * math.exp(-tot / mu0)


def test_gather_mixed_phase_is_the_plane_parallel_closed_form():
    layers = (0.004, 0.003, 0.002, 0.0015, 0.001, 0.0005)
    base = scenes.make_slab(layers=layers, omega=0.95, g=0.85, albedo=0.2, sza=50.0, vza=20.0)
    g = (0.85, 0.0)
    f0 = np.array([0.9, 0.7, 0.5, 0.3, 0.15, 0.05])
    sc = two_component(base, g, f0[:, None, None])
    pix = oracle.run(sc, scatter_order=1)["radiance"]
    ref = closed_single_scatter_mixed(sc, g)
    assert np.abs(pix - ref).max() <= 1e-12 * ref
    # the pure components bracket the mixed image (the fractions matter)
    pure = [oracle.run(dataclasses.replace(base, hg_g=np.array([gk])), scatter_order=1)["radiance"].mean()
            for gk in g]
    assert min(pure) < ref < max(pure) and abs(pure[0] - pure[1]) > 0.05 * ref

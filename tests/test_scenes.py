"""The seeded scene generators: determinism and the scene-format invariants."""
import numpy as np
import pytest

from paper_2503_16037_amd import scenes

S = scenes.FX


def _check_format(sc):
    N = sc.n_nodes
    assert sc.adj_ptr.shape == (N + 1,) and sc.adj_ptr[0] == 0 and sc.adj_ptr[-1] == sc.n_edges
    tails = np.repeat(np.arange(N), np.diff(sc.adj_ptr))
    heads = sc.adj_idx.astype(np.int64)
    assert np.all(tails != heads)
    key = tails * N + heads
    assert np.all(np.diff(key) > 0)                   # sorted by (tail, head), no duplicates
    rkey = np.sort(heads * N + tails)
    assert np.array_equal(rkey, key)                  # symmetric
    if sc.surface_nodes:
        assert not np.any((tails >= sc.nvox) & (heads >= sc.nvox))
    pos = sc.vol_pos_fx.astype(np.int64)
    iz, iy, ix = np.meshgrid(np.arange(sc.nz), np.arange(sc.ny), np.arange(sc.nx), indexing="ij")
    base = np.stack([ix, iy, iz], -1).reshape(-1, 3) * S
    assert np.all(pos > base) and np.all(pos < base + S)  # strictly inside the own voxel
    assert np.all(np.isfinite(sc.mu_s)) and np.all(sc.mu_s >= 0) and np.all(sc.mu_a >= 0)
    assert sc.sun_dir[2] > 0 and sc.view_dir[2] > 0


def test_plain_config_sizes_and_determinism():
    a = scenes.make_plain()
    b = scenes.make_plain()
    assert a.fingerprint() == b.fingerprint()
    assert scenes.make_plain(seed=9).fingerprint() != a.fingerprint()
    _check_format(a)
    assert a.n_nodes == 512 + 64
    assert 13000 < a.n_edges < 14500
    assert np.array_equal(a.view_dir, [0, 0, 1 << 20])


def test_plume_config_sizes():
    sc = scenes.make_plume()
    _check_format(sc)
    assert sc.n_nodes == 131072 + 4096
    assert abs(sc.n_edges - 3.03e6) / 3.03e6 < 0.02
    assert abs(sc.nnz() - 69.6e6) / 69.6e6 < 0.03
    mu_e = sc.mu_s.astype(np.float64) + sc.mu_a
    assert mu_e.max() == pytest.approx(5e-3 + 1.2e-5, rel=0.01)
    assert 0.1 <= sc.surf_albedo.min() and sc.surf_albedo.max() <= 0.3


def test_small_generators_format():
    for sc in (scenes.make_random_small(0), scenes.make_random_small(1, two_phase=True),
               scenes.make_homogeneous(), scenes.make_worked_example(),
               scenes.make_cloud(nx=16, ny=16, nz=12), scenes.make_batched(nx=12, ny=12, nz=8, n_lambda=5)):
        _check_format(sc)
    c = scenes.make_cloud(nx=16, ny=16, nz=12)
    assert c.phase_frac.shape == (2, 12, 16, 16)
    assert np.allclose(c.phase_frac.sum(0), 1.0, atol=1e-6)
    bt = scenes.make_batched(nx=12, ny=12, nz=8, n_lambda=5)
    assert bt.abs_scale.shape == (5,) and np.all((bt.abs_scale >= 0.1) & (bt.abs_scale <= 10))


def test_served_stream_params_are_seeded():
    p = [scenes.served_stream_params(i) for i in range(50)]
    assert p == [scenes.served_stream_params(i) for i in range(50)]
    for gen, nx, ny, nz, nl, seed in p:
        assert 16 <= nx <= 128 and 16 <= ny <= 128 and 16 <= nz <= 48 and 1 <= nl <= 32
        assert gen == ("plume" if seed % 2 == 0 else "cloud")

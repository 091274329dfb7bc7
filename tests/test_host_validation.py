"""Host-side checks of a scene description (no GPU: sg_scene_reservation runs the same
validation as sg_scene_create before anything touches a device).  Each malformed scene
is refused with SG_E_INVALID and a message naming the problem; a descriptor of another
ABI version with SG_E_ABI.  The adjacency's symmetry is checked on the device and is
covered by the GPU tests."""
import ctypes as C
import dataclasses

import numpy as np
import pytest

from paper_2503_16037_amd import scenes, sgrt


def base():
    return scenes.make_random_small(2, nx=5, ny=4, nz=3, kscale=2.0)


def with_array(sc, field, fn):
    a = np.array(getattr(sc, field), copy=True)
    fn(a)
    return dataclasses.replace(sc, **{field: a})


def unsorted_row(sc):
    ai = sc.adj_idx.copy()
    l = int(np.argmax(np.diff(sc.adj_ptr) >= 2))
    o = sc.adj_ptr[l]
    ai[o], ai[o + 1] = ai[o + 1], ai[o]
    return dataclasses.replace(sc, adj_idx=ai)


def self_loop(sc):
    ai = sc.adj_idx.copy()
    ai[sc.adj_ptr[7]] = 7
    return dataclasses.replace(sc, adj_idx=ai)


def surface_pair(sc):
    """Couple the first two surface nodes (both rows stay ascending)."""
    nv = sc.nvox
    rows = [list(sc.adj_idx[sc.adj_ptr[l]:sc.adj_ptr[l + 1]]) for l in range(sc.n_nodes)]
    rows[nv] = sorted(rows[nv] + [nv + 1])
    rows[nv + 1] = sorted(rows[nv + 1] + [nv])
    ap = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    return dataclasses.replace(sc, adj_ptr=ap, adj_idx=np.concatenate(rows).astype(np.int32))


def head_out_of_range(sc):
    ai = sc.adj_idx.copy()
    ai[-1] = sc.n_nodes + 5
    return dataclasses.replace(sc, adj_idx=ai)


CASES = [
    ("unsorted adjacency row", unsorted_row, "ascending"),
    ("self loop", self_loop, "self loop"),
    ("surface-surface coupling", surface_pair, "surface-surface"),
    ("head out of range", head_out_of_range, "out of range"),
    ("node outside its voxel", lambda sc: with_array(sc, "vol_pos_fx", lambda p: p.__setitem__((0, 0), 65536 * 3)),
     "inside its voxel"),
    ("NaN scattering coefficient", lambda sc: with_array(sc, "mu_s", lambda m: m.flat.__setitem__(5, np.nan)),
     "finite"),
    ("negative absorption", lambda sc: with_array(sc, "mu_a", lambda m: m.flat.__setitem__(3, -1.0)), ">= 0"),
    ("albedo above one", lambda sc: with_array(sc, "surf_albedo", lambda a: a.flat.__setitem__(0, 1.5)),
     "surf_albedo"),
    ("sun below the horizon", lambda sc: dataclasses.replace(sc, sun_dir=np.array([100, 0, -5], np.int32)),
     "positive z"),
    ("direction too long", lambda sc: dataclasses.replace(sc, view_dir=np.array([1 << 23, 0, 1 << 20], np.int32)),
     "2^22"),
    ("one-point lattice", lambda sc: dataclasses.replace(sc, n_fib=1), "n_fib"),
    ("oversized lattice", lambda sc: dataclasses.replace(sc, n_fib=129), "n_fib"),
    ("unknown node weight mode", lambda sc: dataclasses.replace(sc, node_weight_mode=2), "node_weight_mode"),
    ("unknown Sigma mode", lambda sc: dataclasses.replace(sc, sigma_mode=3), "sigma_mode"),
    ("|g| = 1", lambda sc: dataclasses.replace(sc, hg_g=np.array([1.0])), "|g|"),
    ("unknown phase kind", lambda sc: dataclasses.replace(sc, phase_kind=np.array([7], np.int32)), "phase_kind"),
    ("table without samples", lambda sc: dataclasses.replace(sc, phase_kind=np.array([2], np.int32)), "phase_lut"),
    ("all-zero table", lambda sc: dataclasses.replace(sc, phase_kind=np.array([2], np.int32),
                                                      phase_lut=np.zeros((1, 9))), "all zero"),
    ("negative table entry", lambda sc: dataclasses.replace(sc, phase_kind=np.array([2], np.int32),
                                                            phase_lut=np.array([[1.0, -0.5, 1.0]])), ">= 0"),
    ("too many wavelengths", lambda sc: dataclasses.replace(sc, abs_scale=np.ones(257, np.float32)), "n_lambda"),
    ("zero absorption multiplier", lambda sc: dataclasses.replace(sc, abs_scale=np.array([1.0, 0.0], np.float32)),
     "abs_scale"),
    ("periodic flag with unknown bits", lambda sc: dataclasses.replace(sc, periodic=8), "periodic"),
]


@pytest.mark.parametrize("name,make,needle", CASES, ids=[c[0] for c in CASES])
def test_malformed_scene_is_refused_on_the_host(name, make, needle):
    with pytest.raises(sgrt.SgError) as e:
        sgrt.scene_reservation(make(base()))
    assert e.value.status == sgrt.SG_E_INVALID
    assert needle in str(e.value), str(e.value)


def test_well_formed_scenes_are_accepted():
    for sc in (base(), scenes.make_plain(), scenes.make_slab(), scenes.make_random_small(5, two_phase=True)):
        assert sgrt.scene_reservation(sc) > 0


def test_other_abi_version_is_refused():
    keep = []
    d = sgrt.make_desc(base(), keep)
    d.abi_version = sgrt.ABI_VERSION + 1
    b = C.c_uint64()
    assert sgrt.lib().sg_scene_reservation(C.byref(d), C.byref(b)) == sgrt.SG_E_ABI


def test_degree_limits():
    """Up to 4096 couplings per node for one wavelength, with either phase-cell rule; 64
    with several wavelengths (one wavefront per node there)."""
    import oracle
    sc = scenes.make_random_small(4, nx=8, ny=8, nz=6, kscale=2.0)
    ap, ai = oracle.coupling_graph(sc, n_pairs=8 * sc.nvox)
    sc = dataclasses.replace(sc, adj_ptr=ap, adj_idx=ai)
    assert np.diff(ap).max() > 64
    assert sgrt.scene_reservation(sc) > 0
    assert sgrt.scene_reservation(dataclasses.replace(sc, sigma_mode=1)) > 0
    with pytest.raises(sgrt.SgError) as e:
        sgrt.scene_reservation(dataclasses.replace(sc, abs_scale=np.array([1.0, 2.0], np.float32)))
    assert "degree above 64" in str(e.value)


def test_first_failure_is_reported_whatever_the_thread_split():
    """Large arrays are checked on several host threads, each over a contiguous range of
    nodes; the failure reported is still the one at the lowest index (here positions
    outside their voxels at nodes 10 and 150,000, in different ranges)."""
    sc = scenes.make_random_small(3, nx=64, ny=64, nz=40, kscale=2.0)
    assert sc.nvox > 2 * 65536  # at least two ranges
    for bad, want in (((10, 150000), 10), ((150000,), 150000)):
        def plant(p):
            for v in bad:
                p[v, 0] = (v % sc.nx + 2) * 65536  # beyond the voxel's x range
        with pytest.raises(sgrt.SgError) as e:
            sgrt.scene_reservation(with_array(sc, "vol_pos_fx", plant))
        assert f"(node {want})" in str(e.value), str(e.value)

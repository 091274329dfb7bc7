"""Host-side scene checks of the library's periodic flag (no GPU needed): unknown bits,
a sun or view ray that would wind round the period beyond the walk's limit, and a
coupled pair exactly half a period apart (two shortest images) are rejected; the same
pair along a bounded axis is accepted."""
import dataclasses

import numpy as np
import pytest

from paper_2503_16037_amd import scenes, sgrt


def test_periodic_flag_checks():
    sc = scenes.make_slab(nx=6, ny=6, nz=3)
    assert sgrt.scene_reservation(sc) > 0
    for bad in (dataclasses.replace(sc, periodic=4),
                dataclasses.replace(sc, sun_dir=scenes.direction_fx(89.999, 10.0)),
                dataclasses.replace(sc, view_dir=scenes.direction_fx(89.999, 200.0))):
        with pytest.raises(sgrt.SgError):
            sgrt.scene_reservation(bad)
    # nodes 0 and 3: voxels (0,0,0) and (3,0,0), 3 voxels apart in a period of 6
    adj_ptr = np.zeros(sc.n_nodes + 1, np.int64)
    adj_ptr[1:] += 1
    adj_ptr[4:] += 1
    half = dataclasses.replace(sc, adj_ptr=adj_ptr, adj_idx=np.array([3, 0], np.int32))
    with pytest.raises(sgrt.SgError):
        sgrt.scene_reservation(half)
    assert sgrt.scene_reservation(dataclasses.replace(half, periodic=2)) > 0

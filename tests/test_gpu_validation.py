"""Malformed scene descriptions are refused by sg_scene_create with SG_E_INVALID
and a message naming the problem; nothing is uploaded and the context stays usable.
The adjacency's symmetry is checked on the device after the upload (a search per
edge), every other property on the host."""
import dataclasses
import sys

import numpy as np
import pytest

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


def _base():
    return scenes.make_random_small(2, nx=5, ny=4, nz=3, kscale=2.0)


def _drop_edge(sc):
    """Remove one direction of the first edge: the adjacency is no longer symmetric."""
    ap, ai = sc.adj_ptr.copy(), sc.adj_idx.copy()
    ai = np.delete(ai, ap[0])
    ap[1:] -= 1
    return dataclasses.replace(sc, adj_ptr=ap, adj_idx=ai)


def _unsorted(sc):
    ai = sc.adj_idx.copy()
    l = int(np.argmax(np.diff(sc.adj_ptr) >= 2))
    o = sc.adj_ptr[l]
    ai[o], ai[o + 1] = ai[o + 1], ai[o]
    return dataclasses.replace(sc, adj_idx=ai)


def _outside(sc):
    p = sc.vol_pos_fx.copy()
    p[0, 0] = 65536 * 3
    return dataclasses.replace(sc, vol_pos_fx=p)


def _nan_mu(sc):
    m = sc.mu_s.copy()
    m.flat[5] = np.nan
    return dataclasses.replace(sc, mu_s=m)


def _self_loop(sc):
    ai = sc.adj_idx.copy()
    l = 7
    ai[sc.adj_ptr[l]] = l  # the row's first entry points back at the node
    return dataclasses.replace(sc, adj_idx=ai)


@pytest.mark.parametrize("make,needle", [(_drop_edge, "symmetric"), (_unsorted, "ascending"),
                                         (_outside, "inside its voxel"), (_nan_mu, "finite"),
                                         (_self_loop, "self loop")])
def test_malformed_scene_is_refused(ctx, make, needle):
    from paper_2503_16037_amd import sgrt
    sc = make(_base())
    say("malformed", make.__name__)
    with pytest.raises(sgrt.SgError) as e:
        sgrt.Scene(ctx, sc)
    assert e.value.status == sgrt.SG_E_INVALID
    assert needle in str(e.value)
    # the context is still usable
    with sgrt.Scene(ctx, _base()) as g:
        _, info = g.solve()
        assert info["converged"] == 1

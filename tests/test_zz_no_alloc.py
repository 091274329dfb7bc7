"""The allocation-free trace entry point (sg_trace_noalloc) against sg_trace through the C
ABI: the same traversals bit for bit (voxel ids, parameter lengths, counts, and the filler of
the slots past each path) on calls in a row of decreasing size, from several threads at once,
and the refusal of a call beyond the staging area."""
import sys
import threading

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


def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def test_noalloc_trace_equals_trace_on_calls_of_decreasing_size(ctx):
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_plume(nx=40, ny=36, nz=20)
    rng = np.random.default_rng(0)
    with sgrt.Scene(ctx, sc) as g:
        calls = [("edge", rng.choice(sc.n_edges, 60000, replace=False), 12),   # 8.6 MB of the 16 MiB
                 ("sun", rng.choice(sc.n_nodes, 3000, replace=False), 96),
                 ("view", np.arange(sc.nx * sc.ny)[::7], 64),
                 ("edge", np.array([0, sc.n_edges - 1]), 4)]
        for kind, ids, cap in calls:
            say("trace_noalloc", sc.name, kind, len(ids), cap)
            ref = g.trace(kind, ids, cap)
            got = g.trace_noalloc(kind, ids, cap)
            assert same(ref, got), (kind, len(ids), cap)
            vox, dt, cnt = got
            assert cnt.min() >= 1
            # slots past each path are filled, not left over from the previous call
            k = np.arange(cap)[None, :]
            past = k >= np.minimum(cnt, cap)[:, None]
            assert np.all(vox[past] == -1) and np.all(dt[past] == 0.0)
            assert np.all(vox[~past] >= 0)


def test_noalloc_trace_from_several_threads(ctx):
    from paper_2503_16037_amd import sgrt
    scs = [scenes.make_plume(nx=24, ny=20, nz=10, seed=s) for s in (2, 7)]
    with sgrt.Scene(ctx, scs[0]) as g0, sgrt.Scene(ctx, scs[1]) as g1:
        gs = [g0, g1]
        refs = [g.trace("edge", np.arange(0, sc.n_edges, 5), 8) for g, sc in zip(gs, scs)]
        out = [[None] * 6 for _ in gs]

        def work(i):
            for r in range(6):
                out[i][r] = gs[i].trace_noalloc("edge", np.arange(0, scs[i].n_edges, 5), 8)

        ths = [threading.Thread(target=work, args=(i,)) for i in range(2)]
        say("trace_noalloc from two threads")
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        for i in range(2):
            assert all(same(refs[i], o) for o in out[i]), i


def test_noalloc_trace_refuses_calls_beyond_the_staging_area(ctx):
    from paper_2503_16037_amd import sgrt
    cap_bytes = sgrt.lib().sg_trace_noalloc_capacity()
    assert cap_bytes == 16 << 20
    sc = scenes.make_plume(nx=16, ny=16, nz=8)
    with sgrt.Scene(ctx, sc) as g:
        n = 2000
        cap = cap_bytes // (12 * n) + 1  # just over the area
        with pytest.raises(sgrt.SgError) as e:
            g.trace_noalloc("edge", np.arange(n) % sc.n_edges, cap)
        assert e.value.status == sgrt.SG_E_INVALID
        # the largest call that fits still works, and equals sg_trace
        cap_ok = (cap_bytes - 4096) // (12 * n) - 1
        ids = np.arange(n) % sc.n_edges
        assert same(g.trace("edge", ids, cap_ok), g.trace_noalloc("edge", ids, cap_ok))

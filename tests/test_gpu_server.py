"""Serving (sg_server_*): continuous batching of scenes of uneven size.

Each served result must be bit-identical to the same scene solved alone
through the plain one-scene path, whatever else is on the device; scenes
larger than the budget are rejected; a full queue answers SG_E_BUSY; every
finished request records its arrival-to-completion latency.
"""
import sys
import threading
import time

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


def small_stream(n, max_voxels=6000):
    return [scenes.make_served(i, max_voxels=max_voxels) for i in range(n)]


def test_served_results_equal_solo_solves(ctx):
    from paper_2503_16037_amd import sgrt
    stream = small_stream(10)
    say("served mix", [s.name for s in stream])
    solo = []
    for sc in stream:
        with sgrt.Scene(ctx, sc) as g:
            r, _ = g.solve()
            solo.append(np.asarray(r).reshape(sc.n_lambda, sc.ny, sc.nx))
    srv = sgrt.Server(ctx, max_resident=4, queue_cap=64, n_streams=4)
    try:
        tickets = [srv.submit(sc) for sc in stream]
        assert all(t is not None for t in tickets)
        out = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for sc, (rad, info), ref in zip(stream, out, solo):
        assert info["status"] == 0 and info["converged"] == 1
        assert np.array_equal(rad, ref), sc.name
    # spot-check two against the oracle
    for k in (0, 3):
        sc = stream[k]
        ora = oracle.run(sc, abs_scale=float(sc.abs_scale[0]))
        err = np.abs(out[k][0][0] - ora["radiance"]) / np.abs(ora["radiance"])
        assert err.max() < 1e-4


def test_served_sample_of_twenty_matches_oracle(ctx):
    """Twenty requests of the seeded served stream (seeds 5000..5019, plume and cloud, 1..32
    wavelengths; grids halved until they hold at most 4000 voxels), solved through the
    server: for each, the smallest, largest and last absorption multipliers meet the
    per-pixel bar against the FP64 oracle."""
    from paper_2503_16037_amd import sgrt
    stream = small_stream(20, max_voxels=4000)
    srv = sgrt.Server(ctx, max_resident=4, queue_cap=64, n_streams=4)
    try:
        tickets = [srv.submit(sc) for sc in stream]
        assert all(t is not None for t in tickets)
        out = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    worst = 0.0
    for sc, (rad, info) in zip(stream, out):
        assert info["status"] == 0 and info["converged"] == 1, sc.name
        lams = sorted({int(np.argmin(sc.abs_scale)), int(np.argmax(sc.abs_scale)), sc.n_lambda - 1})
        for k in lams:
            ora = oracle.run(sc, abs_scale=float(sc.abs_scale[k]), want_matrix=False)
            err = np.abs(rad[k] - ora["radiance"]) / np.abs(ora["radiance"])
            worst = max(worst, float(err.max()))
            assert err.max() < 1e-4, (sc.name, k, float(err.max()))
    say("served sample of 20: worst per-pixel rel err", worst)


def test_served_mix_with_concurrent_arrivals(ctx):
    from paper_2503_16037_amd import sgrt
    stream = small_stream(8, max_voxels=4000)
    say("concurrent arrivals")
    srv = sgrt.Server(ctx, max_resident=3, queue_cap=64, n_streams=3)
    tickets = [None] * len(stream)

    def submitter():
        for i, sc in enumerate(stream):
            tickets[i] = srv.submit(sc)
            time.sleep(0.002)

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    res = [srv.wait(t) for t in tickets]
    lat = srv.latencies()
    srv.close()
    assert len(lat) == len(stream) and np.all(lat > 0)
    for sc, (rad, info) in zip(stream, res):
        with sgrt.Scene(ctx, sc) as g:
            ref, _ = g.solve()
        assert np.array_equal(rad.reshape(np.asarray(ref).shape), np.asarray(ref))


def test_over_budget_scene_is_rejected():
    from paper_2503_16037_amd import sgrt
    say("over budget")
    with sgrt.Context(0, hbm_budget_bytes=8 << 20) as small:
        srv = sgrt.Server(small, max_resident=2, queue_cap=4, n_streams=2)
        try:
            big = scenes.make_plume(nx=32, ny=32, nz=16)
            with pytest.raises(sgrt.SgError) as e:
                srv.submit(big)
            assert e.value.status == sgrt.SG_E_NOMEM
            tiny = scenes.make_random_small(0, nx=3, ny=3, nz=2, kscale=2.0)
            t = srv.submit(tiny)
            rad, info = srv.wait(t)
            assert info["status"] == 0
        finally:
            srv.close()


def test_budget_serialises_scenes_that_fit_one_at_a_time():
    from paper_2503_16037_amd import sgrt
    sc = scenes.make_plume(nx=20, ny=20, nz=10)
    say("budget for one scene at a time")
    with sgrt.Context(0) as c0:
        with sgrt.Scene(c0, sc) as g:
            need = g.sizes["device_bytes"]
            ref, _ = g.solve()
    with sgrt.Context(0, hbm_budget_bytes=int(need * 1.5)) as c1:
        srv = sgrt.Server(c1, max_resident=4, queue_cap=8, n_streams=4)
        try:
            ts = [srv.submit(sc) for _ in range(4)]
            for t in ts:
                rad, info = srv.wait(t)
                assert info["status"] == 0
                assert np.array_equal(rad[0], ref)
        finally:
            srv.close()


def test_queue_full_reports_busy(ctx):
    from paper_2503_16037_amd import sgrt
    say("queue back-pressure")
    # the one slot is busy with a cloud (tens of ms to create and solve) while four small
    # scenes arrive: the queue holds two of them
    head = scenes.make_cloud()
    sc = scenes.make_plume(nx=16, ny=16, nz=8)
    srv = sgrt.Server(ctx, max_resident=1, queue_cap=2, n_streams=1)
    try:
        got = [srv.submit(head)] + [srv.submit(sc) for _ in range(4)]
        assert any(t is None for t in got)
        for t in got:
            if t is not None:
                _, info = srv.wait(t)
                assert info["status"] == 0
    finally:
        srv.close()


def test_reservation_estimate_matches_created_scene(ctx):
    """The server admits by the reservation a scene will make; it must equal what the
    scene actually reserves (single and batched wavelengths)."""
    from paper_2503_16037_amd import sgrt
    for sc in (scenes.make_random_small(1, nx=5, ny=4, nz=3, two_phase=True, kscale=2.0),
               scenes.make_batched(nx=10, ny=9, nz=6, n_lambda=7)):
        with sgrt.Scene(ctx, sc) as g:
            created = g.sizes["device_bytes"]
        srv = sgrt.Server(ctx, max_resident=1, queue_cap=2, n_streams=1)
        try:
            est = srv.reservation(sc)
        finally:
            srv.close()
        assert est == created, (sc.name, est, created)


def test_resident_slots_need_streams_of_their_own(ctx):
    """Two resident slots on one stream would let one slot's launches fall into the
    other's graph capture: the server refuses max_resident > n_streams."""
    from paper_2503_16037_amd import sgrt
    with pytest.raises(sgrt.SgError) as e:
        sgrt.Server(ctx, max_resident=3, queue_cap=4, n_streams=2)
    assert e.value.status == sgrt.SG_E_INVALID
    # more than four resident slots are refused (the configurations covered are 1..4)
    with pytest.raises(sgrt.SgError) as e:
        sgrt.Server(ctx, max_resident=5, queue_cap=4, n_streams=5)
    assert e.value.status == sgrt.SG_E_INVALID


def test_tight_budget_with_a_gmres_fallback_in_the_mix():
    """A scene whose solve falls back to GMRES (literal node weight on clustered nodes)
    allocates the GMRES basis during its solve, beyond its reservation.  Under a budget
    that holds both scenes' reservations but not the basis besides, the request is put
    back and solved again once the other has finished: both results equal their solo
    solves bit for bit."""
    from paper_2503_16037_amd import sgrt
    from test_oracle_matrix_solve import clustered_scene
    a = clustered_scene()
    b = scenes.make_plume(nx=24, ny=24, nz=12)
    say("tight budget with a GMRES fallback")
    with sgrt.Context(0) as c0:
        refs = []
        for sc in (a, b):
            with sgrt.Scene(c0, sc) as g:
                r, info = g.solve()
                refs.append(np.asarray(r))
            if sc is a:
                assert info["gmres_used"] == 1 and info["converged"] == 1
        srv0 = sgrt.Server(c0, max_resident=1, queue_cap=2, n_streams=1)
        try:
            need = srv0.reservation(a) + srv0.reservation(b)
        finally:
            srv0.close()
    with sgrt.Context(0, hbm_budget_bytes=need + 1024) as c1:
        srv = sgrt.Server(c1, max_resident=2, queue_cap=8, n_streams=2)
        try:
            for order in ((b, a), (a, b), (b, a, b, a)):
                ts = [srv.submit(sc) for sc in order]
                for sc, t in zip(order, ts):
                    rad, info = srv.wait(t)
                    assert info["status"] == 0 and info["converged"] == 1, sc.name
                    ref = refs[0 if sc is a else 1]
                    assert np.array_equal(rad.reshape(ref.shape), ref), sc.name
        finally:
            srv.close()


def test_cancel_a_queued_request(ctx):
    """sg_cancel takes a queued request out (its wait reports SG_E_CANCELLED and it never
    runs); the running one is not touched; the one behind it is still the solo result."""
    from paper_2503_16037_amd import sgrt
    head = scenes.make_cloud()  # 128 x 128 x 48: created and solved in tens of ms
    small = [scenes.make_random_small(20 + i, nx=5, ny=4, nz=3, kscale=2.0) for i in range(2)]
    with sgrt.Scene(ctx, small[1]) as g:
        ref = np.asarray(g.solve()[0]).reshape(small[1].n_lambda, small[1].ny, small[1].nx)
    srv = sgrt.Server(ctx, max_resident=1, queue_cap=8, n_streams=1)
    try:
        t0 = srv.submit(head)
        t1 = srv.submit(small[0])
        t2 = srv.submit(small[1])
        assert srv.cancel(t1) == sgrt.SG_OK
        _, info1 = srv.wait(t1)
        assert info1["status"] == sgrt.SG_E_CANCELLED
        _, info0 = srv.wait(t0)
        assert info0["status"] == 0
        rad2, info2 = srv.wait(t2)
        assert info2["status"] == 0 and np.array_equal(rad2, ref)
        with pytest.raises(sgrt.SgError):  # released ticket
            srv.cancel(t2)
    finally:
        srv.close()

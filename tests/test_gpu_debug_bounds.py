"""The bounds-checked build (libsgrt_debug.so, SG_DEBUG_BOUNDS) on the parity cases.

In a child process that loads the checked library (SGRT_LIB=debug): the checker's self-test
(one check that fails by construction, its index never used) reports its site and the report
clears; then per-voxel scenes (one and two phase functions, surface nodes or none, the paper's
colouring, a periodic slab), line-of-sight scenes (layer and step nodes), a 5-wavelength batch,
traversal exports, the CSR export, the graph builder, the placement on the lines of sight and
three served requests all run with every check passing, and their pixels meet the FP32 bar
against the oracle.  The release library reports that it does not check.
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import dataclasses, sys
import numpy as np
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))
import oracle
from paper_2503_16037_amd import scenes, sgrt

def say(*a):
    print(*a, flush=True)

ctx = sgrt.Context(0)
assert sgrt.debug_bounds(ctx) == (True, 0)
assert sgrt.debug_bounds(ctx, selftest=True) == (True, 0xffff)
assert sgrt.debug_bounds(ctx) == (True, 0)
say("self-test ok")

def check(sc, **opts):
    say("scene", sc.name)
    with sgrt.Scene(ctx, sc) as g:
        rad, info = g.solve(**opts)
        assert info["converged"] == 1
        if sc.n_lambda == 1:
            g.export_csr()
            g.trace("edge", np.arange(min(sc.n_edges, 500)), cap=16)
            g.trace("view", np.arange(sc.nx * sc.ny), cap=256)
    rad = np.asarray(rad).reshape(sc.n_lambda, sc.ny, sc.nx)
    for k in sorted({0, sc.n_lambda - 1}):
        ora = oracle.run(sc, abs_scale=float(sc.abs_scale[k]) if sc.n_lambda > 1 else 1.0)
        err = np.abs(rad[k] - ora["radiance"]) / np.abs(ora["radiance"])
        assert err.max() < 1e-4, (sc.name, k, float(err.max()))
    assert sgrt.debug_bounds(ctx) == (True, 0)

check(scenes.make_random_small(0, nx=6, ny=5, nz=4, kscale=2.0))
check(scenes.make_random_small(1, nx=6, ny=5, nz=4, two_phase=True, surface=False, kscale=2.0))
check(scenes.make_random_small(2, nx=5, ny=5, nz=4, kscale=2.0).with_(sigma_mode=1))
check(scenes.make_random_small(3, nx=5, ny=4, nz=4, kscale=2.0), precision="fp64")
check(scenes.make_slab(nx=10, ny=9, nz=4))
sc0 = scenes.make_random_small(4, nx=6, ny=5, nz=4, vza=30.0, vaa=200.0, kscale=2.0)
for mode, step in (("layer", 0.0), ("step", 45.0)):
    got = sgrt.los_nodes(ctx, sc0.nx, sc0.ny, sc0.nz, sc0.view_dir, sc0.voxel_m, mode=mode, step_m=step)
    want = oracle.los_nodes(sc0.nx, sc0.ny, sc0.nz, sc0.view_dir, sc0.voxel_m, mode, step_m=step)
    assert np.array_equal(got[0].astype(np.int64), want[0]) and all(np.array_equal(a, b) for a, b in zip(got[1:], want[1:]))
    check(scenes.with_los_nodes(sc0, *want, radius_vox=1.8))
check(scenes.make_batched(nx=10, ny=9, nz=6, n_lambda=5))
sc = scenes.make_random_small(5, nx=8, ny=7, nz=5, kscale=2.0)
for kw in (dict(n_pairs=300), dict(c_min=0.0)):
    got = sgrt.graph_build(ctx, sc, **kw)
    want = oracle.coupling_graph(sc, **kw)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
assert sgrt.debug_bounds(ctx) == (True, 0)
say("graph ok")
srv = sgrt.Server(ctx, max_resident=2, queue_cap=8, n_streams=2)
try:
    stream = [scenes.make_random_small(30 + i, nx=5, ny=5, nz=4, kscale=2.0) for i in range(3)]
    out = [srv.wait(t) for t in [srv.submit(s) for s in stream]]
    assert all(info["status"] == 0 for _, info in out)
finally:
    srv.close()
assert sgrt.debug_bounds(ctx) == (True, 0)
ctx.close()
print("checked build: clean", flush=True)
'''


def test_release_library_does_not_check():
    from paper_2503_16037_amd import sgrt
    c = sgrt.Context(0)
    try:
        assert sgrt.debug_bounds(c, selftest=True) == (False, 0)
    finally:
        c.close()


@pytest.mark.timeout(600)
def test_checked_build_runs_the_parity_cases_clean():
    lib = os.path.join(ROOT, "paper_2503_16037_amd", "libsgrt_debug.so")
    assert os.path.exists(lib), "libsgrt_debug.so is built by __graft_entry__.build()"
    env = dict(os.environ, SGRT_LIB="debug")
    r = subprocess.run([sys.executable, "-u", "-c", "import os\nROOT = %r\n" % ROOT + CHILD], env=env,
                       capture_output=True, text=True, timeout=580)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "checked build: clean" in r.stdout

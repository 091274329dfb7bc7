"""The oracle built with the host AddressSanitizer and UndefinedBehaviorSanitizer.

sgoracle.c is compiled with -fsanitize=address,undefined (no recovery) and its entry points
are driven on small scenes in a child process that preloads the ASan runtime: the per-voxel
and line-of-sight scenes (one and two phase functions, the table and Rayleigh kinds, surface
nodes, the paper's colouring, periodic slabs, single scattering, the GMRES path), the walks,
the placement on the lines of sight and the coupling graph (top-n, threshold, general nodes).
Any out-of-bounds access, use after free or undefined arithmetic ends the child with a
report, which fails the test.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVE = r'''
import dataclasses, sys
import numpy as np
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))
import oracle
from paper_2503_16037_amd import scenes
from test_oracle_matrix_solve import clustered_scene

def scene_runs():
    yield scenes.make_random_small(0, nx=4, ny=3, nz=3, kscale=2.0)
    yield scenes.make_random_small(1, nx=4, ny=4, nz=3, two_phase=True, surface=False, kscale=2.0)
    yield scenes.make_random_small(2, nx=3, ny=4, nz=3, kscale=2.0).with_(sigma_mode=1)
    yield scenes.make_slab(nx=8, ny=7, nz=3)
    yield clustered_scene()
    sc = scenes.make_random_small(3, nx=4, ny=4, nz=3, vza=30.0, vaa=200.0, kscale=2.0)
    for mode, step in (("layer", 0.0), ("step", 45.0)):
        pos, lp, ln, lt = oracle.los_nodes(sc.nx, sc.ny, sc.nz, sc.view_dir, sc.voxel_m, mode, step_m=step)
        yield scenes.with_los_nodes(sc, pos, lp, ln, lt, radius_vox=1.8)

for sc in scene_runs():
    for order in (0, 1):
        out = oracle.run(sc, scatter_order=order)
        assert np.all(np.isfinite(out["radiance"])), sc.name
    print("ran", sc.name, flush=True)
sc = scenes.make_random_small(4, nx=4, ny=3, nz=3, kscale=2.0)
P = np.array([[100000, 70000, 0], [5000, 150000, 30000]])
oracle.trace_many(sc.nx, sc.ny, sc.nz, P, np.broadcast_to(sc.view_dir, (2, 3)), 1, 32)
for per in (0, 3):
    oracle.los_nodes(5, 4, 3, scenes.direction_fx(35.0, 70.0), 100.0, "step", step_m=61.0, periodic=per)
for kw in (dict(n_pairs=7), dict(n_pairs=10 ** 6), dict(c_min=0.0), dict(c_min=0.01)):
    oracle.coupling_graph(sc, **kw)
pos, lp, ln, lt = oracle.los_nodes(sc.nx, sc.ny, sc.nz, sc.view_dir, sc.voxel_m, "layer")
oracle.coupling_graph(scenes.with_los_nodes(sc, pos, lp, ln, lt), n_pairs=40)
for kind in (0, 1, 2):
    row = np.linspace(0.2, 1.7, 19) if kind == 2 else None
    oracle.phase_value(kind, 0.3, 0.7, row)
print("sanitized oracle: clean", flush=True)
'''


def _runtime(name):
    path = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.timeout(900)
def test_oracle_clean_under_address_and_ub_sanitizers(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    so = str(tmp_path / "libsgoracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", "-std=c11", os.path.join(ROOT, "oracle", "sgoracle.c"), "-o", so, "-lm"],
                   check=True)
    env = dict(os.environ, SGORACLE_LIB=so, LD_PRELOAD=asan, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=97",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=98")
    script = "import os\nROOT = %r\n" % ROOT + DRIVE
    r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=880)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "sanitized oracle: clean" in r.stdout

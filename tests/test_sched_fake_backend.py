"""The server's scheduler on the CPU with a scripted backend (no device).

tests/sched_harness.cpp drives paper_2503_16037_amd/csrc/sched.hpp -- the queue, admission
by reserved bytes against a budget, the requeue of a request that runs out of budget in the
mix, the retry alone after the backend's cache is released, the GMRES basis joining a
reservation, cancellation and the drain at shutdown -- with a backend whose runs take
scripted bytes from the budget, hold them for a few milliseconds, or fail as scripted
(injected allocation failures).  Each scenario runs in a build with the AddressSanitizer and
UndefinedBehaviorSanitizer, and in one with the ThreadSanitizer: the scheduler is threaded
code, and a data race in it fails the scenario.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SCENARIOS = ["admission", "fifo", "backpressure", "over_budget", "requeue_in_mix", "cold_retry", "alone_nomem",
             "gmres_basis", "gmres_over", "injected", "cancel", "drain"]
SANITIZERS = {"asan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
              "tsan": ["-fsanitize=thread"]}


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ is not installed")
    d = tmp_path_factory.mktemp("sched")
    out = {}
    for name, flags in SANITIZERS.items():
        exe = str(d / ("harness_" + name))
        subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-pthread", "-Wall", "-Wextra", "-Werror", *flags,
                        "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2503_16037_amd", "csrc"),
                        os.path.join(ROOT, "tests", "sched_harness.cpp"), "-o", exe], check=True)
        out[name] = exe
    return out


def test_harness_lists_every_scenario(harness):
    r = subprocess.run([harness["asan"]], capture_output=True, text=True, check=True)
    assert sorted(r.stdout.split()) == sorted(SCENARIOS)


@pytest.mark.parametrize("sanitizer", sorted(SANITIZERS))
@pytest.mark.parametrize("scenario", SCENARIOS)
def test_scheduler_scenario(harness, sanitizer, scenario):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", TSAN_OPTIONS="halt_on_error=1:exitcode=66",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([harness[sanitizer], scenario], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert r.stdout.strip() == "ok " + scenario

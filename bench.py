"""Benchmark of the scattering-graph hot path on one MI355X.

One step = one whole solve of a resident scene: CSR structure, edge and sun
transmittance marches, phase cells + flux matrix + source, Neumann sweeps
with FP64 refinement, pixel gather (every row of the hot path).  Inputs are
already in HBM when the timed region starts (the scene is created, i.e.
uploaded, before it).

Prints ONE JSON line.  Per-kernel durations come from HIP events the library
records on the stream its kernels run on (sg_solve_info timings).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "scenes/s & edge couplings/s at 1e-4 rel vs FP64 oracle; p50/p99 scene latency"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6


def make_workload(name: str):
    from paper_2503_16037_amd import scenes
    if name == "plume":
        return scenes.make_plume(), "plume-64x64x32 (seed 2), 1 wavelength"
    if name == "cloud":
        return scenes.make_cloud(), "cloud-128x128x48 (seed 3), 1 wavelength"
    if name == "plain":
        return scenes.make_plain(), "plain-8x8x8 (seed 1), 1 wavelength"
    raise SystemExit(f"unknown workload {name}")


def spmv_bytes(n_nodes: int, n_edges: int, nnz: int, real_bytes: int = 4) -> int:
    """Algorithmic HBM bytes of one sweep y = S + K x (node-blocked, no column index):
    values nnz, and per edge S, y, x (own), x (gathered once), rev; per node adj_ptr and
    the block offset."""
    return real_bytes * nnz + n_edges * (4 * real_bytes + 4) + n_nodes * 16


def qbuild_flops(scene) -> float:
    """FP64 flops of the lattice-ownership dot products (5 per lattice point x out-edge x
    incoming direction; volume nodes see d + 1 incoming directions, surface nodes one)."""
    d = np.diff(scene.adj_ptr).astype(np.float64)
    nvox = scene.nvox
    n_in = np.ones_like(d)
    n_in[:nvox] = d[:nvox] + 1.0
    return 5.0 * float((n_in * d).sum()) * scene.n_fib


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plume")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}), flush=True)
        sys.exit(2)

    import torch

    from paper_2503_16037_amd import sgrt

    scene, wl_name = make_workload(args.workload)
    ctx = sgrt.Context(0)
    g = sgrt.Scene(ctx, scene)
    sz = g.sizes
    for _ in range(args.warmup):
        g.solve(timing=True)
    torch.cuda.synchronize()
    infos, lat = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        rad, info = g.solve(timing=True)
        lat.append((time.perf_counter() - ts) * 1e3)
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed / args.steps * 1e3
    scenes_per_s = args.steps / elapsed

    def avg(k):
        return float(np.mean([i[k] for i in infos]))

    stages = {k: avg(k) for k in ("ms_structure", "ms_march", "ms_qbuild", "ms_solve", "ms_gather", "ms_total")}
    spmv_launches = sum(i["spmv_launches"] for i in infos)
    spmv_avg_ms = sum(i["ms_spmv_sum"] for i in infos) / max(spmv_launches, 1)
    spmv_per_step_ms = sum(i["ms_spmv_sum"] for i in infos) / len(infos)
    sbytes = spmv_bytes(sz["n_nodes"], sz["n_edges"], sz["nnz"])
    qflops = qbuild_flops(scene)
    if stages["ms_qbuild"] >= spmv_per_step_ms:
        achieved = qflops / (stages["ms_qbuild"] * 1e-3) / 1e12
        roof = {"kernel": "k_qbuild (phase cells + K values + source)", "bound": "alu",
                "achieved": round(achieved, 3), "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 4), "traffic": None,
                "algorithmic_per_launch": qflops, "avg_launch_ms": round(stages["ms_qbuild"], 4)}
    else:
        achieved = sbytes / (spmv_avg_ms * 1e-3) / 1e9
        roof = {"kernel": "k_spmv (FP32 sweep)", "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "algorithmic_per_launch": sbytes, "avg_launch_ms": round(spmv_avg_ms, 5)}
    sweep_roof = {"kernel": "k_spmv", "avg_launch_ms": round(spmv_avg_ms, 5), "bytes_per_launch": sbytes,
                  "achieved_GBs": round(sbytes / max(spmv_avg_ms, 1e-9) / 1e6, 1),
                  "launches_per_step": spmv_launches / len(infos)}

    out = {"metric": METRIC, "value": round(scenes_per_s, 3), "unit": "scenes/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": wl_name, "n_lambda": 1, "couplings": sz["n_edges"], "nnz": sz["nnz"],
                      "nodes": sz["n_nodes"], "parallelism": "single GPU"},
           "edge_couplings_per_s": round(scenes_per_s * sz["n_edges"], 1),
           "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                          "p99": round(float(np.percentile(lat, 99)), 4)},
           "stages_ms": {k: round(v, 4) for k, v in stages.items()},
           "sweeps_per_step": avg("sweeps"), "rel_residual": max(i["rel_residual"] for i in infos),
           "roofline": roof, "sweep_kernel": sweep_roof}

    if not args.no_check or not args.no_cpu_baseline:
        import oracle  # test infrastructure: the accuracy check and the CPU baseline only
        t = time.perf_counter()
        ref = oracle.run(scene, want_matrix=False)
        t_cpu = time.perf_counter() - t
        err = np.abs(rad - ref["radiance"]) / np.abs(ref["radiance"])
        out["max_rel_err_vs_oracle"] = float(err.max())
        out["p99_rel_err_vs_oracle"] = float(np.percentile(err, 99))
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = {"value": round(1.0 / t_cpu, 5), "unit": "scenes/s",
                                   "cores": oracle.num_threads(), "kind": "oracle",
                                   "sample": f"one whole {wl_name} scene ({sz['n_edges']} couplings), "
                                             f"FP64, all stages, {t_cpu:.2f} s"}
    g.close()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

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
# FP64 vector issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one FMA, multiply,
# compare, select or max per lane per clock; 78.6 TFLOP/s counts an FMA as two flops)
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def make_workload(name: str):
    from paper_2503_16037_amd import scenes
    if name == "plume":
        return scenes.make_plume(), "plume-64x64x32 (seed 2), 1 wavelength"
    if name == "cloud":
        return scenes.make_cloud(), "cloud-128x128x48 (seed 3), 1 wavelength"
    if name == "plain":
        return scenes.make_plain(), "plain-8x8x8 (seed 1), 1 wavelength"
    if name == "batched":
        return scenes.make_batched(), "batched plume-96x96x32 (seed 4), 64 wavelengths"
    if name == "slab":
        return (scenes.make_plume(periodic=3),
                "plume-64x64x32 (seed 2) repeating in x and y (periodic slab), 1 wavelength")
    raise SystemExit(f"unknown workload {name}")


def spmv_bytes(n_nodes: int, n_edges: int, nnz: int, real_bytes: int = 4, n_lambda: int = 1) -> int:
    """Algorithmic HBM bytes of one sweep y = S + K x (node-blocked, no column index), for a
    sweep that computes no convergence measure (those that do also read the previous x).
    One wavelength: values nnz, per edge S, y, x (gathered once), rev; per node adj_ptr
    and the block offset.  n wavelengths: phase cells nnz (shared), per edge tau_s, tau_a,
    rev, Qsun and per (edge, wavelength) y and x (gathered once); per (node, wavelength)
    rho and the solar factor."""
    if n_lambda == 1:
        return real_bytes * nnz + n_edges * (3 * real_bytes + 4) + n_nodes * 16
    return 4 * nnz + n_edges * 16 + n_edges * n_lambda * 8 + n_nodes * (16 + 8 * n_lambda)


# Lane operations per (incoming direction, out-edge, lattice point) of the phase-cell ownership
# (Eq. 7): the algorithmic count is 5 (a 3-term dot product as one multiply and two FMAs, then
# a compare and a select of the running argmax).  The kernel issues 5.5 full-rate FP32 and
# integer operations per triple instead (its exact screen: three FMAs and a bitfield insert per
# triple, a three-way maximum, a median and a maximum per two out-edges), plus the FP64 scan of
# the rare uncertified pairs; that count is reported beside it
QBUILD_OPS_PER_PAIR = 5
QBUILD_OPS_ISSUED_PER_PAIR = 5.5


def qbuild_pairs(scene) -> float:
    """(incoming direction, out-edge, lattice point) triples of the phase cells: volume nodes
    see d + 1 incoming directions (in-edges and the sun), surface nodes one."""
    d = np.diff(scene.adj_ptr).astype(np.float64)
    nvox = scene.nvox
    n_in = np.ones_like(d)
    n_in[:nvox] = d[:nvox] + 1.0
    return float((n_in * d).sum()) * scene.n_fib


def step_bytes(sz, nvox, infos_avg):
    """Algorithmic HBM bytes of one whole solve of one wavelength (march + matrix + sweeps +
    FP64 residuals + gather), FP32 working precision:
      march: mu_s, mu_a (8 per voxel), positions and adjacency (20 per node, 4 per edge), the two
        optical-depth channels of every undirected pair (4 per directed edge) and of the sun
        path (8 per node), node weights (4 per node);
      matrix: K values (4 nnz), the source and the sun's cell weight (8 per edge), the optical
        depths read back (8 per edge);
      sweeps: spmv_bytes per sweep (the previous iterate of monitored sweeps included);
      FP64 residual: K values (4 nnz), per edge S (4), x64 (8), gathered x64 (8), r (8), rev (4),
        per node 16;
      gather: phi (8 per edge) and the node radiances (8 per node);
      structure (CSR pattern): the adjacency read (4 per edge, 8 per node), the reverse edge
        ids and row pointers written (4 + 8 per edge), the node offsets (8 per node)."""
    N, E, nnz = sz["n_nodes"], sz["n_edges"], sz["nnz"]
    structure = 16 * E + 16 * N
    march = 8 * nvox + 20 * N + 4 * E + 4 * E + 8 * N + 4 * N
    matrix = 4 * nnz + 8 * E + 8 * E
    residual = 4 * nnz + 32 * E + 16 * N
    gather = 8 * E + 8 * N
    return structure + march + matrix + infos_avg["sweep_bytes_total"] + infos_avg["refinements"] * residual + gather


def host_cpu():
    """The host's CPU model and the logical CPUs this process may run on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0))}


def bench_copy(args):
    """Calibration of the HBM byte counters: a plain device copy of known size (read
    and write 512 MiB each per dispatch).  rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE of
    this command gives the counters' reading for known traffic."""
    import torch
    n = 128 << 20
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    nbytes = 4 * n
    print(json.dumps({"metric": "device copy (counter calibration)", "value": round(2 * nbytes / ms / 1e6, 1),
                      "unit": "GB/s", "bytes_read_per_dispatch": nbytes, "bytes_written_per_dispatch": nbytes,
                      "ms_per_copy": round(ms, 4), "steps": args.steps}), flush=True)


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of a kernel from the committed counter summary
    (profiles/traffic.json, FETCH_SIZE and WRITE_SIZE scaled by a device-copy calibration),
    or None when the kernel's sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    srcs = {"k_qbuild": ["qbuild.hip"], "k_spmv": ["solve.hip"], "k_spmm_wide": ["batched.hip"]}[kernel]
    try:
        rec = json.load(open(path))["kernels"][f"{kernel}@{workload}"]
    except (OSError, KeyError, ValueError):
        return None
    h = hashlib.sha256()
    for f in srcs + ["device.hpp"]:
        h.update(open(os.path.join(ROOT, "paper_2503_16037_amd", "csrc", f), "rb").read())
    return int(rec["bytes"]) if h.hexdigest()[:16] == rec["source_sha256_16"] else None


def _gen_served(i):
    from paper_2503_16037_amd import scenes
    return scenes.make_served(i)


def bench_served(args):
    """Served stream: serial plain one-scene solves versus the continuous-batching server
    (Poisson arrivals at 0.8 x the serial throughput, and all requests at t = 0)."""
    import multiprocessing as mp
    import threading

    import torch

    from paper_2503_16037_amd import sgrt

    n = args.served
    t = time.perf_counter()
    with mp.get_context("spawn").Pool(min(16, os.cpu_count() or 1)) as pool:
        stream = pool.map(_gen_served, range(n))
    gen_s = time.perf_counter() - t
    ctx = sgrt.Context(0)
    # warm the kernels once
    with sgrt.Scene(ctx, stream[0]) as g:
        g.solve()
    torch.cuda.synchronize()
    serial, lat_serial, t_solve = [], [], []
    t0 = time.perf_counter()
    for sc in stream:
        ts = time.perf_counter()
        with sgrt.Scene(ctx, sc) as g:
            tc = time.perf_counter()
            r, _ = g.solve()
            t_solve.append(time.perf_counter() - tc)
        lat_serial.append((time.perf_counter() - ts) * 1e3)
        serial.append(np.asarray(r).reshape(sc.n_lambda, sc.ny, sc.nx))
    serial_s = time.perf_counter() - t0
    serial_rate = n / serial_s

    def run_server(arrivals, resident):
        srv = sgrt.Server(ctx, max_resident=resident, queue_cap=4 * n, n_streams=resident)
        tickets = [None] * n
        t_start = time.perf_counter()

        def submitter():
            for i, sc in enumerate(stream):
                delay = arrivals[i] - (time.perf_counter() - t_start)
                if delay > 0:
                    time.sleep(delay)
                tickets[i] = srv.submit(sc)

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        res = [srv.wait(tk) for tk in tickets]
        makespan = time.perf_counter() - t_start
        lat = srv.latencies()
        srv.close()
        same = all(np.array_equal(r[0], ref) for r, ref in zip(res, serial))
        return n / makespan, lat, same

    rng = np.random.default_rng(5)
    gaps = rng.exponential(1.0 / (0.8 * serial_rate), size=n)
    arrivals = np.concatenate([[0.0], np.cumsum(gaps)[:-1]])
    rate_p, lat_p, same_p = run_server(arrivals, args.resident)
    # the plain path behind a queue: one resident scene at a time, same arrivals
    rate_q, lat_q, same_q = run_server(arrivals, 1)
    rate_s, lat_s, same_s = run_server(np.zeros(n), args.resident)
    ctx.close()
    pct = lambda a, q: round(float(np.percentile(a, q)), 2)
    edges = sum(sc.n_edges for sc in stream)
    out = {"metric": METRIC, "value": round(rate_s, 3), "unit": "scenes/s", "n_gpus": 1, "steps": n, "warmup": 1,
           "ms_per_step": round(1e3 / rate_s, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"served stream, requests 0..{n - 1} (seeds 5000+i, 16^3..128x128x48 voxels, "
                                  f"1..32 wavelengths, plume/cloud)", "resident_slots": args.resident},
           "saturation_scenes_per_s": round(rate_s, 3),
           "poisson_0.8x": {"scenes_per_s": round(rate_p, 3),
                            "latency_ms": {"p50": pct(lat_p, 50), "p99": pct(lat_p, 99)},
                            "one_slot_queue": {"scenes_per_s": round(rate_q, 3),
                                               "latency_ms": {"p50": pct(lat_q, 50), "p99": pct(lat_q, 99)},
                                               "note": "the same arrivals served one scene at a time"}},
           "saturation_latency_ms": {"p50": round(float(np.percentile(lat_s, 50)), 2),
                                     "p99": round(float(np.percentile(lat_s, 99)), 2)},
           "serial_plain": {"scenes_per_s": round(serial_rate, 3),
                            "latency_ms": {"p50": round(float(np.percentile(lat_serial, 50)), 2),
                                           "p99": round(float(np.percentile(lat_serial, 99)), 2)},
                            "solve_only_scenes_per_s": round(n / sum(t_solve), 3),
                            "note": "each scene created (host validation, upload) and solved alone on an idle "
                                    "device; solve_only leaves out the creation"},
           "speedup_vs_serial": round(rate_s / serial_rate, 3),
           "edge_couplings_per_s": round(edges / n * rate_s, 1),
           "served_equal_to_serial_bitwise": bool(same_p and same_q and same_s), "generation_s": round(gen_s, 1)}
    print(json.dumps(out), flush=True)


def bench_nfib(args):
    """Sensitivity to the lattice resolution (Sec. 3 integrates the phase function on a
    Fibonacci lattice): a 48x48x24 cloud (g = 0.85, the most forward-peaked phase function
    of the generators) solved with N_fib = 25..128 points, with the Voronoi cells and with
    the paper's colouring; per-pixel differences against N_fib = 128 Voronoi, and the
    phase-cell build time."""
    import torch

    from paper_2503_16037_amd import scenes, sgrt

    base = scenes.make_cloud(nx=48, ny=48, nz=24, seed=3)
    ctx = sgrt.Context(0)
    res = {}
    for mode, mname in ((0, "voronoi"), (1, "colour")):
        for nf in (25, 50, 75, 100, 128):
            sc = base.with_(n_fib=nf, sigma_mode=mode)
            with sgrt.Scene(ctx, sc) as g:
                g.solve()
                rad, info = g.solve(timing=True)
            torch.cuda.synchronize()
            res[(mname, nf)] = (np.asarray(rad), info["ms_qbuild"], info["ms_total"])
    ref = res[("voronoi", 128)][0]
    table = []
    for (mname, nf), (rad, ms_q, ms_t) in res.items():
        d = np.abs(rad - ref) / np.abs(ref)
        table.append({"cells": mname, "n_fib": nf, "mean_rel_diff": float(d.mean()), "p99_rel_diff": float(np.percentile(d, 99)),
                      "max_rel_diff": float(d.max()), "ms_phase_cells": round(ms_q, 3), "ms_solve_total": round(ms_t, 3)})
    ctx.close()
    out = {"metric": "pixel radiance vs Fibonacci lattice size (n_fib sweep)", "value": table[-1]["mean_rel_diff"],
           "unit": "mean relative difference of the 128-point colouring from the 128-point Voronoi cells",
           "n_gpus": 1, "steps": len(table), "warmup": 1, "higher_is_better": False, "data": "synthetic",
           "dtype": "f32", "vs_baseline": None, "scaling": "weak", "ms_per_step": None,
           "config": {"workload": "cloud 48x48x24 (seed 3, g 0.85 in the clouds), n_fib 25..128, both cell definitions"},
           "sweep": table}
    print(json.dumps(out), flush=True)


def bench_coupling(args):
    """Pixel radiance against the amount of scattering coupling (the paper studies the
    transmittance as a function of the number of couplings): the plume 64x64x32's nodes
    coupled by their strongest couplings (Eq. 4), n = k x voxels for k = 1 .. 24, each
    graph built on the GPU and solved; per-pixel differences against the largest graph,
    the graph's size (couplings, nnz, degrees) and the times of the build and the solve."""
    import torch

    from paper_2503_16037_amd import scenes, sgrt

    base = scenes.make_plume()
    if args.sigma == "colour":
        base = base.with_(sigma_mode=1)
    ctx = sgrt.Context(0)
    ks = (args.couplings,) if args.couplings else (1, 2, 4, 8, 11.5, 16, 24)
    res = {}
    for k in ks:
        t = time.perf_counter()
        ap, ai = sgrt.graph_build(ctx, base, n_pairs=int(k * base.nvox))
        ms_build = (time.perf_counter() - t) * 1e3
        sc = base.with_(adj_ptr=ap, adj_idx=ai)
        deg = np.diff(ap)
        with sgrt.Scene(ctx, sc) as g:
            for _ in range(2):  # the second solve tunes the sweep's launch shape
                g.solve()
            rad, info = g.solve(timing=True)
            nnz = g.sizes["nnz"]
        torch.cuda.synchronize()
        res[k] = dict(rad=np.asarray(rad), couplings=int(ap[-1]), nnz=int(nnz), max_degree=int(deg.max()),
                      nodes_above_64=int((deg > 64).sum()), uncoupled_nodes=int((deg == 0).sum()),
                      ms_build=round(ms_build, 2), ms_qbuild=round(info["ms_qbuild"], 2),
                      ms_solve=round(info["ms_solve"], 2), ms_total=round(info["ms_total"], 2), sweeps=info["sweeps"])
    # the radius graph of the same nodes (every node coupled to its neighbours within 1.8 voxels)
    with sgrt.Scene(ctx, base) as g:
        for _ in range(2):
            g.solve()
        rad_r, info_r = g.solve(timing=True)
    ctx.close()
    ref = res[ks[-1]]["rad"]
    table = []
    for k in ks:
        r = res[k]
        d = np.abs(r.pop("rad") - ref) / np.abs(ref)
        table.append({"couplings_per_voxel": k, **r, "mean_rel_diff": float(d.mean()),
                      "p99_rel_diff": float(np.percentile(d, 99)), "max_rel_diff": float(d.max())})
    dr = np.abs(np.asarray(rad_r) - ref) / np.abs(ref)
    out = {"metric": "pixel radiance vs amount of scattering coupling (strongest-coupling graphs)",
           "value": table[-2]["mean_rel_diff"] if len(table) > 1 else 0.0,
           "unit": "mean relative difference of the second largest graph from the largest", "n_gpus": 1, "steps": len(table),
           "warmup": 1, "higher_is_better": False, "data": "synthetic", "dtype": "f32", "vs_baseline": None,
           "scaling": "weak", "ms_per_step": None,
           "config": {"workload": "plume-64x64x32 (seed 2) nodes, strongest couplings k x voxels, k = 1..24",
                      "phase_cells": args.sigma},
           "sweep": table,
           "radius_graph": {"couplings": int(base.adj_ptr[-1]), "mean_rel_diff": float(dr.mean()),
                            "p99_rel_diff": float(np.percentile(dr, 99)), "ms_total": round(info_r["ms_total"], 2)}}
    print(json.dumps(out), flush=True)


GRAPH_OPS_PER_PAIR = 10  # FP64 operations of one coupling: 3 subtractions, 4 products, 2 sums, 1 division


def bench_graph(args):
    """The scattering graph (Eq. 4) of the 64x64x32 plume's nodes: the n strongest
    couplings with n = 11.5 x voxels (mean degree 23, the radius graph's).  The scene's
    arrays are host buffers handed to sg_graph_build; the timed call includes their
    upload and the adjacency's download."""
    import torch

    from paper_2503_16037_amd import scenes, sgrt

    sc = scenes.make_plume()
    nvox = sc.nx * sc.ny * sc.nz
    n_pairs = int(11.5 * nvox)
    ctx = sgrt.Context(0)
    for _ in range(max(1, args.warmup)):
        sgrt.graph_build(ctx, sc, n_pairs=n_pairs)
    torch.cuda.synchronize()
    infos, lat = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        ap_, ai_, info = sgrt.graph_build(ctx, sc, n_pairs=n_pairs, info=True)
        lat.append((time.perf_counter() - ts) * 1e3)
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    deg = np.diff(ap_)
    inf = infos[-1]
    ms_pairs = float(np.mean([i["ms_pairs"] for i in infos]))
    # the count and the fill kernel each evaluate every pair of the boxes
    ops = 2.0 * GRAPH_OPS_PER_PAIR * inf["pairs_evaluated"]
    achieved = ops / (ms_pairs * 1e-3) / 1e12
    N = nvox + sc.nx * sc.ny
    out = {"metric": "scattering-graph builds/s (Eq. 4: the n strongest couplings of a scene's nodes)",
           "value": round(args.steps / elapsed, 3), "unit": "builds/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"coupling graph of plume-64x64x32 (seed 2) nodes ({N} incl. surface), "
                                  f"n = {n_pairs} strongest couplings", "parallelism": "single GPU"},
           "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                          "p99": round(float(np.percentile(lat, 99)), 4)},
           "roofline": {"kernel": "k_graph_pairs (count + fill passes)", "bound": "alu",
                        "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 2), "unit": "T lane-op/s",
                        "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": None,
                        "algorithmic_per_launch": ops / 2, "avg_launch_ms": round(ms_pairs / 2, 5)},
           "graph": {"pairs_in_all": N * (N - 1) // 2, "pairs_evaluated": inf["pairs_evaluated"],
                     "candidates": inf["candidates"], "selected": int(ap_[-1] // 2),
                     "threshold_C2": inf["threshold"], "streamed": inf["streamed"],
                     "ms_pairs": round(ms_pairs, 4),
                     "ms_sort": round(float(np.mean([i["ms_sort"] for i in infos])), 4),
                     "max_degree": int(deg.max()), "isolated_nodes": int((deg == 0).sum())}}
    if not args.no_cpu_baseline:
        import oracle  # test infrastructure: the CPU baseline only
        # bounded sample: the nodes of the lowest 24 of 32 layers, brute force over all
        # their pairs; scaled to the full node set by the pair count
        L = 24
        sub_sc = sc.with_(nz=L, mu_s=sc.mu_s[:L].copy(), mu_a=sc.mu_a[:L].copy(),
                          vol_pos_fx=sc.vol_pos_fx[:L * sc.nx * sc.ny].copy())
        Ns = L * sc.nx * sc.ny + sc.nx * sc.ny
        t = time.perf_counter()
        oracle.coupling_graph(sub_sc, n_pairs=int(11.5 * L * sc.nx * sc.ny))
        t_cpu = time.perf_counter() - t
        scale = (N * (N - 1) / 2) / (Ns * (Ns - 1) / 2)
        out["cpu_baseline"] = {"value": round(1.0 / (t_cpu * scale), 8), "unit": "builds/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"brute force over the {Ns} nodes of the lowest {L} layers plus the surface "
                                         f"({t_cpu:.2f} s), scaled by the pair count x{scale:.1f}"}
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_los(args):
    """Scattering nodes on the pixels' lines of sight (Sec. 2 path points; Sec. 3 step 1) for
    the 64x64x32 plume: the placement (sg_los_nodes, one node per layer crossed or one per
    50 m step) timed on its own, then the layer nodes coupled by their 11.5 x n strongest
    couplings (Eq. 4, sg_graph_build) and whole solves of that scene timed like the main
    workloads; the pixels are checked against the FP64 oracle on the same nodes and graph."""
    import torch

    from paper_2503_16037_amd import scenes, sgrt

    base = scenes.make_plume()
    ctx = sgrt.Context(0)
    place = {}
    for mode, step_m in (("layer", 0.0), ("step", 50.0)):
        for _ in range(max(1, args.warmup)):
            out = sgrt.los_nodes(ctx, base.nx, base.ny, base.nz, base.view_dir, base.voxel_m, mode, step_m=step_m)
        torch.cuda.synchronize()
        lat = []
        for _ in range(args.steps):
            t = time.perf_counter()
            out = sgrt.los_nodes(ctx, base.nx, base.ny, base.nz, base.view_dir, base.voxel_m, mode, step_m=step_m)
            lat.append((time.perf_counter() - t) * 1e3)
        place[mode] = {"nodes": int(len(out[0])), "elements": int(len(out[2])),
                       "ms_p50": round(float(np.percentile(lat, 50)), 4),
                       "ms_p99": round(float(np.percentile(lat, 99)), 4), "out": out}
    pos, lp, ln, lt = place["layer"].pop("out")
    place["step"].pop("out")
    sc = scenes.with_los_nodes(base, pos, lp, ln, lt, name="plume-64x64x32-los-layer")
    n = len(pos) + (sc.nx * sc.ny if sc.surface_nodes else 0)
    t = time.perf_counter()
    ap_, ai_ = sgrt.graph_build(ctx, sc, n_pairs=int(11.5 * n))
    ms_graph = (time.perf_counter() - t) * 1e3
    sc = sc.with_(adj_ptr=ap_, adj_idx=ai_)
    with sgrt.Scene(ctx, sc) as g:
        for _ in range(max(2, args.warmup)):  # the second solve tunes the sweep's launch shape
            g.solve()
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
        nnz = g.sizes["nnz"]
    stages = {k: round(float(np.mean([i[k] for i in infos])), 4)
              for k in ("ms_structure", "ms_march", "ms_qbuild", "ms_solve", "ms_gather", "ms_total")}
    out = {"metric": "scenes/s on line-of-sight nodes (placement, coupling graph, whole solves)",
           "value": round(args.steps / elapsed, 3), "unit": "scenes/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"plume-64x64x32 (seed 2) on its pixels' line-of-sight nodes (one per layer), "
                                  f"{n} nodes incl. surface, {int(ap_[-1])} couplings (the 11.5 x n strongest)",
                      "parallelism": "single GPU"},
           "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                          "p99": round(float(np.percentile(lat, 99)), 4)},
           "stages_ms": stages, "sweeps_per_step": float(np.mean([i["sweeps"] for i in infos])),
           "nnz": int(nnz), "placement": place, "ms_graph_build": round(ms_graph, 3)}
    if not args.no_check or not args.no_cpu_baseline:
        import oracle  # test infrastructure: the check and the CPU baseline only
        t = time.perf_counter()
        ora = oracle.run(sc)
        t_cpu = time.perf_counter() - t
        if not args.no_check:
            err = np.abs(np.asarray(rad, np.float64) - ora["radiance"]) / np.maximum(np.abs(ora["radiance"]), 1e-300)
            out["max_rel_err_vs_oracle"] = float(err.max())
            out["p99_rel_err_vs_oracle"] = float(np.percentile(err, 99))
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = {"value": round(1.0 / t_cpu, 6), "unit": "scenes/s",
                                   "cores": oracle.num_threads(), "kind": "oracle", "host": host_cpu(),
                                   "sample": f"one solve of the same scene, FP64, all stages, {t_cpu:.2f} s"}
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cloud",
                    help="plume | cloud | batched | plain | slab (periodic plume) | served | graph | los | nfib | coupling | copy")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--served", type=int, default=40, help="requests of the served stream (workload served)")
    ap.add_argument("--resident", type=int, default=4, help="resident scenes of the server (workload served)")
    ap.add_argument("--couplings", type=float, default=None,
                    help="workload coupling: only this many couplings per voxel (for profiling)")
    ap.add_argument("--exact-cells", action="store_true",
                    help="phase-cell owners by the FP64 scan alone (no FP32 screen; same results)")
    ap.add_argument("--sigma", default="voronoi", choices=["voronoi", "colour"],
                    help="phase cells: Voronoi ownership (default) or the paper's colouring with flood fill")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}), flush=True)
        sys.exit(2)

    if args.workload == "served":
        bench_served(args)
        return
    if args.workload == "copy":
        bench_copy(args)
        return
    if args.workload == "graph":
        bench_graph(args)
        return
    if args.workload == "nfib":
        bench_nfib(args)
        return
    if args.workload == "coupling":
        bench_coupling(args)
        return
    if args.workload == "los":
        bench_los(args)
        return

    import torch

    from paper_2503_16037_amd import sgrt

    scene, wl_name = make_workload(args.workload)
    if args.sigma == "colour":
        scene = scene.with_(sigma_mode=1)
        wl_name += ", phase cells by nearest-point colouring and flood fill"
    ctx = sgrt.Context(0)
    torch.cuda.synchronize()
    t_up = time.perf_counter()
    g = sgrt.Scene(ctx, scene)  # host buffers -> HBM (validation, upload, reservation)
    torch.cuda.synchronize()
    upload_ms = (time.perf_counter() - t_up) * 1e3
    upload_bytes = scene.nbytes()
    sz = g.sizes
    screen = not args.exact_cells
    for _ in range(args.warmup):
        g.solve(timing=True, screen=screen)
    torch.cuda.synchronize()
    infos, lat = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        rad, info = g.solve(timing=True, screen=screen)
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
    # a sweep that computes the convergence measures also reads the previous iterate
    # (4 bytes per edge and wavelength): average over the timed launches
    monitored = sum(i["spmv_monitored"] for i in infos) / max(spmv_launches, 1)
    sbytes = spmv_bytes(sz["n_nodes"], sz["n_edges"], sz["nnz"], n_lambda=g.n_lambda) + \
        monitored * 4 * sz["n_edges"] * g.n_lambda
    qpairs = qbuild_pairs(scene)
    qops = QBUILD_OPS_PER_PAIR * qpairs
    if stages["ms_qbuild"] >= spmv_per_step_ms and g.n_lambda == 1:
        achieved = qops / (stages["ms_qbuild"] * 1e-3) / 1e12
        issued = QBUILD_OPS_ISSUED_PER_PAIR * qpairs / (stages["ms_qbuild"] * 1e-3) / 1e12
        roof = {"kernel": ("k_qcolour" if args.sigma == "colour" else "k_qbuild") + " (phase cells + K values + source)",
                "bound": "alu",
                "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 2), "unit": "T lane-op/s",
                "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": measured_traffic("k_qbuild", args.workload),
                "algorithmic_per_launch": qops, "ops_per_pair": QBUILD_OPS_PER_PAIR,
                "avg_launch_ms": round(stages["ms_qbuild"], 4),
                "frac_issued": round(issued / ALU_PEAK_TOPS, 4), "ops_issued_per_pair": QBUILD_OPS_ISSUED_PER_PAIR}
    else:
        achieved = sbytes / (spmv_avg_ms * 1e-3) / 1e9
        roof = {"kernel": "k_spmv (FP32 sweep)" if g.n_lambda == 1 else "k_spmm (FP32, all wavelengths)",
                "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic("k_spmv" if g.n_lambda == 1 else "k_spmm_wide", args.workload),
                "algorithmic_per_launch": sbytes, "avg_launch_ms": round(spmv_avg_ms, 5)}
    # the phase cells against the ALU peak whichever kernel dominates the step
    cell_roof = {"kernel": "k_qcolour" if args.sigma == "colour" else "k_qbuild", "bound": "alu",
                 "avg_launch_ms": round(stages["ms_qbuild"], 4), "ops_per_pair": QBUILD_OPS_PER_PAIR,
                 "achieved": round(qops / (stages["ms_qbuild"] * 1e-3) / 1e12, 3), "unit": "T lane-op/s",
                 "frac": round(qops / (stages["ms_qbuild"] * 1e-3) / 1e12 / ALU_PEAK_TOPS, 4),
                 "owners": "FP64 scan only" if args.exact_cells else "FP32 screen, FP64 scan where uncertified"}
    sweep_roof = {"kernel": "k_spmv", "avg_launch_ms": round(spmv_avg_ms, 5), "bytes_per_launch": round(sbytes),
                  "monitored_fraction": round(monitored, 4),
                  "achieved_GBs": round(sbytes / max(spmv_avg_ms, 1e-9) / 1e6, 1),
                  "launches_per_step": spmv_launches / len(infos)}

    step_hbm = None
    if g.n_lambda == 1:
        # bytes of the step: every timed sweep launch (monitored ones read the previous x too)
        sweep_total = (spmv_bytes(sz["n_nodes"], sz["n_edges"], sz["nnz"]) * spmv_launches +
                       4 * sz["n_edges"] * sum(i["spmv_monitored"] for i in infos)) / len(infos)
        sb = step_bytes(sz, scene.nvox, {"sweep_bytes_total": sweep_total, "refinements": avg("refinements")})
        # the same without the phase-cell kernel, whose time is ALU issue (reported against the ALU
        # peak in phase_cell_kernel): its K values and source are taken out of the bytes
        matrix = 4 * sz["nnz"] + 8 * sz["n_edges"] + 8 * sz["n_edges"]
        rest_ms = ms_step - stages["ms_qbuild"]
        # the solve stage alone: the first iterate (rhs read, x written), the timed sweeps and the
        # FP64 residuals, over the stage's own time
        solve_b = (8 * sz["n_edges"] + sweep_total +
                   avg("refinements") * (4 * sz["nnz"] + 32 * sz["n_edges"] + 16 * sz["n_nodes"]))
        step_hbm = {"bytes_per_step": round(sb), "achieved_GBs": round(sb / (ms_step * 1e-3) / 1e9, 1),
                    "frac": round(sb / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "without_phase_cells": {
                        "bytes": round(sb - matrix), "ms": round(rest_ms, 4),
                        "frac": round((sb - matrix) / (rest_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
                    "solve_stage": {
                        "bytes": round(solve_b), "ms": round(stages["ms_solve"], 4),
                        "frac": round(solve_b / (stages["ms_solve"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
                    "note": "algorithmic bytes of structure + march + K write + sweeps + FP64 residuals + gather "
                            "over the whole step's wall time; the phase cells are ALU-bound and count no bytes; "
                            "without_phase_cells: structure, march, sweeps, residuals and gather over the step's "
                            "time less the phase-cell kernel's; solve_stage: the first iterate, the sweeps and the "
                            "FP64 residuals over the solve stage's time"}
    out = {"metric": METRIC, "value": round(scenes_per_s, 3), "unit": "scenes/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": wl_name, "n_lambda": g.n_lambda, "couplings": sz["n_edges"], "nnz": sz["nnz"],
                      "nodes": sz["n_nodes"], "parallelism": "single GPU"},
           "edge_couplings_per_s": round(scenes_per_s * sz["n_edges"], 1),
           "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                          "p99": round(float(np.percentile(lat, 99)), 4)},
           "stages_ms": {k: round(v, 4) for k, v in stages.items()},
           "sweeps_per_step": avg("sweeps"), "rel_residual": max(i["rel_residual"] for i in infos),
           "scene_upload": {"ms": round(upload_ms, 3), "bytes": upload_bytes,
                            "note": "sg_scene_create from host buffers, outside the timed region"},
           "roofline": roof, "phase_cell_kernel": cell_roof, "sweep_kernel": sweep_roof, "step_hbm": step_hbm}

    if g.n_lambda > 1:
        out["wavelength_solves_per_s"] = round(scenes_per_s * g.n_lambda, 2)
    if not args.no_check or not args.no_cpu_baseline:
        import oracle  # test infrastructure: the accuracy check and the CPU baseline only
        t = time.perf_counter()
        k = 0
        ref = oracle.run(scene, want_matrix=False) if g.n_lambda == 1 else \
            oracle.run(scene, abs_scale=float(scene.abs_scale[k]), want_matrix=False)
        t_cpu = time.perf_counter() - t
        got = rad if g.n_lambda == 1 else rad[k]
        err = np.abs(got - ref["radiance"]) / np.abs(ref["radiance"])
        out["max_rel_err_vs_oracle"] = float(err.max())
        out["p99_rel_err_vs_oracle"] = float(np.percentile(err, 99))
        if not args.no_cpu_baseline:
            # the oracle solves one wavelength per run: a whole n-wavelength scene costs n runs
            out["cpu_baseline"] = {"value": round(1.0 / (t_cpu * g.n_lambda), 6), "unit": "scenes/s",
                                   "cores": oracle.num_threads(), "kind": "oracle",
                                   "host": host_cpu(),
                                   "sample": f"one wavelength of {wl_name} ({sz['n_edges']} couplings), "
                                             f"FP64, all stages, {t_cpu:.2f} s"
                                             + (f", x {g.n_lambda} wavelengths" if g.n_lambda > 1 else ""),
                                   "stages_s": {k: round(v, 4) for k, v in ref["stage_s"].items()}}
            if args.workload in ("plain", "plume"):
                # the same run on one thread
                threads = oracle.num_threads()
                oracle.set_threads(1)
                t = time.perf_counter()
                one = oracle.run(scene, want_matrix=False)
                out["cpu_baseline"]["one_thread"] = {
                    "s": round(time.perf_counter() - t, 3),
                    "stages_s": {k: round(v, 4) for k, v in one["stage_s"].items()}}
                oracle.set_threads(threads)
    g.close()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

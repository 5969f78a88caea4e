"""Benchmark of the coupled IB-LBM timestep on one MI355X.

Default workload: the RBC suspension channel -- D3Q19 BGK, tau 0.8, lattice
256 x 128 x 128 (periodic x, walls on y and z), body force gx = 1e-6, seeded
random sequential insertion of biconcave (Evans-Fung) cells of 642 nodes,
diameter 16 lu, to 20 % of the fluid volume, ks 0.005, kb 0.001, cosine delta
kernel, FP32 population storage.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--storage f32|f16]

Prints one JSON line.  `value` is coupled-step MLUPS (all allocated cells x
steps / wall time of the K timed steps, inputs resident in HBM).  The timed
steps run phase by phase with a HIP event after each phase on the
simulation's stream, which gives the dominant kernel's (collide-stream) mean
duration for the roofline object.  The CPU baseline times the FP64 oracle on
a few steps of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2}


def _log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def load_spec(args):
    """The default workload; the generated node arrays are cached (exact
    copies) so repeated runs skip the random sequential insertion."""
    from paper_1704_04551_amd import workloads as W
    cache = args.cache
    if cache and os.path.exists(cache):
        with np.load(cache, allow_pickle=False) as z:
            xs, T = z["x"], z["tris"]
        caps = [W.Capsule(x, x.copy(), T, 0.005, 0.001, "rbc16") for x in xs]
        return W.SimSpec(n=(256, 128, 128), tau=0.8, g_body=(1e-6, 0.0, 0.0), wall=(0, 1, 1),
                         delta="cos", capsules=caps, steps=1000, seed=1002,
                         name="rbc-channel-256x128x128")
    spec = W.config_rbc_channel()
    if cache:
        os.makedirs(os.path.dirname(cache) or ".", exist_ok=True)
        np.savez(cache, x=np.stack([c.x for c in spec.capsules]), tris=spec.capsules[0].tris)
    return spec


def cpu_baseline(spec, steps):
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import oracle
    from parity_util import oracle_from_spec
    o = oracle_from_spec(spec)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {"value": spec.cells * steps / dt / 1e6, "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": "%d FP64 oracle steps of the same %dx%dx%d workload (%d cells, %d nodes), "
                      "%.1f s" % (steps, *spec.n, len(spec.capsules), spec.nodes, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "f64"])
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cache", default=os.path.join(ROOT, "gpurun_out", "rbc_channel_spec.npz"))
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB, 5 times "
                         "(calibrates the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "launches": 5}))
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(the multi-GPU slab decomposition is a design, not built)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1704_04551_amd import ibl

    _log("generating workload")
    spec = load_spec(args)
    _log("%d cells, %d nodes; creating simulation" % (len(spec.capsules), spec.nodes))
    sim = ibl.Sim.from_spec(spec, storage=args.storage, device="cuda:0")
    sim.step(args.warmup)
    sim.sync()
    _log("warmup done")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phases, total_ms = sim.profile_phases(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.sync()
    _log("timed %d steps: %.3f s wall, %.3f ms/step by events" % (args.steps, wall, total_ms / args.steps))

    # the same number of steps replayed as HIP graphs (no per-phase events)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ext = torch.cuda.ExternalStream(sim.stream_handle)
    ev0.record(ext)
    sim.step(args.steps)
    ev1.record(ext)
    sim.sync()
    graph_ms = ev0.elapsed_time(ev1) / args.steps
    mass, mom, health = sim.conservation()

    cells = spec.cells
    ms_per_step = wall * 1e3 / args.steps
    mlups = cells * args.steps / wall / 1e6
    sb = STORAGE_BYTES[args.storage]
    lat_bytes = 2 * 19 * sb * cells
    lat_ms = phases["lattice"]
    achieved = lat_bytes / (lat_ms * 1e-3) / 1e9
    result = {
        "metric": "coupled-step MLUPS + % HBM roofline at stated error vs FP64; served p50/p99",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f16": "f16-offset storage, f32 compute", "f64": "f64"}[args.storage],
        "data": "synthetic (seeded RSA of Evans-Fung cells)",
        "config": {"workload": spec.name, "cells": cells, "capsules": len(spec.capsules),
                   "nodes": spec.nodes, "tau": spec.tau, "g_body": spec.g_body[0],
                   "storage": args.storage, "delta": spec.delta},
        "roofline": {"bound": "hbm", "kernel": "k_lattice (collide-stream)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_launch": lat_bytes, "launch_ms": round(lat_ms, 5)},
        "step_roofline_frac": round(cells * 2 * 19 * sb / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "phase_ms": {k: round(v, 5) for k, v in phases.items()},
        "graph_ms_per_step": round(graph_ms, 4),
        "graph_mlups": round(cells / (graph_ms * 1e-3) / 1e6, 1),
        "health": health,
    }
    if not args.no_cpu:
        _log("cpu baseline (oracle, %d steps)" % args.cpu_steps)
        result["cpu_baseline"] = cpu_baseline(spec, args.cpu_steps)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark of the coupled IB-LBM timestep on one MI355X.

Default workload: the RBC suspension channel -- D3Q19 BGK, tau 0.8, lattice
256 x 128 x 128 (periodic x, walls on y and z), body force gx = 1e-6, seeded
random sequential insertion of biconcave (Evans-Fung) cells of 642 nodes,
diameter 16 lu, to 20 % of the fluid volume, ks 0.005, kb 0.001, cosine delta
kernel, FP32 population storage.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--storage f32|f16|f64]

Prints one JSON line.

* ``value``: coupled-step MLUPS = all allocated cells x K / wall time of K
  steps run the production way (``ibl_step``: replayed HIP graphs), inputs
  resident in HBM, bracketed by device synchronisation.
* ``roofline``: the dominant kernel (collide-stream) against HBM peak.  Its
  mean duration comes from a second run of K steps launched phase by phase
  with a HIP event after each phase, on the simulation's own stream.
  Algorithmic bytes per cell update: 2 x 19 x (storage bytes).
* ``cpu_baseline``: the FP64 oracle timed on a few steps of the same workload
  on the host cores (and one step on a single thread, ``single_thread``); the
  GPU run of the same steps from the same initial
  state is compared with it (``error_vs_oracle``).
* ``batched``: 64 uneven simulations in one batched launch sequence against
  the same simulations run one after another.
* ``served``: Poisson streams of Jeffery-orbit jobs through the serving loop
  (continuous batching): full-length jobs at the stated rate (rejections,
  capacity) and at a sustainable rate (p50/p99 latency), and shortened jobs
  batched against one job at a time (the plain form).
* ``autotune``: the lattice brick width (16 / 32 / 64 cells) and the
  candidate-list skin (0 / 1 cell) are timed on the workload first
  (``--no-autotune``, or ``--brick-x`` with ``--skin``, to skip).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2}


def lattice_traffic(storage, brick_x, skin):
    """Counter-measured HBM bytes of one collide-stream launch, from the
    committed profiler summary of this workload, if the kernel sources, the
    brick width and the skin are still the ones it was measured with (else
    None)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "k_lattice_rbc_channel_256x128x128_%s_traffic.md" % storage)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_b = re.search(r"^traffic_bytes_k_lattice: (\d+)$", text, re.M)
    m_h = re.search(r"^source_sha256: ([0-9a-f]{64})$", text, re.M)
    m_w = re.search(r"^brick_x: (\d+)$", text, re.M)
    m_s = re.search(r"^skin: (\d+)$", text, re.M)
    if not (m_b and m_h and m_w and m_s) or int(m_w.group(1)) != brick_x or int(m_s.group(1)) != skin:
        return None
    csrc = os.path.join(ROOT, "paper_1704_04551_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read()
                   for f in ("ibl_kernels.hip", "ibl_device.h", "ibl_internal.h"))
    return int(m_b.group(1)) if hashlib.sha256(src).hexdigest() == m_h.group(1) else None


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


def cpu_baseline(spec, steps, storage, single_steps=1):
    """The oracle (FP64, OpenMP over the lattice loops) on `steps` steps of the
    workload, and the GPU's error against it after the same steps."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity_util import field_err, fluid_mask, node_err, oracle_from_spec
    from paper_1704_04551_amd import ibl
    import oracle
    o = oracle_from_spec(spec)
    cores = len(os.sched_getaffinity(0))
    threads = oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", "0")) or cores)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    base = {"value": spec.cells * steps / dt / 1e6, "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": "%d FP64 oracle steps of the same %dx%dx%d workload (%d capsules, %d nodes), "
                      "%.1f s" % (steps, *spec.n, len(spec.capsules), spec.nodes, dt)}
    if single_steps > 0:
        # the same oracle on one thread, on a copy of the workload
        o1 = oracle_from_spec(spec)
        oracle.set_threads(1)
        t0 = time.perf_counter()
        o1.step(single_steps)
        d1 = time.perf_counter() - t0
        oracle.set_threads(threads)
        o1.close()
        base["single_thread"] = {"value": spec.cells * single_steps / d1 / 1e6, "unit": "MLUPS", "cores": 1,
                                 "sample": "%d FP64 oracle step(s) of the same workload on one thread, %.1f s"
                                           % (single_steps, d1)}
    g = ibl.Sim.from_spec(spec, storage=storage)
    g.step(steps)
    g.sync()
    _, ug, _ = g.fields(rho=False, g=False)
    _, uo, _ = o.observe()
    umax, ul2 = field_err(ug, uo, fluid_mask(spec))
    xa, xr = 0.0, 0.0
    for m, c in enumerate(spec.capsules):
        a, r = node_err(g.nodes(m)[0], o.nodes(m)[0], c.x)
        xa, xr = max(xa, a), max(xr, r)
    g.close()
    err = {"after_steps": steps, "u_max_rel": umax, "u_l2_rel": ul2, "x_max_abs_lu": xa,
           "x_max_rel_to_displacement": xr}
    return base, err


def run_batched(storage, steps, skin, plain_form=True):
    """Config of 64 uneven simulations: one batched launch sequence vs the
    same simulations one after another (the plain form, unless plain_form is
    False), at one list skin."""
    import torch
    from paper_1704_04551_amd import ibl
    from paper_1704_04551_amd import workloads as W
    specs = W.config_batched(steps=steps)
    cells = sum(s.cells for s in specs)
    ks = [s.steps for s in specs]
    sims = [ibl.Sim.from_spec(s, storage=storage, skin=skin) for s in specs]
    B = ibl.Batch(sims)
    B.step([1] * len(sims))  # capture the graphs
    for s in sims:
        s.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.step(ks)
    sims[0].sync()
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    if not plain_form:
        B.close()
        for s in sims:
            s.close()
        return {"sims": len(specs), "cells": cells, "steps_each": steps, "skin": skin,
                "nodes": sum(s.nodes for s in specs),
                "batched_mlups": round(cells * steps / tb / 1e6, 1), "batched_s": round(tb, 4)}, []
    plain = [ibl.Sim.from_spec(s, storage=storage, skin=skin) for s in specs]
    for p in plain:
        p.step(1)
        p.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, k in zip(plain, ks):
        p.step(k)
        p.sync()
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    same = all(np.array_equal(a.nodes(m)[0], b.nodes(m)[0])
               for a, b, sp in zip(sims, plain, specs) for m in range(len(sp.capsules)))
    xs = [a.nodes(m)[0] for a, sp in zip(sims, specs) for m in range(len(sp.capsules))]
    B.close()
    for s in sims + plain:
        s.close()
    return {"sims": len(specs), "cells": cells, "steps_each": steps, "skin": skin,
            "nodes": sum(s.nodes for s in specs),
            "batched_mlups": round(cells * steps / tb / 1e6, 1),
            "plain_mlups": round(cells * steps / tp / 1e6, 1),
            "batched_s": round(tb, 4), "plain_s": round(tp, 4), "bitwise_same": bool(same)}, xs


def _serve(storage, jobs, pool, slots, queue_cap, time_limit, skin):
    from paper_1704_04551_amd.serve import GpuBackend, Job, Server
    srv = Server(GpuBackend(storage, skin=skin), pool_bytes=pool, chunk=100, max_resident=slots,
                 queue_cap=queue_cap)
    try:
        st = srv.run([Job(j.jid, j.spec, j.arrival, j.steps) for j in jobs], time_limit=time_limit)
    finally:
        srv.close()
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()}


def run_served(storage, seconds, rate, step_scale, skin, seed=1005):
    """Poisson arrivals of Jeffery-orbit jobs (ellipsoid of 642 nodes, ks
    0.05, AR 1.5-4, cubic lattice 48-128, shear rate 0.005, 2000-20000 steps)
    through the serving loop, `seconds` of arrivals per run:

    * stated: `rate` jobs/s of full-length jobs with a bounded queue (64).
      That is several times more work than one GPU does, so jobs are rejected
      and the rest queue; the run stops at 3 x `seconds`.  Its MLUPS is the
      server's capacity.
    * sustainable: full-length jobs at 0.7 x that capacity / the mean work
      per job, run to completion: the meaningful tail latency.
    * scaled: job lengths x `step_scale` at `rate`: continuous batching
      against the plain form (one job at a time, first come first served) on
      the same arrival stream.
    """
    import torch
    from paper_1704_04551_amd import workloads as W
    from paper_1704_04551_amd.serve import poisson_jobs
    free, total = torch.cuda.mem_get_info()
    pool = int(0.5 * free)
    edges = (48, 64, 80, 96, 112, 128)  # the job generator's lattice edges (uniform)
    mean_work = float(np.mean([e ** 3 for e in edges])) * (2000 + 20000) / 2.0
    out = {"window_s": seconds, "pool_bytes": pool, "skin": skin}
    full = poisson_jobs(rate, seconds, lambda rng: W.job_served(rng, edges=edges), seed)
    out["stated"] = dict(_serve(storage, full, pool, 64, 64, 3 * seconds, skin), rate_jobs_s=rate,
                         jobs=len(full))
    _log("served (stated rate): %s" % out["stated"])
    cap = out["stated"]["mlups"] * 1e6
    rate_s = 0.7 * cap / mean_work
    sus = poisson_jobs(rate_s, seconds, lambda rng: W.job_served(rng, edges=edges), seed + 1)
    out["sustainable"] = dict(_serve(storage, sus, pool, 64, 4096, 10 * seconds, skin),
                              rate_jobs_s=round(rate_s, 3), jobs=len(sus))
    _log("served (sustainable rate): %s" % out["sustainable"])
    lo, hi = max(1, int(2000 * step_scale)), max(1, int(20000 * step_scale))
    short = poisson_jobs(rate, seconds, lambda rng: W.job_served(rng, edges=edges, steps=(lo, hi)), seed)
    out["scaled"] = {"rate_jobs_s": rate, "jobs": len(short), "job_steps": [lo, hi]}
    for name, slots in (("batched", 64), ("plain", 1)):
        out["scaled"][name] = _serve(storage, short, pool, slots, 4096, 3 * seconds, skin)
        _log("served (scaled jobs, %s): %s" % (name, out["scaled"][name]))
    out.update({"p50_s": out["sustainable"]["p50_s"], "p99_s": out["sustainable"]["p99_s"],
                "capacity_mlups": out["stated"]["mlups"]})
    return out


# The paper's red blood cell constants (Sec. 3.2 and the parameter table of
# Sec. 3.5) in lattice units of the 256x128x128 channel, whose 16-cell cells
# are 8 um across: dx = 0.5 um, nu = 1e-6 m^2/s at tau = 0.8 (dt = 2.5e-8 s),
# rho = 1000 kg/m^3, so the force unit is rho dx^4 / dt^2 = 1e-7 N.
#   kBT/p = 1e-12 N on 1320 nodes, scaled by sqrt(2636 / 1280) to keep the
#           shear modulus of Eq. (11) on the 642-node mesh: 1.435e-5;
#   kb = 2.3e-19 J / (1e-7 N x 0.5 um) = 4.6e-6;
#   kg = kl = 2.1e-4 N/m / (1e-7 N / 0.5 um) = 1.05e-3;
#   kv = 2.2 N/m^2 / (1e-7 N / (0.5 um)^2) = 5.5e-6.
FULL_MEMBRANE = (1.435e-5, 1.05e-3, 1.05e-3, 5.5e-6)  # kBT/p, kg, kl, kv
FULL_MEMBRANE_KB = 4.6e-6
# The Morse repulsion of Eq. (13) with the same table's constants, r read in
# um and alpha in 1/um: D0 = 1.2e-18 J / (1e-7 N x 0.5 um) = 2.4e-5;
# alpha = 0.5 / um = 0.25 / lu; r0 = rc = 0.66 um = 1.32 lu.
PAPER_MORSE = (2.4e-5, 0.25, 1.32, 1.32)  # D0, alpha, r0, rc


def run_full_membrane(spec, storage, brick_x, skin, steps, warmup):
    """The same workload with the paper's whole membrane energy and its red
    blood cell constants: WLC-POW stretching in place of the linear springs,
    the dihedral bending, the global / local area and volume constraints, and
    the Morse repulsion between cells.  Graph-replayed steps timed like the
    headline, then a phase-by-phase run."""
    import dataclasses
    from paper_1704_04551_amd import ibl
    caps = [dataclasses.replace(c, ks=0.0, kb=FULL_MEMBRANE_KB, membrane=FULL_MEMBRANE) for c in spec.capsules]
    sp = dataclasses.replace(spec, capsules=caps, morse=PAPER_MORSE)
    sim = ibl.Sim.from_spec(sp, storage=storage, device="cuda:0", brick_x=brick_x, skin=skin)
    try:
        sim.step(warmup)
        sim.sync()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        wall = time.perf_counter() - t0
        phases, _ = sim.profile_phases(steps)
        sim.sync()
        _, _, health = sim.conservation()
    finally:
        sim.close()
    return {"terms": dict(zip(("kbt_p", "kg", "kl", "kv"), FULL_MEMBRANE)), "ks": 0.0, "kb": FULL_MEMBRANE_KB,
            "morse": dict(zip(("D0", "alpha", "r0", "rc"), PAPER_MORSE)),
            "constants": "the paper's red blood cell values in lattice units", "steps": steps,
            "mlups": round(spec.cells * steps / wall / 1e6, 1), "ms_per_step": round(wall * 1e3 / steps, 4),
            "phase_ms": {k: round(v, 5) for k, v in phases.items()}, "health": health}


def tile_spec(spec, reps=(2, 2, 2)):
    from paper_1704_04551_amd import workloads as W
    return W.tiled(spec, reps)


def precision_sweep(args):
    """Config of the precision study: throughput of FP32 vs FP16-offset
    storage on a 512x256x256 channel; FP32 and FP16 errors against the FP64
    oracle on a separate 64^3 channel; steady Poiseuille u_max error per
    storage."""
    import torch
    from paper_1704_04551_amd import ibl
    from paper_1704_04551_amd import workloads as W
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity_util import field_err, fluid_mask, node_err, oracle_from_spec
    out = {"mode": "precision-sweep"}
    # (i) throughput, 512 x 256 x 256 (the seeded 256 x 128 x 128 layout tiled 2 x 2 x 2)
    big = tile_spec(load_spec(args))
    _log("sweep: %s, %d cells, %d nodes" % (big.name, len(big.capsules), big.nodes))
    thr = {}
    for st in ("f32", "f16"):
        sim = ibl.Sim.from_spec(big, storage=st)
        sim.step(10)
        sim.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(args.sweep_steps)
        sim.sync()
        dt = time.perf_counter() - t0
        thr[st] = {"mlups": round(big.cells * args.sweep_steps / dt / 1e6, 1),
                   "ms_per_step": round(dt * 1e3 / args.sweep_steps, 4), "health": sim.conservation()[2]}
        _log("sweep: %s %s" % (st, thr[st]))
        sim.close()
        del sim
        torch.cuda.empty_cache()
    out["throughput_512x256x256"] = {"workload": big.name, "cells": big.cells, "capsules": len(big.capsules),
                                     "nodes": big.nodes, "steps": args.sweep_steps, **thr}
    # (ii) 64^3 channel of the same physics vs the FP64 oracle
    crop = W.config_rbc_channel(n=(64, 64, 64), count=200, seed=1003)
    k = args.sweep_crop_steps
    _log("sweep: crop %d cells, %d nodes, %d steps" % (len(crop.capsules), crop.nodes, k))
    o = oracle_from_spec(crop)
    t0 = time.perf_counter()
    for i in range(0, k, 100):
        o.step(min(100, k - i))
        _log("sweep: oracle step %d" % min(k, i + 100))
    tor = time.perf_counter() - t0
    _, uo, _ = o.observe()
    mask = fluid_mask(crop)
    errs = {}
    for st in ("f64", "f32", "f16"):
        g = ibl.Sim.from_spec(crop, storage=st)
        g.step(k)
        g.sync()
        _, ug, _ = g.fields(rho=False, g=False)
        umax, ul2 = field_err(ug, uo, mask)
        xa = xr = 0.0
        for m, c in enumerate(crop.capsules):
            a, r = node_err(g.nodes(m)[0], o.nodes(m)[0], c.x)
            xa, xr = max(xa, a), max(xr, r)
        errs[st] = {"u_max_rel": umax, "u_l2_rel": ul2, "x_max_abs_lu": xa, "x_max_rel_to_displacement": xr}
        _log("sweep: crop %s %s" % (st, errs[st]))
        g.close()
    out["crop_64_vs_fp64_oracle"] = {"cells": crop.cells, "capsules": len(crop.capsules), "nodes": crop.nodes,
                                     "steps": k, "oracle_s": round(tor, 1), **errs}
    # (iii) plane Poiseuille 64 x 64 x 256 (walls on x, flow along z) at steady state
    pz = W.config_poiseuille()
    nu = (pz.tau - 0.5) / 3.0
    lam = (pz.tau - 0.5) ** 2
    nw = pz.n[0]
    zc = np.arange(nw, dtype=float)
    exact = pz.g_body[2] / (2 * nu) * (zc - 0.5) * (nw - 1.5 - zc) + pz.g_body[2] / nu * (2 * lam / 3 - 0.125)
    umax_exact = exact[1:-1].max()
    pois = {}
    for st in ("f64", "f32", "f16"):
        g = ibl.Sim.from_spec(pz, storage=st)
        g.step(args.sweep_poiseuille_steps)
        g.sync()
        _, ug, _ = g.fields(rho=False, g=False)
        pois[st] = {"u_max": float(ug[2].max()), "u_max_rel_err": float(abs(ug[2].max() - umax_exact) / umax_exact)}
        _log("sweep: poiseuille %s %s" % (st, pois[st]))
        g.close()
    out["poiseuille_64x64x256"] = {"steps": args.sweep_poiseuille_steps, "u_max_exact": umax_exact, **pois}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "f64"])
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--cpu-single-steps", type=int, default=1, help="oracle steps of the one-thread leg")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-capsules", action="store_true",
                    help="the lattice of the workload without its capsules (profiling aid)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the built-in brick width and no skin (or --brick-x / --skin)")
    ap.add_argument("--brick-x", type=int, default=0, choices=[0, 16, 32, 64],
                    help="fixed brick width (skips the autotuner)")
    ap.add_argument("--skin", type=int, default=None, choices=[0, 1],
                    help="fixed candidate-list skin (skips the autotuner)")
    ap.add_argument("--batched-steps", type=int, default=500)
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the 64-simulation batched workload, without its plain form "
                         "(its own JSON line; a profiling aid)")
    ap.add_argument("--membrane-steps", type=int, default=300, help="0 skips the full-membrane run")
    ap.add_argument("--serve-seconds", type=float, default=15.0, help="0 skips the served runs")
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-step-scale", type=float, default=0.1)
    ap.add_argument("--serve-skin", type=int, default=1, choices=[0, 1],
                    help="candidate-list skin of the served jobs")
    ap.add_argument("--cache", default=os.path.join(tempfile.gettempdir(), "ibl_rbc_channel_spec.npz"),
                    help="cache of the generated RBC node arrays ('' disables)")
    ap.add_argument("--precision-sweep", action="store_true",
                    help="only run the precision study (its own JSON line; several minutes)")
    ap.add_argument("--sweep-steps", type=int, default=100)
    ap.add_argument("--sweep-crop-steps", type=int, default=1000)
    ap.add_argument("--sweep-poiseuille-steps", type=int, default=150000)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB, 5 times "
                         "(calibrates the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.copy_probe:
        # the library's plain streaming copy kernel: the practical HBM ceiling
        # (read + written bytes over the mean launch time, HIP events on
        # torch's stream, the one the copy is launched on) and the calibration
        # of a profiler's byte counters
        import torch
        from paper_1704_04551_amd import ibl
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            ibl.hbm_copy(src, dst)
        torch.cuda.synchronize()
        reps = 20
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record()
        for i in range(reps):
            ibl.hbm_copy(src, dst)
            ev[i + 1].record()
        torch.cuda.synchronize()
        ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]
        assert bool(torch.equal(src, dst))
        ms_mean = sum(ms) / reps
        # torch's own device copy, for comparison
        dst.zero_()
        ev[0].record()
        for i in range(reps):
            dst.copy_(src)
            ev[i + 1].record()
        torch.cuda.synchronize()
        tms = [ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "launches": reps + 3,
                          "ms_mean": round(ms_mean, 5), "ms_min": round(min(ms), 5),
                          "gbps_mean": round(8 * n / ms_mean / 1e6, 1),
                          "gbps_best": round(8 * n / min(ms) / 1e6, 1),
                          "torch_copy_gbps_mean": round(8 * n * reps / sum(tms) / 1e6, 1)}))
        return
    if args.precision_sweep:
        precision_sweep(args)
        return
    if args.batched_only:
        # the batched workload alone, at one skin (a profiling aid)
        r, _ = run_batched(args.storage, args.batched_steps, args.skin or 0, plain_form=False)
        print(json.dumps(r), flush=True)
        return
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; --gpus %d is not supported "
              "(the multi-GPU slab decomposition is a design, not built)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1704_04551_amd import ibl

    _log("generating workload")
    spec = load_spec(args)
    if args.no_capsules:
        # the same lattice without its capsules: collide-stream alone (a
        # profiling aid for the lattice kernel, not the workload's figure)
        import dataclasses
        spec = dataclasses.replace(spec, capsules=[], name=spec.name + "-no-capsules")
    tuned = None
    brick_x, skin = args.brick_x, args.skin
    if not brick_x and skin is None and not args.no_autotune:
        from paper_1704_04551_amd.autotune import shape_key, tune
        _log("autotuning the brick width and list skin")
        (brick_x, skin), timings = tune(spec, args.storage, steps=30, warmup=5, use_memo=False)
        tuned = {"brick_x": brick_x, "skin": skin,
                 "ms_per_step": {shape_key(k): round(v, 4) for k, v in timings.items()}}
        _log("autotune: %s" % tuned)
    skin = skin or 0
    _log("%d cells, %d nodes; creating simulation" % (len(spec.capsules), spec.nodes))
    sim = ibl.Sim.from_spec(spec, storage=args.storage, device="cuda:0", brick_x=brick_x, skin=skin)
    sim.step(args.warmup)
    sim.sync()
    _log("warmup done")

    # timed region: K steps the production way (replayed HIP graphs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _log("timed %d steps: %.4f s" % (args.steps, wall))

    # the same number of steps phase by phase, HIP events on the sim's stream
    phases, total_ms = sim.profile_phases(args.steps)
    sim.sync()
    mass, mom, health = sim.conservation()
    _log("phase run: %.4f ms/step; %s" % (total_ms / args.steps, phases))

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
        "dtype": {"f32": "f32", "f16": "f32", "f64": "f64"}[args.storage],  # arithmetic; storage in config
        "data": "synthetic (seeded RSA of Evans-Fung cells)",
        "config": {"workload": spec.name, "cells": cells, "capsules": len(spec.capsules),
                   "nodes": spec.nodes, "tau": spec.tau, "g_body": spec.g_body[0],
                   "storage": args.storage, "delta": spec.delta},
        "roofline": {"bound": "hbm", "kernel": "k_lattice (collide-stream)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": lattice_traffic(args.storage, brick_x or 64, skin),
                     "bytes_per_launch": lat_bytes, "launch_ms": round(lat_ms, 5)},
        "step_roofline_frac": round(cells * 2 * 19 * sb / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "phase_ms": {k: round(v, 5) for k, v in phases.items()},
        "brick_x": brick_x or None,
        "skin": skin,
        "autotune": tuned,
        "health": health,
    }
    sim.close()
    if args.membrane_steps > 0:
        _log("full membrane: %d steps" % args.membrane_steps)
        fm = run_full_membrane(spec, args.storage, brick_x, skin, args.membrane_steps, min(args.warmup, 20))
        fm["membrane_kernel_ms"] = round(fm["phase_ms"]["forces"] - result["phase_ms"]["forces"], 5)
        result["full_membrane"] = fm
        _log("full membrane: %s" % fm)
    if not args.no_cpu:
        _log("cpu baseline (oracle, %d steps, then %d on one thread)" % (args.cpu_steps, args.cpu_single_steps))
        result["cpu_baseline"], result["error_vs_oracle"] = cpu_baseline(spec, args.cpu_steps, args.storage,
                                                                         args.cpu_single_steps)
    if not args.no_batched:
        _log("batched: 64 uneven simulations, %d steps" % args.batched_steps)
        runs = {k: run_batched(args.storage, args.batched_steps, k) for k in (0, 1)}
        best = max(runs, key=lambda k: runs[k][0]["batched_mlups"])
        result["batched"] = dict(runs[best][0])
        result["batched"]["other_skin"] = {k: runs[1 - best][0][k] for k in ("skin", "batched_mlups", "plain_mlups")}
        result["batched"]["skins_bitwise_same"] = all(np.array_equal(a, b) for a, b in zip(runs[0][1], runs[1][1]))
        _log("batched: %s" % result["batched"])
    if args.serve_seconds > 0:
        _log("served: %.0f s of arrivals at %.1f jobs/s" % (args.serve_seconds, args.serve_rate))
        result["served"] = run_served(args.storage, args.serve_seconds, args.serve_rate,
                                      args.serve_step_scale, args.serve_skin)
        _log("served: %s" % result["served"])
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

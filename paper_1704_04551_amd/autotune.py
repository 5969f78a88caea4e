"""Autotuner of the lattice brick shape.

The collide-stream kernel processes the lattice in bricks of
``brick_x x (256 / brick_x) x 4`` cells, one workgroup each, and spreads the
brick's candidate nodes into LDS first.  The best width depends on the
lattice shape (long x rows keep the streaming accesses in whole cache lines;
short ones leave lanes idle) and on the node density (the candidate region
of a brick is (brick_x + 3) x (256 / brick_x + 3) x 7 cells).  The tuner
times every width on the actual workload and keeps the fastest.

Results of different widths agree to the spreading's fixed-point resolution
(the per-brick scale depends on which nodes share a brick), not bitwise; a
tuned width is a property of the simulation, chosen once before it runs.
"""
from __future__ import annotations

import time
from typing import Callable, Dict, Optional, Sequence, Tuple

WIDTHS = (64, 32, 16)
_memo: Dict[tuple, int] = {}


def default_width(nx: int) -> int:
    """The library's built-in choice (descriptor brick_x = 0)."""
    return 64 if nx >= 64 else (32 if nx >= 32 else 16)


def pick(timings: Dict[int, float], nx: int, tolerance: float = 0.02) -> int:
    """Fastest width; widths within `tolerance` of the fastest count as ties,
    resolved toward the built-in default, then the wider brick."""
    best = min(timings.values())
    close = [w for w, t in timings.items() if t <= best * (1.0 + tolerance)]
    d = default_width(nx)
    return d if d in close else max(close)


def gpu_runner(spec, storage: str, steps: int, warmup: int, device=None) -> Callable[[int], float]:
    """ms per step of `spec` at a brick width: build, warm up (captures the
    step graphs), then time `steps` graph-replayed steps with HIP events on
    the simulation's stream."""
    def run(width: int) -> float:
        import torch
        from . import ibl
        sim = ibl.Sim.from_spec(spec, storage=storage, device=device, brick_x=width)
        try:
            sim.step(warmup)
            sim.sync()
            ext = torch.cuda.ExternalStream(sim.stream_handle)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(ext)
            sim.step(steps)
            e1.record(ext)
            sim.sync()
            return e0.elapsed_time(e1) / steps
        finally:
            sim.close()
    return run


def tune_brick_x(spec, storage: str = "f32", steps: int = 50, warmup: int = 10,
                 widths: Sequence[int] = WIDTHS, runner: Optional[Callable[[int], float]] = None,
                 use_memo: bool = True) -> Tuple[int, Dict[int, float]]:
    """Time every width in `widths` on `spec` and return (best width,
    {width: ms per step}).  Results are remembered per (lattice shape, walls,
    storage, node count) unless use_memo is False."""
    key = (tuple(spec.n), tuple(spec.wall), storage, spec.nodes)
    if use_memo and key in _memo:
        return _memo[key], {}
    run = runner if runner is not None else gpu_runner(spec, storage, steps, warmup)
    timings = {int(w): float(run(int(w))) for w in widths}
    best = pick(timings, spec.n[0])
    if use_memo:
        _memo[key] = best
    return best, timings


def _main():
    import argparse
    import json
    from . import workloads as W
    ap = argparse.ArgumentParser(description="time the lattice brick widths on a workload")
    ap.add_argument("--workload", default="small", choices=["small", "rbc-channel", "poiseuille"])
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "f64"])
    ap.add_argument("--steps", type=int, default=50)
    args = ap.parse_args()
    spec = {"small": W.config_small, "rbc-channel": W.config_rbc_channel,
            "poiseuille": W.config_poiseuille}[args.workload]()
    t0 = time.perf_counter()
    best, timings = tune_brick_x(spec, args.storage, steps=args.steps, use_memo=False)
    print(json.dumps({"workload": spec.name, "storage": args.storage, "best_brick_x": best,
                      "ms_per_step": timings, "tuning_s": round(time.perf_counter() - t0, 2)}))


if __name__ == "__main__":
    _main()

"""Launch autotuner: times batched calls of a plan over a grid of launch
tunings (workgroup-shape threshold, frame groups, critical group and its
workgroup shape; see
fse_plan_set_tuning in include/fse.h) on the caller's own frames, and leaves
the fastest one set on the plan.  Tuning changes how the work is laid on the
GPU, not what is computed (results stay within the per-shape rounding).

Usage: python -m paper_2207_00233_amd.autotune [--precision fp32_rerank]
runs the grid on the 64-frame benchmark batch with device-resident frames and
prints one JSON object (the best tuning, the default's time, every result).
"""
from __future__ import annotations

import argparse
import itertools
import json
import sys
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

DEFAULT_GRID: Dict[str, Sequence] = {
    "wave_threshold_16": (128, 256, 512),
    "frame_groups": (1, 2, 3, 4),
    "crit_depth": (0.0, 0.75, 0.9),
    "crit_waves": (0, 4),
}


def time_calls(run: Callable[[], object], warmup: int, reps: int) -> float:
    """Milliseconds per call of ``run`` (a synchronous batched call)."""
    for _ in range(warmup):
        run()
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    return (time.perf_counter() - t0) / reps * 1e3


def autotune(plan, run: Callable[[], object], grid: Optional[Dict[str, Sequence]] = None,
             warmup: int = 1, reps: int = 3,
             log: Optional[Callable[[dict, float], None]] = None
             ) -> Tuple[dict, List[Tuple[dict, float]]]:
    """Time ``run`` (one synchronous batched call on ``plan``) for every
    combination of ``grid`` (keys of fse_tuning; the other fields keep the
    plan's values) and set the fastest on the plan.  ``log`` sees each
    (tuning, ms) as it is measured.  Returns (best tuning, [(tuning, ms per
    call), ...])."""
    grid = DEFAULT_GRID if grid is None else grid
    base = plan.get_tuning()
    keys = list(grid)
    results, seen = [], set()
    for vals in itertools.product(*(grid[k] for k in keys)):
        t = dict(base)
        t.update(zip(keys, vals))
        # with one group, or crit_depth 0, there is no critical group: such
        # tunings coincide whatever their critical-group fields
        crit = t["frame_groups"] > 1 and t["crit_depth"] > 0.0
        key = (t["wave_threshold_16"], t["wave_threshold_8"], t["frame_groups"],
               t["crit_depth"] if crit else 0.0, t["crit_prio"] if crit else 0,
               t["crit_waves"] if crit else 0)
        if key in seen:
            continue
        seen.add(key)
        plan.set_tuning(**t)
        results.append((plan.get_tuning(), time_calls(run, warmup, reps)))
        if log is not None:
            log(*results[-1])
    best = min(results, key=lambda r: r[1])[0]
    plan.set_tuning(**best)
    return best, results


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--precision", choices=("fp32", "fp32_rerank", "fp32_f16x3", "fp64"),
                    default="fp32_rerank")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)
    import torch

    import paper_2207_00233_amd as fse
    from paper_2207_00233_amd import synth

    prec = {"fp32": fse.FSE_FP32, "fp32_rerank": fse.FSE_FP32_RERANK,
            "fp32_f16x3": fse.FSE_FP32_F16X3, "fp64": fse.FSE_FP64}[args.precision]
    frames = synth.config3(seed=args.seed)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    imgs = [torch.from_numpy(f.image).to(dev) for f in frames]
    losts = [torch.from_numpy(f.lost).to(dev) for f in frames]
    outs = [torch.empty_like(t) for t in imgs]
    torch.cuda.synchronize()
    descs = [{"image": i.data_ptr(), "lost": l.data_ptr(), "out": o.data_ptr(),
              "width": i.shape[1], "height": i.shape[0]} for i, l, o in zip(imgs, losts, outs)]
    p = fse.Params(border_d=14, iterations=200, precision=prec, flags=fse.FSE_FLAG_DEVICE_PTRS)
    with fse.Plan(p, hip_stream=torch.cuda.current_stream().cuda_stream) as plan:
        def run():
            plan.conceal_device(descs)
        default = plan.get_tuning()
        default_ms = time_calls(run, 1, args.reps)
        print(f"[autotune] default {default}: {default_ms:.2f} ms per batch", file=sys.stderr,
              flush=True)
        best, results = autotune(
            plan, run, reps=args.reps,
            log=lambda t, ms: print(f"[autotune] {t}: {ms:.2f} ms", file=sys.stderr, flush=True))
    best_ms = min(ms for _, ms in results)
    print(json.dumps({"precision": args.precision, "best": best, "best_ms": best_ms,
                      "default": default, "default_ms": default_ms,
                      "results": [{"tuning": t, "ms": ms} for t, ms in results]}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

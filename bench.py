#!/usr/bin/env python3
"""Throughput of the rational-program hot path on one MI355X.

One step = one pass of the hot path over one batch of synthetic input resident in HBM:
  eval : 1024 rational programs (8 fitted degree-2 metrics each, in N, bx, by), 65536 data-size
         queries each, 128 launch configurations: collapse + evaluation + per-query argmin
         (8.59e9 (query, configuration) points).

Prints ONE JSON line (metric, value = launch-configuration evaluations per second over the
whole step, roofline of the dominant kernel, CPU-baseline of the oracle on a bounded sample).
Everything else goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rational fits/s + launch-config evals/s; surrogate vs plain at <=1% cost error"
# MI355X: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz = 39.32 T lane-operations/s for
# unpacked VALU instructions (packed FP32 is disabled in every kernel of this library).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def eval_ops_per_point(degree: int) -> int:
    """Operations of the normative FP32 sequence per (query, configuration) point, each IEEE
    add / mul / div / compare / select / conversion and each integer op counted once.

    per metric (8): scale 1, Horner 4*degree, q > 0 1, divide 1, finiteness 1, clean 1, and 1
    clamps 14, occupancy 13, grid and repetitions 14, cycle estimate 49, argmin update 3,
    data-size conversion 1."""
    return 8 * (6 + 4 * degree) + 14 + 13 + 14 + 49 + 3 + 1


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(pb, budget_s: float):
    """The oracle's FP32 replay + brute-force argmin, timed on a bounded sample of the same
    workload: whole programs' first 16384 queries x all 128 configurations, one program after
    another until the time budget is spent."""
    import numpy as np
    from oracle import cost as oc
    points, t0, progs = 0, time.perf_counter(), 0
    nq = min(16384, int(pb.n_q[0]))
    while time.perf_counter() - t0 < budget_s and progs < pb.n_progs:
        c = oc.program_costs(pb, progs, query_idx=np.arange(nq))
        oc.argmin_lowest(c)
        points += c.size
        progs += 1
    dt = time.perf_counter() - t0
    return {"value": points / dt, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{progs} programs x {nq} queries x {int(pb.n_cfg[0])} configs "
                      f"({points} points, {dt:.1f} s, numpy FP32 replay + argmin, 1 thread)"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--cpu-budget-s", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_1911_02373_amd import klr, synth

    lib = klr.Library.get()
    t = time.perf_counter()
    pb = synth.config3_programs(args.seed, n_progs=1024, n_q=65536)
    de = klr.DeviceEval.from_batch(lib, pb)
    out = (torch.empty(de.queries.numel(), dtype=torch.int32, device="cuda"),
           torch.empty(de.queries.numel(), dtype=torch.float32, device="cuda"), None,
           torch.empty(de.n_progs, dtype=torch.int32, device="cuda"))
    points = int((pb.n_cfg.astype(np.int64) * pb.n_q).sum())
    log(f"workload ready in {time.perf_counter() - t:.1f} s: {pb.n_progs} programs, {points:.3e} points")

    def step():
        lib.eval_argmin(de, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lib.profile_enable(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    eval_ms, n_eval = lib.profile_read(klr.K_EVAL)
    coll_ms, n_coll = lib.profile_read(klr.K_COLLAPSE)
    lib.profile_enable(False)
    st = out[3].cpu().numpy()
    if not np.all(st == 0):
        log("program status nonzero:", np.unique(st))
        return 1
    eval_avg = eval_ms / max(n_eval, 1)
    ops = eval_ops_per_point(2)
    achieved = ops * points / (eval_avg / 1e3) / 1e12
    log(f"step {ms:.3f} ms; eval kernel {eval_avg:.3f} ms x {n_eval}; collapse {coll_ms / max(n_coll, 1):.3f} ms")

    res = {
        "metric": METRIC,
        "value": points / (ms / 1e3),
        "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded)",
        "config": {"workload": "eval/argmin: 1024 rational programs x 65536 queries x 128 launch "
                               "configs, 8 degree-2 fitted metrics each, MWP-CWP-style cycle estimate",
                   "programs": int(pb.n_progs), "queries_per_program": 65536, "configs": 128,
                   "points": points},
        "components": {"eval_kernel_ms": eval_avg, "collapse_kernel_ms": coll_ms / max(n_coll, 1)},
        "roofline": {"bound": "alu", "kernel": "eval_kernel", "achieved": achieved,
                     "peak": VALU_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS,
                     "ops_per_point": ops, "traffic": None},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(pb, args.cpu_budget_s)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

#!/usr/bin/env python3
"""Throughput of the rational-program hot path on one MI355X.

One step = one pass of the hot path over one batch of synthetic input resident in HBM:
  fit  : 4096 independent rational fits of uneven sample counts (m ~ U[64, 512]) over
         (N, bx, by), numerator and denominator of total degree <= 3 (39 unknowns), literal
         domain (bx, by multiples of 16, bx*by <= 1024), FP64 Gram + pivoted Cholesky + FP64
         residual refinement to ||A (y - y*)|| <= 1e-10 ||f||;
  eval : 1024 rational programs (8 fitted degree-2 metrics each, in N, bx, by), 65536 data-size
         queries each, 128 launch configurations: collapse + evaluation + per-query argmin
         (8.59e9 (query, configuration) points).
The reduced-precision Gram paths (FP32, BF16 inputs with FP32 accumulation, same FP64
refinement) are timed on the same fit batch outside the step, as the comparison the
precision change is judged by.

Prints ONE JSON line: value = launch-configuration evaluations per second over the whole step;
fits/s per precision under "components"; roofline of the dominant kernel (the evaluation
sweep); CPU baseline = the oracle timed on bounded samples of the same step, scaled to the step.
Everything else goes to stderr.
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

METRIC = "rational fits/s + launch-config evals/s; surrogate vs plain at <=1% cost error"
# MI355X peaks (published): FP32 vector 157.3 TFLOP/s counts packed FP32 (two lanes' worth per
# instruction); this library builds every kernel with packed FP32 disabled, so its own ceiling
# is half of it: 256 CUs x 64 lanes x 2 flop (FMA) x 2.4 GHz = 78.6 TFLOP/s.  FP64 78.6.
FP32_PEAK_TFLOPS = 157.3
FP32_UNPACKED_TFLOPS = 78.6
FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0
VALU_LANE_OPS_T = 256 * 64 * 2.4e9 / 1e12     # unpacked VALU lane-instructions per second, 1e12
FIT_TOL = {0: 1e-10, 1: 1e-8, 2: 1e-8, 3: 0.0}
FIT_MAX_ITER = 256
N_METRICS = 8


def eval_flops_per_point(degree: int) -> int:
    """FP32 arithmetic of the normative cycle-estimate sequence per (query, configuration)
    point, fused multiply-add = 2, add / sub / mul / div = 1 (compares, selects, min / max,
    conversions and integer steps are not counted): per metric 2 degree fused multiply-adds for
    p and q and one division (8 (4 degree + 1)); occupancy and repetitions 5 (two exact
    quotients, the resident-wave product, the repetition quotient and its + 1); cycle estimate
    37 (I_m 1, L_u 3, mem 3, comp 2, MWP_lat 4, MWP_bw 3, tot 1, the two CWP products 2, comp/I_m
    1, MWP - 1 1, the three case values 2 + 3 + 2, the pure-compute product 1, the
    synchronisation term 5, the final fused multiply-add 2).  Degree 2: 114."""
    return N_METRICS * (4 * degree + 1) + 5 + 37


def eval_ops_per_point(degree: int) -> int:
    """Every operation of the normative sequence counted once (IEEE add / mul / fused
    multiply-add / div / compare / select / conversion and each integer op): a count of issued
    lane-operations, reported as a diagnostic beside the FP32 flop roofline."""
    return 8 * (6 + 2 * degree) + 14 + 13 + 14 + 43 + 3 + 1


def fit_flops(m, n, iters):
    """Algorithmic FP64 flops of one fit: Gram m n (n + 1) (symmetric, with A^T f), Cholesky
    n^3 / 3, refinement per iteration 4 m n (A t and A^T r) + 4 n^2 (two triangular solves),
    initial residual and A^T r 4 m n + 2 n^2."""
    return m * n * (n + 1) + n ** 3 / 3 + (iters + 1) * (4 * m * n + 4 * n * n)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "eval_kernel_hbm_traffic.md")
EVAL_SOURCES = [os.path.join(ROOT, "paper_1911_02373_amd", "csrc", f) for f in ("eval.hip", "eval_point.hpp")]


def measured_traffic():
    """HBM bytes per launch of the evaluation kernel from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, each divided by what the same counter reads
    for a plain device copy of known size), or None when the kernel source changed since the
    counters were taken or no summary exists (the digest covers eval.hip and eval_point.hpp, in
    that order)."""
    import hashlib
    try:
        with open(TRAFFIC_PROFILE) as f:
            lines = f.read().splitlines()
        h = hashlib.sha256()
        for src in EVAL_SOURCES:
            with open(src, "rb") as f:
                h.update(f.read())
        digest = h.hexdigest()
    except OSError:
        return None
    kv = {}
    for ln in lines:
        if ln.startswith("- ") and ": " in ln:
            k, v = ln[2:].split(": ", 1)
            kv[k.strip()] = v.strip().strip("`")
    try:
        if kv.get("eval sources sha256") != digest:
            return None
        fetch = float(kv["FETCH_SIZE KiB per launch"]) / float(kv["FETCH_SIZE copy factor"])
        write = float(kv["WRITE_SIZE KiB per launch"]) / float(kv["WRITE_SIZE copy factor"])
    except (KeyError, ValueError, ZeroDivisionError):
        return None
    return (fetch + write) * 1024.0


# Surrogate training: 16384 samples per Adam step (one 64-sample tile per CU), peak learning rate
# 6e-3 with the cosine schedule; 300 epochs over the 4.2 M samples.
SURR_BATCH = 16384
SURR_LR = 6e-3
SURR_SHORTLIST = 4            # the library default: the network's 4 best predictions re-ranked exactly
LARGE_SURR_QUERIES = 12       # training queries per program of the large batch


def surrogate_component(lib, klr, synth, pb, de, exact_ms, seed, epochs, regret_programs=64):
    """Learned surrogate beside the exact path on the same grid: train on 4.2M samples the
    exact program generates (32 queries x 128 configurations per program), select over the
    full query grid with the 2 % margin fallback, and judge the picks with the exact costs of
    `regret_programs` programs."""
    import numpy as np
    import torch
    tq = synth.surrogate_training_queries(seed + 1, pb, n_q=32)
    de_t = klr.DeviceEval.from_batch(lib, tq, with_costs=True)
    _, _, costs, _ = lib.eval_argmin(de_t, want_costs=True)
    kid, N, L, cost = klr.grid_samples(tq, de_t, costs)
    blob = lib.surrogate_alloc(synth.mlp_init(seed, pb.n_progs), pb.n_progs)
    torch.cuda.synchronize()
    lib.profile_enable(True)
    loss = lib.surrogate_train(blob, pb.n_progs, kid, N, L, cost, lr=SURR_LR, batch=SURR_BATCH, epochs=epochs,
                               seed=seed)
    train_ms, _ = lib.profile_read(klr.K_MLP)
    lib.profile_enable(False)
    del de_t, costs, kid, N, L, cost
    out = lib.surrogate_eval(blob, pb.n_progs, de, margin=0.02)       # warm-up
    torch.cuda.synchronize()
    lib.profile_enable(True)
    am, pc, fb = lib.surrogate_eval(blob, pb.n_progs, de, margin=0.02, out=out)
    sel_ms, _ = lib.profile_read(klr.K_SURR)
    fb_ms, _ = lib.profile_read(klr.K_FALLBACK)
    col_ms, _ = lib.profile_read(klr.K_COLLAPSE)
    lib.profile_enable(False)
    fbr = float(fb.float().mean().cpu())
    sub = regret_programs
    nq = int(pb.n_q[0])
    dex = klr.DeviceEval.from_batch(lib, synth.take_programs(pb, sub), with_costs=True)
    xa, xb, xc, _ = lib.eval_argmin(dex, want_costs=True)
    C = xc.view(sub, int(pb.n_cfg[0]), nq)
    ok = xa >= 0

    def regret(a):
        picked = torch.gather(C, 1, a[: sub * nq].view(sub, 1, nq).long().clamp(min=0)).view(-1).double()
        return (picked[ok] / xb.double()[ok] - 1.0).cpu().numpy()
    r = regret(am)
    am0, _, _ = lib.surrogate_eval(blob, pb.n_progs, dex, margin=0.0)
    r0 = regret(am0)
    lib.set_option(klr.OPT_SURR_SHORTLIST, 1)              # the network's own picks, same rule
    try:
        am1, _, fb1 = lib.surrogate_eval(blob, pb.n_progs, dex, margin=0.02)
        am10, _, _ = lib.surrogate_eval(blob, pb.n_progs, dex, margin=0.0)
    finally:
        lib.set_option(klr.OPT_SURR_SHORTLIST, SURR_SHORTLIST)
    r1, r10 = regret(am1), regret(am10)
    torch.cuda.synchronize()
    nonfb = ~fb[: sub * nq][ok].cpu().numpy().astype(bool)
    total_ms = sel_ms + fb_ms + col_ms
    picks = am[: sub * nq].cpu().numpy()

    def stats(x):
        return {"frac_le_1pct": float(np.mean(x <= 0.01)), "p50": float(np.median(x)),
                "p99": float(np.quantile(x, 0.99)), "max": float(x.max())}
    return {"_picks": picks, "shortlist": SURR_SHORTLIST,
            "train_ms": train_ms, "epochs": epochs, "batch": SURR_BATCH, "lr": SURR_LR,
            "train_samples": int(tq.n_progs * 32 * 128),
            "final_loss_std": float(loss[-1].cpu()), "select_ms": sel_ms, "fallback_ms": fb_ms,
            "collapse_ms": col_ms, "fallback_rate": fbr, "margin": 0.02,
            "speedup_vs_exact": exact_ms / total_ms,
            "regret_programs": sub,
            "regret_with_fallback": {"frac_le_1pct": float(np.mean(r <= 0.01)), "p50": float(np.median(r)),
                                     "p99": float(np.quantile(r, 0.99)), "max": float(r.max()),
                                     "nonfallback_frac_le_1pct": float(np.mean(r[nonfb] <= 0.01)) if nonfb.any() else None},
            "regret_surrogate_alone": stats(r0),
            "regret_shortlist_1_with_fallback": stats(r1),
            "fallback_rate_shortlist_1": float(fb1[: sub * nq].float().mean().cpu()),
            "regret_shortlist_1_alone": stats(r10)}


def large_surrogate(lib, klr, synth, pb, coef, seed, epochs, regret_programs=64):
    """The surrogate beside the exact path on the large batch's programs with two launch
    parameters (the network's inputs are N and one launch pair): trained on samples that the
    fitted programs generate (12 fresh queries x every configuration per program), then selection
    with the 2 % fallback over the programs' full query sets, the exact evaluation of the same
    programs timed beside it, and the picks of `regret_programs` programs judged by exact costs."""
    import numpy as np
    import torch
    idx = np.nonzero(pb.v_launch == 2)[0]
    sub = synth.select_programs(pb, idx)
    nk = sub.n_progs
    tq = synth.surrogate_training_queries(seed + 3, sub, n_q=LARGE_SURR_QUERIES)
    de_t = klr.DeviceEval.from_batch(lib, tq, with_costs=True, coef=coef)
    _, _, costs, _ = lib.eval_argmin(de_t, want_costs=True)
    kid, N, L, cost = klr.program_samples(tq, de_t, costs)
    n_samples = int(kid.numel())
    blob = lib.surrogate_alloc(synth.mlp_init(seed, nk), nk)
    torch.cuda.synchronize()
    lib.profile_enable(True)
    lib.surrogate_train(blob, nk, kid, N, L, cost, lr=SURR_LR, batch=SURR_BATCH, epochs=epochs, seed=seed)
    train_ms, _ = lib.profile_read(klr.K_MLP)
    lib.profile_enable(False)
    del de_t, costs, kid, N, L, cost
    de = klr.DeviceEval.from_batch(lib, sub, coef=coef)
    points = int((sub.n_cfg.astype(np.int64) * sub.n_q).sum())
    ex = lib.eval_argmin(de)                                     # tunes the shape for this set
    out = lib.surrogate_eval(blob, nk, de, margin=0.02)         # warm-up
    torch.cuda.synchronize()
    lib.profile_enable(True)
    lib.eval_argmin(de, out=ex)
    exact_ms, _ = lib.profile_read(klr.K_EVAL)
    exact_col, _ = lib.profile_read(klr.K_COLLAPSE)
    lib.profile_enable(False)
    lib.profile_enable(True)
    am, _, fb = lib.surrogate_eval(blob, nk, de, margin=0.02, out=out)
    sel_ms, _ = lib.profile_read(klr.K_SURR)
    fb_ms, _ = lib.profile_read(klr.K_FALLBACK)
    col_ms, _ = lib.profile_read(klr.K_COLLAPSE)
    lib.profile_enable(False)
    # outputs are indexed by global query position; the subset's queries are its programs' ranges
    qpos = np.concatenate([np.arange(int(sub.q0[p]), int(sub.q0[p]) + int(sub.n_q[p])) for p in range(nk)])
    fbr = float(fb[torch.from_numpy(qpos).to(fb.device)].float().mean().cpu())
    # exact costs of the first programs, per program [n_cfg][n_q] at the program_descs offsets
    rsub = synth.select_programs(sub, np.arange(min(regret_programs, nk)))
    dr = klr.DeviceEval.from_batch(lib, rsub, with_costs=True, coef=coef)
    xa, xb, xc, _ = lib.eval_argmin(dr, want_costs=True)
    ra, _, rf = lib.surrogate_eval(blob, nk, dr, margin=0.02)
    torch.cuda.synchronize()
    xa, xb, xc = xa.cpu().numpy(), xb.cpu().numpy(), xc.cpu().numpy()
    ra, rf = ra.cpu().numpy(), rf.cpu().numpy().astype(bool)
    regrets, nonfb = [], []
    co = 0
    for p in range(rsub.n_progs):
        nc, nq, qo = int(rsub.n_cfg[p]), int(rsub.n_q[p]), int(rsub.q0[p])
        C = xc[co: co + nc * nq].reshape(nc, nq)
        for q in range(nq):
            if xa[qo + q] >= 0 and ra[qo + q] >= 0:
                regrets.append(C[ra[qo + q], q] / xb[qo + q] - 1.0)
                nonfb.append(not rf[qo + q])
        co += nc * nq
    r, nonfb = np.asarray(regrets), np.asarray(nonfb)
    return {"programs": int(nk), "points": points, "train_samples": n_samples, "epochs": epochs,
            "train_ms": train_ms, "exact_ms": exact_ms + exact_col, "select_ms": sel_ms,
            "fallback_ms": fb_ms, "collapse_ms": col_ms, "fallback_rate": fbr,
            "speedup_vs_exact": (exact_ms + exact_col) / (sel_ms + fb_ms + col_ms),
            "regret_programs": int(rsub.n_progs),
            "regret_with_fallback": {"frac_le_1pct": float(np.mean(r <= 0.01)), "p50": float(np.median(r)),
                                     "nonfallback_frac_le_1pct": float(np.mean(r[nonfb] <= 0.01)) if nonfb.any() else None}}


def large_batch_component(lib, klr, synth, seed, replays=3, surrogate_epochs=0):
    """The large persistent batch beside the step: 16384 programs with uneven launch grids
    (32..512 configurations of 2-4 launch parameters), all 131072 metric fits (degree <= 3,
    64..1024 samples, FP64 to tol 1e-5) and the evaluation/argmin of 4096 queries per program
    with the fitted coefficients, captured once in a graph and replayed; per-kernel HIP-event
    times from a timed eager pass."""
    import numpy as np
    import torch
    t = time.perf_counter()
    fb, pb = synth.config5_batch(seed)
    gen_s = time.perf_counter() - t
    df = klr.DeviceFit.from_batch(fb)
    s = torch.cuda.Stream()
    fit_out = (torch.empty(df.n_coef, dtype=torch.float64, device="cuda"),
               torch.empty(df.n_fits * klr.FIT_INFO.itemsize, dtype=torch.uint8, device="cuda"))
    de = klr.DeviceEval.from_batch(lib, pb, coef=fit_out[0])
    nq = de.queries.numel()
    ev_out = (torch.empty(nq, dtype=torch.int32, device="cuda"), torch.empty(nq, dtype=torch.float32, device="cuda"),
              None, torch.empty(de.n_progs, dtype=torch.int32, device="cuda"))
    points = int((pb.n_cfg.astype(np.int64) * pb.n_q).sum())
    with torch.cuda.stream(s):
        lib.profile_enable(True)
        lib.fit_batched(df, klr.KLR_FP64, FIT_MAX_ITER, 1e-5, out=fit_out, stream=s)
        lib.eval_argmin(de, out=ev_out, stream=s)
        s.synchronize()
        fit_ms, _ = lib.profile_read(klr.K_FIT_SOLVE)
        ev_ms, _ = lib.profile_read(klr.K_EVAL)
        col_ms, _ = lib.profile_read(klr.K_COLLAPSE)
        lib.profile_enable(False)
        # the plain method: one workgroup / wavefront per fit in descriptor order, eager
        lib.set_option(klr.OPT_FIT_PERSISTENT, 0)
        try:
            lib.profile_enable(True)
            lib.fit_batched(df, klr.KLR_FP64, FIT_MAX_ITER, 1e-5, out=fit_out, stream=s)
            s.synchronize()
            plain_fit_ms, _ = lib.profile_read(klr.K_FIT_SOLVE)
            lib.profile_enable(False)
        finally:
            lib.set_option(klr.OPT_FIT_PERSISTENT, 1)
    lib.capture_begin(s)
    lib.fit_batched(df, klr.KLR_FP64, FIT_MAX_ITER, 1e-5, out=fit_out, stream=s)
    lib.eval_argmin(de, out=ev_out, stream=s)
    g = lib.capture_end(s)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(replays):
        lib.graph_launch(g, s)
    e1.record(s)
    s.synchronize()
    lib.graph_destroy(g)
    ms = e0.elapsed_time(e1) / replays
    ir = klr.info_records(fit_out[1])
    res = {"programs": int(pb.n_progs), "fits": int(fb.n_fits), "fit_rows": int(fb.m.sum()),
           "points": points, "generate_s": gen_s, "graph_ms": ms,
           "fit_ms": fit_ms, "plain_fit_ms": plain_fit_ms, "eval_ms": ev_ms, "collapse_ms": col_ms,
           "eval_fp32_tflops": eval_flops_per_point(3) * points / (ev_ms / 1e3) / 1e12,
           "eager_total_ms": fit_ms + ev_ms + col_ms,
           "fits_per_s": fb.n_fits / (fit_ms / 1e3), "evals_per_s": points / (ev_ms / 1e3),
           "iters_mean": float(ir["iters"].mean()), "not_converged": float(np.mean((ir["status"] & 4) > 0))}
    if surrogate_epochs > 0:
        del de, ev_out
        res["surrogate_two_launch_params"] = large_surrogate(lib, klr, synth, pb, fit_out[0], seed,
                                                             surrogate_epochs)
    return res


def _one_program(pb, p, nq):
    """Program p of a batch with its first nq queries, as a one-program batch holding only its
    own fits, configurations and queries (small enough to hand to a worker process)."""
    import copy
    out = copy.copy(pb)
    f0 = int(pb.fit0[p])
    fits = slice(f0, f0 + N_METRICS)
    c_lo = int(pb.coef0[f0])
    c_hi = int(pb.coef0[f0 + N_METRICS - 1] + pb.n_num[f0 + N_METRICS - 1]
               + pb.n_den[f0 + N_METRICS - 1] - 1)
    out.coef = pb.coef[c_lo:c_hi].copy()
    out.num0, out.n_num, out.den0, out.n_den = pb.num0[fits], pb.n_num[fits], pb.den0[fits], pb.n_den[fits]
    out.coef0, out.scale_exp = pb.coef0[fits] - c_lo, pb.scale_exp[fits]
    vl, nc = int(pb.v_launch[p]), int(pb.n_cfg[p])
    out.cfgs = pb.cfgs[int(pb.cfg0[p]): int(pb.cfg0[p]) + nc * vl].copy()
    out.queries = pb.queries[int(pb.q0[p]): int(pb.q0[p]) + nq].copy()
    out.v_launch, out.fit0 = pb.v_launch[p:p + 1], np.zeros(1, np.int32)
    out.cfg0, out.n_cfg, out.grid_kind = np.zeros(1, np.int64), pb.n_cfg[p:p + 1], pb.grid_kind[p:p + 1]
    out.q0, out.n_q = np.zeros(1, np.int64), np.array([nq], np.int32)
    return out


def _oracle_eval_task(pb1):
    """Worker: the oracle's FP32 replay + brute-force argmin of one program slice."""
    from oracle import cost as oc
    t = time.perf_counter()
    c = oc.program_costs(pb1, 0)
    oc.argmin_lowest(c)
    return c.size, time.perf_counter() - t


def _oracle_fit_task(fits):
    """Worker: the oracle's pivoted-QR least squares on a list of (X, f, E_num, E_den, s)."""
    from oracle import fit as of
    t = time.perf_counter()
    for Xi, fi, En, Ed, sc in fits:
        of.fit_one(Xi, fi, En, Ed, sc)
    return len(fits), time.perf_counter() - t


def _noop(_):
    return 0


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pb, fb, budget_s: float, points: int, n_fits: int, workers: int):
    """The oracle timed on bounded samples of the same step, at one thread and at `workers`
    threads (worker processes, each single-threaded: numpy's elementwise arithmetic and the
    small QR factorisations run on one core): FP32 replay + brute-force argmin over program
    slices of up to 8192 queries x all configurations, and pivoted-QR fits of the batch's fits.  The
    step time at each thread count is scaled from the two rates.  Runs before the GPU is
    touched (worker processes start from a fresh interpreter)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    nq = min(8192, int(pb.n_q[0]))
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    ctx = mp.get_context("spawn")
    res = {}
    try:
        for nw in (1, workers):
            with ProcessPoolExecutor(max_workers=nw, mp_context=ctx) as ex:
                list(ex.map(_noop, range(nw)))                       # start the workers first
                share = 0.6 * budget_s / 2
                # evaluation: program slices, in waves of nw tasks until the share is spent
                t0, pts, prog = time.perf_counter(), 0, 0
                while time.perf_counter() - t0 < share and prog < pb.n_progs:
                    batch = [_one_program(pb, (prog + i) % pb.n_progs, nq) for i in range(nw)]
                    for n, _ in ex.map(_oracle_eval_task, batch):
                        pts += n
                    prog += nw
                t_ev = time.perf_counter() - t0
                # fits: chunks of 16 fits per task
                share = 0.4 * budget_s / 2
                t1, nf, fi = time.perf_counter(), 0, 0
                while time.perf_counter() - t1 < share:
                    chunks = []
                    for _ in range(nw):
                        chunks.append([fb.fit_arrays((fi + j) % fb.n_fits) for j in range(16)])
                        fi += 16
                    for n, _ in ex.map(_oracle_fit_task, chunks):
                        nf += n
                t_fit = time.perf_counter() - t1
            ev_rate, fit_rate = pts / t_ev, nf / t_fit
            step_s = n_fits / fit_rate + points / ev_rate
            res[nw] = {"value": points / step_s, "evals_per_s": ev_rate, "fits_per_s": fit_rate,
                       "eval_points": pts, "eval_s": t_ev, "fits": nf, "fit_s": t_fit}
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    allc, one = res[workers], res[1]
    return {"value": allc["value"], "unit": "evals/s", "cores": workers, "kind": "oracle",
            "fits_per_s": allc["fits_per_s"], "evals_per_s": allc["evals_per_s"],
            "single_thread": {"value": one["value"], "fits_per_s": one["fits_per_s"],
                              "evals_per_s": one["evals_per_s"]},
            "nproc": os.cpu_count(), "threads_per_worker": 1, "cpu_model": _cpu_model(),
            "sample": f"eval: program slices of {nq} queries x {int(pb.n_cfg[0])} configs, numpy FP32 replay + "
                      f"argmin ({allc['eval_points']} points in {allc['eval_s']:.1f} s at {workers} workers, "
                      f"{one['eval_points']} in {one['eval_s']:.1f} s at 1); fit: numpy pivoted Householder QR "
                      f"({allc['fits']} fits in {allc['fit_s']:.1f} s at {workers} workers, {one['fits']} in "
                      f"{one['fit_s']:.1f} s at 1); step time scaled from the two rates to {n_fits} fits + "
                      f"{points} points"}


def fp64_error(pb, am, bc, n_progs: int, nq: int):
    """Error of the step's FP32 results against the FP64 cycle estimate (the oracle's truth
    mode: each metric the full multivariate p/q in FP64, exact integer parts) on the first
    n_progs programs' first nq queries: argmin disagreement rate, regret of the FP32 pick under
    FP64 costs, relative error of the FP32 best cost."""
    from oracle import cost as oc
    dis = n = adm = 0
    regrets, rel = [], []
    for p in range(n_progs):
        q0 = int(pb.q0[p])
        c64 = oc.program_costs(pb, p, query_idx=np.arange(nq), mode="truth")
        i64, b64 = oc.argmin_lowest(c64)
        a32, b32 = am[q0:q0 + nq], bc[q0:q0 + nq].astype(np.float64)
        dis += int(np.sum(a32 != i64))
        adm += int(np.sum((a32 >= 0) != (i64 >= 0)))
        n += nq
        ok = (a32 >= 0) & (i64 >= 0)
        regrets.append(c64[np.maximum(a32, 0), np.arange(nq)][ok] / b64[ok] - 1.0)
        rel.append(np.abs(b32[ok] - b64[ok]) / b64[ok])
    r, e = np.concatenate(regrets), np.concatenate(rel)
    return {"queries": n, "argmin_mismatch_rate": dis / n, "admissibility_mismatch": adm,
            "regret_max": float(r.max()), "best_cost_rel_err_max": float(e.max()),
            "best_cost_rel_err_median": float(np.median(e)),
            "sample": f"first {nq} queries of the first {n_progs} programs, all configurations"}


def surrogate_fp64_regret(pb, picks, n_progs: int, nq: int):
    """Regret of the surrogate's picks (shortlist and 2 % fallback) under the FP64 cycle estimate
    (the oracle's truth mode) on the first n_progs programs' first nq queries: the FP64 cost of
    the pick over the FP64 optimum, minus one."""
    from oracle import cost as oc
    regrets = []
    n_all = int(pb.n_q[0])
    for p in range(n_progs):
        c64 = oc.program_costs(pb, p, query_idx=np.arange(nq), mode="truth")
        i64, b64 = oc.argmin_lowest(c64)
        a = picks[p * n_all: p * n_all + nq]
        ok = (a >= 0) & (i64 >= 0)
        regrets.append(c64[np.maximum(a, 0), np.arange(nq)][ok] / b64[ok] - 1.0)
    r = np.concatenate(regrets)
    return {"queries": int(r.size), "frac_le_1pct": float(np.mean(r <= 0.01)), "p50": float(np.median(r)),
            "p99": float(np.quantile(r, 0.99)), "max": float(r.max()),
            "sample": f"first {nq} queries of the first {n_progs} programs"}


def single_fit_component(lib, klr, synth, replays=200, seeds=100):
    """The single-fit workload: one FP64 fit of 200 samples over (N, B), then its fitted
    function over the 11 x 32 grid with the per-N argmin, captured as one graph; the median of
    `replays` individually timed replays (HIP events on the stream) is the time per fit +
    decision.  Decision quality against the generator's noise-free argmin over `seeds` seeds
    (each fitted on the device)."""
    import torch
    s = torch.cuda.Stream()
    picks_equal, regrets = [], []
    g = None
    times = []
    for seed in range(1, seeds + 1):
        fb = synth.config1_fit(seed)
        df = klr.DeviceFit.from_batch(fb)
        fit_out = (torch.empty(df.n_coef, dtype=torch.float64, device="cuda"),
                   torch.empty(klr.FIT_INFO.itemsize, dtype=torch.uint8, device="cuda"))
        de = klr.DeviceEval.from_batch(lib, synth.config1_program(fb), coef=fit_out[0])
        ev_out = (torch.empty(11, dtype=torch.int32, device="cuda"), torch.empty(11, dtype=torch.float32, device="cuda"),
                  None, torch.empty(1, dtype=torch.int32, device="cuda"))
        with torch.cuda.stream(s):
            lib.fit_batched(df, klr.KLR_FP64, 64, 1e-12, out=fit_out, stream=s)
            lib.eval_argmin(de, out=ev_out, stream=s)
        s.synchronize()
        if seed == 1:          # the timed graph: fit + grid evaluation + argmin of seed 1
            lib.capture_begin(s)
            lib.fit_batched(df, klr.KLR_FP64, 64, 1e-12, out=fit_out, stream=s)
            lib.eval_argmin(de, out=ev_out, stream=s)
            g = lib.capture_end(s)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(replays)]
            for _ in range(10):
                lib.graph_launch(g, s)
            for a, b in ev:
                a.record(s)
                lib.graph_launch(g, s)
                b.record(s)
            s.synchronize()
            times = sorted(a.elapsed_time(b) * 1e3 for a, b in ev)
            lib.graph_destroy(g)
        pick = ev_out[0].cpu().numpy()
        truth = synth.config1_truth_grid(fb)
        tp = np.argmin(truth, axis=0)
        picks_equal.append(float(np.mean(pick == tp)))
        regrets.append(truth[pick, np.arange(11)] / truth[tp, np.arange(11)] - 1.0)
    r = np.concatenate(regrets)
    return {"us_per_fit_and_decision_median": times[len(times) // 2], "us_p10": times[len(times) // 10],
            "us_p90": times[(9 * len(times)) // 10], "replays": replays,
            "decision_quality": {"seeds": seeds, "picks_equal_truth": float(np.mean(picks_equal)),
                                 "regret_under_truth_median": float(np.median(r)),
                                 "regret_under_truth_p90": float(np.quantile(r, 0.9)),
                                 "regret_under_truth_max": float(r.max())},
            "workload": "1 FP64 fit (200 of the 11 x 32 (N, B) grid points, degree <= 2, 1 % noise), "
                        "then the fitted function on all 352 points and the argmin over B per N"}


def collection_component(lib, klr, synth, seed):
    """Data collection on this GPU: each target kernel timed at 240 sample points (N, bx, by),
    the times fitted (FP64, degree <= 2 rational), the fitted time minimised over the 45 block
    shapes at 13 data sizes, and the pick compared with the exhaustively measured best shape
    (best time / chosen time, the paper's Table 1 measure; >= 0.85 counts as a good choice)."""
    import torch
    shapes = synth.block_shapes()
    out = {}
    for target, name in ((klr.TARGET_TRANSPOSE, "transpose"), (klr.TARGET_STENCIL, "stencil")):
        t0 = time.perf_counter()
        plan = synth.collection_plan(seed + target, 240)
        times = lib.collect_times(target, plan, reps=5)
        collect_s = time.perf_counter() - t0
        fb = synth.measured_fit(plan, times)
        df = klr.DeviceFit.from_batch(fb)
        coef, info = lib.fit_batched(df, klr.KLR_FP64, FIT_MAX_ITER, 1e-12)
        queries = np.rint(2.0 ** (8 + np.arange(13) / 3.0)).astype(np.int32)
        pb = synth.measured_program(fb, shapes, queries)
        de = klr.DeviceEval.from_batch(lib, pb, coef=coef)
        am, _, _, _ = lib.eval_argmin(de)
        torch.cuda.synchronize()
        am = am.cpu().numpy()
        grid = np.array([(n, bx, by) for n in queries for bx, by in shapes if max(bx, by) <= n], np.int32)
        tg = lib.collect_times(target, grid, reps=5)
        ratios = []
        for qi, n in enumerate(queries):
            sel = grid[:, 0] == n
            meas = dict(zip(map(tuple, grid[sel, 1:]), tg[sel]))
            chosen = meas.get(tuple(shapes[am[qi]]), np.inf) if am[qi] >= 0 else np.inf
            ratios.append(min(meas.values()) / chosen)
        r = np.array(ratios)
        ir = klr.info_records(info)
        out[name] = {"samples": int(plan.shape[0]), "collect_s": collect_s, "attributes": lib.target_attributes(target),
                     "fit_rel_resid": float(ir["resid_norm"][0] / np.linalg.norm(times)),
                     "best_over_chosen": [round(float(x), 4) for x in r], "median_ratio": float(np.median(r)),
                     "frac_ge_0.85": float(np.mean(r >= 0.85)), "sizes": [int(x) for x in queries]}
    return out


def piecewise_component(lib, klr, synth, seed):
    """Piecewise rational programs with a fitted decision node: 256 programs (3 fits each: the
    decision, and the two regime costs), 4096 queries x 128 configurations; fit and evaluation
    times, and the picks' regret under the generator's costs on 16 programs."""
    import copy
    import torch
    fb, pb, truth = synth.piecewise_batch(seed, n_progs=256, n_q=4096)
    df = klr.DeviceFit.from_batch(fb)
    coef, _ = lib.fit_batched(df, klr.KLR_FP64, FIT_MAX_ITER, 1e-12)
    torch.cuda.synchronize()
    lib.profile_enable(True)
    coef, _ = lib.fit_batched(df, klr.KLR_FP64, FIT_MAX_ITER, 1e-12)
    fit_ms, _ = lib.profile_read(klr.K_FIT_SOLVE)
    lib.profile_enable(False)
    pb2 = copy.copy(pb)
    de = klr.DeviceEval.from_batch(lib, pb2, coef=coef)
    am, _, _, _ = lib.eval_argmin(de)
    torch.cuda.synchronize()
    lib.profile_enable(True)
    am, _, _, _ = lib.eval_argmin(de)
    ev_ms, _ = lib.profile_read(klr.K_EVAL)
    col_ms, _ = lib.profile_read(klr.K_COLLAPSE)
    lib.profile_enable(False)
    am = am.cpu().numpy()
    regrets = []
    for p in range(16):
        q0, nq = int(pb.q0[p]), int(pb.n_q[p])
        t = truth(p, pb.queries[q0:q0 + nq])
        best = t.min(axis=0)
        a = am[q0:q0 + nq]
        ok = np.isfinite(best) & (a >= 0)
        regrets.append(t[a[ok], np.nonzero(ok)[0]] / best[ok] - 1.0)
    r = np.concatenate(regrets)
    points = int((pb.n_cfg.astype(np.int64) * pb.n_q).sum())
    return {"programs": int(pb.n_progs), "fits": int(fb.n_fits), "points": points, "fit_ms": fit_ms,
            "eval_ms": ev_ms, "collapse_ms": col_ms, "evals_per_s": points / ((ev_ms + col_ms) / 1e3),
            "regret_under_truth": {"median": float(np.median(r)), "frac_le_1pct": float(np.mean(r <= 0.01)),
                                   "frac_le_5pct": float(np.mean(r <= 0.05)), "queries": int(r.size)}}


def service_component(lib, klr, synth, pb, de, n_calls=2000):
    """The launch-time decision service over the 1024 c3 programs: single-size decisions as a
    launching program makes them, first for sizes never seen (each an evaluation on the GPU)
    and then repeated (answered from the history); microseconds per decision on the host."""
    svc = klr.Service(lib, de, pb, max_batch=256)
    try:
        rng = np.random.default_rng(5)
        progs = rng.integers(0, pb.n_progs, n_calls)
        sizes = np.rint(2.0 ** rng.uniform(8, 26, n_calls)).astype(np.int32)
        svc.decide(0, sizes[:4])                       # warm-up
        t = time.perf_counter()
        for p, n in zip(progs, sizes):
            svc.decide(int(p), [int(n)])
        miss_us = (time.perf_counter() - t) / n_calls * 1e6
        t = time.perf_counter()
        for p, n in zip(progs, sizes):
            svc.decide(int(p), [int(n)])
        hit_us = (time.perf_counter() - t) / n_calls * 1e6
        t = time.perf_counter()
        batch = svc.decide(7, np.rint(2.0 ** rng.uniform(8, 26, 4096)).astype(np.int32))
        batch_ms = (time.perf_counter() - t) * 1e3
        st = svc.stats()
        return {"decision_us_new_size": miss_us, "decision_us_from_history": hit_us,
                "batch_4096_new_sizes_ms": batch_ms, "stats": st,
                "admissible_picks": float(np.mean(batch["config"] >= 0))}
    finally:
        svc.close()


def fit_component(lib, klr, fb, prec, reps=3, persistent=True):
    """Eager HIP-event time of one precision / schedule on a fit batch, with iteration and
    status statistics and the FP64 roofline fraction."""
    import torch
    df = klr.DeviceFit.from_batch(fb)
    fit_out = (torch.empty(df.n_coef, dtype=torch.float64, device="cuda"),
               torch.empty(df.n_fits * klr.FIT_INFO.itemsize, dtype=torch.uint8, device="cuda"))
    lib.set_option(klr.OPT_FIT_PERSISTENT, 1 if persistent else 0)
    try:
        lib.fit_batched(df, prec, FIT_MAX_ITER, FIT_TOL[prec], out=fit_out)
        torch.cuda.synchronize()
        lib.profile_enable(True)
        for _ in range(reps):
            lib.fit_batched(df, prec, FIT_MAX_ITER, FIT_TOL[prec], out=fit_out)
        kms, kn = lib.profile_read(klr.K_FIT_SOLVE)
        lib.profile_enable(False)
    finally:
        lib.set_option(klr.OPT_FIT_PERSISTENT, 1)
    ir = klr.info_records(fit_out[1])
    kavg = kms / max(kn, 1)
    n_unk = (fb.n_num + fb.n_den - 1).astype(np.float64)
    m = fb.m.astype(np.float64)
    it = ir["iters"].astype(np.float64)
    if prec == klr.KLR_FP64_SVD:
        # one-sided Jacobi: per sweep n (n - 1) / 2 column pairs, each an inner product (2 m) and
        # a rotation of both columns (6 m), plus the column norms (2 m n)
        fl = float(np.sum(it * (4.0 * m * n_unk * (n_unk - 1.0) + 2.0 * m * n_unk)))
    else:
        fl = float(np.sum(fit_flops(m, n_unk, it)))
    return {"kernel_ms": kavg, "fits_per_s": fb.n_fits / (kavg / 1e3), "tol": FIT_TOL[prec],
            "iters_mean": float(ir["iters"].mean()), "iters_max": int(ir["iters"].max()),
            "rank_deficient": float(np.mean((ir["status"] & 1) > 0)),
            "fell_back_fp64": float(np.mean((ir["status"] & 8) > 0)),
            "not_converged": float(np.mean((ir["status"] & 4) > 0)),
            "err_est_max": float(ir["err_est"].max()),
            "fp64_tflops": fl / (kavg / 1e3) / 1e12, "fp64_frac": fl / (kavg / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
            "schedule": "persistent longest-first" if persistent else "plain (one wavefront / workgroup per fit)"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--cpu-budget-s", type=float, default=24.0)
    ap.add_argument("--cpu-workers", type=int, default=min(os.cpu_count() or 1, 16))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision-sweep", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-large-batch", action="store_true")
    ap.add_argument("--no-single-fit", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the data-collection, piecewise-program and decision-service components")
    ap.add_argument("--kernel-only", choices=("eval", "fit", "copy", "large", "mlp"), default=None,
                    help="run only this kernel --steps times (for hardware-counter runs); "
                         "'copy' is a plain 1 GiB device copy used to calibrate byte counters")
    ap.add_argument("--surrogate-epochs", type=int, default=300)
    ap.add_argument("--large-surrogate-epochs", type=int, default=150)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (fits and programs "
              "would be sharded by descriptor ranges, one process per GPU); run with --gpus 1", file=sys.stderr)
        return 2

    from paper_1911_02373_amd import synth
    t = time.perf_counter()
    pb = synth.config3_programs(args.seed, n_progs=1024, n_q=65536)
    fb = synth.config2_fits(args.seed, n_fits=4096, domain="2a")
    points = int((pb.n_cfg.astype(np.int64) * pb.n_q).sum())
    log(f"workload generated in {time.perf_counter() - t:.1f} s: {fb.n_fits} fits "
        f"({int(fb.m.sum())} rows), {pb.n_progs} programs, {points:.3e} points")
    cpu = None
    if not args.no_cpu_baseline and args.kernel_only is None:
        # before the GPU is touched: the oracle's worker processes start from a fresh interpreter
        t = time.perf_counter()
        cpu = cpu_baseline(pb, fb, args.cpu_budget_s, points, fb.n_fits, args.cpu_workers)
        log(f"cpu baseline in {time.perf_counter() - t:.1f} s: {cpu['evals_per_s']:.3e} evals/s and "
            f"{cpu['fits_per_s']:.0f} fits/s at {cpu['cores']} workers; "
            f"{cpu['single_thread']['evals_per_s']:.3e} / {cpu['single_thread']['fits_per_s']:.0f} at 1")

    import torch
    from paper_1911_02373_amd import klr

    lib = klr.Library.get()
    if args.kernel_only == "copy":
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(args.steps):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"kernel_only": "copy", "bytes_read": x.numel() * 4, "bytes_written": y.numel() * 4,
                          "launches": args.steps}), flush=True)
        return 0
    if args.kernel_only == "large":
        # the large persistent batch alone (fits, then collapse + evaluation), eagerly
        fb5, pb5 = synth.config5_batch(args.seed)
        df5 = klr.DeviceFit.from_batch(fb5)
        fo = (torch.empty(df5.n_coef, dtype=torch.float64, device="cuda"),
              torch.empty(df5.n_fits * klr.FIT_INFO.itemsize, dtype=torch.uint8, device="cuda"))
        de5 = klr.DeviceEval.from_batch(lib, pb5, coef=fo[0])
        nq5 = de5.queries.numel()
        eo = (torch.empty(nq5, dtype=torch.int32, device="cuda"), torch.empty(nq5, dtype=torch.float32, device="cuda"),
              None, torch.empty(de5.n_progs, dtype=torch.int32, device="cuda"))
        torch.cuda.synchronize()
        for _ in range(args.steps):
            lib.fit_batched(df5, klr.KLR_FP64, FIT_MAX_ITER, 1e-5, out=fo)
            lib.eval_argmin(de5, out=eo)
            torch.cuda.synchronize()
            log("large batch pass done")
        print(json.dumps({"kernel_only": "large", "launches": args.steps, "fits": int(fb5.n_fits),
                          "fit_rows": int(fb5.m.sum()),
                          "points": int((pb5.n_cfg.astype(np.int64) * pb5.n_q).sum())}), flush=True)
        return 0
    de = klr.DeviceEval.from_batch(lib, pb)
    df = klr.DeviceFit.from_batch(fb)
    dev = "cuda"
    out = (torch.empty(de.queries.numel(), dtype=torch.int32, device=dev),
           torch.empty(de.queries.numel(), dtype=torch.float32, device=dev), None,
           torch.empty(de.n_progs, dtype=torch.int32, device=dev))
    fit_out = (torch.empty(df.n_coef, dtype=torch.float64, device=dev),
               torch.empty(df.n_fits * klr.FIT_INFO.itemsize, dtype=torch.uint8, device=dev))

    def step():
        lib.fit_batched(df, klr.KLR_FP64, FIT_MAX_ITER, FIT_TOL[0], out=fit_out)
        lib.eval_argmin(de, out=out)

    if args.kernel_only == "mlp":
        # surrogate training (a few epochs) and one selection over the full grid
        comp = surrogate_component(lib, klr, synth, pb, de, 1.0, args.seed, args.steps, regret_programs=2)
        print(json.dumps({"kernel_only": "mlp", "epochs": args.steps, "select_ms": comp["select_ms"]}), flush=True)
        return 0
    if args.kernel_only is not None:
        lib.eval_argmin(de, out=out)          # tune the sweep's launch shape outside the counted run
        torch.cuda.synchronize()
        for _ in range(args.steps):
            if args.kernel_only == "eval":
                lib.eval_argmin(de, out=out)
            else:
                lib.fit_batched(df, klr.KLR_FP64, FIT_MAX_ITER, FIT_TOL[0], out=fit_out)
        torch.cuda.synchronize()
        print(json.dumps({"kernel_only": args.kernel_only, "launches": args.steps, "points": points,
                          "fits": int(fb.n_fits), "fit_rows": int(fb.m.sum())}), flush=True)
        return 0

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
    kt = {k: lib.profile_read(k) for k in (klr.K_EVAL, klr.K_COLLAPSE, klr.K_FIT_SOLVE)}
    lib.profile_enable(False)
    st = out[3].cpu().numpy()
    info = klr.info_records(fit_out[1])
    if not np.all(st == 0) or np.any(info["status"] & 16):
        log("bad status:", np.unique(st), np.unique(info["status"]))
        return 1
    avg = {k: v[0] / max(v[1], 1) for k, v in kt.items()}
    eval_avg = avg[klr.K_EVAL]
    flops = eval_flops_per_point(2)
    achieved = flops * points / (eval_avg / 1e3) / 1e12
    n_unk = (fb.n_num + fb.n_den - 1).astype(np.float64)
    fit_fl = float(np.sum(fit_flops(fb.m.astype(np.float64), n_unk, info["iters"].astype(np.float64))))
    comps = {
        "eval": {"kernel_ms": eval_avg, "collapse_ms": avg[klr.K_COLLAPSE],
                 "evals_per_s": points / ((eval_avg + avg[klr.K_COLLAPSE]) / 1e3),
                 "lane_ops_per_point": eval_ops_per_point(2),
                 "issue_rate_T_lane_ops": eval_ops_per_point(2) * points / (eval_avg / 1e3) / 1e12,
                 "issue_rate_note": "normative operations (each compare / select / integer op counted once) per "
                                    "second; a diagnostic, not a roofline"},
        "fit_fp64": {"kernel_ms": avg[klr.K_FIT_SOLVE], "fits_per_s": fb.n_fits / (avg[klr.K_FIT_SOLVE] / 1e3),
                     "iters_mean": float(info["iters"].mean()), "iters_max": int(info["iters"].max()),
                     "tol": FIT_TOL[0], "err_est_max": float(info["err_est"].max()),
                     "roofline": {"bound": "fp64", "achieved": fit_fl / (avg[klr.K_FIT_SOLVE] / 1e3) / 1e12,
                                  "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                  "frac": fit_fl / (avg[klr.K_FIT_SOLVE] / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
                                  "flops_per_launch": fit_fl}},
    }
    log(f"step {ms:.3f} ms; eval {eval_avg:.3f} ms; collapse {avg[klr.K_COLLAPSE]:.3f} ms; "
        f"fit {avg[klr.K_FIT_SOLVE]:.3f} ms")
    am_h, bc_h = out[0].cpu().numpy(), out[1].cpu().numpy()
    del de
    comps["fit_fp64_plain"] = fit_component(lib, klr, fb, klr.KLR_FP64, persistent=False)
    fb2b = synth.config2_fits(args.seed, n_fits=4096, domain="2b")
    comps["fit_fp64_c2b"] = fit_component(lib, klr, fb2b, klr.KLR_FP64)
    log(f"fit plain schedule {comps['fit_fp64_plain']['kernel_ms']:.3f} ms; c2b {comps['fit_fp64_c2b']['kernel_ms']:.3f} ms")
    if not args.no_precision_sweep:
        for prec, name in ((klr.KLR_FP32_REFINED, "fit_fp32_refined"), (klr.KLR_BF16_REFINED, "fit_bf16_refined")):
            comps[name] = fit_component(lib, klr, fb, prec)
            comps[name]["speedup_vs_fp64"] = avg[klr.K_FIT_SOLVE] / comps[name]["kernel_ms"]
            comps[name + "_c2b"] = fit_component(lib, klr, fb2b, prec)
            log(f"{name}: {comps[name]['kernel_ms']:.3f} ms, iters mean {comps[name]['iters_mean']:.1f}; "
                f"c2b {comps[name + '_c2b']['kernel_ms']:.3f} ms")
    comps["fit_svd_c2a"] = fit_component(lib, klr, fb, klr.KLR_FP64_SVD, reps=1)
    comps["fit_svd_c2b"] = fit_component(lib, klr, fb2b, klr.KLR_FP64_SVD, reps=1)
    log(f"SVD fits: c2a {comps['fit_svd_c2a']['kernel_ms']:.2f} ms, c2b {comps['fit_svd_c2b']['kernel_ms']:.2f} ms")
    if not args.no_extras:
        comps["data_collection"] = dc = collection_component(lib, klr, synth, args.seed)
        log("data collection: " + ", ".join(f"{k} median best/chosen {v['median_ratio']:.3f}" for k, v in dc.items()))
        comps["piecewise"] = pw = piecewise_component(lib, klr, synth, args.seed)
        log(f"piecewise: eval {pw['eval_ms']:.2f} ms, median regret {pw['regret_under_truth']['median']:.4f}")
        de_s = klr.DeviceEval.from_batch(lib, pb)
        comps["service"] = sv = service_component(lib, klr, synth, pb, de_s)
        log(f"service: {sv['decision_us_new_size']:.1f} us per new size, {sv['decision_us_from_history']:.2f} us "
            f"from the history")
        del de_s
    if not args.no_single_fit:
        comps["single_fit"] = sf = single_fit_component(lib, klr, synth)
        log(f"single fit + grid decision: median {sf['us_per_fit_and_decision_median']:.1f} us per graph replay; "
            f"picks equal to the truth's {sf['decision_quality']['picks_equal_truth']:.3f}")

    surr_picks = None
    if not args.no_surrogate:
        de = klr.DeviceEval.from_batch(lib, pb)
        comps["surrogate"] = surrogate_component(lib, klr, synth, pb, de, eval_avg + avg[klr.K_COLLAPSE],
                                                 args.seed, args.surrogate_epochs)
        sc = comps["surrogate"]
        surr_picks = sc.pop("_picks")
        log(f"surrogate: train {sc['train_ms']:.0f} ms, select {sc['select_ms']:.0f} ms, fallback rate "
            f"{sc['fallback_rate']:.3f}, speedup vs exact {sc['speedup_vs_exact']:.3f}")
        del de

    if not args.no_large_batch:
        del df
        torch.cuda.empty_cache()
        comps["large_batch"] = lb = large_batch_component(
            lib, klr, synth, args.seed, surrogate_epochs=0 if args.no_surrogate else args.large_surrogate_epochs)
        log(f"large batch: {lb['fits']} fits + {lb['points']:.3e} points, graph {lb['graph_ms']:.1f} ms "
            f"(fit {lb['fit_ms']:.1f}, plain fit {lb['plain_fit_ms']:.1f}, eval {lb['eval_ms']:.1f}); "
            f"generated in {lb['generate_s']:.0f} s")
        if "surrogate_two_launch_params" in lb:
            ls = lb["surrogate_two_launch_params"]
            log(f"large batch surrogate ({ls['programs']} programs): train {ls['train_ms']:.0f} ms, select + "
                f"fallback {ls['select_ms'] + ls['fallback_ms']:.0f} ms vs exact {ls['exact_ms']:.1f} ms, fallback "
                f"rate {ls['fallback_rate']:.3f}, within 1 % {ls['regret_with_fallback']['frac_le_1pct']:.3f}")

    res = {
        "metric": METRIC,
        "value": points / (ms / 1e3),
        "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 eval / f64 fit", "data": "synthetic (seeded)",
        "config": {"workload": "fit 4096 uneven degree-3 rational fits over (N, bx, by) + eval/argmin "
                               "of 1024 rational programs x 65536 queries x 128 launch configs",
                   "fits": int(fb.n_fits), "fit_rows": int(fb.m.sum()), "unknowns": 39,
                   "programs": int(pb.n_progs), "queries_per_program": 65536, "configs": 128,
                   "points": points},
        "fits_per_s": comps["fit_fp64"]["fits_per_s"],
        "evals_per_s": comps["eval"]["evals_per_s"],
        "components": comps,
        "roofline": {"bound": "alu", "kernel": "eval_kernel", "achieved": achieved,
                     "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                     "frac_of_unpacked_fp32": achieved / FP32_UNPACKED_TFLOPS,
                     "flops_per_point": flops, "points_per_launch": points,
                     "traffic": measured_traffic()},
    }
    if cpu is not None:
        t = time.perf_counter()
        cpu["fp64_error"] = fp64_error(pb, am_h, bc_h, 8, 2048)
        log(f"FP64 check in {time.perf_counter() - t:.1f} s: {cpu['fp64_error']}")
        if surr_picks is not None:
            comps["surrogate"]["regret_fp64_truth"] = surrogate_fp64_regret(pb, surr_picks, 8, 2048)
            log(f"surrogate regret under FP64 truth: {comps['surrogate']['regret_fp64_truth']}")
        res["cpu_baseline"] = cpu
        res["fp64_error"] = cpu["fp64_error"]
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

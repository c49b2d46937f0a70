"""Seeded synthetic workloads for the rational-program fit and the launch-configuration search.

This module only draws random inputs and lays them out in flat arrays.  It holds none of the
method's arithmetic (no design matrix, no least squares, no cost model, no argmin).  The one
computation it performs is the data-generating process itself: evaluating a seeded ground-truth
rational function at the sample points to produce the "measured" metric values, which stand in
for the profiler readings of the paper's data-collection step (section "An Algorithm to Build
and Deploy a Performance-Predicting Rational Program", step 1).

Both the GPU path and the CPU oracle consume these arrays; neither shares any other code.

Layouts (structure of arrays, all numpy):
  fits:  X   int32 flat, fit i's samples at X[x0[i] : x0[i] + m[i]*v[i]] as rows of v[i]
         f   float64 flat, fit i's targets at f[f0[i] : f0[i] + m[i]]
         exps uint8 [rows][8], exponent tuples; a fit uses rows [num0, num0+n_num) for the
             numerator and [den0, den0+n_den) for the denominator (row den0 is all-zero: the
             denominator's constant coefficient is fixed to 1)
         coef0 offset of the fit's n_num + n_den - 1 coefficients (numerator first)
         scale_exp int8 [n_fits][8]: variable k enters the monomials as x_k * 2**-scale_exp[k]
  programs (eval): eight consecutive fits per program in the metric order
         (I_comp, I_mc, I_mu, U, I_sync, R, Z, B_w); configs int32 rows of v_launch;
         queries int32 data sizes N.
"""
from __future__ import annotations

import itertools
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

MAX_VARS = 8
N_METRICS = 8
METRIC_NAMES = ("I_comp", "I_mc", "I_mu", "U", "I_sync", "R", "Z", "B_w")
# Value ranges [lo, hi] of the synthetic metrics (per-thread instruction counts, transactions
# per uncoalesced wave access, sync instructions, registers per thread, LDS bytes per block,
# bytes per wave memory transaction).
METRIC_RANGES = ((10.0, 4000.0), (1.0, 200.0), (0.0, 50.0), (1.0, 16.0), (0.0, 8.0),
                 (16.0, 128.0), (0.0, 65536.0), (64.0, 512.0))


def monomials(v: int, d: int) -> np.ndarray:
    """All exponent tuples in v variables of total degree <= d, graded order.

    Within one total degree the tuples are in descending lexicographic order, so the constant
    monomial is row 0 and, for v=2, d=2 the order is 1, x, y, x^2, xy, y^2.
    Returned as uint8 [n][MAX_VARS] (unused variables zero)."""
    rows = []
    for deg in range(d + 1):
        tup = [t for t in itertools.product(range(deg + 1), repeat=v) if sum(t) == deg]
        tup.sort(reverse=True)
        rows.extend(tup)
    out = np.zeros((len(rows), MAX_VARS), np.uint8)
    for i, t in enumerate(rows):
        out[i, :v] = t
    return out


def _truth_value(xt: np.ndarray, e_num: np.ndarray, e_den: np.ndarray,
                 c_num: np.ndarray, c_den: np.ndarray) -> np.ndarray:
    """Ground-truth p/q at scaled points xt [m][v] (data generation only)."""
    v = xt.shape[1]
    def poly(E, c):
        acc = np.zeros(xt.shape[0])
        for e, ce in zip(E, c):
            term = np.full(xt.shape[0], ce)
            for k in range(v):
                for _ in range(int(e[k])):
                    term = term * xt[:, k]
            acc = acc + term
        return acc
    return poly(e_num, c_num) / poly(e_den, c_den)


@dataclass
class FitBatch:
    """A batch of independent rational fits (structure of arrays)."""
    X: np.ndarray
    f: np.ndarray
    exps: np.ndarray
    x0: np.ndarray
    f0: np.ndarray
    m: np.ndarray
    v: np.ndarray
    num0: np.ndarray
    n_num: np.ndarray
    den0: np.ndarray
    n_den: np.ndarray
    coef0: np.ndarray
    scale_exp: np.ndarray
    n_coef: int
    truth_coef: np.ndarray | None = None     # same layout as the fitted coefficients
    meta: dict = field(default_factory=dict)

    @property
    def n_fits(self) -> int:
        return int(self.m.shape[0])

    def fit_arrays(self, i: int):
        """(X_i [m][v] int32, f_i [m], E_num, E_den, scale_exp[:v]) of fit i."""
        v, m = int(self.v[i]), int(self.m[i])
        Xi = self.X[self.x0[i]: self.x0[i] + m * v].reshape(m, v)
        fi = self.f[self.f0[i]: self.f0[i] + m]
        En = self.exps[self.num0[i]: self.num0[i] + self.n_num[i], :v]
        Ed = self.exps[self.den0[i]: self.den0[i] + self.n_den[i], :v]
        return Xi, fi, En, Ed, self.scale_exp[i, :v]


def _pack_fits(samples, exps, num0, n_num, den0, n_den, scale, truth=None, meta=None) -> FitBatch:
    n = len(samples)
    v = np.array([s[0].shape[1] for s in samples], np.int32)
    m = np.array([s[0].shape[0] for s in samples], np.int32)
    x0 = np.zeros(n, np.int64)
    f0 = np.zeros(n, np.int64)
    x0[1:] = np.cumsum((m.astype(np.int64) * v)[:-1])
    f0[1:] = np.cumsum(m.astype(np.int64)[:-1])
    X = np.concatenate([s[0].reshape(-1) for s in samples]).astype(np.int32) if n else np.zeros(0, np.int32)
    f = np.concatenate([s[1] for s in samples]).astype(np.float64) if n else np.zeros(0)
    n_num = np.asarray(n_num, np.int32)
    n_den = np.asarray(n_den, np.int32)
    ncoef = n_num.astype(np.int64) + n_den - 1
    coef0 = np.zeros(n, np.int64)
    coef0[1:] = np.cumsum(ncoef[:-1])
    tc = None
    if truth is not None:
        tc = np.concatenate(truth) if n else np.zeros(0)
    return FitBatch(X=X, f=f, exps=exps, x0=x0, f0=f0, m=m, v=v,
                    num0=np.asarray(num0, np.int32), n_num=n_num,
                    den0=np.asarray(den0, np.int32), n_den=n_den, coef0=coef0,
                    scale_exp=np.asarray(scale, np.int8), n_coef=int(ncoef.sum()),
                    truth_coef=tc, meta=meta or {})


def config1_fit(seed: int, noise: float = 0.01, n_samples: int = 200) -> FitBatch:
    """One fit in (N, B): N = 2^10..2^20, B = 32..1024 step 32, total degree <= 2 num and den.

    200 distinct points of the 11 x 32 grid; coefficients U(0.1, 2) in the scaled variables
    N/2^20, B/2^10; targets times (1 + eps), eps ~ N(0, noise^2)."""
    rng = np.random.default_rng(seed)
    Ns = 2 ** np.arange(10, 21)
    Bs = 32 * np.arange(1, 33)
    grid = np.array([(n, b) for n in Ns for b in Bs], np.int64)
    pick = rng.choice(grid.shape[0], size=n_samples, replace=False)
    Xi = grid[pick].astype(np.int32)
    E = monomials(2, 2)
    c_num = rng.uniform(0.1, 2.0, E.shape[0])
    c_den = np.concatenate([[1.0], rng.uniform(0.1, 2.0, E.shape[0] - 1)])
    scale = np.zeros((1, MAX_VARS), np.int8)
    scale[0, :2] = (20, 10)
    xt = Xi.astype(np.float64) * 2.0 ** -scale[0, :2].astype(np.float64)
    ftrue = _truth_value(xt, E[:, :2], E[:, :2], c_num, c_den)
    eps = rng.normal(0.0, 1.0, n_samples) * noise
    fi = ftrue * (1.0 + eps)
    exps = np.concatenate([E, E])
    truth = np.concatenate([c_num, c_den[1:]])
    return _pack_fits([(Xi, fi)], exps, [0], [E.shape[0]], [E.shape[0]], [E.shape[0]], scale,
                      truth=[truth], meta={"grid": grid.astype(np.int32), "noise": noise})


def config1_program(fb: FitBatch, coef: np.ndarray | None = None) -> "ProgramBatch":
    """The rational program of the single-fit workload: its one fitted function (fit 0 of `fb`,
    over (N, B)) is the cost, evaluated on the full 11 x 32 grid (queries N = 2^10..2^20,
    configurations B = 32..1024 step 32, one launch parameter) with the per-N argmin over B.
    The wavefront is 32 wide here (the paper's warp), so every B is a whole number of waves.
    `coef` defaults to the generator's truth coefficients."""
    grid = fb.meta["grid"]
    Ns = np.unique(grid[:, 0]).astype(np.int32)
    Bs = np.unique(grid[:, 1]).astype(np.int32)
    c = fb.truth_coef if coef is None else coef
    return ProgramBatch(
        fits=None, coef=np.asarray(c, np.float64), exps=fb.exps, num0=fb.num0[:1], n_num=fb.n_num[:1],
        den0=fb.den0[:1], n_den=fb.n_den[:1], coef0=np.zeros(1, np.int64), scale_exp=fb.scale_exp[:1],
        v_launch=np.ones(1, np.int32), fit0=np.zeros(1, np.int32), cfg0=np.zeros(1, np.int64),
        n_cfg=np.array([Bs.size], np.int32), grid_kind=np.zeros(1, np.int32), q0=np.zeros(1, np.int64),
        n_q=np.array([Ns.size], np.int32), cfgs=Bs.copy(), queries=Ns.copy(), hw=HW(wave=32),
        cost_kind=np.ones(1, np.int32))


def config1_truth_grid(fb: FitBatch) -> np.ndarray:
    """The generator's noise-free metric on the 11 x 32 grid, [B][N] (the decision-quality
    reference of the single-fit workload)."""
    grid = fb.meta["grid"]
    Ns = np.unique(grid[:, 0])
    Bs = np.unique(grid[:, 1])
    n_num = int(fb.n_num[0])
    E = fb.exps[:n_num, :2]
    t = fb.truth_coef
    c_den = np.concatenate([[1.0], t[n_num:]])
    pts = np.array([(n, b) for b in Bs for n in Ns], np.float64)
    xt = pts * 2.0 ** -fb.scale_exp[0, :2].astype(np.float64)
    return _truth_value(xt, E, fb.exps[fb.den0[0]: fb.den0[0] + fb.n_den[0], :2], t[:n_num], c_den).reshape(Bs.size, Ns.size)


def block_shapes(t_min: int = 64, t_max: int = 1024) -> np.ndarray:
    """Power-of-two block shapes (bx, by) with t_min <= bx by <= t_max (45 shapes for 64..1024)."""
    return pow2_launch_tuples(2, t_min, t_max)


def collection_plan(seed: int, n_samples: int = 200, log2_range=(8.0, 12.5), shapes=None) -> np.ndarray:
    """Sample points K for timing a target kernel: rows (N, bx, by), N = round(2^u) with
    u ~ U(log2_range), the block shape uniform over `shapes` (default block_shapes())."""
    rng = np.random.default_rng(seed)
    shapes = block_shapes() if shapes is None else shapes
    N = np.rint(2.0 ** rng.uniform(log2_range[0], log2_range[1], n_samples)).astype(np.int32)
    S = shapes[rng.integers(0, shapes.shape[0], n_samples)]
    return np.stack([N, S[:, 0], S[:, 1]], 1).astype(np.int32)


def measured_fit(samples: np.ndarray, values: np.ndarray, degree: int = 2, scale=(13, 10, 10)) -> FitBatch:
    """One fit of measured values at sample rows (N, bx, by): numerator and denominator over the
    monomials of total degree <= `degree` in the scaled variables (N / 2^13, bx / 2^10, by / 2^10)."""
    E = monomials(3, degree)
    sc = np.zeros((1, MAX_VARS), np.int8)
    sc[0, :3] = scale
    return _pack_fits([(np.asarray(samples, np.int32), np.asarray(values, np.float64))], np.concatenate([E, E]),
                      [0], [E.shape[0]], [E.shape[0]], [E.shape[0]], sc, meta={"kind": "measured"})


def measured_program(fb: FitBatch, shapes: np.ndarray, queries, coef=None) -> "ProgramBatch":
    """A metric-cost program over fit 0 of `fb` (a fitted kernel time): configurations `shapes`
    (bx, by), queries the data sizes `queries`, wavefront 64."""
    q = np.asarray(queries, np.int32)
    c = np.zeros(fb.n_coef) if coef is None else np.asarray(coef, np.float64)
    return ProgramBatch(
        fits=None, coef=c, exps=fb.exps, num0=fb.num0[:1], n_num=fb.n_num[:1], den0=fb.den0[:1],
        n_den=fb.n_den[:1], coef0=np.zeros(1, np.int64), scale_exp=fb.scale_exp[:1],
        v_launch=np.full(1, 2, np.int32), fit0=np.zeros(1, np.int32), cfg0=np.zeros(1, np.int64),
        n_cfg=np.array([shapes.shape[0]], np.int32), grid_kind=np.ones(1, np.int32), q0=np.zeros(1, np.int64),
        n_q=np.array([q.size], np.int32), cfgs=np.ascontiguousarray(shapes.reshape(-1).astype(np.int32)),
        queries=q, hw=HW(), cost_kind=np.ones(1, np.int32))


LITERAL_PAIRS = np.array([(bx, by) for bx in (16, 32, 48, 64) for by in (16, 32, 48, 64)
                          if bx * by <= 1024], np.int32)
POW2_PAIRS = np.array([(1 << a, 1 << b) for a in range(11) for b in range(11)
                       if 16 <= (1 << (a + b)) <= 1024], np.int32)


def config2_fits(seed: int, n_fits: int = 4096, domain: str = "2a", noise: float = 0.01,
                 degree: int = 3, m_range=(64, 512)) -> FitBatch:
    """Batched uneven fits over (N, bx, by).

    domain "2a": (bx, by) from the 8 pairs of multiples of 16 with bx*by <= 1024;
    domain "2b": power-of-two (bx, by) with 16 <= bx*by <= 1024.
    N = round(2^u), u ~ U(8, 24); m ~ U{m_range}; truth of total degree <= `degree` with
    coefficients U(0.1, 2) in (N/2^24, bx/2^10, by/2^10); f = truth * exp(noise * z)."""
    rng = np.random.default_rng(seed)
    pairs = LITERAL_PAIRS if domain == "2a" else POW2_PAIRS
    E = monomials(3, degree)
    nm = E.shape[0]
    scale = np.zeros((n_fits, MAX_VARS), np.int8)
    scale[:, :3] = (24, 10, 10)
    sdiv = 2.0 ** -np.array([24.0, 10.0, 10.0])
    samples, truth = [], []
    ms = rng.integers(m_range[0], m_range[1] + 1, n_fits)
    for i in range(n_fits):
        m = int(ms[i])
        N = np.rint(2.0 ** rng.uniform(8.0, 24.0, m)).astype(np.int64)
        pr = pairs[rng.integers(0, pairs.shape[0], m)]
        Xi = np.stack([N, pr[:, 0], pr[:, 1]], axis=1).astype(np.int32)
        c_num = rng.uniform(0.1, 2.0, nm)
        c_den = np.concatenate([[1.0], rng.uniform(0.1, 2.0, nm - 1)])
        ftrue = _truth_value(Xi.astype(np.float64) * sdiv, E[:, :3], E[:, :3], c_num, c_den)
        fi = ftrue * np.exp(noise * rng.normal(0.0, 1.0, m))
        samples.append((Xi, fi))
        truth.append(np.concatenate([c_num, c_den[1:]]))
    exps = np.concatenate([E, E])
    return _pack_fits(samples, exps, [0] * n_fits, [nm] * n_fits, [nm] * n_fits, [nm] * n_fits,
                      scale, truth=truth, meta={"domain": domain, "noise": noise})


# ----------------------------------------------------------------------------------------------
# Rational programs for the evaluation / argmin sweep.

@dataclass
class HW:
    """Hardware parameters H, fixed per call."""
    n_cu: int = 256
    wave: int = 64
    w_max: int = 32          # resident waves per CU
    b_max: int = 32          # resident workgroups per CU
    r_max: int = 131072      # register-lanes per CU (512 VGPRs x 64 lanes x 4 SIMDs)
    z_max: int = 163840      # LDS bytes per CU
    t_max: int = 1024        # threads per workgroup
    mem_lat: float = 600.0   # memory latency, cycles
    dep_delay: float = 40.0  # departure delay between consecutive memory requests, cycles
    issue_cycles: float = 4.0
    bw: float = 13.0         # bytes per cycle per CU


def config3_launch_configs() -> np.ndarray:
    """128 launch configs (bx, by): bx = 2^a (a = 0..10), integer by, bx*by in 64*{1..16}
    (127 tuples), plus one pad (1, 1) that is never admissible."""
    out = []
    for a in range(11):
        bx = 1 << a
        for k in range(1, 17):
            t = 64 * k
            if t % bx == 0:
                out.append((bx, t // bx))
    out.append((1, 1))
    return np.array(out, np.int32)


@dataclass
class ProgramBatch:
    fits: FitBatch | None      # coefficient holders (8 per program); X/f empty
    coef: np.ndarray           # float64 coefficients (scaled basis), fits' layout
    exps: np.ndarray
    num0: np.ndarray
    n_num: np.ndarray
    den0: np.ndarray
    n_den: np.ndarray
    coef0: np.ndarray
    scale_exp: np.ndarray      # [n_fits][8]
    v_launch: np.ndarray       # per program
    fit0: np.ndarray
    cfg0: np.ndarray           # element offset into cfgs
    n_cfg: np.ndarray
    grid_kind: np.ndarray      # 0: blocks = ceil(N/prod L); 1: ceil(N/L0)*ceil(N/L1)
    q0: np.ndarray
    n_q: np.ndarray
    cfgs: np.ndarray           # int32 flat
    queries: np.ndarray        # int32 flat
    hw: HW
    cost_kind: np.ndarray | None = None    # per program: 0 cycle estimate (default), 1 fitted metric

    @property
    def n_progs(self) -> int:
        return int(self.fit0.shape[0])


def config3_programs(seed: int, n_progs: int = 1024, n_q: int = 65536, degree: int = 2,
                     log2_range=(8.0, 26.0), cfgs: np.ndarray | None = None) -> ProgramBatch:
    """Rational programs with 8 fitted metrics each, degree <= `degree` rationals in
    (N/2^26, bx/2^10, by/2^10).  Metric j is lo_j + s_j * p/q with p, q coefficients U(0.1, 2),
    q's constant 1, s_j = (hi_j - lo_j)/20 (p/q stays below 20 on the unit cube), so the
    numerator coefficients are lo_j * q + s_j * p.  Queries N = round(2^u), u ~ U(log2_range)."""
    rng = np.random.default_rng(seed)
    E = monomials(3, degree)
    nm = E.shape[0]
    n_fits = n_progs * N_METRICS
    coef = np.empty(n_fits * (2 * nm - 1))
    for i in range(n_fits):
        lo, hi = METRIC_RANGES[i % N_METRICS]
        s = (hi - lo) / 20.0
        p = rng.uniform(0.1, 2.0, nm)
        q = np.concatenate([[1.0], rng.uniform(0.1, 2.0, nm - 1)])
        coef[i * (2 * nm - 1): (i + 1) * (2 * nm - 1)] = np.concatenate([lo * q + s * p, q[1:]])
    if cfgs is None:
        cfgs = config3_launch_configs()
    n_cfg = cfgs.shape[0]
    queries = np.rint(2.0 ** rng.uniform(log2_range[0], log2_range[1], n_progs * n_q)).astype(np.int32)
    scale = np.zeros((n_fits, MAX_VARS), np.int8)
    scale[:, :3] = (26, 10, 10)
    return ProgramBatch(
        fits=None, coef=coef, exps=np.concatenate([E, E]),
        num0=np.zeros(n_fits, np.int32), n_num=np.full(n_fits, nm, np.int32),
        den0=np.full(n_fits, nm, np.int32), n_den=np.full(n_fits, nm, np.int32),
        coef0=np.arange(n_fits, dtype=np.int64) * (2 * nm - 1), scale_exp=scale,
        v_launch=np.full(n_progs, 2, np.int32),
        fit0=np.arange(n_progs, dtype=np.int32) * N_METRICS,
        cfg0=np.zeros(n_progs, np.int64), n_cfg=np.full(n_progs, n_cfg, np.int32),
        grid_kind=np.zeros(n_progs, np.int32),
        q0=np.arange(n_progs, dtype=np.int64) * n_q, n_q=np.full(n_progs, n_q, np.int32),
        cfgs=cfgs.reshape(-1).astype(np.int32), queries=queries, hw=HW())


def pow2_launch_tuples(v_launch: int, t_min: int = 64, t_max: int = 1024) -> np.ndarray:
    """All power-of-two tuples of v_launch launch parameters with product in [t_min, t_max]."""
    lo, hi = int(np.log2(t_min)), int(np.log2(t_max))
    out = [tuple(1 << a for a in t) for t in itertools.product(range(hi + 1), repeat=v_launch)
           if lo <= sum(t) <= hi]
    return np.array(sorted(out), np.int32).reshape(-1, v_launch)


def mixed_programs(seed: int, n_progs: int, n_q_range=(1, 700), n_cfg_range=(1, 160),
                   degree: int = 3, log2_range=(4.0, 26.0), v_launch_choices=(1, 2, 3, 4),
                   p_2d: float = 0.3, p_bad_cfg: float = 0.05,
                   launch_degree: int | None = None) -> ProgramBatch:
    """Uneven programs: v_launch from `v_launch_choices`, n_cfg and n_q uniform in the given
    ranges, metrics of total degree <= `degree` in (N/2^26, L_k/2^10) with the same lo + s*p/q
    construction as config3_programs (s = (hi - lo) / (2 * #monomials)).  With
    `launch_degree`, the monomials are instead N^a L^b with a <= `degree` and total launch degree
    <= `launch_degree` (large monomial sets).  Configurations are power-of-two tuples with
    product 64..1024 (the 2-parameter case uses the 127 config-3 tuples), plus a few random
    tuples that may be inadmissible.  Two-dimensional grids are drawn with probability p_2d when
    v_launch >= 2."""
    rng = np.random.default_rng(seed)
    vls = rng.choice(np.asarray(v_launch_choices), n_progs)
    exps_blocks, exps_index = [], {}
    row = 0
    for vl in sorted(set(int(x) for x in vls)):
        if launch_degree is None:
            E = monomials(1 + vl, degree)
        else:
            E = monomials(1 + vl, degree + launch_degree)
            E = E[(E[:, 0] <= degree) & (E[:, 1:].sum(1) <= launch_degree)]
        exps_index[vl] = (row, E.shape[0])
        exps_blocks.append(E)
        row += E.shape[0]
    exps = np.concatenate(exps_blocks)
    fit_num0, fit_nn, coef_parts, coef0 = [], [], [], []
    scale_rows, fit0, cfg0, n_cfg, gk, q0, n_q = [], [], [], [], [], [], []
    cfg_parts, q_parts = [], []
    c_off = q_off = k_off = 0
    for p in range(n_progs):
        vl = int(vls[p])
        r0, nm = exps_index[vl]
        fit0.append(p * N_METRICS)
        for j in range(N_METRICS):
            lo, hi = METRIC_RANGES[j]
            s = (hi - lo) / (2.0 * nm)
            pc = rng.uniform(0.1, 2.0, nm)
            qc = np.concatenate([[1.0], rng.uniform(0.1, 2.0, nm - 1)])
            coef_parts.append(np.concatenate([lo * qc + s * pc, qc[1:]]))
            coef0.append(k_off)
            k_off += 2 * nm - 1
            fit_num0.append(r0)
            fit_nn.append(nm)
            sc = np.zeros(MAX_VARS, np.int8)
            sc[0] = 26
            sc[1: 1 + vl] = 10
            scale_rows.append(sc)
        base = config3_launch_configs()[:127] if vl == 2 else pow2_launch_tuples(vl)
        nc = int(rng.integers(n_cfg_range[0], n_cfg_range[1] + 1))
        pick = base[rng.integers(0, base.shape[0], nc)]
        bad = rng.random(nc) < p_bad_cfg
        pick[bad] = rng.integers(1, 96, (int(bad.sum()), vl))
        cfg_parts.append(pick.reshape(-1))
        cfg0.append(c_off)
        c_off += pick.size
        n_cfg.append(nc)
        gk.append(1 if (vl >= 2 and rng.random() < p_2d) else 0)
        nq = int(rng.integers(n_q_range[0], n_q_range[1] + 1))
        q_parts.append(np.rint(2.0 ** rng.uniform(log2_range[0], log2_range[1], nq)).astype(np.int32))
        q0.append(q_off)
        q_off += nq
        n_q.append(nq)
    n_fits = n_progs * N_METRICS
    return ProgramBatch(
        fits=None, coef=np.concatenate(coef_parts), exps=exps,
        num0=np.array(fit_num0, np.int32), n_num=np.array(fit_nn, np.int32),
        den0=np.array(fit_num0, np.int32), n_den=np.array(fit_nn, np.int32),
        coef0=np.array(coef0, np.int64), scale_exp=np.array(scale_rows, np.int8).reshape(n_fits, MAX_VARS),
        v_launch=vls.astype(np.int32), fit0=np.array(fit0, np.int32),
        cfg0=np.array(cfg0, np.int64), n_cfg=np.array(n_cfg, np.int32),
        grid_kind=np.array(gk, np.int32), q0=np.array(q0, np.int64), n_q=np.array(n_q, np.int32),
        cfgs=np.concatenate(cfg_parts).astype(np.int32), queries=np.concatenate(q_parts), hw=HW())


def piecewise_batch(seed: int, n_progs: int = 64, n_q: int = 512, m: int = 240, noise: float = 0.01):
    """Programs with two regimes and a decision between them (a piecewise rational program):
    over (N, bx, by) scaled by (2^26, 2^10, 2^10), the decision d = (c - x_N (1 + a x_bx)) /
    (1 + b x_by) (c ~ U(0.002, 0.05), a, b ~ U(0.1, 2); positive below a data size that moves with
    the block shape) and two costs g_a, g_b, polynomials of total degree <= 2 with coefficients
    U(0.1, 2) (g_b scaled up by 1.5 - 3, the slower regime).  Each program has three fits over
    the monomials of total degree <= 2: d as a rational function (numerator and denominator) from
    m samples over the whole domain (its exact value, a measured quantity such as a working set
    minus a cache size), g_a and g_b as polynomials (denominator 1) from m samples where d >= 0,
    respectively d < 0 (each regime is observed only where it holds), times exp(noise z).  Configurations: the c3 launch set; queries N = round(2^u),
    u ~ U(8, 26).  Returns (FitBatch of 3 n_progs fits, ProgramBatch with the truth's
    coefficients in the fit layout, truth function)."""
    rng = np.random.default_rng(seed)
    E = monomials(3, 2)
    nm = E.shape[0]
    cfgs = config3_launch_configs()
    adm = cfgs[:127]
    sc = np.array([26, 10, 10], np.int8)

    def scaled(X):
        return X.astype(np.float64) * 2.0 ** -sc.astype(np.float64)

    params = []
    samples, truth = [], []
    for p in range(n_progs):
        c = rng.uniform(0.002, 0.05)
        a, b = rng.uniform(0.1, 2.0, 2)
        one = np.zeros(nm)
        one[0] = 1.0
        ga_n, ga_d = rng.uniform(0.1, 2.0, nm), one
        gb_n, gb_d = rng.uniform(0.1, 2.0, nm) * rng.uniform(1.5, 3.0), one
        # d in the monomial basis 1, x_N, x_bx, x_by, x_N^2, x_N x_bx, ...: numerator c - x_N - a x_N x_bx
        d_n = np.zeros(nm)
        d_d = np.zeros(nm)
        d_d[0] = 1.0
        for r in range(nm):
            e = tuple(E[r, :3])
            if e == (0, 0, 0):
                d_n[r] = c
            elif e == (1, 0, 0):
                d_n[r] = -1.0
            elif e == (1, 1, 0):
                d_n[r] = -a
            elif e == (0, 0, 1):
                d_d[r] = b
        params.append((d_n, d_d, ga_n, ga_d, gb_n, gb_d))
        for j, (cn, cd) in enumerate(((d_n, d_d), (ga_n, ga_d), (gb_n, gb_d))):
            Xs = []
            while sum(len(x) for x in Xs) < m:
                N = np.rint(2.0 ** rng.uniform(8, 26, 4 * m)).astype(np.int64)
                L = adm[rng.integers(0, adm.shape[0], 4 * m)]
                X = np.stack([N, L[:, 0], L[:, 1]], 1)
                if j > 0:
                    dv = _truth_value(scaled(X), E[:, :3], E[:, :3], d_n, d_d)
                    X = X[dv >= 0] if j == 1 else X[dv < 0]
                Xs.append(X)
            X = np.concatenate(Xs)[:m]
            f = _truth_value(scaled(X), E[:, :3], E[:, :3], cn, cd)
            if j > 0:
                f = f * np.exp(noise * rng.normal(size=f.shape[0]))
            samples.append((X.astype(np.int32), f))
            truth.append(np.concatenate([cn, cd[1:]]) if j == 0 else cn.copy())
    n_fits = 3 * n_progs
    exps = np.concatenate([E, E])
    # the decision is a full rational fit; the regime costs are polynomials (denominator 1)
    n_den = [nm if i % 3 == 0 else 1 for i in range(n_fits)]
    fb = _pack_fits(samples, exps, [0] * n_fits, [nm] * n_fits, [nm] * n_fits, n_den,
                    np.tile(np.concatenate([sc, np.zeros(5, np.int8)]), (n_fits, 1)), truth=truth,
                    meta={"kind": "piecewise"})
    queries = np.rint(2.0 ** rng.uniform(8, 26, n_progs * n_q)).astype(np.int32)
    pb = ProgramBatch(
        fits=None, coef=fb.truth_coef.copy(), exps=exps, num0=fb.num0, n_num=fb.n_num, den0=fb.den0,
        n_den=fb.n_den, coef0=fb.coef0, scale_exp=fb.scale_exp, v_launch=np.full(n_progs, 2, np.int32),
        fit0=np.arange(n_progs, dtype=np.int32) * 3, cfg0=np.zeros(n_progs, np.int64),
        n_cfg=np.full(n_progs, cfgs.shape[0], np.int32), grid_kind=np.zeros(n_progs, np.int32),
        q0=np.arange(n_progs, dtype=np.int64) * n_q, n_q=np.full(n_progs, n_q, np.int32),
        cfgs=cfgs.reshape(-1).astype(np.int32), queries=queries, hw=HW(), cost_kind=np.full(n_progs, 2, np.int32))

    def truth_costs(prog, N):
        """The generator's regime cost at data sizes N, [n_cfg][len(N)] (+inf where the launch
        constraints fail)."""
        d_n, d_d, ga_n, ga_d, gb_n, gb_d = params[prog]
        out = np.full((cfgs.shape[0], len(N)), np.inf)
        for k in range(cfgs.shape[0]):
            bx, by = int(cfgs[k, 0]), int(cfgs[k, 1])
            T = bx * by
            if T % 64 or T > 1024:
                continue
            X = np.stack([np.asarray(N, np.int64), np.full(len(N), bx), np.full(len(N), by)], 1)
            xt = scaled(X)
            dv = _truth_value(xt, E[:, :3], E[:, :3], d_n, d_d)
            va = _truth_value(xt, E[:, :3], E[:, :3], ga_n, ga_d)
            vb = _truth_value(xt, E[:, :3], E[:, :3], gb_n, gb_d)
            v = np.where(dv >= 0, va, vb)
            out[k] = np.where(np.asarray(N) >= max(bx, by), v, np.inf)
        return out

    return fb, pb, truth_costs


def config5_batch(seed: int, n_progs: int = 16384, n_q: int = 4096, m_range=(64, 1024),
                  n_cfg_range=(32, 512), v_launch_choices=(2, 3, 4), degree: int = 3,
                  noise: float = 0.01, log2_range=(8.0, 26.0), chunk_rows: int = 1 << 18):
    """Large persistent batch: programs with uneven launch grids whose 8 metrics are FITTED.

    Program p: v_launch ~ U(v_launch_choices); n_cfg ~ U{n_cfg_range} configurations drawn
    without replacement from the power-of-two tuples with product in 64..1024 (the 127 config-3
    tuples when v_launch = 2, all of them when fewer exist); n_q data sizes N = round(2^u),
    u ~ U(log2_range).  Its metric j has the ground truth lo_j + s_j p/q of total degree
    <= `degree` in (N/2^26, L_k/2^10) (coefficients U(0.1, 2), q's constant 1, s_j = (hi_j -
    lo_j) / (2 #monomials)).  Fit (p, j) has m ~ U{m_range} samples at (N, L) with N drawn like
    the queries and L one of the program's configurations, target truth * exp(noise z).

    Returns (fits, programs): the FitBatch of all 8 n_progs fits and the ProgramBatch whose
    fit descriptors are the same (its coef holds the ground truth; the workload replaces it by
    the fitted coefficients).  Rows are generated per v_launch class in chunks."""
    rng = np.random.default_rng(seed)
    vls = rng.choice(np.asarray(v_launch_choices), n_progs).astype(np.int32)
    E_of, r0_of, blocks, row = {}, {}, [], 0
    for vl in sorted(set(int(x) for x in vls)):
        E = monomials(1 + vl, degree)
        E_of[vl], r0_of[vl] = E, row
        blocks.append(E)
        row += E.shape[0]
    exps = np.concatenate(blocks)
    n_fits = n_progs * N_METRICS
    nm_p = np.array([E_of[int(v)].shape[0] for v in vls], np.int64)
    nm_f = np.repeat(nm_p, N_METRICS)
    v_f = np.repeat(vls + 1, N_METRICS).astype(np.int32)
    # ground-truth coefficients, fits' layout (numerator lo q + s p, denominator q without q0)
    ncoef = 2 * nm_f - 1
    coef0 = np.zeros(n_fits, np.int64)
    coef0[1:] = np.cumsum(ncoef[:-1])
    coef = np.empty(int(ncoef.sum()))
    cnum, cden = {}, {}           # per v_launch class: [fits of the class][nm]
    fit_ids = {}
    for vl in E_of:
        nm = E_of[vl].shape[0]
        ids = np.nonzero(v_f == vl + 1)[0]
        lo = np.array([METRIC_RANGES[j][0] for j in range(N_METRICS)])[ids % N_METRICS]
        hi = np.array([METRIC_RANGES[j][1] for j in range(N_METRICS)])[ids % N_METRICS]
        sj = (hi - lo) / (2.0 * nm)
        pc = rng.uniform(0.1, 2.0, (ids.size, nm))
        qc = np.concatenate([np.ones((ids.size, 1)), rng.uniform(0.1, 2.0, (ids.size, nm - 1))], axis=1)
        cn = lo[:, None] * qc + sj[:, None] * pc
        cnum[vl], cden[vl], fit_ids[vl] = cn, qc, ids
        for t, i in enumerate(ids):
            coef[coef0[i]: coef0[i] + 2 * nm - 1] = np.concatenate([cn[t], qc[t, 1:]])
    # launch configurations
    n_cfg = rng.integers(n_cfg_range[0], n_cfg_range[1] + 1, n_progs).astype(np.int32)
    base_of = {vl: (config3_launch_configs()[:127] if vl == 2 else pow2_launch_tuples(vl)) for vl in E_of}
    cfg_parts, cfg0, off = [], np.zeros(n_progs, np.int64), 0
    for p in range(n_progs):
        base = base_of[int(vls[p])]
        k = min(int(n_cfg[p]), base.shape[0])
        n_cfg[p] = k
        pick = base[np.sort(rng.choice(base.shape[0], k, replace=False))]
        cfg_parts.append(pick.reshape(-1))
        cfg0[p] = off
        off += pick.size
    cfgs = np.concatenate(cfg_parts).astype(np.int32)
    queries = np.rint(2.0 ** rng.uniform(log2_range[0], log2_range[1], n_progs * n_q)).astype(np.int32)
    # samples
    m = rng.integers(m_range[0], m_range[1] + 1, n_fits).astype(np.int32)
    f0 = np.zeros(n_fits, np.int64)
    f0[1:] = np.cumsum(m.astype(np.int64)[:-1])
    x0 = np.zeros(n_fits, np.int64)
    x0[1:] = np.cumsum((m.astype(np.int64) * v_f)[:-1])
    X = np.empty(int((m.astype(np.int64) * v_f).sum()), np.int32)
    f = np.empty(int(m.sum()))
    for vl in E_of:
        E = E_of[vl][:, :1 + vl].astype(np.int64)
        ids = fit_ids[vl]
        pos = np.empty(n_fits, np.int64)
        pos[ids] = np.arange(ids.size)
        rows_fit = np.repeat(ids, m[ids])                         # fit of every row of the class
        R = rows_fit.size
        Nv = np.rint(2.0 ** rng.uniform(log2_range[0], log2_range[1], R)).astype(np.int64)
        prog = rows_fit // N_METRICS
        pick = (rng.random(R) * n_cfg[prog]).astype(np.int64)
        Lv = cfgs[(cfg0[prog] + pick * vl)[:, None] + np.arange(vl)[None, :]].astype(np.int64)
        Xc = np.concatenate([Nv[:, None], Lv], axis=1)          # [R][1 + vl]
        z = rng.normal(0.0, 1.0, R)
        start = np.repeat(f0[ids], m[ids])
        within = np.arange(R) - np.repeat(np.cumsum(np.concatenate([[0], m[ids][:-1].astype(np.int64)])), m[ids])
        frow = start + within
        xrow = np.repeat(x0[ids], m[ids]) + within * (1 + vl)
        X[xrow[:, None] + np.arange(1 + vl)[None, :]] = Xc.astype(np.int32)
        sdiv = 2.0 ** -np.array([26.0] + [10.0] * vl)

        def chunk(c0, vl=vl, E=E, R=R, Xc=Xc, sdiv=sdiv, pos=pos, rows_fit=rows_fit, frow=frow, z=z):
            c1 = min(R, c0 + chunk_rows)
            xt = Xc[c0:c1].astype(np.float64) * sdiv
            powk = [[np.ones(c1 - c0)] for _ in range(1 + vl)]
            for k in range(1 + vl):
                for d in range(1, degree + 1):
                    powk[k].append(powk[k][-1] * xt[:, k])
            mono = np.empty((c1 - c0, E.shape[0]))
            for t in range(E.shape[0]):
                col = powk[0][E[t, 0]]
                for k in range(1, 1 + vl):
                    if E[t, k]:
                        col = col * powk[k][E[t, k]]
                mono[:, t] = col
            fr = pos[rows_fit[c0:c1]]
            pv = np.einsum("ij,ij->i", mono, cnum[vl][fr])
            qv = np.einsum("ij,ij->i", mono, cden[vl][fr])
            f[frow[c0:c1]] = pv / qv * np.exp(noise * z[c0:c1])

        # chunks write disjoint rows and every random draw is made above, so the thread pool
        # changes nothing but the wall time
        with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
            list(ex.map(chunk, range(0, R, chunk_rows)))
    scale = np.zeros((n_fits, MAX_VARS), np.int8)
    scale[:, 0] = 26
    for k in range(1, 5):
        scale[v_f > k, k] = 10
    num0 = np.array([r0_of[int(v) - 1] for v in v_f], np.int32)
    fits = FitBatch(X=X, f=f, exps=exps, x0=x0, f0=f0, m=m, v=v_f, num0=num0,
                    n_num=nm_f.astype(np.int32), den0=num0.copy(), n_den=nm_f.astype(np.int32),
                    coef0=coef0, scale_exp=scale, n_coef=int(ncoef.sum()), truth_coef=coef.copy(),
                    meta={"noise": noise})
    progs = ProgramBatch(
        fits=fits, coef=coef, exps=exps, num0=fits.num0, n_num=fits.n_num, den0=fits.den0,
        n_den=fits.n_den, coef0=coef0, scale_exp=scale, v_launch=vls,
        fit0=np.arange(n_progs, dtype=np.int32) * N_METRICS, cfg0=cfg0, n_cfg=n_cfg,
        grid_kind=np.zeros(n_progs, np.int32),
        q0=np.arange(n_progs, dtype=np.int64) * n_q, n_q=np.full(n_progs, n_q, np.int32),
        cfgs=cfgs, queries=queries, hw=HW())
    return fits, progs


def mlp_init(seed: int, n_kernels: int, hidden: int = 256):
    """He-uniform initial weights of the surrogate network (bound sqrt(6 / fan_in)), zero
    biases, embeddings U(0, 1).  Returns float32 arrays keyed W1 [h][4], b1, W2 [h][h], b2,
    w3, b3 (shape ()), emb [n_kernels]."""
    rng = np.random.default_rng(seed)
    def he(shape, fan_in):
        b = np.sqrt(6.0 / fan_in)
        return rng.uniform(-b, b, shape).astype(np.float32)
    return {"W1": he((hidden, 4), 4), "b1": np.zeros(hidden, np.float32),
            "W2": he((hidden, hidden), hidden), "b2": np.zeros(hidden, np.float32),
            "w3": he((hidden,), hidden), "b3": np.zeros((), np.float32),
            "emb": rng.uniform(0.0, 1.0, n_kernels).astype(np.float32)}


def surrogate_training_queries(seed: int, pb: "ProgramBatch", n_q: int = 32,
                               log2_range=(8.0, 26.0)) -> "ProgramBatch":
    """The programs of `pb` with fresh training queries: n_q data sizes per program,
    N = round(2^u), u ~ U(log2_range); every configuration of every query is a training sample
    (so configurations are uniform over each program's set)."""
    import copy
    rng = np.random.default_rng(seed)
    out = copy.copy(pb)
    out.queries = np.rint(2.0 ** rng.uniform(log2_range[0], log2_range[1], pb.n_progs * n_q)).astype(np.int32)
    out.q0 = np.arange(pb.n_progs, dtype=np.int64) * n_q
    out.n_q = np.full(pb.n_progs, n_q, np.int32)
    return out


def select_programs(pb: "ProgramBatch", idx) -> "ProgramBatch":
    """The programs `idx` of a batch as a new batch over the same fits, coefficients,
    configurations and queries (only the per-program arrays are subset)."""
    import copy
    idx = np.asarray(idx, np.int64)
    out = copy.copy(pb)
    out.v_launch, out.fit0, out.cfg0 = pb.v_launch[idx], pb.fit0[idx], pb.cfg0[idx]
    out.n_cfg, out.grid_kind, out.q0, out.n_q = pb.n_cfg[idx], pb.grid_kind[idx], pb.q0[idx], pb.n_q[idx]
    return out


def take_programs(pb: "ProgramBatch", n: int) -> "ProgramBatch":
    """The first n programs of a batch (their fits, configurations and queries), re-based."""
    import copy
    out = copy.copy(pb)
    nf = n * N_METRICS
    out.num0, out.n_num, out.den0, out.n_den = pb.num0[:nf], pb.n_num[:nf], pb.den0[:nf], pb.n_den[:nf]
    out.coef0, out.scale_exp = pb.coef0[:nf], pb.scale_exp[:nf]
    out.coef = pb.coef[: int(pb.coef0[nf - 1] + pb.n_num[nf - 1] + pb.n_den[nf - 1] - 1)]
    out.v_launch, out.fit0, out.cfg0 = pb.v_launch[:n], pb.fit0[:n], pb.cfg0[:n]
    out.n_cfg, out.grid_kind, out.n_q = pb.n_cfg[:n], pb.grid_kind[:n], pb.n_q[:n]
    qend = int(pb.q0[n - 1] + pb.n_q[n - 1])
    out.q0, out.queries = pb.q0[:n], pb.queries[:qend]
    return out

"""Oracle: rational-program evaluation over launch configurations and brute-force argmin.

Test infrastructure only (see the package docstring); never imported by the product path.

What it follows.
  * Occupancy: the flowchart of the paper's Example "Hardware occupancy" (figure of the
    occupancy rational program) deciding B_active by four guarded branches plus the failure
    terminal, and eq. (occupancy) W_active = min(floor(B_active T / wave), W_max).  The warp
    width 32 of the paper is the wavefront width `wave` here; R_max and Z_max are per compute
    unit.
  * Execution time: the paper's Example "execution time" names the MWP-CWP model (Hong & Kim)
    without printing its equations; the cycle estimate below is this project's normative
    MWP-CWP-style reading (memory warp parallelism, computation warp parallelism, three cases,
    synchronisation term, repetitions = blocks over resident blocks of all CUs).
  * Grid: blocks = ceil(N / prod L) for one-dimensional data, ceil(N/bx) * ceil(N/by) for the
    two-dimensional example of section "Annotating the source code".
  * Admissible ("practically meaningful") configurations: T = prod L is a multiple of the wave
    and at most T_max (section "An Algorithm ...", discussion of F), every launch parameter is at
    most N (the constraint-file example, read non-strictly), every fitted metric has q > 0 and a
    finite value, B_active >= 1, and the cost is finite.
  * Selection (step 5): exhaustive search, strict "<" in configuration order, so ties go to the
    lowest index; no admissible configuration gives -1 and +inf.
  * A program may instead take its one fitted function as the cost (the sampled metric was the
    quantity to minimise), with the same launch constraints and no occupancy or grid terms; or
    be piecewise, a fitted decision function choosing between two fitted cost functions.

Two precisions:
  truth  - FP64: each metric is the full multivariate p/q evaluated directly at (N~, L~).
  replay - FP32: the normative FP32 operation sequence: per (program, config) the metric
           polynomials are collapsed to polynomials in N~ (FP64, monomial order, then rounded to
           FP32); per point Horner by fused multiply-add (one rounding per step), the a*b + c
           terms of the cycle estimate fused the same way, every other operation rounded on its
           own, correctly rounded division, explicit compare-select min/max, exact integer
           parts.  The argmin is decided in this precision on both sides.

Fused multiply-add in FP32 (fma32): a*b is exact in FP64 (two 24-bit significands); the FP64 sum
with a*b is rounded to odd (the exact error of the FP64 addition, from the two-sum, decides
whether the result moves to its odd neighbour), and rounding that to FP32 by round-to-nearest-even
gives the correctly rounded a*b + c, since FP64 carries more than FP32's precision plus two bits
(Boldo and Melquiond, "Emulation of FMA and correctly rounded sums: proved algorithms using
rounding to odd", IEEE Trans. Computers 57(4), 2008).

Metric order: I_comp, I_mc, I_mu, U, I_sync, R, Z, B_w.
"""
from __future__ import annotations

import numpy as np

N_METRICS = 8
MAX_NDEG = 3     # highest power of N~ in a collapsed metric polynomial


# ---------------------------------------------------------------------------------------------
# occupancy

def occupancy_flowchart(T, R, Z, hw):
    """B_active by the paper's four-branch flowchart, exact integer (int64) arithmetic.

    T threads per block, R registers per thread (>= 1), Z LDS bytes per block (>= 0)."""
    T = np.asarray(T, np.int64)
    R = np.asarray(R, np.int64)
    Z = np.asarray(Z, np.int64)
    W = np.int64(hw.wave * hw.w_max)     # resident threads per CU, "32 W_max" of the paper
    Bm, Rm, Zm = np.int64(hw.b_max), np.int64(hw.r_max), np.int64(hw.z_max)
    c1 = (T * Bm <= W) & (R * T * Bm <= Rm) & (Z * Bm <= Zm)
    c2 = (W <= T * Bm) & (W * R <= Rm) & (W * Z <= Zm * T)
    c3 = (Rm <= R * T * Bm) & (Rm <= R * W) & (Rm * Z <= R * T * Zm)
    c4 = (Zm <= Bm * Z) & (Zm * T <= W * Z) & (Zm * R * T <= Z * Rm)
    Zs = np.where(Z > 0, Z, 1)
    return np.select([c1, c2, c3, c4],
                     [np.broadcast_to(Bm, T.shape), W // T, Rm // (R * T), Zm // Zs],
                     default=0).astype(np.int64)


def waves_active(B, T, hw):
    """eq. (occupancy): W_active = min(floor(B_active T / wave), W_max)."""
    return np.minimum((np.asarray(B, np.int64) * T) // hw.wave, hw.w_max)


# ---------------------------------------------------------------------------------------------
# metric polynomials

def _mono(values, e):
    """prod_k values[k]^e[k] by repeated multiplication in variable order (FP64)."""
    acc = np.float64(1.0) if np.ndim(values[0]) == 0 else np.ones_like(values[0])
    for k, vk in enumerate(values):
        for _ in range(int(e[k])):
            acc = acc * vk
    return acc


def metric_truth(coef, E_num, E_den, s, N, L):
    """FP64 value of p/q at data size N (array) and launch tuple L (ints); returns (p, q)."""
    v = E_num.shape[1]
    vals = [np.ldexp(np.asarray(N, np.float64), -int(s[0]))]
    vals += [np.float64(np.ldexp(float(L[k - 1]), -int(s[k]))) for k in range(1, v)]
    nn = E_num.shape[0]
    p = np.zeros_like(vals[0])
    for t in range(nn):
        p = p + coef[t] * _mono(vals, E_num[t])
    q = np.ones_like(vals[0])
    for t in range(1, E_den.shape[0]):
        q = q + coef[nn + t - 1] * _mono(vals, E_den[t])
    return p, q


def collapse(coef, E_num, E_den, s, L):
    """Polynomials in N~ of one metric at a fixed launch tuple L.

    FP64: a_d = sum over monomials (in order) with N-exponent d of coef * prod_k L~_k^e_k,
    accumulated left to right with separately rounded multiply and add; then each a_d is
    rounded to FP32.  Returns (num[MAX_NDEG+1], den[MAX_NDEG+1]) float32, index = power."""
    v = E_num.shape[1]
    Lt = [np.float64(np.ldexp(float(L[k - 1]), -int(s[k]))) for k in range(1, v)]
    nn = E_num.shape[0]
    a = [np.float64(0.0)] * (MAX_NDEG + 1)
    for t in range(nn):
        mono = np.float64(1.0)
        for k in range(1, v):
            for _ in range(int(E_num[t, k])):
                mono = mono * Lt[k - 1]
        d = int(E_num[t, 0])
        a[d] = a[d] + np.float64(coef[t]) * mono
    b = [np.float64(0.0)] * (MAX_NDEG + 1)
    for t in range(E_den.shape[0]):
        c = np.float64(1.0) if t == 0 else np.float64(coef[nn + t - 1])
        mono = np.float64(1.0)
        for k in range(1, v):
            for _ in range(int(E_den[t, k])):
                mono = mono * Lt[k - 1]
        d = int(E_den[t, 0])
        b[d] = b[d] + c * mono
    return np.array(a, np.float32), np.array(b, np.float32)


def fma32(a, b, c):
    """Correctly rounded FP32 a*b + c (one rounding), elementwise, by rounding to odd in FP64."""
    a, b, c = np.broadcast_arrays(np.asarray(a, np.float32), np.asarray(b, np.float32),
                                  np.asarray(c, np.float32))
    with np.errstate(all="ignore"):
        p = a.astype(np.float64) * b.astype(np.float64)          # exact
        c64 = c.astype(np.float64)
        s = p + c64
        bv = s - p                                                # two-sum: s + e = p + c exactly
        e = (p - (s - bv)) + (c64 - bv)
        even = (s.view(np.int64) & 1) == 0
        move = np.isfinite(s) & np.isfinite(e) & (e != 0) & even
        toward = np.where(e > 0, np.inf, -np.inf)
        s = np.where(move, np.nextafter(s, toward), s)
        return s.astype(np.float32)


def _fma(a, b, c, dt):
    """a*b + c with one rounding in the replay (FP32); plain FP64 arithmetic for the truth."""
    if dt == np.float32:
        return fma32(a, b, c)
    return np.asarray(a, dt) * np.asarray(b, dt) + np.asarray(c, dt)


def horner32(c, x):
    """FP32 Horner over powers MAX_NDEG..0 by fused multiply-add (zero padding at the top is exact)."""
    acc = np.full(x.shape, c[MAX_NDEG], np.float32)
    for d in range(MAX_NDEG - 1, -1, -1):
        acc = fma32(acc, x, c[d])
    return acc


# ---------------------------------------------------------------------------------------------
# the cycle estimate

def _min(a, b):
    return np.where(b < a, b, a)


def _max(a, b):
    return np.where(b > a, b, a)


def cycles_from_metrics(g, N, L, grid_kind, hw, dt):
    """Cost of one configuration L at data sizes N (1-D int array) from metric values g[8][nq].

    dt is np.float64 (truth) or np.float32 (replay); every floating operation stays in dt.
    Inadmissible points get +inf."""
    F = dt
    N = np.asarray(N, np.int64)
    L = [int(x) for x in L]
    T = int(np.prod(L))
    ok = np.ones(N.shape, bool)
    ok &= (T <= hw.t_max) and (T % hw.wave == 0) and all(x >= 1 for x in L)
    ok &= N >= max(L)
    with np.errstate(all="ignore"):
        for j in range(N_METRICS):
            ok &= np.isfinite(g[j])
        gz = [np.where(np.isfinite(g[j]), g[j], F(0)).astype(dt) for j in range(N_METRICS)]
        Icomp = _max(gz[0], F(0))
        Imc = _max(gz[1], F(0))
        Imu = _max(gz[2], F(0))
        U = _max(gz[3], F(1))
        Isync = _max(gz[4], F(0))
        Rc = _min(_max(np.ceil(gz[5]), F(1)), F(2 ** 24)).astype(np.int64)
        Zc = _min(_max(np.ceil(gz[6]), F(0)), F(2 ** 24)).astype(np.int64)
        Bw = _max(gz[7], F(1))

        B = occupancy_flowchart(np.full(N.shape, T, np.int64), Rc, Zc, hw)
        ok &= B >= 1
        Bs = np.where(B >= 1, B, 1)
        Nw = waves_active(Bs, T, hw)
        if grid_kind == 0:
            blocks = (N - 1) // T + 1
        else:
            blocks = ((N - 1) // L[0] + 1) * ((N - 1) // L[1] + 1)
        rep = (blocks - 1) // (Bs * hw.n_cu) + 1
        Nwf = Nw.astype(dt)
        repf = rep.astype(dt)
        Bf = Bs.astype(dt)
        lat, dep = F(hw.mem_lat), F(hw.dep_delay)
        iss, bw = F(hw.issue_cycles), F(hw.bw)

        Im = Imc + Imu
        Lu = _fma(U - F(1), dep, lat, dt)            # (U - 1) dep + lat
        mem = _fma(Lu, Imu, lat * Imc, dt)           # lat I_mc + L_u I_mu
        comp = Icomp + Im
        comp = iss * comp

        # memory-bound branch quantities (computed everywhere, selected where Im > 0)
        d1 = _fma(U, Imu, Imc, dt)                   # I_mc + U I_mu
        d1 = dep * d1
        mwp_lat = mem / d1
        n2 = bw * mem
        d2 = Im * Bw
        mwp_bw = n2 / d2
        mwp = _min(mwp_lat, mwp_bw)
        mwp = _min(mwp, Nwf)
        mwp = _max(mwp, F(1))
        tot = mem + comp
        cwp_full = tot >= Nwf * comp
        cwp_ge_mwp = tot >= mwp * comp
        cpm = comp / Im
        m1 = mwp - F(1)
        e1 = _fma(cpm, m1, tot, dt)                  # tot + cpm (MWP - 1)
        t2 = mem * Nwf
        t2 = t2 / mwp
        e2 = _fma(cpm, m1, t2, dt)                   # mem N_w / MWP + cpm (MWP - 1)
        e3 = _fma(comp, Nwf, lat, dt)                # lat + comp N_w
        case1 = (mwp >= Nwf) & cwp_full
        case2 = cwp_ge_mwp | (comp > mem)
        ex_mem = np.where(case1, e1, np.where(case2, e2, e3))

        pure = Im == F(0)
        mwp = np.where(pure, F(1), mwp)
        ex = np.where(pure, comp * Nwf, ex_mem)

        sy = mwp - F(1)
        sy = dep * sy
        sy = sy * Isync
        sy = sy * Bf
        sy = sy * repf
        cost = _fma(ex, repf, sy, dt)                # exec rep + sync
        ok &= np.isfinite(cost)
    return np.where(ok, cost, dt(np.inf)).astype(dt)


# ---------------------------------------------------------------------------------------------
# programs

COST_CYCLES, COST_METRIC, COST_PIECEWISE = 0, 1, 2


def cost_kind(pb, prog):
    """KLR_COST_CYCLES (the cycle estimate from 8 metrics) or KLR_COST_METRIC (the program's one
    fitted function is the cost)."""
    ck = getattr(pb, "cost_kind", None)
    return COST_CYCLES if ck is None else int(ck[prog])


def metric_cost(g, N, L, hw):
    """Cost of a program whose one fitted function g = p/q is the cost (the rational program
    is the fitted metric itself, e.g. when the sampled metric was the kernel's time): g where q > 0
    and the value is finite and the launch constraints hold (every L >= 1 and <= N, T = prod L a
    multiple of the wave and <= T_max); +inf elsewhere."""
    N = np.asarray(N, np.int64)
    L = [int(x) for x in L]
    T = int(np.prod(L))
    ok = np.isfinite(g) & (N >= max(L))
    ok &= (T <= hw.t_max) and (T % hw.wave == 0) and all(x >= 1 for x in L)
    return np.where(ok, g, np.inf).astype(np.asarray(g).dtype)


def piecewise_cost(d, ga, gb, N, L, hw):
    """A piecewise rational program whose decision node is a fitted function too (the paper
    remarks that a decision node is given by rational functions, so it can be determined by
    curve fitting like the metrics): cost ga where d >= 0, gb elsewhere; +inf where d or the
    branch taken is invalid (q <= 0 or not finite) or the launch constraints fail.  Invalid
    values arrive as NaN."""
    d = np.asarray(d)
    take_a = d >= 0
    g = np.where(take_a, ga, gb)
    return metric_cost(np.where(np.isfinite(d), g, np.nan).astype(d.dtype), N, L, hw)


def program_metrics(pb, prog):
    return {COST_METRIC: 1, COST_PIECEWISE: 3}.get(cost_kind(pb, prog), N_METRICS)


def _metric_slices(pb, prog):
    out = []
    for j in range(program_metrics(pb, prog)):
        fi = int(pb.fit0[prog]) + j
        v = 1 + int(pb.v_launch[prog])
        En = pb.exps[pb.num0[fi]: pb.num0[fi] + pb.n_num[fi], :v]
        Ed = pb.exps[pb.den0[fi]: pb.den0[fi] + pb.n_den[fi], :v]
        nc = En.shape[0] + Ed.shape[0] - 1
        c = pb.coef[pb.coef0[fi]: pb.coef0[fi] + nc]
        out.append((c, En, Ed, pb.scale_exp[fi, :v]))
    return out


def program_configs(pb, prog):
    vl = int(pb.v_launch[prog])
    c0 = int(pb.cfg0[prog])
    return pb.cfgs[c0: c0 + int(pb.n_cfg[prog]) * vl].reshape(-1, vl)


def program_costs(pb, prog, query_idx=None, mode="replay", coef=None):
    """Costs [n_cfg][nq] of one program at its queries (optionally a subset, by index)."""
    if coef is not None:
        pb = _with_coef(pb, coef)
    q0, nq = int(pb.q0[prog]), int(pb.n_q[prog])
    N = pb.queries[q0: q0 + nq].astype(np.int64)
    if query_idx is not None:
        N = N[np.asarray(query_idx)]
    cfgs = program_configs(pb, prog)
    mets = _metric_slices(pb, prog)
    gk = int(pb.grid_kind[prog])
    dt = np.float32 if mode == "replay" else np.float64
    out = np.empty((cfgs.shape[0], N.shape[0]), dt)
    if mode == "replay":
        x = np.ldexp(N.astype(np.float32), -int(mets[0][3][0])).astype(np.float32)
    for c in range(cfgs.shape[0]):
        g = []
        for (cf, En, Ed, s) in mets:
            if mode == "replay":
                a, b = collapse(cf, En, Ed, s, cfgs[c])
                xs = np.ldexp(N.astype(np.float32), -int(s[0])).astype(np.float32)
                p = horner32(a, xs)
                q = horner32(b, xs)
                with np.errstate(all="ignore"):
                    val = p / q
                g.append(np.where(q > np.float32(0), val, np.float32(np.nan)))
            else:
                p, q = metric_truth(cf, En, Ed, s, N, cfgs[c])
                with np.errstate(all="ignore"):
                    val = p / q
                g.append(np.where(q > 0, val, np.nan))
        if cost_kind(pb, prog) == COST_METRIC:
            out[c] = metric_cost(g[0], N, cfgs[c], pb.hw)
        elif cost_kind(pb, prog) == COST_PIECEWISE:
            out[c] = piecewise_cost(g[0], g[1], g[2], N, cfgs[c], pb.hw)
        else:
            out[c] = cycles_from_metrics(g, N, cfgs[c], gk, pb.hw, dt)
    return out


def argmin_lowest(costs):
    """Brute force over configurations in index order: strict "<", so ties keep the lowest
    index; NaN and +inf never win; nothing admissible gives (-1, +inf)."""
    n_cfg, nq = costs.shape
    best = np.full(nq, np.inf, costs.dtype)
    idx = np.full(nq, -1, np.int32)
    for c in range(n_cfg):
        better = costs[c] < best
        best = np.where(better, costs[c], best)
        idx = np.where(better, np.int32(c), idx)
    return idx, best


def program_argmin(pb, prog, query_idx=None, mode="replay", coef=None):
    return argmin_lowest(program_costs(pb, prog, query_idx, mode, coef))


def _with_coef(pb, coef):
    import copy
    pb2 = copy.copy(pb)
    pb2.coef = coef
    return pb2

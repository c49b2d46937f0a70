"""Pins of the evaluation / argmin oracle against things the paper and arithmetic fix."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import cost as oc
from paper_1911_02373_amd import synth
from tests.helpers import constant_programs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cost_cases.json")


def _closed_form_occupancy(T, R, Z, hw):
    """B_active = min(B_max, floor(wave W_max / T), floor(R_max / (R T)), floor(Z_max / Z))."""
    cand = [hw.b_max, (hw.wave * hw.w_max) // T, hw.r_max // (R * T)]
    if Z > 0:
        cand.append(hw.z_max // Z)
    return min(cand)


@pytest.mark.parametrize("hw", [
    synth.HW(),
    # the paper's CUDA setting: warp 32, 64 warps and 32 blocks per SM, 64K registers,
    # 48 KiB shared memory
    synth.HW(wave=32, w_max=64, b_max=32, r_max=65536, z_max=49152),
    synth.HW(wave=64, w_max=40, b_max=16, r_max=98304, z_max=65536),
])
def test_occupancy_flowchart_equals_closed_form(hw):
    Ts = list(range(hw.wave, 1025, hw.wave)) + [1, 3, 17, 100]
    Rs = list(range(1, 260, 3))
    Zs = [0, 1, 7, 100, 1000, 4096, 6000, 16384, 20000, 40000, 49152, 65536, 100000, 163840, 200000]
    T, R, Z = (np.array(a) for a in zip(*itertools.product(Ts, Rs, Zs)))
    got = oc.occupancy_flowchart(T, R, Z, hw)
    want = np.array([_closed_form_occupancy(t, r, z, hw) for t, r, z in zip(T, R, Z)])
    assert np.array_equal(got, want)


def test_occupancy_eq_waves():
    hw = synth.HW()
    # eq. (occupancy): W_active = min(floor(B T / wave), W_max)
    assert oc.waves_active(8, 256, hw) == 32
    assert oc.waves_active(1, 512, hw) == 8
    assert oc.waves_active(32, 1024, hw) == 32


@pytest.mark.parametrize("mode", ["replay", "truth"])
def test_hand_derived_costs(mode):
    cases = json.load(open(GOLDEN))["cases"]
    for cs in cases:
        pb = constant_programs([cs["metrics"]], [cs["L"]], [[cs["N"]]], grid_kind=cs["grid"])
        c = oc.program_costs(pb, 0, mode=mode)[0, 0]
        want = np.inf if cs["expect"] == "inf" else cs["expect"]
        assert c == want, (cs["name"], c, want)


def test_argmin_ties_lowest_index_and_none_admissible():
    costs = np.array([[3.0, np.inf, 5.0, np.nan],
                      [2.0, np.inf, 5.0, np.nan],
                      [2.0, np.inf, 4.0, np.inf],
                      [np.nan, np.inf, 4.0, np.inf]], np.float32)
    idx, best = oc.argmin_lowest(costs)
    assert idx.tolist() == [1, -1, 2, -1]
    assert best[0] == 2.0 and best[2] == 4.0 and np.isinf(best[1]) and np.isinf(best[3])


def test_argmin_matches_numpy_first_occurrence():
    rng = np.random.default_rng(5)
    costs = rng.integers(0, 6, (37, 500)).astype(np.float32)   # many exact ties
    idx, best = oc.argmin_lowest(costs)
    assert np.array_equal(idx, np.argmin(costs, axis=0))
    assert np.array_equal(best, costs.min(axis=0))


def test_duplicate_configs_tie_to_lowest_index():
    pb = synth.config3_programs(3, n_progs=2, n_q=64)
    base = synth.config3_launch_configs()[:40]
    dup = np.concatenate([base, base])          # every cost appears twice
    pb.cfgs = dup.reshape(-1)
    pb.n_cfg[:] = dup.shape[0]
    for p in range(2):
        costs = oc.program_costs(pb, p)
        assert np.array_equal(costs[:40], costs[40:])
        idx, _ = oc.argmin_lowest(costs)
        assert np.all(idx < 40)


def test_collapse_matches_direct_evaluation():
    pb = synth.config3_programs(11, n_progs=3, n_q=200)
    cfgs = synth.config3_launch_configs()
    rng = np.random.default_rng(0)
    for prog in range(3):
        mets = oc._metric_slices(pb, prog)
        N = pb.queries[pb.q0[prog]: pb.q0[prog] + 200].astype(np.int64)
        for c in rng.choice(127, 12, replace=False):
            for cf, En, Ed, s in mets:
                a, b = oc.collapse(cf, En, Ed, s, cfgs[c])
                x = np.ldexp(N.astype(np.float64), -int(s[0]))
                pc = sum(float(a[d]) * x ** d for d in range(4))
                qc = sum(float(b[d]) * x ** d for d in range(4))
                p, q = oc.metric_truth(cf, En, Ed, s, N, cfgs[c])
                # FP32 rounding of the collapsed coefficients only
                assert np.allclose(pc, p, rtol=3e-7, atol=0)
                assert np.allclose(qc, q, rtol=3e-7, atol=0)


def test_replay_close_to_truth():
    pb = synth.config3_programs(21, n_progs=4, n_q=512)
    for prog in range(4):
        c32 = oc.program_costs(pb, prog, mode="replay").astype(np.float64)
        c64 = oc.program_costs(pb, prog, mode="truth")
        fin = np.isfinite(c32) & np.isfinite(c64)
        # admissibility agrees except where an FP32 ceil / compare flips
        assert np.mean(np.isfinite(c32) == np.isfinite(c64)) > 0.999
        rel = np.abs(c32[fin] - c64[fin]) / c64[fin]
        assert np.median(rel) < 1e-6
        assert np.mean(rel < 1e-4) > 0.999


def test_cost_non_decreasing_in_N_for_constant_metrics():
    rows = [[100, 10, 2, 3, 1, 40, 2048, 128], [2000, 50, 0, 1, 0, 64, 0, 256]]
    Ns = np.arange(1024, 1 << 22, 4093)
    cfgs = synth.config3_launch_configs()[:127]
    pb = constant_programs(rows, cfgs, [Ns, Ns])
    for p in range(2):
        c = oc.program_costs(pb, p, mode="truth")
        fin = np.isfinite(c).all(axis=1)
        assert np.all(np.diff(c[fin], axis=1) >= 0)


def test_config3_launch_configs():
    cfg = synth.config3_launch_configs()
    assert cfg.shape == (128, 2)
    T = cfg[:127, 0] * cfg[:127, 1]
    assert np.all(T % 64 == 0) and np.all(T <= 1024) and len(set(map(tuple, cfg[:127]))) == 127
    # the pad is never admissible
    pb = synth.config3_programs(1, n_progs=1, n_q=100)
    assert np.all(np.isinf(oc.program_costs(pb, 0)[127]))


# ---------------------------------------------------------------------------------------------
# FP32 fused multiply-add of the replay, against exact rational arithmetic

def _round_f32_exact(x):
    """Correctly rounded (nearest, ties to even) FP32 of an exact Fraction, by comparing the
    FP32 neighbours of a nearby candidate exactly."""
    from fractions import Fraction
    f = np.float32(float(x))
    cands = [np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))]
    best = None
    for c in cands:
        if not np.isfinite(c):
            continue
        d = abs(Fraction(float(c)) - x)
        if best is None or d < best[0] or (d == best[0] and (int(np.float32(c).view(np.int32)) & 1) == 0):
            best = (d, c)
    return np.float32(best[1])


def _fma_exact(a, b, c):
    from fractions import Fraction
    return _round_f32_exact(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def test_fma32_matches_exact_rounding_on_random_inputs():
    rng = np.random.default_rng(7)
    n = 3000
    a = (rng.standard_normal(n) * 2.0 ** rng.integers(-20, 20, n)).astype(np.float32)
    b = (rng.standard_normal(n) * 2.0 ** rng.integers(-20, 20, n)).astype(np.float32)
    c = (rng.standard_normal(n) * 2.0 ** rng.integers(-30, 30, n)).astype(np.float32)
    c[: n // 3] = -(a[: n // 3] * b[: n // 3])                # near cancellation
    got = oc.fma32(a, b, c)
    want = np.array([_fma_exact(x, y, z) for x, y, z in zip(a, b, c)], np.float32)
    assert np.array_equal(got.view(np.int32), want.view(np.int32))


def test_fma32_single_rounding_where_double_rounding_fails():
    """a b + c lands a hair off an FP32 halfway point, inside FP64's last place: rounding to FP64
    first produces an exact tie that ties-to-even resolves the wrong way; one rounding does not."""
    cases = []
    for i in (1, 3, 77, 300):
        for c in (np.float32(1 + 2.0 ** -23), np.float32(3.0 + 2.0 ** -22), np.float32(-(1 + 2.0 ** -23))):
            ulp = float(np.spacing(np.float32(abs(c))))
            a = np.float32(1 + i * 2.0 ** -23)
            b = np.float32((1 - i * 2.0 ** -23) * ulp / 2)     # a b = ulp/2 (1 - i^2 2^-46)
            cases.append((a, b, c))
            cases.append((a, np.float32(-b), c))
    naive_wrong = 0
    for a, b, c in cases:
        want = _fma_exact(a, b, c)
        got = oc.fma32(np.float32(a), np.float32(b), np.float32(c))
        assert got.view(np.int32) == want.view(np.int32), (a, b, c, got, want)
        naive = np.float32(float(a) * float(b) + float(c))
        naive_wrong += int(naive != want)
    assert naive_wrong >= len(cases) // 2      # the cases do separate one rounding from two


def test_fma32_special_values():
    inf, nan = np.float32(np.inf), np.float32(np.nan)
    assert oc.fma32(np.float32(2), np.float32(3), np.float32(1)) == np.float32(7)
    assert oc.fma32(np.float32(0), np.float32(5), np.float32(-0.0)).view(np.int32) == 0   # +0
    assert oc.fma32(inf, np.float32(1), np.float32(1)) == inf
    assert np.isnan(oc.fma32(inf, np.float32(0), np.float32(1)))
    assert np.isnan(oc.fma32(inf, np.float32(1), -inf))
    assert np.isnan(oc.fma32(nan, np.float32(1), np.float32(1)))
    big = np.float32(3e38)
    assert oc.fma32(big, np.float32(2), np.float32(0)) == inf


def _generator_truth(pb, fi, j, N, L):
    """lo_j + s_j p/q of fit fi at (N, L), from the generator's own description of the c3
    programs (numerator coefficients lo_j q + s_j p, q's constant 1, total degree <= 2 in
    (N/2^26, bx/2^10, by/2^10)), evaluated with numpy powers: no code shared with the oracle."""
    E = synth.monomials(3, 2)[:, :3].astype(np.float64)
    nm = E.shape[0]
    c = pb.coef[fi * (2 * nm - 1): (fi + 1) * (2 * nm - 1)]
    q = np.concatenate([[1.0], c[nm:]])
    lo, hi = synth.METRIC_RANGES[j]
    s = (hi - lo) / 20.0
    p = (c[:nm] - lo * q) / s
    x = np.stack([np.asarray(N, np.float64) / 2.0 ** 26, np.full(len(N), L[0] / 2.0 ** 10),
                  np.full(len(N), L[1] / 2.0 ** 10)], axis=1)
    mono = np.prod(x[:, None, :] ** E[None, :, :], axis=2)
    return lo + s * (mono @ p) / (mono @ q)


def test_metric_truth_and_collapse_match_the_generators_metrics():
    """metric_truth (p/q of each metric's own coefficient slice) and the FP32 collapse of the
    same slice, against the generator's lo_j + s_j p/q for non-constant metrics of c3 programs:
    a wrong coefficient slice, scale exponent or denominator constant fails here."""
    pb = synth.config3_programs(12, n_progs=3, n_q=300)
    cfgs = synth.config3_launch_configs()
    rng = np.random.default_rng(3)
    for prog in range(3):
        N = pb.queries[pb.q0[prog]: pb.q0[prog] + 300].astype(np.int64)
        mets = oc._metric_slices(pb, prog)
        for c in rng.choice(127, 10, replace=False):
            for j, (cf, En, Ed, s) in enumerate(mets):
                want = _generator_truth(pb, int(pb.fit0[prog]) + j, j, N, cfgs[c])
                p, q = oc.metric_truth(cf, En, Ed, s, N, cfgs[c])
                assert np.allclose(p / q, want, rtol=1e-12, atol=0), (prog, c, j)
                a, b = oc.collapse(cf, En, Ed, s, cfgs[c])
                x = np.asarray(N, np.float64) / 2.0 ** 26
                val = np.polyval(a[::-1].astype(np.float64), x) / np.polyval(b[::-1].astype(np.float64), x)
                assert np.allclose(val, want, rtol=2e-6, atol=0), (prog, c, j)


def test_metric_truth_matches_fitted_rational_value():
    """A metric fitted by the oracle's least squares and read back through a program's
    coefficient layout: metric_truth equals oracle.fit.rational_value at the same points (both
    are p/q of the fitted coefficients), and noise-free samples give back the generator's truth."""
    from oracle import fit as of
    pb = synth.config3_programs(13, n_progs=1, n_q=64)
    cfgs = synth.config3_launch_configs()
    rng = np.random.default_rng(4)
    E = synth.monomials(3, 2)
    nm = E.shape[0]
    for j in range(synth.N_METRICS):
        # 120 samples of metric j at (N, bx, by) on the program's configurations
        Ns = np.rint(2.0 ** rng.uniform(8, 26, 120)).astype(np.int64)
        cs = cfgs[rng.integers(0, 127, 120)]
        f = np.array([_generator_truth(pb, j, j, Ns[i:i + 1], cs[i])[0] for i in range(120)])
        Xi = np.stack([Ns, cs[:, 0], cs[:, 1]], 1).astype(np.int32)
        s = np.array([26, 10, 10], np.int8)
        coef, info = of.fit_one(Xi, f, E[:, :3], E[:, :3], s)
        assert info["rank"] == 2 * nm - 1
        for c in rng.choice(127, 4, replace=False):
            N = np.rint(2.0 ** rng.uniform(8, 26, 50)).astype(np.int64)
            p, q = oc.metric_truth(coef, E[:, :3], E[:, :3], s, N, cfgs[c])
            Xq = np.stack([N, np.full(50, cfgs[c][0]), np.full(50, cfgs[c][1])], 1).astype(np.int32)
            rv = of.rational_value(Xq, E[:, :3], E[:, :3], s, coef)
            assert np.allclose(p / q, rv, rtol=1e-12, atol=0), (j, c)
            assert np.allclose(p / q, _generator_truth(pb, j, j, N, cfgs[c]), rtol=1e-7, atol=0), (j, c)


def test_metric_cost_program_is_the_fitted_function():
    """A program whose one fitted function is the cost (the single-fit workload: N = 2^10..2^20,
    B = 32..1024 step 32): in FP64 its cost matrix is oracle.fit.rational_value of the fitted
    coefficients on the grid, the FP32 replay agrees to FP32 rounding, and the argmin over B per
    N is numpy's argmin of the fitted values (first index among equal values)."""
    from oracle import fit as of
    fb = synth.config1_fit(3)
    coef, info = of.fit_batch(fb)
    pb = synth.config1_program(fb, coef)
    c64 = oc.program_costs(pb, 0, mode="truth")
    c32 = oc.program_costs(pb, 0, mode="replay")
    Ns, Bs = pb.queries, pb.cfgs
    Xq = np.array([(n, b) for b in Bs for n in Ns], np.int32)
    Xi, fi, En, Ed, s = fb.fit_arrays(0)
    rv = of.rational_value(Xq, En, Ed, s, coef).reshape(Bs.size, Ns.size)
    assert np.all(np.isfinite(rv))
    assert np.allclose(c64, rv, rtol=1e-13, atol=0)
    assert np.allclose(c32, rv, rtol=1e-6, atol=0)
    idx, best = oc.argmin_lowest(c64)
    assert np.array_equal(idx, np.argmin(rv, axis=0)) and np.allclose(best, rv.min(axis=0), rtol=1e-13, atol=0)
    # the launch constraints still apply: B above N or off the wave is inadmissible
    pb2 = synth.config1_program(fb, coef)
    pb2.queries = np.array([500, 1 << 12], np.int32)
    pb2.n_q = np.array([2], np.int32)
    pb2.hw = synth.HW(wave=64)
    c = oc.program_costs(pb2, 0, mode="truth")
    assert np.all(np.isinf(c[Bs > 500, 0])) and np.all(np.isinf(c[Bs % 64 != 0]))
    assert np.all(np.isfinite(c[(Bs <= 500) & (Bs % 64 == 0), 0]))


def test_metric_cost_noise_free_fit_recovers_truth_decisions():
    """Noise-free samples: the fitted rational function is the generator's, so its per-N argmin
    over B is the truth's."""
    from oracle import fit as of
    fb = synth.config1_fit(5, noise=0.0)
    coef, _ = of.fit_batch(fb)
    pb = synth.config1_program(fb, coef)
    idx, _ = oc.argmin_lowest(oc.program_costs(pb, 0, mode="truth"))
    truth = synth.config1_truth_grid(fb)
    assert np.array_equal(idx, np.argmin(truth, axis=0))


def test_piecewise_program_matches_the_generators_regimes():
    """A piecewise program built from the generator's own decision and regime functions: the
    oracle's FP64 cost is the generator's regime cost (d >= 0: g_a, else g_b) wherever the
    launch constraints hold, and +inf elsewhere; the FP32 replay agrees to FP32 rounding except
    where the decision is within FP32 resolution of 0."""
    fb, pb, truth = synth.piecewise_batch(5, n_progs=3, n_q=200)
    for p in range(3):
        q0 = int(pb.q0[p])
        N = pb.queries[q0:q0 + 200]
        want = truth(p, N)
        c64 = oc.program_costs(pb, p, mode="truth")
        c32 = oc.program_costs(pb, p, mode="replay").astype(np.float64)
        assert np.array_equal(np.isinf(c64), np.isinf(want))
        fin = np.isfinite(want)
        assert np.allclose(c64[fin], want[fin], rtol=1e-12, atol=0)
        close = np.isclose(c32[fin], want[fin], rtol=2e-6, atol=0)
        assert close.mean() > 0.999


def test_piecewise_fits_recover_the_decision_and_pick_well():
    """Fitted from the generator's samples by the oracle's least squares: the decision function
    (exact samples, representable in the monomial set) comes back to rounding, and the per-query
    argmin of the fitted piecewise program has small regret under the generator's costs."""
    from oracle import fit as of
    fb, pb, truth = synth.piecewise_batch(6, n_progs=4, n_q=256)
    coef, infos = of.fit_batch(fb)
    for p in range(4):
        d0 = int(fb.coef0[3 * p])
        n = int(fb.n_num[0] + fb.n_den[0] - 1)
        assert np.allclose(coef[d0:d0 + n], fb.truth_coef[d0:d0 + n], rtol=0, atol=1e-8)
    regrets = []
    for p in range(4):
        q0 = int(pb.q0[p])
        N = pb.queries[q0:q0 + 256]
        idx, _ = oc.argmin_lowest(oc.program_costs(pb, p, mode="truth", coef=coef))
        t = truth(p, N)
        best = t.min(axis=0)
        ok = np.isfinite(best) & (idx >= 0)
        regrets.append(t[idx[ok], np.nonzero(ok)[0]] / best[ok] - 1.0)
    r = np.concatenate(regrets)
    assert np.median(r) < 0.01 and np.mean(r <= 0.05) > 0.9, (np.median(r), np.mean(r <= 0.05))

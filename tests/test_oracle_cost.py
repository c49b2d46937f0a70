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

"""GPU parity of klr_eval_argmin against the oracle's FP32 replay (bit-exact costs and argmin)."""
import json
import os

import numpy as np
import pytest

from oracle import cost as oc
from paper_1911_02373_amd import synth
from tests.helpers import constant_programs

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cost_cases.json")


def _run(klr, pb, want_costs=True):
    from paper_1911_02373_amd.klr import DeviceEval
    de = DeviceEval.from_batch(klr, pb, with_costs=want_costs)
    am, bc, costs, st = klr.eval_argmin(de, want_costs=want_costs)
    import torch
    torch.cuda.synchronize()
    return (am.cpu().numpy(), bc.cpu().numpy(),
            None if costs is None else costs.cpu().numpy(), st.cpu().numpy())


def _check_program_exact(pb, p, am, bc, costs, cost_off):
    want = oc.program_costs(pb, p, mode="replay")
    q0, nq, nc = int(pb.q0[p]), int(pb.n_q[p]), int(pb.n_cfg[p])
    if costs is not None:
        got = costs[cost_off: cost_off + nc * nq].reshape(nc, nq)
        bad = np.argwhere(got.view(np.uint32) != want.view(np.uint32))
        assert bad.size == 0, (p, bad[:5], got[tuple(bad[0])], want[tuple(bad[0])])
    wi, wb = oc.argmin_lowest(want)
    assert np.array_equal(am[q0:q0 + nq], wi), p
    assert np.array_equal(bc[q0:q0 + nq].view(np.uint32), wb.view(np.uint32)), p


def test_hand_derived_costs_on_gpu(klr):
    cases = json.load(open(GOLDEN))["cases"]
    for cs in cases:
        pb = constant_programs([cs["metrics"]], [cs["L"]], [[cs["N"]]], grid_kind=cs["grid"])
        am, bc, costs, st = _run(klr, pb)
        want = np.inf if cs["expect"] == "inf" else cs["expect"]
        assert st[0] == 0
        assert costs[0] == want, (cs["name"], costs[0], want)


def test_config3_small_bit_exact(klr):
    """8 programs x 1000 queries (ragged against the 256-lane blocks) x 128 configurations."""
    pb = synth.config3_programs(101, n_progs=8, n_q=1000)
    am, bc, costs, st = _run(klr, pb)
    assert np.all(st == 0)
    off = 0
    for p in range(pb.n_progs):
        _check_program_exact(pb, p, am, bc, costs, off)
        off += int(pb.n_cfg[p]) * int(pb.n_q[p])


def _slot_records(de):
    """Configuration records of the collapse workspace after an evaluation, as int32 rows of 12:
    T, Wb, Bcap, rTh, Lmax, L0, L1, ok, magTC, shTC, fast, pad (slot p * max_cfg + c)."""
    ws = de.ws.cpu().numpy()
    off = de.n_progs * de.max_cfg * 72 * 4
    return ws[off: off + de.n_progs * de.max_cfg * 48].view(np.int32).reshape(de.n_progs, de.max_cfg, 12)


def test_short_division_taken_on_config3(klr):
    """Every admissible configuration of the c3 workload's programs (metric numerators and
    denominators, and the cycle estimate's quotient operands, far inside [2^-40, 2^40] over the
    queries) takes the short division for all twelve quotients; the pad configuration, ruled out
    statically, takes none."""
    import torch
    from paper_1911_02373_amd.klr import DeviceEval
    pb = synth.config3_programs(104, n_progs=8, n_q=1000)
    de = DeviceEval.from_batch(klr, pb)
    klr.eval_argmin(de)
    torch.cuda.synchronize()
    rec = _slot_records(de)
    ok, fast = rec[:, :, 7], rec[:, :, 10]
    assert np.array_equal(fast, 2 * ok)
    assert ok.sum() == 8 * 127 and not ok[:, 127].any()


def test_short_division_metrics_only_bit_exact(klr):
    """A memory latency of 2^42 cycles puts the cycle estimate's quotient operands past 2^40
    while the metrics stay moderate: every admissible configuration takes the short division
    for its eight metric quotients only, and costs and argmin equal the oracle's replay bit for
    bit."""
    import dataclasses

    import torch
    from paper_1911_02373_amd.klr import DeviceEval
    pb = synth.config3_programs(106, n_progs=6, n_q=600)
    pb = dataclasses.replace(pb, hw=dataclasses.replace(pb.hw, mem_lat=2.0 ** 42))
    de = DeviceEval.from_batch(klr, pb, with_costs=True)
    am, bc, costs, st = klr.eval_argmin(de, want_costs=True)
    torch.cuda.synchronize()
    am, bc, costs, st = am.cpu().numpy(), bc.cpu().numpy(), costs.cpu().numpy(), st.cpu().numpy()
    assert np.all(st == 0)
    rec = _slot_records(de)
    assert np.array_equal(rec[:, :, 10], rec[:, :, 7])            # 1 exactly where admissible
    off = 0
    for p in range(pb.n_progs):
        _check_program_exact(pb, p, am, bc, costs, off)
        off += int(pb.n_cfg[p]) * int(pb.n_q[p])


def test_short_division_wide_exponents_bit_exact(klr):
    """Metric numerators scaled by 2^k (k in [-36, 36]) and denominators' non-constant terms by
    2^m (m in [0, 30]) per fit, so the quotients span most of [2^-40, 2^40]: some configurations
    take the short division (for the metrics, or for all twelve quotients), others (an enclosure
    reaching past the range) the IEEE one, and every cost and argmin equals the oracle's replay
    bit for bit."""
    import dataclasses

    import torch
    from paper_1911_02373_amd.klr import DeviceEval
    pb = synth.config3_programs(105, n_progs=16, n_q=700)
    rng = np.random.default_rng(105)
    coef = pb.coef.copy()
    nm = int(pb.n_num[0])
    for fi in range(pb.num0.shape[0]):
        c0 = int(pb.coef0[fi])
        coef[c0: c0 + nm] *= 2.0 ** int(rng.integers(-36, 37))
        coef[c0 + nm: c0 + 2 * nm - 1] *= 2.0 ** int(rng.integers(0, 31))
    pb = dataclasses.replace(pb, coef=coef)
    de = DeviceEval.from_batch(klr, pb, with_costs=True)
    am, bc, costs, st = klr.eval_argmin(de, want_costs=True)
    torch.cuda.synchronize()
    am, bc, costs, st = am.cpu().numpy(), bc.cpu().numpy(), costs.cpu().numpy(), st.cpu().numpy()
    assert np.all(st == 0)
    rec = _slot_records(de)
    fast = rec[:, :127, 10]
    print("configurations by short quotients (none, metrics, all):", np.bincount(fast.ravel(), minlength=3))
    assert (fast == 0).any() and (fast > 0).any()
    off = 0
    for p in range(pb.n_progs):
        _check_program_exact(pb, p, am, bc, costs, off)
        off += int(pb.n_cfg[p]) * int(pb.n_q[p])


def test_short_quotient_is_ieee_sampled(klr):
    """The short quotient (reciprocal, one Newton step, one remainder correction) equals the
    correctly rounded FP32 division for every a mantissa against b mantissas at both ends of
    [1, 2) and spread over it, and the reciprocal estimate scales exactly with b's exponent and
    sign (the library's self-test kernel)."""
    top = 1 << 23
    slices = [(0, 1024), (top - 1024, 1024)] + [(k << 19, 128) for k in range(1, 16)]
    for b0, nb in slices:
        assert klr.lib.klr_selftest_short_division(b0, nb) == 0, (b0, nb)
    assert klr.lib.klr_selftest_short_division(-1, 4) == -1
    assert klr.lib.klr_selftest_short_division(top - 2, 4) == -1
    assert klr.lib.klr_selftest_short_division(5, 0) == 0


def test_short_quotient_is_ieee_exhaustive(klr):
    """Every pair of mantissas (2^46 pairs, about half a minute): with the exponent and sign
    scaling above this makes the short quotient the IEEE quotient for all operands in
    [2^-40, 2^40], the range the collapse admits it for."""
    step = 1 << 20
    for b0 in range(0, 1 << 23, step):
        assert klr.lib.klr_selftest_short_division(b0, step) == 0, b0
        print(f"b mantissas [0, {b0 + step}) checked", flush=True)


def test_mixed_uneven_programs_bit_exact(klr):
    """1-4 launch parameters, degree-3 metrics, 1-D and 2-D grids, uneven n_cfg and n_q,
    inadmissible configurations, tiny and huge N."""
    pb = synth.mixed_programs(202, 24)
    am, bc, costs, st = _run(klr, pb)
    assert np.all(st == 0)
    off = 0
    for p in range(pb.n_progs):
        _check_program_exact(pb, p, am, bc, costs, off)
        off += int(pb.n_cfg[p]) * int(pb.n_q[p])


def test_large_monomial_sets_bit_exact(klr):
    """Metrics with 280 numerator and 280 denominator monomials (N^a L^b, a <= 3, launch degree
    <= 4 over 4 launch parameters): more exponent rows than the collapse stages in LDS, so the
    collapse reads them from device memory."""
    pb = synth.mixed_programs(203, 4, n_q_range=(1, 200), n_cfg_range=(1, 48), v_launch_choices=(4,),
                              launch_degree=4)
    assert int(pb.n_num[0]) == 280
    am, bc, costs, st = _run(klr, pb)
    assert np.all(st == 0)
    off = 0
    for p in range(pb.n_progs):
        _check_program_exact(pb, p, am, bc, costs, off)
        off += int(pb.n_cfg[p]) * int(pb.n_q[p])


def test_config3_full_size_sampled(klr):
    """1024 programs x 65536 queries x 128 configurations as timed; argmin and best cost of
    sampled queries against the oracle's replay."""
    pb = synth.config3_programs(7, n_progs=1024, n_q=65536)
    am, bc, _, st = _run(klr, pb, want_costs=False)
    assert np.all(st == 0)
    rng = np.random.default_rng(0)
    for p in rng.choice(1024, 24, replace=False):
        qi = rng.choice(65536, 64, replace=False)
        wi, wb = oc.argmin_lowest(oc.program_costs(pb, int(p), query_idx=qi))
        q0 = int(pb.q0[p])
        assert np.array_equal(am[q0 + qi], wi)
        assert np.array_equal(bc[q0 + qi].view(np.uint32), wb.view(np.uint32))
    # properties over every query: an index in range or -1 exactly when the cost is +inf
    assert np.all((am >= -1) & (am < 128))
    assert np.array_equal(am == -1, np.isinf(bc))
    assert np.all(am != 127)            # the pad configuration is never admissible


def test_ties_duplicates_and_empty(klr):
    pb = synth.config3_programs(9, n_progs=3, n_q=300)
    base = synth.config3_launch_configs()[:50]
    pb.cfgs = np.concatenate([base, base]).reshape(-1)
    pb.n_cfg[:] = 100
    pb.n_cfg[2] = 0                    # a program without configurations
    am, bc, costs, st = _run(klr, pb)
    assert np.all(st == 0)
    assert np.all(am[:600] < 50) and np.all(am[:600] >= 0)
    assert np.all(am[600:] == -1) and np.all(np.isinf(bc[600:]))


def test_all_inadmissible_and_small_N(klr):
    rows = [[10, 10, 0, 1, 0, 300, 0, 128]]            # R = 300: B_active = 0 for T >= 512
    cfgs = [[512, 1], [1024, 1], [1, 1], [32, 33]]
    pb = constant_programs(rows, cfgs, [[1 << 20, 100, 1, 0, -5]])
    am, bc, costs, st = _run(klr, pb)
    assert np.all(am == -1) and np.all(np.isinf(bc)) and np.all(np.isinf(costs))


@pytest.mark.parametrize("grid", [0, 1])
@pytest.mark.parametrize("n_cu", [1, 3, 32768])
def test_occupancy_edges_and_huge_block_counts(klr, grid, n_cu):
    """Few compute units (and a 32768-CU machine with 65536-thread blocks) and N up to 2^31 - 1, so ceil(blocks / n_cu) reaches 2^25 on both sides
    of the 2^20 switch of the repetition count; register and LDS terms at their clamps: R = 1,
    fractional R, R past 2^24, Z = 0 (no LDS bound), Z = z_max, Z = z_max + 1 (no block fits), and
    R, Z in (-1, 0) and below (ceil gives -0: clamped to 1 and to no LDS bound)."""
    base = [40.0, 6.0, 3.0, 2.0, 1.0, 1.0, 0.0, 64.0]
    rows = []
    for r_val, z_val in [(1.0, 0.0), (37.2, 0.0), (1e9, 0.0), (2.0, 163840.0), (2.0, 163841.0),
                         (5.0, 4096.0), (64.0, 1.5), (2048.0, 0.0), (2.0, -0.5), (-0.5, 7.0),
                         (-3.0, -2.0)]:
        m = list(base)
        m[5], m[6] = r_val, z_val
        rows.append(m)
    cfgs = [[64, 1], [128, 1], [1024, 1], [96, 2], [1, 64], [32, 32], [65536, 1], [256, 256]]
    big = [2 ** 31 - 1, 2 ** 30 + 7, 2 ** 25 + 3, 123456789, 64 * 2 ** 20, 64 * 2 ** 20 + 1,
           64 * 2 ** 20 - 1, 3 * 64 * 2 ** 20 + 5, 1, 0, 64, 65]
    # the 32768-CU machine admits 65536-thread blocks (T n_cu = 2^31: repetition quotient 0)
    hw = synth.HW(n_cu=n_cu) if n_cu < 32768 else synth.HW(n_cu=n_cu, w_max=1024, t_max=65536)
    pb = constant_programs(rows, cfgs, [big] * len(rows), grid_kind=grid, hw=hw)
    am, bc, costs, st = _run(klr, pb)
    assert np.all(st == 0)
    off = 0
    for p in range(pb.n_progs):
        _check_program_exact(pb, p, am, bc, costs, off)
        off += int(pb.n_cfg[p]) * int(pb.n_q[p])
    assert np.isfinite(costs).any() and np.isinf(costs).any()


def test_bad_descriptors_reported_not_read(klr):
    pb = synth.config3_programs(5, n_progs=4, n_q=100)
    pb.fit0[1] = 10 ** 6               # fit range out of bounds: program skipped
    pb.n_den = pb.n_den.copy()
    pb.n_den[2 * 8 + 3] = 0            # a metric without a denominator row: fits invalid
    pb.n_q[3] = 10 ** 6                # query range out of bounds: program skipped
    pb.q0[3] = 0
    am, bc, costs, st = _run(klr, pb, want_costs=False)
    assert st[0] == 0
    assert st[1] & 1 and st[3] & 1
    assert st[2] == 2
    assert np.all(am[200:300] == -1) and np.all(np.isinf(bc[200:300]))


def test_deterministic(klr):
    pb = synth.mixed_programs(77, 16)
    a = _run(klr, pb)
    b = _run(klr, pb)
    for x, y in zip(a, b):
        assert np.array_equal(np.asarray(x).view(np.uint8), np.asarray(y).view(np.uint8))


def fp64_truth_report(pb, am, bc, costs, progs):
    """Error of the FP32 results against the FP64 cycle estimate (each metric the full
    multivariate p/q in FP64, exact integer parts) for the listed programs: the rate at which
    the FP32 argmin differs from the FP64 one, the regret of the FP32 pick under the FP64
    costs, the relative error of the FP32 best cost and of every FP32 cost, and admissibility
    disagreements."""
    dis = n = adm = 0
    regrets, rel, rel_all = [], [], []
    off = 0
    for p in progs:
        q0, nq, nc = int(pb.q0[p]), int(pb.n_q[p]), int(pb.n_cfg[p])
        c64 = oc.program_costs(pb, p, mode="truth")
        c32 = costs[off: off + nc * nq].reshape(nc, nq).astype(np.float64)
        off += nc * nq
        fin = np.isfinite(c32) & np.isfinite(c64)
        rel_all.append(np.abs(c32[fin] - c64[fin]) / c64[fin])
        i64, b64 = oc.argmin_lowest(c64)
        a32, b32 = am[q0:q0 + nq], bc[q0:q0 + nq].astype(np.float64)
        dis += int(np.sum(a32 != i64))
        n += nq
        adm += int(np.sum((i64 >= 0) != (a32 >= 0)))
        ok = (i64 >= 0) & (a32 >= 0)
        picked = c64[np.maximum(a32, 0), np.arange(nq)]
        regrets.append(picked[ok] / b64[ok] - 1.0)
        rel.append(np.abs(b32[ok] - b64[ok]) / b64[ok])
    r, e, ea = np.concatenate(regrets), np.concatenate(rel), np.concatenate(rel_all)
    return {"queries": n, "argmin_mismatch_rate": dis / max(n, 1), "admissible_mismatch": adm,
            "cost_rel_err_max": float(ea.max()) if ea.size else 0.0,
            "regret_max": float(r.max()) if r.size else 0.0, "regret_p999": float(np.quantile(r, 0.999)) if r.size else 0.0,
            "best_cost_rel_err_max": float(e.max()) if e.size else 0.0,
            "best_cost_rel_err_median": float(np.median(e)) if e.size else 0.0}


@pytest.mark.parametrize("kind", ["c3", "mixed"])
def test_fp32_results_against_fp64_truth(klr, kind):
    """The FP32 evaluation against the FP64 cycle estimate: on c3 programs (degree 2, 2048
    queries each) and on uneven programs (1-4 launch parameters, degree 3, 1-D and 2-D grids)
    the FP32 argmin is the FP64 argmin wherever the FP64 runner-up is more than the FP32 error
    away; the regret of every FP32 pick under FP64 costs stays within twice the FP32 cost error
    (so near-ties at FP32 resolution are the only place the two can part); best costs agree to
    a few FP32 ulps in the median."""
    if kind == "c3":
        pb = synth.config3_programs(41, n_progs=6, n_q=2048)
    else:
        pb = synth.mixed_programs(42, 16, n_q_range=(50, 400), n_cfg_range=(16, 160))
    am, bc, costs, st = _run(klr, pb, want_costs=True)
    assert np.all(st == 0)
    rep = fp64_truth_report(pb, am, bc, costs, range(pb.n_progs))
    print(kind, rep)
    eps = rep["cost_rel_err_max"]
    assert eps < 1e-5 and rep["best_cost_rel_err_median"] < 1e-6, rep
    assert rep["admissible_mismatch"] <= 1e-3 * rep["queries"], rep
    assert rep["argmin_mismatch_rate"] <= 1e-3, rep
    assert rep["regret_max"] <= 2 * eps / (1 - eps) + 1e-12, rep

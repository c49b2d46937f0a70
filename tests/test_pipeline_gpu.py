"""Batching machinery: eval launch-shape variants and autotuner, hipGraph capture and replay of
the fit -> eval pipeline."""
import os

import numpy as np
import pytest

from paper_1911_02373_amd import synth

pytestmark = pytest.mark.gpu


def test_eval_variants_bit_identical(klr):
    import torch
    from paper_1911_02373_amd.klr import OPT_EVAL_VARIANT, DeviceEval
    pb = synth.mixed_programs(31, 12, n_q_range=(1, 1500))
    de = DeviceEval.from_batch(klr, pb, with_costs=True)
    ref = None
    try:
        for v in range(6):
            klr.set_option(OPT_EVAL_VARIANT, v)
            am, bc, costs, _ = klr.eval_argmin(de, want_costs=True)
            torch.cuda.synchronize()
            cur = (am.cpu().numpy(), bc.cpu().numpy().view(np.uint32), costs.cpu().numpy().view(np.uint32))
            if ref is None:
                ref = cur
            else:
                for x, y in zip(cur, ref):
                    assert np.array_equal(x, y), v
    finally:
        klr.set_option(OPT_EVAL_VARIANT, -1)


def test_autotuner_choice_is_used_and_results_unchanged(klr):
    import torch
    from paper_1911_02373_amd.klr import DeviceEval
    pb = synth.config3_programs(33, n_progs=16, n_q=4096)
    de = DeviceEval.from_batch(klr, pb)
    a1, b1, _, _ = klr.eval_argmin(de)          # first call of this shape: tunes
    a2, b2, _, _ = klr.eval_argmin(de)          # cached choice
    torch.cuda.synchronize()
    assert np.array_equal(a1.cpu().numpy(), a2.cpu().numpy())
    assert np.array_equal(b1.cpu().numpy().view(np.uint32), b2.cpu().numpy().view(np.uint32))


def test_graph_replay_matches_eager(klr):
    """Fit batch + evaluation captured once and replayed three times; eager work of another
    batch runs between the replays; every replay equals the eager result bit for bit."""
    import torch
    from paper_1911_02373_amd.klr import FIT_INFO, DeviceEval, DeviceFit
    fb = synth.config2_fits(41, 200, "2b")
    pb = synth.config3_programs(42, n_progs=24, n_q=3000)
    pb_other = synth.config3_programs(43, n_progs=24, n_q=3000)
    df = DeviceFit.from_batch(fb)
    de = DeviceEval.from_batch(klr, pb)
    de_o = DeviceEval.from_batch(klr, pb_other)
    s = torch.cuda.Stream()
    fit_out = (torch.empty(df.n_coef, dtype=torch.float64, device="cuda"),
               torch.empty(df.n_fits * FIT_INFO.itemsize, dtype=torch.uint8, device="cuda"))
    ev_out = (torch.empty(de.queries.numel(), dtype=torch.int32, device="cuda"),
              torch.empty(de.queries.numel(), dtype=torch.float32, device="cuda"), None,
              torch.empty(de.n_progs, dtype=torch.int32, device="cuda"))
    with torch.cuda.stream(s):
        klr.fit_batched(df, 0, 64, 1e-10, out=fit_out, stream=s)       # eager reference (+ tuning)
        klr.eval_argmin(de, out=ev_out, stream=s)
    s.synchronize()
    ref = [fit_out[0].cpu().clone(), fit_out[1].cpu().clone(), ev_out[0].cpu().clone(), ev_out[1].cpu().clone()]
    klr.capture_begin(s)
    klr.fit_batched(df, 0, 64, 1e-10, out=fit_out, stream=s)
    klr.eval_argmin(de, out=ev_out, stream=s)
    g = klr.capture_end(s)
    try:
        for rep in range(3):
            for t in (fit_out[0], ev_out[1]):
                t.fill_(0)
            torch.cuda.synchronize()
            klr.graph_launch(g, s)
            s.synchronize()
            got = [fit_out[0].cpu(), fit_out[1].cpu(), ev_out[0].cpu(), ev_out[1].cpu()]
            for x, y in zip(got, ref):
                assert torch.equal(x.view(torch.uint8), y.view(torch.uint8)), rep
            klr.eval_argmin(de_o)                                          # eager work in between
            torch.cuda.synchronize()
    finally:
        klr.graph_destroy(g)


def test_single_fit_workload_end_to_end(klr):
    """The single-fit workload on the device: FP64 fit of 200 samples over (N, B), then its
    fitted function over the full 11 x 32 grid as a metric-cost program with the per-N argmin
    over B, eager and as a captured graph replayed several times.  Costs and argmin bit-exact
    against the oracle's FP32 replay of the GPU's coefficients; fitted values within 1e-9 of the
    oracle's least squares; decision quality against the truth's per-N argmin reported (the
    1 % noise can move a pick between near-equal block sizes)."""
    import torch
    from oracle import cost as oc
    from oracle import fit as of
    from paper_1911_02373_amd.klr import FIT_INFO, DeviceEval, DeviceFit, info_records
    for seed in (1, 2, 3):
        fb = synth.config1_fit(seed)
        df = DeviceFit.from_batch(fb)
        s = torch.cuda.Stream()
        fit_out = (torch.empty(df.n_coef, dtype=torch.float64, device="cuda"),
                   torch.empty(FIT_INFO.itemsize, dtype=torch.uint8, device="cuda"))
        pb = synth.config1_program(fb)
        de = DeviceEval.from_batch(klr, pb, with_costs=True, coef=fit_out[0])
        ev_out = (torch.empty(11, dtype=torch.int32, device="cuda"), torch.empty(11, dtype=torch.float32, device="cuda"),
                  torch.empty(11 * 32, dtype=torch.float32, device="cuda"), torch.empty(1, dtype=torch.int32, device="cuda"))
        with torch.cuda.stream(s):
            klr.fit_batched(df, 0, 64, 1e-12, out=fit_out, stream=s)
            klr.eval_argmin(de, out=ev_out, want_costs=True, stream=s)
        s.synchronize()
        ref = [t.cpu().clone() for t in (fit_out[0], ev_out[0], ev_out[1], ev_out[2])]
        coef = ref[0].numpy()
        info = info_records(fit_out[1])
        assert info["status"][0] & (of.BAD_INPUT | of.NOT_CONVERGED) == 0
        ora, _ = of.fit_batch(fb)
        Xi, fi, En, Ed, sc = fb.fit_arrays(0)
        A, _ = of.design_matrix(Xi, fi, En, Ed, sc)
        assert np.linalg.norm(A @ (coef - ora)) <= 1e-9 * np.linalg.norm(fi)
        want = oc.program_costs(synth.config1_program(fb, coef), 0, mode="replay")
        assert np.array_equal(ref[3].numpy().reshape(32, 11).view(np.uint32), want.view(np.uint32))
        wi, wb = oc.argmin_lowest(want)
        assert np.array_equal(ref[1].numpy(), wi) and np.array_equal(ref[2].numpy().view(np.uint32), wb.view(np.uint32))
        assert int(ev_out[3].cpu()[0]) == 0
        truth = synth.config1_truth_grid(fb)
        tpick = np.argmin(truth, axis=0)
        regret = truth[wi, np.arange(11)] / truth[tpick, np.arange(11)] - 1.0
        print(f"seed {seed}: per-N picks equal to the truth's {np.mean(wi == tpick):.2f}, "
              f"max regret under the truth {regret.max():.4f}")
        # graph capture of fit + grid evaluation, replayed with eager work in between
        klr.capture_begin(s)
        klr.fit_batched(df, 0, 64, 1e-12, out=fit_out, stream=s)
        klr.eval_argmin(de, out=ev_out, want_costs=True, stream=s)
        g = klr.capture_end(s)
        try:
            for rep in range(3):
                for t in (fit_out[0], ev_out[1], ev_out[2]):
                    t.fill_(0)
                torch.cuda.synchronize()
                klr.graph_launch(g, s)
                s.synchronize()
                got = [t.cpu() for t in (fit_out[0], ev_out[0], ev_out[1], ev_out[2])]
                for x, y in zip(got, ref):
                    assert torch.equal(x.view(torch.uint8), y.view(torch.uint8)), rep
                klr.fit_batched(df, 0, 64, 1e-12)                     # eager work in between
                torch.cuda.synchronize()
        finally:
            klr.graph_destroy(g)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_fit_variants_bit_identical(klr, prec):
    """Every fit launch variant (fits per workgroup of the one-wavefront kernel: 4, 2, 1), under
    both schedules, gives bit-identical coefficients and info records; the autotuned call too."""
    import torch
    from paper_1911_02373_amd.klr import OPT_FIT_PERSISTENT, OPT_FIT_VARIANT, DeviceFit, info_records
    fb = synth.config2_fits(91, 333, "2b", m_range=(20, 1000))
    df = DeviceFit.from_batch(fb)
    ref = None
    try:
        for pers in (1, 0):
            klr.set_option(OPT_FIT_PERSISTENT, pers)
            for v in (-1, 0, 1, 2):
                klr.set_option(OPT_FIT_VARIANT, v)
                c, i = klr.fit_batched(df, prec, 256, 1e-9)
                torch.cuda.synchronize()
                cur = (c.cpu().numpy().view(np.uint64), info_records(i).view(np.uint8))
                if ref is None:
                    ref = cur
                else:
                    assert np.array_equal(cur[0], ref[0]) and np.array_equal(cur[1], ref[1]), (pers, v)
    finally:
        klr.set_option(OPT_FIT_PERSISTENT, 1)
        klr.set_option(OPT_FIT_VARIANT, -1)

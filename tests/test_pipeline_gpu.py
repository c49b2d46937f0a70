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

"""Data collection on the device: target kernels timed at sample points, the measured times
fitted by klr_fit_batched, the fitted time evaluated over every block shape by a metric-cost
program, and the pick compared with the exhaustively measured best block shape (the paper's
Table 1 measure: best time / chosen time)."""
import numpy as np
import pytest

from oracle import cost as oc
from oracle import fit as of
from paper_1911_02373_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("target", [0, 1])
def test_collect_fit_decide_on_measured_times(klr, target):
    import torch
    from paper_1911_02373_amd.klr import DeviceEval, DeviceFit, info_records
    shapes = synth.block_shapes()
    attrs = klr.target_attributes(target)
    assert attrs["regs"] > 0 and attrs["lds_bytes"] >= 0
    plan = synth.collection_plan(11 + target, 240)
    t = klr.collect_times(target, plan, reps=5)
    assert np.all(np.isfinite(t)) and np.all(t > 0)
    again = klr.collect_times(target, plan[:60], reps=5)
    assert np.median(np.abs(again / t[:60] - 1.0)) < 0.25
    fb = synth.measured_fit(plan, t)
    df = DeviceFit.from_batch(fb)
    coef, info = klr.fit_batched(df, 0, 256, 1e-12)
    torch.cuda.synchronize()
    info = info_records(info)
    assert not (info["status"][0] & (of.BAD_INPUT | of.NOT_CONVERGED))
    queries = np.rint(2.0 ** (8 + np.arange(13) / 3.0)).astype(np.int32)
    ch = coef.cpu().numpy()
    pb = synth.measured_program(fb, shapes, queries, coef=ch)
    de = DeviceEval.from_batch(klr, pb, with_costs=True, coef=coef)
    am, bc, costs, st = klr.eval_argmin(de, want_costs=True)
    torch.cuda.synchronize()
    am, costs = am.cpu().numpy(), costs.cpu().numpy()
    want = oc.program_costs(pb, 0, mode="replay")
    assert np.array_equal(costs.view(np.uint32), want.reshape(-1).view(np.uint32))
    assert np.array_equal(am, oc.argmin_lowest(want)[0])
    # every admissible block shape measured at every query size
    grid = np.array([(n, bx, by) for n in queries for bx, by in shapes if max(bx, by) <= n], np.int32)
    tg = klr.collect_times(target, grid, reps=5)
    ratios = []
    for n in queries:
        sel = grid[:, 0] == n
        meas = dict(zip(map(tuple, grid[sel, 1:]), tg[sel]))
        best = min(meas.values())
        c = am[list(queries).index(n)]
        chosen = meas.get(tuple(shapes[c]), np.inf) if c >= 0 else np.inf
        ratios.append(best / chosen)
    r = np.array(ratios)
    print(f"target {target} (regs {attrs['regs']}): best / chosen time per N: {np.round(r, 3).tolist()}; "
          f"median {np.median(r):.3f}, >= 0.85 for {np.mean(r >= 0.85):.2f} of the sizes")
    assert np.median(r) >= 0.5


def test_collect_rejects_bad_samples(klr):
    """Samples outside the limits are refused on the host before any launch."""
    from paper_1911_02373_amd.klr import KlrError
    for bad in ([[0, 32, 2]], [[1024, 64, 32]], [[1024, 0, 4]], [[1 << 20, 32, 2]]):
        with pytest.raises(KlrError):
            klr.collect_times(0, bad)

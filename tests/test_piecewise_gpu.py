"""Piecewise rational programs with a fitted decision node on the device: the decision and the
two regime costs are fitted by klr_fit_batched, the programs (KLR_COST_PIECEWISE) evaluated by
klr_eval_argmin bit-exactly against the oracle's FP32 replay of the same coefficients, and the
picks judged by the generator's own regime costs."""
import copy

import numpy as np
import pytest

from oracle import cost as oc
from oracle import fit as of
from paper_1911_02373_amd import synth

pytestmark = pytest.mark.gpu


def test_piecewise_fit_then_evaluate(klr):
    import torch
    from paper_1911_02373_amd.klr import DeviceEval, DeviceFit, info_records
    fb, pb, truth = synth.piecewise_batch(81, n_progs=12, n_q=700)
    df = DeviceFit.from_batch(fb)
    coef, info = klr.fit_batched(df, 0, 256, 1e-12)
    torch.cuda.synchronize()
    info = info_records(info)
    assert not np.any(info["status"] & (of.BAD_INPUT | of.NOT_CONVERGED))
    # the decision functions come back from their exact samples
    ch = coef.cpu().numpy()
    for p in range(pb.n_progs):
        d0 = int(fb.coef0[3 * p])
        n = int(fb.n_num[3 * p] + fb.n_den[3 * p] - 1)
        assert np.allclose(ch[d0:d0 + n], fb.truth_coef[d0:d0 + n], rtol=0, atol=1e-7), p
    pb2 = copy.copy(pb)
    pb2.coef = ch
    de = DeviceEval.from_batch(klr, pb2, with_costs=True, coef=coef)
    am, bc, costs, st = klr.eval_argmin(de, want_costs=True)
    torch.cuda.synchronize()
    am, bc, costs = am.cpu().numpy(), bc.cpu().numpy(), costs.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    off = 0
    regrets = []
    for p in range(pb.n_progs):
        q0, nq, nc = int(pb.q0[p]), int(pb.n_q[p]), int(pb.n_cfg[p])
        want = oc.program_costs(pb2, p, mode="replay")
        got = costs[off: off + nc * nq].reshape(nc, nq)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), p
        wi, wb = oc.argmin_lowest(want)
        assert np.array_equal(am[q0:q0 + nq], wi) and np.array_equal(bc[q0:q0 + nq].view(np.uint32), wb.view(np.uint32))
        t = truth(p, pb.queries[q0:q0 + nq])
        best = t.min(axis=0)
        ok = np.isfinite(best) & (wi >= 0)
        regrets.append(t[wi[ok], np.nonzero(ok)[0]] / best[ok] - 1.0)
        off += nc * nq
    r = np.concatenate(regrets)
    print(f"piecewise picks under the generator's costs: median regret {np.median(r):.4f}, "
          f"within 1 % {np.mean(r <= 0.01):.3f}, within 5 % {np.mean(r <= 0.05):.3f}")
    assert np.median(r) < 0.01 and np.mean(r <= 0.05) > 0.9

"""klr_eval_argmin_noalloc (the entry point for callers that cannot allocate) against
klr_eval_argmin: identical argmin, best costs, cost matrix and program status, on two calls in
a row (the second on a smaller batch, so the fixed workspace still holds the first call's
larger contents), and the size limit rejected on the host."""
import numpy as np
import pytest

from paper_1911_02373_amd import synth

pytestmark = pytest.mark.gpu


def _noalloc(klr, de, want_costs=True):
    import torch
    from paper_1911_02373_amd.klr import _ptr
    ql = int(de.queries.numel())
    am = torch.full((ql,), -5, dtype=torch.int32, device="cuda")
    bc = torch.full((ql,), -1.0, dtype=torch.float32, device="cuda")
    costs = torch.full((de.costs_len,), -1.0, dtype=torch.float32, device="cuda") if want_costs else None
    st = torch.full((de.n_progs,), -1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    rc = klr.lib.klr_eval_argmin_noalloc(
        klr.h, _ptr(de.progs), de.n_progs, de.max_cfg, de.max_q, de.hw.ctypes.data, _ptr(de.desc), de.n_fits,
        _ptr(de.exps), de.n_exp_rows, _ptr(de.coef), int(de.coef.numel()), _ptr(de.cfgs), int(de.cfgs.numel()),
        _ptr(de.queries), ql, _ptr(am), _ptr(bc), _ptr(costs), int(costs.numel()) if costs is not None else 0,
        _ptr(st), stream)
    return rc, am, bc, costs, st


def _same(klr, pb):
    import torch
    from paper_1911_02373_amd.klr import DeviceEval
    de = DeviceEval.from_batch(klr, pb, with_costs=True)
    rc, am, bc, costs, st = _noalloc(klr, de)
    assert rc == 0, klr.lib.klr_last_error(klr.h)
    ea, eb, ec, est = klr.eval_argmin(de, want_costs=True)
    torch.cuda.synchronize()
    assert np.array_equal(am.cpu().numpy(), ea.cpu().numpy())
    assert np.array_equal(bc.cpu().numpy().view(np.uint32), eb.cpu().numpy().view(np.uint32))
    assert np.array_equal(costs.cpu().numpy().view(np.uint32), ec.cpu().numpy().view(np.uint32))
    assert np.array_equal(st.cpu().numpy(), est.cpu().numpy())


def test_noalloc_matches_eval_argmin_twice(klr):
    # a larger batch first (uneven programs, 1-4 launch parameters, 1-D and 2-D grids), then a
    # smaller one over the same fixed workspace
    _same(klr, synth.mixed_programs(61, 40, n_q_range=(1, 900), n_cfg_range=(1, 300)))
    _same(klr, synth.config3_programs(62, n_progs=5, n_q=333))


def test_noalloc_rejects_batches_above_the_limit(klr):
    """A batch whose workspace exceeds the fixed array is refused on the host (nothing runs)."""
    from paper_1911_02373_amd.klr import KLR_E_WORKSPACE, DeviceEval
    pb = synth.config3_programs(63, n_progs=1, n_q=16)
    de = DeviceEval.from_batch(klr, pb)
    need_progs = (64 << 20) // int(klr.lib.klr_eval_workspace(1, 65536)) + 2
    de.n_progs, de.max_cfg = need_progs, 65536
    rc, *_ = _noalloc(klr, de, want_costs=False)
    assert rc == KLR_E_WORKSPACE

"""The C-ABI library loads without a GPU and exports every symbol include/klr.h declares."""
import os
import re

import pytest

from paper_1911_02373_amd import klr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "klr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(klr_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(klr.LIB_PATH):
        pytest.fail("libklr.so missing: run python -m paper_1911_02373_amd.build (or __graft_entry__.build())")
    return klr.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert set(klr.EXPORTS) <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_struct_layouts_match_binding(lib):
    assert klr.abi_layout(lib) == klr.expected_layout()


def test_workspace_sizes_are_host_computable(lib):
    assert lib.klr_eval_workspace(0, 128) == 0
    assert lib.klr_eval_workspace(1024, 128) > 0
    assert lib.klr_fit_workspace(4096, 1 << 20, klr.KLR_FP64) >= 16 << 20


def test_null_handle_rejected_without_launch(lib):
    # host-detectable errors return before touching the device
    assert lib.klr_eval_argmin(None, None, 0, 0, 0, None, None, 0, None, 0, None, 0, None, 0, None,
                               0, None, None, None, 0, None, None, 0, None) == klr.KLR_E_INVALID


def test_invariant_divisor_multiplication_exact(lib):
    """floor(n / d) by multiply-high and shift, for every divisor up to 70000 (block sizes and
    CU counts) on dividends around its multiples and at the top of [0, 2^31)."""
    assert lib.klr_selftest_divisors(70000) == 0


def test_invariant_divisor_products_exact(lib):
    """The one-step divisor of the repetition count, T * n_cu: every wave multiple T up to 65536
    times CU counts from 1 to 65536 (products up to 2^32; from 2^31 on the quotient is 0), and
    seeded random divisors below 2^31."""
    import numpy as np
    t = np.arange(32, 65537, 32, dtype=np.uint64)
    cus = np.array([1, 2, 3, 7, 80, 104, 120, 228, 256, 304, 1000, 32768, 65535, 65536], np.uint64)
    ds = np.unique(np.concatenate([(t[:, None] * cus[None, :]).reshape(-1),
                                   np.random.default_rng(5).integers(1, 1 << 31, 4000, dtype=np.int64).astype(np.uint64),
                                   np.array([(1 << 31) - 1, 1 << 31, (1 << 31) + 1, 1 << 32], np.uint64)]))
    ds = np.ascontiguousarray(ds)
    assert lib.klr_selftest_divisor_list(ds.ctypes.data, int(ds.size)) == 0
    zero = np.zeros(1, np.uint64)
    assert lib.klr_selftest_divisor_list(zero.ctypes.data, 1) == 1


def test_short_division_selftest_rejects_bad_ranges_on_host(lib):
    """The GPU self-test of the short quotient checks its b-mantissa range before any HIP call."""
    assert lib.klr_selftest_short_division(-1, 4) == -1
    assert lib.klr_selftest_short_division(0, -1) == -1
    assert lib.klr_selftest_short_division((1 << 23) - 2, 4) == -1


def test_program_samples_bookkeeping():
    """The (program, configuration, query) training samples of uneven two-launch-parameter
    programs, against a brute-force listing of the same points (host tensors)."""
    import numpy as np
    import torch
    from paper_1911_02373_amd import klr as K
    from paper_1911_02373_amd import synth
    _, pb = synth.config5_batch(3, n_progs=24, n_q=5)
    sub = synth.select_programs(pb, np.nonzero(pb.v_launch == 2)[0])
    tq = synth.surrogate_training_queries(4, sub, n_q=3)

    class _DE:
        queries = torch.from_numpy(tq.queries.astype(np.int32))
        cfgs = torch.from_numpy(tq.cfgs.astype(np.int32))
    n = int((tq.n_cfg.astype(np.int64) * tq.n_q).sum())
    kid, N, L, c = K.program_samples(tq, _DE, torch.arange(n, dtype=torch.float32))
    rows = [(p, tq.queries[tq.q0[p] + q], tq.cfgs[tq.cfg0[p] + 2 * ci], tq.cfgs[tq.cfg0[p] + 2 * ci + 1])
            for p in range(tq.n_progs) for ci in range(int(tq.n_cfg[p])) for q in range(int(tq.n_q[p]))]
    rows = np.array(rows)
    assert tq.n_progs > 1 and len(set(tq.n_cfg.tolist())) > 1
    assert np.array_equal(kid.numpy(), rows[:, 0]) and np.array_equal(N.numpy(), rows[:, 1])
    assert np.array_equal(L.numpy().reshape(-1, 2), rows[:, 2:4])
    assert np.array_equal(c.numpy(), np.arange(n, dtype=np.float32))


def test_eval_fit_descs_out_of_range_program():
    """A program whose fit range lies outside the batch leaves the descriptors alone (the
    device reports it as a bad descriptor); the other programs' fits take 1 + v_launch."""
    import numpy as np
    from paper_1911_02373_amd import synth
    pb = synth.config3_programs(5, n_progs=4, n_q=16)
    pb.fit0 = np.asarray(pb.fit0).copy()
    pb.fit0[1] = 10 ** 6
    pb.fit0[2] = -3
    d = klr.eval_fit_descs(pb)
    n = pb.num0.shape[0]
    want = np.zeros(n, np.int64)
    for p in (0, 3):
        want[pb.fit0[p]:pb.fit0[p] + 8] = 1 + pb.v_launch[p]
    assert np.array_equal(d["v"].astype(np.int64), want)

"""Small builders shared by the tests (inputs only, no method arithmetic)."""
import numpy as np

from paper_1911_02373_amd import synth


def constant_programs(metric_rows, cfg_rows, queries_per_prog, grid_kind=0, hw=None):
    """Programs whose 8 metrics are constants (numerator = value, denominator = 1).

    metric_rows: [n_progs][8] values; cfg_rows: [n_cfg][2] (shared by all programs);
    queries_per_prog: [n_progs][n_q] data sizes."""
    metric_rows = np.asarray(metric_rows, np.float64)
    n_progs = metric_rows.shape[0]
    n_fits = n_progs * synth.N_METRICS
    exps = np.zeros((2, synth.MAX_VARS), np.uint8)
    cfgs = np.asarray(cfg_rows, np.int32)
    qs = np.asarray(queries_per_prog, np.int32)
    n_q = qs.shape[1]
    scale = np.zeros((n_fits, synth.MAX_VARS), np.int8)
    scale[:, :3] = (26, 10, 10)
    return synth.ProgramBatch(
        fits=None, coef=metric_rows.reshape(-1).copy(), exps=exps,
        num0=np.zeros(n_fits, np.int32), n_num=np.ones(n_fits, np.int32),
        den0=np.ones(n_fits, np.int32), n_den=np.ones(n_fits, np.int32),
        coef0=np.arange(n_fits, dtype=np.int64), scale_exp=scale,
        v_launch=np.full(n_progs, 2, np.int32),
        fit0=np.arange(n_progs, dtype=np.int32) * synth.N_METRICS,
        cfg0=np.zeros(n_progs, np.int64), n_cfg=np.full(n_progs, cfgs.shape[0], np.int32),
        grid_kind=np.full(n_progs, grid_kind, np.int32),
        q0=np.arange(n_progs, dtype=np.int64) * n_q, n_q=np.full(n_progs, n_q, np.int32),
        cfgs=cfgs.reshape(-1), queries=qs.reshape(-1), hw=hw or synth.HW())

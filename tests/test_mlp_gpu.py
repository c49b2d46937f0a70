"""GPU parity of the surrogate network kernels against the FP64 oracle, and the semantics of
surrogate selection with exact fallback."""
import numpy as np
import pytest

from oracle import cost as oc
from oracle import mlp as om
from paper_1911_02373_amd import synth

pytestmark = pytest.mark.gpu


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t if dtype is None else t.to(dtype)).cuda()


def _samples(rng, B, nk):
    kid = rng.integers(0, nk, B).astype(np.int32)
    N = np.rint(2.0 ** rng.uniform(8, 26, B)).astype(np.int32)
    bx = (2 ** rng.integers(0, 11, B)).astype(np.int32)
    by = rng.integers(1, 65, B).astype(np.int32)
    return kid, N, bx, by


def _f64(p):
    return {k: np.asarray(v, np.float64) for k, v in p.items()}


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-30)


def _cos(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))


def test_forward_matches_oracle(klr):
    import torch
    rng = np.random.default_rng(0)
    nk = 16
    p = synth.mlp_init(1, nk)
    blob = klr.surrogate_alloc(p, nk)
    kid, N, bx, by = _samples(rng, 1000, nk)                    # ragged against 64-row tiles
    L = np.stack([bx, by], 1).reshape(-1)
    pred = klr.surrogate_predict(blob, nk, _dev(kid), _dev(N), _dev(L))
    torch.cuda.synchronize()
    y = pred.cpu().numpy().astype(np.float64)
    yo, _ = om.forward(_f64(p), kid, N, bx, by)
    # BF16 h1 and W2 (2^-9 relative rounding) on the 256 x 256 layer, FP32 elsewhere
    assert _rel(y, yo) < 2e-2 and _cos(y, yo) > 0.999
    assert np.max(np.abs(y - yo)) < 0.05 * np.sqrt(np.mean(yo ** 2)) + 1e-3


def test_gradients_match_oracle(klr):
    import torch
    rng = np.random.default_rng(1)
    nk = 32
    p = synth.mlp_init(2, nk)
    blob = klr.surrogate_alloc(p, nk)
    B = 512
    kid, N, bx, by = _samples(rng, B, nk)
    t = rng.normal(size=B).astype(np.float32)
    grads, loss = klr.surrogate_step(blob, nk, _dev(kid), _dev(N), _dev(np.stack([bx, by], 1).reshape(-1)),
                                     _dev(t), lr=0.0, step=1)
    torch.cuda.synchronize()
    from paper_1911_02373_amd.klr import grads_to_dict
    g = grads_to_dict(klr.lib, grads.cpu().numpy(), nk)
    lo, go = om.loss_and_grads(_f64(p), kid, N, bx, by, t.astype(np.float64))
    assert abs(float(loss.cpu()[0]) - lo) <= 1e-2 * lo
    for k in om.PARAM_NAMES:
        if k == "b3":
            assert abs(float(g[k]) - float(go[k])) <= 2e-2 * abs(float(go[k])) + 1e-4, k
            continue
        assert _rel(g[k], go[k]) < 2e-2, (k, _rel(g[k], go[k]))
        assert _cos(g[k], go[k]) > 0.999, (k, _cos(g[k], go[k]))


def test_adam_update_matches_oracle(klr):
    """Given the gradients the GPU computed, its Adam update equals the oracle's (FP32)."""
    import torch
    rng = np.random.default_rng(2)
    nk = 8
    p = synth.mlp_init(3, nk)
    blob = klr.surrogate_alloc(p, nk)
    B = 256
    kid, N, bx, by = _samples(rng, B, nk)
    t = rng.normal(size=B).astype(np.float32)
    grads, _ = klr.surrogate_step(blob, nk, _dev(kid), _dev(N), _dev(np.stack([bx, by], 1).reshape(-1)),
                                  _dev(t), lr=1e-3, step=1)
    torch.cuda.synchronize()
    from paper_1911_02373_amd.klr import grads_to_dict
    g = grads_to_dict(klr.lib, grads.cpu().numpy(), nk)
    got = klr.surrogate_params(blob, nk)
    # the kernel's hyper-parameters are FP32 values: give the oracle the same numbers
    b1, b2, eps, lr = (float(np.float32(x)) for x in (0.9, 0.999, 1e-8, 1e-3))
    p2, m2, v2 = om.adam_step(_f64(p), g, om.zeros_like(_f64(p)), om.zeros_like(_f64(p)), 1, lr=lr,
                              beta1=b1, beta2=b2, eps=eps)
    for k in om.PARAM_NAMES:
        assert np.max(np.abs(got["P"][k] - p2[k])) <= 2e-6, k
        assert np.allclose(got["M"][k], m2[k], rtol=1e-5, atol=1e-12), k
        assert np.allclose(got["V"][k], v2[k], rtol=1e-5, atol=1e-15), k


def _trained(klr, n_progs=64, epochs=6, seed=4):
    import torch
    from paper_1911_02373_amd.klr import DeviceEval, grid_samples
    pb = synth.config3_programs(seed, n_progs=n_progs, n_q=256)
    tq = synth.surrogate_training_queries(seed + 1, pb, n_q=32)
    de = DeviceEval.from_batch(klr, tq, with_costs=True)
    _, _, costs, _ = klr.eval_argmin(de, want_costs=True)
    kid, N, L, cost = grid_samples(tq, de, costs)
    p = synth.mlp_init(seed, n_progs)
    blob = klr.surrogate_alloc(p, n_progs)
    loss = klr.surrogate_train(blob, n_progs, kid, N, L, cost, lr=2e-3, batch=1024, epochs=epochs, seed=seed)
    torch.cuda.synchronize()
    return pb, blob, loss.cpu().numpy()


@pytest.fixture(scope="module")
def trained(klr):
    return _trained(klr)


def test_training_reduces_loss(trained):
    _, _, loss = trained
    assert np.all(np.isfinite(loss))
    assert loss[-1] < 0.25 * loss[0], loss


def test_selection_fallback_semantics(klr, trained):
    import torch
    from paper_1911_02373_amd.klr import DeviceEval
    pb, blob, _ = trained
    nk = pb.n_progs
    de = DeviceEval.from_batch(klr, pb)
    ea, eb, _, _ = klr.eval_argmin(de)
    torch.cuda.synchronize()
    ea, eb = ea.cpu().numpy(), eb.cpu().numpy()
    # every query falls back: identical to the exact path, bit for bit
    am, pc, fb = klr.surrogate_eval(blob, nk, de, margin=1e9)
    torch.cuda.synchronize()
    assert np.all(fb.cpu().numpy() == 1)
    assert np.array_equal(am.cpu().numpy(), ea)
    assert np.array_equal(pc.cpu().numpy().view(np.uint32), eb.view(np.uint32))
    # the 2 % margin: fallback queries equal the exact path; the others are admissible
    am, pc, fb = klr.surrogate_eval(blob, nk, de, margin=0.02)
    torch.cuda.synchronize()
    am, pc, fb = am.cpu().numpy(), pc.cpu().numpy(), fb.cpu().numpy().astype(bool)
    assert np.array_equal(am[fb], ea[fb])
    assert np.array_equal(pc[fb].view(np.uint32), eb[fb].view(np.uint32))
    cfg = synth.config3_launch_configs()
    picked = cfg[am[~fb]]
    Nq = pb.queries[~fb]
    assert np.all(am[~fb] >= 0) and np.all(am[~fb] < 127)
    assert np.all(picked.max(axis=1) <= Nq) and np.all(np.isfinite(pc[~fb])) and np.all(pc[~fb] > 0)
    assert 0.0 < fb.mean() < 1.0


def test_selection_regret_small(klr, trained):
    """Regret of the surrogate+fallback picks, judged by the exact rational program."""
    import torch
    from paper_1911_02373_amd.klr import DeviceEval
    pb, blob, _ = trained
    de = DeviceEval.from_batch(klr, pb, with_costs=True)
    ea, eb, costs, _ = klr.eval_argmin(de, want_costs=True)
    am, _, fb = klr.surrogate_eval(blob, pb.n_progs, de, margin=0.02)
    torch.cuda.synchronize()
    ea, eb, am = ea.cpu().numpy(), eb.cpu().numpy(), am.cpu().numpy()
    C = costs.cpu().numpy().reshape(pb.n_progs, 128, -1)
    nq = int(pb.n_q[0])
    picked = C[np.repeat(np.arange(pb.n_progs), nq), am, np.tile(np.arange(nq), pb.n_progs)]
    ok = ea >= 0
    assert np.all(np.isfinite(picked[ok & ~fb.cpu().numpy().astype(bool)]))
    regret = picked[ok].astype(np.float64) / eb[ok] - 1.0
    assert np.all(regret >= 0)
    assert np.median(regret) < 0.01


def test_training_gain_over_untrained_network(klr, trained):
    """What learning buys, with the same network, kernels and 2 % fallback rule: the untrained
    weights are confidently wrong (large predicted margins, so almost no query falls back and
    the picks are poor), while the trained weights' margins are informative, so the combined
    picks are within 1 % of the exact optimum far more often.  The network alone is reported,
    not asserted: its log-cycle error is too coarse to separate configurations within 1 %."""
    import torch
    from paper_1911_02373_amd.klr import DeviceEval
    pb, blob, _ = trained
    nk = pb.n_progs
    blob0 = klr.surrogate_alloc(synth.mlp_init(4, nk), nk)       # the trained net's initial weights
    de = DeviceEval.from_batch(klr, pb, with_costs=True)
    ea, eb, costs, _ = klr.eval_argmin(de, want_costs=True)
    torch.cuda.synchronize()
    C = costs.cpu().numpy().reshape(nk, 128, -1)
    nq = int(pb.n_q[0])
    ea, eb = ea.cpu().numpy(), eb.cpu().numpy()
    ok = ea >= 0

    def judge(b, margin):
        am, _, fb = klr.surrogate_eval(b, nk, de, margin=margin)
        torch.cuda.synchronize()
        a = am.cpu().numpy()
        picked = C[np.repeat(np.arange(nk), nq), np.maximum(a, 0), np.tile(np.arange(nq), nk)]
        regret = picked[ok].astype(np.float64) / eb[ok] - 1.0
        return float(np.mean(regret <= 0.01)), 1.0 - float(fb.cpu().numpy().astype(bool).mean())

    fb_t, settled_t = judge(blob, 0.02)
    fb_0, settled_0 = judge(blob0, 0.02)
    alone_t, _ = judge(blob, 0.0)
    alone_0, _ = judge(blob0, 0.0)
    print(f"with the 2 % fallback, picks within 1 %: trained {fb_t:.3f}, untrained {fb_0:.3f}; settled "
          f"without the exact program: trained {settled_t:.3f}, untrained {settled_0:.3f}; network alone "
          f"within 1 %: trained {alone_t:.3f}, untrained {alone_0:.3f}")
    assert settled_0 > 0.5                      # the untrained net is (over)confident
    assert fb_t >= 0.8 and fb_t >= fb_0 + 0.3, (fb_t, fb_0)


def test_uneven_programs_train_and_select(klr):
    """Programs with two launch parameters but uneven configuration lists and query counts
    (including configurations that are not admissible), trained from klr.program_samples; with
    an infinite margin the selection equals the exact path bit for bit, with 2 % the fallback
    queries equal it and the others pick one of their program's configurations.  Data sizes
    N >= 2^10.5 keep at least two configurations statically admissible per query (with a
    single candidate the margin is infinite and no query falls back)."""
    import torch
    from paper_1911_02373_amd.klr import DeviceEval, program_samples
    pb = synth.mixed_programs(31, 12, n_q_range=(1, 300), n_cfg_range=(8, 127), v_launch_choices=(2,),
                              log2_range=(10.5, 26.0))
    tq = synth.surrogate_training_queries(32, pb, n_q=16)
    de_t = DeviceEval.from_batch(klr, tq, with_costs=True)
    _, _, costs, _ = klr.eval_argmin(de_t, want_costs=True)
    kid, N, L, cost = program_samples(tq, de_t, costs)
    blob = klr.surrogate_alloc(synth.mlp_init(5, pb.n_progs), pb.n_progs)
    loss = klr.surrogate_train(blob, pb.n_progs, kid, N, L, cost, lr=2e-3, batch=1024, epochs=4, seed=5)
    de = DeviceEval.from_batch(klr, pb)
    ea, eb, _, _ = klr.eval_argmin(de)
    am, pc, fb = klr.surrogate_eval(blob, pb.n_progs, de, margin=1e9)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(loss.cpu().numpy()))
    ea, eb = ea.cpu().numpy(), eb.cpu().numpy()
    assert np.all(fb.cpu().numpy() == 1)
    assert np.array_equal(am.cpu().numpy(), ea)
    assert np.array_equal(pc.cpu().numpy().view(np.uint32), eb.view(np.uint32))
    am, pc, fb = klr.surrogate_eval(blob, pb.n_progs, de, margin=0.02)
    torch.cuda.synchronize()
    am, pc, fb = am.cpu().numpy(), pc.cpu().numpy(), fb.cpu().numpy().astype(bool)
    assert np.array_equal(am[fb], ea[fb])
    # every pick the network keeps has a finite exact cost (an inadmissible pick falls back)
    dc = DeviceEval.from_batch(klr, pb, with_costs=True)
    _, _, xc, _ = klr.eval_argmin(dc, want_costs=True)
    torch.cuda.synchronize()
    xc = xc.cpu().numpy()
    co = 0
    for p in range(pb.n_progs):
        nc, nq, q0 = int(pb.n_cfg[p]), int(pb.n_q[p]), int(pb.q0[p])
        q = np.arange(q0, q0 + nq)
        own = q[~fb[q]]
        assert np.all((am[own] >= 0) & (am[own] < nc))
        Cp = xc[co: co + nc * nq].reshape(nc, nq)
        assert np.all(np.isfinite(Cp[am[own], own - q0])), p
        co += nc * nq


def test_selection_ranks_only_admissible_configurations(klr):
    """With sigma = 0 every prediction is equal, so the network ranks configurations by index.
    Configurations 0 and 1 (512 and 1024 threads at R = 300 registers per thread) leave no
    block resident, so the exact program rules them out and the selection never ranks them.
    With margin 0 (the margin rule never fires) and a shortlist of one, every query keeps the
    first admissible configuration, 2; with a shortlist of four the three admissible
    configurations are re-ranked by their exact costs, so the pick is the exact argmin."""
    import torch
    from paper_1911_02373_amd.klr import OPT_SURR_SHORTLIST, DeviceEval
    from tests.helpers import constant_programs
    rows = [[40.0, 6.0, 3.0, 2.0, 1.0, 300.0, 0.0, 64.0]] * 3
    cfgs = [[512, 1], [1024, 1], [64, 1], [128, 1], [32, 8]]
    pb = constant_programs(rows, cfgs, [[1024, 4096, 65536, 1 << 20]] * 3)
    nk = pb.n_progs
    blob = klr.surrogate_alloc(synth.mlp_init(9, nk), nk, mu=0.0, sigma=0.0)
    de = DeviceEval.from_batch(klr, pb)
    ea, _, _, _ = klr.eval_argmin(de)
    klr.set_option(OPT_SURR_SHORTLIST, 1)
    try:
        am, pc, fb = klr.surrogate_eval(blob, nk, de, margin=0.0)
        torch.cuda.synchronize()
    finally:
        klr.set_option(OPT_SURR_SHORTLIST, 4)
    ea = ea.cpu().numpy()
    assert np.all(np.isin(ea, [2, 3, 4]))                       # the exact picks are the admissible ones
    assert np.all(fb.cpu().numpy() == 0)
    assert np.all(am.cpu().numpy() == 2)
    assert np.all(pc.cpu().numpy() == 1.0)                     # exp(mu + 0 * y)
    am4, pc4, fb4 = klr.surrogate_eval(blob, nk, de, margin=0.0)
    torch.cuda.synchronize()
    assert np.all(fb4.cpu().numpy() == 0)
    assert np.array_equal(am4.cpu().numpy(), ea)
    assert np.all(pc4.cpu().numpy() == 1.0)


def test_shortlist_reranks_the_networks_best_by_exact_cost(klr, trained):
    """Shortlist of four with margin 0 (only an all-inadmissible shortlist falls back), query by
    query (8 programs x 256 queries): where the oracle network's four best predictions are
    separated from the rest by more than twice the accumulation bound 2^-15 S (so the shortlist
    is unambiguous up to a rare first-layer bfloat16 flip), a query falls back exactly when the
    four exact costs are all +inf, and otherwise picks the configuration of lowest exact FP32
    cost (oracle replay, lowest index on ties) among those four - all but at most 1 % of them -
    and never one worse than the network's own pick."""
    import torch
    from paper_1911_02373_amd.klr import OPT_SURR_SHORTLIST, DeviceEval
    pb, blob, _ = trained
    nk = pb.n_progs
    sub = synth.take_programs(pb, 8)
    de = DeviceEval.from_batch(klr, sub)
    am4, _, fb4 = klr.surrogate_eval(blob, nk, de, margin=0.0)
    klr.set_option(OPT_SURR_SHORTLIST, 1)
    try:
        am1, _, fb1 = klr.surrogate_eval(blob, nk, de, margin=0.0)
        torch.cuda.synchronize()
    finally:
        klr.set_option(OPT_SURR_SHORTLIST, 4)
    am4, fb4 = am4.cpu().numpy(), fb4.cpu().numpy().astype(bool)
    am1, fb1 = am1.cpu().numpy(), fb1.cpu().numpy().astype(bool)
    prm = klr.surrogate_params(blob, nk)
    refs, scales = _select_reference(prm, sub, sub.n_progs)
    checked = off = 0
    for p in range(sub.n_progs):
        nq, q0 = int(sub.n_q[p]), int(sub.q0[p])
        X = oc.program_costs(sub, p)                         # exact FP32 costs [n_cfg][nq]
        R, S = refs[p], scales[p]
        for i in range(nq):
            o = q0 + i
            row = R[i]
            fin = np.isfinite(row)
            if fin.sum() < 5:
                continue
            order = np.argsort(row, kind="stable")
            acc = 2.0 ** -15 * float(S[i][fin].max())
            if row[order[4]] - row[order[3]] <= 2 * acc:
                continue
            short = order[:4]
            xs = X[short, i]
            assert fb4[o] == (not np.isfinite(xs).any()), (p, i)
            if fb4[o]:
                continue
            if not fb1[o]:
                assert X[am4[o], i] <= X[am1[o], i], (p, i)
            want = short[np.lexsort((short, xs))[0]]
            checked += 1
            off += int(am4[o] != want)
    print(f"shortlist picks checked: {checked}, different from the oracle shortlist's best: {off}")
    assert checked > 100 and off <= 0.01 * checked, (checked, off)


def test_pick_check_sends_inadmissible_picks_to_the_exact_path(klr):
    """A pick whose cycle estimate overflows FP32 is admissible by every constraint the
    selection checks (metrics defined, blocks resident) but has exact cost +inf: I_comp = 1e38
    makes the compute cycles 4 (I_comp + I_m) overflow.  With margin 0 only the pick check can
    send a query to the exact path: every query falls back and the result equals the exact
    path bit for bit (no admissible configuration: -1 and +inf)."""
    import torch
    from paper_1911_02373_amd.klr import DeviceEval
    from tests.helpers import constant_programs
    rows = [[1e38, 6.0, 3.0, 2.0, 1.0, 300.0, 0.0, 64.0]] * 3
    cfgs = [[512, 1], [1024, 1], [64, 1], [128, 1], [32, 8]]
    pb = constant_programs(rows, cfgs, [[1024, 4096, 65536, 1 << 20]] * 3)
    nk = pb.n_progs
    blob = klr.surrogate_alloc(synth.mlp_init(9, nk), nk, mu=0.0, sigma=0.0)
    de = DeviceEval.from_batch(klr, pb)
    ea, eb, _, _ = klr.eval_argmin(de)
    am, pc, fb = klr.surrogate_eval(blob, nk, de, margin=0.0)
    torch.cuda.synchronize()
    ea, eb = ea.cpu().numpy(), eb.cpu().numpy()
    assert np.all(ea == -1) and np.all(np.isinf(eb))
    assert np.all(fb.cpu().numpy() == 1)
    assert np.array_equal(am.cpu().numpy(), ea)
    assert np.array_equal(pc.cpu().numpy().view(np.uint32), eb.view(np.uint32))


def _select_reference(prm, pb, n_progs):
    """Oracle predictions (ln C) of every admissible configuration of each query of the first
    n_progs programs (finite cost in the oracle's FP32 replay of the exact program; these
    programs' costs never overflow, so that is exactly the set the selection ranks), with the
    operands the selection kernel rounds to bfloat16 rounded the same way; +inf elsewhere.  Also S = sum |w3| (|W2| h1 +
    |b2|) per point (times sigma): the FP32 accumulations of layers 2 and 3 (exact bfloat16
    products, 257-term sums) stay within 2 * 257 * 2^-24 S < 2^-15 S of the FP64 values; a
    first-layer value that the kernel's FP32 products round to the other neighbour in bfloat16
    (rare: the two FP32 values differ by a few units of 2^-24) moves the output by at most one
    bfloat16 step of that value's term, below 2^-8 S."""
    P = prm["P"]
    cfg = pb.cfgs.reshape(-1, 2)
    out, scale = [], []
    for p in range(n_progs):
        nq, nc = int(pb.n_q[p]), int(pb.n_cfg[p])
        q0, c0 = int(pb.q0[p]), int(pb.cfg0[p]) // 2
        N = pb.queries[q0:q0 + nq].astype(np.int64)
        C = cfg[c0:c0 + nc].astype(np.int64)
        kid = np.full(nq * nc, p)
        NN = np.repeat(N, nc)
        bx, by = np.tile(C[:, 0], nq), np.tile(C[:, 1], nq)
        y = om.forward_bf16(P, kid, NN, bx, by).reshape(nq, nc)
        x = om.features(NN, bx, by, P["emb"][kid])
        h1 = om.bf16_round(np.maximum(x @ P["W1"].T + P["b1"], 0.0))
        s = (np.abs(h1) @ np.abs(om.bf16_round(P["W2"])).T + np.abs(P["b2"])) @ np.abs(P["w3"])
        ok = np.isfinite(oc.program_costs(pb, p)).T
        out.append(np.where(ok, prm["mu"] + prm["sigma"] * y, np.inf))
        scale.append(s.reshape(nq, nc) * abs(prm["sigma"]))
    return out, scale


def test_selection_matches_network_elementwise(klr, trained):
    """mlp_select against the network oracle, query by query (8 programs x 256 queries x 128
    configurations), with a shortlist of one (the network's own pick).  Every query: the predicted ln C of its pick and its predicted margin
    (second best minus best) are within the bfloat16-flip bound 2^-8 S of the oracle's minimum
    and margin over the admissible configurations, and 99 % within the accumulation
    bound 2^-15 S.  Wherever the oracle's margin exceeds twice the accumulation bound the pick
    is the oracle's argmin, except for at most 1 % of those queries (a first-layer bfloat16
    flip), whose pick is then within the flip bound of the oracle's minimum (at least a tenth of
    the queries are that far from a tie).  With margin 0 only
    a pick the exact program rules out falls back; at 2 % the fallback flag follows the
    oracle's margin away from the threshold."""
    import torch
    from paper_1911_02373_amd.klr import DeviceEval
    from paper_1911_02373_amd.klr import OPT_SURR_SHORTLIST
    pb, blob, _ = trained
    nk = pb.n_progs
    sub = synth.take_programs(pb, 8)
    de = DeviceEval.from_batch(klr, sub)
    ql = int(sub.queries.size)
    marg = torch.empty(ql, dtype=torch.float32, device="cuda")
    st = torch.empty(sub.n_progs, dtype=torch.int32, device="cuda")
    ea, eb, _, _ = klr.eval_argmin(de)
    klr.set_option(OPT_SURR_SHORTLIST, 1)                    # the network's own picks
    try:
        am, pc, fb = klr.surrogate_eval(blob, nk, de, margin=0.0, pred_margin=marg, prog_status=st)
        am2, _, fb2 = klr.surrogate_eval(blob, nk, de, margin=0.02)
        torch.cuda.synchronize()
    finally:
        klr.set_option(OPT_SURR_SHORTLIST, 4)
    am, pc, fb, marg = am.cpu().numpy(), pc.cpu().numpy(), fb.cpu().numpy().astype(bool), marg.cpu().numpy()
    ea, eb = ea.cpu().numpy(), eb.cpu().numpy()
    fb2, am2 = fb2.cpu().numpy().astype(bool), am2.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    prm = klr.surrogate_params(blob, nk)
    refs, scales = _select_reference(prm, sub, sub.n_progs)
    checked = tight = strict = strict_off = 0
    worst = 0.0
    for p in range(sub.n_progs):
        nq, q0 = int(sub.n_q[p]), int(sub.q0[p])
        R, S = refs[p], scales[p]
        for i in range(nq):
            o = q0 + i
            row = R[i]
            fin = np.isfinite(row)
            if fin.sum() < 2:
                continue
            order = np.argsort(row, kind="stable")          # lowest index among equal values
            b0, b1 = row[order[0]], row[order[1]]
            smax = float(S[i][fin].max())
            loose, acc = 2.0 ** -8 * smax, 2.0 ** -15 * smax
            d_marg = abs(marg[o] - (b1 - b0))
            assert d_marg <= 2 * loose, (p, i, marg[o], b1 - b0, loose)
            d_val = 0.0
            if not fb[o]:
                assert np.isfinite(row[am[o]]), (p, i, am[o])
                d_val = abs(np.log(pc[o]) - b0)
                assert d_val <= loose + 1e-6 * abs(b0), (p, i, np.log(pc[o]), b0, loose)
                if b1 - b0 > 2 * acc:
                    strict += 1
                    if am[o] != order[0]:
                        strict_off += 1
                        assert row[am[o]] - b0 <= 2 * loose, (p, i, am[o], order[0])
            else:
                # margin 0: a fallback means the exact program rules the pick out
                assert not np.isfinite(eb[o]) or am[o] == ea[o]
            tight += int(d_marg <= 2 * acc + 1e-6 * abs(b0) and d_val <= acc + 1e-6 * abs(b0))
            worst = max(worst, d_val / max(acc, 1e-30))
            # the 2 % rule, away from its threshold
            if not fb[o] and (b1 - b0) > np.log1p(0.02) + 2 * loose:
                assert not fb2[o] and am2[o] == am[o], (p, i)
            if (b1 - b0) < np.log1p(0.02) - 2 * loose:
                assert fb2[o], (p, i)
            checked += 1
    print(f"checked {checked} queries: within the accumulation bound {tight / checked:.4f}; picks compared "
          f"{strict}, off the oracle's {strict_off}; worst value error {worst:.2f} accumulation bounds")
    assert checked > 0.9 * ql
    assert tight >= 0.99 * checked, (tight, checked)
    assert strict > 0.1 * checked and strict_off <= 0.01 * strict, (strict, strict_off, checked)


def test_surrogate_bad_descriptor_and_shared_query_ranges(klr, trained):
    """Program 1's fit range lies outside the batch: it gets KLR_PROG_BAD_DESC and the selection
    writes none of its outputs (as klr_eval_argmin does); programs 0 and 2 are answered as
    usual.  Programs 3 and 4 are the same program over the same query range: each counts its
    flagged queries over that range, so the compacted lists (2 n_q entries for n_q queries)
    stay inside the workspace, and both answer with the exact path's result."""
    import copy

    import torch
    from paper_1911_02373_amd.klr import DeviceEval
    pb, blob, _ = trained
    sub = copy.copy(synth.take_programs(pb, 5))
    sub.fit0 = sub.fit0.copy()
    sub.q0, sub.cfg0 = sub.q0.copy(), sub.cfg0.copy()
    sub.fit0[1] = 10 ** 6
    sub.fit0[4], sub.cfg0[4], sub.q0[4] = sub.fit0[3], sub.cfg0[3], sub.q0[3]
    de = DeviceEval.from_batch(klr, sub)
    ql = int(sub.queries.size)
    ea, eb, _, est = klr.eval_argmin(de)
    out = (torch.full((ql,), -7, dtype=torch.int32, device="cuda"),
           torch.full((ql,), 123.0, dtype=torch.float32, device="cuda"),
           torch.full((ql,), 9, dtype=torch.uint8, device="cuda"))
    st = torch.full((sub.n_progs,), -1, dtype=torch.int32, device="cuda")
    am, pc, fb = klr.surrogate_eval(blob, pb.n_progs, de, margin=1e9, out=out, prog_status=st)
    torch.cuda.synchronize()
    am, pc, fb = am.cpu().numpy(), pc.cpu().numpy(), fb.cpu().numpy()
    ea, eb = ea.cpu().numpy(), eb.cpu().numpy()
    assert list(st.cpu().numpy()) == [0, 1, 0, 0, 0] == list(est.cpu().numpy())
    r1 = slice(int(sub.q0[1]), int(sub.q0[1] + sub.n_q[1]))
    assert np.all(am[r1] == -7) and np.all(pc[r1] == 123.0) and np.all(fb[r1] == 9)
    for p in (0, 2, 3):
        r = slice(int(sub.q0[p]), int(sub.q0[p] + sub.n_q[p]))
        assert np.all(fb[r] == 1)
        assert np.array_equal(am[r], ea[r]) and np.array_equal(pc[r].view(np.uint32), eb[r].view(np.uint32))

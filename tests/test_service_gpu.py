"""The launch-time decision service on the device: decisions equal klr_eval_argmin's, repeated
data sizes come from the history, constraints restrict the argmin exactly as a host-side
masked argmin over the device's cost rows does, and launch dimensions follow the grid kind."""
import numpy as np
import pytest

from paper_1911_02373_amd import synth

pytestmark = pytest.mark.gpu


def _py_ok(expr, N, L):
    env = {"N": N, "bx": L[0], "by": L[1] if len(L) > 1 else 1, "bz": L[2] if len(L) > 2 else 1}
    env["T"] = int(np.prod(L))
    env.update(min=min, max=max, abs=abs)
    try:
        return bool(eval(expr, {"__builtins__": {}}, env))
    except ZeroDivisionError:
        return False


def test_service_decisions_history_and_constraints(klr):
    import torch
    from paper_1911_02373_amd.klr import DeviceEval, Service
    pb = synth.mixed_programs(71, 10, n_q_range=(50, 300), n_cfg_range=(20, 160))
    de = DeviceEval.from_batch(klr, pb, with_costs=True)
    ea, eb, costs, st = klr.eval_argmin(de, want_costs=True)
    torch.cuda.synchronize()
    ea, eb, costs = ea.cpu().numpy(), eb.cpu().numpy(), costs.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    svc = Service(klr, de, pb, max_batch=128)
    try:
        off = 0
        offs = []
        for p in range(pb.n_progs):
            offs.append(off)
            off += int(pb.n_cfg[p]) * int(pb.n_q[p])
        total_miss = 0
        for p in range(pb.n_progs):
            q0, nq = int(pb.q0[p]), int(pb.n_q[p])
            N = pb.queries[q0:q0 + nq]
            out = svc.decide(p, N)                     # more than max_batch sizes: several evaluations
            total_miss += len(np.unique(N))
            assert np.array_equal(out["config"], ea[q0:q0 + nq]), p
            assert np.array_equal(out["cost"].view(np.uint32), eb[q0:q0 + nq].view(np.uint32)), p
            # launch dimensions
            vl = int(pb.v_launch[p])
            cfg = pb.cfgs[int(pb.cfg0[p]): int(pb.cfg0[p]) + int(pb.n_cfg[p]) * vl].reshape(-1, vl)
            for j in np.nonzero(out["config"] >= 0)[0][:20]:
                L = cfg[out["config"][j]]
                n = int(N[j])
                assert out["bx"][j] == L[0] and out["by"][j] == (L[1] if vl > 1 else 1)
                if int(pb.grid_kind[p]) == 1:
                    assert out["gx"][j] == -(-n // L[0]) and out["gy"][j] == -(-n // L[1])
                else:
                    assert out["gx"][j] == -(-n // int(np.prod(L))) and out["gy"][j] == 1
            # the same sizes again: every one from the history
            st0 = svc.stats()
            again = svc.decide(p, N[::-1])
            assert np.array_equal(again["config"], out["config"][::-1])
            assert svc.stats()["hits"] - st0["hits"] == nq and svc.stats()["misses"] == st0["misses"]
        s = svc.stats()
        assert s["misses"] == sum(int(x) for x in pb.n_q) and s["entries"] == total_miss, (s, total_miss)
        # constraints: the masked argmin over the cost rows, strict "<" in configuration order
        exprs = ["bx * by <= 256 and bx <= N // 64", "bx >= 8 or T < 128"]
        for e in exprs:
            svc.add_constraint(-1, e)
        for p in range(pb.n_progs):
            q0, nq, nc = int(pb.q0[p]), int(pb.n_q[p]), int(pb.n_cfg[p])
            vl = int(pb.v_launch[p])
            cfg = pb.cfgs[int(pb.cfg0[p]): int(pb.cfg0[p]) + nc * vl].reshape(-1, vl)
            C = costs[offs[p]: offs[p] + nc * nq].reshape(nc, nq)
            N = pb.queries[q0:q0 + nq]
            out = svc.decide(p, N)
            for q in range(nq):
                best, bi = np.float32(np.inf), -1
                for c in range(nc):
                    if C[c, q] < best and all(_py_ok(e, int(N[q]), list(cfg[c])) for e in exprs):
                        best, bi = C[c, q], c
                assert out["config"][q] == bi and (bi < 0 or out["cost"][q] == best), (p, q)
    finally:
        svc.close()

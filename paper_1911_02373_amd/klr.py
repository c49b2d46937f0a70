"""ctypes binding of libklr.so (include/klr.h): argument marshalling only.

Every step of the fit, evaluation and argmin runs in the HIP library; this module only lays
out descriptors, uploads arrays with torch (device memory and streams), and calls the C ABI.
There is no CPU fallback: without the built library or a GPU, `Library.get()` raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libklr.so")

KLR_OK, KLR_E_INVALID, KLR_E_WORKSPACE, KLR_E_HIP, KLR_E_UNSUPPORTED = 0, -1, -2, -3, -4
KLR_FP64, KLR_FP32_REFINED, KLR_BF16_REFINED, KLR_FP64_SVD = 0, 1, 2, 3
GRID_1D, GRID_2D = 0, 1
N_METRICS = 8
MAX_VARS = 8

FIT_DESC = np.dtype([("x0", "<i8"), ("f0", "<i8"), ("coef0", "<i8"), ("m", "<i4"), ("v", "<i4"),
                     ("num0", "<i4"), ("n_num", "<i4"), ("den0", "<i4"), ("n_den", "<i4"),
                     ("scale_exp", "i1", (MAX_VARS,))])
FIT_INFO = np.dtype([("status", "<u4"), ("rank", "<i4"), ("iters", "<i4"), ("q_nonpos", "<i4"),
                     ("resid_norm", "<f8"), ("err_est", "<f8")])
HW = np.dtype([("n_cu", "<i4"), ("wave", "<i4"), ("w_max", "<i4"), ("b_max", "<i4"),
               ("r_max", "<i4"), ("z_max", "<i4"), ("t_max", "<i4"), ("reserved", "<i4"),
               ("mem_lat", "<f4"), ("dep_delay", "<f4"), ("issue_cycles", "<f4"), ("bw", "<f4")])
PROGRAM = np.dtype([("cfg0", "<i8"), ("q0", "<i8"), ("cost0", "<i8"), ("fit0", "<i4"),
                    ("v_launch", "<i4"), ("n_cfg", "<i4"), ("n_q", "<i4"), ("grid_kind", "<i4"),
                    ("cost_kind", "<i4")])

EXPORTS = ("klr_create", "klr_destroy", "klr_last_error", "klr_fit_workspace", "klr_fit_batched",
           "klr_eval_workspace", "klr_eval_argmin", "klr_abi_layout", "klr_profile_enable",
           "klr_profile_read", "klr_surrogate_param_bytes", "klr_surrogate_layout",
           "klr_surrogate_train_workspace", "klr_surrogate_train", "klr_surrogate_predict",
           "klr_surrogate_step", "klr_surrogate_eval_workspace", "klr_surrogate_eval", "klr_surrogate_init",
           "klr_set_option", "klr_capture_begin", "klr_capture_end", "klr_graph_launch", "klr_graph_destroy",
           "klr_selftest_divisors", "klr_selftest_divisor_list", "klr_selftest_short_division",
           "klr_eval_argmin_noalloc", "klr_service_workspace", "klr_service_create", "klr_service_destroy",
           "klr_service_add_constraint", "klr_service_decide", "klr_service_stats",
           "klr_service_set_history_limit", "klr_constraint_check", "klr_collect_buffer",
           "klr_target_attributes", "klr_collect_times")
TARGET_TRANSPOSE, TARGET_STENCIL = 0, 1
OPT_FIT_PERSISTENT, OPT_EVAL_VARIANT, OPT_FIT_VARIANT, OPT_SURR_SHORTLIST = 0, 1, 2, 3
K_COLLAPSE, K_EVAL, K_FIT_GRAM, K_FIT_SOLVE, K_MLP, K_SURR, K_FALLBACK = 0, 1, 2, 3, 4, 5, 6
TRAIN_CFG = np.dtype([("lr", "<f4"), ("beta1", "<f4"), ("beta2", "<f4"), ("eps", "<f4"),
                      ("batch", "<i4"), ("epochs", "<i4"), ("seed", "<u8")])
MLP_PARAMS = ("W2", "W1", "b1", "b2", "w3", "b3", "emb")


class KlrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"klr status {status}: {msg}")
        self.status = status


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libklr.so and declare the C signatures (no GPU needed)."""
    if not os.path.exists(path):
        raise RuntimeError(f"libklr.so not built at {path}: run `python -m paper_1911_02373_amd.build`")
    lib = ctypes.CDLL(path)
    P, I32, I64, SZ, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
    lib.klr_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
    lib.klr_create.restype = I32
    lib.klr_destroy.argtypes = [P]
    lib.klr_destroy.restype = None
    lib.klr_last_error.argtypes = [P]
    lib.klr_last_error.restype = ctypes.c_char_p
    lib.klr_abi_layout.argtypes = [ctypes.POINTER(I64), I32]
    lib.klr_abi_layout.restype = I32
    lib.klr_fit_workspace.argtypes = [I32, I64, I32]
    lib.klr_fit_workspace.restype = SZ
    lib.klr_fit_batched.argtypes = [P, P, I32, P, I32, P, I64, P, I64, I32, I32, D, P, I64, P, P, SZ, P]
    lib.klr_fit_batched.restype = I32
    lib.klr_eval_workspace.argtypes = [I32, I32]
    lib.klr_eval_workspace.restype = SZ
    lib.klr_eval_argmin.argtypes = [P, P, I32, I32, I32, P, P, I32, P, I32, P, I64, P, I64, P, I64,
                                    P, P, P, I64, P, P, SZ, P]
    lib.klr_eval_argmin.restype = I32
    lib.klr_eval_argmin_noalloc.argtypes = [P, P, I32, I32, I32, P, P, I32, P, I32, P, I64, P, I64, P, I64,
                                            P, P, P, I64, P, P]
    lib.klr_eval_argmin_noalloc.restype = I32
    lib.klr_profile_enable.argtypes = [P, I32]
    lib.klr_profile_enable.restype = I32
    lib.klr_profile_read.argtypes = [P, I32, ctypes.POINTER(D), ctypes.POINTER(I64)]
    lib.klr_profile_read.restype = I32
    F = ctypes.c_float
    lib.klr_surrogate_param_bytes.argtypes = [I32]
    lib.klr_surrogate_param_bytes.restype = SZ
    lib.klr_capture_begin.argtypes = [P, P]
    lib.klr_capture_begin.restype = I32
    lib.klr_capture_end.argtypes = [P, P, ctypes.POINTER(P)]
    lib.klr_capture_end.restype = I32
    lib.klr_graph_launch.argtypes = [P, P, P]
    lib.klr_graph_launch.restype = I32
    lib.klr_graph_destroy.argtypes = [P]
    lib.klr_graph_destroy.restype = None
    lib.klr_selftest_divisors.argtypes = [ctypes.c_uint32]
    lib.klr_selftest_divisors.restype = I64
    lib.klr_selftest_divisor_list.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.klr_selftest_divisor_list.restype = I64
    lib.klr_selftest_short_division.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.klr_selftest_short_division.restype = I64
    lib.klr_set_option.argtypes = [P, I32, I64]
    lib.klr_set_option.restype = I32
    lib.klr_surrogate_init.argtypes = [P, P, I32, P]
    lib.klr_surrogate_init.restype = I32
    lib.klr_surrogate_layout.argtypes = [I32, ctypes.POINTER(I64), I32]
    lib.klr_surrogate_layout.restype = I32
    lib.klr_surrogate_train_workspace.argtypes = [I32, I32]
    lib.klr_surrogate_train_workspace.restype = SZ
    lib.klr_surrogate_train.argtypes = [P, P, I32, P, P, P, P, I64, P, P, P, SZ, P]
    lib.klr_surrogate_train.restype = I32
    lib.klr_surrogate_predict.argtypes = [P, P, I32, P, P, P, I64, P, P]
    lib.klr_surrogate_predict.restype = I32
    lib.klr_surrogate_step.argtypes = [P, P, I32, P, P, P, P, I32, F, I32, F, F, F, P, P, P, SZ, P]
    lib.klr_surrogate_step.restype = I32
    lib.klr_surrogate_eval_workspace.argtypes = [I32, I32, I32]
    lib.klr_surrogate_eval_workspace.restype = SZ
    lib.klr_surrogate_eval.argtypes = [P, P, I32, P, I32, I32, I32, P, P, I32, P, I32, P, I64, P, I64,
                                       P, I64, F, P, P, P, P, P, P, SZ, P]
    lib.klr_surrogate_eval.restype = I32
    lib.klr_service_workspace.argtypes = [I32, I32]
    lib.klr_service_workspace.restype = SZ
    lib.klr_service_create.argtypes = [P, ctypes.POINTER(P), P, I32, P, P, I32, P, I32, P, I64, P, P, I64, I32,
                                       P, SZ]
    lib.klr_service_create.restype = I32
    lib.klr_service_destroy.argtypes = [P]
    lib.klr_service_destroy.restype = None
    lib.klr_service_add_constraint.argtypes = [P, I32, ctypes.c_char_p]
    lib.klr_service_add_constraint.restype = I32
    lib.klr_service_decide.argtypes = [P, I32, P, I32, P, P]
    lib.klr_service_decide.restype = I32
    lib.klr_service_stats.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64),
                                      ctypes.POINTER(I64)]
    lib.klr_service_stats.restype = I32
    lib.klr_service_set_history_limit.argtypes = [P, I64]
    lib.klr_service_set_history_limit.restype = I32
    lib.klr_constraint_check.argtypes = [ctypes.c_char_p, I32, P, I32, ctypes.c_char_p, I32]
    lib.klr_constraint_check.restype = I32
    lib.klr_collect_buffer.argtypes = [I32, I32]
    lib.klr_collect_buffer.restype = SZ
    lib.klr_target_attributes.argtypes = [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    lib.klr_target_attributes.restype = I32
    lib.klr_collect_times.argtypes = [P, I32, P, I32, I32, P, P, SZ, P]
    lib.klr_collect_times.restype = I32
    return lib


def constraint_check(lib, expr: str, N: int, L) -> int:
    """[host] 1 / 0 for the constraint at (N, L), -1 on a parse error (raises KlrError)."""
    arr = np.ascontiguousarray(np.asarray(L, np.int32))
    err = ctypes.create_string_buffer(256)
    r = lib.klr_constraint_check(expr.encode(), int(N), arr.ctypes.data if arr.size else None, int(arr.size),
                                 err, 256)
    if r < 0:
        raise KlrError(KLR_E_INVALID, err.value.decode())
    return int(r)


LAUNCH = np.dtype([("gx", "<i4"), ("gy", "<i4"), ("gz", "<i4"), ("bx", "<i4"), ("by", "<i4"), ("bz", "<i4"),
                   ("config", "<i4"), ("cost", "<f4")])


def surrogate_layout(lib, n_kernels: int) -> dict:
    buf = (ctypes.c_int64 * 32)()
    cnt = lib.klr_surrogate_layout(n_kernels, buf, 32)
    v = [int(buf[i]) for i in range(cnt)]
    keys = ("np", "P", "M", "V", "W2b", "W2Tb", "bytes", "W2", "W1", "b1", "b2", "w3", "b3", "emb")
    return dict(zip(keys, v))


def pack_params(lib, params: dict, n_kernels: int, mu: float = 0.0, sigma: float = 1.0) -> np.ndarray:
    """Host blob (uint8) of the surrogate: header (mu, sigma), P from `params`, M = V = 0; the
    BF16 working copies are written by the library."""
    lay = surrogate_layout(lib, n_kernels)
    blob = np.zeros(lay["bytes"], np.uint8)
    f = blob[: (16 + 3 * lay["np"]) * 4].view(np.float32)
    f[0], f[1] = mu, sigma
    P = f[lay["P"]: lay["P"] + lay["np"]]
    for k in MLP_PARAMS:
        a = np.asarray(params[k], np.float32).reshape(-1)
        P[lay[k]: lay[k] + a.size] = a
    return blob


def unpack_params(lib, blob: np.ndarray, n_kernels: int, hidden: int = 256) -> dict:
    lay = surrogate_layout(lib, n_kernels)
    f = np.asarray(blob, np.uint8)[: (16 + 3 * lay["np"]) * 4].view(np.float32)
    out = {"mu": float(f[0]), "sigma": float(f[1])}
    shapes = {"W2": (hidden, hidden), "W1": (hidden, 4), "b1": (hidden,), "b2": (hidden,),
              "w3": (hidden,), "b3": (), "emb": (n_kernels,)}
    for tag in ("P", "M", "V"):
        base = f[lay[tag]: lay[tag] + lay["np"]]
        d = {}
        for k, shp in shapes.items():
            size = int(np.prod(shp)) if shp else 1
            d[k] = base[lay[k]: lay[k] + size].reshape(shp).astype(np.float64)
        out[tag] = d
    return out


def grads_to_dict(lib, g: np.ndarray, n_kernels: int, hidden: int = 256) -> dict:
    lay = surrogate_layout(lib, n_kernels)
    shapes = {"W2": (hidden, hidden), "W1": (hidden, 4), "b1": (hidden,), "b2": (hidden,),
              "w3": (hidden,), "b3": (), "emb": (n_kernels,)}
    out = {}
    for k, shp in shapes.items():
        size = int(np.prod(shp)) if shp else 1
        out[k] = np.asarray(g[lay[k]: lay[k] + size], np.float64).reshape(shp)
    return out


def abi_layout(lib) -> list:
    buf = (ctypes.c_int64 * 32)()
    n = lib.klr_abi_layout(buf, 32)
    return [int(buf[i]) for i in range(n)]


def expected_layout() -> list:
    return [FIT_DESC.itemsize, FIT_INFO.itemsize, HW.itemsize, PROGRAM.itemsize,
            FIT_DESC.fields["coef0"][1], FIT_DESC.fields["m"][1], FIT_DESC.fields["scale_exp"][1],
            FIT_INFO.fields["resid_norm"][1], HW.fields["mem_lat"][1], PROGRAM.fields["fit0"][1],
            PROGRAM.fields["grid_kind"][1]]


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _torch():
    import torch
    return torch


def to_device(arr: np.ndarray, device="cuda"):
    """Upload a numpy array (structured arrays as raw bytes) to a torch device tensor."""
    torch = _torch()
    a = np.ascontiguousarray(arr)
    if a.dtype.fields is not None or a.dtype == np.uint8:
        t = torch.from_numpy(a.view(np.uint8).reshape(-1).copy())
    else:
        t = torch.from_numpy(a.reshape(-1).copy())
    return t.to(device)


def hw_struct(hw) -> np.ndarray:
    h = np.zeros(1, HW)
    for k in ("n_cu", "wave", "w_max", "b_max", "r_max", "z_max", "t_max"):
        h[k] = getattr(hw, k)
    h["mem_lat"], h["dep_delay"] = hw.mem_lat, hw.dep_delay
    h["issue_cycles"], h["bw"] = hw.issue_cycles, hw.bw
    return h


def fit_descs(fb) -> np.ndarray:
    d = np.zeros(fb.n_fits, FIT_DESC)
    d["x0"], d["f0"], d["coef0"] = fb.x0, fb.f0, fb.coef0
    d["m"], d["v"] = fb.m, fb.v
    d["num0"], d["n_num"], d["den0"], d["n_den"] = fb.num0, fb.n_num, fb.den0, fb.n_den
    d["scale_exp"] = fb.scale_exp
    return d


def program_descs(pb, with_costs: bool = False) -> np.ndarray:
    d = np.zeros(pb.n_progs, PROGRAM)
    d["cfg0"], d["q0"] = pb.cfg0, pb.q0
    d["fit0"], d["v_launch"], d["n_cfg"], d["n_q"] = pb.fit0, pb.v_launch, pb.n_cfg, pb.n_q
    d["grid_kind"] = pb.grid_kind
    if getattr(pb, "cost_kind", None) is not None:
        d["cost_kind"] = pb.cost_kind
    if with_costs:
        sizes = pb.n_cfg.astype(np.int64) * pb.n_q
        d["cost0"][1:] = np.cumsum(sizes)[:-1]
    return d


def eval_fit_descs(pb) -> np.ndarray:
    """Fit descriptors of a ProgramBatch (coefficient holders: no samples)."""
    n = pb.num0.shape[0]
    d = np.zeros(n, FIT_DESC)
    d["coef0"], d["m"] = pb.coef0, 0
    # each program's eight fits take its variable count (fits no program refers to keep v = 0;
    # a program whose fit range lies outside the batch is left to the device check, which
    # reports it as a bad descriptor)
    fit0 = np.asarray(pb.fit0, np.int64)
    ck = getattr(pb, "cost_kind", None)
    ck_a = np.asarray(ck) if ck is not None else np.zeros(fit0.shape, np.int32)
    nmet = np.where(ck_a == 1, 1, np.where(ck_a == 2, 3, N_METRICS))
    for k in (1, 3, N_METRICS):
        sel = (nmet == k) & (fit0 >= 0) & (fit0 + k <= n)
        fit_idx = (fit0[sel][:, None] + np.arange(k)).reshape(-1)
        d["v"][fit_idx] = np.repeat(1 + np.asarray(pb.v_launch)[sel], k)
    d["num0"], d["n_num"], d["den0"], d["n_den"] = pb.num0, pb.n_num, pb.den0, pb.n_den
    d["scale_exp"] = pb.scale_exp
    return d


@dataclass
class DeviceEval:
    """Device-resident inputs of klr_eval_argmin for one ProgramBatch."""
    progs: object
    n_progs: int
    max_cfg: int
    max_q: int
    desc: object
    n_fits: int
    exps: object
    n_exp_rows: int
    coef: object
    cfgs: object
    queries: object
    hw: np.ndarray
    costs_len: int
    ws: object
    sws: object = None

    @classmethod
    def from_batch(cls, lib: "Library", pb, with_costs: bool = False, device="cuda", coef=None):
        torch = _torch()
        pd = program_descs(pb, with_costs)
        costs_len = int((pb.n_cfg.astype(np.int64) * pb.n_q).sum()) if with_costs else 0
        max_cfg, max_q = int(pb.n_cfg.max()), int(pb.n_q.max())
        ws_bytes = lib.eval_workspace(pb.n_progs, max_cfg)
        c = pb.coef if coef is None else coef
        coef_t = c if hasattr(c, "data_ptr") else to_device(np.asarray(c, np.float64), device)
        return cls(progs=to_device(pd, device), n_progs=pb.n_progs, max_cfg=max_cfg, max_q=max_q,
                   desc=to_device(eval_fit_descs(pb), device), n_fits=int(pb.num0.shape[0]),
                   exps=to_device(pb.exps.astype(np.uint8), device), n_exp_rows=int(pb.exps.shape[0]),
                   coef=coef_t, cfgs=to_device(pb.cfgs.astype(np.int32), device),
                   queries=to_device(pb.queries.astype(np.int32), device), hw=hw_struct(pb.hw),
                   costs_len=costs_len,
                   ws=torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=device))


class Library:
    _inst = None

    def __init__(self, path: str = LIB_PATH):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the klr product path runs only on the HIP device")
        self.lib = load_library(path)
        self.device = torch.cuda.current_device()
        h = ctypes.c_void_p()
        st = self.lib.klr_create(ctypes.byref(h), self.device)
        if st != KLR_OK:
            raise KlrError(st, "klr_create failed")
        self.h = h

    @classmethod
    def get(cls) -> "Library":
        if cls._inst is None:
            cls._inst = cls()
        return cls._inst

    def _check(self, st: int):
        if st != KLR_OK:
            raise KlrError(st, self.lib.klr_last_error(self.h).decode())

    @staticmethod
    def _stream(stream=None) -> int:
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream()
        return s.cuda_stream

    # ---- graph capture --------------------------------------------------------------------
    def capture_begin(self, stream):
        self._check(self.lib.klr_capture_begin(self.h, stream.cuda_stream))

    def capture_end(self, stream):
        g = ctypes.c_void_p()
        self._check(self.lib.klr_capture_end(self.h, stream.cuda_stream, ctypes.byref(g)))
        return g

    def graph_launch(self, g, stream):
        self._check(self.lib.klr_graph_launch(self.h, g, stream.cuda_stream))

    def graph_destroy(self, g):
        self.lib.klr_graph_destroy(g)

    def set_option(self, option: int, value: int):
        self._check(self.lib.klr_set_option(self.h, option, int(value)))

    # ---- kernel timing ------------------------------------------------------------------
    def profile_enable(self, on: bool = True):
        self._check(self.lib.klr_profile_enable(self.h, 1 if on else 0))

    def profile_read(self, kind: int):
        """(summed milliseconds, launches) of one kernel kind since profile_enable."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(self.lib.klr_profile_read(self.h, kind, ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)

    # ---- eval ---------------------------------------------------------------------------
    def eval_workspace(self, n_progs: int, max_cfg: int) -> int:
        return int(self.lib.klr_eval_workspace(n_progs, max_cfg))

    def eval_argmin(self, de: DeviceEval, want_costs: bool = False, out=None, stream=None,
                    want_status: bool = True):
        """Returns (argmin int32, best_cost float32, all_costs float32 | None, status | None)."""
        torch = _torch()
        ql = int(de.queries.numel())
        if out is None:
            am = torch.empty(ql, dtype=torch.int32, device=de.queries.device)
            bc = torch.empty(ql, dtype=torch.float32, device=de.queries.device)
            costs = torch.empty(de.costs_len, dtype=torch.float32, device=de.queries.device) \
                if want_costs else None
            status = torch.empty(de.n_progs, dtype=torch.int32, device=de.queries.device) \
                if want_status else None
        else:
            am, bc, costs, status = out
        st = self.lib.klr_eval_argmin(
            self.h, _ptr(de.progs), de.n_progs, de.max_cfg, de.max_q, de.hw.ctypes.data,
            _ptr(de.desc), de.n_fits, _ptr(de.exps), de.n_exp_rows, _ptr(de.coef),
            int(de.coef.numel()), _ptr(de.cfgs), int(de.cfgs.numel()), _ptr(de.queries), ql,
            _ptr(am), _ptr(bc), _ptr(costs), int(costs.numel()) if costs is not None else 0,
            _ptr(status), _ptr(de.ws), int(de.ws.numel()), self._stream(stream))
        self._check(st)
        return am, bc, costs, status

    # ---- surrogate ----------------------------------------------------------------------
    def surrogate_alloc(self, params: dict, n_kernels: int, mu=0.0, sigma=1.0, device="cuda"):
        """Device parameter blob (256-byte aligned torch uint8 tensor) from host parameters."""
        torch = _torch()
        blob = pack_params(self.lib, params, n_kernels, mu, sigma)
        t = torch.empty(blob.size + 256, dtype=torch.uint8, device=device)
        off = (-t.data_ptr()) % 256
        v = t[off: off + blob.size]
        v.copy_(torch.from_numpy(blob))
        v._klr_base = t        # keep the allocation alive
        self._check(self.lib.klr_surrogate_init(self.h, _ptr(v), n_kernels, self._stream(None)))
        return v

    def surrogate_params(self, blob_t, n_kernels: int) -> dict:
        return unpack_params(self.lib, blob_t.cpu().numpy(), n_kernels)

    def _aligned(self, nbytes: int, device="cuda"):
        torch = _torch()
        t = torch.empty(max(nbytes, 1) + 256, dtype=torch.uint8, device=device)
        off = (-t.data_ptr()) % 256
        v = t[off: off + max(nbytes, 1)]
        v._klr_base = t
        return v

    def surrogate_train(self, blob_t, n_kernels: int, kid, N, L, cost, lr=1e-3, beta1=0.9,
                        beta2=0.999, eps=1e-8, batch=4096, epochs=1, seed=0, stream=None):
        """Returns the per-epoch mean loss (device float32 tensor)."""
        torch = _torch()
        cfg = np.zeros(1, TRAIN_CFG)
        cfg["lr"], cfg["beta1"], cfg["beta2"], cfg["eps"] = lr, beta1, beta2, eps
        cfg["batch"], cfg["epochs"], cfg["seed"] = batch, epochs, seed
        ws = self._aligned(int(self.lib.klr_surrogate_train_workspace(n_kernels, batch)), kid.device)
        loss = torch.zeros(max(epochs, 1), dtype=torch.float32, device=kid.device)
        st = self.lib.klr_surrogate_train(self.h, _ptr(blob_t), n_kernels, _ptr(kid), _ptr(N), _ptr(L),
                                          _ptr(cost), int(kid.numel()), cfg.ctypes.data, _ptr(loss),
                                          _ptr(ws), int(ws.numel()), self._stream(stream))
        self._check(st)
        return loss

    def surrogate_predict(self, blob_t, n_kernels: int, kid, N, L, stream=None):
        torch = _torch()
        pred = torch.empty(int(kid.numel()), dtype=torch.float32, device=kid.device)
        st = self.lib.klr_surrogate_predict(self.h, _ptr(blob_t), n_kernels, _ptr(kid), _ptr(N), _ptr(L),
                                            int(kid.numel()), _ptr(pred), self._stream(stream))
        self._check(st)
        return pred

    def surrogate_step(self, blob_t, n_kernels: int, kid, N, L, t_std, lr=0.0, step=1, beta1=0.9,
                       beta2=0.999, eps=1e-8, stream=None):
        """One step over the first `batch` = len(kid) samples; returns (grads float32[NP], loss)."""
        torch = _torch()
        B = int(kid.numel())
        lay = surrogate_layout(self.lib, n_kernels)
        grads = torch.zeros(lay["np"], dtype=torch.float32, device=kid.device)
        loss = torch.zeros(1, dtype=torch.float32, device=kid.device)
        ws = self._aligned(int(self.lib.klr_surrogate_train_workspace(n_kernels, B)), kid.device)
        st = self.lib.klr_surrogate_step(self.h, _ptr(blob_t), n_kernels, _ptr(kid), _ptr(N), _ptr(L),
                                         _ptr(t_std), B, lr, step, beta1, beta2, eps, _ptr(grads),
                                         _ptr(loss), _ptr(ws), int(ws.numel()), self._stream(stream))
        self._check(st)
        return grads, loss

    def surrogate_eval(self, blob_t, n_kernels: int, de: DeviceEval, margin: float = 0.02, out=None,
                       stream=None, pred_margin=None, prog_status=None):
        """Returns (argmin int32, pred_cost float32, fell_back uint8); pred_margin (float32
        [q_len]) and prog_status (int32 [n_progs]) are optional output tensors."""
        torch = _torch()
        ql = int(de.queries.numel())
        if out is None:
            am = torch.empty(ql, dtype=torch.int32, device=de.queries.device)
            pc = torch.empty(ql, dtype=torch.float32, device=de.queries.device)
            fb = torch.empty(ql, dtype=torch.uint8, device=de.queries.device)
        else:
            am, pc, fb = out
        need = int(self.lib.klr_surrogate_eval_workspace(de.n_progs, de.max_cfg, de.max_q))
        if getattr(de, "sws", None) is None or de.sws.numel() < need:
            de.sws = self._aligned(need, de.queries.device)
        st = self.lib.klr_surrogate_eval(
            self.h, _ptr(blob_t), n_kernels, _ptr(de.progs), de.n_progs, de.max_cfg, de.max_q,
            de.hw.ctypes.data, _ptr(de.desc), de.n_fits, _ptr(de.exps), de.n_exp_rows, _ptr(de.coef),
            int(de.coef.numel()), _ptr(de.cfgs), int(de.cfgs.numel()), _ptr(de.queries), ql, margin,
            _ptr(am), _ptr(pc), _ptr(fb), _ptr(pred_margin), _ptr(prog_status), _ptr(de.sws),
            int(de.sws.numel()), self._stream(stream))
        self._check(st)
        return am, pc, fb

    # ---- data collection ----------------------------------------------------------------
    def target_attributes(self, target: int) -> dict:
        r, z = ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.klr_target_attributes(self.h, target, ctypes.byref(r), ctypes.byref(z)))
        return {"regs": int(r.value), "lds_bytes": int(z.value)}

    def collect_times(self, target: int, samples, reps: int = 5, stream=None) -> np.ndarray:
        """Mean kernel time in microseconds at each (N, bx, by) row of `samples`."""
        torch = _torch()
        smp = np.ascontiguousarray(np.asarray(samples, np.int32).reshape(-1, 3))
        out = np.zeros(smp.shape[0], np.float64)
        if smp.shape[0] == 0:
            return out
        need = int(self.lib.klr_collect_buffer(target, int(smp[:, 0].max())))
        buf = getattr(self, "_collect_buf", None)
        if buf is None or buf.numel() < need:
            buf = torch.zeros(max(need, 1), dtype=torch.uint8, device="cuda")
            self._collect_buf = buf
        self._check(self.lib.klr_collect_times(self.h, target, smp.ctypes.data, smp.shape[0], reps,
                                               out.ctypes.data, _ptr(buf), int(buf.numel()), self._stream(stream)))
        return out

    # ---- fit ----------------------------------------------------------------------------
    def fit_workspace(self, n_fits: int, total_rows: int, precision: int) -> int:
        return int(self.lib.klr_fit_workspace(n_fits, total_rows, precision))

    def fit_batched(self, df: "DeviceFit", precision: int = KLR_FP64, max_iter: int = 32,
                    tol: float = 1e-12, out=None, stream=None):
        """Returns (coef float64, info bytes [n_fits * 32] uint8 tensor)."""
        torch = _torch()
        if out is None:
            coef = torch.empty(max(df.n_coef, 1), dtype=torch.float64, device=df.f.device)
            info = torch.empty(max(df.n_fits, 1) * FIT_INFO.itemsize, dtype=torch.uint8, device=df.f.device)
        else:
            coef, info = out
        wsb = self.fit_workspace(df.n_fits, df.total_rows, precision)
        if df.ws is None or df.ws.numel() < wsb:
            df.ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=df.f.device)
        st = self.lib.klr_fit_batched(
            self.h, _ptr(df.desc), df.n_fits, _ptr(df.exps), df.n_exp_rows, _ptr(df.X),
            int(df.X.numel()), _ptr(df.f), int(df.f.numel()), precision, max_iter, tol,
            _ptr(coef), df.n_coef, _ptr(info), _ptr(df.ws), int(df.ws.numel()), self._stream(stream))
        self._check(st)
        return coef, info


@dataclass
class DeviceFit:
    desc: object
    n_fits: int
    exps: object
    n_exp_rows: int
    X: object
    f: object
    n_coef: int
    total_rows: int = 0          # sum of the fits' sample counts (sizes the private scratch)
    ws: object = None

    @classmethod
    def from_batch(cls, fb, device="cuda"):
        return cls(desc=to_device(fit_descs(fb), device), n_fits=fb.n_fits,
                   exps=to_device(fb.exps.astype(np.uint8), device), n_exp_rows=int(fb.exps.shape[0]),
                   X=to_device(fb.X.astype(np.int32), device), f=to_device(fb.f.astype(np.float64), device),
                   n_coef=int(fb.n_coef), total_rows=int(np.clip(fb.m, 0, None).sum()))


def info_records(info) -> np.ndarray:
    """Info bytes (device tensor or host array) -> numpy structured array of klr_fit_info."""
    arr = info.cpu().numpy() if hasattr(info, "cpu") else np.asarray(info)
    return arr.view(np.uint8).view(FIT_INFO)


def program_samples(pb, de: DeviceEval, costs):
    """Training samples (kernel id = program index, N, launch pair, exact cost) of every
    (program, configuration, query) point of a batch of two-launch-parameter programs with
    uneven configuration and query counts, from its cost array (laid out per program as
    [n_cfg][n_q] at the offsets program_descs assigns); device tensors, index bookkeeping only."""
    torch = _torch()
    if not np.all(pb.v_launch == 2):
        raise ValueError("program_samples needs programs with two launch parameters")
    dev = de.queries.device
    nc = pb.n_cfg.astype(np.int64)
    nq = pb.n_q.astype(np.int64)
    sizes = nc * nq
    total = int(sizes.sum())
    cost0 = np.zeros(pb.n_progs, np.int64)
    cost0[1:] = np.cumsum(sizes)[:-1]
    prog = np.repeat(np.arange(pb.n_progs, dtype=np.int64), sizes)
    local = np.arange(total, dtype=np.int64) - cost0[prog]
    c = local // nq[prog]
    q = local % nq[prog]
    qi = torch.from_numpy(pb.q0.astype(np.int64)[prog] + q).to(dev)
    ci = torch.from_numpy(pb.cfg0.astype(np.int64)[prog] + 2 * c).to(dev)
    kid = torch.from_numpy(prog.astype(np.int32)).to(dev)
    N = de.queries[qi]
    L = torch.stack([de.cfgs[ci], de.cfgs[ci + 1]], dim=1).reshape(-1)
    return kid.contiguous(), N.contiguous(), L.contiguous(), costs[:total].contiguous()


def grid_samples(pb, de: DeviceEval, costs):
    """Training samples (kernel id, N, launch pair, exact cost) of a uniform ProgramBatch from
    its full cost matrix: every (program, query, configuration) point, as device tensors
    (index bookkeeping only)."""
    torch = _torch()
    P, C, Q = pb.n_progs, int(pb.n_cfg[0]), int(pb.n_q[0])
    if not (np.all(pb.n_cfg == C) and np.all(pb.n_q == Q) and np.all(pb.v_launch == 2)
            and np.all(pb.cfg0 == pb.cfg0[0])):
        raise ValueError("grid_samples needs programs of one shape sharing one configuration list")
    dev = de.queries.device
    kid = torch.arange(P, dtype=torch.int32, device=dev).view(P, 1, 1).expand(P, C, Q).reshape(-1)
    N = de.queries.view(P, 1, Q).expand(P, C, Q).reshape(-1)
    c0 = int(pb.cfg0[0])
    L = de.cfgs[c0: c0 + 2 * C].view(1, C, 1, 2).expand(P, C, Q, 2).reshape(-1)
    return kid.contiguous(), N.contiguous(), L.contiguous(), costs[: P * C * Q].contiguous()


class Service:
    """Launch-time decision service over the programs of a DeviceEval (klr_service_*): decisions
    for data sizes with a history, optional Python-syntax constraints per program."""

    def __init__(self, lib: "Library", de: DeviceEval, pb, max_batch: int = 1024):
        torch = _torch()
        self.lib, self.L = lib, lib.lib
        self.progs_host = program_descs(pb)
        self.cfgs_host = np.ascontiguousarray(pb.cfgs.astype(np.int32))
        max_cfg = int(max(1, pb.n_cfg.max()))
        self.ws = lib._aligned(int(self.L.klr_service_workspace(max_cfg, max_batch)), de.queries.device)
        self.de = de                                   # keeps the device arrays alive
        s = ctypes.c_void_p()
        st = self.L.klr_service_create(lib.h, ctypes.byref(s), self.progs_host.ctypes.data, int(pb.n_progs),
                                       de.hw.ctypes.data, _ptr(de.desc), de.n_fits, _ptr(de.exps), de.n_exp_rows,
                                       _ptr(de.coef), int(de.coef.numel()), self.cfgs_host.ctypes.data,
                                       _ptr(de.cfgs), int(self.cfgs_host.size), max_batch, _ptr(self.ws),
                                       int(self.ws.numel()))
        lib._check(st)
        self.s = s
        del torch

    def close(self):
        if self.s:
            self.L.klr_service_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_constraint(self, prog: int, expr: str):
        self.lib._check(self.L.klr_service_add_constraint(self.s, int(prog), expr.encode()))

    def decide(self, prog: int, N, stream=None) -> np.ndarray:
        Nh = np.ascontiguousarray(np.asarray(N, np.int32))
        out = np.zeros(Nh.size, LAUNCH)
        self.lib._check(self.L.klr_service_decide(self.s, int(prog), Nh.ctypes.data if Nh.size else None,
                                                  int(Nh.size), out.ctypes.data if Nh.size else None,
                                                  self.lib._stream(stream)))
        return out

    def stats(self) -> dict:
        v = [ctypes.c_int64() for _ in range(4)]
        self.lib._check(self.L.klr_service_stats(self.s, *[ctypes.byref(x) for x in v]))
        return dict(zip(("hits", "misses", "evaluations", "entries"), (int(x.value) for x in v)))

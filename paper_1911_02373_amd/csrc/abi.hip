// C ABI entry points of libklr: argument validation on the host, workspace sizing, dispatch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "internal.hpp"

namespace klr {

klr_status fail(klr_handle h, klr_status st, const std::string& msg) {
  if (h) h->err = msg;
  return st;
}

klr_status hip_check(klr_handle h, hipError_t e, const char* what) {
  if (e == hipSuccess) return KLR_OK;
  return fail(h, KLR_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

hipEvent_t Timer::get() {
  if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int Timer::begin(int kind, hipStream_t s) {
  if (!on) return -1;
  Rec r{kind, get(), get()};
  if (!r.a || !r.b) return -1;
  hipEventRecord(r.a, s);
  pending.push_back(r);
  return (int)pending.size() - 1;
}

void Timer::end(int idx, hipStream_t s) {
  if (idx >= 0) hipEventRecord(pending[idx].b, s);
}

hipError_t Timer::drain() {
  hipError_t err = hipSuccess;
  for (auto& r : pending) {
    hipError_t e = hipEventSynchronize(r.b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e == hipSuccess) { total_ms[r.kind] += ms; count[r.kind] += 1; } else { err = e; }
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  pending.clear();
  return err;
}

void Timer::reset() {
  drain();
  for (int k = 0; k < KLR_K_COUNT; ++k) { total_ms[k] = 0.0; count[k] = 0; }
}

Timer::~Timer() {
  for (auto& r : pending) { pool.push_back(r.a); pool.push_back(r.b); }
  for (hipEvent_t e : pool) hipEventDestroy(e);
}

namespace {

bool hw_ok(const klr_hw& hw, std::string& why) {
  if (hw.wave != 32 && hw.wave != 64) { why = "hw.wave must be 32 or 64"; return false; }
  if (hw.n_cu < 1 || hw.n_cu > 65536) { why = "hw.n_cu out of [1, 65536]"; return false; }
  if (hw.w_max < 1 || hw.w_max > 1024) { why = "hw.w_max out of [1, 1024]"; return false; }
  if (hw.b_max < 1 || hw.b_max > 1024) { why = "hw.b_max out of [1, 1024]"; return false; }
  if (hw.r_max < 1 || hw.z_max < 0) { why = "hw.r_max must be >= 1 and hw.z_max >= 0"; return false; }
  if (hw.t_max < hw.wave || hw.t_max > 65536) { why = "hw.t_max out of [wave, 65536]"; return false; }
  if (hw.reserved != 0) { why = "hw.reserved must be 0"; return false; }
  const float fl[4] = {hw.mem_lat, hw.dep_delay, hw.issue_cycles, hw.bw};
  for (float x : fl)
    if (!(x > 0.0f) || !std::isfinite(x)) { why = "hw float parameters must be finite and > 0"; return false; }
  return true;
}

}  // namespace
}  // namespace klr

using klr::fail;

extern "C" {

klr_status klr_create(klr_handle* out, int device) {
  if (!out) return KLR_E_INVALID;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return KLR_E_INVALID;
  if (hipSetDevice(device) != hipSuccess) return KLR_E_HIP;
  klr_handle h = new (std::nothrow) klr_handle_s;
  if (!h) return KLR_E_HIP;
  h->device = device;
  *out = h;
  return KLR_OK;
}

void klr_destroy(klr_handle h) { delete h; }

const char* klr_last_error(klr_handle h) { return h ? h->err.c_str() : "null handle"; }

klr_status klr_profile_enable(klr_handle h, int32_t on) {
  if (!h) return KLR_E_INVALID;
  h->timer.reset();
  h->timer.on = on != 0;
  return KLR_OK;
}

klr_status klr_profile_read(klr_handle h, int32_t kind, double* total_ms, int64_t* launches) {
  if (!h || kind < 0 || kind >= KLR_K_COUNT || !total_ms || !launches) return KLR_E_INVALID;
  klr_status st = klr::hip_check(h, h->timer.drain(), "klr_profile_read");
  *total_ms = h->timer.total_ms[kind];
  *launches = h->timer.count[kind];
  return st;
}

int32_t klr_abi_layout(int64_t* out, int32_t n) {
  const int64_t v[] = {
      (int64_t)sizeof(klr_fit_desc), (int64_t)sizeof(klr_fit_info), (int64_t)sizeof(klr_hw),
      (int64_t)sizeof(klr_program),
      (int64_t)offsetof(klr_fit_desc, coef0), (int64_t)offsetof(klr_fit_desc, m),
      (int64_t)offsetof(klr_fit_desc, scale_exp), (int64_t)offsetof(klr_fit_info, resid_norm),
      (int64_t)offsetof(klr_hw, mem_lat), (int64_t)offsetof(klr_program, fit0),
      (int64_t)offsetof(klr_program, grid_kind),
  };
  const int32_t cnt = (int32_t)(sizeof(v) / sizeof(v[0]));
  for (int32_t i = 0; i < n && i < cnt; ++i) out[i] = v[i];
  return cnt;
}

size_t klr_eval_workspace(int32_t n_progs, int32_t max_cfg) {
  return klr::eval_workspace_bytes(n_progs, max_cfg);
}

klr_status klr_eval_argmin(klr_handle h, const klr_program* progs, int32_t n_progs,
                           int32_t max_cfg, int32_t max_q, const klr_hw* hw,
                           const klr_fit_desc* desc, int32_t n_fits,
                           const uint8_t* exps, int32_t n_exp_rows,
                           const double* coef, int64_t coef_len,
                           const int32_t* cfgs, int64_t cfgs_len,
                           const int32_t* queries, int64_t q_len,
                           int32_t* argmin, float* best_cost,
                           float* all_costs, int64_t costs_len, int32_t* prog_status,
                           void* ws, size_t ws_bytes, void* stream) {
  if (!h) return KLR_E_INVALID;
  h->err.clear();
  if (!hw) return fail(h, KLR_E_INVALID, "hw is NULL");
  std::string why;
  if (!klr::hw_ok(*hw, why)) return fail(h, KLR_E_INVALID, why);
  if (n_progs < 0 || max_cfg < 0 || max_q < 0 || n_fits < 0 || n_exp_rows < 0 || coef_len < 0 ||
      cfgs_len < 0 || q_len < 0 || costs_len < 0)
    return fail(h, KLR_E_INVALID, "negative size");
  if (n_progs == 0) return KLR_OK;
  if (max_cfg > 65536) return fail(h, KLR_E_UNSUPPORTED, "max_cfg above 65536");
  if (!progs || !desc || !exps || !coef || !cfgs || (q_len > 0 && (!queries || !argmin || !best_cost)))
    return fail(h, KLR_E_INVALID, "NULL array argument");
  if (max_q > 0 && (!queries || !argmin || !best_cost))
    return fail(h, KLR_E_INVALID, "NULL query or output array");
  const size_t need = klr::eval_workspace_bytes(n_progs, max_cfg);
  if (need > 0 && (!ws || ws_bytes < need))
    return fail(h, KLR_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(h, KLR_E_INVALID, "workspace must be 256-byte aligned");
  // one work-item per (program, configuration) and per (program, query): 32-bit grid limit
  const int64_t items_c = (int64_t)n_progs * (((int64_t)max_cfg + 127) / 128) * 128;
  const int64_t items_q = (int64_t)n_progs * (((int64_t)max_q + 255) / 256) * 256;
  if (items_c >= (int64_t(1) << 32) || items_q >= (int64_t(1) << 32))
    return fail(h, KLR_E_UNSUPPORTED, "launch grid above 2^32 work-items; split the batch");
  klr::EvalArgs a{progs, n_progs, max_cfg, max_q, *hw, desc, n_fits, exps, n_exp_rows, coef, coef_len,
                  cfgs, cfgs_len, queries, q_len, argmin, best_cost, all_costs,
                  all_costs ? costs_len : 0, prog_status, ws, ws_bytes,
                  reinterpret_cast<hipStream_t>(stream), &h->timer};
  return klr::hip_check(h, klr::launch_eval(a), "klr_eval_argmin launch");
}

size_t klr_fit_workspace(int32_t n_fits, int64_t f_len, int32_t precision) {
  return klr::fit_workspace_bytes(n_fits, f_len, precision);
}

klr_status klr_fit_batched(klr_handle h, const klr_fit_desc* desc, int32_t n_fits,
                           const uint8_t* exps, int32_t n_exp_rows,
                           const int32_t* X, int64_t x_len, const double* f, int64_t f_len,
                           int32_t precision, int32_t max_iter, double tol,
                           double* coef, int64_t coef_len, klr_fit_info* info,
                           void* ws, size_t ws_bytes, void* stream) {
  if (!h) return KLR_E_INVALID;
  h->err.clear();
  if (n_fits < 0 || n_exp_rows < 0 || x_len < 0 || f_len < 0 || coef_len < 0)
    return fail(h, KLR_E_INVALID, "negative size");
  if (precision != KLR_FP64 && precision != KLR_FP32_REFINED && precision != KLR_BF16_REFINED)
    return fail(h, KLR_E_INVALID, "unknown precision");
  if (max_iter < 0 || max_iter > 10000 || !(tol >= 0.0) || !std::isfinite(tol))
    return fail(h, KLR_E_INVALID, "max_iter must be in [0, 10000] and tol finite >= 0");
  if (n_fits == 0) return KLR_OK;
  if (!desc || !exps || !coef || !info || (x_len > 0 && !X) || (f_len > 0 && !f))
    return fail(h, KLR_E_INVALID, "NULL array argument");
  const size_t need = klr::fit_workspace_bytes(n_fits, f_len, precision);
  if (need > 0 && (!ws || ws_bytes < need))
    return fail(h, KLR_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(h, KLR_E_INVALID, "workspace must be 256-byte aligned");
  klr::FitArgs a{desc, n_fits, exps, n_exp_rows, X, x_len, f, f_len, precision, max_iter, tol,
                 coef, coef_len, info, ws, ws_bytes, reinterpret_cast<hipStream_t>(stream), &h->timer};
  return klr::hip_check(h, klr::launch_fit(a), "klr_fit_batched launch");
}

}  // extern "C"

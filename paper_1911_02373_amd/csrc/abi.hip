// C ABI entry points of libklr: argument validation on the host, workspace sizing, dispatch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "internal.hpp"

// Workspace of klr_eval_argmin_noalloc: one copy of this array per GPU, resident from the
// library's load until the process ends.  In host code `scratch` is a host-side stand-in, not
// a device address: each GPU's copy is found with hipGetSymbolAddress while that GPU is current
// (in klr_create), and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[KLR_NOALLOC_SCRATCH_BYTES];

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

void Tuner::record(uint64_t key, int variant, float ms) {
  entries.emplace_back(key, variant);
  if (path.empty()) return;
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%llu %d %.6f\n", (unsigned long long)key, variant, ms);
  std::fclose(f);
}

void Tuner::load() {
  const char* p = std::getenv("KLR_TUNE_CACHE");
  if (!p || !*p) return;
  path = p;
  FILE* f = std::fopen(p, "r");
  if (!f) return;
  unsigned long long k = 0;
  int v = 0;
  float ms = 0.0f;
  while (std::fscanf(f, "%llu %d %f", &k, &v, &ms) == 3) {
    const int nv = (k & kTuneFitTag) ? kFitVariants : eval_num_variants();
    if (v >= 0 && v < nv && find(k) < 0) entries.emplace_back((uint64_t)k, v);
  }
  std::fclose(f);
}

namespace {

// Device address of `scratch` on each GPU (found once per device by klr_create).
constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

void find_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess && p) g_scratch_ptr[device] = p;
  else g_scratch_err[device] = e == hipSuccess ? hipErrorInvalidSymbol : e;
}

uint64_t ceil_log2(int64_t x) {
  int b = 0;
  while ((int64_t(1) << b) < x && b < 40) ++b;
  return (uint64_t)b;
}

uint64_t eval_tune_key(int32_t n_progs, int32_t max_cfg, int32_t max_q) {
  return kTuneEvalTag | (ceil_log2(n_progs) << 32) | (ceil_log2(max_cfg) << 16) | ceil_log2(max_q);
}

// A fit batch's shape: precision, schedule, and the batch size and sample rows per fit in
// powers of two.
uint64_t fit_tune_key(int32_t n_fits, int64_t f_len, int32_t precision, bool persistent) {
  const int64_t per = n_fits > 0 ? f_len / n_fits : 0;
  return kTuneFitTag | ((uint64_t)precision << 48) | ((uint64_t)persistent << 44) | (ceil_log2(n_fits) << 16) |
         ceil_log2(per);
}

bool hw_ok(const klr_hw& hw, std::string& why) {
  if (hw.wave != 32 && hw.wave != 64) { why = "hw.wave must be 32 or 64"; return false; }
  if (hw.n_cu < 1 || hw.n_cu > 65536) { why = "hw.n_cu out of [1, 65536]"; return false; }
  if (hw.w_max < 1 || hw.w_max > 1024) { why = "hw.w_max out of [1, 1024]"; return false; }
  if (hw.b_max < 1 || hw.b_max > 1024) { why = "hw.b_max out of [1, 1024]"; return false; }
  if (hw.r_max < 1 || hw.r_max >= (1 << 20) || hw.z_max < 0 || hw.z_max >= (1 << 20)) {
    why = "hw.r_max must be in [1, 2^20) and hw.z_max in [0, 2^20)";
    return false;
  }
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
  klr::find_scratch(device);     // with `device` current: its copy of the no-allocation workspace
  h->tuner.load();
  *out = h;
  return KLR_OK;
}

void klr_destroy(klr_handle h) { delete h; }

const char* klr_last_error(klr_handle h) { return h ? h->err.c_str() : "null handle"; }

struct klr_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

klr_status klr_capture_begin(klr_handle h, void* stream) {
  if (!h) return KLR_E_INVALID;
  h->err.clear();
  if (!stream) return fail(h, KLR_E_INVALID, "the null stream cannot be captured");
  if (h->capturing) return fail(h, KLR_E_INVALID, "already capturing");
  klr_status st = klr::hip_check(h, hipStreamBeginCapture(reinterpret_cast<hipStream_t>(stream),
                                                          hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
  if (st == KLR_OK) h->capturing = true;
  return st;
}

klr_status klr_capture_end(klr_handle h, void* stream, klr_graph* out) {
  if (!h || !out) return KLR_E_INVALID;
  *out = nullptr;
  if (!h->capturing) return fail(h, KLR_E_INVALID, "not capturing");
  h->capturing = false;
  hipGraph_t g = nullptr;
  klr_status st = klr::hip_check(h, hipStreamEndCapture(reinterpret_cast<hipStream_t>(stream), &g),
                                 "hipStreamEndCapture");
  if (st != KLR_OK) return st;
  hipGraphExec_t ex = nullptr;
  st = klr::hip_check(h, hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "hipGraphInstantiate");
  if (st != KLR_OK) { hipGraphDestroy(g); return st; }
  klr_graph r = new (std::nothrow) klr_graph_s;
  if (!r) { hipGraphExecDestroy(ex); hipGraphDestroy(g); return fail(h, KLR_E_HIP, "out of host memory"); }
  r->graph = g;
  r->exec = ex;
  *out = r;
  return KLR_OK;
}

klr_status klr_graph_launch(klr_handle h, klr_graph g, void* stream) {
  if (!h || !g) return KLR_E_INVALID;
  h->err.clear();
  return klr::hip_check(h, hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(stream)), "hipGraphLaunch");
}

void klr_graph_destroy(klr_graph g) {
  if (!g) return;
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  delete g;
}

klr_status klr_set_option(klr_handle h, int32_t option, int64_t value) {
  if (!h) return KLR_E_INVALID;
  if (option < 0 || option >= KLR_OPT_COUNT) return fail(h, KLR_E_INVALID, "unknown option");
  h->opt[option] = value;
  return KLR_OK;
}

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

int64_t klr_selftest_divisors(uint32_t d_max) { return klr::selftest_divisors(d_max); }

int64_t klr_selftest_divisor_list(const uint64_t* ds, int32_t n_ds) {
  return ds == nullptr || n_ds < 0 ? -1 : klr::selftest_divisor_list(ds, n_ds);
}

int64_t klr_selftest_short_division(int32_t b_first, int32_t b_count) {
  return klr::selftest_short_division(b_first, b_count);
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

}  // extern "C"

namespace klr {
namespace {

// Validation and launch of the evaluation; no_alloc: the workspace is this GPU's `scratch`, the
// launch shape is the cached tuned one (or the default) and no kernel timing is recorded, so
// the call creates no events and allocates nothing.
klr_status eval_argmin_impl(klr_handle h, const klr_program* progs, int32_t n_progs,
                            int32_t max_cfg, int32_t max_q, const klr_hw* hw,
                            const klr_fit_desc* desc, int32_t n_fits,
                            const uint8_t* exps, int32_t n_exp_rows,
                            const double* coef, int64_t coef_len,
                            const int32_t* cfgs, int64_t cfgs_len,
                            const int32_t* queries, int64_t q_len,
                            int32_t* argmin, float* best_cost,
                            float* all_costs, int64_t costs_len, int32_t* prog_status,
                            void* ws, size_t ws_bytes, void* stream, bool no_alloc) {
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
                  reinterpret_cast<hipStream_t>(stream), (h->capturing || no_alloc) ? nullptr : &h->timer,
                  -1, nullptr, 0};
  a.tune_key = klr::eval_tune_key(n_progs, max_cfg, max_q);
  if (h->opt[KLR_OPT_EVAL_VARIANT] >= 0) {
    a.variant = (int)(h->opt[KLR_OPT_EVAL_VARIANT] % klr::eval_num_variants());
  } else {
    a.variant = h->tuner.find(a.tune_key);
    if (a.variant < 0 && !h->capturing && !no_alloc) a.tuner = &h->tuner;
    if (a.variant < 0 && (h->capturing || no_alloc)) a.variant = 0;
  }
  return klr::hip_check(h, klr::launch_eval(a), no_alloc ? "klr_eval_argmin_noalloc launch" : "klr_eval_argmin launch");
}

}  // namespace
}  // namespace klr

extern "C" {

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
  return klr::eval_argmin_impl(h, progs, n_progs, max_cfg, max_q, hw, desc, n_fits, exps, n_exp_rows, coef,
                               coef_len, cfgs, cfgs_len, queries, q_len, argmin, best_cost, all_costs,
                               costs_len, prog_status, ws, ws_bytes, stream, false);
}

klr_status klr_eval_argmin_noalloc(klr_handle h, const klr_program* progs, int32_t n_progs,
                                   int32_t max_cfg, int32_t max_q, const klr_hw* hw,
                                   const klr_fit_desc* desc, int32_t n_fits,
                                   const uint8_t* exps, int32_t n_exp_rows,
                                   const double* coef, int64_t coef_len,
                                   const int32_t* cfgs, int64_t cfgs_len,
                                   const int32_t* queries, int64_t q_len,
                                   int32_t* argmin, float* best_cost,
                                   float* all_costs, int64_t costs_len, int32_t* prog_status,
                                   void* stream) {
  if (!h) return KLR_E_INVALID;
  h->err.clear();
  if (n_progs < 0 || max_cfg < 0) return fail(h, KLR_E_INVALID, "negative size");
  const size_t need = klr::eval_workspace_bytes(n_progs, max_cfg);
  if (need > (size_t)KLR_NOALLOC_SCRATCH_BYTES)
    return fail(h, KLR_E_WORKSPACE, "klr_eval_argmin_noalloc: the batch needs " + std::to_string(need) +
                                    " bytes of workspace, above the fixed " +
                                    std::to_string((size_t)KLR_NOALLOC_SCRATCH_BYTES) +
                                    " (KLR_NOALLOC_SCRATCH_BYTES); split the batch");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != h->device)
    return fail(h, KLR_E_INVALID, "klr_eval_argmin_noalloc: the handle's device must be current");
  void* ws = nullptr;
  if (dev >= 0 && dev < klr::kMaxDevices) {
    std::lock_guard<std::mutex> lk(klr::g_scratch_mu);
    ws = klr::g_scratch_ptr[dev];
    if (!ws)
      return fail(h, KLR_E_HIP, std::string("klr_eval_argmin_noalloc: no device address for the fixed workspace: ") +
                                    hipGetErrorString(klr::g_scratch_err[dev]));
  } else {
    return fail(h, KLR_E_UNSUPPORTED, "klr_eval_argmin_noalloc: device index above the supported range");
  }
  return klr::eval_argmin_impl(h, progs, n_progs, max_cfg, max_q, hw, desc, n_fits, exps, n_exp_rows, coef,
                               coef_len, cfgs, cfgs_len, queries, q_len, argmin, best_cost, all_costs,
                               costs_len, prog_status, ws, (size_t)KLR_NOALLOC_SCRATCH_BYTES, stream, true);
}

size_t klr_fit_workspace(int32_t n_fits, int64_t total_rows, int32_t precision) {
  return klr::fit_workspace_bytes(n_fits, total_rows, precision);
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
  if (precision != KLR_FP64 && precision != KLR_FP32_REFINED && precision != KLR_BF16_REFINED &&
      precision != KLR_FP64_SVD)
    return fail(h, KLR_E_INVALID, "unknown precision");
  if (max_iter < 0 || max_iter > 10000 || !(tol >= 0.0) || !std::isfinite(tol))
    return fail(h, KLR_E_INVALID, "max_iter must be in [0, 10000] and tol finite >= 0");
  if (n_fits == 0) return KLR_OK;
  if (!desc || !exps || !coef || !info || (x_len > 0 && !X) || (f_len > 0 && !f))
    return fail(h, KLR_E_INVALID, "NULL array argument");
  // the fixed part (schedule and scratch offsets); the scratch rows the fits need are only known
  // on the device, so a shortfall there is reported per fit (KLR_FIT_NO_SCRATCH)
  const size_t need = klr::fit_workspace_bytes(n_fits, 0, precision);
  if (need > 0 && (!ws || ws_bytes < need))
    return fail(h, KLR_E_WORKSPACE, "workspace too small: need at least " + std::to_string(need) + " bytes");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(h, KLR_E_INVALID, "workspace must be 256-byte aligned");
  klr::FitArgs a{desc, n_fits, exps, n_exp_rows, X, x_len, f, f_len, precision, max_iter, tol,
                 coef, coef_len, info, ws, ws_bytes, reinterpret_cast<hipStream_t>(stream),
                 h->capturing ? nullptr : &h->timer, h->opt[KLR_OPT_FIT_PERSISTENT] != 0,
                 nullptr, nullptr, 0};
  klr::fit_workspace_split(a);
  a.tune_key = klr::fit_tune_key(n_fits, f_len, precision, a.persistent);
  if (h->opt[KLR_OPT_FIT_VARIANT] >= 0) {
    a.variant = (int)(h->opt[KLR_OPT_FIT_VARIANT] % klr::kFitVariants);
  } else {
    a.variant = h->tuner.find(a.tune_key);
    if (a.variant < 0 && !h->capturing) a.tuner = &h->tuner;
    if (a.variant < 0 && h->capturing) a.variant = 0;
  }
  return klr::hip_check(h, klr::launch_fit(a), "klr_fit_batched launch");
}

size_t klr_surrogate_param_bytes(int32_t n_kernels) {
  return n_kernels < 0 ? 0 : klr::mlp_param_bytes(n_kernels);
}

klr_status klr_surrogate_init(klr_handle h, void* params, int32_t n_kernels, void* stream) {
  if (!h) return KLR_E_INVALID;
  h->err.clear();
  if (!params || n_kernels < 1) return fail(h, KLR_E_INVALID, "bad arguments");
  if (reinterpret_cast<uintptr_t>(params) % 256 != 0) return fail(h, KLR_E_INVALID, "params must be 256-byte aligned");
  return klr::hip_check(h, klr::launch_refresh(klr::blob_of(params, n_kernels), reinterpret_cast<hipStream_t>(stream)),
                        "klr_surrogate_init");
}

int32_t klr_surrogate_layout(int32_t n_kernels, int64_t* out, int32_t n) {
  const int64_t np = klr::mlp_np(n_kernels);
  const int64_t v[] = {np, 16, 16 + np, 16 + 2 * np, (16 + 3 * np) * 4,
                       (16 + 3 * np) * 4 + 2 * KLR_MLP_HIDDEN * KLR_MLP_HIDDEN,
                       (int64_t)klr::mlp_param_bytes(n_kernels), klr::kO_W2, klr::kO_W1, klr::kO_B1,
                       klr::kO_B2, klr::kO_W3, klr::kO_B3, klr::kO_EMB};
  const int32_t cnt = (int32_t)(sizeof(v) / sizeof(v[0]));
  for (int32_t i = 0; i < n && i < cnt; ++i) out[i] = v[i];
  return cnt;
}

size_t klr_surrogate_train_workspace(int32_t n_kernels, int32_t batch) {
  if (n_kernels < 0 || batch <= 0) return 0;
  return klr::mlp_train_ws_bytes(n_kernels, batch);
}

}  // extern "C"

namespace klr {

size_t mlp_train_ws_bytes(int32_t nk, int32_t B) {
  const size_t t = (size_t)KLR_MLP_HIDDEN * B * sizeof(uint16_t);
  const size_t part = (size_t)(B / 64) * kPartialStride * sizeof(float);
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t dw2 = (size_t)kDw2Slices * KLR_MLP_HIDDEN * KLR_MLP_HIDDEN * sizeof(float);
  return 2 * al(t) + al(part) + al((size_t)nk * 8) + al(dw2) + 256;
}

namespace {

TrainTile tile_args(void* ws, int32_t nk, int32_t B) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  char* c = reinterpret_cast<char*>(ws);
  const size_t t = (size_t)KLR_MLP_HIDDEN * B * sizeof(uint16_t);
  TrainTile tt{};
  tt.H1T = reinterpret_cast<uint16_t*>(c);
  tt.dH2T = reinterpret_cast<uint16_t*>(c + al(t));
  tt.partial = reinterpret_cast<float*>(c + 2 * al(t));
  const size_t emb_off = 2 * al(t) + al((size_t)(B / 64) * kPartialStride * 4);
  tt.emb_acc = reinterpret_cast<unsigned long long*>(c + emb_off);
  const size_t dw2_off = emb_off + al((size_t)nk * 8);
  tt.dw2_part = reinterpret_cast<float*>(c + dw2_off);
  tt.B = B;
  tt.nk = nk;
  return tt;
}

float* loss_slot(void* ws, int32_t nk, int32_t B) {
  return reinterpret_cast<float*>(reinterpret_cast<char*>(ws) + mlp_train_ws_bytes(nk, B) - 256);
}

AdamArgs adam_args(float lr, float b1, float b2, float eps, int64_t step) {
  AdamArgs a{lr, b1, b2, eps, (float)(1.0 - std::pow((double)b1, (double)step)),
             (float)(1.0 - std::pow((double)b2, (double)step))};
  return a;
}

bool batch_ok(int32_t B) { return B >= 128 && B <= 65536 && B % 128 == 0; }

}  // namespace
}  // namespace klr

extern "C" {

klr_status klr_surrogate_train(klr_handle h, void* params, int32_t n_kernels,
                               const int32_t* kernel_id, const int32_t* N, const int32_t* launch,
                               const float* cost, int64_t n, const klr_train_cfg* cfg,
                               float* loss_per_epoch, void* ws, size_t ws_bytes, void* stream) {
  if (!h) return KLR_E_INVALID;
  h->err.clear();
  if (!cfg || !params || n_kernels < 1 || n < 0) return fail(h, KLR_E_INVALID, "bad arguments");
  if (!klr::batch_ok(cfg->batch)) return fail(h, KLR_E_INVALID, "batch must be a multiple of 128 in [128, 65536]");
  if (cfg->epochs < 0 || !(cfg->lr >= 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) ||
      !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) || !(cfg->eps > 0.0f))
    return fail(h, KLR_E_INVALID, "bad optimiser settings");
  if (n > 0 && (!kernel_id || !N || !launch || !cost)) return fail(h, KLR_E_INVALID, "NULL sample array");
  if (cfg->epochs > 0 && !loss_per_epoch) return fail(h, KLR_E_INVALID, "loss_per_epoch is NULL");
  const size_t need = klr::mlp_train_ws_bytes(n_kernels, cfg->batch);
  if (!ws || ws_bytes < need) return fail(h, KLR_E_WORKSPACE, "workspace too small: need " + std::to_string(need));
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0 || reinterpret_cast<uintptr_t>(params) % 256 != 0)
    return fail(h, KLR_E_INVALID, "params and workspace must be 256-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  klr::Blob w = klr::blob_of(params, n_kernels);
  klr::TrainTile t = klr::tile_args(ws, n_kernels, cfg->batch);
  t.kid = kernel_id; t.N = N; t.L = launch; t.cost = cost; t.tstd = nullptr; t.n = n;
  int bits = 1;
  while (bits < 62 && (int64_t(1) << bits) < n) ++bits;
  t.perm_bits = bits;
  const int64_t nb = n / cfg->batch;
  const int64_t total = nb * cfg->epochs;
  const int tm = h->timer.begin(KLR_K_MLP, s);
  hipError_t e = klr::launch_stats(cost, n, w.hdr, s);
  if (e == hipSuccess) e = klr::launch_refresh(w, s);
  if (e == hipSuccess) e = hipMemsetAsync(t.emb_acc, 0, (size_t)n_kernels * 8, s);
  if (e == hipSuccess && cfg->epochs > 0) e = hipMemsetAsync(loss_per_epoch, 0, (size_t)cfg->epochs * 4, s);
  int64_t step = 0;
  for (int ep = 0; ep < cfg->epochs && e == hipSuccess; ++ep) {
    uint64_t z = cfg->seed * 0x9E3779B97F4A7C15ull + (uint64_t)ep * 0xD1B54A32D192ED03ull + 0x1234567ull;
    t.perm_key = z;
    for (int64_t b = 0; b < nb && e == hipSuccess; ++b) {
      ++step;
      const double prog = total > 1 ? (double)(step - 1) / (double)(total - 1) : 0.0;
      const float lr = (float)(cfg->lr * 0.5 * (1.0 + std::cos(3.14159265358979323846 * prog)));
      t.batch_start = b * cfg->batch;
      e = klr::launch_train_step(t, w, klr::adam_args(lr, cfg->beta1, cfg->beta2, cfg->eps, step), nullptr,
                                 nullptr, loss_per_epoch + ep, 1.0f / (float)nb, s);
    }
  }
  h->timer.end(tm, s);
  return klr::hip_check(h, e, "klr_surrogate_train");
}

klr_status klr_surrogate_predict(klr_handle h, const void* params, int32_t n_kernels,
                                 const int32_t* kernel_id, const int32_t* N, const int32_t* launch,
                                 int64_t n, float* pred, void* stream) {
  if (!h) return KLR_E_INVALID;
  h->err.clear();
  if (!params || n_kernels < 1 || n < 0) return fail(h, KLR_E_INVALID, "bad arguments");
  if (n == 0) return KLR_OK;
  if (!kernel_id || !N || !launch || !pred) return fail(h, KLR_E_INVALID, "NULL array");
  if ((n + 63) / 64 >= (int64_t(1) << 31)) return fail(h, KLR_E_UNSUPPORTED, "too many samples");
  klr::Blob w = klr::blob_of(const_cast<void*>(params), n_kernels);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return klr::hip_check(h, klr::launch_predict(kernel_id, N, launch, n, n_kernels, w, pred, s),
                        "klr_surrogate_predict");
}

klr_status klr_surrogate_step(klr_handle h, void* params, int32_t n_kernels,
                              const int32_t* kernel_id, const int32_t* N, const int32_t* launch,
                              const float* target_std, int32_t batch, float lr, int32_t step,
                              float beta1, float beta2, float eps, float* grads, float* loss,
                              void* ws, size_t ws_bytes, void* stream) {
  if (!h) return KLR_E_INVALID;
  h->err.clear();
  if (!params || n_kernels < 1 || !klr::batch_ok(batch) || step < 1 || !kernel_id || !N || !launch ||
      !target_std)
    return fail(h, KLR_E_INVALID, "bad arguments (batch must be a multiple of 128, step >= 1)");
  const size_t need = klr::mlp_train_ws_bytes(n_kernels, batch);
  if (!ws || ws_bytes < need) return fail(h, KLR_E_WORKSPACE, "workspace too small");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0 || reinterpret_cast<uintptr_t>(params) % 256 != 0)
    return fail(h, KLR_E_INVALID, "params and workspace must be 256-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  klr::Blob w = klr::blob_of(params, n_kernels);
  klr::TrainTile t = klr::tile_args(ws, n_kernels, batch);
  t.kid = kernel_id; t.N = N; t.L = launch; t.cost = nullptr; t.tstd = target_std; t.n = batch;
  t.perm_bits = 0; t.batch_start = 0;
  float* ls = loss ? loss : klr::loss_slot(ws, n_kernels, batch);
  hipError_t e = klr::launch_refresh(w, s);
  if (e == hipSuccess) e = hipMemsetAsync(t.emb_acc, 0, (size_t)n_kernels * 8, s);
  if (e == hipSuccess)
    e = klr::launch_train_step(t, w, klr::adam_args(lr, beta1, beta2, eps, step), grads, ls, nullptr, 0.0f, s);
  return klr::hip_check(h, e, "klr_surrogate_step");
}

size_t klr_surrogate_eval_workspace(int32_t n_progs, int32_t max_cfg, int32_t max_q) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  return al(klr::eval_workspace_bytes(n_progs, max_cfg)) + al(klr::fallback_ws_bytes(n_progs, max_q));
}

klr_status klr_surrogate_eval(klr_handle h, const void* params, int32_t n_kernels,
                              const klr_program* progs, int32_t n_progs, int32_t max_cfg,
                              int32_t max_q, const klr_hw* hw, const klr_fit_desc* desc,
                              int32_t n_fits, const uint8_t* exps, int32_t n_exp_rows,
                              const double* coef, int64_t coef_len, const int32_t* cfgs,
                              int64_t cfgs_len, const int32_t* queries, int64_t q_len,
                              float margin, int32_t* argmin, float* pred_cost, uint8_t* fell_back,
                              float* pred_margin, int32_t* prog_status,
                              void* ws, size_t ws_bytes, void* stream) {
  if (!h) return KLR_E_INVALID;
  h->err.clear();
  if (!hw) return fail(h, KLR_E_INVALID, "hw is NULL");
  std::string why;
  if (!klr::hw_ok(*hw, why)) return fail(h, KLR_E_INVALID, why);
  if (!params || n_kernels < 1 || n_progs < 0 || max_cfg < 0 || max_q < 0 || q_len < 0 || cfgs_len < 0 ||
      coef_len < 0 || n_fits < 0 || n_exp_rows < 0 || !(margin >= 0.0f))
    return fail(h, KLR_E_INVALID, "bad arguments");
  if (n_progs == 0) return KLR_OK;
  if (max_cfg > 65536) return fail(h, KLR_E_UNSUPPORTED, "max_cfg above 65536");
  if (!progs || !desc || !exps || !coef || !cfgs || !queries || !argmin || !pred_cost || !fell_back)
    return fail(h, KLR_E_INVALID, "NULL array argument");
  const size_t need = klr_surrogate_eval_workspace(n_progs, max_cfg, max_q);
  if (!ws || ws_bytes < need) return fail(h, KLR_E_WORKSPACE, "workspace too small: need " + std::to_string(need));
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0 || reinterpret_cast<uintptr_t>(params) % 256 != 0)
    return fail(h, KLR_E_INVALID, "params and workspace must be 256-byte aligned");
  const int64_t items = (int64_t)n_progs * (((int64_t)max_q + 255) / 256) * 256;
  const int64_t items_c = (int64_t)n_progs * (((int64_t)max_cfg + 127) / 128) * 128;
  if (items >= (int64_t(1) << 31) || items_c >= (int64_t(1) << 32))
    return fail(h, KLR_E_UNSUPPORTED, "more than 2^31 query slots or 2^32 configuration slots; split the batch");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  klr::Blob w = klr::blob_of(const_cast<void*>(params), n_kernels);
  klr::SelectArgs sa{progs, n_progs, max_cfg, max_q, n_kernels, n_fits, hw->t_max, hw->wave, cfgs, cfgs_len,
                     queries, q_len, margin, argmin, pred_cost, fell_back, pred_margin, ws, *hw,
                     (int32_t)(h->opt[KLR_OPT_SURR_SHORTLIST] < 1 ? 1
                               : (h->opt[KLR_OPT_SURR_SHORTLIST] > klr::kMaxShortlist ? klr::kMaxShortlist
                                                                                       : h->opt[KLR_OPT_SURR_SHORTLIST]))};
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t ews = klr::eval_workspace_bytes(n_progs, max_cfg);
  klr::EvalArgs a{progs, n_progs, max_cfg, max_q, *hw, desc, n_fits, exps, n_exp_rows, coef, coef_len,
                  cfgs, cfgs_len, queries, q_len, argmin, pred_cost, nullptr, 0, prog_status, ws, ews, s,
                  h->capturing ? nullptr : &h->timer, 0, nullptr, 0};
  // collapse (program status, per-configuration records), network selection, then the pick
  // check, compaction and exact sweep of the flagged queries
  hipError_t e = klr::launch_collapse_only(a);
  const int t0 = h->capturing ? -1 : h->timer.begin(KLR_K_SURR, s);
  if (e == hipSuccess) e = klr::launch_select(sa, w, s);
  if (!h->capturing) h->timer.end(t0, s);
  if (e == hipSuccess) e = klr::launch_fallback(a, fell_back, pred_cost, reinterpret_cast<char*>(ws) + al(ews));
  return klr::hip_check(h, e, "klr_surrogate_eval");
}

}  // extern "C"

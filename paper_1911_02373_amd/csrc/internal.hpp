// Internal declarations shared by the HIP translation units of libklr (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "klr.h"

namespace klr {

// Optional per-kernel event timing (see klr_profile_enable).
struct Timer {
  bool on = false;
  struct Rec { int kind; hipEvent_t a, b; };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  double total_ms[KLR_K_COUNT] = {0};
  int64_t count[KLR_K_COUNT] = {0};
  hipEvent_t get();
  // Record the start event of a kernel of `kind` on `s` (returns the index or -1 when off).
  int begin(int kind, hipStream_t s);
  void end(int idx, hipStream_t s);
  hipError_t drain();
  void reset();
  ~Timer();
};

}  // namespace klr

struct klr_handle_s {
  int device = 0;
  std::string err;
  klr::Timer timer;
};

namespace klr {

// Record the error text on the handle and return the status.
klr_status fail(klr_handle h, klr_status st, const std::string& msg);
klr_status hip_check(klr_handle h, hipError_t e, const char* what);

// ---- eval ---------------------------------------------------------------------------------
struct EvalArgs {
  const klr_program* progs;
  int32_t n_progs, max_cfg, max_q;
  klr_hw hw;
  const klr_fit_desc* desc;
  int32_t n_fits;
  const uint8_t* exps;
  int32_t n_exp_rows;
  const double* coef;
  int64_t coef_len;
  const int32_t* cfgs;
  int64_t cfgs_len;
  const int32_t* queries;
  int64_t q_len;
  int32_t* argmin;
  float* best_cost;
  float* all_costs;
  int64_t costs_len;
  int32_t* prog_status;
  void* ws;
  size_t ws_bytes;
  hipStream_t stream;
  Timer* timer;
};

size_t eval_workspace_bytes(int32_t n_progs, int32_t max_cfg);
hipError_t launch_eval(const EvalArgs& a);

// ---- fit ----------------------------------------------------------------------------------
struct FitArgs {
  const klr_fit_desc* desc;
  int32_t n_fits;
  const uint8_t* exps;
  int32_t n_exp_rows;
  const int32_t* X;
  int64_t x_len;
  const double* f;
  int64_t f_len;
  int32_t precision, max_iter;
  double tol;
  double* coef;
  int64_t coef_len;
  klr_fit_info* info;
  void* ws;
  size_t ws_bytes;
  hipStream_t stream;
  Timer* timer;
};

size_t fit_workspace_bytes(int32_t n_fits, int64_t f_len, int32_t precision);
hipError_t launch_fit(const FitArgs& a);

}  // namespace klr

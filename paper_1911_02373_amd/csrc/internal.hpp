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

// Launch-shape autotuner cache: shape key -> chosen variant (kept per handle; optionally
// persisted in the text file named by KLR_TUNE_CACHE, one "key variant ms" line per entry).
struct Tuner {
  std::vector<std::pair<uint64_t, int>> entries;
  std::string path;
  int find(uint64_t key) const {
    for (const auto& e : entries)
      if (e.first == key) return e.second;
    return -1;
  }
  void record(uint64_t key, int variant, float ms);
  void load();
};
// Tune-cache keys: bit 56 marks an evaluation shape, bit 57 a fit batch.
constexpr uint64_t kTuneEvalTag = 1ull << 56;
constexpr uint64_t kTuneFitTag = 2ull << 56;

}  // namespace klr

struct klr_handle_s {
  int device = 0;
  std::string err;
  klr::Timer timer;
  klr::Tuner tuner;
  bool capturing = false;
  int64_t opt[8] = {1, -1, -1, 4, 0, 0, 0, 0};   // see KLR_OPT_* in klr.h
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
  int variant;             // launch shape of the sweep; < 0: autotune with `tuner`
  Tuner* tuner;
  uint64_t tune_key;
};

size_t eval_workspace_bytes(int32_t n_progs, int32_t max_cfg);
hipError_t launch_eval(const EvalArgs& a);
int eval_num_variants();
int64_t selftest_divisors(uint32_t d_max);
int64_t selftest_divisor_list(const uint64_t* ds, int32_t n_ds);
int64_t selftest_short_division(int32_t b_first, int32_t b_count);

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
  bool persistent;         // longest-first persistent schedule (else one workgroup per fit)
  int64_t* rowoff;         // per-fit first scratch row (workspace, set by fit_workspace_split)
  double* scratch;         // 2 x scratch_rows FP64 residual scratch (workspace)
  int64_t scratch_rows;
  int wave_group = 4;      // fits per workgroup of the one-wavefront kernel (1, 2 or 4)
  int variant = -1;        // index into the fit launch variants; < 0: autotune with `tuner`
  Tuner* tuner = nullptr;
  uint64_t tune_key = 0;
};
// Fit launch variants (all give bit-identical results): fits per workgroup of the one-wavefront
// kernel.
constexpr int kFitVariants = 3;
constexpr int kFitWaveGroups[kFitVariants] = {4, 2, 1};

size_t fit_workspace_bytes(int32_t n_fits, int64_t total_rows, int32_t precision);
// Point rowoff / scratch / scratch_rows of `a` into its workspace (a.ws, a.ws_bytes, a.n_fits).
void fit_workspace_split(FitArgs& a);
hipError_t launch_fit(const FitArgs& a);
// Fits by one-sided Jacobi SVD (KLR_FP64_SVD), one workgroup per fit.
hipError_t launch_fit_svd(const FitArgs& a);

// Rows per lane of the one-wavefront fit kernel for this fit: 8 (m <= 512) or 16 (m <= 1024)
// when n <= 48, v <= 4 and every exponent is <= 3; 0 when the fit takes the workgroup kernel.
__device__ inline int wave_fit_rows(const FitArgs& a, const klr_fit_desc& d) {
  const int n = d.n_num + d.n_den - 1;
  if (!(d.n_num >= 0 && d.n_den >= 1 && n >= 1 && n <= 48 && d.v >= 1 && d.v <= 4 && d.m >= 1 && d.m <= 1024))
    return 0;
  if (d.num0 < 0 || (int64_t)d.num0 + d.n_num > a.n_exp_rows || d.den0 < 0 ||
      (int64_t)d.den0 + d.n_den > a.n_exp_rows)
    return 0;
  for (int r = 0; r < d.n_num + d.n_den; ++r) {
    const int64_t row = r < d.n_num ? (int64_t)d.num0 + r : (int64_t)d.den0 + (r - d.n_num);
    for (int k = 0; k < d.v; ++k)
      if (a.exps[row * KLR_MAX_VARS + k] > 3) return 0;
  }
  return d.m <= 512 ? 8 : 16;
}
// ---- cross-lane moves on the VALU (no LDS round trip) ----------------------------------------
// Lane l's value of v, broadcast through scalar registers (l wave-uniform).
__device__ __forceinline__ double readlane_d(double v, int l) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, l);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// DPP move of a double within rows of 16 lanes (CTRL: quad_perm, row_mirror, ...).  Every lane
// of the wavefront must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141; // lane i <- 7 - i within each 8 lanes
constexpr int kDppMirror = 0x140;     // lane i <- 15 - i within each 16 lanes

// Sum over aligned groups of G lanes (G = 4, 8 or 16); every lane of a group receives the same
// value (each step adds a value from the other half of the group, and addition commutes).
// Every lane of the wavefront must be active.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  static_assert(G == 4 || G == 8 || G == 16, "group of 4, 8 or 16 lanes");
  v += dpp_d<kDppXor1>(v);
  v += dpp_d<kDppXor2>(v);
  if (G >= 8) v += dpp_d<kDppHalfMirror>(v);
  if (G >= 16) v += dpp_d<kDppMirror>(v);
  return v;
}

// Sum of lane l and lane l ^ 16 (resp. l ^ 32) through the gfx950 lane-swap instructions:
// swapping a register with itself leaves the value of one half of each lane pair in each of the
// two results, so their sum is the pair sum, in the same order in every lane.
__device__ __forceinline__ double pair_sum16(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)u, (unsigned)u, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
  const double a = __longlong_as_double((long long)(((unsigned long long)(unsigned)hi[0] << 32) | (unsigned)lo[0]));
  const double b = __longlong_as_double((long long)(((unsigned long long)(unsigned)hi[1] << 32) | (unsigned)lo[1]));
  return a + b;
}
__device__ __forceinline__ double pair_sum32(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)u, (unsigned)u, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
  const double a = __longlong_as_double((long long)(((unsigned long long)(unsigned)hi[0] << 32) | (unsigned)lo[0]));
  const double b = __longlong_as_double((long long)(((unsigned long long)(unsigned)hi[1] << 32) | (unsigned)lo[1]));
  return a + b;
}

// Sum over the 64 lanes of the wavefront, the same value in every lane (all lanes active).
__device__ __forceinline__ double wave_sum_d(double v) {
  return pair_sum32(pair_sum16(group_sum<16>(v)));
}

// FP32 versions: sum over aligned groups of 16 lanes by DPP, and the pair sum of lanes l and
// l ^ 16 by the lane-swap instruction (all lanes active).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float group16_sum_f(float v) {
  v += dpp_f<kDppXor1>(v);
  v += dpp_f<kDppXor2>(v);
  v += dpp_f<kDppHalfMirror>(v);
  v += dpp_f<kDppMirror>(v);
  return v;
}
__device__ __forceinline__ float pair_sum16_f(float v) {
  const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float((unsigned)s[0]) + __uint_as_float((unsigned)s[1]);
}
__device__ __forceinline__ float pair_sum32_f(float v) {
  const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float((unsigned)s[0]) + __uint_as_float((unsigned)s[1]);
}

// Largest key over the 64 lanes, lowest index among equal keys (keys are never NaN); every
// lane receives the same (key, index).  All lanes active.
__device__ __forceinline__ void argmax_take(double& best, int& bi, double ob, int oi) {
  const bool take = (ob > best) | ((ob == best) & (oi < bi));   // selects, no branch
  best = take ? ob : best;
  bi = take ? oi : bi;
}
template <int CTRL>
__device__ __forceinline__ void argmax_dpp(double& best, int& bi) {
  const double ob = dpp_d<CTRL>(best);
  const int oi = dpp_i<CTRL>(bi);
  argmax_take(best, bi, ob, oi);
}
template <bool K32>
__device__ __forceinline__ void argmax_swap(double& best, int& bi) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(best);
  const unsigned ulo = (unsigned)u, uhi = (unsigned)(u >> 32), ui = (unsigned)bi;
  const auto lo = K32 ? __builtin_amdgcn_permlane32_swap(ulo, ulo, false, false)
                      : __builtin_amdgcn_permlane16_swap(ulo, ulo, false, false);
  const auto hi = K32 ? __builtin_amdgcn_permlane32_swap(uhi, uhi, false, false)
                      : __builtin_amdgcn_permlane16_swap(uhi, uhi, false, false);
  const auto ix = K32 ? __builtin_amdgcn_permlane32_swap(ui, ui, false, false)
                      : __builtin_amdgcn_permlane16_swap(ui, ui, false, false);
  best = __longlong_as_double((long long)(((unsigned long long)(unsigned)hi[0] << 32) | (unsigned)lo[0]));
  bi = (int)ix[0];
  const double ob = __longlong_as_double((long long)(((unsigned long long)(unsigned)hi[1] << 32) | (unsigned)lo[1]));
  argmax_take(best, bi, ob, (int)ix[1]);
}
__device__ __forceinline__ void wave_argmax(double& best, int& bi) {
  argmax_dpp<kDppXor1>(best, bi);
  argmax_dpp<kDppXor2>(best, bi);
  argmax_dpp<kDppHalfMirror>(best, bi);
  argmax_dpp<kDppMirror>(best, bi);
  argmax_swap<false>(best, bi);
  argmax_swap<true>(best, bi);
}

// Rounds an FP32 value to the nearest BF16 value (ties to even), kept in FP32.
__device__ __forceinline__ float round_bf16(float x) {
  uint32_t b = __float_as_uint(x);
  b = (b + 0x7FFFu + ((b >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(b);
}

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Gram products on the matrix cores, per Gram precision.  One MFMA covers SUB steps of 4 sample
// rows.  FP64 and FP32 (SUB = 1, v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  BF16 (SUB = 4, v_mfma_f32_16x16x16_bf16): lane l
// supplies A[l % 16][4 (l / 16) + e] and B[4 (l / 16) + e][l % 16], e = 0..3; the callers give
// reduction index 4 (l / 16) + e the row of sub-step e that the lane's group reads (row 4 e +
// l / 16 of the 16-row block), the same for both operands, so every product pairs two values of
// one row.  Result register r of lane l is D[out_row(l / 16, r)][l % 16]: row 4 r + l / 16 for
// the FP64 instruction, 4 (l / 16) + r for the FP32 and BF16 ones.  The reduced paths round the
// design-matrix values to FP32 or BF16 (through FP32) and accumulate in FP32 (products of BF16
// values are exact in FP32).
typedef short s16x4 __attribute__((ext_vector_type(4)));
template <int GP>
struct GramTypes;
template <>
struct GramTypes<KLR_FP64> {
  typedef f64x4 acc_t;
  typedef double op_t;
  static constexpr int SUB = 1;
  static __device__ __forceinline__ void put(op_t& o, int, double v) { o = v; }
  static __device__ __forceinline__ op_t zero() { return 0.0; }
  static __device__ __forceinline__ acc_t mma(op_t a, op_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int grp, int r) { return 4 * r + grp; }
};
template <>
struct GramTypes<KLR_FP32_REFINED> {
  typedef f32x4 acc_t;
  typedef float op_t;
  static constexpr int SUB = 1;
  static __device__ __forceinline__ void put(op_t& o, int, double v) { o = (float)v; }
  static __device__ __forceinline__ op_t zero() { return 0.0f; }
  static __device__ __forceinline__ acc_t mma(op_t a, op_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int grp, int r) { return 4 * grp + r; }
};
template <>
struct GramTypes<KLR_BF16_REFINED> {
  typedef f32x4 acc_t;
  typedef s16x4 op_t;
  static constexpr int SUB = 4;
  static __device__ __forceinline__ void put(op_t& o, int e, double v) {
    const short b = (short)(__float_as_uint(round_bf16((float)v)) >> 16);
    if (e == 0) o[0] = b;
    else if (e == 1) o[1] = b;
    else if (e == 2) o[2] = b;
    else o[3] = b;
  }
  static __device__ __forceinline__ op_t zero() { return (op_t){0, 0, 0, 0}; }
  static __device__ __forceinline__ acc_t mma(op_t a, op_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int grp, int r) { return 4 * grp + r; }
};

struct WavePlanView {        // the wave-fit part of the longest-first order
  const int32_t* order;
  const int32_t* total;
  const int32_t* base;
};
hipError_t launch_fit_wave(const FitArgs& a, bool ordered, const WavePlanView& pv8, const WavePlanView& pv16);

// ---- surrogate network ----------------------------------------------------------------------
// Parameter vector layout (floats): W2[256][256] | W1[256][4] | b1 | b2 | w3 | b3 | pad | emb.
constexpr int kO_W2 = 0;
constexpr int kO_W1 = KLR_MLP_HIDDEN * KLR_MLP_HIDDEN;
constexpr int kO_B1 = kO_W1 + KLR_MLP_HIDDEN * KLR_MLP_IN;
constexpr int kO_B2 = kO_B1 + KLR_MLP_HIDDEN;
constexpr int kO_W3 = kO_B2 + KLR_MLP_HIDDEN;
constexpr int kO_B3 = kO_W3 + KLR_MLP_HIDDEN;
constexpr int kO_EMB = kO_B3 + 16;
constexpr int kLossSlot = kO_B3 - kO_W1 + 1;          // per-tile partial row: small grads, loss
constexpr int kPartialStride = kO_EMB - kO_W1;
inline int64_t mlp_np(int32_t nk) { return ((int64_t)kO_EMB + nk + 63) / 64 * 64; }
inline size_t mlp_param_bytes(int32_t nk) {
  return (size_t)(16 + 3 * mlp_np(nk)) * sizeof(float) +
         (size_t)2 * KLR_MLP_HIDDEN * KLR_MLP_HIDDEN * sizeof(uint16_t);
}

struct Blob {
  float* hdr;
  float* P;
  float* M;
  float* V;
  uint16_t* W2b;
  uint16_t* W2Tb;
};
Blob blob_of(void* base, int32_t nk);

struct AdamArgs {
  float lr, b1, b2, eps, bc1, bc2;   // bc = 1 - beta^step
};

struct TrainTile {
  const int32_t* kid;
  const int32_t* N;
  const int32_t* L;
  const float* cost;       // exact costs (ln taken in the kernel), or
  const float* tstd;       // standardised targets (when non-null)
  int64_t n;
  int32_t B;
  int64_t batch_start;     // position of the batch in the epoch order
  uint64_t perm_key;
  int32_t perm_bits;       // 0: no permutation (samples in order)
  int32_t nk;
  uint16_t* H1T;           // [256][B] bf16
  uint16_t* dH2T;          // [256][B] bf16
  float* partial;          // [B / 64][kPartialStride]
  unsigned long long* emb_acc;   // [nk] fixed point 2^-44
  float* dw2_part;         // [kDw2Slices][256][256] slice partials of dW2
};
constexpr int kDw2Slices = 16;
size_t mlp_train_ws_bytes(int32_t nk, int32_t B);

constexpr int kMaxShortlist = 4;      // configurations the selection re-ranks exactly per query
struct SelectArgs {
  const klr_program* progs;
  int32_t n_progs, max_cfg, max_q, nk, n_fits;
  int32_t t_max, wave;
  const int32_t* cfgs;
  int64_t cfgs_len;
  const int32_t* queries;
  int64_t q_len;
  float margin;
  int32_t* argmin;
  float* pred_cost;
  uint8_t* fell_back;
  float* pred_margin;      // optional: second-best minus best prediction (ln units) per query
  const void* eval_ws;     // the collapse workspace of the same programs (launch_collapse_only)
  klr_hw hw;
  int32_t shortlist;       // predicted-best configurations re-ranked by their exact costs (1..4)
};

hipError_t launch_refresh(const Blob& w, hipStream_t s);
hipError_t launch_stats(const float* cost, int64_t n, float* hdr, hipStream_t s);
hipError_t launch_train_step(const TrainTile& t, const Blob& w, const AdamArgs& ad, float* grads,
                             float* loss_step, float* loss_epoch, float epoch_scale, hipStream_t s);
hipError_t launch_predict(const int32_t* kid, const int32_t* N, const int32_t* L, int64_t n, int32_t nk,
                          const Blob& w, float* pred, hipStream_t s);
hipError_t launch_select(const SelectArgs& a, const Blob& w, hipStream_t s);

// Exact re-evaluation of the queries flagged by the surrogate (compaction by program, then the
// exact sweep over the compacted list); the collapse workspace must already hold the program
// coefficients (launch_eval's collapse).  Workspace beyond eval_workspace_bytes:
size_t fallback_ws_bytes(int32_t n_progs, int32_t max_q);
hipError_t launch_fallback(const EvalArgs& a, uint8_t* flags, float* best_cost, void* fws);
hipError_t launch_collapse_only(const EvalArgs& a);

}  // namespace klr

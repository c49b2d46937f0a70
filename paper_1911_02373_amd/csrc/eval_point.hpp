// Per-point pieces of the rational-program evaluation, shared by the exact sweep (eval.hip) and
// the surrogate selection (mlp.hip): the layout of the collapse workspace, the fitted metric
// values and the occupancy terms.  One definition of each FP32 step keeps the selection's
// admissibility mask identical to the exact sweep's decisions.
//
// Paper: step 4 ("Rational program evaluation") of the section "An Algorithm to Build and Deploy
// a Performance-Predicting Rational Program" and the occupancy flowchart of Example "Hardware
// occupancy" (with eq. (occupancy)).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "internal.hpp"

namespace klr {

constexpr int kNdeg = KLR_MAX_NDEG;            // powers 0..3 of N~
constexpr int kSlotFloats = KLR_N_METRICS * 2 * (kNdeg + 1) + KLR_N_METRICS;   // 72

struct CfgRec {          // per (program, configuration) occupancy terms
  int32_t T;             // threads per block = prod L
  float Wb;              // waves per block = T / wave (an integer, exact in FP32)
  float Bcap;            // min(b_max, floor(wave * w_max / T)) (an integer below 2^11)
  float rTh;             // floor(r_max / T) + 1/2; floor(r_max / (R T)) = floor(floor(r_max / T) / R)
  int32_t Lmax;          // largest launch parameter (admissible only if <= N)
  int32_t L0, L1;        // first two launch parameters (two-dimensional grid)
  int32_t ok;            // configuration admissible and the program's fits valid
  uint32_t magTC;        // floor(n / (T n_cu)) = mulhi(n, magTC) >> shTC for 0 <= n < 2^31
  int32_t shTC;
  int32_t fast;          // quotients taking the short division at every query: 0 none, 1 the
                         //   metrics', 2 the metrics' and the cycle estimate's
  int32_t pad;
};

struct Hw32 {
  int32_t n_cu;
  float w_max;           // integers below 2^11, exact in FP32
  float zh;              // z_max + 1/2 (z_max < 2^20)
  float lat, dep, iss, bw;
};

__host__ __device__ inline Hw32 make_hw32(const klr_hw& h) {
  return Hw32{h.n_cu, (float)h.w_max, (float)h.z_max + 0.5f, h.mem_lat, h.dep_delay, h.issue_cycles, h.bw};
}

// Collapse workspace: n_progs * max_cfg coefficient slots of kSlotFloats floats (slot p max_cfg
// + c), then one CfgRec per slot, then the per-program highest power of N~.
__host__ __device__ inline const float* slot_coefs(const void* ws) { return reinterpret_cast<const float*>(ws); }
__host__ __device__ inline const CfgRec* slot_recs(const void* ws, int32_t n_progs, int32_t max_cfg) {
  return reinterpret_cast<const CfgRec*>(reinterpret_cast<const char*>(ws) +
                                         (int64_t)n_progs * max_cfg * kSlotFloats * (int64_t)sizeof(float));
}

// Exact floor(a / b) for integers 0 <= a < 2^20 and 1 <= b <= 2^24, given ah = a + 1/2 (exact
// in FP32).  With a = k b + j, 0 <= j < b, the quotient (a + 1/2) / b = k + (j + 1/2) / b lies at
// least 1/(2b) from every integer.  The reciprocal is within one ulp (relative error <= 2^-23)
// and the product adds at most 2^-24, so ah b^-1 is within ((a + 1/2) / b) 2^-22 < 1/(2b) of
// the quotient and its floor is k.  b = +0 gives +inf.
__device__ __forceinline__ float floor_div(float ah, float b) {
  return floorf(ah * __builtin_amdgcn_rcpf(b));
}

__device__ __forceinline__ float sel_min(float a, float b) { return b < a ? b : a; }
__device__ __forceinline__ float sel_max(float a, float b) { return b > a ? b : a; }
// sel_max(good ? v : +0, lo) for lo in {+0, 1}: a failed metric yields lo either way.
__device__ __forceinline__ float clean_max(bool good, float v, float lo) {
  return (good && !(lo > v)) ? v : lo;
}

// Two adjacent wave-uniform floats (8-byte aligned) copied into a vector register pair.
__device__ __forceinline__ float2 vgpr_pair(const float* p) {
  const uint64_t s = *reinterpret_cast<const uint64_t*>(p);
  uint64_t v;
  asm("v_mov_b64 %0, %1" : "=v"(v) : "s"(s));
  return make_float2(__uint_as_float((uint32_t)v), __uint_as_float((uint32_t)(v >> 32)));
}

// Scaled query size per metric, x_j = N * 2^-s_j with s_j the scale exponent of metric j's fit.
// The collapse kernel writes the same scales into every configuration slot of a program (a
// program whose fits are invalid gets 1 and an inadmissible record in every slot), so the
// products are formed once per query from the first slot and reused across configurations.
__device__ __forceinline__ void scaled_n(int32_t N, const float* __restrict__ slot0, float* x) {
#pragma clang fp contract(off)
  const float fN = (float)N;
#pragma unroll
  for (int j = 0; j < KLR_N_METRICS; ++j) x[j] = fN * slot0[KLR_N_METRICS * 2 * (kNdeg + 1) + j];
}

// One fitted function j of a configuration slot at the scaled size x: p / q by Horner from
// power DEG (fused multiply-adds), then the correctly rounded quotient; *good = q > 0 and the
// value finite.  UNI: the slot is the same in every lane (its coefficients sit in scalar
// registers); otherwise each lane reads its own slot.
template <int DEG = kNdeg, bool UNI = true>
__device__ __forceinline__ float fitted_value(const float* __restrict__ cf, int j, float x, bool* good) {
#pragma clang fp contract(off)
  const float* c = cf + j * 2 * (kNdeg + 1);
  const float2 lo = UNI ? vgpr_pair(c + 2 * (DEG - 1)) : make_float2(c[2 * (DEG - 1)], c[2 * DEG - 1]);
  float p = __builtin_fmaf(c[2 * DEG], x, lo.x);
  float q = __builtin_fmaf(c[2 * DEG + 1], x, lo.y);
#pragma unroll
  for (int d = DEG - 2; d >= 0; --d) {
    p = __builtin_fmaf(p, x, c[2 * d]);
    q = __builtin_fmaf(q, x, c[2 * d + 1]);
  }
  const float g = p / q;
  *good = (q > 0.0f) & (fabsf(g) <= 3.402823466e38f);
  return g;
}

// Resident blocks per compute unit from the fitted register (g5) and LDS (g6) metrics:
// R = min(max(ceil g5, 1), 2^24), Z = min(max(ceil g6, 0), 2^24) (a failed metric counts as its
// lower clamp), B = min(b_max, floor(wave w_max / T), floor(r_max / (R T)), floor(z_max / Z)).
// Every term is an integer held exactly in FP32 (the LDS term is +inf when Z = 0: no LDS bound).
__device__ __forceinline__ float resident_blocks(float g5, bool good5, float g6, bool good6, const CfgRec& r,
                                                 const Hw32& hw) {
#pragma clang fp contract(off)
  const float R = fminf(clean_max(good5, ceilf(g5), 1.0f), 16777216.0f);
  const float Z = fminf(clean_max(good6, ceilf(g6), 0.0f), 16777216.0f);   // -0 for g in (-1, 0)
  const float breg = floor_div(r.rTh, R);
  const float blds = floor_div(hw.zh, fabsf(Z));   // Z = -0 counts as 0
  return fminf(fminf(r.Bcap, breg), blds);
}

// The same for metrics known to be defined, finite and nonzero (the clamps are then maxima; a
// ceiling of -0 for Z counts as 0 through the absolute value either way).
__device__ __forceinline__ float resident_blocks_defined(float g5, float g6, const CfgRec& r, const Hw32& hw) {
#pragma clang fp contract(off)
  const float R = fminf(fmaxf(ceilf(g5), 1.0f), 16777216.0f);
  const float Z = fminf(fmaxf(ceilf(g6), 0.0f), 16777216.0f);
  const float breg = floor_div(r.rTh, R);
  const float blds = floor_div(hw.zh, fabsf(Z));
  return fminf(fminf(r.Bcap, breg), blds);
}

// Whether the exact evaluation can give a point a finite cost: the configuration is admissible
// for the program, no launch parameter exceeds N, every fitted function the cost reads is
// defined (q > 0, finite value) and, for the cycle estimate, at least one block is resident.
// A point this rejects has cost +inf in the exact sweep; the converse fails only where the
// cycle estimate itself overflows.  Slots are per lane (UNI = false); powers from kNdeg.
__device__ __forceinline__ bool point_admissible(int kind, int32_t N, const float* xs, const float* __restrict__ cf,
                                                 const CfgRec& r, const Hw32& hw) {
  bool ok = (r.ok != 0) & (N >= r.Lmax);
  if (kind == KLR_COST_METRIC) {
    bool g0;
    (void)fitted_value<kNdeg, false>(cf, 0, xs[0], &g0);
    return ok & g0;
  }
  if (kind == KLR_COST_PIECEWISE) {
    bool gd, ga, gb;
    const float d = fitted_value<kNdeg, false>(cf, 0, xs[0], &gd);
    (void)fitted_value<kNdeg, false>(cf, 1, xs[1], &ga);
    (void)fitted_value<kNdeg, false>(cf, 2, xs[2], &gb);
    return ok & gd & (d >= 0.0f ? ga : gb);
  }
  float g5 = 0.0f, g6 = 0.0f;
  bool good5 = false, good6 = false;
#pragma unroll
  for (int j = 0; j < KLR_N_METRICS; ++j) {
    bool gj;
    const float g = fitted_value<kNdeg, false>(cf, j, xs[j], &gj);
    ok = ok & gj;
    if (j == 5) { g5 = g; good5 = gj; }
    if (j == 6) { g6 = g; good6 = gj; }
  }
  return ok & (resident_blocks(g5, good5, g6, good6, r, hw) >= 1.0f);
}

}  // namespace klr

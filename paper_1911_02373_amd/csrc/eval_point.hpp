// Per-point pieces of the rational-program evaluation, shared by the exact sweep (eval.hip) and
// the surrogate selection (mlp.hip): the layout of the collapse workspace, the fitted metric
// values, the occupancy terms and the normative FP32 cost of a point.  One definition of each
// FP32 step keeps the selection's admissibility mask and its exact re-ranking identical to the
// exact sweep's decisions.
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

__device__ __forceinline__ uint32_t udiv_magic(uint32_t n, uint32_t m, int32_t sh) {
  return sh < 0 ? n : (__umulhi(n, m) >> sh);
}

// Quotient a / b for operands of moderate size: reciprocal estimate, one Newton step, then one
// correction of the quotient by its exact FMA remainder (six instructions, against the eleven of
// the correctly rounded FP32 division with its range scaling and special-case fix-up).  For
// finite a, b with |a| and |b| in [2^-40, 2^40] the result is the IEEE quotient bit for bit:
// klr_selftest_short_division compares the two over every pair of mantissas in [1, 2) and checks
// that the reciprocal estimate scales exactly with b's exponent and sign.  In that range every
// step's rounded result is a normal number or zero (a nonzero remainder is at least 2^-87 in
// magnitude; the product inside an FMA is not rounded), so each step, and the correctly rounded
// quotient, scale with the operands' exponents and signs.
__device__ __forceinline__ float div_moderate(float a, float b) {
#pragma clang fp contract(off)
  const float y0 = __builtin_amdgcn_rcpf(b);
  const float e0 = __builtin_fmaf(-b, y0, 1.0f);
  const float y1 = __builtin_fmaf(e0, y0, y0);
  const float q0 = a * y1;
  const float r0 = __builtin_fmaf(-b, q0, a);
  return __builtin_fmaf(r0, y1, q0);
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

// Whether the exact evaluation can give a point a finite cost, from the cheap part of the
// rational program: the configuration is admissible for the program and no launch parameter
// exceeds N; for a cycle-estimate program every metric denominator is positive and, from the
// register and LDS metrics, at least one block is resident; for the other kinds every fitted
// function the cost reads is defined (q > 0, finite value).  A point this rejects has cost +inf
// in the exact sweep (the same FP32 steps); the converse fails where a metric value or the
// cycle estimate overflows FP32.  Slots are per lane (UNI = false); powers from kNdeg.
__device__ __forceinline__ bool point_admissible(int kind, int32_t N, const float* xs, const float* __restrict__ cf,
                                                 const CfgRec& r, const Hw32& hw) {
#pragma clang fp contract(off)
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
#pragma unroll
  for (int j = 0; j < KLR_N_METRICS; ++j) {
    if (j == 5 || j == 6) continue;
    const float* c = cf + j * 2 * (kNdeg + 1);       // the denominator: odd entries, by power
    float q = __builtin_fmaf(c[2 * kNdeg + 1], xs[j], c[2 * kNdeg - 1]);
#pragma unroll
    for (int d = kNdeg - 2; d >= 0; --d) q = __builtin_fmaf(q, xs[j], c[2 * d + 1]);
    ok = ok & (q > 0.0f);
  }
  bool good5, good6;
  const float g5 = fitted_value<kNdeg, false>(cf, 5, xs[5], &good5);
  const float g6 = fitted_value<kNdeg, false>(cf, 6, xs[6], &good6);
  return ok & good5 & good6 & (resident_blocks(g5, good5, g6, good6, r, hw) >= 1.0f);
}

// The cycle estimate of one point from its metric values g (g[j] = p_j / q_j; good[j]: q > 0
// and the value finite; ok: the point admissible so far), steps 2-6 of the normative sequence.
// SHORT (the configuration record's `fast`): 1 - every metric is defined, finite and nonzero, so
// the clamps reduce to maxima; 2 - besides, the four quotients of the cycle estimate have
// operands in [2^-40, 2^40] and take div_moderate, so MWP's bounds are positive and finite and
// its compare-select clamps equal the minimum and maximum.
template <int GRID, int SHORT>
__device__ __forceinline__ float cycle_cost(int32_t N, const float* g, const bool* good, bool ok, const CfgRec& r,
                                            const Hw32& hw) {
#pragma clang fp contract(off)
  // A metric failing the check is cleaned to +0 before its clamp; clean_max takes both steps.
  // The upper clamps of R (>= 1) and Z (>= -0) see no NaN, so fminf equals the compare-select.
  // (with SHORT every value is finite and nonzero, so the compare-select equals the maximum)
  const float Icomp = SHORT ? fmaxf(g[0], 0.0f) : clean_max(good[0], g[0], 0.0f);
  const float Imc = SHORT ? fmaxf(g[1], 0.0f) : clean_max(good[1], g[1], 0.0f);
  const float Imu = SHORT ? fmaxf(g[2], 0.0f) : clean_max(good[2], g[2], 0.0f);
  const float U = SHORT ? fmaxf(g[3], 1.0f) : clean_max(good[3], g[3], 1.0f);
  const float Isync = SHORT ? fmaxf(g[4], 0.0f) : clean_max(good[4], g[4], 0.0f);
  const float Bw = SHORT ? fmaxf(g[7], 1.0f) : clean_max(good[7], g[7], 1.0f);

  // occupancy from the register and LDS metrics; the minima and the products below equal their
  // integer counterparts
  const float B = SHORT ? resident_blocks_defined(g[5], g[6], r, hw)
                        : resident_blocks(g[5], good[5], g[6], good[6], r, hw);
  ok = ok & (B >= 1.0f);
  const float Bf = fmaxf(B, 1.0f);
  const float Nwf = fminf(Bf * r.Wb, hw.w_max);     // a product above 2^24 is above w_max too
  const int32_t Nc = N >= 1 ? N : 1;
  float repf;
  if (GRID == KLR_GRID_1D) {
    // rep = ceil(blocks / (B n_cu)) = ceil(ceil(blocks / n_cu) / B), blocks = ceil(N / T);
    // ceil(blocks / n_cu) - 1 = floor(floor((N - 1) / T) / n_cu) = floor((N - 1) / (T n_cu))
    const uint32_t cm1 = udiv_magic((uint32_t)(Nc - 1), r.magTC, r.shTC);
    if (cm1 < (1u << 20))
      repf = floor_div((float)cm1 + 0.5f, Bf) + 1.0f;
    else
      repf = (float)(cm1 / (uint32_t)Bf + 1u);
  } else {
    const uint64_t blocks = (uint64_t)((uint32_t)(Nc - 1) / (uint32_t)r.L0 + 1u) *
                            (uint64_t)((uint32_t)(Nc - 1) / (uint32_t)r.L1 + 1u);
    const uint64_t rep = (blocks - 1u) / (uint64_t)((uint32_t)Bf * (uint32_t)hw.n_cu) + 1u;
    repf = (float)rep;
  }

  const float Im = Imc + Imu;
  const float Lu = __builtin_fmaf(U - 1.0f, hw.dep, hw.lat);      // (U - 1) dep + lat
  const float mem = __builtin_fmaf(Lu, Imu, hw.lat * Imc);         // lat I_mc + L_u I_mu
  float comp = Icomp + Im;
  comp = hw.iss * comp;

  float d1 = __builtin_fmaf(U, Imu, Imc);                          // I_mc + U I_mu
  d1 = hw.dep * d1;
  const float mwp_lat = SHORT == 2 ? div_moderate(mem, d1) : mem / d1;
  const float n2 = hw.bw * mem;
  const float d2 = Im * Bw;
  const float mwp_bw = SHORT == 2 ? div_moderate(n2, d2) : n2 / d2;
  float mwp = SHORT == 2 ? fminf(mwp_lat, mwp_bw) : sel_min(mwp_lat, mwp_bw);
  mwp = SHORT == 2 ? fminf(mwp, Nwf) : sel_min(mwp, Nwf);
  mwp = SHORT == 2 ? fmaxf(mwp, 1.0f) : sel_max(mwp, 1.0f);
  const float tot = mem + comp;
  const bool cwp_full = tot >= Nwf * comp;
  const bool cwp_ge_mwp = tot >= mwp * comp;
  const float cpm = SHORT == 2 ? div_moderate(comp, Im) : comp / Im;
  const float m1 = mwp - 1.0f;
  const float e1 = __builtin_fmaf(cpm, m1, tot);                   // tot + cpm (MWP - 1)
  float t2 = mem * Nwf;
  t2 = SHORT == 2 ? div_moderate(t2, mwp) : t2 / mwp;
  const float e2 = __builtin_fmaf(cpm, m1, t2);                    // mem N_w / MWP + cpm (MWP - 1)
  const float e3 = __builtin_fmaf(comp, Nwf, hw.lat);              // lat + comp N_w
  const bool case1 = (mwp >= Nwf) & cwp_full;
  const bool case2 = cwp_ge_mwp | (comp > mem);
  float ex = case1 ? e1 : (case2 ? e2 : e3);
  const bool pure = (Im == 0.0f);
  mwp = pure ? 1.0f : mwp;
  ex = pure ? comp * Nwf : ex;

  float sy = mwp - 1.0f;
  sy = hw.dep * sy;
  sy = sy * Isync;
  sy = sy * Bf;
  sy = sy * repf;
  const float cost = __builtin_fmaf(ex, repf, sy);                 // exec rep + sync
  ok = ok & (fabsf(cost) <= 3.402823466e38f);
  return ok ? cost : INFINITY;
}

// Cost of one (query, configuration) point; +inf where inadmissible.  DEG: the program's highest
// power of N~ (Horner from there; the normative sequence starts at power 3 with zero
// coefficients above DEG, which gives bit-identical values because fma(0, x, a) = a exactly for
// finite x and a != -0, and collapsed coefficients are sums that start from +0).
// UNI: cf and r are the same in every lane (the coefficients then sit in scalar registers); a
// per-lane configuration takes plain vector loads.  SHORT (the configuration record's `fast`):
// 1 - every metric's numerator and denominator stay in [2^-40, 2^40] (denominators positive)
// over the program's queries, so each metric quotient takes div_moderate (the same bits as the
// IEEE division), every metric is defined and finite and nonzero, and the clamps reduce to
// maxima; 2 - the four quotients of the cycle estimate take div_moderate as well.
template <int GRID, int DEG = kNdeg, bool UNI = true, int SHORT = 0>
__device__ __forceinline__ float point_cost(int32_t N, const float* xs, const float* __restrict__ cf,
                                            const CfgRec& r, const Hw32& hw) {
#pragma clang fp contract(off)
  static_assert(DEG >= 1 && DEG <= kNdeg, "Horner degree");
  bool ok = (r.ok != 0) & (N >= r.Lmax);
  float g[KLR_N_METRICS];
  bool good[KLR_N_METRICS];
#pragma unroll
  for (int j = 0; j < KLR_N_METRICS; ++j) {
    const float* c = cf + j * 2 * (kNdeg + 1);     // c[2 d] numerator, c[2 d + 1] denominator
    const float x = xs[j];
    // First Horner step: both addends enter vector registers through one 64-bit move (the
    // wave-uniform coefficients sit in scalar registers, and a VALU instruction reads at most
    // one of them).
    const float2 lo = UNI ? vgpr_pair(c + 2 * (DEG - 1)) : make_float2(c[2 * (DEG - 1)], c[2 * DEG - 1]);
    float p = __builtin_fmaf(c[2 * DEG], x, lo.x);
    float q = __builtin_fmaf(c[2 * DEG + 1], x, lo.y);
#pragma unroll
    for (int d = DEG - 2; d >= 0; --d) {
      p = __builtin_fmaf(p, x, c[2 * d]);
      q = __builtin_fmaf(q, x, c[2 * d + 1]);
    }
    if (SHORT) {
      g[j] = div_moderate(p, q);
      good[j] = true;
    } else {
      g[j] = p / q;
      good[j] = (q > 0.0f) & (fabsf(g[j]) <= 3.402823466e38f);
      ok = ok & good[j];
    }
  }
  return cycle_cost<GRID, SHORT>(N, g, good, ok, r, hw);
}

// Costs of QPL points (one configuration slot, wave-uniform, all of whose metric quotients take
// the short form: SHORT = 1 or 2) by the same steps as point_cost: per metric the two
// coefficients that enter vector registers do so once for all QPL queries.
template <int QPL, int GRID, int DEG, int SHORT>
__device__ __forceinline__ void point_costs_short(const int32_t* N, const float (*xs)[KLR_N_METRICS],
                                                  const float* __restrict__ cf, const CfgRec& r, const Hw32& hw,
                                                  float* cost) {
#pragma clang fp contract(off)
  static_assert(DEG >= 1 && DEG <= kNdeg && SHORT >= 1, "short metrics");
  float g[QPL][KLR_N_METRICS];
#pragma unroll
  for (int j = 0; j < KLR_N_METRICS; ++j) {
    const float* c = cf + j * 2 * (kNdeg + 1);
    const float2 lo = vgpr_pair(c + 2 * (DEG - 1));
#pragma unroll
    for (int u = 0; u < QPL; ++u) {
      const float x = xs[u][j];
      float p = __builtin_fmaf(c[2 * DEG], x, lo.x);
      float q = __builtin_fmaf(c[2 * DEG + 1], x, lo.y);
#pragma unroll
      for (int d = DEG - 2; d >= 0; --d) {
        p = __builtin_fmaf(p, x, c[2 * d]);
        q = __builtin_fmaf(q, x, c[2 * d + 1]);
      }
      g[u][j] = div_moderate(p, q);
    }
  }
  const bool good[KLR_N_METRICS] = {true, true, true, true, true, true, true, true};
#pragma unroll
  for (int u = 0; u < QPL; ++u)
    cost[u] = cycle_cost<GRID, SHORT>(N[u], g[u], good, (r.ok != 0) & (N[u] >= r.Lmax), r, hw);
}

// Cost of one point of a program whose one fitted function is the cost: p/q of metric 0 by the
// same Horner steps and division as the cycle estimate's metrics; +inf where q <= 0, the value is
// not finite, a launch parameter exceeds N or the configuration is not admissible.
template <int DEG = kNdeg, bool UNI = true>
__device__ __forceinline__ float metric_cost(int32_t N, const float* xs, const float* __restrict__ cf,
                                             const CfgRec& r) {
  bool good;
  const float g = fitted_value<DEG, UNI>(cf, 0, xs[0], &good);
  const bool ok = (r.ok != 0) & (N >= r.Lmax) & good;
  return ok ? g : INFINITY;
}

// A piecewise rational program with a fitted decision node (paper: the decision nodes of a
// rational program are themselves rational functions, so they can be fitted like the metrics):
// fits 0, 1, 2 are the decision d, the cost where d >= 0 and the cost where d < 0.  The point
// is inadmissible where d or the branch taken is (q <= 0 or not finite), or where the launch
// constraints fail.
template <int DEG = kNdeg, bool UNI = true>
__device__ __forceinline__ float piecewise_cost(int32_t N, const float* xs, const float* __restrict__ cf,
                                                const CfgRec& r) {
  bool gd, ga, gb;
  const float d = fitted_value<DEG, UNI>(cf, 0, xs[0], &gd);
  const float a = fitted_value<DEG, UNI>(cf, 1, xs[1], &ga);
  const float b = fitted_value<DEG, UNI>(cf, 2, xs[2], &gb);
  const bool first = d >= 0.0f;
  const bool ok = (r.ok != 0) & (N >= r.Lmax) & gd & (first ? ga : gb);
  return ok ? (first ? a : b) : INFINITY;
}

// Any cost, chosen per program (wave-uniform).
template <int GRID, int DEG = kNdeg, bool UNI = true>
__device__ __forceinline__ float any_cost(int kind, int32_t N, const float* xs, const float* __restrict__ cf,
                                          const CfgRec& r, const Hw32& hw) {
  if (kind == KLR_COST_METRIC) return metric_cost<DEG, UNI>(N, xs, cf, r);
  if (kind == KLR_COST_PIECEWISE) return piecewise_cost<DEG, UNI>(N, xs, cf, r);
  return point_cost<GRID, DEG, UNI>(N, xs, cf, r, hw);
}

}  // namespace klr

// Rational-program evaluation over launch configurations + per-query argmin, gfx950.
//
// Paper: steps 4 ("Rational program evaluation") and 5 ("Selection of optimal values of
// program parameters") of the section "An Algorithm to Build and Deploy a
// Performance-Predicting Rational Program"; occupancy by the flowchart of Example "Hardware
// occupancy" and eq. (occupancy); execution time by an MWP-CWP-style estimate (Example
// "execution time" names the model without its equations; the operation sequence below is
// this library's normative definition).
//
// Two kernels:
//   collapse  - one thread per (program, configuration): validates the descriptors, fixes the
//               launch parameters in each metric's p and q (FP64, monomial order), rounds the
//               resulting polynomials in N~ to FP32, and precomputes the configuration's
//               integer occupancy terms.
//   eval      - one lane per query, looping over the program's configurations in index order;
//               the configuration's coefficients are wave-uniform (scalar loads), so each lane
//               keeps its own running (cost, index) minimum with a strict "<" and no cross-lane
//               reduction is needed.  All decisions are taken in FP32 with the exact operation
//               order: fused multiply-adds exactly where written (the Horner steps and the
//               a b + c terms of the cycle estimate), every other operation rounded on its own
//               (no contraction: this file is compiled with -ffp-contract=off), correctly
//               rounded division and compare-select min/max, so a CPU replay reproduces every
//               cost and index bit for bit.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "eval_point.hpp"
#include "internal.hpp"

namespace klr {
namespace {

constexpr int kEvalBlock = 256;
constexpr int kCollapseBlock = 128;

// Division by an invariant divisor d in [1, 2^31): with l = ceil(log2 d) and
// m = ceil(2^(31 + l) / d) (fits 32 bits), floor(n / d) = floor(n m / 2^(31 + l)) for every
// 0 <= n < 2^31, because n (m d - 2^(31 + l)) / (d 2^(31 + l)) < 1/d (round-up method of
// Granlund and Montgomery).  sh = l - 1; d = 1 is marked by sh = -1.
__host__ __device__ inline void magic_u31(uint32_t d, uint32_t* m, int32_t* sh) {
  int l = 0;
  while (l < 31 && (1u << l) < d) ++l;
  if (l == 0) { *m = 0u; *sh = -1; return; }
  const uint64_t p = (uint64_t)1 << (31 + l);
  *m = (uint32_t)((p + d - 1) / d);
  *sh = l - 1;
}

// The same for a divisor d >= 1 of up to 64 bits: every d >= 2^31 gives the quotient 0 for
// 0 <= n < 2^31, which m = 0, sh = 0 encode.
__host__ __device__ inline void magic_u31_wide(uint64_t d, uint32_t* m, int32_t* sh) {
  if (d >= ((uint64_t)1 << 31)) { *m = 0u; *sh = 0; return; }
  magic_u31((uint32_t)d, m, sh);
}




// Per-program highest power of N~, stored after the configuration records, then each program's
// smallest and largest query size.
__host__ __device__ inline int32_t* prog_degree(const EvalArgs& a) {
  char* base = reinterpret_cast<char*>(a.ws);
  const int64_t slots = (int64_t)a.n_progs * a.max_cfg;
  return reinterpret_cast<int32_t*>(base + slots * (kSlotFloats * (int64_t)sizeof(float) + (int64_t)sizeof(CfgRec)));
}
__host__ __device__ inline int32_t* prog_nrange(const EvalArgs& a) { return prog_degree(a) + a.n_progs; }

// Enclosure of every FP32 Horner value (fused multiply-adds from power 3, c[2 d] the coefficient
// of power d) at FP32 points x in [xl, xh]: interval Horner in FP64 over the exact coefficients,
// widened by 2^-20 sum |c_d| max|x|^d, above the FP32 Horner error bound 3 u sum |c_d| |x|^d
// (u = 2^-24) and the FP64 rounding of the interval steps.  Returns false when a partial value
// could leave the FP32 range.
__device__ inline bool horner_enclosure(const float* c, double xl, double xh, double* lo, double* hi) {
  const double xm = fmax(fabs(xl), fabs(xh));
  double pl = c[2 * kNdeg], ph = pl, sa = fabs(pl);
  bool fin = sa <= 0x1p100;
  for (int d = kNdeg - 1; d >= 0; --d) {
    const double a0 = pl * xl, a1 = pl * xh, a2 = ph * xl, a3 = ph * xh;
    const double cd = c[2 * d];
    pl = fmin(fmin(a0, a1), fmin(a2, a3)) + cd;
    ph = fmax(fmax(a0, a1), fmax(a2, a3)) + cd;
    sa = sa * xm + fabs(cd);
    fin = fin && sa <= 0x1p100;
  }
  const double E = sa * 0x1p-20;
  *lo = pl - E;
  *hi = ph + E;
  return fin && xm <= 0x1p100;
}

// Fitted metrics a program reads: the eight of the cycle estimate, or its one cost function.
__host__ __device__ inline int program_metrics(const klr_program& P) {
  return P.cost_kind == KLR_COST_METRIC ? 1 : (P.cost_kind == KLR_COST_PIECEWISE ? 3 : KLR_N_METRICS);
}

__device__ bool program_desc_ok(const klr_program& P, const EvalArgs& a) {
  if (P.cost_kind != KLR_COST_CYCLES && P.cost_kind != KLR_COST_METRIC && P.cost_kind != KLR_COST_PIECEWISE)
    return false;
  if (P.fit0 < 0 || (int64_t)P.fit0 + program_metrics(P) > a.n_fits) return false;
  if (P.v_launch < 1 || P.v_launch > KLR_MAX_LAUNCH) return false;
  if (P.n_cfg < 0 || P.n_cfg > a.max_cfg || P.n_q < 0 || P.n_q > a.max_q) return false;
  if (P.cfg0 < 0 || P.cfg0 + (int64_t)P.n_cfg * P.v_launch > a.cfgs_len) return false;
  if (P.q0 < 0 || P.q0 + (int64_t)P.n_q > a.q_len) return false;
  if (P.grid_kind != KLR_GRID_1D && P.grid_kind != KLR_GRID_2D) return false;
  if (P.grid_kind == KLR_GRID_2D && P.v_launch < 2) return false;
  if (a.all_costs && (P.cost0 < 0 || P.cost0 + (int64_t)P.n_cfg * P.n_q > a.costs_len)) return false;
  return true;
}

__device__ bool fit_desc_ok(const klr_fit_desc& d, int v_expected, const EvalArgs& a) {
  if (d.v != v_expected) return false;
  if (d.n_num < 0 || d.n_den < 1) return false;
  if (d.num0 < 0 || (int64_t)d.num0 + d.n_num > a.n_exp_rows) return false;
  if (d.den0 < 0 || (int64_t)d.den0 + d.n_den > a.n_exp_rows) return false;
  if (d.coef0 < 0 || d.coef0 + (int64_t)d.n_num + d.n_den - 1 > a.coef_len) return false;
  for (int k = 0; k < d.v; ++k)
    if (d.scale_exp[k] < -100 || d.scale_exp[k] > 100) return false;
  const uint8_t* r0 = a.exps + (int64_t)d.den0 * KLR_MAX_VARS;
  for (int k = 0; k < d.v; ++k)
    if (r0[k] != 0) return false;
  return true;
}

// Polynomial in N~ of one metric polynomial at fixed launch parameters.  FP64, monomials in set
// order, each monomial value by repeated multiplication in variable order.  `rows` points at
// the polynomial's exponent rows (8 bytes each), `coef` at its coefficients (the denominator's
// constant 1 is implicit).  Every exponent of N~ has been checked to be <= kNdeg.
__device__ __forceinline__ uint64_t exp_row(const uint8_t* exps, int64_t row) {
  const uint8_t* e = exps + row * KLR_MAX_VARS;
  if ((reinterpret_cast<uintptr_t>(e) & 7u) == 0) return *reinterpret_cast<const uint64_t*>(e);
  uint64_t w = 0;
  for (int k = 0; k < KLR_MAX_VARS; ++k) w |= (uint64_t)e[k] << (8 * k);
  return w;
}

template <bool STAGED>
__device__ __forceinline__ void collapse_poly(const uint64_t* srows, const uint8_t* exps, int64_t row0, int nrows,
                                              int v, const double* Lt, const double* coef, bool den,
                                              double out[kNdeg + 1]) {
  double o[kNdeg + 1] = {0.0, 0.0, 0.0, 0.0};
  static_assert(kNdeg == 3, "four powers of N~");
  // rows in groups of 4: the group's exponent words and coefficients are loaded first; each row
  // is the same for every thread, so its exponents go to scalar registers
  for (int t0 = 0; t0 < nrows; t0 += 4) {
    uint64_t w[4];
    double cf[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + u < nrows ? t0 + u : nrows - 1;
      w[u] = STAGED ? srows[t] : exp_row(exps, row0 + t);
      cf[u] = den ? (t == 0 ? 1.0 : coef[t > 0 ? t - 1 : 0]) : coef[t];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (t0 + u < nrows) {
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)w[u]);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(w[u] >> 32));
        double mono = 1.0;
#pragma unroll
        for (int k = 1; k <= KLR_MAX_LAUNCH; ++k) {
          if (k < v) {
            const int ek = (int)(((k < 4 ? lo >> (8 * k) : hi >> (8 * (k - 4)))) & 0xFFu);
            for (int r = 0; r < ek; ++r) mono = mono * Lt[k - 1];
          }
        }
        const double term = cf[u] * mono;
        switch (lo & 0xFFu) {
          case 0: o[0] = o[0] + term; break;
          case 1: o[1] = o[1] + term; break;
          case 2: o[2] = o[2] + term; break;
          default: o[3] = o[3] + term; break;
        }
      }
    }
  }
  for (int e = 0; e <= kNdeg; ++e) out[e] = o[e];
}

// Smallest and largest query size of each program (one workgroup per program); a program
// without queries gets an empty range (lo > hi).
constexpr int kRangeBlock = 256;
__global__ void __launch_bounds__(kRangeBlock) query_range_kernel(EvalArgs a) {
  __shared__ int32_t s_lo[kRangeBlock / 64], s_hi[kRangeBlock / 64];
  const int p = blockIdx.x;
  const klr_program P = a.progs[p];
  int32_t lo = 0x7fffffff, hi = (int32_t)0x80000000;
  if (program_desc_ok(P, a))
#pragma unroll 8
    for (int i = threadIdx.x; i < P.n_q; i += kRangeBlock) {     // eight loads in flight
      const int32_t N = a.queries[P.q0 + i];
      lo = N < lo ? N : lo;
      hi = N > hi ? N : hi;
    }
  for (int off = 32; off >= 1; off >>= 1) {
    const int32_t ol = __shfl_xor(lo, off), oh = __shfl_xor(hi, off);
    lo = ol < lo ? ol : lo;
    hi = oh > hi ? oh : hi;
  }
  if ((threadIdx.x & 63) == 0) { s_lo[threadIdx.x >> 6] = lo; s_hi[threadIdx.x >> 6] = hi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kRangeBlock / 64; ++w) {
      lo = s_lo[w] < lo ? s_lo[w] : lo;
      hi = s_hi[w] > hi ? s_hi[w] : hi;
    }
    prog_nrange(a)[2 * p] = lo;
    prog_nrange(a)[2 * p + 1] = hi;
  }
}

// Enclosures of nonnegative FP32 results: each FP32 step below rounds once, so widening the
// exact-arithmetic bounds by 2^-22 per step (relative) keeps every FP32 value inside.
struct Ival { double lo, hi; };
__device__ inline Ival iv_round(Ival a) { return Ival{a.lo * (1.0 - 0x1p-22), a.hi * (1.0 + 0x1p-22)}; }
__device__ inline Ival iv_add(Ival a, Ival b) { return iv_round(Ival{a.lo + b.lo, a.hi + b.hi}); }
__device__ inline Ival iv_mul(Ival a, Ival b) { return iv_round(Ival{a.lo * b.lo, a.hi * b.hi}); }
__device__ inline Ival iv_max(Ival a, double c) { return Ival{fmax(a.lo, c), fmax(a.hi, c)}; }
__device__ inline bool iv_moderate(Ival a) { return a.lo >= 0x1p-40 && a.hi <= 0x1p40; }

// Which quotients of a configuration slot can take the short division at every query of the
// program (0: none; 1: the eight metric quotients; 2: those and the four of the cycle
// estimate).  Over the program's range of scaled sizes every metric numerator and denominator
// must stay in [2^-40, 2^40] in magnitude with positive denominators (so every metric is also
// defined there, as the exact sweep would find); then the clamped metric values are enclosed
// and carried through the cycle estimate's sums and products (all nonnegative), and the
// operands of its quotients must stay in [2^-40, 2^40] as well.
__device__ inline int slot_divides_short(const float* out, int32_t n_lo, int32_t n_hi, const klr_hw& hw) {
  if (n_lo > n_hi) return 0;
  const double xn_lo = (double)(float)n_lo, xn_hi = (double)(float)n_hi;
  Ival g[KLR_N_METRICS];
  for (int j = 0; j < KLR_N_METRICS; ++j) {
    const double sc = out[KLR_N_METRICS * 2 * (kNdeg + 1) + j];     // a power of two
    const double xl = xn_lo * sc, xh = xn_hi * sc;
    double pl, ph, ql, qh;
    if (!horner_enclosure(out + j * 2 * (kNdeg + 1), xl, xh, &pl, &ph)) return 0;
    if (!horner_enclosure(out + j * 2 * (kNdeg + 1) + 1, xl, xh, &ql, &qh)) return 0;
    if (!(ql >= 0x1p-40 && qh <= 0x1p40)) return 0;
    if (!(pl >= -0x1p40 && ph <= 0x1p40 && (pl >= 0x1p-40 || ph <= -0x1p-40))) return 0;
    // p / q over the box, then the quotient's own rounding
    const double a = pl / ql, b = pl / qh, c = ph / ql, d = ph / qh;
    const double lo = fmin(fmin(a, b), fmin(c, d)), hi = fmax(fmax(a, b), fmax(c, d));
    g[j] = Ival{lo - fabs(lo) * 0x1p-22, hi + fabs(hi) * 0x1p-22};
  }
  if (!(hw.mem_lat > 0.0f && hw.dep_delay > 0.0f && hw.issue_cycles > 0.0f && hw.bw > 0.0f && hw.w_max >= 1 &&
        hw.mem_lat <= 0x1p40f && hw.dep_delay <= 0x1p40f && hw.issue_cycles <= 0x1p40f && hw.bw <= 0x1p40f))
    return 1;
  const Ival Icomp = iv_max(g[0], 0.0), Imc = iv_max(g[1], 0.0), Imu = iv_max(g[2], 0.0);
  const Ival U = iv_max(g[3], 1.0), Bw = iv_max(g[7], 1.0);
  const Ival lat{hw.mem_lat, hw.mem_lat}, dep{hw.dep_delay, hw.dep_delay};
  const Ival iss{hw.issue_cycles, hw.issue_cycles}, bw{hw.bw, hw.bw};
  const Ival Nw{1.0, (double)hw.w_max};
  const Ival Im = iv_add(Imc, Imu);
  const Ival Lu = iv_round(Ival{(U.lo - 1.0) * dep.lo + lat.lo, (U.hi - 1.0) * dep.hi + lat.hi});
  const Ival mem = iv_add(iv_mul(Lu, Imu), iv_mul(lat, Imc));
  const Ival comp = iv_mul(iss, iv_add(Icomp, Im));
  const Ival d1 = iv_mul(dep, iv_add(iv_mul(U, Imu), Imc));
  const Ival n2 = iv_mul(bw, mem), d2 = iv_mul(Im, Bw), t2 = iv_mul(mem, Nw);
  const bool cyc = iv_moderate(mem) && iv_moderate(d1) && iv_moderate(n2) && iv_moderate(d2) &&
                   iv_moderate(comp) && iv_moderate(Im) && iv_moderate(t2) && hw.w_max <= (1 << 11);
  return cyc ? 2 : 1;
}

// One workgroup per (program, block of configurations).  The program's eight fit descriptors
// are validated once per workgroup, and their exponent rows and coefficients are staged in LDS
// when they fit (every thread then reads the same LDS rows); one thread per configuration
// computes its record and the collapsed coefficients of the eight metrics.
constexpr int kCollapseCapRows = KLR_N_METRICS * (KLR_MAX_UNKNOWNS + 1);
__global__ void __launch_bounds__(kCollapseBlock)
collapse_kernel(EvalArgs a, int chunks) {
  __shared__ uint64_t s_rows[kCollapseCapRows];       // exponent rows, numerator then denominator
  __shared__ double s_coef[kCollapseCapRows];
  __shared__ klr_fit_desc s_desc[KLR_N_METRICS];
  __shared__ int s_off[KLR_N_METRICS + 1];
  __shared__ int s_bad, s_deg, s_staged;
  const int p = blockIdx.x / chunks;
  const int c = (blockIdx.x % chunks) * kCollapseBlock + threadIdx.x;
  if (p >= a.n_progs) return;
  const klr_program P = a.progs[p];
  const bool pd_ok = program_desc_ok(P, a);
  const int v = 1 + (pd_ok ? P.v_launch : 0);
  const int nmet = program_metrics(P);
  if (threadIdx.x == 0) { s_bad = 0; s_deg = 0; }
  __syncthreads();
  if (pd_ok && (int)threadIdx.x < nmet) {
    const klr_fit_desc d = a.desc[P.fit0 + threadIdx.x];
    s_desc[threadIdx.x] = d;
    if (!fit_desc_ok(d, v, a)) atomicOr(&s_bad, 1);
  }
  __syncthreads();
  bool fits_ok = pd_ok && s_bad == 0;
  if (threadIdx.x == 0 && fits_ok) {
    int off = 0;
    for (int j = 0; j < nmet; ++j) {
      s_off[j] = off;
      off += s_desc[j].n_num + s_desc[j].n_den;
    }
    s_off[nmet] = off;
    s_staged = off <= kCollapseCapRows;
  }
  __syncthreads();
  // one pass over the exponent rows: powers of N~ checked, the highest one found, rows and
  // coefficients staged in LDS when they fit
  const bool stage = fits_ok && s_staged;
  if (fits_ok) {
    int emax = 0;
    for (int j = 0; j < nmet; ++j) {
      const klr_fit_desc& d = s_desc[j];
      const int nr = d.n_num + d.n_den;
      for (int t = threadIdx.x; t < nr; t += kCollapseBlock) {
        const int64_t row = t < d.n_num ? (int64_t)d.num0 + t : (int64_t)d.den0 + (t - d.n_num);
        const uint64_t w = exp_row(a.exps, row);
        const int e0 = (int)(w & 0xFFu);
        emax = e0 > emax ? e0 : emax;
        if (stage) {
          s_rows[s_off[j] + t] = w;
          if (t < nr - 1) s_coef[s_off[j] + t] = a.coef[d.coef0 + t];
        }
      }
    }
    if (emax > kNdeg) atomicOr(&s_bad, 1);
    if (emax > 0) atomicMax(&s_deg, emax);
  }
  __syncthreads();
  fits_ok = fits_ok && s_bad == 0;
  const bool staged = fits_ok && stage;
  if (c == 0 && a.prog_status)
    a.prog_status[p] = (pd_ok ? 0 : KLR_PROG_BAD_DESC) | (pd_ok && !fits_ok ? KLR_PROG_BAD_FIT : 0);
  if (c == 0) {   // highest power of N~ over the program's metric polynomials (Horner start)
    const int deg = fits_ok ? s_deg : 0;
    prog_degree(a)[p] = deg > kNdeg ? kNdeg : deg;
  }
  if (!pd_ok || c >= P.n_cfg || c >= a.max_cfg) return;

  const int64_t slot = (int64_t)p * a.max_cfg + c;
  float* out = reinterpret_cast<float*>(a.ws) + slot * kSlotFloats;
  CfgRec* rec = reinterpret_cast<CfgRec*>(reinterpret_cast<char*>(a.ws) +
                                          (int64_t)a.n_progs * a.max_cfg * kSlotFloats * sizeof(float)) + slot;

  int32_t L[KLR_MAX_LAUNCH] = {1, 1, 1, 1};
  bool cfg_ok = true;
  int64_t T = 1;
  int32_t Lmax = 1;
#pragma unroll
  for (int k = 0; k < KLR_MAX_LAUNCH; ++k) {
    if (k < P.v_launch) {
      L[k] = a.cfgs[P.cfg0 + (int64_t)c * P.v_launch + k];
      if (L[k] < 1) cfg_ok = false;
      if (L[k] > Lmax) Lmax = L[k];
      if (cfg_ok) { T *= L[k]; if (T > (int64_t)a.hw.t_max) cfg_ok = false; }
    }
  }
  if (cfg_ok && (T % a.hw.wave) != 0) cfg_ok = false;
  CfgRec r;
  r.T = cfg_ok ? (int32_t)T : a.hw.wave;
  const int32_t bwarp = (a.hw.wave * a.hw.w_max) / r.T;
  r.Wb = (float)(r.T / a.hw.wave);
  r.Bcap = (float)(a.hw.b_max < bwarp ? a.hw.b_max : bwarp);
  r.rTh = (float)(a.hw.r_max / r.T) + 0.5f;
  r.Lmax = Lmax;
  r.L0 = L[0] < 1 ? 1 : L[0];
  r.L1 = L[1] < 1 ? 1 : L[1];
  r.ok = (cfg_ok && fits_ok) ? 1 : 0;
  magic_u31_wide((uint64_t)r.T * (uint64_t)a.hw.n_cu, &r.magTC, &r.shTC);
  r.fast = 0;
  r.pad = 0;

  for (int j = 0; j < KLR_N_METRICS; ++j) {
    double num[kNdeg + 1] = {0, 0, 0, 0}, den[kNdeg + 1] = {1, 0, 0, 0};
    float sc = 1.0f;
    if (fits_ok && j < nmet) {         // a metric-cost program leaves the other slots 0 / 1
      const klr_fit_desc& d = s_desc[j];
      double Lt[KLR_MAX_LAUNCH];
#pragma unroll
      for (int k = 1; k <= KLR_MAX_LAUNCH; ++k)
        Lt[k - 1] = k < v ? ldexp((double)L[k - 1], -(int)d.scale_exp[k]) : 1.0;
      if (staged) {
        const uint64_t* rows = s_rows + s_off[j];
        collapse_poly<true>(rows, nullptr, 0, d.n_num, v, Lt, s_coef + s_off[j], false, num);
        collapse_poly<true>(rows + d.n_num, nullptr, 0, d.n_den, v, Lt, s_coef + s_off[j] + d.n_num, true, den);
      } else {
        collapse_poly<false>(nullptr, a.exps, d.num0, d.n_num, v, Lt, a.coef + d.coef0, false, num);
        collapse_poly<false>(nullptr, a.exps, d.den0, d.n_den, v, Lt, a.coef + d.coef0 + d.n_num, true, den);
      }
      sc = ldexpf(1.0f, -(int)d.scale_exp[0]);
    }
    for (int e = 0; e <= kNdeg; ++e) {        // (numerator, denominator) pairs by power
      out[j * 2 * (kNdeg + 1) + 2 * e] = (float)num[e];
      out[j * 2 * (kNdeg + 1) + 2 * e + 1] = (float)den[e];
    }
    out[KLR_N_METRICS * 2 * (kNdeg + 1) + j] = sc;
  }
  if (r.ok && P.cost_kind == KLR_COST_CYCLES)
    r.fast = slot_divides_short(out, prog_nrange(a)[2 * p], prog_nrange(a)[2 * p + 1], a.hw);
  *rec = r;
}

struct SweepOut {
  int32_t* __restrict__ argmin;
  float* __restrict__ best_cost;
  float* __restrict__ all_costs;
};

// One lane per query; all control flow is wave-uniform (lanes without a query compute a
// clamped one and skip only the stores), so the per-configuration terms are scalar loads.
template <int GRID>
__device__ __forceinline__ void sweep(const float* __restrict__ slot0, const CfgRec* __restrict__ rec0,
                                      const int32_t* __restrict__ queries, const SweepOut& o,
                                      const Hw32& hw, const klr_program& P, int qi, bool live) {
  const int32_t N = queries[P.q0 + qi];
  float best = INFINITY;
  int32_t bi = -1;
  float* costs = o.all_costs ? o.all_costs + P.cost0 + qi : nullptr;
  float xs[KLR_N_METRICS];
  if (P.n_cfg > 0) scaled_n(N, slot0, xs);
  for (int c = 0; c < P.n_cfg; ++c) {
    const CfgRec r = rec0[c];
    const float cost = any_cost<GRID>(P.cost_kind, N, xs, slot0 + (int64_t)c * kSlotFloats, r, hw);
    if (costs && live) costs[(int64_t)c * P.n_q] = cost;
    if (cost < best) { best = cost; bi = c; }
  }
  if (live) {
    o.argmin[P.q0 + qi] = bi;
    o.best_cost[P.q0 + qi] = best;
  }
}

template <int QPL, int GRID, int DEG, int KIND = KLR_COST_CYCLES>
__device__ __forceinline__ void sweep_cfgs(const klr_program& P, const float* __restrict__ slot0,
                                           const CfgRec* __restrict__ rec0, const Hw32& hw,
                                           const int32_t* N, const bool* live, const int* qi,
                                           float* costs, float* best, int32_t* bi) {
  if (P.n_cfg <= 0) return;
  float xs[QPL][KLR_N_METRICS];
#pragma unroll
  for (int u = 0; u < QPL; ++u) scaled_n(N[u], slot0, xs[u]);
  for (int c = 0; c < P.n_cfg; ++c) {
    const CfgRec r = rec0[c];
    const float* cf = slot0 + (int64_t)c * kSlotFloats;
    if (KIND == KLR_COST_CYCLES && r.fast >= 1) {     // wave-uniform
      float cost[QPL];
      if (r.fast == 2)
        point_costs_short<QPL, GRID, DEG, 2>(N, xs, cf, r, hw, cost);
      else
        point_costs_short<QPL, GRID, DEG, 1>(N, xs, cf, r, hw, cost);
#pragma unroll
      for (int u = 0; u < QPL; ++u) {
        if (costs && live[u]) costs[(int64_t)c * P.n_q + qi[u]] = cost[u];
        if (cost[u] < best[u]) { best[u] = cost[u]; bi[u] = c; }
      }
      continue;
    }
#pragma unroll
    for (int u = 0; u < QPL; ++u) {
      const float cost = KIND == KLR_COST_METRIC      ? metric_cost<DEG>(N[u], xs[u], cf, r)
                         : KIND == KLR_COST_PIECEWISE ? piecewise_cost<DEG>(N[u], xs[u], cf, r)
                                                      : point_cost<GRID, DEG>(N[u], xs[u], cf, r, hw);
      if (costs && live[u]) costs[(int64_t)c * P.n_q + qi[u]] = cost;
      if (cost < best[u]) { best[u] = cost; bi[u] = c; }
    }
  }
}

// QPL queries per lane, BLOCK lanes per workgroup: each lane carries QPL independent
// (query, running minimum) chains through the same configuration loop.  The sweep is bound by
// instruction issue, and an extra wave per SIMD hides more of its dependent latencies: the
// two-query shapes are held to 80 VGPRs (six waves; 85 unconstrained, five), the four-query
// shape to 128 (four waves; 135 unconstrained, three).
template <int QPL, int BLOCK>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(QPL == 2 ? 6 : (QPL == 4 ? 4 : 1))))
eval_kernel(const klr_program* __restrict__ progs, const float* __restrict__ coefs,
            const CfgRec* __restrict__ recs, const int32_t* __restrict__ queries,
            int32_t* __restrict__ argmin, float* __restrict__ best_cost,
            float* __restrict__ all_costs, EvalArgs a, Hw32 hw, int chunks) {
  // workgroup b runs on XCD b mod 8 (the dispatcher deals workgroups to the eight XCDs in
  // turn): program p's chunks take the workgroups of XCD p mod 8, so one L2 holds its slots
  const int xcd = (int)(blockIdx.x & 7u), j = (int)(blockIdx.x >> 3);
  const int p = xcd + 8 * (j / chunks);
  const int qb = (j % chunks) * BLOCK * QPL;
  if (p >= a.n_progs) return;
  const klr_program P = progs[p];
  if (!program_desc_ok(P, a) || qb >= P.n_q) return;
  const float* slot0 = coefs + (int64_t)p * a.max_cfg * kSlotFloats;
  const CfgRec* rec0 = recs + (int64_t)p * a.max_cfg;
  int32_t N[QPL];
  bool live[QPL];
  int qi[QPL];
#pragma unroll
  for (int u = 0; u < QPL; ++u) {
    qi[u] = qb + u * BLOCK + (int)threadIdx.x;
    live[u] = qi[u] < P.n_q;
    qi[u] = live[u] ? qi[u] : P.n_q - 1;
    N[u] = queries[P.q0 + qi[u]];
  }
  float best[QPL];
  int32_t bi[QPL];
#pragma unroll
  for (int u = 0; u < QPL; ++u) { best[u] = INFINITY; bi[u] = -1; }
  float* costs = all_costs ? all_costs + P.cost0 : nullptr;
  const int deg = prog_degree(a)[p];
  if (P.cost_kind == KLR_COST_METRIC)
    sweep_cfgs<QPL, KLR_GRID_1D, kNdeg, KLR_COST_METRIC>(P, slot0, rec0, hw, N, live, qi, costs, best, bi);
  else if (P.cost_kind == KLR_COST_PIECEWISE)
    sweep_cfgs<QPL, KLR_GRID_1D, kNdeg, KLR_COST_PIECEWISE>(P, slot0, rec0, hw, N, live, qi, costs, best, bi);
  else if (P.grid_kind == KLR_GRID_1D && deg <= 2)
    sweep_cfgs<QPL, KLR_GRID_1D, 2>(P, slot0, rec0, hw, N, live, qi, costs, best, bi);
  else if (P.grid_kind == KLR_GRID_1D)
    sweep_cfgs<QPL, KLR_GRID_1D, kNdeg>(P, slot0, rec0, hw, N, live, qi, costs, best, bi);
  else
    sweep_cfgs<QPL, KLR_GRID_2D, kNdeg>(P, slot0, rec0, hw, N, live, qi, costs, best, bi);
#pragma unroll
  for (int u = 0; u < QPL; ++u)
    if (live[u]) {
      argmin[P.q0 + qi[u]] = bi[u];
      best_cost[P.q0 + qi[u]] = best[u];
    }
}

struct EvalVariant { int qpl, block; };
constexpr EvalVariant kVariants[] = {{1, 256}, {2, 256}, {1, 128}, {2, 128}, {1, 64}, {4, 64}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

template <int QPL, int BLOCK>
hipError_t launch_variant(const EvalArgs& a, const Hw32& hw, const float* coefs, const CfgRec* recs) {
  const int chunks = (a.max_q + BLOCK * QPL - 1) / (BLOCK * QPL);
  const unsigned groups = 8u * (unsigned)((a.n_progs + 7) / 8) * (unsigned)chunks;
  hipLaunchKernelGGL((eval_kernel<QPL, BLOCK>), dim3(groups), dim3(BLOCK), 0, a.stream,
                     a.progs, coefs, recs, a.queries, a.argmin, a.best_cost, a.all_costs, a, hw, chunks);
  return hipGetLastError();
}

hipError_t launch_sweep(int v, const EvalArgs& a, const Hw32& hw, const float* coefs, const CfgRec* recs) {
  switch (v) {
    case 1: return launch_variant<2, 256>(a, hw, coefs, recs);
    case 2: return launch_variant<1, 128>(a, hw, coefs, recs);
    case 3: return launch_variant<2, 128>(a, hw, coefs, recs);
    case 4: return launch_variant<1, 64>(a, hw, coefs, recs);
    case 5: return launch_variant<4, 64>(a, hw, coefs, recs);
    default: return launch_variant<1, 256>(a, hw, coefs, recs);
  }
}

// ---- exact re-evaluation of flagged queries --------------------------------------------------
// pick_check: one lane per query; a query the network answered (flag 0) is flagged when the
// exact cost of its pick is +inf (the network never sees inadmissible configurations in training,
// so its prediction for one carries no information).
__global__ void __launch_bounds__(kEvalBlock)
pick_check(EvalArgs a, Hw32 hw, const float* __restrict__ coefs, const CfgRec* __restrict__ recs,
           const int32_t* __restrict__ picks, uint8_t* flags, int chunks) {
  const int p = blockIdx.x / chunks;
  const int qi = (blockIdx.x % chunks) * kEvalBlock + (int)threadIdx.x;
  if (p >= a.n_progs) return;
  const klr_program P = a.progs[p];
  if (!program_desc_ok(P, a) || qi >= P.n_q || P.n_cfg <= 0) return;
  const int64_t o = P.q0 + qi;
  if (flags[o] != 0) return;
  const int c = picks[o];
  if (c < 0 || c >= P.n_cfg) { flags[o] = 1; return; }
  const float* slot0 = coefs + (int64_t)p * a.max_cfg * kSlotFloats;
  const int32_t N = a.queries[o];
  float xs[KLR_N_METRICS];
  scaled_n(N, slot0, xs);
  const float cost = P.grid_kind == KLR_GRID_1D
      ? any_cost<KLR_GRID_1D, kNdeg, false>(P.cost_kind, N, xs, slot0 + (int64_t)c * kSlotFloats, recs[(int64_t)p * a.max_cfg + c], hw)
      : any_cost<KLR_GRID_2D, kNdeg, false>(P.cost_kind, N, xs, slot0 + (int64_t)c * kSlotFloats, recs[(int64_t)p * a.max_cfg + c], hw);
  if (!(cost < INFINITY)) flags[o] = 1;
}

// fb_count: flagged queries per program; fb_scan: exclusive offsets of queries and of 256-query
// chunks; fb_compact: order-preserving list of flagged query indices per program; fb_exact: one
// workgroup per chunk, the exact sweep over the listed queries (all lanes of a workgroup belong
// to one program, so the configuration loop stays wave-uniform).
__global__ void __launch_bounds__(kEvalBlock)
fb_count(EvalArgs a, const uint8_t* __restrict__ flags, int32_t* cnt) {
  __shared__ int red[kEvalBlock / 64];
  const int p = blockIdx.x;
  const klr_program P = a.progs[p];
  int c = 0;
  if (program_desc_ok(P, a))
    for (int qi = threadIdx.x; qi < P.n_q; qi += kEvalBlock) c += flags[P.q0 + qi] != 0 ? 1 : 0;
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) cnt[p] = red[0] + red[1] + red[2] + red[3];
}

__global__ void fb_scan(int32_t n_progs, const int32_t* __restrict__ cnt, int32_t* off, int32_t* choff,
                        int32_t* total) {
  if (threadIdx.x != 0) return;
  int32_t o = 0, ch = 0;
  for (int p = 0; p < n_progs; ++p) {
    off[p] = o;
    choff[p] = ch;
    o += cnt[p];
    ch += (cnt[p] + kEvalBlock - 1) / kEvalBlock;
  }
  *total = ch;
}

__global__ void __launch_bounds__(kEvalBlock)
fb_compact(EvalArgs a, const uint8_t* __restrict__ flags, const int32_t* __restrict__ off, int32_t* list) {
  __shared__ int wsum[kEvalBlock / 64];
  const int p = blockIdx.x;
  const klr_program P = a.progs[p];
  if (!program_desc_ok(P, a)) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int running = off[p];
  for (int q0 = 0; q0 < P.n_q; q0 += kEvalBlock) {
    const int qi = q0 + (int)threadIdx.x;
    const bool f = qi < P.n_q && flags[P.q0 + qi] != 0;
    const unsigned long long m = __ballot(f);
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wv] = __popcll(m);
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wv; ++w) before += wsum[w];
    if (f) list[running + before + rank] = qi;
    running += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kEvalBlock)
fb_exact(const klr_program* __restrict__ progs, const float* __restrict__ coefs,
         const CfgRec* __restrict__ recs, const int32_t* __restrict__ queries,
         int32_t* __restrict__ argmin, float* __restrict__ best_cost, EvalArgs a, Hw32 hw,
         const int32_t* __restrict__ cnt, const int32_t* __restrict__ off,
         const int32_t* __restrict__ choff, const int32_t* __restrict__ total,
         const int32_t* __restrict__ list) {
  const int b = blockIdx.x;
  if (b >= *total) return;
  int lo = 0, hi = a.n_progs - 1;          // last p with choff[p] <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (choff[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const int p = lo;
  const klr_program P = progs[p];
  if (!program_desc_ok(P, a)) return;
  const int n = cnt[p];
  const int li = (b - choff[p]) * kEvalBlock + (int)threadIdx.x;
  const bool live = li < n;
  const int qi = list[off[p] + (live ? li : n - 1)];
  const float* slot0 = coefs + (int64_t)p * a.max_cfg * kSlotFloats;
  const CfgRec* rec0 = recs + (int64_t)p * a.max_cfg;
  const SweepOut o{argmin, best_cost, nullptr};
  if (P.grid_kind == KLR_GRID_1D)
    sweep<KLR_GRID_1D>(slot0, rec0, queries, o, hw, P, qi, live);
  else
    sweep<KLR_GRID_2D>(slot0, rec0, queries, o, hw, P, qi, live);
}

// ---- self-test of the short quotient ---------------------------------------------------------
// div_moderate against the correctly rounded division for every a mantissa in [1, 2) and the b
// mantissas [b_first, b_first + nb); the first thread of each b also checks that the reciprocal
// estimate of b 2^e is that of b times 2^-e, and that of -b 2^e its negation, for e in [-60, 60].
constexpr int kSdA = 4096;                        // a mantissas per thread
constexpr int kSdThreadsPerB = (1 << 23) / kSdA;  // 2048

__global__ void __launch_bounds__(256) short_div_check(uint32_t b_first, uint32_t nb, unsigned long long* bad) {
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (uint64_t)nb * kSdThreadsPerB) return;
  const uint32_t bm = b_first + (uint32_t)(g / kSdThreadsPerB);
  const uint32_t a0 = (uint32_t)(g % kSdThreadsPerB) * kSdA;
  const float b = __uint_as_float(0x3f800000u | bm);
  uint32_t n = 0;
  for (int i = 0; i < kSdA; ++i) {
    const float a = __uint_as_float(0x3f800000u | (a0 + (uint32_t)i));
    n += __float_as_uint(div_moderate(a, b)) != __float_as_uint(a / b) ? 1u : 0u;
  }
  if (g % kSdThreadsPerB == 0) {
    const float r = __builtin_amdgcn_rcpf(b);
    for (int e = -60; e <= 60; ++e) {
      const float x = __builtin_ldexpf(b, e);
      const uint32_t want = __float_as_uint(__builtin_ldexpf(r, -e));
      n += __float_as_uint(__builtin_amdgcn_rcpf(x)) != want ? 1u : 0u;
      n += __float_as_uint(__builtin_amdgcn_rcpf(-x)) != (want ^ 0x80000000u) ? 1u : 0u;
    }
  }
  if (n) atomicAdd(bad, (unsigned long long)n);
}

}  // namespace

size_t eval_workspace_bytes(int32_t n_progs, int32_t max_cfg) {
  if (n_progs <= 0) return 0;
  const size_t slots = (size_t)(n_progs > 0 ? n_progs : 0) * (size_t)(max_cfg > 0 ? max_cfg : 0);
  return slots * (kSlotFloats * sizeof(float) + sizeof(CfgRec)) + (size_t)(n_progs > 0 ? n_progs : 0) * 12 + 256;
}

hipError_t launch_collapse_only(const EvalArgs& a) {
  const int cchunks = a.max_cfg > 0 ? (a.max_cfg + kCollapseBlock - 1) / kCollapseBlock : 1;
  int t = a.timer ? a.timer->begin(KLR_K_COLLAPSE, a.stream) : -1;
  hipLaunchKernelGGL(query_range_kernel, dim3((unsigned)a.n_progs), dim3(kRangeBlock), 0, a.stream, a);
  hipLaunchKernelGGL(collapse_kernel, dim3((unsigned)a.n_progs * cchunks), dim3(kCollapseBlock), 0,
                     a.stream, a, cchunks);
  if (a.timer) a.timer->end(t, a.stream);
  return hipGetLastError();
}

// Counts, offsets, chunk offsets, the chunk total, then the compacted list: every program
// contributes at most n_q <= max_q flagged queries (counted over its own query range), so
// n_progs * max_q entries hold the list whatever the programs' query ranges.
size_t fallback_ws_bytes(int32_t n_progs, int32_t max_q) {
  const size_t np = (size_t)(n_progs > 0 ? n_progs : 0);
  return (3 * np + 64 + np * (size_t)(max_q > 0 ? max_q : 0)) * sizeof(int32_t);
}

hipError_t launch_fallback(const EvalArgs& a, uint8_t* flags, float* best_cost, void* fws) {
  int32_t* cnt = reinterpret_cast<int32_t*>(fws);
  int32_t* off = cnt + a.n_progs;
  int32_t* choff = off + a.n_progs;
  int32_t* total = choff + a.n_progs;
  int32_t* list = total + 64;
  int t = a.timer ? a.timer->begin(KLR_K_FALLBACK, a.stream) : -1;
  hipError_t e = hipSuccess;
  if (a.max_q > 0) {
    const Hw32 hw = make_hw32(a.hw);
    const float* coefs = reinterpret_cast<const float*>(a.ws);
    const CfgRec* recs = reinterpret_cast<const CfgRec*>(
        reinterpret_cast<const char*>(a.ws) + (int64_t)a.n_progs * a.max_cfg * kSlotFloats * sizeof(float));
    const int chunks = (a.max_q + kEvalBlock - 1) / kEvalBlock;
    hipLaunchKernelGGL(pick_check, dim3((unsigned)a.n_progs * chunks), dim3(kEvalBlock), 0, a.stream, a, hw,
                       coefs, recs, a.argmin, flags, chunks);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(fb_count, dim3((unsigned)a.n_progs), dim3(kEvalBlock), 0, a.stream, a, flags, cnt);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(fb_scan, dim3(1), dim3(64), 0, a.stream, a.n_progs, cnt, off, choff, total);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(fb_compact, dim3((unsigned)a.n_progs), dim3(kEvalBlock), 0, a.stream, a, flags, off, list);
    e = hipGetLastError();
  }
  if (e == hipSuccess && a.max_q > 0) {
    const Hw32 hw = make_hw32(a.hw);
    const float* coefs = reinterpret_cast<const float*>(a.ws);
    const CfgRec* recs = reinterpret_cast<const CfgRec*>(
        reinterpret_cast<const char*>(a.ws) + (int64_t)a.n_progs * a.max_cfg * kSlotFloats * sizeof(float));
    const unsigned grid = (unsigned)a.n_progs * ((a.max_q + kEvalBlock - 1) / kEvalBlock);
    hipLaunchKernelGGL(fb_exact, dim3(grid), dim3(kEvalBlock), 0, a.stream, a.progs, coefs, recs, a.queries,
                       a.argmin, best_cost, a, hw, cnt, off, choff, total, list);
    e = hipGetLastError();
  }
  if (a.timer) a.timer->end(t, a.stream);
  return e;
}

int eval_num_variants() { return kNumVariants; }

int64_t selftest_short_division(int32_t b_first, int32_t b_count) {
  if (b_first < 0 || b_count < 0 || (int64_t)b_first + b_count > (1 << 23)) return -1;
  unsigned long long* d = nullptr;
  if (hipMalloc(&d, sizeof *d) != hipSuccess) return -1;
  bool ok = hipMemset(d, 0, sizeof *d) == hipSuccess;
  // slices of 2^16 b mantissas (2^39 pairs, a fraction of a second each)
  constexpr int32_t kSlice = 1 << 16;
  for (int32_t b0 = b_first; ok && b0 < b_first + b_count; b0 += kSlice) {
    const int32_t nb = b_first + b_count - b0 < kSlice ? b_first + b_count - b0 : kSlice;
    const uint64_t threads = (uint64_t)nb * kSdThreadsPerB;
    hipLaunchKernelGGL(short_div_check, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, nullptr,
                       (uint32_t)b0, (uint32_t)nb, d);
    ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  }
  unsigned long long h = 0;
  ok = ok && hipMemcpy(&h, d, sizeof h, hipMemcpyDeviceToHost) == hipSuccess;
  const bool freed = hipFree(d) == hipSuccess;
  return ok && freed ? (int64_t)h : -1;
}

int64_t selftest_divisor_list(const uint64_t* ds, int32_t n_ds) {
  // each listed divisor (up to 64 bits) against dividends at and around its multiples, small
  // values and the top of the range, with the host form of the device arithmetic
  int64_t bad = 0;
  for (int32_t i = 0; i < n_ds; ++i) {
    const uint64_t d = ds[i];
    if (d == 0) { ++bad; continue; }
    uint32_t m = 0;
    int32_t sh = 0;
    magic_u31_wide(d, &m, &sh);
    auto chk = [&](uint64_t n) {
      if (n >= (1ull << 31)) return;
      const uint32_t q = sh < 0 ? (uint32_t)n : (uint32_t)((n * m) >> 32) >> sh;
      if ((uint64_t)q != n / d) ++bad;
    };
    for (uint64_t n = 0; n < 4096; ++n) chk(n);
    for (uint64_t k = 0; k < 64; ++k) chk((1ull << 31) - 1 - k);
    for (uint64_t k = d; k < (1ull << 31); k = k * 3 + 7) {
      chk(k / d * d);
      chk(k / d * d - 1);
      chk(k / d * d + d - 1);
    }
  }
  return bad;
}

int64_t selftest_divisors(uint32_t d_max) {
  // every divisor 1..d_max against dividends at and around its multiples, small values and the
  // top of the range, with the host form of the same arithmetic (64-bit product, high word)
  int64_t bad = 0;
  for (uint32_t d = 1; d <= d_max; ++d) {
    uint32_t m = 0;
    int32_t sh = 0;
    magic_u31(d, &m, &sh);
    auto chk = [&](uint32_t n) {
      if (n >= (1u << 31)) return;
      const uint32_t q = sh < 0 ? n : (uint32_t)(((uint64_t)n * m) >> 32) >> sh;
      if (q != n / d) ++bad;
    };
    for (uint32_t n = 0; n < 4096; ++n) chk(n);
    const uint32_t top = (1u << 31) - 1u;
    for (uint32_t k = 0; k < 64; ++k) chk(top - k);
    for (uint64_t k = d; k < (1ull << 31); k = k * 3 + 7) {
      chk((uint32_t)(k / d * d));
      chk((uint32_t)(k / d * d - 1));
      chk((uint32_t)(k / d * d + d - 1));
    }
  }
  return bad;
}

hipError_t launch_eval(const EvalArgs& a) {
  hipError_t e = launch_collapse_only(a);
  if (e != hipSuccess) return e;
  if (a.max_q == 0) return hipSuccess;
  const Hw32 hw = make_hw32(a.hw);
  const float* coefs = reinterpret_cast<const float*>(a.ws);
  const CfgRec* recs = reinterpret_cast<const CfgRec*>(
      reinterpret_cast<const char*>(a.ws) + (int64_t)a.n_progs * a.max_cfg * kSlotFloats * sizeof(float));
  int v = a.variant;
  if (v < 0 && a.tuner) {
    // autotune: time every variant once on this problem (all produce identical outputs)
    float best = 0.0f;
    int bv = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int i = 0; i < kNumVariants && e == hipSuccess; ++i) {
      e = hipEventRecord(e0, a.stream);
      if (e == hipSuccess) e = launch_sweep(i, a, hw, coefs, recs);
      if (e == hipSuccess) e = hipEventRecord(e1, a.stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && (i == 0 || ms < best)) { best = ms; bv = i; }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    a.tuner->record(a.tune_key, bv, best);
    v = bv;
  }
  if (v < 0) v = 0;
  int t = a.timer ? a.timer->begin(KLR_K_EVAL, a.stream) : -1;
  e = launch_sweep(v % kNumVariants, a, hw, coefs, recs);
  if (a.timer) a.timer->end(t, a.stream);
  return e;
}

}  // namespace klr

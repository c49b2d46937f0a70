// Batched rational least-squares fits, one wavefront per fit (small fits), gfx950.
//
// Same problem and numerical method as the workgroup kernel in fit.hip (paper: step 2 of the
// section "An Algorithm to Build and Deploy a Performance-Predicting Rational Program" and
// section "Building a Driver Program: Rational function estimation"), organised for fits with
// n <= 48 unknowns, v <= 4 variables, m <= 1024 samples and exponents <= 3:
//   * lane l owns sample rows l, l + 64, ... (scaled variables, target and residual in VGPRs;
//     8 rows per lane for m <= 512 at two waves per SIMD, 16 for m <= 1024 at one);
//   * Gram on MFMA (v_mfma_f64_16x16x4f64 for the FP64 path, v_mfma_f32_16x16x4f32 with FP32
//     values, v_mfma_f32_16x16x16_bf16 with BF16 values over four steps): for each step of 4 rows the
//     lanes build a table of x_k^p (p <= 3) of the step's rows in LDS, one entry per lane, and
//     every lane forms exactly the design-matrix elements of its MFMA operand slots (column
//     l % 16 of each 16-column tile, row l / 16 of the step) from four table entries, so A is
//     never stored;
//   * equilibration, shift, diagonally pivoted Cholesky kept in pivot order (rows and columns
//     swapped in place), triangular solves and reductions are wave-synchronous (no workgroup
//     barriers); four independent fits per workgroup;
//   * refinement: CGLS on the right-preconditioned problem with one pass over the rows per
//     iteration: q = A t stays in registers, alpha needs only ||q||^2 (one wave reduction), the
//     FP64 residual is updated in place and A^T r accumulated in the same pass; column
//     exponents are read into scalar registers so the monomial loops are uniform; stopping by
//     the delayed Hestenes-Stiefel estimate of ||A(y - y*)||.
// MFMA layouts (wave64): see GramTypes in internal.hpp.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "internal.hpp"

namespace klr {
namespace {

constexpr int kNP = 48;            // padded unknowns: three 16-column tiles
static_assert(kNP <= 48, "the 8 x 8 update grid of the factorization covers 48 rows");
constexpr int kV = 4;              // variables
constexpr int kSP = kNP * (kNP + 1) / 2;


struct WaveLds {
  double S[kSP];                   // equilibrated, shifted Gram -> pivoted Cholesky factor
  double D[kNP];                   // power-of-two column scales
  double c[kNP];                   // D A^T f
  double z[kNP];                   // iterate (equilibrated coefficients)
  double dz[kNP];                  // direction in the equilibrated coefficients
  double t[kNP];                   // coefficient vector read by the row passes (unscaled)
  double s[kNP], p[kNP];           // preconditioned normal residual and search direction
  double g[kNP];                   // D A^T w written by the row passes
  double piv[kNP];
  double rd[kNP];                  // 1 / L_kk, pivot-indexed
  int perm[kNP];
  int ex[kNP];                     // exponents of column j, one byte per variable
  double T[64];                    // per Gram step: x_k^p of the step's 4 rows, [row][k][p]
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Row base of the packed lower triangle: element (i, j), j <= i, is at rbase(i) + j.
__device__ __forceinline__ int rbase(int i) { return i * (i + 1) / 2; }

__device__ __forceinline__ int symi(int a, int b) {
  return a >= b ? a * (a + 1) / 2 + b : b * (b + 1) / 2 + a;
}

__device__ __forceinline__ double wsum(double v) { return wave_sum_d(v); }

// Sample rows of one fit held in registers: lane l owns rows l, l + 64, ..., RPL rows per lane
// (RPL = 8 for m <= 512, 16 for m <= 1024).
template <int RPL>
struct Rows {
  double x[RPL][kV];
  double f[RPL];
  double r[RPL];
};

// Gram of the equilibrated problem's unscaled matrix: S (packed lower) and c = A^T f.
template <int GP, int RPL>
__device__ void gram(WaveLds& L, const Rows<RPL>& R, int m, int n, int n_num) {
  using GT = GramTypes<GP>;
  typename GT::acc_t acc[6];
#pragma unroll
  for (int t = 0; t < 6; ++t) acc[t] = (typename GT::acc_t){0, 0, 0, 0};
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  // table position of x_k^(e_k) for each of the lane's three columns, as byte offsets packed
  // two per word: entry (row g, variable k, power p) is T[16 g + 4 k + p]
  unsigned offs[3][2];
  bool numc[3], inr[3];
#pragma unroll
  for (int ct = 0; ct < 3; ++ct) {
    const int j = ct * 16 + col, ew = L.ex[j];
    unsigned o[4];
#pragma unroll
    for (int k = 0; k < kV; ++k) {
      const int ek = (ew >> (8 * k)) & 0xFF;
      o[k] = 8u * (unsigned)(16 * grp + 4 * k + ek);
    }
    offs[ct][0] = o[0] | (o[1] << 16);
    offs[ct][1] = o[2] | (o[3] << 16);
    numc[ct] = j < n_num;
    inr[ct] = j < n;
  }
  const int tk_var = (lane >> 2) & 3, tk_pow = lane & 3;   // the table entry this lane writes
  const char* Tb = reinterpret_cast<const char*>(L.T);
  double cacc[3] = {0.0, 0.0, 0.0};
  typename GT::op_t op[3];
  const int steps = (m + 3) / 4;
  for (int st = 0; st < steps; ++st) {
    const int row = 4 * st + grp;             // this lane's row of the step
    const int src = row & 63, slot = (4 * st) >> 6;
    double xv[kV], fv = 0.0;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      if (s == slot) {
#pragma unroll
        for (int k = 0; k < kV; ++k) xv[k] = __shfl(R.x[s][k], src);
        fv = __shfl(R.f[s], src);
      }
    }
    const bool live = row < m;
    double a[3];
    {
      const double xk = tk_var == 0 ? xv[0] : (tk_var == 1 ? xv[1] : (tk_var == 2 ? xv[2] : xv[3]));
      const double x2 = xk * xk;
      L.T[lane] = tk_pow == 0 ? 1.0 : (tk_pow == 1 ? xk : (tk_pow == 2 ? x2 : x2 * xk));
      wave_sync();
#pragma unroll
      for (int ct = 0; ct < 3; ++ct) {
        const double m0 = *reinterpret_cast<const double*>(Tb + (offs[ct][0] & 0xFFFFu));
        const double m1 = *reinterpret_cast<const double*>(Tb + (offs[ct][0] >> 16));
        const double m2 = *reinterpret_cast<const double*>(Tb + (offs[ct][1] & 0xFFFFu));
        const double m3 = *reinterpret_cast<const double*>(Tb + (offs[ct][1] >> 16));
        const double mo = (m0 * m1) * (m2 * m3);
        a[ct] = (live && inr[ct]) ? (numc[ct] ? mo : -fv * mo) : 0.0;
      }
      wave_sync();                           // the table is rewritten by the next step
    }
#pragma unroll
    for (int ct = 0; ct < 3; ++ct) cacc[ct] += a[ct] * fv;
    const int e = st % GT::SUB;                // sub-step of the MFMA's reduction block
    if (e == 0) {
#pragma unroll
      for (int ct = 0; ct < 3; ++ct) op[ct] = GT::zero();
    }
#pragma unroll
    for (int ct = 0; ct < 3; ++ct) GT::put(op[ct], e, a[ct]);
    if (e == GT::SUB - 1 || st == steps - 1) {
      acc[0] = GT::mma(op[0], op[0], acc[0]);   // tile (0, 0)
      acc[1] = GT::mma(op[1], op[0], acc[1]);   // tile (1, 0)
      acc[2] = GT::mma(op[1], op[1], acc[2]);   // tile (1, 1)
      acc[3] = GT::mma(op[2], op[0], acc[3]);   // tile (2, 0)
      acc[4] = GT::mma(op[2], op[1], acc[4]);   // tile (2, 1)
      acc[5] = GT::mma(op[2], op[2], acc[5]);   // tile (2, 2)
    }
  }
  const int tj[6] = {0, 1, 1, 2, 2, 2}, tk[6] = {0, 0, 1, 0, 1, 2};
#pragma unroll
  for (int t = 0; t < 6; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = tj[t] * 16 + GT::out_row(grp, r), k = tk[t] * 16 + col;
      if (j < n && k < n && k <= j) L.S[rbase(j) + k] = (double)acc[t][r];
    }
#pragma unroll
  for (int ct = 0; ct < 3; ++ct) {
    const double v = pair_sum32(pair_sum16(cacc[ct]));
    if (grp == 0 && ct * 16 + col < n) L.c[ct * 16 + col] = v;
  }
  wave_sync();
}

// Equilibrate, shift by mu = 8 u tr / n, diagonally pivoted Cholesky.  Returns the rank.
// The factor is kept in pivot order: at step k the rows and columns k and bi are swapped in
// place (the computed part of L and the Schur complement alike), so element (i, j) of L is at
// rbase(i) + j and perm maps a pivot position to the original column.
__device__ int factor_wave(WaveLds& L, int n, double unit) {
  const int lane = threadIdx.x & 63;
  const int myb = rbase(lane);
  if (lane < n) {
    const double gjj = L.S[myb + lane];
    int e = 0;
    if (gjj > 0.0 && isfinite(gjj)) frexp(sqrt(gjj), &e);
    L.D[lane] = ldexp(1.0, -e);
    L.perm[lane] = lane;
  }
  wave_sync();
  if (lane < n) {                       // row `lane` of the lower triangle
    const double dl = L.D[lane];
#pragma unroll 8
    for (int j = 0; j <= lane; ++j) L.S[myb + j] *= dl * L.D[j];
    L.c[lane] *= dl;
  }
  wave_sync();
  double tr = lane < n ? L.S[myb + lane] : 0.0;
  tr = wsum(tr);
  const double mu = 8.0 * unit * tr / n + 1e-300;
  if (lane < n) L.S[myb + lane] += mu;
  wave_sync();
  for (int k = 0; k < n; ++k) {
    double best = -INFINITY;
    int bi = n;
    if (lane >= k && lane < n) {
      const double vv = L.S[myb + lane];
      best = vv == vv ? vv : -INFINITY;
      bi = lane;
    }
    wave_argmax(best, bi);
    if (!(best > 4.0 * mu)) {
      const double smu = sqrt(mu);
      if (lane >= k && lane < n) {
        L.piv[lane] = L.S[myb + lane];
        for (int j = k; j < lane; ++j) L.S[myb + j] = 0.0;
        L.S[myb + lane] = smu;
      }
      wave_sync();
      break;
    }
    if (bi != k) {                      // symmetric swap of positions k < bi
      const int ba = rbase(k), bb = rbase(bi);
      int p0 = -1, p1 = -1;
      if (lane < k) { p0 = ba + lane; p1 = bb + lane; }
      else if (lane == k) { p0 = ba + k; p1 = bb + bi; }
      else if (lane < bi) { p0 = myb + k; p1 = bb + lane; }
      else if (lane > bi && lane < n) { p0 = myb + k; p1 = myb + bi; }
      if (p0 >= 0) {
        const double t0 = L.S[p0], t1 = L.S[p1];
        L.S[p0] = t1;
        L.S[p1] = t0;
      }
      if (lane == 0) {
        const int t = L.perm[k];
        L.perm[k] = L.perm[bi];
        L.perm[bi] = t;
      }
      wave_sync();
    }
    const double lkk = sqrt(best);
    if (lane == k) {
      L.piv[k] = best;
      L.S[myb + k] = lkk;
    } else if (lane > k && lane < n) {
      L.S[myb + k] = L.S[myb + k] / lkk;
    }
    wave_sync();
    // S(i, j) -= L(i, k) L(j, k) for k < j <= i: lane (ty, tx) of an 8 x 8 grid takes rows
    // k + 1 + ty + 8 a and columns k + 1 + tx + 8 b (n <= 48: a, b < 6), so the entries of
    // the trailing triangle are spread evenly and the loads of a row are independent
    {
      const int ty = lane >> 3, tx = lane & 7;
      double lj[6];
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        const int j = k + 1 + tx + 8 * b;
        lj[b] = j < n ? L.S[rbase(j) + k] : 0.0;
      }
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        const int i = k + 1 + ty + 8 * a;
        if (i < n) {
          const int rb = rbase(i);
          const double li = L.S[rb + k];
#pragma unroll
          for (int b = 0; b < 6; ++b) {
            const int j = k + 1 + tx + 8 * b;
            if (j <= i) L.S[rb + j] -= li * lj[b];
          }
        }
      }
    }
    wave_sync();
  }
  if (lane < n) L.rd[lane] = 1.0 / L.S[myb + lane];
  const unsigned long long full = __ballot(lane < n && L.piv[lane] > 4.0 * mu);
  wave_sync();
  return __popcll(full);
}

// L u = in[perm] (out pivot-indexed).  Step k reads b_k, forms u_k = b_k / L(k, k) (a product
// with the stored reciprocal) and subtracts L(i, k) u_k from the rows i > k (the factor entry of
// rows i <= k is taken as zero, which leaves them unchanged while u_k is finite); row k keeps
// b_k, and every u_k is formed again at the end from the same operands.  Lanes past n hold values
// never stored.
__device__ void fwd_wave(const WaveLds& L, int n, const double* in, double* out) {
  const int lane = threadIdx.x & 63;
  n = __builtin_amdgcn_readfirstlane(n);
  const int myb = rbase(lane < n ? lane : 0);
  double b = lane < n ? in[L.perm[lane]] : 0.0;
  // steps in groups of 4: the factor entries of a group are loaded before its dependent chain
  for (int k0 = 0; k0 < n; k0 += 4) {
    double rp[4], sv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + u < n ? k0 + u : n - 1;
      rp[u] = L.rd[k];
      sv[u] = lane > k ? L.S[myb + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + u;
      if (k < n) {
        const double uk = readlane_d(b, k) * rp[u];
        b -= sv[u] * uk;
      }
    }
  }
  if (lane < n) out[lane] = b * L.rd[lane];
  wave_sync();
}
// L^T v = in (pivot-indexed); out[perm[i]] = v_i.  Step k (from n - 1 down) forms v_k = b_k /
// L(k, k) and subtracts L(k, i) v_k from the rows i < k; row k keeps b_k and the v_k are formed
// again at the end.
__device__ void bwd_wave(const WaveLds& L, int n, const double* in, double* out) {
  const int lane = threadIdx.x & 63;
  n = __builtin_amdgcn_readfirstlane(n);
  double b = lane < n ? in[lane] : 0.0;
  for (int k0 = n - 1; k0 >= 0; k0 -= 4) {
    double rp[4], sv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 - u >= 0 ? k0 - u : 0;
      rp[u] = L.rd[k];
      sv[u] = lane < k ? L.S[rbase(k) + lane] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 - u;
      if (k >= 0) {
        const double vk = readlane_d(b, k) * rp[u];
        b -= sv[u] * vk;
      }
    }
  }
  if (lane < n) out[L.perm[lane]] = b * L.rd[lane];
  wave_sync();
}

__device__ __forceinline__ double dotw(const double* a, const double* b, int n) {
  const int lane = threadIdx.x & 63;
  return wsum(lane < n ? a[lane] * b[lane] : 0.0);
}

// Monomial x~^e of column e (packed exponents, wave-uniform) for the lane's first NS rows.
template <int NS, int RPL>
__device__ __forceinline__ void mono_rows(const Rows<RPL>& R, int e, double* mo) {
#pragma unroll
  for (int s = 0; s < NS; ++s) mo[s] = 1.0;
#pragma unroll
  for (int k = 0; k < kV; ++k) {
    const int ek = (e >> (8 * k)) & 0xFF;
    for (int q = 0; q < ek; ++q)
#pragma unroll
      for (int s = 0; s < NS; ++s) mo[s] *= R.x[s][k];
  }
}

// One pass over the rows with the coefficient vector y held in L.t (D z of the iterate or of the
// direction): d_i = A_i . y = p_i - f_i s_i with p_i, s_i the numerator and denominator parts.
//   mode 0: r = f - d, then g = D A^T r;
//   mode 1: d is the CGLS image q = A D dz: *qq = ||q||^2, alpha = gamma / ||q||^2, the FP64
//           residual is updated in place (r -= alpha q) and g = D A^T r from the updated residual;
//   mode 2: returns ||f - d||^2 and counts q(x~_i) = 1 + s_i <= 0 into *qneg.
// Column exponents are read into scalar registers, so the monomial loops are uniform.  Only the
// lane's first NS row slots are visited (m <= 64 NS: the others hold no sample).
// Returns alpha in mode 1.
template <int MODE, int RPL, int NS>
__device__ double row_pass_ns(WaveLds& L, Rows<RPL>& R, int m, int n, int n_num, double gamma, double* qq,
                              int* qneg) {
  const int lane = threadIdx.x & 63;
  // lane j holds column j's exponents and coefficient; the column loops broadcast them by
  // readlane instead of an LDS round trip per column
  const int exv = lane < kNP ? L.ex[lane] : 0;
  const double tv = lane < kNP ? L.t[lane] : 0.0;
  double pn[NS], pd[NS], mo[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) pn[s] = pd[s] = 0.0;
  for (int j = 0; j < n_num; ++j) {
    mono_rows<NS>(R, __builtin_amdgcn_readlane(exv, j), mo);
    const double tj = readlane_d(tv, j);
#pragma unroll
    for (int s = 0; s < NS; ++s) pn[s] += mo[s] * tj;
  }
  for (int j = n_num; j < n; ++j) {
    mono_rows<NS>(R, __builtin_amdgcn_readlane(exv, j), mo);
    const double tj = readlane_d(tv, j);
#pragma unroll
    for (int s = 0; s < NS; ++s) pd[s] += mo[s] * tj;
  }
  double sq = 0.0;
  int qn = 0;
  double d[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const bool live = lane + 64 * s < m;
    d[s] = live ? pn[s] - R.f[s] * pd[s] : 0.0;
    if (MODE == 0 && live) R.r[s] = R.f[s] - d[s];
    if (MODE == 1) sq += d[s] * d[s];
    if (MODE == 2 && live) {
      const double res = R.f[s] - d[s];
      sq += res * res;
      if (!(1.0 + pd[s] > 0.0)) ++qn;
    }
  }
  if (MODE == 2) {
    *qneg = (int)wsum((double)qn);     // a count: exact in FP64
    return wsum(sq);
  }
  double alpha = 0.0;
  if (MODE == 1) {
    const double qn2 = wsum(sq);
    *qq = qn2;
    alpha = qn2 > 0.0 ? gamma / qn2 : 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) R.r[s] -= alpha * d[s];
  }
  // g_j = D_j sum_i A_ij r_i: numerator columns weigh r_i, denominator columns -f_i r_i
  double wf[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) wf[s] = -R.f[s] * R.r[s];
  // column sums collected in lane j of gv (one wavefront sum per column, two columns per step
  // so that their reductions overlap)
  double gv = 0.0;
  for (int j0 = 0; j0 < n; j0 += 2) {
    double v2[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int j = j0 + u < n ? j0 + u : j0;
      mono_rows<NS>(R, __builtin_amdgcn_readlane(exv, j), mo);
      double v = 0.0;
      if (j < n_num) {
#pragma unroll
        for (int s = 0; s < NS; ++s) v += mo[s] * R.r[s];
      } else {
#pragma unroll
        for (int s = 0; s < NS; ++s) v += mo[s] * wf[s];
      }
      v2[u] = v;
    }
    const double s0 = wsum(v2[0]), s1 = wsum(v2[1]);
    if (lane == j0) gv = s0;
    if (lane == j0 + 1) gv = s1;
  }
  if (lane < n) L.g[lane] = gv * L.D[lane];
  wave_sync();
  return alpha;
}

// row_pass_ns for the smallest listed slot count that covers the fit's m rows (wave-uniform):
// 2, 4 or 8 slots with 8 rows per lane; 12 or 16 with 16 rows per lane (its fits have m > 512).
template <int MODE, int RPL>
__device__ __forceinline__ double row_pass(WaveLds& L, Rows<RPL>& R, int m, int n, int n_num, double gamma,
                                           double* qq, int* qneg) {
  if constexpr (RPL == 8) {
    if (m <= 128) return row_pass_ns<MODE, RPL, 2>(L, R, m, n, n_num, gamma, qq, qneg);
    if (m <= 256) return row_pass_ns<MODE, RPL, 4>(L, R, m, n, n_num, gamma, qq, qneg);
  } else {
    if (m <= 768) return row_pass_ns<MODE, RPL, 12>(L, R, m, n, n_num, gamma, qq, qneg);
  }
  return row_pass_ns<MODE, RPL, RPL>(L, R, m, n, n_num, gamma, qq, qneg);
}

template <int PREC, int RPL>
__device__ void fit_wave_one(const FitArgs& a, int fi, WaveLds& L) {
  const int lane = threadIdx.x & 63;
  const klr_fit_desc d = a.desc[fi];
  const int n = d.n_num + d.n_den - 1;
  const bool coef_ok = d.n_num >= 0 && d.n_den >= 1 && n >= 1 && n <= kNP && d.coef0 >= 0 &&
                       d.coef0 + (int64_t)n <= a.coef_len;
  bool ok = coef_ok && d.v >= 1 && d.v <= kV && d.m >= 1 && d.m <= RPL * 64 && d.x0 >= 0 &&
            d.x0 + (int64_t)d.m * d.v <= a.x_len && d.f0 >= 0 && d.f0 + (int64_t)d.m <= a.f_len &&
            d.num0 >= 0 && (int64_t)d.num0 + d.n_num <= a.n_exp_rows && d.den0 >= 0 &&
            (int64_t)d.den0 + d.n_den <= a.n_exp_rows;
  if (ok)
#pragma unroll
    for (int k = 0; k < kV; ++k)
      if (k < d.v) {
        if (d.scale_exp[k] < -100 || d.scale_exp[k] > 100) ok = false;
        if (a.exps[(int64_t)d.den0 * KLR_MAX_VARS + k] != 0) ok = false;
      }
  klr_fit_info info{};
  Rows<RPL> R;
#pragma unroll
  for (int s = 0; s < RPL; ++s) {
#pragma unroll
    for (int k = 0; k < kV; ++k) R.x[s][k] = 0.0;
    R.f[s] = 0.0;
    R.r[s] = 0.0;
  }
  bool bad = !ok;
  if (ok) {
    if (lane < kNP) {
      int w = 0;
      if (lane < n) {
        const int row = lane < d.n_num ? d.num0 + lane : d.den0 + (lane - d.n_num + 1);
        for (int k = 0; k < d.v; ++k) w |= (int)a.exps[(int64_t)row * KLR_MAX_VARS + k] << (8 * k);
      }
      L.ex[lane] = w;
    }
    bool nonfinite = false;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int i = lane + 64 * s;
      if (i < d.m) {
#pragma unroll
        for (int k = 0; k < kV; ++k)
          if (k < d.v) R.x[s][k] = ldexp((double)a.X[d.x0 + (int64_t)i * d.v + k], -(int)d.scale_exp[k]);
        R.f[s] = a.f[d.f0 + i];
        nonfinite |= !isfinite(R.f[s]);
      }
    }
    bad = __any(nonfinite);
    wave_sync();
  }
  if (bad) {
    if (coef_ok)
      for (int j = lane; j < n; j += 64) a.coef[d.coef0 + j] = 0.0;
    if (lane == 0) {
      info.status = KLR_FIT_BAD_INPUT;
      info.resid_norm = NAN;
      info.err_est = NAN;
      a.info[fi] = info;
    }
    return;
  }
  double fn2 = 0.0;
#pragma unroll
  for (int s = 0; s < RPL; ++s) fn2 += R.f[s] * R.f[s];
  const double fnorm = sqrt(wsum(fn2));

  int prec = PREC, iters = 0, rank = 0;
  bool converged = false;
  double err = 0.0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    double unit;
    if (prec == KLR_FP64) { gram<KLR_FP64, RPL>(L, R, d.m, n, d.n_num); unit = 0x1p-53; }
    else if (prec == KLR_FP32_REFINED) { gram<KLR_FP32_REFINED, RPL>(L, R, d.m, n, d.n_num); unit = 0x1p-24; }
    else { gram<KLR_BF16_REFINED, RPL>(L, R, d.m, n, d.n_num); unit = 0x1p-8; }
    rank = factor_wave(L, n, unit);
    fwd_wave(L, n, L.c, L.s);                          // z0 = (G~ + mu I)^-1 D A^T f
    bwd_wave(L, n, L.s, L.z);
    if (lane < n) L.t[lane] = L.D[lane] * L.z[lane];
    wave_sync();
    row_pass<0, RPL>(L, R, d.m, n, d.n_num, 0.0, nullptr, nullptr);   // r0 = f - A y0, g = D A^T r0
    fwd_wave(L, n, L.g, L.s);                          // s0 = R^-T Pi^T g
    if (lane < n) L.p[lane] = L.s[lane];
    wave_sync();
    double gamma = dotw(L.s, L.s, n);
    iters = 0;
    converged = a.max_iter == 0 || gamma == 0.0;
    err = 0.0;
    double h0 = 0.0, h1 = 0.0, h2 = 0.0;   // the last three alpha gamma terms
    const int need = a.max_iter < 3 ? a.max_iter : 3;
    for (int it = 0; it < a.max_iter && !converged; ++it) {
      bwd_wave(L, n, L.p, L.dz);                       // dz = Pi R^-1 p
      if (lane < n) L.t[lane] = L.D[lane] * L.dz[lane];
      wave_sync();
      double qq = 0.0;   // ||A D dz||^2; r -= alpha A D dz; g = D A^T r
      const double alpha = row_pass<1, RPL>(L, R, d.m, n, d.n_num, gamma, &qq, nullptr);
      if (lane < n) L.z[lane] += alpha * L.dz[lane];
      wave_sync();
      h0 = h1;
      h1 = h2;
      h2 = alpha * gamma;
      ++iters;
      if (it + 1 >= need) {
        const double est = sqrt(h0 + h1 + h2);
        err = fnorm > 0.0 ? est / fnorm : 0.0;
        if (est <= a.tol * fnorm) { converged = true; break; }
      }
      if (qq == 0.0) { converged = true; break; }
      fwd_wave(L, n, L.g, L.s);                        // s = B^T r from the updated residual
      const double gnew = dotw(L.s, L.s, n);
      const double beta = gamma > 0.0 ? gnew / gamma : 0.0;
      if (lane < n) L.p[lane] = L.s[lane] + beta * L.p[lane];
      wave_sync();
      gamma = gnew;
      if (gamma == 0.0) { converged = true; break; }
    }
    if (converged || prec == KLR_FP64) break;
    info.status |= KLR_FIT_FELL_BACK_FP64;
    prec = KLR_FP64;
  }
  if (lane < n) L.t[lane] = L.D[lane] * L.z[lane];
  wave_sync();
  int qneg = 0;
  const double rr = row_pass<2, RPL>(L, R, d.m, n, d.n_num, 0.0, nullptr, &qneg);
  if (lane < n) a.coef[d.coef0 + lane] = L.t[lane];
  if (lane == 0) {
    if (rank < n) info.status |= KLR_FIT_RANK_DEFICIENT;
    if (d.m < n) info.status |= KLR_FIT_UNDERDETERMINED;
    if (!converged) info.status |= KLR_FIT_NOT_CONVERGED;
    if (qneg > 0) info.status |= KLR_FIT_Q_NONPOS;
    info.rank = rank;
    info.iters = iters;
    info.q_nonpos = qneg;
    info.resid_norm = sqrt(rr);
    info.err_est = err;
    a.info[fi] = info;
  }
  wave_sync();
}

// Longest-first schedule: wave w of workgroup b takes position WG b + w of its row class's part
// of the plan's order (the dispatcher starts workgroups in index order, so the longest fits
// start first); positions past the class's count leave at once.  Fits with 8 rows per lane run
// two waves per SIMD; those with 16 rows per lane need the whole register file of one.  WG
// (fits per workgroup: 1, 2 or 4) changes only how the fits are grouped into workgroups (a
// workgroup's LDS is released when its last fit ends), never a fit's arithmetic.
template <int PREC, int RPL, int WG>
__device__ __forceinline__ void ordered_body(const FitArgs& a, const WavePlanView& pv, WaveLds* lds) {
  const int i = blockIdx.x * WG + (threadIdx.x >> 6);
  if (i >= *pv.total) return;
  fit_wave_one<PREC, RPL>(a, pv.order[*pv.base + i], lds[threadIdx.x >> 6]);
}
template <int PREC, int RPL, int WG>
__device__ __forceinline__ void plain_body(const FitArgs& a, WaveLds* lds) {
  const int fi = blockIdx.x * WG + (threadIdx.x >> 6);
  if (fi >= a.n_fits || wave_fit_rows(a, a.desc[fi]) != RPL) return;
  fit_wave_one<PREC, RPL>(a, fi, lds[threadIdx.x >> 6]);
}

template <int PREC, int WG>
__global__ void __launch_bounds__(64 * WG) __attribute__((amdgpu_waves_per_eu(2)))
fit_wave_ordered(FitArgs a, WavePlanView pv) {
  __shared__ WaveLds lds[WG];
  ordered_body<PREC, 8, WG>(a, pv, lds);
}
template <int PREC, int WG>
__global__ void __launch_bounds__(64 * WG) __attribute__((amdgpu_waves_per_eu(1)))
fit_wave_ordered16(FitArgs a, WavePlanView pv) {
  __shared__ WaveLds lds[WG];
  ordered_body<PREC, 16, WG>(a, pv, lds);
}

// One wave per fit in descriptor order; waves whose fit is not of the kernel's row class leave.
template <int PREC, int WG>
__global__ void __launch_bounds__(64 * WG) __attribute__((amdgpu_waves_per_eu(2)))
fit_wave_plain(FitArgs a) {
  __shared__ WaveLds lds[WG];
  plain_body<PREC, 8, WG>(a, lds);
}
template <int PREC, int WG>
__global__ void __launch_bounds__(64 * WG) __attribute__((amdgpu_waves_per_eu(1)))
fit_wave_plain16(FitArgs a) {
  __shared__ WaveLds lds[WG];
  plain_body<PREC, 16, WG>(a, lds);
}

template <int PREC, int WG>
hipError_t launch_wave_g(const FitArgs& a, bool ordered, const WavePlanView& pv8, const WavePlanView& pv16) {
  const dim3 grid((unsigned)((a.n_fits + WG - 1) / WG)), block(64 * WG);
  if (ordered) {
    hipLaunchKernelGGL((fit_wave_ordered16<PREC, WG>), grid, block, 0, a.stream, a, pv16);
    hipLaunchKernelGGL((fit_wave_ordered<PREC, WG>), grid, block, 0, a.stream, a, pv8);
  } else {
    hipLaunchKernelGGL((fit_wave_plain16<PREC, WG>), grid, block, 0, a.stream, a);
    hipLaunchKernelGGL((fit_wave_plain<PREC, WG>), grid, block, 0, a.stream, a);
  }
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_wave_t(const FitArgs& a, bool ordered, const WavePlanView& pv8, const WavePlanView& pv16) {
  if (a.wave_group == 1) return launch_wave_g<PREC, 1>(a, ordered, pv8, pv16);
  if (a.wave_group == 2) return launch_wave_g<PREC, 2>(a, ordered, pv8, pv16);
  return launch_wave_g<PREC, 4>(a, ordered, pv8, pv16);
}

}  // namespace

hipError_t launch_fit_wave(const FitArgs& a, bool ordered, const WavePlanView& pv8, const WavePlanView& pv16) {
  if (a.precision == KLR_FP64) return launch_wave_t<KLR_FP64>(a, ordered, pv8, pv16);
  if (a.precision == KLR_FP32_REFINED) return launch_wave_t<KLR_FP32_REFINED>(a, ordered, pv8, pv16);
  return launch_wave_t<KLR_BF16_REFINED>(a, ordered, pv8, pv16);
}

}  // namespace klr

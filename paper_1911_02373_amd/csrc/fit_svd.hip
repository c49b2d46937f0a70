// Batched rational least-squares fits by singular value decomposition, gfx950.
//
// Paper: section "Building a Driver Program: Rational function estimation" - the Vandermonde-like
// least-squares systems of the rational fits are ill-conditioned and possibly rank deficient,
// so the paper solves them through an SVD (LAPACK) rather than a QR factorisation.  This is
// that solver on the GPU, as an alternative to the Gram + pivoted Cholesky + CGLS path and as
// the rank reference.
//
// One workgroup per fit; thread t < m holds row t of the column-equilibrated design matrix
// B = A D (power-of-two D, exact) in registers, and one-sided Jacobi (Hestenes) rotations
// orthogonalise B's columns: B V = U S.  Columns are paired by the round-robin ordering
// (pairs (k, NC - 1 - k) of positions, position 0 fixed and positions 1 .. NC - 1 rotated one
// place after every step, so each pair of columns meets once per sweep of NC - 1 steps and the
// positions return to their places at the end of the sweep).  Per step, the NC / 2 inner
// products b_i . b_j are summed over the rows by a deterministic workgroup reduction, the
// rotations are formed by NC / 2 threads, and every thread rotates its row; V (n x n) lives in
// LDS and takes the same rotations.  Column norms are recomputed at the start of every sweep
// and updated in between; a sweep without a rotation (|b_i . b_j| <= sqrt(m) eps ||b_i|| ||b_j||
// for every pair) ends the iteration.  Then sigma_j = ||b_j||, the numerical rank counts
// sigma_j > 10 max(m, n) eps sigma_max (the oracle's threshold), and the minimum-norm solution
// of the equilibrated problem is z = V S^+ U^T f, y = D z.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "internal.hpp"

namespace klr {
namespace {

constexpr int kMaxSweeps = 30;

// Largest sample count per padded width: the rows sit in registers, one per thread.
__device__ __forceinline__ int svd_class(const FitArgs& a, const klr_fit_desc& d) {
  const int n = d.n_num + d.n_den - 1;
  if (!(d.n_num >= 0 && d.n_den >= 1 && n >= 1 && n <= 48)) return -1;
  if (d.m < 1 || d.v < 1 || d.v > KLR_MAX_VARS) return -1;
  const int nc = n <= 16 ? 16 : (n <= 32 ? 32 : 48);
  const int wmax = nc == 16 ? 1024 : 512;
  if (d.m > wmax) return -1;
  const int w = d.m <= 256 ? 256 : (d.m <= 512 ? 512 : 1024);
  return (nc / 16 - 1) * 3 + (w == 256 ? 0 : (w == 512 ? 1 : 2));
}

// Workgroup sums of K per-thread values (K a multiple of 8): inside each wavefront the value
// set is halved at lane distances 32, 16 and 8 (each lane keeps one half and adds its partner's
// copy of it), then summed over the last three lane bits; one LDS row per wavefront; thread
// k < K adds the rows in wavefront order.  The association is the same on every call, so the
// sums are reproducible.  out[k] is valid after the call (which ends with a barrier).
template <int K, int W>
__device__ __forceinline__ void block_sums(const double (&v)[K], double* red, double* out) {
  static_assert(K % 8 == 0, "value count");
  constexpr int K1 = K / 2, K2 = K / 4, K3 = K / 8;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool h5 = (lane & 32) != 0, h4 = (lane & 16) != 0, h3 = (lane & 8) != 0;
  double a1[K1], a2[K2], a3[K3];
#pragma unroll
  for (int i = 0; i < K1; ++i) {
    const double keep = h5 ? v[K1 + i] : v[i];
    const double send = h5 ? v[i] : v[K1 + i];
    a1[i] = keep + __shfl_xor(send, 32);
  }
#pragma unroll
  for (int i = 0; i < K2; ++i) {
    const double keep = h4 ? a1[K2 + i] : a1[i];
    const double send = h4 ? a1[i] : a1[K2 + i];
    a2[i] = keep + __shfl_xor(send, 16);
  }
#pragma unroll
  for (int i = 0; i < K3; ++i) {
    const double keep = h3 ? a2[K3 + i] : a2[i];
    const double send = h3 ? a2[i] : a2[K3 + i];
    a3[i] = keep + __shfl_xor(send, 8);
  }
#pragma unroll
  for (int i = 0; i < K3; ++i) {
    a3[i] += __shfl_xor(a3[i], 4);
    a3[i] += __shfl_xor(a3[i], 2);
    a3[i] += __shfl_xor(a3[i], 1);
  }
  const int base = (h5 ? K1 : 0) + (h4 ? K2 : 0) + (h3 ? K3 : 0);
  if ((lane & 7) == 0) {
#pragma unroll
    for (int i = 0; i < K3; ++i) red[wv * K + base + i] = a3[i];
  }
  __syncthreads();
  if ((int)threadIdx.x < K) {
    double s = 0.0;
    for (int w = 0; w < W / 64; ++w) s += red[w * K + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

template <int NC, int W>
struct SvdLds {
  double red[(W / 64) * NC];         // per-wavefront partial sums
  double V[NC * NC];                 // [row][physical column]
  double nrm[NC];                    // squared column norms by position
  double newn[NC];
  double gam[2 * NC];                // reduction results
  double cs[NC];                     // (c, s) of pair k at 2k, 2k + 1
  double D[NC];
  double w[NC];
  double y[NC];
  int slot[2][NC];                   // physical V column of each position (double-buffered)
  uint8_t ex[NC * 8];                // column exponents
  int flag;
  int rank;
};

// Scaled variables x~_k = x_k 2^-s_k (exact; unused variables 1) and the target of row t.
__device__ __forceinline__ void load_row(const FitArgs& a, const klr_fit_desc& d, int t, double* xt, double* f) {
  const int32_t* xr = a.X + d.x0 + (int64_t)t * d.v;
  for (int k = 0; k < KLR_MAX_VARS; ++k) xt[k] = k < d.v ? ldexp((double)xr[k], -(int)d.scale_exp[k]) : 1.0;
  *f = a.f[d.f0 + t];
}

// Monomial of column j at the thread's scaled variables: repeated multiplication in variable
// order (exponents from LDS, wave-uniform).
__device__ __forceinline__ double mono(const uint8_t* e, const double* xt, int v) {
  double r = 1.0;
  for (int k = 0; k < v; ++k)
    for (int p = 0; p < e[k]; ++p) r *= xt[k];
  return r;
}

template <int NC, int W>
__device__ void svd_fit(const FitArgs& a, int fi, SvdLds<NC, W>& L) {
  const klr_fit_desc d = a.desc[fi];
  const int n = d.n_num + d.n_den - 1;
  const int m = d.m, v = d.v;
  const int t = threadIdx.x;
  bool ok = d.x0 >= 0 && d.x0 + (int64_t)m * v <= a.x_len && d.f0 >= 0 && d.f0 + (int64_t)m <= a.f_len &&
            d.num0 >= 0 && (int64_t)d.num0 + d.n_num <= a.n_exp_rows && d.den0 >= 0 &&
            (int64_t)d.den0 + d.n_den <= a.n_exp_rows && d.coef0 >= 0 && d.coef0 + (int64_t)n <= a.coef_len;
  if (ok)
    for (int k = 0; k < v; ++k) {
      if (d.scale_exp[k] < -100 || d.scale_exp[k] > 100) ok = false;
      if (a.exps[(int64_t)d.den0 * KLR_MAX_VARS + k] != 0) ok = false;
    }
  if (t == 0) L.flag = 0;
  for (int q = t; ok && q < NC * 8; q += W) {      // NC * 8 entries: more than the threads when NC = 48
    const int j = q / 8, k = q % 8;
    uint8_t e = 0;
    if (j < n && k < v) {
      const int64_t row = j < d.n_num ? (int64_t)d.num0 + j : (int64_t)d.den0 + (j - d.n_num + 1);
      e = a.exps[row * KLR_MAX_VARS + k];
    }
    L.ex[q] = e;
  }
  __syncthreads();
  // the sample row: design-matrix row from the scaled variables and the target (the variables
  // and target are read again after the rotations, so only the row stays live through them)
  double col[NC];
  const bool own = ok && t < m;
  bool bad = false;
  {
    double xt[KLR_MAX_VARS];
    double f = 0.0;
    if (own) {
      load_row(a, d, t, xt, &f);
      bad = !isfinite(f);
    }
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      double e = 0.0;
      if (own && j < n) {
        const double mo = mono(L.ex + 8 * j, xt, v);
        e = j < d.n_num ? mo : -f * mo;
      }
      col[j] = e;
    }
  }
  if (bad) atomicOr(&L.flag, 1);
  __syncthreads();
  if (L.flag) ok = false;
  __syncthreads();
  if (!ok) {
    for (int j = t; j < n; j += W)
      if (d.coef0 >= 0 && d.coef0 + (int64_t)n <= a.coef_len) a.coef[d.coef0 + j] = 0.0;
    if (t == 0) {
      klr_fit_info info{};
      info.status = KLR_FIT_BAD_INPUT;
      info.resid_norm = NAN;
      info.err_est = NAN;
      a.info[fi] = info;
    }
    return;
  }
  // column equilibration by powers of two: D_j = 2^-e with ||A_j|| = frac 2^e, frac in [1/2, 1)
  {
    double sq[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) sq[j] = col[j] * col[j];
    block_sums<NC, W>(sq, L.red, L.gam);
    if (t < NC) {
      int e = 0;
      const double nr = sqrt(L.gam[t]);
      if (nr > 0.0) frexp(nr, &e);
      L.D[t] = ldexp(1.0, -e);
    }
    for (int i = t; i < NC * NC; i += W) L.V[i] = (i / NC == i % NC) ? 1.0 : 0.0;
    if (t < NC) { L.slot[0][t] = t; L.slot[1][t] = t; }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NC; ++j) col[j] *= L.D[j];
  }
  const double tol = sqrt((double)m) * 0x1p-52;
  int sweeps = 0;
  bool converged = false;
  int cur = 0;
  for (; sweeps < kMaxSweeps && !converged; ++sweeps) {
    double sq[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) sq[j] = col[j] * col[j];
    block_sums<NC, W>(sq, L.red, L.nrm);
    if (t == 0) L.flag = 0;
    for (int step = 0; step < NC - 1; ++step) {
      double g[NC / 2];
#pragma unroll
      for (int k = 0; k < NC / 2; ++k) g[k] = col[k] * col[NC - 1 - k];
      block_sums<NC / 2, W>(g, L.red, L.gam);
      if (t < NC / 2) {
        const int k = t;
        const double al = L.nrm[k], be = L.nrm[NC - 1 - k], ga = L.gam[k];
        double c = 1.0, s = 0.0, na = al, nb = be;
        if (ga != 0.0 && fabs(ga) > tol * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = c * tt;
          na = al - tt * ga;
          nb = be + tt * ga;
          atomicOr(&L.flag, 1);
        }
        L.cs[2 * k] = c;
        L.cs[2 * k + 1] = s;
        L.newn[k] = na;
        L.newn[NC - 1 - k] = nb;
      }
      __syncthreads();
      // rotate the row, then the rows of V (items (row i, pair k))
#pragma unroll
      for (int k = 0; k < NC / 2; ++k) {
        const double c = L.cs[2 * k], s = L.cs[2 * k + 1];
        const double x = col[k], y = col[NC - 1 - k];
        col[k] = c * x - s * y;
        col[NC - 1 - k] = s * x + c * y;
      }
      for (int it = t; it < n * (NC / 2); it += W) {
        const int i = it / (NC / 2), k = it % (NC / 2);
        const int sa = L.slot[cur][k], sb = L.slot[cur][NC - 1 - k];
        const double c = L.cs[2 * k], s = L.cs[2 * k + 1];
        const double x = L.V[i * NC + sa], y = L.V[i * NC + sb];
        L.V[i * NC + sa] = c * x - s * y;
        L.V[i * NC + sb] = s * x + c * y;
      }
      // next positions: 0 stays, NC - 1 moves to 1, p moves to p + 1
      if (t < NC) {
        const int dst = t == 0 ? 0 : (t == NC - 1 ? 1 : t + 1);
        L.nrm[dst] = L.newn[t];
        L.slot[cur ^ 1][dst] = L.slot[cur][t];
      }
      cur ^= 1;
      {
        const double last = col[NC - 1];
#pragma unroll
        for (int j = NC - 1; j >= 2; --j) col[j] = col[j - 1];
        col[1] = last;
      }
      __syncthreads();
    }
    converged = L.flag == 0;
    __syncthreads();
  }
  // singular values, U^T f, rank and the minimum-norm solution
  double xt[KLR_MAX_VARS];
  double f = 0.0;
  if (own) load_row(a, d, t, xt, &f);
  {
    double q[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) q[j] = col[j] * col[j];
    block_sums<NC, W>(q, L.red, L.gam);
#pragma unroll
    for (int j = 0; j < NC; ++j) q[j] = col[j] * f;
    block_sums<NC, W>(q, L.red, L.gam + NC);
  }
  if (t == 0) {
    double smax = 0.0;
    for (int j = 0; j < NC; ++j) smax = fmax(smax, sqrt(L.gam[j]));
    const double thr = 10.0 * (double)(m > n ? m : n) * 0x1p-52 * smax;
    int r = 0;
    double smin = smax;
    for (int j = 0; j < NC; ++j) {
      const double sj = sqrt(L.gam[j]);
      const bool keep = sj > thr && sj > 0.0;
      L.w[j] = keep ? L.gam[NC + j] / L.gam[j] : 0.0;
      if (keep) { ++r; smin = fmin(smin, sj); }
    }
    L.rank = r;
    L.gam[0] = smin > 0.0 ? smax / smin : 0.0;   // condition number of the kept part
  }
  __syncthreads();
  if (t < n) {
    double z = 0.0;
    for (int j = 0; j < NC; ++j) z += L.V[t * NC + L.slot[cur][j]] * L.w[j];
    const double yv = L.D[t] * z;
    L.y[t] = yv;
    a.coef[d.coef0 + t] = yv;
  }
  const double kappa = L.gam[0];
  const int rank = L.rank;
  __syncthreads();
  // residual ||f - A y|| and the count of samples with q(x~) <= 0, from the samples again
  double rs[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (t < m) {
    double p = 0.0, qd = 1.0;
    for (int j = 0; j < n; ++j) {
      const double mo = mono(L.ex + 8 * j, xt, v);
      if (j < d.n_num) p += L.y[j] * mo; else qd += L.y[j] * mo;
    }
    const double r = f - (p - f * (qd - 1.0));
    rs[0] = r * r;
    rs[1] = qd <= 0.0 ? 1.0 : 0.0;
  }
  block_sums<8, W>(rs, L.red, L.gam);
  if (t == 0) {
    klr_fit_info info{};
    if (rank < n) info.status |= KLR_FIT_RANK_DEFICIENT;
    if (m < n) info.status |= KLR_FIT_UNDERDETERMINED;
    if (!converged) info.status |= KLR_FIT_NOT_CONVERGED;
    const int qneg = (int)L.gam[1];
    if (qneg > 0) info.status |= KLR_FIT_Q_NONPOS;
    info.rank = rank;
    info.iters = sweeps;
    info.q_nonpos = qneg;
    info.resid_norm = sqrt(L.gam[0]);
    info.err_est = 0x1p-53 * kappa;
    a.info[fi] = info;
  }
}

template <int NC, int W>
__global__ void __launch_bounds__(W) fit_svd_kernel(FitArgs a, int cls) {
  __shared__ SvdLds<NC, W> L;
  const int fi = blockIdx.x;
  if (fi >= a.n_fits) return;
  const klr_fit_desc d = a.desc[fi];
  const int c = svd_class(a, d);
  if (c == cls) {
    svd_fit<NC, W>(a, fi, L);
  } else if (c < 0 && cls == 0 && threadIdx.x == 0) {
    // outside the limits of this path (n > 48, or more samples than a class holds) or an
    // invalid descriptor: no coefficients
    const int n = d.n_num + d.n_den - 1;
    const bool shape = d.n_num >= 0 && d.n_den >= 1 && n >= 1 && n <= KLR_MAX_UNKNOWNS;
    if (shape && d.coef0 >= 0 && d.coef0 + (int64_t)n <= a.coef_len)
      for (int j = 0; j < n; ++j) a.coef[d.coef0 + j] = 0.0;
    klr_fit_info info{};
    const bool valid = shape && d.m >= 1 && d.v >= 1 && d.v <= KLR_MAX_VARS;
    info.status = valid ? KLR_FIT_UNSUPPORTED : KLR_FIT_BAD_INPUT;
    info.resid_norm = NAN;
    info.err_est = NAN;
    a.info[fi] = info;
  }
}

template <int NC, int W>
hipError_t launch_svd_class(const FitArgs& a, int cls) {
  hipLaunchKernelGGL((fit_svd_kernel<NC, W>), dim3((unsigned)a.n_fits), dim3(W), 0, a.stream, a, cls);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fit_svd(const FitArgs& a) {
  const int t = a.timer ? a.timer->begin(KLR_K_FIT_SOLVE, a.stream) : -1;
  hipError_t e = launch_svd_class<16, 256>(a, 0);
  if (e == hipSuccess) e = launch_svd_class<16, 512>(a, 1);
  if (e == hipSuccess) e = launch_svd_class<16, 1024>(a, 2);
  if (e == hipSuccess) e = launch_svd_class<32, 256>(a, 3);
  if (e == hipSuccess) e = launch_svd_class<32, 512>(a, 4);
  if (e == hipSuccess) e = launch_svd_class<48, 256>(a, 6);
  if (e == hipSuccess) e = launch_svd_class<48, 512>(a, 7);
  if (a.timer) a.timer->end(t, a.stream);
  return e;
}

}  // namespace klr

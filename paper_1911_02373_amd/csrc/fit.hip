// Batched rational least-squares fits, gfx950.
//
// Paper: step 2 ("Rational function estimation") of the section "An Algorithm to Build and
// Deploy a Performance-Predicting Rational Program" and the section "Building a Driver
// Program: Rational function estimation": each low-level metric is fitted by a rational
// function p/q over given monomial sets, as a linear least-squares problem on a Vandermonde-like
// design matrix (ill-conditioned, possibly rank deficient).
//
// One workgroup (4 waves) per fit, one launch per size class of padded width 32, 64, 96, 112 or
// 128 columns (the 96- and 112-column classes at two workgroups per CU); fits small enough for
// one wavefront go to fit_wave.hip.  Persistent workgroups pop fits of their class from a
// longest-first order; the plain schedule launches one workgroup per fit, and workgroups whose
// fit belongs to another class leave at once.  Per fit:
//   1. the samples are staged in chunks of rows as a table of x~_k^p (x~ = x 2^-s exact in
//      FP64; A_ij = x~^e_j, or -f_i x~^e_j for denominator columns), the next chunk's samples
//      being loaded into registers meanwhile; the Gram pass builds each chunk of A in LDS, the
//      refinement and final passes form their elements from the table, sixteen threads per row
//      (column sums in registers until the end of the pass) when every exponent is <= 3;
//   2. Gram G = A^T A on MFMA (16-column tiles dealt to the waves as lower tile pairs; FP64, or
//      FP32 / BF16-rounded inputs with FP32 accumulation) and c = A^T f in FP64;
//   3. power-of-two column equilibration (exact), diagonal shift mu = 8 u tr/n;
//   4. diagonally pivoted Cholesky in FP64 in LDS, kept in pivot order (rows and columns swapped
//      in place); rank = pivots above 4 mu, the rest of the factor sqrt(mu) I;
//   5. z0 = normal-equations solution, then CGLS on min || A D Pi R^-1 w - f ||, i.e. right-
//      preconditioned by the factor, one sweep over the rows per iteration with the FP64
//      residual of the samples kept in the workspace; stop when the delayed Hestenes-Stiefel
//      estimate of ||A (y - y*)|| (error of the fitted linearised values) is <= tol ||f||;
//   6. reduced-precision Gram paths that do not converge are redone with the FP64 Gram;
//   7. epilogue: y = D z, ||f - A y||, count of samples with q(x~_i) <= 0, status.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "internal.hpp"

namespace klr {
namespace {

constexpr int kFitBlock = 256;

// Rows per chunk.  The 96- and 112-column classes are sized so that two workgroups share a CU
// (at most 80 KB of LDS each).
template <int NM>
struct Chunk { static constexpr int CH = 64; };
template <>
struct Chunk<96> { static constexpr int CH = 32; };
template <>
struct Chunk<112> { static constexpr int CH = 16; };
template <>
struct Chunk<128> { static constexpr int CH = 32; };

template <int NM>
struct Lds {
  static constexpr int CH = Chunk<NM>::CH;
  static constexpr int S = 0;                         // packed symmetric NM x NM (doubles)
  static constexpr int A = S + NM * (NM + 1) / 2;     // design-matrix chunk CH x NM
  static constexpr int PT = A + CH * NM;              // powers x~_k^p of the chunk, CH x 8 x 4
  static constexpr int F = PT + CH * 32;              // targets of the chunk
  static constexpr int R = F + CH;                    // residuals of the chunk
  static constexpr int Q = R + CH;                    // A t of the chunk
  static constexpr int V = Q + CH;                    // 10 vectors of NM
  static constexpr int NDOUBLE = V + 10 * NM;
  static constexpr int BYTES = NDOUBLE * 8 + NM * 8 + NM * 4 + 64 + NM * 4;
  // reduction scratch (kFitBlock doubles) shares the power table: no reduction value is kept
  // across a pass over the rows
  static_assert(CH * 32 >= kFitBlock, "reduction scratch must fit in the power table");
  static_assert(CH % 4 == 0 && kFitBlock % CH == 0 && NM % 16 == 0, "chunk and tile shapes");
};

__device__ __forceinline__ int symi(int a, int b) {
  return a >= b ? a * (a + 1) / 2 + b : b * (b + 1) / 2 + a;
}

__device__ __forceinline__ double wave_sum(double v) { return wave_sum_d(v); }

// Deterministic sum over the workgroup (result valid in every thread).
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
}

struct FitCtx {
  int n, n_num, n_den, m, v;
  int64_t x0, f0;
  int64_t r0;      // first row of the fit's private residual scratch in the workspace
  double* S; double* A; double* pt; double* fch; double* rch; double* qch;
  double *D, *c, *z, *t, *s, *p, *g, *gq, *tp;
  double* piv;     // pivots during the factorization, then 1 / L(k, k)
  double* red;
  uint8_t* ex;
  int* perm;
  int* flags;
  uint32_t* ep;    // exponents of column j, two bits per variable (when every exponent <= 3)
  bool pow3;       // every exponent of the fit is <= 3: monomials are products of table entries
};

// Samples of one chunk held in registers (thread t < rows holds row i0 + t), so that the loads
// of the next chunk are in flight while the current one is processed.
struct RowLoad {
  int32_t x[KLR_MAX_VARS];
  double f;
};

__device__ __forceinline__ void load_rows(const FitArgs& a, const FitCtx& C, int i0, int rows, RowLoad& L) {
  const int t = threadIdx.x;
  if (t < rows) {
    const int32_t* xr = a.X + C.x0 + (int64_t)(i0 + t) * C.v;
#pragma unroll
    for (int k = 0; k < KLR_MAX_VARS; ++k) L.x[k] = k < C.v ? xr[k] : 0;
    L.f = a.f[C.f0 + i0 + t];
  }
}

__device__ __forceinline__ int chunk_rows(const FitCtx& C, int i0, int ch) {
  return C.m - i0 < ch ? C.m - i0 : ch;
}

// Stage the loaded rows: scaled variables x~_k and their powers 0..3, and targets.  The
// 0-th power entry of the unused variables k >= v is 1 as well, so a monomial is the product
// of all KLR_MAX_VARS table entries and needs no branch on v.  Returns true if a target is not
// finite; adds the squared targets to *ff when given.
__device__ __forceinline__ bool put_rows(const FitCtx& C, uint64_t sc, int rows, const RowLoad& L,
                                         double* ff = nullptr) {
  bool bad = false;
  const int t = threadIdx.x;
  if (t < rows) {
#pragma unroll
    for (int k = 0; k < KLR_MAX_VARS; ++k) {
      double* pw = C.pt + t * 32 + k * 4;
      pw[0] = 1.0;
      if (k < C.v) {
        const double x = ldexp((double)L.x[k], -(int)(int8_t)(uint8_t)(sc >> (8 * k)));
        const double x2 = x * x;
        pw[1] = x;
        pw[2] = x2;
        pw[3] = x2 * x;
      }
    }
    C.fch[t] = L.f;
    bad = !isfinite(L.f);
    if (ff) *ff += L.f * L.f;
  }
  return bad;
}

// Monomial of column j at staged row i: a product of table entries x~_k^(e_k) when every
// exponent is <= 3, otherwise repeated multiplication by x~_k = pt[i][k][1].
__device__ __forceinline__ double monomial(const FitCtx& C, int i, int j) {
  const double* pw = C.pt + i * 32;
  double mono = 1.0;
  if (C.pow3) {                         // same product order as build_chunk
    const uint32_t w = C.ep[j];
    double pv[KLR_MAX_VARS];
#pragma unroll
    for (int k = 0; k < KLR_MAX_VARS; ++k) pv[k] = pw[k * 4 + ((w >> (2 * k)) & 3u)];
    mono = ((pv[0] * pv[1]) * (pv[2] * pv[3])) * ((pv[4] * pv[5]) * (pv[6] * pv[7]));
  } else {
    const uint8_t* e = C.ex + j * 8;
    for (int k = 0; k < C.v; ++k)
      for (int r = 0; r < e[k]; ++r) mono *= pw[k * 4 + 1];
  }
  return mono;
}

// Design-matrix chunk: A[i][j] for j < n, zero up to the 4-padded width.  Each thread owns one
// column (its exponents are read once) and the rows i = g, g + G, ... of its row group g.
template <int NM, int CHR = Chunk<NM>::CH>
__device__ __forceinline__ void build_chunk(const FitCtx& C, int rows) {
  constexpr int G = kFitBlock / NM;
  const int j = threadIdx.x % NM, g = threadIdx.x / NM;
  const int nb4 = ((C.n + 3) / 4) * 4;
  if (j >= nb4 || g >= G) return;
  if (j >= C.n) {
    for (int i = g; i < rows; i += G) C.A[i * NM + j] = 0.0;
    return;
  }
  const bool num = j < C.n_num;
  if (C.pow3) {
    const uint32_t w = C.ep[j];
    int off[KLR_MAX_VARS];
#pragma unroll
    for (int k = 0; k < KLR_MAX_VARS; ++k) off[k] = k * 4 + (int)((w >> (2 * k)) & 3u);
    constexpr int CH = CHR;
    // all table loads of a row are issued before its products; full chunks skip the row guard
    auto row = [&](int i) {
      const double* pw = C.pt + i * 32;
      double pv[KLR_MAX_VARS];
#pragma unroll
      for (int k = 0; k < KLR_MAX_VARS; ++k) pv[k] = pw[off[k]];
      const double fi = C.fch[i];
      static_assert(KLR_MAX_VARS == 8, "product tree over 8 table entries");
      const double mono = ((pv[0] * pv[1]) * (pv[2] * pv[3])) * ((pv[4] * pv[5]) * (pv[6] * pv[7]));
      C.A[i * NM + j] = num ? mono : -fi * mono;
    };
    if (rows == CH) {
      // four rows per step with every table load issued before the stores (the chunk and the
      // power table are separate LDS arrays, which the compiler cannot see through C)
      constexpr int RPT = CH / G, NB = 2;
      static_assert(RPT % NB == 0, "rows per thread");
#pragma unroll 1
      for (int u0 = 0; u0 < RPT; u0 += NB) {
        double pv[NB][KLR_MAX_VARS], fv[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const double* pw = C.pt + (g + (u0 + b) * G) * 32;
#pragma unroll
          for (int k = 0; k < KLR_MAX_VARS; ++k) pv[b][k] = pw[off[k]];
          fv[b] = C.fch[g + (u0 + b) * G];
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const double mono = ((pv[b][0] * pv[b][1]) * (pv[b][2] * pv[b][3])) *
                              ((pv[b][4] * pv[b][5]) * (pv[b][6] * pv[b][7]));
          C.A[(g + (u0 + b) * G) * NM + j] = num ? mono : -fv[b] * mono;
        }
      }
    } else {
      for (int i = g; i < rows; i += G) row(i);
    }
  } else {
    for (int i = g; i < rows; i += G) {
      const double mono = monomial(C, i, j);
      C.A[i * NM + j] = num ? mono : -C.fch[i] * mono;
    }
  }
}

// Row base of the packed lower triangle: element (i, j), j <= i, is at rbase(i) + j.
__device__ __forceinline__ int rbase(int i) { return i * (i + 1) / 2; }

// Rows per chunk of the Gram pass, which stages its chunks of A and the power table in the LDS
// span of S (written only after the last chunk) and of the usual chunk: a multiple of 16 rows
// whose staging fits in that span, with four rows per thread in each build step.
template <int NM>
struct GramChunk { static constexpr int CH = NM == 112 ? 48 : 64; };

template <int NM>
__device__ __forceinline__ FitCtx gram_staging(const FitCtx& C) {
  constexpr int CH = GramChunk<NM>::CH;
  static_assert(CH * (NM + 32 + 1) <= Lds<NM>::F && CH % 16 == 0, "Gram staging span");
  FitCtx W = C;
  W.A = C.S;                             // the span starts at S
  W.pt = C.S + CH * NM;
  W.fch = W.pt + CH * 32;
  return W;
}

// Gram pass: S (packed lower, unscaled), c = A^T f and ||f||^2 (into *fnorm2).
// GP: Gram precision.  Returns true if a target is not finite.
// S is formed on the matrix cores: the 16-column tiles of A give nt (nt + 1) / 2 lower tile
// pairs, dealt round-robin to the waves; at every step of 4 chunk rows the wave issues one MFMA
// per pair it owns, each lane reading its operand slots (row l / 16, column l % 16 of the two
// tiles) from LDS.  c = A^T f stays in FP64 on the vector units.
template <int NM, int GP>
__device__ __forceinline__ bool gram_pass(const FitArgs& a, const FitCtx& C, uint64_t sc, double* fnorm2) {
  using GT = GramTypes<GP>;
  using acc_t = typename GT::acc_t;
  constexpr int CH = GramChunk<NM>::CH;
  const FitCtx Wc = gram_staging<NM>(C);
  constexpr int NT = NM / 16;                       // column tiles
  constexpr int W = kFitBlock / 64;                 // waves
  constexpr int PPW = (NT * (NT + 1) / 2 + W - 1) / W;
  constexpr int TPC = kFitBlock / NM;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int grp = lane >> 4, col = lane & 15;
  const int nt = (C.n + 15) / 16;
  const int npair = nt * (nt + 1) / 2;
  const int mine = npair > wv ? (npair - wv + W - 1) / W : 0;   // pairs of this wave
  int tj[PPW], tk[PPW];
  acc_t acc[PPW];
#pragma unroll
  for (int q = 0; q < PPW; ++q) {
    const int p = q < mine ? wv + W * q : 0;
    int r = 0;
    while ((r + 1) * (r + 2) / 2 <= p) ++r;
    tj[q] = r;
    tk[q] = p - r * (r + 1) / 2;
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[q][u] = 0;
  }
  const int cj = threadIdx.x % NM, csub = threadIdx.x / NM;
  double cacc = 0.0, ff = 0.0;
  bool bad = false;
  RowLoad rl;
  load_rows(a, C, 0, chunk_rows(C, 0, CH), rl);
  for (int i0 = 0; i0 < C.m; i0 += CH) {
    const int rows = chunk_rows(C, i0, CH);
    const int rows4 = (rows + 3) & ~3;
    bad |= put_rows(Wc, sc, rows, rl, &ff);
    if (i0 + CH < C.m) load_rows(a, C, i0 + CH, chunk_rows(C, i0 + CH, CH), rl);
    __syncthreads();
    build_chunk<NM, CH>(Wc, rows);
    for (int e = threadIdx.x; e < (rows4 - rows) * NM; e += kFitBlock) Wc.A[rows * NM + e] = 0.0;
    __syncthreads();
    // blocks of 4 SUB rows: sub-step e gives reduction slot e the block's row 4 e + grp
    for (int i = 0; i < rows4; i += 4 * GT::SUB) {
      typename GT::op_t xa[PPW], xb[PPW];
#pragma unroll
      for (int q = 0; q < PPW; ++q) xa[q] = xb[q] = GT::zero();
#pragma unroll
      for (int e = 0; e < GT::SUB; ++e) {
        if (i + 4 * e < rows4) {
          const double* ar = Wc.A + (i + 4 * e + grp) * NM + col;
#pragma unroll
          for (int q = 0; q < PPW; ++q) {
            GT::put(xa[q], e, ar[16 * tj[q]]);
            GT::put(xb[q], e, ar[16 * tk[q]]);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < PPW; ++q)
        if (q < mine) acc[q] = GT::mma(xa[q], xb[q], acc[q]);
    }
    if (cj < C.n && csub < TPC) {
#pragma unroll 4
      for (int u = 0; u < CH / TPC; ++u) {
        const int i = csub + u * TPC;
        if (i < rows) cacc += Wc.A[i * NM + cj] * Wc.fch[i];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < PPW; ++q) {
    if (q < mine) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = 16 * tj[q] + GT::out_row(grp, r), k = 16 * tk[q] + col;
        if (j < C.n && k <= j) C.S[rbase(j) + k] = (double)acc[q][r];
      }
    }
  }
  C.red[threadIdx.x] = cacc;
  __syncthreads();
  if ((int)threadIdx.x < C.n) {
    double v = 0.0;
    for (int s2 = 0; s2 < TPC; ++s2) v += C.red[threadIdx.x + s2 * NM];
    C.c[threadIdx.x] = v;
  }
  if (bad) C.flags[0] = 1;
  *fnorm2 = block_sum(ff, C.red);
  return C.flags[0] != 0;
}

// Forward solve L u = in[perm[.]] by wave 0 (L in pivot order, see factor).  out is
// pivot-indexed.  A lane holds the right-hand side of rows lane and lane + 64.  Step k reads b_k,
// forms u_k = b_k / L(k, k) (a product with the stored reciprocal) and subtracts L(i, k) u_k from
// the rows i > k (the factor entry of rows i <= k is taken as zero, which leaves them unchanged
// while u_k is finite); row k keeps b_k, and every u_k is formed again at the end from the same
// operands.  Rows past n hold values that are never read or stored.
__device__ __forceinline__ void solve_fwd(const FitCtx& C, const double* in, double* out) {
  const int lane = threadIdx.x & 63;
  const int n = __builtin_amdgcn_readfirstlane(C.n);
  const int r1 = lane + 64;
  const int b0r = rbase(lane < n ? lane : 0), b1r = rbase(r1 < n ? r1 : 0);
  double b0 = lane < n ? in[C.perm[lane]] : 0.0;
  double b1 = r1 < n ? in[C.perm[r1]] : 0.0;
  const int n0 = n < 64 ? n : 64;
  // steps 0 .. 63 update both rows of a lane; the factor entries of a group of four steps are
  // loaded before its dependent chain
  for (int k0 = 0; k0 < n0; k0 += 4) {
    double rp[4], s0[4], s1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + u < n0 ? k0 + u : n0 - 1;
      rp[u] = C.piv[k];
      s0[u] = lane > k ? C.S[b0r + k] : 0.0;
      s1[u] = C.S[b1r + k];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + u;
      if (k < n0) {
        const double uk = readlane_d(b0, k) * rp[u];
        b0 -= s0[u] * uk;
        b1 -= s1[u] * uk;
      }
    }
  }
  // steps 64 .. n - 1: the first row of every lane is final
  for (int k0 = 64; k0 < n; k0 += 4) {
    double rp[4], s1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + u < n ? k0 + u : n - 1;
      rp[u] = C.piv[k];
      s1[u] = r1 > k ? C.S[b1r + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + u;
      if (k < n) {
        const double uk = readlane_d(b1, k - 64) * rp[u];
        b1 -= s1[u] * uk;
      }
    }
  }
  if (lane < n) out[lane] = b0 * C.piv[lane];
  if (r1 < n) out[r1] = b1 * C.piv[r1];
}

// Backward solve L^T v = in (pivot-indexed) by wave 0; out[perm[i]] = v_i.  Step k (from n - 1
// down) forms v_k = b_k / L(k, k) and subtracts L(k, i) v_k from the rows i < k; as in the
// forward solve, row k keeps b_k and the v_k are formed again at the end.
__device__ __forceinline__ void solve_bwd(const FitCtx& C, const double* in, double* out) {
  const int lane = threadIdx.x & 63;
  const int n = __builtin_amdgcn_readfirstlane(C.n);
  const int r1 = lane + 64;
  double b0 = lane < n ? in[lane] : 0.0;
  double b1 = r1 < n ? in[r1] : 0.0;
  // steps n - 1 .. 64: every first row lies below k; second rows below k only
  for (int k0 = n - 1; k0 >= 64; k0 -= 4) {
    double rp[4], s0[4], s1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 - u >= 64 ? k0 - u : 64;
      const int rk = rbase(k);
      rp[u] = C.piv[k];
      s0[u] = C.S[rk + lane];
      s1[u] = r1 < k ? C.S[rk + r1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 - u;
      if (k >= 64) {
        const double vk = readlane_d(b1, k - 64) * rp[u];
        b0 -= s0[u] * vk;
        b1 -= s1[u] * vk;
      }
    }
  }
  // steps min(n, 64) - 1 .. 0: only first rows lie below k
  for (int k0 = (n < 64 ? n : 64) - 1; k0 >= 0; k0 -= 4) {
    double rp[4], s0[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 - u >= 0 ? k0 - u : 0;
      rp[u] = C.piv[k];
      s0[u] = lane < k ? C.S[rbase(k) + lane] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 - u;
      if (k >= 0) {
        const double vk = readlane_d(b0, k) * rp[u];
        b0 -= s0[u] * vk;
      }
    }
  }
  if (lane < n) out[C.perm[lane]] = b0 * C.piv[lane];
  if (r1 < n) out[C.perm[r1]] = b1 * C.piv[r1];
}

// sum_j x_j y_j over n entries, by wave 0 (valid in wave 0).
__device__ __forceinline__ double dot_w0(const double* x, const double* y, int n) {
  const int lane = threadIdx.x & 63;
  double v = 0.0;
  for (int j = lane; j < n; j += 64) v += x[j] * y[j];
  return wave_sum(v);
}

// Final pass: returns sum (f_i - d_i)^2 with d = A tp (tp holds y) and counts the samples with
// q(x~_i) <= 0 into *qneg_out.
template <int NM>
__device__ __forceinline__ double final_pass(const FitArgs& a, const FitCtx& C, uint64_t sc, int* qneg_out) {
  constexpr int CH = Chunk<NM>::CH;
  constexpr int TPR = kFitBlock / CH;
  const int i = threadIdx.x / TPR, sub = threadIdx.x % TPR;
  double acc = 0.0;
  int qneg = 0;
  RowLoad rl;
  load_rows(a, C, 0, chunk_rows(C, 0, CH), rl);
  for (int i0 = 0; i0 < C.m; i0 += CH) {
    const int rows = chunk_rows(C, i0, CH);
    put_rows(C, sc, rows, rl);
    if (i0 + CH < C.m) load_rows(a, C, i0 + CH, chunk_rows(C, i0 + CH, CH), rl);
    __syncthreads();
    build_chunk<NM>(C, rows);
    __syncthreads();
    // d_i = A_i tp and q(x~_i) - 1, each split over the TPR threads of row i
    double dsum = 0.0, qs = 0.0;
    if (i < rows) {
#pragma unroll 4
      for (int u = 0; u < NM / TPR; ++u) {
        const int j = sub + u * TPR;
        if (j < C.n) dsum += C.A[i * NM + j] * C.tp[j];
      }
      for (int j = C.n_num + sub; j < C.n; j += TPR) qs += C.tp[j] * monomial(C, i, j);
    }
    dsum = group_sum<TPR>(dsum);
    qs = group_sum<TPR>(qs);
    if (i < rows && sub == 0) {
      const double res = C.fch[i] - dsum;
      acc += res * res;
      const double qv = 1.0 + qs;
      if (!(qv > 0.0)) ++qneg;
    }
    __syncthreads();
  }
  const double qn = block_sum((double)qneg, C.red);
  *qneg_out = (int)qn;
  return block_sum(acc, C.red);
}

enum CgMode { kR0 = 0, kQ = 1 };

// One sweep over the fit's rows for the refinement, each chunk of A built once:
//   kR0: r = f - A tp (stored), C.g = A^T r;
//   kQ : when `upd`, r = r - alpha_prev q_prev (the residual update of the previous iteration,
//        applied to the stored rows first); q = A tp (stored), C.g = A^T r, C.gq = A^T q;
//        returns ||q||^2.
// The caller forms D A^T r_next = D (C.g - alpha C.gq) once alpha is known, so every iteration
// reads the FP64 residual of the samples and builds each chunk once.
template <int NM, int MODE>
__device__ __forceinline__ double cg_pass(const FitArgs& a, const FitCtx& C, uint64_t sc, double* wsr, double* wsq,
                          bool upd, double alpha_prev) {
  constexpr int CH = Chunk<NM>::CH;
  constexpr int TPR = kFitBlock / CH;
  constexpr int TPC = kFitBlock / NM;
  const int ri = threadIdx.x / TPR, rsub = threadIdx.x % TPR;
  const int cj = threadIdx.x % NM, csub = threadIdx.x / NM;
  double accr = 0.0, accq = 0.0, qq = 0.0;
  RowLoad rl;
  load_rows(a, C, 0, chunk_rows(C, 0, CH), rl);
  // kQ: the stored residual and previous image of the row are read one chunk ahead by the
  // thread that owns the row (the one that wrote them)
  const bool owner = rsub == 0;
  double rn = 0.0, qn = 0.0;
  if (MODE == kQ && owner && ri < chunk_rows(C, 0, CH)) {
    rn = wsr[C.r0 + ri];
    if (upd) qn = wsq[C.r0 + ri];
  }
  for (int i0 = 0; i0 < C.m; i0 += CH) {
    const int rows = chunk_rows(C, i0, CH);
    put_rows(C, sc, rows, rl);
    double rn2 = 0.0, qn2 = 0.0;
    if (i0 + CH < C.m) {
      const int rows2 = chunk_rows(C, i0 + CH, CH);
      load_rows(a, C, i0 + CH, rows2, rl);
      if (MODE == kQ && owner && ri < rows2) {
        rn2 = wsr[C.r0 + i0 + CH + ri];
        if (upd) qn2 = wsq[C.r0 + i0 + CH + ri];
      }
    }
    __syncthreads();
    build_chunk<NM>(C, rows);
    __syncthreads();
    double dsum = 0.0;
    if (ri < rows) {
#pragma unroll 4
      for (int u = 0; u < NM / TPR; ++u) {
        const int j = rsub + u * TPR;
        if (j < C.n) dsum += C.A[ri * NM + j] * C.tp[j];
      }
    }
    dsum = group_sum<TPR>(dsum);
    if (ri < rows && rsub == 0) {
      const int64_t row = C.r0 + i0 + ri;
      if (MODE == kR0) {
        const double r = C.fch[ri] - dsum;
        wsr[row] = r;
        C.rch[ri] = r;
      } else {
        double r = rn;
        if (upd) {
          r -= alpha_prev * qn;
          wsr[row] = r;
        }
        C.rch[ri] = r;
        C.qch[ri] = dsum;
        wsq[row] = dsum;
        qq += dsum * dsum;
      }
    }
    __syncthreads();
    if (cj < C.n && csub < TPC) {
#pragma unroll 4
      for (int u = 0; u < CH / TPC; ++u) {
        const int i = csub + u * TPC;
        if (i < rows) {
          const double av = C.A[i * NM + cj];
          accr += av * C.rch[i];
          if (MODE == kQ) accq += av * C.qch[i];
        }
      }
    }
    __syncthreads();
    rn = rn2;
    qn = qn2;
  }
  C.red[threadIdx.x] = accr;
  __syncthreads();
  if ((int)threadIdx.x < C.n) {
    double v = 0.0;
    for (int s2 = 0; s2 < TPC; ++s2) v += C.red[threadIdx.x + s2 * NM];
    C.g[threadIdx.x] = v;
  }
  __syncthreads();
  if (MODE == kQ) {
    C.red[threadIdx.x] = accq;
    __syncthreads();
    if ((int)threadIdx.x < C.n) {
      double v = 0.0;
      for (int s2 = 0; s2 < TPC; ++s2) v += C.red[threadIdx.x + s2 * NM];
      C.gq[threadIdx.x] = v;
    }
    __syncthreads();
    return block_sum(qq, C.red);
  }
  return 0.0;
}

// ---- row-parallel passes (every exponent of the fit <= 3) --------------------------------------
// Sixteen threads share a row: thread `sub` owns the columns j = sub + 16 u (u < NM / 16) and
// forms their design-matrix elements straight from the row's power table, so no chunk of A is
// staged.  A t is a sum over the sixteen threads of the row (DPP); the column sums A^T r and
// A^T q stay in registers for the whole pass and are reduced once at its end.  Each chunk needs
// one barrier after its rows are staged and one before they are overwritten.

// Byte offsets of a column's table entries k * 4 + e_k (one byte each: variables 0-3 in o0,
// 4-7 in o1).
__device__ __forceinline__ void col_offsets(uint32_t w, uint32_t& o0, uint32_t& o1) {
  o0 = 0;
  o1 = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    o0 |= (uint32_t)((k * 4 + (int)((w >> (2 * k)) & 3u)) * 8) << (8 * k);
    o1 |= (uint32_t)(((k + 4) * 4 + (int)((w >> (2 * (k + 4))) & 3u)) * 8) << (8 * k);
  }
}

// Monomial of one column at a staged row: the product tree of build_chunk over the eight table
// entries.  VV = 4: variables 4-7 are unused, their entries are exactly 1 and the tree reduces
// exactly to (p0 p1)(p2 p3).
template <int VV>
__device__ __forceinline__ double row_mono(const double* pw, uint32_t o0, uint32_t o1) {
  const char* b = reinterpret_cast<const char*>(pw);
  double p[8];
#pragma unroll
  for (int k = 0; k < 4; ++k) p[k] = *reinterpret_cast<const double*>(b + ((o0 >> (8 * k)) & 255u));
  if (VV <= 4) return (p[0] * p[1]) * (p[2] * p[3]);
#pragma unroll
  for (int k = 0; k < 4; ++k) p[4 + k] = *reinterpret_cast<const double*>(b + ((o1 >> (8 * k)) & 255u));
  return ((p[0] * p[1]) * (p[2] * p[3])) * ((p[4] * p[5]) * (p[6] * p[7]));
}

// The row-parallel passes stage kRowChunk rows at a time in the LDS span of the Gram pass's
// chunk of A and its power table (free outside the Gram pass): tables from the start of the
// span, targets after them.
constexpr int kRowChunk = 64;
template <int NM>
__device__ __forceinline__ FitCtx row_staging(const FitCtx& C) {
  static_assert((Lds<NM>::PT - Lds<NM>::A) + Lds<NM>::CH * 32 >= kRowChunk * 33, "row staging span");
  FitCtx W = C;
  W.pt = C.A;
  W.fch = C.A + kRowChunk * 32;
  return W;
}

// Per-thread column set of the row-parallel passes.
template <int NM>
struct RowCols {
  static constexpr int CPT = NM / 16;
  uint32_t o0[CPT], o1[CPT];
  double tpj[CPT];     // tp of the column (0 past n)
  bool num[CPT];       // numerator column
  __device__ __forceinline__ void load(const FitCtx& C, int sub) {
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int j = sub + 16 * u;
      col_offsets(j < C.n ? C.ep[j] : 0u, o0[u], o1[u]);
      tpj[u] = j < C.n ? C.tp[j] : 0.0;
      num[u] = j < C.n_num;
    }
  }
};

// Column sums of the row-parallel passes: the four lanes of a wave that own the same columns
// are summed by lane swaps, then the four waves through LDS scratch (the chunk region of A,
// which these passes do not use), in a fixed order.
template <int NM>
__device__ __forceinline__ void col_reduce(const FitCtx& C, const double* acc, double* out) {
  constexpr int CPT = NM / 16;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, sub = threadIdx.x & 15;
#pragma unroll
  for (int u = 0; u < CPT; ++u) {
    const double v = pair_sum32(pair_sum16(acc[u]));
    if (lane < 16) C.A[(w * CPT + u) * 16 + sub] = v;
  }
  __syncthreads();
  const int j = threadIdx.x;
  if (j < C.n) {
    const int u = j >> 4, sj = j & 15;
    out[j] = (C.A[(0 * CPT + u) * 16 + sj] + C.A[(1 * CPT + u) * 16 + sj]) +
             (C.A[(2 * CPT + u) * 16 + sj] + C.A[(3 * CPT + u) * 16 + sj]);
  }
  __syncthreads();
}

// The refinement sweep of cg_pass (same modes and outputs) in the row-parallel form.
template <int NM, int MODE, int VV>
__device__ __forceinline__ double cg_rows(const FitArgs& a, const FitCtx& C, uint64_t sc, double* wsr, double* wsq,
                                          bool upd, double alpha_prev) {
  constexpr int CH = kRowChunk;
  constexpr int CPT = NM / 16;
  constexpr int RPC = CH / 16;                      // rows per thread and chunk
  static_assert(CH % 16 == 0 && NM % 16 == 0, "row groups");
  const int sub = threadIdx.x & 15, rg = threadIdx.x >> 4;
  const FitCtx W = row_staging<NM>(C);
  RowCols<NM> cs;
  cs.load(C, sub);
  double accr[CPT], accq[CPT];
#pragma unroll
  for (int u = 0; u < CPT; ++u) accr[u] = accq[u] = 0.0;
  double qq = 0.0;
  RowLoad rl;
  load_rows(a, C, 0, chunk_rows(C, 0, CH), rl);
  for (int i0 = 0; i0 < C.m; i0 += CH) {
    const int rows = chunk_rows(C, i0, CH);
    put_rows(W, sc, rows, rl);
    if (i0 + CH < C.m) load_rows(a, C, i0 + CH, chunk_rows(C, i0 + CH, CH), rl);
    double rv[RPC], qv[RPC];
#pragma unroll
    for (int s2 = 0; s2 < RPC; ++s2) {
      const int i = rg + 16 * s2;
      rv[s2] = 0.0;
      qv[s2] = 0.0;
      if (MODE == kQ && i < rows) {
        rv[s2] = wsr[C.r0 + i0 + i];
        if (upd) qv[s2] = wsq[C.r0 + i0 + i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int s2 = 0; s2 < RPC; ++s2) {
      const int i = rg + 16 * s2;
      const bool live = i < rows;
      const double* pw = W.pt + (live ? i : 0) * 32;
      const double fi = W.fch[live ? i : 0];
      double mv[CPT];
      double dsum = 0.0;
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const double mo = row_mono<VV>(pw, cs.o0[u], cs.o1[u]);
        mv[u] = cs.num[u] ? mo : -fi * mo;
        dsum += mv[u] * cs.tpj[u];
      }
      dsum = group_sum<16>(live ? dsum : 0.0);
      if (live) {
        const int64_t row = C.r0 + i0 + i;
        double r, q = dsum;
        if (MODE == kR0) {
          r = fi - dsum;
          if (sub == 0) wsr[row] = r;
        } else {
          r = rv[s2];
          if (upd) {
            r -= alpha_prev * qv[s2];
            if (sub == 0) wsr[row] = r;
          }
          if (sub == 0) {
            wsq[row] = q;
            qq += q * q;
          }
        }
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
          accr[u] += mv[u] * r;
          if (MODE == kQ) accq[u] += mv[u] * q;
        }
      }
    }
    __syncthreads();
  }
  col_reduce<NM>(C, accr, C.g);
  if (MODE == kQ) {
    col_reduce<NM>(C, accq, C.gq);
    return block_sum(qq, C.red);
  }
  return 0.0;
}

// final_pass in the row-parallel form.
template <int NM, int VV>
__device__ __forceinline__ double final_rows(const FitArgs& a, const FitCtx& C, uint64_t sc, int* qneg_out) {
  constexpr int CH = kRowChunk;
  constexpr int CPT = NM / 16;
  constexpr int RPC = CH / 16;
  const int sub = threadIdx.x & 15, rg = threadIdx.x >> 4;
  const FitCtx W = row_staging<NM>(C);
  RowCols<NM> cs;
  cs.load(C, sub);
  double acc = 0.0;
  int qneg = 0;
  RowLoad rl;
  load_rows(a, C, 0, chunk_rows(C, 0, CH), rl);
  for (int i0 = 0; i0 < C.m; i0 += CH) {
    const int rows = chunk_rows(C, i0, CH);
    put_rows(W, sc, rows, rl);
    if (i0 + CH < C.m) load_rows(a, C, i0 + CH, chunk_rows(C, i0 + CH, CH), rl);
    __syncthreads();
#pragma unroll
    for (int s2 = 0; s2 < RPC; ++s2) {
      const int i = rg + 16 * s2;
      const bool live = i < rows;
      const double* pw = W.pt + (live ? i : 0) * 32;
      const double fi = W.fch[live ? i : 0];
      double dsum = 0.0, qs = 0.0;
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const double mo = row_mono<VV>(pw, cs.o0[u], cs.o1[u]);
        const double av = cs.num[u] ? mo : -fi * mo;
        dsum += av * cs.tpj[u];
        if (!cs.num[u]) qs += cs.tpj[u] * mo;
      }
      dsum = group_sum<16>(live ? dsum : 0.0);
      qs = group_sum<16>(live ? qs : 0.0);
      if (live && sub == 0) {
        const double res = fi - dsum;
        acc += res * res;
        const double qv = 1.0 + qs;
        if (!(qv > 0.0)) ++qneg;
      }
    }
    __syncthreads();
  }
  const double qn = block_sum((double)qneg, C.red);
  *qneg_out = (int)qn;
  return block_sum(acc, C.red);
}

// Pass selection: the row-parallel form when every exponent is <= 3, else the chunked one.
template <int NM, int MODE>
__device__ __forceinline__ double cg_sweep(const FitArgs& a, const FitCtx& C, uint64_t sc, double* wsr, double* wsq,
                                           bool upd, double alpha_prev) {
  if (C.pow3) return C.v <= 4 ? cg_rows<NM, MODE, 4>(a, C, sc, wsr, wsq, upd, alpha_prev)
                              : cg_rows<NM, MODE, 8>(a, C, sc, wsr, wsq, upd, alpha_prev);
  return cg_pass<NM, MODE>(a, C, sc, wsr, wsq, upd, alpha_prev);
}

template <int NM>
__device__ __forceinline__ double final_sweep(const FitArgs& a, const FitCtx& C, uint64_t sc, int* qneg_out) {
  if (C.pow3) return C.v <= 4 ? final_rows<NM, 4>(a, C, sc, qneg_out) : final_rows<NM, 8>(a, C, sc, qneg_out);
  return final_pass<NM>(a, C, sc, qneg_out);
}

// Equilibrate, shift and factor S.  Returns the numerical rank.  The factor is kept in pivot
// order: at step k the rows and columns k and bi are swapped in place (the computed part of L
// and the Schur complement alike), so element (i, j) of L is at rbase(i) + j and perm maps a
// pivot position to the original column.
__device__ __forceinline__ int factor(const FitCtx& C, double unit) {
  const int n = C.n;
  const int tid = threadIdx.x;
  if (tid < n) {
    const double gjj = C.S[rbase(tid) + tid];
    int e = 0;
    if (gjj > 0.0 && isfinite(gjj)) frexp(sqrt(gjj), &e);
    C.D[tid] = ldexp(1.0, -e);
    C.perm[tid] = tid;
  }
  __syncthreads();
  {                                    // rows over a 16 x 16 thread grid, loads before stores
    const int ty = tid >> 4, tx = tid & 15;
    for (int i = ty; i < n; i += 16) {
      const int rb = rbase(i);
      const double di = C.D[i];
      double sv[8], dv[8];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int j = tx + 16 * b, jj = j <= i ? j : 0;
        sv[b] = C.S[rb + jj];
        dv[b] = C.D[jj];
      }
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int j = tx + 16 * b;
        if (j <= i) C.S[rb + j] = sv[b] * (di * dv[b]);
      }
    }
    if (tid < n) C.c[tid] *= C.D[tid];
  }
  __syncthreads();
  if (tid < 64) {
    double tr = 0.0;
    for (int j = tid; j < n; j += 64) tr += C.S[rbase(j) + j];
    tr = wave_sum(tr);
    if (tid == 0) C.red[kFitBlock - 1] = 8.0 * unit * tr / n + 1e-300;
  }
  __syncthreads();
  const double mu = C.red[kFitBlock - 1];
  // the diagonal of the Schur complement, kept apart from S (C.t is free during the
  // factorization) and updated column by column
  double* const dg = C.t;
  if (tid < n) {
    const double dv = C.S[rbase(tid) + tid] + mu;
    C.S[rbase(tid) + tid] = dv;
    dg[tid] = dv;
  }
  __syncthreads();
  // Blocked, left-looking: panels of kPanel columns.  Step k of a panel: (A) every wave picks
  // the largest remaining diagonal; (B) symmetric swap of positions k and bi (the computed part of
  // L and the not yet updated trailing part alike, so L(i, j) sits at rbase(i) + j in pivot
  // order); (C) column k of L: S(i, k) less the products of the panel's earlier columns, over
  // L(k, k), one thread per row, and the diagonal loses its square.  After the panel the
  // trailing triangle takes the panel's rank-kPanel product in one pass (16 x 16 thread grid).
  constexpr int kPanel = 16;
  const int ty = tid >> 4, tx = tid & 15;
  bool stopped = false;
  for (int k0 = 0; k0 < n && !stopped; k0 += kPanel) {
    const int kend = k0 + kPanel < n ? k0 + kPanel : n;
    for (int k = k0; k < kend; ++k) {
      // every wave picks the pivot itself (the same pick in each: dg is written only in phase
      // (C), behind a barrier): the largest remaining diagonal, lowest index on ties; NaN
      // ranks below every number, so the pick is always one of the remaining positions k..n-1
      double best = -INFINITY;
      int bi = n;
      for (int i = k + (tid & 63); i < n; i += 64) {
        const double vv = dg[i];
        const double key = vv == vv ? vv : -INFINITY;
        argmax_take(best, bi, key, i);
      }
      wave_argmax(best, bi);
      bi = __builtin_amdgcn_readfirstlane(bi);
      if (!(best > 4.0 * mu)) {
        // numerical rank reached: every remaining diagonal is at most 4 mu, i.e. the remaining
        // Schur complement is rounding noise; the rest of the factor becomes sqrt(mu) I (the
        // shift alone), so the noise is never divided by a tiny pivot
        const double smu = sqrt(mu);
        const int i = k + tid;
        if (i < n) {
          const int rb = rbase(i);
          C.piv[i] = dg[i];
          for (int j = k; j < i; ++j) C.S[rb + j] = 0.0;
          C.S[rb + i] = smu;
        }
        __syncthreads();
        stopped = true;
        break;
      }
      if (bi != k) {                   // symmetric swap of positions k < bi
        const int ba = rbase(k), bb = rbase(bi);
        const int i = tid;
        int p0 = -1, p1 = -1;
        if (i < k) { p0 = ba + i; p1 = bb + i; }
        else if (i == k) { p0 = ba + k; p1 = bb + bi; }
        else if (i < bi) { p0 = rbase(i) + k; p1 = bb + i; }
        else if (i > bi && i < n) { p0 = rbase(i) + k; p1 = rbase(i) + bi; }
        if (p0 >= 0) {
          const double t0 = C.S[p0], t1 = C.S[p1];
          C.S[p0] = t1;
          C.S[p1] = t0;
        }
        if (tid == 0) {
          const int t = C.perm[k];
          C.perm[k] = C.perm[bi];
          C.perm[bi] = t;
        }
      }
      __syncthreads();
      const double lkk = sqrt(best);
      if (tid == 0) {                  // nothing reads (k, k) in this step
        C.piv[k] = best;
        C.S[rbase(k) + k] = lkk;
      }
      {
        const int i = k + 1 + tid;     // rows k+1.. (n <= 128)
        if (i < n) {
          const int rb = rbase(i), rk = rbase(k);
          double lv[kPanel - 1], kv[kPanel - 1];
#pragma unroll
          for (int p = 0; p < kPanel - 1; ++p) {
            const bool in = k0 + p < k;
            lv[p] = in ? C.S[rb + k0 + p] : 0.0;
            kv[p] = in ? C.S[rk + k0 + p] : 0.0;
          }
          double acc = C.S[rb + k];
#pragma unroll
          for (int p = 0; p < kPanel - 1; ++p)
            if (k0 + p < k) acc -= lv[p] * kv[p];
          const double l = acc / lkk;
          C.S[rb + k] = l;
          dg[i] = (i == bi ? dg[k] : dg[i]) - l * l;   // position bi now holds old position k
        }
      }
      __syncthreads();
    }
    if (stopped || kend >= n) continue;
    // trailing update: S(i, j) -= sum over the panel of L(i, p) L(j, p), kend <= j <= i
    for (int i = kend + ty; i < n; i += 16) {
      const int rb = rbase(i);
      double li[kPanel];
#pragma unroll
      for (int p = 0; p < kPanel; ++p) li[p] = k0 + p < kend ? C.S[rb + k0 + p] : 0.0;
#pragma unroll 2
      for (int c = 0; c < 8; ++c) {
        const int j = kend + tx + 16 * c;
        if (j <= i) {
          const int rj = rbase(j);
          double lj[kPanel];
#pragma unroll
          for (int p = 0; p < kPanel; ++p) lj[p] = k0 + p < kend ? C.S[rj + k0 + p] : 0.0;
          double acc = C.S[rb + j];
#pragma unroll
          for (int p = 0; p < kPanel; ++p) acc -= li[p] * lj[p];
          C.S[rb + j] = acc;
        }
      }
    }
    __syncthreads();
  }
  int rank = 0;
  for (int k = 0; k < n; ++k) rank += C.piv[k] > 4.0 * mu ? 1 : 0;
  __syncthreads();
  if (tid < n) C.piv[tid] = 1.0 / C.S[rbase(tid) + tid];   // the solves multiply by 1 / L(k, k)
  __syncthreads();
  return rank;
}

// Size class of a fit: kWaveClass (8 rows per lane) and kWaveClass16 (16) = one wavefront per
// fit (fit_wave.hip); otherwise one workgroup per fit with padded width 32 (class 0), 64 (1),
// 96 (2), 112 (3) or 128 (4, which also takes every invalid descriptor and reports it as bad
// input).
constexpr int kWaveClass = 5;
constexpr int kWaveClass16 = 6;
__device__ __forceinline__ int fit_class(const FitArgs& a, const klr_fit_desc& d) {
  const int rpl = wave_fit_rows(a, d);
  if (rpl == 8) return kWaveClass;
  if (rpl == 16) return kWaveClass16;
  const int n = d.n_num + d.n_den - 1;
  const bool shape_ok = d.n_num >= 0 && d.n_den >= 1 && n >= 1 && n <= KLR_MAX_UNKNOWNS;
  if (!shape_ok) return 4;
  return n <= 32 ? 0 : (n <= 64 ? 1 : (n <= 96 ? 2 : (n <= 112 ? 3 : 4)));
}

// One fit by the whole workgroup (all threads call it with the same fi).
template <int NM, int PREC>
__device__ __forceinline__ void fit_one(const FitArgs& a, int fi, double* smem) {
  using L = Lds<NM>;
  const klr_fit_desc d = a.desc[fi];
  const int n = d.n_num + d.n_den - 1;
  const bool shape_ok = d.n_num >= 0 && d.n_den >= 1 && n >= 1 && n <= KLR_MAX_UNKNOWNS;
  const int tid = threadIdx.x;
  bool ok = shape_ok && d.v >= 1 && d.v <= KLR_MAX_VARS && d.m >= 1 && d.m <= KLR_MAX_SAMPLES &&
            d.x0 >= 0 && d.x0 + (int64_t)d.m * d.v <= a.x_len && d.f0 >= 0 &&
            d.f0 + (int64_t)d.m <= a.f_len && d.num0 >= 0 &&
            (int64_t)d.num0 + d.n_num <= a.n_exp_rows && d.den0 >= 0 &&
            (int64_t)d.den0 + d.n_den <= a.n_exp_rows;
  const bool coef_ok = shape_ok && d.coef0 >= 0 && d.coef0 + (int64_t)n <= a.coef_len;
  ok = ok && coef_ok;
  if (ok)
    for (int k = 0; k < d.v; ++k) {
      if (d.scale_exp[k] < -100 || d.scale_exp[k] > 100) ok = false;
      if (a.exps[(int64_t)d.den0 * KLR_MAX_VARS + k] != 0) ok = false;
    }

  FitCtx C;
  C.n = n; C.n_num = d.n_num; C.n_den = d.n_den; C.m = d.m; C.v = d.v; C.x0 = d.x0; C.f0 = d.f0;
  // private residual rows: an exclusive prefix of m over the fits of the workgroup classes, so
  // fits that share targets never share scratch; a workspace sized for fewer rows than the
  // fits need is reported per fit
  C.r0 = a.rowoff[fi];
  const bool scratch_ok = C.r0 >= 0 && C.r0 + (int64_t)(d.m > 0 ? d.m : 0) <= a.scratch_rows;
  C.S = smem + L::S; C.A = smem + L::A; C.pt = smem + L::PT; C.fch = smem + L::F; C.rch = smem + L::R;
  C.qch = smem + L::Q;
  double* V = smem + L::V;
  C.D = V; C.c = V + NM; C.z = V + 2 * NM; C.t = V + 3 * NM; C.s = V + 4 * NM; C.p = V + 5 * NM;
  C.g = V + 6 * NM; C.tp = V + 7 * NM; C.piv = V + 8 * NM; C.gq = V + 9 * NM;
  C.red = smem + L::PT;
  C.ex = reinterpret_cast<uint8_t*>(smem + L::NDOUBLE);
  C.perm = reinterpret_cast<int*>(C.ex + NM * 8);
  C.flags = C.perm + NM;
  C.ep = reinterpret_cast<uint32_t*>(C.flags + 16);

  klr_fit_info info{};
  if (tid == 0) { C.flags[0] = 0; C.flags[1] = 0; }
  __syncthreads();
  if (ok && tid < n) {
    const int row = tid < d.n_num ? d.num0 + tid : d.den0 + (tid - d.n_num + 1);
    uint32_t w = 0;
    bool big = false;
    for (int k = 0; k < KLR_MAX_VARS; ++k) {
      const int e = k < d.v ? (int)a.exps[(int64_t)row * KLR_MAX_VARS + k] : 0;
      C.ex[tid * 8 + k] = (uint8_t)e;
      w |= (uint32_t)(e & 3) << (2 * k);
      big |= e > 3;
    }
    C.ep[tid] = w;
    if (big) atomicOr(&C.flags[1], 1);
  }
  __syncthreads();
  C.pow3 = C.flags[1] == 0;
  uint64_t sc = 0;                     // scale exponents s_k, one byte each
#pragma unroll
  for (int k = 0; k < KLR_MAX_VARS; ++k) sc |= (uint64_t)(uint8_t)d.scale_exp[k] << (8 * k);
  double* wsr = a.scratch;
  double* wsq = wsr + a.scratch_rows;

  bool bad = !ok || !scratch_ok;
  int prec = PREC;
  int iters = 0, rank = 0;
  bool converged = false;
  double err = 0.0;
  for (int attempt = 0; attempt < 2 && !bad; ++attempt) {
    bool fbad;
    double unit, fn2 = 0.0;
    if (prec == KLR_FP64) { fbad = gram_pass<NM, KLR_FP64>(a, C, sc, &fn2); unit = 0x1p-53; }
    else if (prec == KLR_FP32_REFINED) { fbad = gram_pass<NM, KLR_FP32_REFINED>(a, C, sc, &fn2); unit = 0x1p-24; }
    else { fbad = gram_pass<NM, KLR_BF16_REFINED>(a, C, sc, &fn2); unit = 0x1p-8; }
    const double fnorm = sqrt(fn2);
    if (fbad) { bad = true; break; }
    rank = factor(C, unit);
    // z0 = (G + mu I)^-1 c
    if (tid < 64) solve_fwd(C, C.c, C.s);
    __syncthreads();
    if (tid < 64) solve_bwd(C, C.s, C.z);
    __syncthreads();
    if (tid < n) C.tp[tid] = C.D[tid] * C.z[tid];
    __syncthreads();
    cg_sweep<NM, kR0>(a, C, sc, wsr, wsq, false, 0.0);
    if (tid < n) C.g[tid] *= C.D[tid];
    __syncthreads();
    if (tid < 64) solve_fwd(C, C.g, C.s);
    __syncthreads();
    if (tid < n) C.p[tid] = C.s[tid];
    if (tid < 64) { const double gg = dot_w0(C.s, C.s, n); if (tid == 0) C.red[kFitBlock - 2] = gg; }
    __syncthreads();
    double gamma = C.red[kFitBlock - 2];
    iters = 0;
    converged = a.max_iter == 0 || gamma == 0.0;
    err = 0.0;
    // CGLS increments are B^T B-orthogonal, so sum_{j >= k} alpha_j gamma_j = ||A (y* - y_k)||^2:
    // the last kDelay terms estimate the error of the fitted values (Hestenes-Stiefel).
    constexpr int kDelay = 3;
    double h0 = 0.0, h1 = 0.0, h2 = 0.0;     // the last kDelay alpha gamma terms
    const int need = a.max_iter < kDelay ? a.max_iter : kDelay;
    double alpha_prev = 0.0;
    for (int it = 0; it < a.max_iter && !converged; ++it) {
      if (tid < 64) solve_bwd(C, C.p, C.t);
      __syncthreads();
      if (tid < n) C.tp[tid] = C.D[tid] * C.t[tid];
      __syncthreads();
      const double qq = cg_sweep<NM, kQ>(a, C, sc, wsr, wsq, it > 0, alpha_prev);
      const double alpha = qq > 0.0 ? gamma / qq : 0.0;
      if (tid < n) C.z[tid] += alpha * C.t[tid];
      __syncthreads();
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
      if (tid < n) C.g[tid] = C.D[tid] * (C.g[tid] - alpha * C.gq[tid]);   // D A^T (r - alpha q)
      __syncthreads();
      alpha_prev = alpha;
      if (tid < 64) solve_fwd(C, C.g, C.s);
      __syncthreads();
      if (tid < 64) { const double gg = dot_w0(C.s, C.s, n); if (tid == 0) C.red[kFitBlock - 2] = gg; }
      __syncthreads();
      const double gnew = C.red[kFitBlock - 2];
      const double beta = gamma > 0.0 ? gnew / gamma : 0.0;
      if (tid < n) C.p[tid] = C.s[tid] + beta * C.p[tid];
      __syncthreads();
      gamma = gnew;
      if (gamma == 0.0) { converged = true; break; }
    }
    if (converged || prec == KLR_FP64) break;
    info.status |= KLR_FIT_FELL_BACK_FP64;
    prec = KLR_FP64;
  }

  if (bad) {
    if (coef_ok)
      for (int j = tid; j < n; j += kFitBlock) a.coef[d.coef0 + j] = 0.0;
    if (tid == 0) {
      info.status = ok ? KLR_FIT_NO_SCRATCH : KLR_FIT_BAD_INPUT;
      info.resid_norm = NAN;
      info.err_est = NAN;
      a.info[fi] = info;
    }
    return;
  }
  if (tid < n) C.tp[tid] = C.D[tid] * C.z[tid];
  __syncthreads();
  int qneg = 0;
  const double rr = final_sweep<NM>(a, C, sc, &qneg);
  if (tid < n) a.coef[d.coef0 + tid] = C.tp[tid];
  if (tid == 0) {
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
}

// Plain schedule: one workgroup per fit and size class (workgroups of other classes leave).
// The classes whose LDS allows two workgroups per CU are compiled for two waves per SIMD.
template <int NM, int PREC>
__device__ __forceinline__ void fit_plain_body(const FitArgs& a, int cls, double* smem) {
  const int fi = blockIdx.x;
  if (fi >= a.n_fits || fit_class(a, a.desc[fi]) != cls) return;
  fit_one<NM, PREC>(a, fi, smem);
}

template <int NM, int PREC>
__global__ void __launch_bounds__(kFitBlock) fit_kernel(FitArgs a, int cls) {
  extern __shared__ double smem[];
  fit_plain_body<NM, PREC>(a, cls, smem);
}

template <int NM, int PREC>
__global__ void __launch_bounds__(kFitBlock) __attribute__((amdgpu_waves_per_eu(2)))
fit_kernel2(FitArgs a, int cls) {
  extern __shared__ double smem[];
  fit_plain_body<NM, PREC>(a, cls, smem);
}

// ---- persistent, longest-first schedule ------------------------------------------------------
// plan: fits are bucketed by (class, 31 - floor(log2(m n^2 + 1))) so that an ascending scan of
// the buckets lists each class's fits from the most to the least work; the persistent
// workgroups of a workgroup class then pop positions from that class's queue counter, and the
// wave class (one wavefront per fit) is launched as a grid that takes positions in order.  A
// fit's result does not depend on which workgroup computes it, so outputs are deterministic.
constexpr int kBuckets = 32;
constexpr int kClasses = 7;
struct Plan {
  int32_t counts[kClasses * kBuckets];
  int32_t offs[kClasses * kBuckets];
  int32_t cursor[kClasses * kBuckets];
  int32_t totals[kClasses];
  int32_t base[kClasses];
  int32_t queue[kClasses];
  int32_t pad[4];
};

__device__ __forceinline__ int cost_bucket(const klr_fit_desc& d) {
  const int n = d.n_num + d.n_den - 1;
  const double w = (double)(d.m > 0 ? d.m : 0) * (double)(n > 0 ? n : 0) * (double)(n > 0 ? n : 0) + 1.0;
  int e = 0;
  frexp(w, &e);                      // w in [2^(e-1), 2^e)
  const int lg = e - 1 < kBuckets - 1 ? e - 1 : kBuckets - 1;
  return kBuckets - 1 - lg;
}

__global__ void fit_plan_zero(Plan* pl) {
  const int i = threadIdx.x;
  if (i < kClasses * kBuckets) pl->counts[i] = 0;
}

// Per-workgroup histograms in LDS, then one global atomic per non-empty bin and workgroup (a
// single bucket can hold every fit of the batch).
// The bin of each fit is kept in `keys` for the scatter.
__global__ void __launch_bounds__(kFitBlock) fit_plan_count(FitArgs a, Plan* pl, int32_t* keys) {
  __shared__ int32_t hist[kClasses * kBuckets];
  for (int b = threadIdx.x; b < kClasses * kBuckets; b += kFitBlock) hist[b] = 0;
  __syncthreads();
  const int fi = blockIdx.x * kFitBlock + threadIdx.x;
  if (fi < a.n_fits) {
    const klr_fit_desc d = a.desc[fi];
    const int key = fit_class(a, d) * kBuckets + cost_bucket(d);
    keys[fi] = key;
    atomicAdd(&hist[key], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kClasses * kBuckets; b += kFitBlock)
    if (hist[b] > 0) atomicAdd(&pl->counts[b], hist[b]);
}

__global__ void fit_plan_scan(Plan* pl) {
  if (threadIdx.x != 0) return;
  int32_t base = 0;
  for (int c = 0; c < kClasses; ++c) {
    pl->base[c] = base;
    int32_t run = 0;
    for (int b = 0; b < kBuckets; ++b) {
      pl->offs[c * kBuckets + b] = base + run;
      pl->cursor[c * kBuckets + b] = 0;
      run += pl->counts[c * kBuckets + b];
    }
    pl->totals[c] = run;
    pl->queue[c] = 0;
    base += run;
  }
}

// Each workgroup reserves one range per bin with a global atomic and places its fits in it by
// their LDS rank (the order inside a bucket is arbitrary; a fit's result does not depend on it).
__global__ void __launch_bounds__(kFitBlock) fit_plan_scatter(FitArgs a, Plan* pl, const int32_t* keys,
                                                               int32_t* order) {
  __shared__ int32_t hist[kClasses * kBuckets];
  __shared__ int32_t start[kClasses * kBuckets];
  for (int b = threadIdx.x; b < kClasses * kBuckets; b += kFitBlock) hist[b] = 0;
  __syncthreads();
  const int fi = blockIdx.x * kFitBlock + threadIdx.x;
  int key = -1, rank = 0;
  if (fi < a.n_fits) {
    key = keys[fi];
    rank = atomicAdd(&hist[key], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kClasses * kBuckets; b += kFitBlock)
    start[b] = hist[b] > 0 ? pl->offs[b] + atomicAdd(&pl->cursor[b], hist[b]) : 0;
  __syncthreads();
  if (key >= 0) order[start[key] + rank] = fi;
}

template <int NM, int PREC>
__device__ __forceinline__ void fit_persistent_body(const FitArgs& a, Plan* pl, const int32_t* order, int cls,
                                                    double* smem, int* next) {
  const int total = pl->totals[cls], base = pl->base[cls];
  if (total == 0) return;              // an empty class: no queue traffic at all
  for (;;) {
    // the counter only grows: once a plain read shows the queue exhausted, no atomic is needed
    // (every workgroup of an exhausted class would otherwise meet at one address)
    if (threadIdx.x == 0) {
      const int seen = __hip_atomic_load(&pl->queue[cls], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      *next = seen >= total ? seen : atomicAdd(&pl->queue[cls], 1);
    }
    __syncthreads();
    const int i = *next;
    __syncthreads();
    if (i >= total) break;
    fit_one<NM, PREC>(a, order[base + i], smem);
  }
}

template <int NM, int PREC>
__global__ void __launch_bounds__(kFitBlock)
fit_persistent(FitArgs a, Plan* pl, const int32_t* __restrict__ order, int cls) {
  extern __shared__ double smem[];
  __shared__ int next;
  fit_persistent_body<NM, PREC>(a, pl, order, cls, smem, &next);
}

template <int NM, int PREC>
__global__ void __launch_bounds__(kFitBlock) __attribute__((amdgpu_waves_per_eu(2)))
fit_persistent2(FitArgs a, Plan* pl, const int32_t* __restrict__ order, int cls) {
  extern __shared__ double smem[];
  __shared__ int next;
  fit_persistent_body<NM, PREC>(a, pl, order, cls, smem, &next);
}

// Exclusive prefix of the sample counts of the fits that take a workgroup class (the one-
// wavefront classes keep their residuals in registers): each such fit owns scratch rows
// [rowoff[fi], rowoff[fi] + m).  Three launches: every workgroup of kScanBlock fits writes the
// exclusive prefix within its block and the block total; one workgroup scans the totals; every
// workgroup adds the total of the blocks before its own.  A block total is at most
// kScanBlock * KLR_MAX_SAMPLES = 2^22, so the in-block sums stay in int32.
constexpr int kScanBlock = 1024;

__device__ __forceinline__ int32_t scratch_need(const FitArgs& a, int fi) {
  if (fi >= a.n_fits) return 0;
  const klr_fit_desc d = a.desc[fi];
  const int cls = fit_class(a, d);
  if (cls == kWaveClass || cls == kWaveClass16) return 0;
  return d.m < 0 ? 0 : (d.m > KLR_MAX_SAMPLES ? KLR_MAX_SAMPLES : d.m);
}

// Exclusive scan of v over the workgroup (kScanBlock threads); *total gets the sum.
template <typename T>
__device__ __forceinline__ T block_exclusive(T v, T* wsum, T* total) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  T inc = v;                                   // inclusive scan within the wavefront
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T o = __shfl_up(inc, off);
    if (lane >= off) inc += o;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  T before = 0;
  for (int w = 0; w < wv; ++w) before += wsum[w];
  T t = 0;
  for (int w = 0; w < kScanBlock / 64; ++w) t += wsum[w];
  *total = t;
  __syncthreads();
  return before + (inc - v);
}

__global__ void __launch_bounds__(kScanBlock) fit_rows_local(FitArgs a, int64_t* rowoff, int64_t* bsum) {
  __shared__ int32_t wsum[kScanBlock / 64];
  const int fi = blockIdx.x * kScanBlock + (int)threadIdx.x;
  int32_t total;
  const int32_t ex = block_exclusive<int32_t>(scratch_need(a, fi), wsum, &total);
  if (fi < a.n_fits) rowoff[fi] = ex;
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanBlock) fit_rows_scan(int64_t* bsum, int nblk) {
  __shared__ int64_t wsum[kScanBlock / 64];
  int64_t carry = 0;
  for (int b0 = 0; b0 < nblk; b0 += kScanBlock) {
    const int b = b0 + (int)threadIdx.x;
    int64_t total;
    const int64_t ex = block_exclusive<int64_t>(b < nblk ? bsum[b] : 0, wsum, &total);
    if (b < nblk) bsum[b] = carry + ex;
    carry += total;
  }
}

__global__ void __launch_bounds__(kScanBlock) fit_rows_add(FitArgs a, int64_t* rowoff, const int64_t* bsum) {
  const int fi = blockIdx.x * kScanBlock + (int)threadIdx.x;
  if (fi < a.n_fits) rowoff[fi] += bsum[blockIdx.x];
}

__host__ __device__ inline int scan_blocks(int32_t n_fits) {
  return n_fits > 0 ? (n_fits + kScanBlock - 1) / kScanBlock : 0;
}

// Workspace: the plan, the longest-first order and bucket keys (int32 per fit), the scratch
// offsets (int64 per fit) and the scan's block totals (int64 per kScanBlock fits), then two
// FP64 scratch values per sample row (residual and A t).
size_t head_bytes(int32_t n_fits) {
  const size_t nf = (size_t)(n_fits > 0 ? n_fits : 0);
  return (sizeof(Plan) + nf * 2 * sizeof(int32_t) + (nf + (size_t)scan_blocks(n_fits)) * sizeof(int64_t) + 255) /
         256 * 256;
}

// Two workgroups per CU when the dynamic LDS of a class leaves room for a second one (160 KB
// per CU, with a margin for the static queue slot and allocation granularity).
template <int NM>
constexpr bool two_per_cu() { return Lds<NM>::BYTES <= 80 * 1024 - 512; }

template <int NM, int PREC>
hipError_t launch_class(const FitArgs& a, int cls, bool persistent, Plan* pl, const int32_t* order) {
  const size_t lds = (size_t)Lds<NM>::BYTES;
  const void* fn;
  if constexpr (two_per_cu<NM>())
    fn = persistent ? reinterpret_cast<const void*>(&fit_persistent2<NM, PREC>)
                    : reinterpret_cast<const void*>(&fit_kernel2<NM, PREC>);
  else
    fn = persistent ? reinterpret_cast<const void*>(&fit_persistent<NM, PREC>)
                    : reinterpret_cast<const void*>(&fit_kernel<NM, PREC>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (!persistent) {
    if constexpr (two_per_cu<NM>())
      hipLaunchKernelGGL((fit_kernel2<NM, PREC>), dim3((unsigned)a.n_fits), dim3(kFitBlock), lds, a.stream, a, cls);
    else
      hipLaunchKernelGGL((fit_kernel<NM, PREC>), dim3((unsigned)a.n_fits), dim3(kFitBlock), lds, a.stream, a, cls);
    return hipGetLastError();
  }
  int dev = 0, ncu = 0, occ = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, kFitBlock, lds);
  if (e != hipSuccess) return e;
  int64_t g = (int64_t)ncu * (occ > 0 ? occ : 1);
  if (g > a.n_fits) g = a.n_fits;
  if constexpr (two_per_cu<NM>())
    hipLaunchKernelGGL((fit_persistent2<NM, PREC>), dim3((unsigned)g), dim3(kFitBlock), lds, a.stream, a, pl,
                       order, cls);
  else
    hipLaunchKernelGGL((fit_persistent<NM, PREC>), dim3((unsigned)g), dim3(kFitBlock), lds, a.stream, a, pl,
                       order, cls);
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_all(const FitArgs& a, bool persistent) {
  Plan* pl = reinterpret_cast<Plan*>(a.ws);
  int32_t* order = reinterpret_cast<int32_t*>(pl + 1);
  int32_t* keys = order + (a.n_fits > 0 ? a.n_fits : 0);
  const int nblk = scan_blocks(a.n_fits);
  int64_t* bsum = a.rowoff + (a.n_fits > 0 ? a.n_fits : 0);
  if (nblk > 0)       // one block: its in-block prefix is the whole prefix
    hipLaunchKernelGGL(fit_rows_local, dim3((unsigned)nblk), dim3(kScanBlock), 0, a.stream, a, a.rowoff, bsum);
  if (nblk > 1) {
    hipLaunchKernelGGL(fit_rows_scan, dim3(1), dim3(kScanBlock), 0, a.stream, bsum, nblk);
    hipLaunchKernelGGL(fit_rows_add, dim3((unsigned)nblk), dim3(kScanBlock), 0, a.stream, a, a.rowoff, bsum);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && persistent) {
    const unsigned g = (unsigned)((a.n_fits + kFitBlock - 1) / kFitBlock);
    hipLaunchKernelGGL(fit_plan_zero, dim3(1), dim3(kClasses * kBuckets), 0, a.stream, pl);
    hipLaunchKernelGGL(fit_plan_count, dim3(g), dim3(kFitBlock), 0, a.stream, a, pl, keys);
    hipLaunchKernelGGL(fit_plan_scan, dim3(1), dim3(64), 0, a.stream, pl);
    hipLaunchKernelGGL(fit_plan_scatter, dim3(g), dim3(kFitBlock), 0, a.stream, a, pl, keys, order);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    const WavePlanView pv8{order, &pl->totals[kWaveClass], &pl->base[kWaveClass]};
    const WavePlanView pv16{order, &pl->totals[kWaveClass16], &pl->base[kWaveClass16]};
    e = launch_fit_wave(a, persistent, pv8, pv16);
  }
  if (e == hipSuccess) e = launch_class<32, PREC>(a, 0, persistent, pl, order);
  if (e == hipSuccess) e = launch_class<64, PREC>(a, 1, persistent, pl, order);
  if (e == hipSuccess) e = launch_class<96, PREC>(a, 2, persistent, pl, order);
  if (e == hipSuccess) e = launch_class<112, PREC>(a, 3, persistent, pl, order);
  if (e == hipSuccess) e = launch_class<128, PREC>(a, 4, persistent, pl, order);
  return e;
}

}  // namespace

size_t fit_workspace_bytes(int32_t n_fits, int64_t total_rows, int32_t precision) {
  (void)precision;
  return head_bytes(n_fits) + (size_t)(total_rows > 0 ? total_rows : 0) * 2 * sizeof(double);
}

void fit_workspace_split(FitArgs& a) {
  const size_t head = head_bytes(a.n_fits);
  char* base = reinterpret_cast<char*>(a.ws);
  a.rowoff = reinterpret_cast<int64_t*>(base + sizeof(Plan) + (size_t)(a.n_fits > 0 ? a.n_fits : 0) * 2 * sizeof(int32_t));
  a.scratch = reinterpret_cast<double*>(base + head);
  a.scratch_rows = a.ws_bytes > head ? (int64_t)((a.ws_bytes - head) / (2 * sizeof(double))) : 0;
}

hipError_t launch_fit_once(const FitArgs& a) {
  if (a.precision == KLR_FP64) return launch_all<KLR_FP64>(a, a.persistent);
  if (a.precision == KLR_FP32_REFINED) return launch_all<KLR_FP32_REFINED>(a, a.persistent);
  return launch_all<KLR_BF16_REFINED>(a, a.persistent);
}

hipError_t launch_fit(const FitArgs& a0) {
  if (a0.precision == KLR_FP64_SVD) return launch_fit_svd(a0);
  FitArgs a = a0;
  int v = a.variant;
  if (v < 0 && a.tuner) {
    // autotune: every variant once on this batch (they give identical results), HIP events on
    // the caller's stream; the fastest is cached under the batch's shape key
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 0.0f;
    int bv = 0;
    for (int i = 0; i < kFitVariants && e == hipSuccess; ++i) {
      a.wave_group = kFitWaveGroups[i];
      e = hipEventRecord(e0, a.stream);
      if (e == hipSuccess) e = launch_fit_once(a);
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
  a.wave_group = kFitWaveGroups[v >= 0 && v < kFitVariants ? v : 0];
  const int t = a.timer ? a.timer->begin(KLR_K_FIT_SOLVE, a.stream) : -1;
  const hipError_t e = launch_fit_once(a);
  if (a.timer) a.timer->end(t, a.stream);
  return e;
}

}  // namespace klr

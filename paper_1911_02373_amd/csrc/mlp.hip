// Surrogate network of the log-cycle estimate (not in the paper), gfx950.
//
// Network: x = (log2 N / 26, log2 bx / 10, log2 by / 10, e_k); h1 = relu(W1 x + b1) [256];
// h2 = relu(W2 h1 + b2) [256]; y = w3 . h2 + b3 predicts (ln C - mu) / sigma.
//
// Kernels
//   mlp_stats       mu, sigma of ln C over the valid training samples (one workgroup, FP64,
//                   fixed reduction order)
//   mlp_refresh     BF16 working copies W2b = bf16(W2), W2Tb = bf16(W2^T)
//   mlp_fwd_bwd     one 64-sample tile per workgroup: layer 1 (FP32 VALU) -> h1 (BF16, LDS) ->
//                   layer 2 on v_mfma_f32_32x32x16_bf16 (each wave owns 64 output columns:
//                   2 x 2 tiles of 32 x 32) -> y, dy -> dA2 (BF16, LDS) -> dH1 = dA2 W2 on the
//                   same MFMA (B operand from the transposed copy) -> per-tile partial gradients
//                   of the small parameters, h1^T and dA2^T to global memory for dW2, embedding
//                   gradients accumulated in 2^-44 fixed point with integer atomics (exact and
//                   order independent, so results are deterministic)
//   mlp_dw2_part    dW2 = dA2^T h1 over the batch on v_mfma_f32_16x16x32_bf16: 64 x 64 output
//                   tiles x 16 batch slices, one slice partial per workgroup
//   mlp_small_adam  fixed-order sums of the 16 dW2 slice partials (one thread per W2 entry,
//                   Adam on W2 and refresh of W2b / W2Tb) and of the per-tile partials of the
//                   small parameters (8 lanes per parameter), Adam on W1, b1, b2, w3, b3 and
//                   the embeddings, batch loss
//   mlp_predict     forward pass for arbitrary samples
//   mlp_select      surrogate selection over the (query x configuration) grid of a program
//
// MFMA operand layouts used (wave64): for v_mfma_f32_32x32x16_bf16 lane l holds
// A[l % 32][8 (l / 32) + e] and B[8 (l / 32) + e][l % 32] (e = 0..7); result register r of
// lane l is D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].  For v_mfma_f32_16x16x32_bf16 lane l
// holds A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16]; register r is
// D[4 (l / 16) + r][l % 16].
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "eval_point.hpp"
#include "internal.hpp"

namespace klr {

namespace {

constexpr int H = KLR_MLP_HIDDEN;
constexpr int TS = 64;          // rows (samples or configurations) per tile
constexpr int HP = H + 8;       // padded LDS row of BF16 values
constexpr int kBlock = 256;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t b = __float_as_uint(x);
  b += 0x7FFFu + ((b >> 16) & 1u);       // round to nearest even (finite inputs)
  return (uint16_t)(b >> 16);
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

__device__ __forceinline__ void features(int32_t N, int32_t bx, int32_t by, float e, float* x) {
  x[0] = log2f((float)N) * (1.0f / 26.0f);
  x[1] = log2f((float)bx) * 0.1f;
  x[2] = log2f((float)by) * 0.1f;
  x[3] = e;
}

// ---- permutation of the samples of one epoch: a bijection on [0, 2^bits) (odd multiply +
// xorshift rounds with keyed constants) with cycle walking into [0, n).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ int64_t permute(int64_t i, int64_t n, int bits, uint64_t key) {
  const uint64_t mask = (bits >= 64) ? ~0ull : ((1ull << bits) - 1ull);
  const int sh = bits / 2 > 0 ? bits / 2 : 1;
  uint64_t x = (uint64_t)i;
  do {
    for (int r = 0; r < 4; ++r) {
      const uint64_t k = mix64(key + (uint64_t)r * 0x632BE59BD9B4E019ull);
      x = (x * (k | 1ull) + (k >> 17)) & mask;
      x ^= x >> sh;
    }
  } while (x >= (uint64_t)n);
  return (int64_t)x;
}

// ---- layer 1 of one tile into LDS (row-major [row][k], BF16) and optionally to h1^T in HBM.
// Row r has features xs[r][0..3]; rows with valid[r] == 0 get h1 = 0.
__device__ void layer1(const Blob& w, const float (*xs)[4], uint16_t* H1s, uint16_t* H1T, int64_t ld,
                       int64_t col0) {
  const int k = threadIdx.x;
  const float w0 = w.P[kO_W1 + 4 * k], w1 = w.P[kO_W1 + 4 * k + 1];
  const float w2 = w.P[kO_W1 + 4 * k + 2], w3 = w.P[kO_W1 + 4 * k + 3];
  const float b = w.P[kO_B1 + k];
  uint16_t pack[8];
  for (int s = 0; s < TS; ++s) {
    float a = w0 * xs[s][0] + w1 * xs[s][1];
    a += w2 * xs[s][2] + w3 * xs[s][3];
    a += b;
    const uint16_t u = f2bf(a > 0.0f ? a : 0.0f);
    H1s[s * HP + k] = u;
    pack[s & 7] = u;
    if (H1T && (s & 7) == 7) {
      uint4 v;
      v.x = pack[0] | ((uint32_t)pack[1] << 16);
      v.y = pack[2] | ((uint32_t)pack[3] << 16);
      v.z = pack[4] | ((uint32_t)pack[5] << 16);
      v.w = pack[6] | ((uint32_t)pack[7] << 16);
      *reinterpret_cast<uint4*>(H1T + (int64_t)k * ld + col0 + (s - 7)) = v;
    }
  }
}

// ---- layer 2 of one tile: acc[rt][ct] = H1 (64 x 256) x B^T for the wave's 64 output columns,
// where B rows are read from Bmat (row-major [col][k], 256 columns of 256).
__device__ __forceinline__ void gemm_tile(const uint16_t* As, const uint16_t* Bmat, f32x16 acc[2][2]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[rt][ct][r] = 0.0f;
  const int row = lane & 31, kh = 8 * (lane >> 5);
#pragma unroll 4
  for (int kk = 0; kk < H / 16; ++kk) {
    const int kb = kk * 16 + kh;
    const bf16x8 a0 = ld8(As + row * HP + kb);
    const bf16x8 a1 = ld8(As + (32 + row) * HP + kb);
    const bf16x8 b0 = ld8(Bmat + (wv * 64 + row) * H + kb);
    const bf16x8 b1 = ld8(Bmat + (wv * 64 + 32 + row) * H + kb);
    acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
  }
}

__device__ __forceinline__ int acc_row(int rt, int r, int lane) {
  return rt * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

// Sum over the 32 lanes of each half-wavefront (all lanes active): DPP within rows of 16, then
// the lane-swap pair sum of rows 0 and 1 (2 and 3).
__device__ __forceinline__ float sum32(float v) { return pair_sum16_f(group16_sum_f(v)); }

// y[row] partial of this wave: sum over its columns of w3[j] relu(acc + b2[j]); written to
// part[wave][row].
__device__ void layer3_partial(const Blob& w, f32x16 acc[2][2], float (*part)[TS]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float b2v[2], w3v[2];
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int j = wv * 64 + ct * 32 + (lane & 31);
    b2v[ct] = w.P[kO_B2 + j];
    w3v[ct] = w.P[kO_W3 + j];
  }
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      float v = 0.0f;
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        const float a2 = acc[rt][ct][r] + b2v[ct];
        v += w3v[ct] * (a2 > 0.0f ? a2 : 0.0f);
      }
      v = sum32(v);
      if ((lane & 31) == 0) part[wv][acc_row(rt, r, lane)] = v;
    }
}

}  // namespace

// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(1024)
mlp_stats(const float* __restrict__ cost, int64_t n, float* hdr) {
  __shared__ double s1[1024], s2[1024], sc[1024];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const float v = cost[i];
    if (v > 0.0f && v <= 3.402823466e38f) {
      const double l = log((double)v);
      a += l;
      b += l * l;
      c += 1.0;
    }
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int st = 512; st >= 1; st >>= 1) {
    if ((int)threadIdx.x < st) {
      s1[threadIdx.x] += s1[threadIdx.x + st];
      s2[threadIdx.x] += s2[threadIdx.x + st];
      sc[threadIdx.x] += sc[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double cnt = sc[0] > 0.0 ? sc[0] : 1.0;
    const double mu = s1[0] / cnt;
    double var = s2[0] / cnt - mu * mu;
    if (!(var > 1e-12)) var = 1.0;
    hdr[0] = (float)mu;
    hdr[1] = (float)sqrt(var);
  }
}

__global__ void __launch_bounds__(kBlock) mlp_refresh(Blob w) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= H * H) return;
  const int j = i / H, k = i % H;
  const uint16_t u = f2bf(w.P[kO_W2 + i]);
  w.W2b[i] = u;
  w.W2Tb[k * H + j] = u;
}

__global__ void __launch_bounds__(kBlock) mlp_fwd_bwd(TrainTile a, Blob w) {
  __shared__ __attribute__((aligned(16))) uint16_t H1s[TS * HP];
  __shared__ __attribute__((aligned(16))) uint16_t dAs[TS * HP];
  __shared__ float xs[TS][4];
  __shared__ float ts[TS], vs[TS], dys[TS], lss[TS];
  __shared__ int ks[TS];
  __shared__ float part[4][TS];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t s0 = (int64_t)blockIdx.x * TS;
  const float mu = w.hdr[0], sig = w.hdr[1];
  if (tid < TS) {
    const int64_t pos = a.batch_start + s0 + tid;
    const int64_t i = a.perm_bits > 0 ? permute(pos, a.n, a.perm_bits, a.perm_key) : pos;
    const int32_t k = a.kid[i], Nv = a.N[i], bx = a.L[2 * i], by = a.L[2 * i + 1];
    bool ok = k >= 0 && k < a.nk && Nv >= 1 && bx >= 1 && by >= 1;
    float t = 0.0f;
    if (a.tstd) {
      t = a.tstd[i];
    } else {
      const float c = a.cost[i];
      ok = ok && c > 0.0f && c <= 3.402823466e38f;
      t = ok ? (logf(c) - mu) / sig : 0.0f;
    }
    ok = ok && fabsf(t) <= 3.402823466e38f;
    float x[4];
    features(Nv >= 1 ? Nv : 1, bx >= 1 ? bx : 1, by >= 1 ? by : 1, ok ? w.P[kO_EMB + k] : 0.0f, x);
    for (int f = 0; f < 4; ++f) xs[tid][f] = x[f];
    ts[tid] = t;
    vs[tid] = ok ? 1.0f : 0.0f;
    ks[tid] = ok ? k : -1;
  }
  __syncthreads();
  layer1(w, xs, H1s, a.H1T, a.B, s0);
  __syncthreads();
  f32x16 acc[2][2];
  gemm_tile(H1s, w.W2b, acc);
  layer3_partial(w, acc, part);
  __syncthreads();
  if (tid < TS) {
    const float y = ((part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid])) + w.P[kO_B3];
    const float r = y - ts[tid];
    dys[tid] = vs[tid] != 0.0f ? 2.0f * r / (float)a.B : 0.0f;
    lss[tid] = vs[tid] != 0.0f ? r * r : 0.0f;
  }
  __syncthreads();
  float* prt = a.partial + (int64_t)blockIdx.x * kPartialStride;
  {
    float b2v[2], w3v[2];
    int jc[2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      jc[ct] = wv * 64 + ct * 32 + (lane & 31);
      b2v[ct] = w.P[kO_B2 + jc[ct]];
      w3v[ct] = w.P[kO_W3 + jc[ct]];
    }
    float gw3[2] = {0.0f, 0.0f}, gb2[2] = {0.0f, 0.0f};
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int s = acc_row(rt, r, lane);
        const float dy = dys[s];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const float a2 = acc[rt][ct][r] + b2v[ct];
          const float h2 = a2 > 0.0f ? a2 : 0.0f;
          const float da2 = a2 > 0.0f ? dy * w3v[ct] : 0.0f;
          gw3[ct] += dy * h2;
          gb2[ct] += da2;
          dAs[s * HP + jc[ct]] = f2bf(da2);
        }
      }
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      gw3[ct] = pair_sum32_f(gw3[ct]);
      gb2[ct] = pair_sum32_f(gb2[ct]);
      if (lane < 32) {
        prt[kO_W3 - kO_W1 + jc[ct]] = gw3[ct];
        prt[kO_B2 - kO_W1 + jc[ct]] = gb2[ct];
      }
    }
  }
  __syncthreads();
  {  // dA2^T to HBM for the dW2 product: row j = tid, 64 samples
    const int j = tid;
    for (int s = 0; s < TS; s += 8) {
      uint4 v;
      v.x = dAs[(s + 0) * HP + j] | ((uint32_t)dAs[(s + 1) * HP + j] << 16);
      v.y = dAs[(s + 2) * HP + j] | ((uint32_t)dAs[(s + 3) * HP + j] << 16);
      v.z = dAs[(s + 4) * HP + j] | ((uint32_t)dAs[(s + 5) * HP + j] << 16);
      v.w = dAs[(s + 6) * HP + j] | ((uint32_t)dAs[(s + 7) * HP + j] << 16);
      *reinterpret_cast<uint4*>(a.dH2T + (int64_t)j * a.B + s0 + s) = v;
    }
  }
  gemm_tile(dAs, w.W2Tb, acc);   // dH1 = dA2 W2
  {
    float gw1[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, gb1[2] = {0.0f, 0.0f};
    float w13[2];
    int kc[2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      kc[ct] = wv * 64 + ct * 32 + (lane & 31);
      w13[ct] = w.P[kO_W1 + 4 * kc[ct] + 3];
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int s = acc_row(rt, r, lane);
        float de = 0.0f;
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const float da1 = H1s[s * HP + kc[ct]] != 0 ? acc[rt][ct][r] : 0.0f;
#pragma unroll
          for (int f = 0; f < 4; ++f) gw1[ct][f] += da1 * xs[s][f];
          gb1[ct] += da1;
          de += da1 * w13[ct];
        }
        de = sum32(de);
        if ((lane & 31) == 0) part[wv][s] = de;
      }
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
#pragma unroll
      for (int f = 0; f < 4; ++f) gw1[ct][f] = pair_sum32_f(gw1[ct][f]);
      gb1[ct] = pair_sum32_f(gb1[ct]);
      if (lane < 32) {
#pragma unroll
        for (int f = 0; f < 4; ++f) prt[4 * kc[ct] + f] = gw1[ct][f];
        prt[kO_B1 - kO_W1 + kc[ct]] = gb1[ct];
      }
    }
  }
  __syncthreads();
  if (tid < TS && ks[tid] >= 0) {
    const float de = (part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid]);
    const long long q = __double2ll_rn((double)de * 0x1p44);
    atomicAdd(a.emb_acc + ks[tid], (unsigned long long)q);
  }
  if (tid < TS) {               // wave 0: butterfly sums over the tile (fixed pattern, deterministic)
    float sdy = dys[tid], sl = lss[tid];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      sdy += __shfl_xor(sdy, off);
      sl += __shfl_xor(sl, off);
    }
    if (tid == 0) {
      prt[kO_B3 - kO_W1] = sdy;
      prt[kLossSlot] = sl;
    }
  }
}

// dW2 over the batch, first half: workgroup (tile, slice) forms the 64 x 64 output tile `tile`
// over batch slice `slice` (one sixteenth of the 32-sample chunks; its four waves take the
// chunks round-robin with the next chunk's operands loaded ahead, each wave the whole tile as
// 4 x 4 MFMA blocks), sums the four wave partials in a fixed order and stores the slice
// partial.  mlp_small_adam sums the 16 slice partials in a fixed order and applies Adam.
constexpr int kDw2Tile = 64;
constexpr int kDw2Waves = 4;
constexpr int kDw2Tiles = (H / kDw2Tile) * (H / kDw2Tile);
__global__ void __launch_bounds__(64 * kDw2Waves)
mlp_dw2_part(const uint16_t* __restrict__ dH2T, const uint16_t* __restrict__ H1T, int32_t B,
             float* __restrict__ part) {
  __shared__ float red[kDw2Waves][kDw2Tile][kDw2Tile];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, tid = threadIdx.x;
  const int tile = blockIdx.x % kDw2Tiles, slice = blockIdx.x / kDw2Tiles;
  const int tj = tile / (H / kDw2Tile), tk = tile % (H / kDw2Tile);
  const int row = lane & 15, kh = 8 * (lane >> 4);
  const uint16_t* pa = dH2T + (int64_t)(kDw2Tile * tj + row) * B + kh;
  const uint16_t* pb = H1T + (int64_t)(kDw2Tile * tk + row) * B + kh;
  const int nch = B / 32;
  const int c_lo = (int)((int64_t)slice * nch / kDw2Slices), c_hi = (int)((int64_t)(slice + 1) * nch / kDw2Slices);
  f32x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  int c = c_lo + wv;
  bf16x8 av[4], bv[4];
  if (c < c_hi) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[u] = ld8(pa + (int64_t)16 * u * B + (int64_t)c * 32);
      bv[u] = ld8(pb + (int64_t)16 * u * B + (int64_t)c * 32);
    }
  }
  for (; c < c_hi; c += kDw2Waves) {
    bf16x8 an[4], bn[4];
    const int cn = c + kDw2Waves < c_hi ? c + kDw2Waves : c;   // reload of c on the last chunk
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      an[u] = ld8(pa + (int64_t)16 * u * B + (int64_t)cn * 32);
      bn[u] = ld8(pb + (int64_t)16 * u * B + (int64_t)cn * 32);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < 4; ++u) { av[u] = an[u]; bv[u] = bn[u]; }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wv][16 * a + 4 * (lane >> 4) + r][16 * b + (lane & 15)] = acc[a][b][r];
  __syncthreads();
  float* myp = part + (int64_t)slice * H * H;
  for (int e = tid; e < kDw2Tile * kDw2Tile; e += 64 * kDw2Waves) {
    const int rr = e / kDw2Tile, cc = e % kDw2Tile;
    myp[(kDw2Tile * tj + rr) * H + kDw2Tile * tk + cc] =
        (red[0][rr][cc] + red[1][rr][cc]) + (red[2][rr][cc] + red[3][rr][cc]);
  }
}

// Small parameters: eight consecutive lanes per parameter sum interleaved tiles (lane s takes
// tiles s, s + 8, ...), then the eight partial sums are combined by DPP in a fixed order; the
// embeddings' fixed-point sums take one lane each.
constexpr int kSmallLanes = 8;
__global__ void __launch_bounds__(kBlock)
mlp_small_adam(const float* __restrict__ partial, int32_t ntiles, unsigned long long* emb_acc,
               int32_t nk, Blob w, AdamArgs ad, float* grads, float* loss_step, float* loss_epoch,
               float epoch_scale, int32_t B, const float* __restrict__ dw2_part) {
  int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (gt < H * H) {                    // W2: the 16 slice partials of dW2 in a fixed order
    const int j = (int)(gt / H), k = (int)(gt % H);
    float q[kDw2Slices / 2];
#pragma unroll
    for (int i = 0; i < kDw2Slices / 2; ++i)
      q[i] = dw2_part[(int64_t)(2 * i) * H * H + gt] + dw2_part[(int64_t)(2 * i + 1) * H * H + gt];
#pragma unroll
    for (int h = kDw2Slices / 4; h >= 1; h >>= 1)
#pragma unroll
      for (int i = 0; i < h; ++i) q[i] = q[2 * i] + q[2 * i + 1];
    const float g = q[0];
    const int idx = kO_W2 + (int)gt;
    if (grads) grads[idx] = g;
    const float m = ad.b1 * w.M[idx] + (1.0f - ad.b1) * g;
    const float v = ad.b2 * w.V[idx] + (1.0f - ad.b2) * g * g;
    w.M[idx] = m;
    w.V[idx] = v;
    const float p = w.P[idx] - ad.lr * (m / ad.bc1) / (sqrtf(v / ad.bc2) + ad.eps);
    w.P[idx] = p;
    const uint16_t u = f2bf(p);
    w.W2b[j * H + k] = u;
    w.W2Tb[k * H + j] = u;
    return;
  }
  gt -= H * H;                         // a multiple of the block size: groups of 8 stay aligned
  const int nsmall = kO_B3 - kO_W1 + 1;
  const int64_t nsum = (int64_t)(nsmall + 1) * kSmallLanes;    // the small parameters and the loss
  int idx = -1;
  float g = 0.0f;
  if (gt < nsum) {                     // whole groups of 8 lanes: the DPP moves stay inside a group
    const int i = (int)(gt / kSmallLanes), sub = (int)(gt % kSmallLanes);
    const int slot = i < nsmall ? i : kLossSlot;
    float s = 0.0f;
#pragma unroll 8
    for (int t = sub; t < ntiles; t += kSmallLanes) s += partial[(int64_t)t * kPartialStride + slot];
    s += dpp_f<kDppXor1>(s);
    s += dpp_f<kDppXor2>(s);
    s += dpp_f<kDppHalfMirror>(s);
    if (sub == 0) {
      if (i < nsmall) {
        g = s;
        idx = kO_W1 + i;
      } else {
        const float L = s / (float)B;
        if (loss_step) *loss_step = L;
        if (loss_epoch) *loss_epoch += L * epoch_scale;
      }
    }
  } else if (gt - nsum < nk) {
    const int k = (int)(gt - nsum);
    g = (float)((double)(long long)emb_acc[k] * 0x1p-44);
    emb_acc[k] = 0ull;
    idx = kO_EMB + k;
  }
  if (idx >= 0) {
    if (grads) grads[idx] = g;
    const float m = ad.b1 * w.M[idx] + (1.0f - ad.b1) * g;
    const float v = ad.b2 * w.V[idx] + (1.0f - ad.b2) * g * g;
    w.M[idx] = m;
    w.V[idx] = v;
    w.P[idx] = w.P[idx] - ad.lr * (m / ad.bc1) / (sqrtf(v / ad.bc2) + ad.eps);
  }
}

__global__ void __launch_bounds__(kBlock)
mlp_predict(const int32_t* __restrict__ kid, const int32_t* __restrict__ Nq, const int32_t* __restrict__ L,
            int64_t n, int32_t nk, Blob w, float* pred) {
  __shared__ __attribute__((aligned(16))) uint16_t H1s[TS * HP];
  __shared__ float xs[TS][4];
  __shared__ float part[4][TS];
  const int tid = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * TS;
  if (tid < TS) {
    const int64_t i = s0 + tid < n ? s0 + tid : n - 1;
    const int32_t k = kid[i], Nv = Nq[i], bx = L[2 * i], by = L[2 * i + 1];
    const bool ok = k >= 0 && k < nk;
    float x[4];
    features(Nv >= 1 ? Nv : 1, bx >= 1 ? bx : 1, by >= 1 ? by : 1, ok ? w.P[kO_EMB + k] : 0.0f, x);
    for (int f = 0; f < 4; ++f) xs[tid][f] = x[f];
  }
  __syncthreads();
  layer1(w, xs, H1s, nullptr, 0, 0);
  __syncthreads();
  f32x16 acc[2][2];
  gemm_tile(H1s, w.W2b, acc);
  layer3_partial(w, acc, part);
  __syncthreads();
  if (tid < TS && s0 + tid < n) {
    const float y = ((part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid])) + w.P[kO_B3];
    pred[s0 + tid] = w.hdr[0] + w.hdr[1] * y;
  }
}

// Surrogate selection.  Persistent workgroups of 8 waves; each holds W2 in LDS (BF16, in
// MFMA fragment order) and loops over work items of (program, 64 queries).  A wave takes one
// query at a time through the whole network for 64 configurations at once, with no LDS round
// trip of the activations:
//   layer 1: H1^T = W1 X^T + b1 on v_mfma_f32_32x32x2f32 (A = W1 rows from registers, B = the
//            features of 32 configurations, C = b1), relu, v_cvt_pk_bf16_f32;
//   layer 2: D2^T = W2 H1^T + b2 on v_mfma_f32_32x32x16_bf16 (A = W2 fragments from LDS,
//            B = the layer-1 registers: k-block kb holds hidden units 16 kb .. 16 kb + 15, lane
//            group g the units 16 kb + 8 (e / 4) + 4 g + e % 4, which is exactly where the
//            32 x 32 FP32 output of layer 1 keeps them, so H1 never leaves registers);
//   layer 3: y = w3 . relu(D2^T) + b3 summed over the lane's 16 output registers, then the two
//            lane groups in a fixed order.
// Only configurations the exact program admits at the query's N enter the ranking (the fitted
// metrics defined, at least one block resident, the launch constraints met: the same FP32 steps
// as the exact sweep, so a configuration left out has cost +inf there); the network never sees
// inadmissible points in training, so its predictions for them carry no information.
// Each lane keeps its lowest predictions; rounds of 32-lane minima give the query's best
// predictions in order, hence the pick and the margin; a query that does not fall back has its
// shortlist (the best a.shortlist predictions) evaluated exactly, and the lowest exact cost wins.
constexpr int kSelMaxCfg = 1024;
constexpr int kSelWaves = 8;
constexpr int kSelQ = 64;            // queries per work item

struct SelLds {
  uint4 w2f[8 * 16 * 64];            // [h2 tile][k block][lane] -> 8 BF16 of W2
  float b1f[8][2][16];               // b1, b2, w3 in the 32 x 32 output layout: [tile][group][reg]
  float b2f[8][2][16];
  float w3f[8][2][16];
  float2 cfx[kSelMaxCfg];            // (log2 bx / 10, log2 by / 10)
};

__device__ __forceinline__ int out_hidden(int tile, int g, int r) {   // 32 x 32 output row index
  return 32 * tile + 8 * (r >> 2) + 4 * g + (r & 3);
}

__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  bf16x2 v;
  v[0] = (__bf16)a;
  v[1] = (__bf16)b;
  return *reinterpret_cast<uint32_t*>(&v);
}

__global__ void __launch_bounds__(64 * kSelWaves)
mlp_select(SelectArgs a, Blob w, int chunks, int64_t n_items) {
  extern __shared__ __attribute__((aligned(16))) char sel_raw[];
  SelLds& S = *reinterpret_cast<SelLds*>(sel_raw);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = lane >> 5;
  for (int i = tid; i < 8 * 16 * 64; i += 64 * kSelWaves) {
    const int t2 = i >> 10, kb = (i >> 6) & 15, ln = i & 63;
    const uint16_t* src = w.W2b + (int64_t)(32 * t2 + (ln & 31)) * H + 16 * kb + 4 * (ln >> 5);
    const uint2 lo = *reinterpret_cast<const uint2*>(src);
    const uint2 hi = *reinterpret_cast<const uint2*>(src + 8);
    S.w2f[i] = make_uint4(lo.x, lo.y, hi.x, hi.y);
  }
  for (int i = tid; i < 8 * 2 * 16; i += 64 * kSelWaves) {
    const int t = i >> 5, gg = (i >> 4) & 1, r = i & 15;
    const int h = out_hidden(t, gg, r);
    S.b1f[t][gg][r] = w.P[kO_B1 + h];
    S.b2f[t][gg][r] = w.P[kO_B2 + h];
    S.w3f[t][gg][r] = w.P[kO_W3 + h];
  }
  float w1r[8][2];                   // A operand of layer 1: W1[32 t + lane % 32][2 s + lane / 32]
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int st = 0; st < 2; ++st) w1r[t][st] = w.P[kO_W1 + 4 * (32 * t + (lane & 31)) + 2 * st + g];
  const float mu = w.hdr[0], sig = w.hdr[1], b3 = w.P[kO_B3];
  const Hw32 hw = make_hw32(a.hw);
  const float lnm = logf(1.0f + a.margin);
  int loaded = -1;
  for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    const int p = (int)(item / chunks);
    const int qb = (int)(item % chunks) * kSelQ;
    const klr_program P = a.progs[p];
    // the descriptor checks of the exact path: a program it rejects gets no output here either
    const int nmet = P.cost_kind == KLR_COST_METRIC ? 1 : (P.cost_kind == KLR_COST_PIECEWISE ? 3 : KLR_N_METRICS);
    const bool desc_ok = (P.cost_kind == KLR_COST_CYCLES || P.cost_kind == KLR_COST_METRIC ||
                          P.cost_kind == KLR_COST_PIECEWISE) && P.fit0 >= 0 &&
                         (int64_t)P.fit0 + nmet <= a.n_fits &&
                         P.v_launch >= 1 && P.v_launch <= KLR_MAX_LAUNCH && P.n_cfg >= 0 &&
                         P.n_cfg <= a.max_cfg && P.n_q >= 0 && P.n_q <= a.max_q && P.cfg0 >= 0 &&
                         P.cfg0 + (int64_t)P.n_cfg * P.v_launch <= a.cfgs_len && P.q0 >= 0 &&
                         P.q0 + (int64_t)P.n_q <= a.q_len &&
                         (P.grid_kind == KLR_GRID_1D || (P.grid_kind == KLR_GRID_2D && P.v_launch >= 2));
    if (!desc_ok || qb >= P.n_q) continue;
    const bool sel_ok = P.v_launch == 2 && P.n_cfg <= kSelMaxCfg;
    const int qe = qb + kSelQ < P.n_q ? qb + kSelQ : P.n_q;
    if (!sel_ok) {   // not representable by the network: the exact path answers these queries
      for (int qi = qb + tid; qi < qe; qi += 64 * kSelWaves) {
        const int64_t o = P.q0 + qi;
        a.argmin[o] = -1;
        a.pred_cost[o] = INFINITY;
        a.fell_back[o] = 1;
        if (a.pred_margin) a.pred_margin[o] = NAN;
      }
      continue;
    }
    if (p != loaded) {
      __syncthreads();               // every wave is done with the previous program's tables
      for (int c = tid; c < P.n_cfg; c += 64 * kSelWaves) {
        const int32_t bx = a.cfgs[P.cfg0 + 2 * c], by = a.cfgs[P.cfg0 + 2 * c + 1];
        S.cfx[c] = make_float2(log2f((float)(bx >= 1 ? bx : 1)) * 0.1f, log2f((float)(by >= 1 ? by : 1)) * 0.1f);
      }
      __syncthreads();
      loaded = p;
    }
    const float emb = p < a.nk ? w.P[kO_EMB + p] : 0.0f;
    const float* slot0 = slot_coefs(a.eval_ws) + (int64_t)p * a.max_cfg * kSlotFloats;
    const CfgRec* rec0 = slot_recs(a.eval_ws, a.n_progs, a.max_cfg) + (int64_t)p * a.max_cfg;
    for (int qi = qb + wv; qi < qe; qi += kSelWaves) {
      const int32_t N = a.queries[P.q0 + qi];
      const float fN = log2f((float)(N >= 1 ? N : 1)) * (1.0f / 26.0f);
      float xs[KLR_N_METRICS];
      scaled_n(N, slot0, xs);
      // the lane's kMaxShortlist lowest predictions (value, index), ascending; configurations
      // arrive in increasing index order, so an equal value stays behind the earlier one
      float tv[kMaxShortlist];
      int ti[kMaxShortlist];
#pragma unroll
      for (int s2 = 0; s2 < kMaxShortlist; ++s2) { tv[s2] = INFINITY; ti[s2] = 0x7fffffff; }
      for (int c0 = 0; c0 < P.n_cfg; c0 += 64) {
        // the network ranks only the configurations the exact program admits at this N: lane
        // group g checks configuration c0 + 32 g + lane % 32, the other group's result arrives by
        // one lane swap
        bool adm[2];
        {
          const int c = c0 + 32 * g + (lane & 31);
          const int cc = c < P.n_cfg ? c : P.n_cfg - 1;
          const bool mine = c < P.n_cfg &&
                            point_admissible(P.cost_kind, N, xs, slot0 + (int64_t)cc * kSlotFloats, rec0[cc], hw);
          const bool theirs = __shfl_xor((int)mine, 32) != 0;
          adm[0] = g == 0 ? mine : theirs;
          adm[1] = g == 0 ? theirs : mine;
        }
        // layer 1 for two tiles of 32 configurations
        bf16x8 h1[2][16];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
          int c = c0 + 32 * rt + (lane & 31);
          c = c < P.n_cfg ? c : P.n_cfg - 1;
          const float2 cx = S.cfx[c];
          const float xb0 = g == 0 ? fN : cx.x;       // features 0, 1 (k-step 0)
          const float xb1 = g == 0 ? cx.y : emb;      // features 2, 3 (k-step 1)
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            f32x16 acc;
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = S.b1f[t][g][r];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(w1r[t][0], xb0, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(w1r[t][1], xb1, acc, 0, 0, 0);
#pragma unroll
            for (int half = 0; half < 2; ++half) {
              uint4 u;
              u.x = pack_bf16(fmaxf(acc[8 * half + 0], 0.0f), fmaxf(acc[8 * half + 1], 0.0f));
              u.y = pack_bf16(fmaxf(acc[8 * half + 2], 0.0f), fmaxf(acc[8 * half + 3], 0.0f));
              u.z = pack_bf16(fmaxf(acc[8 * half + 4], 0.0f), fmaxf(acc[8 * half + 5], 0.0f));
              u.w = pack_bf16(fmaxf(acc[8 * half + 6], 0.0f), fmaxf(acc[8 * half + 7], 0.0f));
              h1[rt][2 * t + half] = *reinterpret_cast<bf16x8*>(&u);
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        // layers 2 and 3
        float yp[2] = {0.0f, 0.0f};
        for (int t2 = 0; t2 < 8; ++t2) {
          f32x16 acc0, acc1;
#pragma unroll
          for (int r = 0; r < 16; ++r) acc0[r] = acc1[r] = S.b2f[t2][g][r];
          // W2 fragments are loaded one k-block ahead; the scheduling barriers keep the compiler
          // from hoisting all sixteen loads (64 registers) next to the 128 registers of H1
          uint4 wa = S.w2f[(t2 * 16) * 64 + lane];
#pragma unroll
          for (int kb = 0; kb < 16; ++kb) {
            uint4 wn = wa;
            if (kb + 1 < 16) wn = S.w2f[(t2 * 16 + kb + 1) * 64 + lane];
            const bf16x8 av = *reinterpret_cast<const bf16x8*>(&wa);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, h1[0][kb], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, h1[1][kb], acc1, 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
            wa = wn;
          }
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const float w3 = S.w3f[t2][g][r];
            yp[0] += w3 * fmaxf(acc0[r], 0.0f);
            yp[1] += w3 * fmaxf(acc1[r], 0.0f);
          }
        }
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
          const float other = __shfl_xor(yp[rt], 32);
          const float y = (g == 0 ? yp[rt] + other : other + yp[rt]) + b3;   // same order in both groups
          const int c = c0 + 32 * rt + (lane & 31);
          if (adm[rt]) {
            float nv = mu + sig * y;
            int ni = c;
#pragma unroll
            for (int s2 = 0; s2 < kMaxShortlist; ++s2) {
              const bool lt = nv < tv[s2];
              const float t = tv[s2];
              const int u = ti[s2];
              tv[s2] = lt ? nv : t;
              ti[s2] = lt ? ni : u;
              nv = lt ? t : nv;
              ni = lt ? u : ni;
            }
          }
        }
      }
      // the group's lowest predictions in order: each round takes the (value, index) minimum of
      // the 32 configuration lanes' list heads and the lane that held it drops its head (both
      // lane groups hold the same lists and take the same steps); at least two rounds, for the
      // margin
      const int rounds = a.shortlist > 2 ? a.shortlist : 2;
      float cv[kMaxShortlist];
      int ci[kMaxShortlist];
#pragma unroll
      for (int r = 0; r < kMaxShortlist; ++r) {
        cv[r] = INFINITY;
        ci[r] = 0x7fffffff;
        if (r < rounds) {
          float hv = tv[0];
          int hi = ti[0];
#pragma unroll
          for (int off = 1; off <= 16; off <<= 1) {
            const float ov = __shfl_xor(hv, off);
            const int oi = __shfl_xor(hi, off);
            if (ov < hv || (ov == hv && oi < hi)) { hv = ov; hi = oi; }
          }
          cv[r] = hv;
          ci[r] = hi;
          if (ti[0] == hi) {
#pragma unroll
            for (int s2 = 0; s2 + 1 < kMaxShortlist; ++s2) { tv[s2] = tv[s2 + 1]; ti[s2] = ti[s2 + 1]; }
            tv[kMaxShortlist - 1] = INFINITY;
            ti[kMaxShortlist - 1] = 0x7fffffff;
          }
        }
      }
      const bool found = ci[0] != 0x7fffffff;
      const float marg = cv[1] - cv[0];                 // +inf with a single candidate
      bool fell = !found || !(marg >= lnm);
      int pick = found ? ci[0] : -1;
      float pv = cv[0];
      if (!fell) {                                      // wave-uniform
        // exact costs of the shortlist, lane r < shortlist taking candidate r; the lowest exact
        // cost wins, lowest index on ties; none finite falls back
        int c = 0x7fffffff;
        float cp = INFINITY;
#pragma unroll
        for (int r = 0; r < kMaxShortlist; ++r)
          if (lane == r && r < a.shortlist) { c = ci[r]; cp = cv[r]; }
        float xc = INFINITY;
        if (c != 0x7fffffff) {
          const float* cf = slot0 + (int64_t)c * kSlotFloats;
          xc = P.grid_kind == KLR_GRID_1D ? any_cost<KLR_GRID_1D, kNdeg, false>(P.cost_kind, N, xs, cf, rec0[c], hw)
                                          : any_cost<KLR_GRID_2D, kNdeg, false>(P.cost_kind, N, xs, cf, rec0[c], hw);
        }
#pragma unroll
        for (int off = 1; off < kMaxShortlist; off <<= 1) {
          const float ox = __shfl_xor(xc, off);
          const int oc = __shfl_xor(c, off);
          const float op = __shfl_xor(cp, off);
          if (ox < xc || (ox == xc && oc < c)) { xc = ox; c = oc; cp = op; }
        }
        xc = __shfl(xc, 0);
        c = __shfl(c, 0);
        cp = __shfl(cp, 0);
        if (xc < INFINITY) {
          pick = c;
          pv = cp;
        } else {
          fell = true;
        }
      }
      if (lane == 0) {
        const int64_t o = P.q0 + qi;
        a.argmin[o] = pick;
        a.pred_cost[o] = found ? expf(pv) : INFINITY;
        a.fell_back[o] = fell ? 1 : 0;
        if (a.pred_margin) a.pred_margin[o] = found ? marg : NAN;
      }
    }
  }
}

Blob blob_of(void* base, int32_t nk) {
  float* f = reinterpret_cast<float*>(base);
  const int64_t np = mlp_np(nk);
  Blob b;
  b.hdr = f;
  b.P = f + 16;
  b.M = b.P + np;
  b.V = b.M + np;
  b.W2b = reinterpret_cast<uint16_t*>(b.V + np);
  b.W2Tb = b.W2b + H * H;
  return b;
}

hipError_t launch_refresh(const Blob& w, hipStream_t s) {
  hipLaunchKernelGGL(mlp_refresh, dim3(H * H / kBlock), dim3(kBlock), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_stats(const float* cost, int64_t n, float* hdr, hipStream_t s) {
  hipLaunchKernelGGL(mlp_stats, dim3(1), dim3(1024), 0, s, cost, n, hdr);
  return hipGetLastError();
}

hipError_t launch_train_step(const TrainTile& t, const Blob& w, const AdamArgs& ad, float* grads,
                             float* loss_step, float* loss_epoch, float epoch_scale, hipStream_t s) {
  const int ntiles = t.B / TS;
  hipLaunchKernelGGL(mlp_fwd_bwd, dim3(ntiles), dim3(kBlock), 0, s, t, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_dw2_part, dim3(kDw2Tiles * kDw2Slices), dim3(64 * kDw2Waves), 0, s, t.dH2T, t.H1T,
                     t.B, t.dw2_part);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nsmall = kO_B3 - kO_W1 + 1;
  const int64_t nthr = (int64_t)H * H + (int64_t)(nsmall + 1) * kSmallLanes + t.nk;
  hipLaunchKernelGGL(mlp_small_adam, dim3((nthr + kBlock - 1) / kBlock), dim3(kBlock), 0, s, t.partial,
                     ntiles, t.emb_acc, t.nk, w, ad, grads, loss_step, loss_epoch, epoch_scale, t.B,
                     t.dw2_part);
  return hipGetLastError();
}

hipError_t launch_predict(const int32_t* kid, const int32_t* N, const int32_t* L, int64_t n, int32_t nk,
                          const Blob& w, float* pred, hipStream_t s) {
  const int64_t tiles = (n + TS - 1) / TS;
  hipLaunchKernelGGL(mlp_predict, dim3((unsigned)tiles), dim3(kBlock), 0, s, kid, N, L, n, nk, w, pred);
  return hipGetLastError();
}

hipError_t launch_select(const SelectArgs& a, const Blob& w, hipStream_t s) {
  if (a.max_q <= 0 || a.n_progs <= 0) return hipSuccess;
  const int chunks = (a.max_q + kSelQ - 1) / kSelQ;
  const int64_t n_items = (int64_t)a.n_progs * chunks;
  const size_t lds = sizeof(SelLds);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mlp_select),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int dev = 0, ncu = 0;
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int64_t grid = n_items < ncu ? n_items : ncu;     // one persistent workgroup per CU
  hipLaunchKernelGGL(mlp_select, dim3((unsigned)grid), dim3(64 * kSelWaves), lds, s, a, w, chunks, n_items);
  return hipGetLastError();
}

}  // namespace klr

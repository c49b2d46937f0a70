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
//   mlp_dw2_adam    dW2 = dA2^T h1 over the batch on v_mfma_f32_16x16x32_bf16 (one 16 x 16
//                   output tile per workgroup, the batch split over its 4 waves and summed in a
//                   fixed order), Adam on W2, refresh of W2b / W2Tb
//   mlp_small_adam  fixed-order sum of the per-tile partials, Adam on W1, b1, b2, w3, b3 and
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

__device__ __forceinline__ float sum32(float v) {
#pragma unroll
  for (int off = 16; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

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
      gw3[ct] += __shfl_xor(gw3[ct], 32);
      gb2[ct] += __shfl_xor(gb2[ct], 32);
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
      for (int f = 0; f < 4; ++f) gw1[ct][f] += __shfl_xor(gw1[ct][f], 32);
      gb1[ct] += __shfl_xor(gb1[ct], 32);
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
  if (tid == 0) {
    float sdy = 0.0f, sl = 0.0f;
    for (int s = 0; s < TS; ++s) { sdy += dys[s]; sl += lss[s]; }
    prt[kO_B3 - kO_W1] = sdy;
    prt[kLossSlot] = sl;
  }
}

__global__ void __launch_bounds__(kBlock)
mlp_dw2_adam(const uint16_t* __restrict__ dH2T, const uint16_t* __restrict__ H1T, int32_t B, Blob w,
             AdamArgs ad, float* grads) {
  __shared__ float red[4][16][16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tj = blockIdx.x / (H / 16), tk = blockIdx.x % (H / 16);
  const int per = B / 4;
  const int sbeg = wv * per, send = sbeg + per;
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  const int row = lane & 15, kh = 8 * (lane >> 4);
  const uint16_t* pa = dH2T + (int64_t)(16 * tj + row) * B + kh;
  const uint16_t* pb = H1T + (int64_t)(16 * tk + row) * B + kh;
  for (int s = sbeg; s < send; s += 32)
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(pa + s), ld8(pb + s), acc, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < 4; ++r) red[wv][4 * (lane >> 4) + r][lane & 15] = acc[r];
  __syncthreads();
  const int rr = threadIdx.x / 16, cc = threadIdx.x % 16;
  const float g = (red[0][rr][cc] + red[1][rr][cc]) + (red[2][rr][cc] + red[3][rr][cc]);
  const int j = 16 * tj + rr, k = 16 * tk + cc;
  const int idx = kO_W2 + j * H + k;
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
}

__global__ void __launch_bounds__(kBlock)
mlp_small_adam(const float* __restrict__ partial, int32_t ntiles, unsigned long long* emb_acc,
               int32_t nk, Blob w, AdamArgs ad, float* grads, float* loss_step, float* loss_epoch,
               float epoch_scale, int32_t B) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int nsmall = kO_B3 - kO_W1 + 1;
  int idx = -1;
  float g = 0.0f;
  if (i < nsmall) {
    for (int t = 0; t < ntiles; ++t) g += partial[(int64_t)t * kPartialStride + i];
    idx = kO_W1 + i;
  } else if (i - nsmall < nk) {
    const int k = i - nsmall;
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
  if (i == 0) {
    float L = 0.0f;
    for (int t = 0; t < ntiles; ++t) L += partial[(int64_t)t * kPartialStride + kLossSlot];
    L /= (float)B;
    if (loss_step) *loss_step = L;
    if (loss_epoch) *loss_epoch += L * epoch_scale;
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

// Surrogate selection: one workgroup = one program x kSelQ queries; each query's configurations
// are processed in 64-row tiles; the running best / second-best predictions live in LDS.
constexpr int kSelQ = 8;
constexpr int kSelMaxCfg = 1024;

__global__ void __launch_bounds__(kBlock)
mlp_select(SelectArgs a, Blob w, int chunks) {
  __shared__ __attribute__((aligned(16))) uint16_t H1s[TS * HP];
  __shared__ float xs[TS][4];
  __shared__ float part[4][TS];
  __shared__ float cfx[kSelMaxCfg][2];
  __shared__ int cT[kSelMaxCfg], cL[kSelMaxCfg];
  __shared__ float best_v, second_v;
  __shared__ int best_i;
  const int tid = threadIdx.x;
  const int p = blockIdx.x / chunks;
  const int qb = (blockIdx.x % chunks) * kSelQ;
  if (p >= a.n_progs) return;
  const klr_program P = a.progs[p];
  const bool range_ok = P.reserved == 0 && P.n_q >= 0 && P.n_q <= a.max_q && P.q0 >= 0 &&
                        P.q0 + (int64_t)P.n_q <= a.q_len;
  if (!range_ok || qb >= P.n_q) return;
  const bool sel_ok = P.v_launch == 2 && P.n_cfg >= 0 && P.n_cfg <= a.max_cfg && P.n_cfg <= kSelMaxCfg &&
                      P.cfg0 >= 0 && P.cfg0 + 2 * (int64_t)P.n_cfg <= a.cfgs_len;
  if (!sel_ok) {   // not representable by the network: leave the whole query to the exact path
    if (tid < kSelQ && qb + tid < P.n_q) {
      const int64_t o = P.q0 + qb + tid;
      a.argmin[o] = -1;
      a.pred_cost[o] = INFINITY;
      a.fell_back[o] = 1;
    }
    return;
  }
  const float emb = p < a.nk ? w.P[kO_EMB + p] : 0.0f;
  for (int c = tid; c < P.n_cfg; c += kBlock) {
    const int32_t bx = a.cfgs[P.cfg0 + 2 * c], by = a.cfgs[P.cfg0 + 2 * c + 1];
    const bool pos = bx >= 1 && by >= 1;
    const int64_t T = pos ? (int64_t)bx * by : 0;
    const bool ok = pos && T <= a.t_max && (T % a.wave) == 0;
    cfx[c][0] = log2f((float)(bx >= 1 ? bx : 1)) * 0.1f;
    cfx[c][1] = log2f((float)(by >= 1 ? by : 1)) * 0.1f;
    cT[c] = ok ? 1 : 0;
    cL[c] = bx > by ? bx : by;
  }
  __syncthreads();
  const float mu = w.hdr[0], sig = w.hdr[1];
  const float lnm = logf(1.0f + a.margin);
  const float b3 = w.P[kO_B3];
  for (int qi = qb; qi < qb + kSelQ && qi < P.n_q; ++qi) {
    const int32_t N = a.queries[P.q0 + qi];
    const float fN = log2f((float)(N >= 1 ? N : 1)) * (1.0f / 26.0f);
    if (tid == 0) { best_v = INFINITY; second_v = INFINITY; best_i = -1; }
    for (int c0 = 0; c0 < P.n_cfg; c0 += TS) {
      if (tid < TS) {
        const int c = c0 + tid < P.n_cfg ? c0 + tid : P.n_cfg - 1;
        xs[tid][0] = fN;
        xs[tid][1] = cfx[c][0];
        xs[tid][2] = cfx[c][1];
        xs[tid][3] = emb;
      }
      __syncthreads();
      layer1(w, xs, H1s, nullptr, 0, 0);
      __syncthreads();
      f32x16 acc[2][2];
      gemm_tile(H1s, w.W2b, acc);
      layer3_partial(w, acc, part);
      __syncthreads();
      if (tid < 64) {
        // (best, index, second) over the tile: lexicographic (value, index) minimum; the
        // second best collects the loser of every comparison, so equal values give margin 0
        const int c = c0 + tid;
        float b = INFINITY, sec = INFINITY;
        int bi = 0x7fffffff;
        if (c < P.n_cfg && cT[c] && cL[c] <= N) {
          const float y = ((part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid])) + b3;
          b = mu + sig * y;
          bi = c;
        }
#pragma unroll
        for (int off = 1; off <= 32; off <<= 1) {
          const float ob = __shfl_xor(b, off), os = __shfl_xor(sec, off);
          const int oi = __shfl_xor(bi, off);
          if (ob < b || (ob == b && oi < bi)) {
            sec = fminf(b, os);
            b = ob;
            bi = oi;
          } else {
            sec = fminf(sec, ob);
          }
        }
        if (tid == 0) {     // the running result holds lower indices: it wins ties
          if (b < best_v) {
            second_v = fminf(best_v, sec);
            best_v = b;
            best_i = bi;
          } else {
            second_v = fminf(second_v, b);
          }
        }
      }
      __syncthreads();
    }
    if (tid == 0) {
      const int64_t o = P.q0 + qi;
      a.argmin[o] = best_i;
      a.pred_cost[o] = best_i >= 0 ? expf(best_v) : INFINITY;
      a.fell_back[o] = (best_i < 0 || !(second_v - best_v >= lnm)) ? 1 : 0;
    }
    __syncthreads();
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
  hipLaunchKernelGGL(mlp_dw2_adam, dim3((H / 16) * (H / 16)), dim3(kBlock), 0, s, t.dH2T, t.H1T, t.B, w,
                     ad, grads);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nsmall = kO_B3 - kO_W1 + 1;
  const int nthr = nsmall + t.nk;
  hipLaunchKernelGGL(mlp_small_adam, dim3((nthr + kBlock - 1) / kBlock), dim3(kBlock), 0, s, t.partial,
                     ntiles, t.emb_acc, t.nk, w, ad, grads, loss_step, loss_epoch, epoch_scale, t.B);
  return hipGetLastError();
}

hipError_t launch_predict(const int32_t* kid, const int32_t* N, const int32_t* L, int64_t n, int32_t nk,
                          const Blob& w, float* pred, hipStream_t s) {
  const int64_t tiles = (n + TS - 1) / TS;
  hipLaunchKernelGGL(mlp_predict, dim3((unsigned)tiles), dim3(kBlock), 0, s, kid, N, L, n, nk, w, pred);
  return hipGetLastError();
}

hipError_t launch_select(const SelectArgs& a, const Blob& w, hipStream_t s) {
  const int chunks = (a.max_q + kSelQ - 1) / kSelQ;
  if (a.max_q == 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_select, dim3((unsigned)a.n_progs * chunks), dim3(kBlock), 0, s, a, w, chunks);
  return hipGetLastError();
}

}  // namespace klr

// Data collection on the GPU: timing target kernels at sample points (N, launch configuration).
//
// Paper: step 1 of the section "An Algorithm to Build and Deploy a Performance-Predicting
// Rational Program" and section "Building a Driver Program: Data collection" - the program is run
// at a set K of sample points (data and program parameters) and a performance metric is measured
// at each, giving the values V that the rational functions are fitted to.  Here the metric is
// the kernel's time (HIP events around repeated launches on the caller's stream), which a
// metric-cost program (KLR_COST_METRIC) then fits and minimises directly, and the static
// resource usage (registers per thread, LDS bytes per block) comes from the compiled kernel's
// attributes.
//
// Target kernels (single-precision N x N grids, one thread per element, 2-D blocks bx x by):
//   KLR_TARGET_TRANSPOSE  out[x][y] = in[y][x]: reads coalesced along x, writes strided;
//   KLR_TARGET_STENCIL    five-point Jacobi step with a fixed boundary;
// both launch ceil(N / bx) x ceil(N / by) blocks and guard every access by the grid bounds.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "internal.hpp"

namespace klr {
namespace {

__global__ void target_transpose(const float* __restrict__ in, float* __restrict__ out, int n) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x < n && y < n) out[(int64_t)x * n + y] = in[(int64_t)y * n + x];
}

__global__ void target_stencil(const float* __restrict__ in, float* __restrict__ out, int n) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= n || y >= n) return;
  const int64_t i = (int64_t)y * n + x;
  if (x == 0 || y == 0 || x == n - 1 || y == n - 1) {
    out[i] = in[i];
    return;
  }
  out[i] = 0.2f * (in[i] + in[i - 1] + in[i + 1] + in[i - n] + in[i + n]);
}

const void* target_fn(int32_t target) {
  switch (target) {
    case KLR_TARGET_TRANSPOSE: return reinterpret_cast<const void*>(&target_transpose);
    case KLR_TARGET_STENCIL: return reinterpret_cast<const void*>(&target_stencil);
    default: return nullptr;
  }
}

hipError_t launch_target(int32_t target, int32_t n, int32_t bx, int32_t by, const float* in, float* out,
                         hipStream_t s) {
  const dim3 grid((unsigned)((n + bx - 1) / bx), (unsigned)((n + by - 1) / by));
  const dim3 block((unsigned)bx, (unsigned)by);
  if (target == KLR_TARGET_TRANSPOSE)
    hipLaunchKernelGGL(target_transpose, grid, block, 0, s, in, out, n);
  else
    hipLaunchKernelGGL(target_stencil, grid, block, 0, s, in, out, n);
  return hipGetLastError();
}

}  // namespace
}  // namespace klr

using klr::fail;

extern "C" {

size_t klr_collect_buffer(int32_t target, int32_t max_n) {
  if (!klr::target_fn(target) || max_n < 1 || max_n > KLR_COLLECT_MAX_N) return 0;
  return (size_t)2 * (size_t)max_n * (size_t)max_n * sizeof(float);
}

klr_status klr_target_attributes(klr_handle h, int32_t target, int32_t* regs, int32_t* lds_bytes) {
  if (!h) return KLR_E_INVALID;
  h->err.clear();
  const void* fn = klr::target_fn(target);
  if (!fn || !regs || !lds_bytes) return fail(h, KLR_E_INVALID, "klr_target_attributes: bad arguments");
  hipFuncAttributes at{};
  klr_status st = klr::hip_check(h, hipFuncGetAttributes(&at, fn), "hipFuncGetAttributes");
  if (st != KLR_OK) return st;
  *regs = at.numRegs;
  *lds_bytes = (int32_t)at.sharedSizeBytes;
  return KLR_OK;
}

klr_status klr_collect_times(klr_handle h, int32_t target, const int32_t* samples, int32_t n_samples,
                             int32_t reps, double* time_us, void* buf, size_t buf_bytes, void* stream) {
  if (!h) return KLR_E_INVALID;
  h->err.clear();
  if (!klr::target_fn(target) || n_samples < 0 || reps < 1 || reps > 1000 || (n_samples > 0 && (!samples || !time_us)))
    return fail(h, KLR_E_INVALID, "klr_collect_times: bad arguments");
  if (n_samples == 0) return KLR_OK;
  // every sample checked before anything is launched: sizes, block shapes, buffer capacity
  int32_t max_n = 0;
  for (int32_t i = 0; i < n_samples; ++i) {
    const int32_t n = samples[3 * i], bx = samples[3 * i + 1], by = samples[3 * i + 2];
    if (n < 1 || n > KLR_COLLECT_MAX_N || bx < 1 || by < 1 || (int64_t)bx * by > 1024 || by > 1024)
      return fail(h, KLR_E_INVALID, "klr_collect_times: sample " + std::to_string(i) +
                                        " outside 1 <= N <= KLR_COLLECT_MAX_N, bx by <= 1024");
    max_n = n > max_n ? n : max_n;
  }
  const size_t need = klr_collect_buffer(target, max_n);
  if (!buf || buf_bytes < need)
    return fail(h, KLR_E_WORKSPACE, "klr_collect_times: buffer too small: need " + std::to_string(need));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  float* in = reinterpret_cast<float*>(buf);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (int32_t i = 0; i < n_samples && e == hipSuccess; ++i) {
    const int32_t n = samples[3 * i], bx = samples[3 * i + 1], by = samples[3 * i + 2];
    float* out = in + (size_t)n * n;
    e = klr::launch_target(target, n, bx, by, in, out, s);              // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int32_t r = 0; r < reps && e == hipSuccess; ++r) e = klr::launch_target(target, n, bx, by, in, out, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) time_us[i] = 1e3 * (double)ms / reps;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return klr::hip_check(h, e, "klr_collect_times");
}

}  // extern "C"

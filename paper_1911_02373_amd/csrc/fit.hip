// Batched rational least-squares fits (placeholder until the kernels land).
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace klr {

size_t fit_workspace_bytes(int32_t n_fits, int32_t precision) {
  (void)precision;
  return (size_t)(n_fits > 0 ? n_fits : 0) * 256;
}

hipError_t launch_fit(const FitArgs& a) {
  (void)a;
  return hipErrorNotSupported;
}

}  // namespace klr

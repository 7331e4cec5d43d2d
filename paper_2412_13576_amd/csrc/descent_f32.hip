// Binary32 descent on MFMA (placeholder until the MFMA kernel lands).
#include <hip/hip_runtime.h>

#include "graver_internal.h"

namespace graver {

bool descent_f32_supported(int, int) { return false; }
size_t f32_pack_floats(int n, int d) { return (size_t)n * d; }
size_t f32_state_floats(int n, int d, int64_t N) { return (size_t)N * d * 3; }
hipError_t launch_f32_pack(hipStream_t, int, int, const int64_t*, float*, float*, int*) {
  return hipErrorNotSupported;
}
hipError_t launch_f32_state_io(hipStream_t, int, int, int64_t, float*, double*, double*, double*, int) {
  return hipErrorNotSupported;
}
hipError_t launch_descent_f32(hipStream_t, const DescentArgs&, const float*, const float*, float*, PoolDev,
                              unsigned long long*, float) {
  return hipErrorNotSupported;
}

}  // namespace graver

// Kernels for k = 16, r = 2^62 + 2^36.
#include "gfp_kernels.hpp"

namespace gfpk {

hipError_t launch_pass_16_62_36(const PassArgs& p, hipStream_t st) { return launch_pass_t<16, 62, 36>(p, st); }
hipError_t launch_elementwise_16_62_36(const EwArgs& a, hipStream_t st) {
  return launch_elementwise_t<16, 62, 36>(a, st);
}

}  // namespace gfpk

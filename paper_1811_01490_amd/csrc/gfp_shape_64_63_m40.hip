// Kernels for k = 64, r = 2^63 - 2^40.
#include "gfp_kernels.hpp"

namespace gfpk {

hipError_t launch_pass_64_63_m40(const PassArgs& p, hipStream_t st) { return launch_pass_t<64, 63, -40>(p, st); }
hipError_t launch_elementwise_64_63_m40(const EwArgs& a, hipStream_t st) {
  return launch_elementwise_t<64, 63, -40>(a, st);
}

}  // namespace gfpk

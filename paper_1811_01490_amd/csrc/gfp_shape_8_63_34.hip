// Kernels for k = 8, r = 2^63 + 2^34.
#include "gfp_kernels.hpp"

namespace gfpk {

hipError_t launch_pass_8_63_34(const PassArgs& p, hipStream_t st) { return launch_pass_t<8, 63, 34>(p, st); }
hipError_t launch_elementwise_8_63_34(const EwArgs& a, hipStream_t st) {
  return launch_elementwise_t<8, 63, 34>(a, st);
}

}  // namespace gfpk

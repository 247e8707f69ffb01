// Kernels for k = 32, r = 2^56 + 2^21.
#include "gfp_kernels.hpp"

namespace gfpk {

hipError_t launch_pass_32_56_21(const PassArgs& p, hipStream_t st) { return launch_pass_t<32, 56, 21>(p, st); }
hipError_t launch_elementwise_32_56_21(const EwArgs& a, hipStream_t st) {
  return launch_elementwise_t<32, 56, 21>(a, st);
}

hipError_t launch_persistent_32_56_21(const PLevel* levels, uint32_t nlevels, const PRec* recs, uint32_t* sync,
                                     uint32_t grid, hipStream_t st) {
  return launch_persistent_t<32, 56, 21>(levels, nlevels, recs, sync, grid, st);
}
int persistent_capacity_32_56_21(int* grid) { return persistent_capacity_t<32, 56, 21>(grid); }

hipError_t launch_table_build_32_56_21(const uint64_t* lo, const uint64_t* hi, int log2b, uint64_t cnt, uint32_t* tab,
                                      uint64_t* raw, hipStream_t st) {
  return launch_table_build_t<32, 56, 21>(lo, hi, log2b, cnt, tab, raw, st);
}

}  // namespace gfpk

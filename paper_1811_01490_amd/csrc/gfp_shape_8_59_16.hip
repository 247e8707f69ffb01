// Kernels for k = 8, r = 2^59 + 2^16.
#include "gfp_kernels.hpp"

namespace gfpk {

hipError_t launch_pass_8_59_16(const PassArgs& p, hipStream_t st) { return launch_pass_t<8, 59, 16>(p, st); }
hipError_t launch_elementwise_8_59_16(const EwArgs& a, hipStream_t st) {
  return launch_elementwise_t<8, 59, 16>(a, st);
}

hipError_t launch_persistent_8_59_16(const PLevel* levels, uint32_t nlevels, const PRec* recs, uint32_t* sync,
                                     uint32_t grid, hipStream_t st) {
  return launch_persistent_t<8, 59, 16>(levels, nlevels, recs, sync, grid, st);
}
int persistent_capacity_8_59_16(int* grid) { return persistent_capacity_t<8, 59, 16>(grid); }

hipError_t launch_table_build_8_59_16(const uint64_t* lo, const uint64_t* hi, int log2b, uint64_t cnt, uint32_t* tab,
                                      uint64_t* raw, hipStream_t st) {
  return launch_table_build_t<8, 59, 16>(lo, hi, log2b, cnt, tab, raw, st);
}

}  // namespace gfpk

// Kernels for k = 16, r = 2^62 + 2^36.
#include "gfp_kernels.hpp"

namespace gfpk {

hipError_t launch_pass_16_62_36(const PassArgs& p, hipStream_t st) { return launch_pass_t<16, 62, 36>(p, st); }
hipError_t launch_elementwise_16_62_36(const EwArgs& a, hipStream_t st) {
  return launch_elementwise_t<16, 62, 36>(a, st);
}

hipError_t launch_persistent_16_62_36(const PLevel* levels, uint32_t nlevels, const PRec* recs, uint32_t* sync,
                                     uint32_t grid, hipStream_t st) {
  return launch_persistent_t<16, 62, 36>(levels, nlevels, recs, sync, grid, st);
}
int persistent_capacity_16_62_36(int* grid) { return persistent_capacity_t<16, 62, 36>(grid); }

hipError_t launch_table_build_16_62_36(const uint64_t* lo, const uint64_t* hi, int log2b, uint64_t cnt, uint32_t* tab,
                                      uint64_t* raw, hipStream_t st) {
  return launch_table_build_t<16, 62, 36>(lo, hi, log2b, cnt, tab, raw, st);
}

}  // namespace gfpk

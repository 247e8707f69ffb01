// Kernels for k = 64, r = 2^63 - 2^40.
#include "gfp_kernels.hpp"

namespace gfpk {

hipError_t launch_pass_64_63_m40(const PassArgs& p, hipStream_t st) { return launch_pass_t<64, 63, -40>(p, st); }
hipError_t launch_elementwise_64_63_m40(const EwArgs& a, hipStream_t st) {
  return launch_elementwise_t<64, 63, -40>(a, st);
}

hipError_t launch_persistent_64_63_m40(const PLevel* levels, uint32_t nlevels, const PRec* recs, uint32_t* sync,
                                     uint32_t grid, hipStream_t st) {
  return launch_persistent_t<64, 63, -40>(levels, nlevels, recs, sync, grid, st);
}
int persistent_capacity_64_63_m40(int* grid) { return persistent_capacity_t<64, 63, -40>(grid); }

hipError_t launch_table_build_64_63_m40(const uint64_t* lo, const uint64_t* hi, int log2b, uint64_t cnt, uint32_t* tab,
                                      uint64_t* raw, hipStream_t st) {
  return launch_table_build_t<64, 63, -40>(lo, hi, log2b, cnt, tab, raw, st);
}

}  // namespace gfpk

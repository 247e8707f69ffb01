// Dispatch from a runtime radix shape to the kernels compiled for it.
#include "gfp_internal.hpp"

namespace gfpk {

// Radix shapes compiled in (k, W, U; r = 2^W + 2^U, or 2^W - 2^-U for U < 0):
// the k = 8, 16, 32 and 64 primes of Table 1 and the three test primes of
// section 5.3 (Table testprimes).
#define GFP_FOR_EACH_SHAPE(X) \
  X(8, 63, 34, 8_63_34)       \
  X(8, 59, 16, 8_59_16)       \
  X(16, 62, 36, 16_62_36)     \
  X(16, 58, 10, 16_58_10)     \
  X(32, 62, 56, 32_62_56)     \
  X(32, 56, 21, 32_56_21)     \
  X(64, 63, -40, 64_63_m40)

#define GFP_DECLARE(K, W, U, TAG)                                                                             \
  hipError_t launch_pass_##TAG(const PassArgs& p, hipStream_t st);                                           \
  hipError_t launch_elementwise_##TAG(const EwArgs& a, hipStream_t st);                                      \
  hipError_t launch_persistent_##TAG(const PLevel* levels, uint32_t nlevels, const PRec* recs, uint32_t* sync, \
                                     uint32_t grid, hipStream_t st);                                           \
  int persistent_capacity_##TAG(int* grid);                                                                  \
  hipError_t launch_table_build_##TAG(const uint64_t* lo, const uint64_t* hi, int log2b, uint64_t cnt,        \
                                      uint32_t* tab, uint64_t* raw, hipStream_t st);
GFP_FOR_EACH_SHAPE(GFP_DECLARE)
#undef GFP_DECLARE

bool shape_supported(int k, int w, int u) {
#define GFP_SHAPE_CASE(K, W, U, TAG) \
  if (k == K && w == W && u == U) return true;
  GFP_FOR_EACH_SHAPE(GFP_SHAPE_CASE)
#undef GFP_SHAPE_CASE
  return false;
}

bool span2_supported(int k) { return k == 8 || k == 16; }
bool wide_supported(int k) { return k == 8; }

hipError_t launch_pass(int k, int w, int u, const PassArgs& p, hipStream_t st) {
#define GFP_SHAPE_CASE(K, W, U, TAG) \
  if (k == K && w == W && u == U) return launch_pass_##TAG(p, st);
  GFP_FOR_EACH_SHAPE(GFP_SHAPE_CASE)
#undef GFP_SHAPE_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_elementwise(int k, int w, int u, const EwArgs& a, hipStream_t st) {
#define GFP_SHAPE_CASE(K, W, U, TAG) \
  if (k == K && w == W && u == U) return launch_elementwise_##TAG(a, st);
  GFP_FOR_EACH_SHAPE(GFP_SHAPE_CASE)
#undef GFP_SHAPE_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_persistent(int k, int w, int u, const PLevel* levels, uint32_t nlevels, const PRec* recs,
                             uint32_t* sync, uint32_t grid, hipStream_t st) {
#define GFP_SHAPE_CASE(K, W, U, TAG) \
  if (k == K && w == W && u == U) return launch_persistent_##TAG(levels, nlevels, recs, sync, grid, st);
  GFP_FOR_EACH_SHAPE(GFP_SHAPE_CASE)
#undef GFP_SHAPE_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_table_build(int k, int w, int u, const uint64_t* lo, const uint64_t* hi, int log2b, uint64_t cnt,
                              uint32_t* tab, uint64_t* raw, hipStream_t st) {
#define GFP_SHAPE_CASE(K, W, U, TAG) \
  if (k == K && w == W && u == U) return launch_table_build_##TAG(lo, hi, log2b, cnt, tab, raw, st);
  GFP_FOR_EACH_SHAPE(GFP_SHAPE_CASE)
#undef GFP_SHAPE_CASE
  return hipErrorInvalidValue;
}

int persistent_capacity(int k, int w, int u, int* grid) {
#define GFP_SHAPE_CASE(K, W, U, TAG) \
  if (k == K && w == W && u == U) return persistent_capacity_##TAG(grid);
  GFP_FOR_EACH_SHAPE(GFP_SHAPE_CASE)
#undef GFP_SHAPE_CASE
  *grid = 0;
  return 0;
}

}  // namespace gfpk

// Declarations shared by the host side (gfp_host.cpp) and the kernel
// launchers (gfp_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gfp.h"

namespace gfpk {

// Vector addressing: digit d of element i is at base[i * se + d * sd].
// Digit-major (the ABI's layout): se = 1, sd = ld.  Element-major (used
// between passes, one element = k contiguous digits): se = k, sd = 1.
struct PassArgs {
  const uint64_t* in;
  uint64_t se_in, sd_in;
  uint64_t* out;
  uint64_t se_out, sd_out;
  const uint32_t* tw;  // twiddle table (or the single scale entry when scale)
  int log2n;
  int log2ns;
  uint64_t ngroups;  // n / K
  bool inverse;
  bool scale;  // inverse pass 0: multiply every slot by tw[0] (1/n)
  bool last;   // canonical output
};

struct EwArgs {
  int op;
  const uint64_t* x;
  uint64_t ldx;
  const uint64_t* y;
  uint64_t ldy;
  uint64_t* z;
  uint64_t ldz;
  uint64_t n;
  int64_t s;
  const uint32_t* cst;  // one twiddle-layout entry (device)
};

bool shape_supported(int k, int w, int u);
hipError_t launch_pass(int k, int w, int u, const PassArgs& p, hipStream_t st);
hipError_t launch_elementwise(int k, int w, int u, const EwArgs& a, hipStream_t st);

// words per twiddle-table entry (see TwLayout in gfp_device.hpp)
inline int tw_words(int k) { return (6 * k + 6) & ~3; }

}  // namespace gfpk

// Device side of the copies between caller vectors and work vectors, shared
// by the copy kernels and the persistent batch kernel.
#pragma once
#include <hip/hip_runtime.h>

#include "gfp_internal.hpp"

namespace gfpk {

// Unpad through LDS, one tile of E = 1024 / k elements per workgroup: the
// tile's 1024 element-major words are read contiguously (4 per thread,
// coalesced), transposed in LDS (rows padded to k + 1 words, so that the
// column reads of the second phase spread over the banks) and written as k
// digit rows of E consecutive coefficients (coalesced).  Reading the work
// vector with a stride of k words instead fetched 8x (k = 8) to 16x (k = 16)
// its bytes, as each 64- or 128-byte line left L2 before its other digits
// were read: the 2^19 x 2^19 products went 816 -> 760 us (k = 8) and
// 2167 -> 1916 us (k = 16).  Tiles of 4096 words were 1-7% slower on small
// products (fewer workgroups), 1024 equal to the strided copy there.  Only
// elements i < len are read or written; the tile index is uniform, so the
// early exit keeps every barrier whole.
constexpr int kUnpadWords = (int)kUnpadTileWords;
template <int KD>
__device__ __forceinline__ void unpad_tile(const CopyDesc& cd, const uint64_t* __restrict__ w, uint64_t tile,
                                           uint64_t* __restrict__ lds) {
  constexpr int E = kUnpadWords / KD;
  constexpr int PITCH = KD + 1;
  const uint64_t i0 = tile * E;
  if (i0 >= cd.len) return;
  const uint64_t* src = w + i0 * KD;
#pragma unroll
  for (int s = 0; s < kUnpadWords / 256; ++s) {
    const int o = (int)threadIdx.x + 256 * s;
    const int e = o / KD, d = o % KD;
    lds[e * PITCH + d] = (i0 + e < cd.len) ? src[o] : 0ull;
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < kUnpadWords / 256; ++s) {
    const int o = (int)threadIdx.x + 256 * s;
    const int d = o / E, e = o % E;
    if (i0 + e < cd.len) cd.dst[(uint64_t)d * cd.ld + i0 + e] = lds[e * PITCH + d];
  }
}

}  // namespace gfpk

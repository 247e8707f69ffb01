// Copies between caller vectors (digit-major) and the padded element-major
// work vectors of the batched product.  Zero padding is written by the
// kernel (no memset), so a captured graph can be replayed safely.
#include "gfp_copy.hpp"

namespace gfpk {

struct CopyBatch {
  CopyDesc d[kCopyBatch];
};

// thread -> (element i, digit d) of work vector blockIdx.y: work[v n k + i k + d],
// for the first cols elements
__global__ __launch_bounds__(256) void k_pad(const CopyBatch desc, uint64_t* __restrict__ work, uint64_t n,
                                             uint64_t cols, uint32_t k, uint32_t log2k) {
  const uint32_t v = blockIdx.y;
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cols * k) return;
  const uint64_t i = t >> log2k;
  const uint32_t d = (uint32_t)(t & (k - 1));
  const CopyDesc cd = desc.d[v];
  work[(uint64_t)v * n * k + t] = (i < cd.len) ? cd.src[(uint64_t)d * cd.ld + i] : 0ull;
}

// caller vector blockIdx.y, tile blockIdx.x (coefficients below len)
template <int KD>
__global__ __launch_bounds__(256) void k_unpad(const CopyBatch desc, const uint64_t* __restrict__ work, uint64_t n) {
  __shared__ uint64_t lds[kUnpadWords + kUnpadWords / KD];
  const uint32_t v = blockIdx.y;
  unpad_tile<KD>(desc.d[v], work + (uint64_t)v * n * KD, blockIdx.x, lds);
}

// The same two copies with the descriptors read from device memory (entry
// base + blockIdx.y), so that a captured launch sequence can be replayed for
// new requests by rewriting the descriptor table; unpad covers all n
// elements of each vector (entries past a descriptor's len write nothing).
__global__ __launch_bounds__(256) void k_pad_dev(const CopyDesc* __restrict__ desc, uint64_t* __restrict__ work,
                                                 uint64_t n, uint32_t k, uint32_t log2k) {
  const uint32_t v = blockIdx.y;
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * k) return;
  const uint64_t i = t >> log2k;
  const uint32_t d = (uint32_t)(t & (k - 1));
  const CopyDesc cd = desc[v];
  work[(uint64_t)v * n * k + t] = (i < cd.len) ? cd.src[(uint64_t)d * cd.ld + i] : 0ull;
}

template <int KD>
__global__ __launch_bounds__(256) void k_unpad_dev(const CopyDesc* __restrict__ desc,
                                                   const uint64_t* __restrict__ work, uint64_t n) {
  __shared__ uint64_t lds[kUnpadWords + kUnpadWords / KD];
  const uint32_t v = blockIdx.y;
  const CopyDesc cd = desc[v];
  unpad_tile<KD>(cd, work + (uint64_t)v * n * KD, blockIdx.x, lds);
}

// Elements of a digit-major vector that are not canonical (section 2: every
// digit below r, or p - 1 written as (0, ..., 0, r)), counted into *bad
// (vector atomics).  One thread per element.
__global__ __launch_bounds__(256) void k_check_canonical(const uint64_t* __restrict__ x, uint64_t ld, uint64_t n,
                                                         uint32_t k, uint64_t r, unsigned long long* bad) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ok = true;
  if (i < n) {
    const uint64_t top = x[(uint64_t)(k - 1) * ld + i];
    bool low_zero = true, below = top < r;
    for (uint32_t d = 0; d + 1 < k; ++d) {
      const uint64_t v = x[(uint64_t)d * ld + i];
      below = below && v < r;
      low_zero = low_zero && v == 0;
    }
    ok = below || (top == r && low_zero);
  }
  const uint64_t m = __ballot(!ok);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(bad, (unsigned long long)__popcll(m));
}

hipError_t launch_check_canonical(const uint64_t* x, uint64_t ld, uint64_t n, int k, uint64_t r, uint64_t* bad,
                                  hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_canonical, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, ld, n, (uint32_t)k, r,
                     (unsigned long long*)bad);
  return hipGetLastError();
}

hipError_t launch_pad(int k, const CopyDesc* d, uint32_t nvec, uint64_t* work, uint64_t n, uint64_t cols,
                      hipStream_t st) {
  if (nvec == 0 || cols == 0) return hipSuccess;
  if (nvec > kCopyBatch || cols > n) return hipErrorInvalidValue;
  CopyBatch b;
  for (uint32_t i = 0; i < nvec; ++i) b.d[i] = d[i];
  const uint64_t tot = cols * (uint64_t)k;
  dim3 grid((unsigned)((tot + 255) / 256), nvec);
  uint32_t lk = 0;
  while ((1u << lk) < (uint32_t)k) ++lk;
  hipLaunchKernelGGL(k_pad, grid, dim3(256), 0, st, b, work, n, cols, (uint32_t)k, lk);
  return hipGetLastError();
}

hipError_t launch_unpad(int k, const CopyDesc* d, uint32_t nvec, const uint64_t* work, uint64_t n, uint64_t maxlen,
                        hipStream_t st) {
  if (nvec == 0 || maxlen == 0) return hipSuccess;
  if (nvec > kCopyBatch || maxlen > n) return hipErrorInvalidValue;
  CopyBatch b;
  for (uint32_t i = 0; i < nvec; ++i) b.d[i] = d[i];
  const uint64_t E = kUnpadWords / (uint64_t)k;
  dim3 grid((unsigned)((maxlen + E - 1) / E), nvec);
  switch (k) {
    case 8: hipLaunchKernelGGL(k_unpad<8>, grid, dim3(256), 0, st, b, work, n); break;
    case 16: hipLaunchKernelGGL(k_unpad<16>, grid, dim3(256), 0, st, b, work, n); break;
    case 32: hipLaunchKernelGGL(k_unpad<32>, grid, dim3(256), 0, st, b, work, n); break;
    case 64: hipLaunchKernelGGL(k_unpad<64>, grid, dim3(256), 0, st, b, work, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pad_dev(int k, const CopyDesc* dev_desc, uint32_t nvec, uint64_t* work, uint64_t n,
                          hipStream_t st) {
  if (nvec == 0) return hipSuccess;
  if (nvec > 65535) return hipErrorInvalidValue;
  uint32_t lk = 0;
  while ((1u << lk) < (uint32_t)k) ++lk;
  dim3 grid((unsigned)((n * (uint64_t)k + 255) / 256), nvec);
  hipLaunchKernelGGL(k_pad_dev, grid, dim3(256), 0, st, dev_desc, work, n, (uint32_t)k, lk);
  return hipGetLastError();
}

hipError_t launch_unpad_dev(int k, const CopyDesc* dev_desc, uint32_t nvec, const uint64_t* work, uint64_t n,
                            hipStream_t st) {
  if (nvec == 0) return hipSuccess;
  if (nvec > 65535) return hipErrorInvalidValue;
  const uint64_t E = kUnpadWords / (uint64_t)k;
  dim3 grid((unsigned)((n + E - 1) / E), nvec);  // a descriptor's len is at most n
  switch (k) {
    case 8: hipLaunchKernelGGL(k_unpad_dev<8>, grid, dim3(256), 0, st, dev_desc, work, n); break;
    case 16: hipLaunchKernelGGL(k_unpad_dev<16>, grid, dim3(256), 0, st, dev_desc, work, n); break;
    case 32: hipLaunchKernelGGL(k_unpad_dev<32>, grid, dim3(256), 0, st, dev_desc, work, n); break;
    case 64: hipLaunchKernelGGL(k_unpad_dev<64>, grid, dim3(256), 0, st, dev_desc, work, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gfpk

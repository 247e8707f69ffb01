// Integer multiplication through the polynomial product over Z/pZ (the
// application of section 1: an integer is a polynomial evaluated at a power
// of two, so an integer product is a polynomial product followed by the
// evaluation, i.e. carries).
//
// An integer of n 64-bit words is cut into chunks of CW bits, CW = W for
// r = 2^W + 2^U and CW = W - 1 for r = 2^W - 2^U, so a chunk is below r and
// is one radix-r digit: no radix conversion on the way in.  The product's coefficients C_m = sum a_i b_(m-i) < L 2^(2W) are
// far below p, so their canonical digits give C_m = d0 + d1 r + d2 r^2 + d3 r^3
// exactly.  Output word w sums the 64-bit slices of every C_m 2^(W m) that
// overlaps it into lo_w + 2^64 hi_w; the carries between words are resolved
// by a carry-lookahead scan: word w holds c'_w = lo_w + hi_(w-1) mod 2^64,
// generates a carry when that sum overflowed and propagates one when
// c'_w = 2^64 - 1.
#include "gfp_internal.hpp"

namespace gfpk {

constexpr int kScanThreads = 1024;  // words per scan block

// coefficient i of a = bits [W i, W i + W) (digit 0; W here is the chunk
// width); digits 1..k-1 are 0
__global__ __launch_bounds__(256) void k_bigint_split(const uint64_t* __restrict__ a, uint64_t na,
                                                      uint64_t* __restrict__ A, uint64_t la, uint32_t k, uint32_t W) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= la * k) return;
  const uint64_t d = t / la, i = t - d * la;
  if (d != 0) {
    A[t] = 0;
    return;
  }
  const uint64_t bit = (uint64_t)W * i;
  const uint64_t w = bit >> 6;
  const uint32_t s = (uint32_t)(bit & 63);
  uint64_t v = a[w] >> s;
  if (s != 0 && w + 1 < na) v |= a[w + 1] << (64 - s);
  A[i] = v & ((1ull << W) - 1);
}

// v (5 words) = v r + d, r = 2^W + 2^U (U > 0) or 2^W - 2^-U (U < 0); the
// caller keeps v r below 2^320
__device__ __forceinline__ void mul_r_add(uint64_t (&v)[5], uint64_t d, uint32_t W, int U) {
  const uint32_t ua = (uint32_t)(U < 0 ? -U : U);
  uint64_t hw[5], hu[5];
  hw[0] = v[0] << W;
  hu[0] = v[0] << ua;
#pragma unroll
  for (int i = 1; i < 5; ++i) {
    hw[i] = (v[i] << W) | (v[i - 1] >> (64 - W));
    hu[i] = (v[i] << ua) | (v[i - 1] >> (64 - ua));
  }
  if (U > 0) {
    unsigned __int128 c = (unsigned __int128)d;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      c += (unsigned __int128)hw[i] + hu[i];
      v[i] = (uint64_t)c;
      c >>= 64;
    }
  } else {
    // v 2^W - v 2^ua + d >= 0: add d, subtract with borrow
    __int128 c = (__int128)d;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      c += (__int128)hw[i] - (__int128)hu[i];
      v[i] = (uint64_t)c;
      c >>= 64;  // arithmetic: -1, 0 or +1
    }
  }
}

// word w of sum_m C_m 2^(W m) as lo_w + 2^64 hi_w (hi_w small)
// (CW: chunk width; W, U: the radix)
__global__ __launch_bounds__(256) void k_bigint_combine(const uint64_t* __restrict__ C, uint64_t lc, uint32_t CW,
                                                        uint32_t W, int U, uint64_t nw, uint64_t* __restrict__ lo,
                                                        uint64_t* __restrict__ hi) {
  const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  // C_m 2^(CW m) spans bits [CW m, CW m + 320): it meets word w when
  // CW m < 64 w + 64 and CW m + 320 > 64 w
  const uint64_t top = (64 * w + 63) / CW;
  const uint64_t m_hi = top < lc - 1 ? top : lc - 1;
  const uint64_t m_lo = (64 * w >= 320) ? (64 * w - 320) / CW : 0;
  unsigned __int128 acc = 0;
  for (uint64_t m = m_lo; m <= m_hi; ++m) {
    uint64_t v[5] = {0, 0, 0, 0, 0};
    mul_r_add(v, C[3 * lc + m], W, U);
    mul_r_add(v, C[2 * lc + m], W, U);
    mul_r_add(v, C[1 * lc + m], W, U);
    mul_r_add(v, C[0 * lc + m], W, U);
    const int64_t s = (int64_t)((uint64_t)CW * m) - (int64_t)(64 * w);  // bit 0 of C_m relative to word w
    uint64_t slice;
    if (s >= 64 || s <= -320) {
      slice = 0;
    } else if (s >= 0) {
      slice = v[0] << s;
    } else {
      const uint32_t off = (uint32_t)(-s);
      const uint32_t q = off >> 6, sh = off & 63;
      const uint64_t x0 = v[q], x1 = (q + 1 < 5) ? v[q + 1] : 0;
      slice = sh ? ((x0 >> sh) | (x1 << (64 - sh))) : x0;
    }
    acc += slice;
  }
  lo[w] = (uint64_t)acc;
  hi[w] = (uint64_t)(acc >> 64);
}

// carry-lookahead within a wavefront: g, p per lane, carry into lane 0 = cin;
// returns the carry into this lane.  Adding X = G and Y = G | P bit by bit
// generates where g, propagates where p and kills elsewhere, so the carries
// of X + Y + cin are exactly the carries wanted: carry into bit i =
// bit i of (X + Y + cin) ^ X ^ Y.
__device__ __forceinline__ bool wave_carry(bool g, bool p, bool cin) {
  const uint64_t G = __ballot(g), P = __ballot(p);
  const uint64_t X = G, Y = G | P;
  const uint64_t S = X + Y + (cin ? 1ull : 0ull);
  const uint64_t carries = S ^ X ^ Y;
  const int lane = (int)(threadIdx.x & 63);
  return (carries >> lane) & 1;
}

// (generate, propagate) of a wavefront: carry out with carry-in 0, all propagate
__device__ __forceinline__ void wave_aggregate(bool g, bool p, bool& wg, bool& wp) {
  const uint64_t G = __ballot(g), P = __ballot(p);
  const uint64_t X = G, Y = G | P;
  const uint64_t S = X + Y;
  wg = S < X;  // unsigned overflow of X + Y
  wp = (P == ~0ull);
}

// word w: c'_w = lo_w + hi_(w-1), flags; block aggregate (generate, propagate)
__global__ __launch_bounds__(kScanThreads) void k_carry_prep(const uint64_t* __restrict__ lo,
                                                             const uint64_t* __restrict__ hi, uint64_t nw,
                                                             uint64_t* __restrict__ c, uint8_t* __restrict__ flags,
                                                             uint8_t* __restrict__ agg) {
  __shared__ uint8_t wgs[kScanThreads / 64], wps[kScanThreads / 64];
  const uint64_t w = (uint64_t)blockIdx.x * kScanThreads + threadIdx.x;
  bool g = false, p = false;
  if (w < nw) {
    const uint64_t a = lo[w], b = (w > 0) ? hi[w - 1] : 0;
    const uint64_t s = a + b;
    g = s < a;
    p = s == ~0ull;
    c[w] = s;
    flags[w] = (uint8_t)((g ? 1 : 0) | (p ? 2 : 0));
  }
  bool wg, wp;
  wave_aggregate(g, p, wg, wp);
  const int wv = (int)(threadIdx.x >> 6);
  if ((threadIdx.x & 63) == 0) {
    wgs[wv] = wg;
    wps[wv] = wp;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    bool cg = false, cp = true;
    for (int i = 0; i < kScanThreads / 64; ++i) {
      cg = wgs[i] || (wps[i] && cg);
      cp = cp && wps[i];
    }
    agg[blockIdx.x] = (uint8_t)((cg ? 1 : 0) | (cp ? 2 : 0));
  }
}

// carry into every block, from the block aggregates (one workgroup)
__global__ __launch_bounds__(kScanThreads) void k_carry_blocks(const uint8_t* __restrict__ agg, uint64_t nb,
                                                               uint8_t* __restrict__ cin) {
  __shared__ uint8_t wgs[kScanThreads / 64], wps[kScanThreads / 64];
  const uint64_t per = (nb + kScanThreads - 1) / kScanThreads;
  const uint64_t b0 = threadIdx.x * per, b1 = (b0 + per < nb) ? b0 + per : nb;
  // this thread's range as one (generate, propagate) pair
  bool g = false, p = true;
  for (uint64_t b = b0; b < b1; ++b) {
    const bool bg = agg[b] & 1, bp = (agg[b] >> 1) & 1;
    g = bg || (bp && g);
    p = p && bp;
  }
  bool wg, wp;
  wave_aggregate(g, p, wg, wp);
  const int wv = (int)(threadIdx.x >> 6);
  if ((threadIdx.x & 63) == 0) {
    wgs[wv] = wg;
    wps[wv] = wp;
  }
  __syncthreads();
  bool c = false;  // carry into this wavefront
  for (int i = 0; i < wv; ++i) c = wgs[i] || (wps[i] && c);
  bool ct = wave_carry(g, p, c);  // carry into this thread's range
  for (uint64_t b = b0; b < b1; ++b) {
    cin[b] = ct;
    const bool bg = agg[b] & 1, bp = (agg[b] >> 1) & 1;
    ct = bg || (bp && ct);
  }
}

// final words: c_w = c'_w + carry into w
__global__ __launch_bounds__(kScanThreads) void k_carry_apply(uint64_t* __restrict__ c,
                                                              const uint8_t* __restrict__ flags, uint64_t nw,
                                                              const uint8_t* __restrict__ cin) {
  __shared__ uint8_t wgs[kScanThreads / 64], wps[kScanThreads / 64];
  const uint64_t w = (uint64_t)blockIdx.x * kScanThreads + threadIdx.x;
  bool g = false, p = false;
  if (w < nw) {
    g = flags[w] & 1;
    p = (flags[w] >> 1) & 1;
  }
  bool wg, wp;
  wave_aggregate(g, p, wg, wp);
  const int wv = (int)(threadIdx.x >> 6);
  if ((threadIdx.x & 63) == 0) {
    wgs[wv] = wg;
    wps[wv] = wp;
  }
  __syncthreads();
  bool cw = cin[blockIdx.x] != 0;  // carry into this wavefront
  for (int i = 0; i < wv; ++i) cw = wgs[i] || (wps[i] && cw);
  const bool ci = wave_carry(g, p, cw);
  if (w < nw && ci) c[w] += 1;
}

hipError_t launch_bigint_split(const uint64_t* a, uint64_t na, uint64_t* A, uint64_t la, int k, int W,
                               hipStream_t st) {
  const uint64_t tot = la * (uint64_t)k;
  hipLaunchKernelGGL(k_bigint_split, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a, na, A, la,
                     (uint32_t)k, (uint32_t)W);
  return hipGetLastError();
}

hipError_t launch_bigint_combine(const uint64_t* C, uint64_t lc, int CW, int W, int U, uint64_t nw, uint64_t* lo,
                                 uint64_t* hi, hipStream_t st) {
  hipLaunchKernelGGL(k_bigint_combine, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st, C, lc, (uint32_t)CW,
                     (uint32_t)W, U, nw, lo, hi);
  return hipGetLastError();
}

uint64_t bigint_scan_blocks(uint64_t nw) { return (nw + kScanThreads - 1) / kScanThreads; }

hipError_t launch_bigint_carry(const uint64_t* lo, const uint64_t* hi, uint64_t nw, uint64_t* c, uint8_t* flags,
                               uint8_t* agg, uint8_t* cin, hipStream_t st) {
  const uint64_t nb = bigint_scan_blocks(nw);
  hipLaunchKernelGGL(k_carry_prep, dim3((unsigned)nb), dim3(kScanThreads), 0, st, lo, hi, nw, c, flags, agg);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_carry_blocks, dim3(1), dim3(kScanThreads), 0, st, agg, nb, cin);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_carry_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, st, c, flags, nw, cin);
  return hipGetLastError();
}

}  // namespace gfpk

// Integer multiplication through the polynomial product over Z/pZ (the
// application of section 1: an integer is a polynomial evaluated at a power
// of two, so an integer product is a polynomial product followed by the
// evaluation, i.e. carries).
//
// An integer of n 64-bit words is cut into chunks of b bits, b as large as
// the field allows: the product's coefficients C_m < min(la, lb) 2^(2b) must
// stay below p (about 2^(k W)), so b is about (k W - log2 min(la, lb)) / 2,
// at most 448.  Each chunk is converted to k radix-r digits by division
// (r = 2^U' d with d = 2^D +- 1).  The canonical digits of the product's
// coefficients give each C_m exactly; it is evaluated back to binary
// (Horner with r: shifts and adds), and output word w sums the 64-bit slices
// of every C_m 2^(b m) that overlaps it into lo_w + 2^64 hi_w; the carries
// between words are resolved by a carry-lookahead scan: word w holds
// c'_w = lo_w + hi_(w-1) mod 2^64, generates a carry when that sum overflowed
// and propagates one when c'_w = 2^64 - 1.
#include "gfp_device.hpp"
#include "gfp_internal.hpp"

namespace gfpk {

constexpr int kScanThreads = 1024;  // words per scan block

constexpr int kChunkWords = 7;  // chunk bits b <= 448
constexpr int kEvalWords = 16;  // product coefficients < 2^(2b + 64) <= 2^960

// x := x / r, returning x mod r, for r = 2^ua d (ua < 64, d < 2^49): the low
// ua bits are the low part of the remainder, and x >> ua is divided by d by
// long division in 15-bit pieces from the top (a remainder below 2^49 times
// 2^15 stays within 64 bits).
__device__ __forceinline__ uint64_t divmod_r(uint64_t (&x)[kChunkWords], uint32_t ua, uint64_t d) {
  const uint64_t lo = x[0] & ((1ull << ua) - 1);
  uint64_t y[kChunkWords];
  static_for<kChunkWords>([&](auto J) {
    constexpr int j = decltype(J)::value;
    y[j] = (x[j] >> ua) | ((j + 1 < kChunkWords) ? (x[j + 1 < kChunkWords ? j + 1 : j] << (64 - ua)) : 0ull);
    x[j] = 0;
  });
  constexpr int P = (64 * kChunkWords + 14) / 15;
  uint64_t rem = 0;
  static_for<P>([&](auto Q) {
    constexpr int pc = P - 1 - decltype(Q)::value;  // piece index, from the top
    constexpr int bit = 15 * pc, w0 = bit / 64, sh = bit % 64;
    uint64_t piece = y[w0] >> sh;
    if constexpr (sh > 64 - 15 && w0 + 1 < kChunkWords) piece |= y[w0 + 1] << (64 - sh);
    piece &= 0x7FFF;
    const uint64_t cur = (rem << 15) | piece;
    const uint64_t qd = cur / d;
    rem = cur - qd * d;
    x[w0] |= qd << sh;
    if constexpr (sh > 64 - 15 && w0 + 1 < kChunkWords) x[w0 + 1] |= qd >> (64 - sh);
  });
  return lo | (rem << ua);
}

// coefficient i of a = bits [b i, b i + b), converted to k radix-r digits
// (digit-major: A[d la + i]); the chunk is below 2^b < r^k
__global__ __launch_bounds__(256) void k_bigint_split(const uint64_t* __restrict__ a, uint64_t na,
                                                      uint64_t* __restrict__ A, uint64_t la, uint32_t k, uint32_t b,
                                                      uint32_t ua, uint64_t d) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= la) return;
  const uint64_t bit = (uint64_t)b * i;
  const uint64_t w = bit >> 6;
  const uint32_t s = (uint32_t)(bit & 63);
  const uint32_t nwb = (b + 63) / 64;
  uint64_t x[kChunkWords];
  static_for<kChunkWords>([&](auto J) {
    constexpr int j = decltype(J)::value;
    uint64_t v = 0;
    if ((uint32_t)j < nwb) {
      v = (w + j < na) ? a[w + j] >> s : 0ull;
      if (s != 0 && w + j + 1 < na) v |= a[w + j + 1] << (64 - s);
      const uint32_t top = b - 64 * j;  // bits of the chunk in this word
      if (top < 64) v &= (1ull << top) - 1;
    }
    x[j] = v;
  });
  for (uint32_t dg = 0; dg < k; ++dg) {
    uint64_t nz = 0;
    static_for<kChunkWords>([&](auto J) { nz |= x[decltype(J)::value]; });
    A[(uint64_t)dg * la + i] = nz ? divmod_r(x, ua, d) : 0ull;
  }
}

// v (kEvalWords words) = v r + dg, r = 2^W + 2^U (U > 0) or 2^W - 2^-U
// (U < 0); the caller keeps v r below 2^(64 kEvalWords)
__device__ __forceinline__ void mul_r_add(uint64_t (&v)[kEvalWords], uint64_t dg, uint32_t W, int U) {
  const uint32_t ua = (uint32_t)(U < 0 ? -U : U);
  if (U > 0) {
    unsigned __int128 c = (unsigned __int128)dg;
    uint64_t pw = 0, pu = 0;  // the word below, before this step
    static_for<kEvalWords>([&](auto J) {
      constexpr int j = decltype(J)::value;
      const uint64_t cur = v[j];
      const uint64_t hw = (cur << W) | (j ? pw >> (64 - W) : 0ull);
      const uint64_t hu = (cur << ua) | (j ? pu >> (64 - ua) : 0ull);
      pw = cur;
      pu = cur;
      c += (unsigned __int128)hw + hu;
      v[j] = (uint64_t)c;
      c >>= 64;
    });
  } else {
    // v 2^W - v 2^ua + dg >= 0: add dg, subtract with borrow
    __int128 c = (__int128)dg;
    uint64_t pw = 0;
    static_for<kEvalWords>([&](auto J) {
      constexpr int j = decltype(J)::value;
      const uint64_t cur = v[j];
      const uint64_t hw = (cur << W) | (j ? pw >> (64 - W) : 0ull);
      const uint64_t hu = (cur << ua) | (j ? pw >> (64 - ua) : 0ull);
      pw = cur;
      c += (__int128)hw - (__int128)hu;
      v[j] = (uint64_t)c;
      c >>= 64;  // arithmetic: -1, 0 or +1
    });
  }
}

// E[m] (kEvalWords words) = C_m as a binary integer, from its k canonical
// digits (Horner from the top nonzero digit)
__global__ __launch_bounds__(256) void k_bigint_eval(const uint64_t* __restrict__ C, uint64_t lc, uint32_t k,
                                                     uint32_t W, int U, uint64_t* __restrict__ E) {
  const uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= lc) return;
  int top = (int)k - 1;
  while (top > 0 && C[(uint64_t)top * lc + m] == 0) --top;
  uint64_t v[kEvalWords];
  static_for<kEvalWords>([&](auto J) { v[decltype(J)::value] = 0; });
  for (int dg = top; dg >= 0; --dg) mul_r_add(v, C[(uint64_t)dg * lc + m], W, U);
  static_for<kEvalWords>([&](auto J) {
    constexpr int j = decltype(J)::value;
    E[m * kEvalWords + j] = v[j];
  });
}

// word w of sum_m C_m 2^(b m) as lo_w + 2^64 hi_w (hi_w small)
__global__ __launch_bounds__(256) void k_bigint_gather(const uint64_t* __restrict__ E, uint64_t lc, uint32_t b,
                                                       uint64_t nw, uint64_t* __restrict__ lo,
                                                       uint64_t* __restrict__ hi) {
  const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  // C_m 2^(b m) spans bits [b m, b m + 64 kEvalWords): it meets word w when
  // b m < 64 w + 64 and b m + 64 kEvalWords > 64 w
  const uint64_t span = 64ull * kEvalWords;
  const uint64_t top = (64 * w + 63) / b;
  const uint64_t m_hi = top < lc - 1 ? top : lc - 1;
  const uint64_t m_lo = (64 * w >= span) ? (64 * w - span) / b : 0;
  unsigned __int128 acc = 0;
  for (uint64_t m = m_lo; m <= m_hi; ++m) {
    const uint64_t* v = E + m * kEvalWords;
    const int64_t s = (int64_t)((uint64_t)b * m) - (int64_t)(64 * w);  // bit 0 of C_m relative to word w
    uint64_t slice;
    if (s >= 64 || s <= -(int64_t)span) {
      slice = 0;
    } else if (s >= 0) {
      slice = v[0] << s;
    } else {
      const uint64_t off = (uint64_t)(-s);
      const uint64_t q = off >> 6, sh = off & 63;
      const uint64_t x0 = v[q], x1 = (q + 1 < kEvalWords) ? v[q + 1] : 0;
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

hipError_t launch_bigint_split(const uint64_t* a, uint64_t na, uint64_t* A, uint64_t la, int k, int b, int ua,
                               uint64_t d, hipStream_t st) {
  if (b < 1 || b > 64 * kChunkWords || ua < 1 || ua > 63 || d >= (1ull << 49)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_bigint_split, dim3((unsigned)((la + 255) / 256)), dim3(256), 0, st, a, na, A, la, (uint32_t)k,
                     (uint32_t)b, (uint32_t)ua, d);
  return hipGetLastError();
}

hipError_t launch_bigint_combine(const uint64_t* C, uint64_t lc, int k, int b, int W, int U, uint64_t nw, uint64_t* E,
                                 uint64_t* lo, uint64_t* hi, hipStream_t st) {
  if (b < 1 || lc == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_bigint_eval, dim3((unsigned)((lc + 255) / 256)), dim3(256), 0, st, C, lc, (uint32_t)k,
                     (uint32_t)W, U, E);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bigint_gather, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st, E, lc, (uint32_t)b, nw, lo,
                     hi);
  return hipGetLastError();
}

uint64_t bigint_eval_words() { return kEvalWords; }
int bigint_max_chunk_bits() { return 64 * kChunkWords; }

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

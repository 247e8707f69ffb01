// HIP kernels for the Generalized Fermat prime field FFT (gfx950).
//
// The transform of size N = K^e (K = 2k) runs as e radix-K passes of an
// out-of-place, self-sorting (Stockham) decimation-in-time schedule.  Pass s
// (stride Ns = K^s) takes, for every j < N/K, the K elements
// x[j + t N/K] (t < K), multiplies element t by the twiddle w_L^(a t)
// (L = Ns K, a = j mod Ns), runs the base case DFT_K at w^(N/K) = r on them
// and writes output t to (j - a) K + a + t Ns.  This is the Cooley-Tukey
// factorisation of section 1.1 (eq. CTCT) unrolled e times, with the stride
// permutations of section 4.1 folded into the load/store indexing.  The
// twiddle w_L^(a t) = r^rho w^(c N/L) with rho = floor(a t / Ns) and
// c = a t mod Ns (section 4.1: w^(i N/K + j) = r^i w^j): only w^j for
// j < N/K is tabulated and r^rho is a digit rotation.
#pragma once

#include "gfp_copy.hpp"
#include "gfp_device.hpp"
#include "gfp_internal.hpp"

namespace gfpk {

// ---------------------------------------------------------------------------
// XCD-aware workgroup order
// ---------------------------------------------------------------------------
// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.
// Mapping dispatch index b to logical index (b mod 8) (G / 8) + b / 8 gives
// every XCD one contiguous range of logical workgroups, run in order, so
// neighbouring workgroups meet in the same L2.  That pays when the input or
// the output is digit-major (a workgroup touches half of each 128-byte line,
// its neighbour the other half) and costs 1-3% otherwise (measured), so it is
// used only then.  A pure permutation of the work; identity when G is not a multiple
// of 8.
// A kernel body runs on a virtual block: a launch's blockIdx.x of gridDim.x,
// or one tile of a persistent launch (k_batch_persistent).
struct VB {
  uint64_t idx, cnt;
};
__device__ __forceinline__ VB launch_vb() { return VB{blockIdx.x, gridDim.x}; }

__device__ __forceinline__ uint64_t xcd_block(bool on, VB vb) {
  const uint64_t b = vb.idx, g = vb.cnt;
  if (!on || (g & 7)) return b;
  return (b & 7) * (g >> 3) + (b >> 3);
}
__device__ __forceinline__ uint64_t xcd_block(bool on) { return xcd_block(on, launch_vb()); }

// ---------------------------------------------------------------------------
// one radix-K Stockham pass
// ---------------------------------------------------------------------------
// MODE_PLAIN: twiddles from the table (forward or inverse table).
// MODE_SCALE: every slot multiplied by one constant (inverse pass 0: 1/N).
// MODE_PRODUCT: the slots are the pointwise products of two transforms
// (section 1: the product of polynomials is the inverse transform of the
// product of their transforms), each then multiplied by the constant, so
// the pointwise step of a polynomial product costs no launch of its own.
enum { MODE_PLAIN = 0, MODE_SCALE = 1, MODE_PRODUCT = 2 };

// MODE_SCALE / MODE_PRODUCT slot value.  x: this lane's digit of the first
// factor; y: the second factor's element, k contiguous digits (every lane
// of the element reads all of them, 16 bytes at a time); c: the constant
// (UC: its limbs read with scalar loads into SGPRs, 3k of them).
template <int KD, int W, int U, int MODE, bool UC = false>
__device__ __forceinline__ L96 first_slot(uint64_t x, const uint64_t* __restrict__ y, const uint32_t* __restrict__ c,
                                          int l, int m) {
  if constexpr (MODE == MODE_PRODUCT && KD == 64) {
    slot_fence();
    x = seminorm<KD, W, U>(mul_data_ptr<KD, W, U>(x, y, 1, l, m), m);
  } else if constexpr (MODE == MODE_PRODUCT) {
    slot_fence();
    uint64_t yd[KD];
    const ulonglong2* y2 = reinterpret_cast<const ulonglong2*>(y);
    static_for<KD / 2>([&](auto T) {
      constexpr int i = decltype(T)::value;
      const ulonglong2 v = y2[i];
      yd[2 * i] = v.x;
      yd[2 * i + 1] = v.y;
    });
    x = seminorm<KD, W, U>(mul_data<KD, W, U>(x, yd, m), m);
  }
  if constexpr (UC) {
    return mul_twiddle_uniform<KD, W, U>(x, c, 0, l, m);
  } else {
    return mul_twiddle<KD, W, U>(x, c, 0, l, m);
  }
}

// UNIF: the K^(e-1-s) groups sharing one twiddle base a are spread over
// whole wavefronts (group g of a wavefront is j = a + (qb G + g) Ns), so the
// twiddles and rotations of a wavefront are uniform: the table entry is read
// with scalar loads into SGPRs and feeds v_mad_u64_u32 as its SGPR operand.
// Used when every a has at least G groups (all passes but the last).
// T2: the twiddles come from the table of w^(K i) without rotations (every
// pass but the last); otherwise from the table of w^j with r^rho rotations.
// k = 16 passes take the shorter product tail (LN).  Per-group passes: at
// most 2 wavefronts per SIMD expected, so the scheduler keeps their
// instruction-level parallelism (with fewer registers it aims at 3 and runs
// slower).  Uniform-twiddle passes: at most 3 (145 VGPRs); with the longer
// tail at 4 wavefronts (128 VGPRs) the N = 2^20 forward transform took
// 538.7 us against 536.4, a 2^15 product 180.3 against 176.4 us.
template <int KD, int W, int U, bool INV, int MODE, bool LAST, bool UNIF, bool T2, bool BND = false>
__device__ __forceinline__ void pass_body(
    const uint64_t* __restrict__ in, const uint64_t* __restrict__ in2, uint64_t se_in, uint64_t sd_in,
    uint64_t* __restrict__ out, uint64_t se_out, uint64_t sd_out, const uint32_t* __restrict__ tw,
    const uint32_t* __restrict__ tw2, const uint64_t* __restrict__ twr1, const uint64_t* __restrict__ twr2, int log2n,
    int log2ns, uint64_t ngroups, uint64_t nvec, uint64_t vin, uint64_t vout, int staged, VB vb,
    uint32_t* __restrict__ stg, uint64_t in_len = ~0ull) {
  typedef Geo<KD> Gm;
  constexpr bool LN = Gm::LEAN || KD == 16;
  constexpr int KB = Gm::KB;
  constexpr int LOGKB = ilog2(KB);
  const int l = Gm::lane();
  const int m = Gm::digit(l);
  // A launch covers nvec transforms of the same size: vector v reads
  // in + v vin and writes out + v vout.
  const uint64_t wave = xcd_block(se_in == 1 || se_out == 1, vb) * (blockDim.x / 64) + (threadIdx.x >> 6);
  const uint64_t nk = ngroups;  // N / K
  const int log2nk = log2n - LOGKB;
  const uint64_t ns = 1ull << log2ns;
  uint64_t j, a, vec;
  if constexpr (UNIF) {
    const int log2wpv = log2nk - ilog2(Gm::G);       // wavefronts per vector
    const int log2wpa = log2wpv - log2ns;            // wavefronts per twiddle base
    vec = wave >> log2wpv;
    const uint64_t w = wave & ((1ull << log2wpv) - 1);
    a = (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(w >> log2wpa));
    const uint64_t qb = w & ((1ull << log2wpa) - 1);
    j = a + ((qb * Gm::G + Gm::group(l)) << log2ns);
  } else {
    const uint64_t J = wave * Gm::G + Gm::group(l);  // group index over all vectors
    vec = J >> log2nk;
    j = J & (nk - 1);
    a = j & (ns - 1);
  }
  // inactive groups (past the last vector) compute on element 0 of vector 0
  // and store nothing; with UNIF the grid covers the groups exactly
  const bool active = UNIF || vec < nvec;
  const uint64_t jj = active ? j : 0;
  if (!active) {
    a = 0;
    vec = 0;
  }
  in += vec * vin;
  if constexpr (MODE == MODE_PRODUCT) in2 += vec * vin;
  out += vec * vout;

  // all slots loaded up front, except for the pointwise product, whose
  // second operand loads already keep enough reads in flight
  // BND: elements at or past in_len are zero and not read (a product's
  // zero padding, first launch of its forward transforms; a variant of its
  // own, so that the transforms' kernels carry no bound check)
  uint64_t x[KB];
  if constexpr (MODE != MODE_PRODUCT) {
    static_for<KB>([&](auto T) {
      constexpr int t = decltype(T)::value;
      const uint64_t i = jj + (uint64_t)t * nk;
      x[t] = (!BND || i < in_len) ? in[(uint64_t)m * sd_in + i * se_in] : 0ull;
    });
  }

  // Twiddle of slot t: w_L^(a t) = r^rho w^(c N/L) with rho = (a t) / Ns,
  // c = (a t) mod Ns.  r^rho is a digit rotation: lane m takes digit
  // (m - rho) mod k of the element from the lane holding it.
  L96 v[KB];
  if constexpr (MODE != MODE_PLAIN) {
    static_for<KB>([&](auto T) {
      constexpr int t = decltype(T)::value;
      if constexpr (MODE == MODE_PRODUCT) {
        slot_fence();
        x[t] = in[(uint64_t)m * sd_in + (jj + (uint64_t)t * nk) * se_in];
      }
      v[t] = first_slot<KD, W, U, MODE, (KD <= 16)>(x[t], in2 + (jj + (uint64_t)t * nk) * se_in, tw, l, m);
    });
  } else {
    v[0] = l96(x[0]);
    if (log2ns == 0 || __all(a == 0)) {
      static_for<KB - 1>([&](auto T) {
        constexpr int t = decltype(T)::value + 1;
        v[t] = l96(x[t]);
      });
    } else if constexpr (T2 && UNIF) {
      // every exponent a t N / (K Ns) is a multiple of K: w^(a t N / (K Ns))
      // is entry (a t) N / (K^2 Ns) of the table of w^(K i), no rotation
      const int sh2 = log2n - 2 * LOGKB - log2ns;
      static_for<KB - 1>([&](auto T) {
        constexpr int t = decltype(T)::value + 1;
        v[t] = mul_entry_uniform<KD, W, U, LN>(x[t], tw2 + ((a * (uint64_t)t) << sh2) * TwLayout<KD>::WORDS, m);
      });
    } else if constexpr (UNIF) {
      const int shift = log2n - log2ns - LOGKB;  // table stride N / (Ns K)
      static_for<KB - 1>([&](auto T) {
        constexpr int t = decltype(T)::value + 1;
        const uint64_t e = a * (uint64_t)t;
        const int rho = (int)(e >> log2ns);
        const uint64_t c = e & (ns - 1);
        const int rot = INV ? ((2 * KD - rho) & (2 * KD - 1)) : rho;
        v[t] = mul_twiddle_uniform<KD, W, U, LN>(x[t], tw + (c << shift) * TwLayout<KD>::WORDS, rot, l, m);
      });
    } else if (!staged) {
      // per-group twiddles, each lane reading the whole entry from the limb
      // tables (small transforms: shorter latency per slot than staging)
      if constexpr (T2) {
        const int sh2 = log2n - 2 * LOGKB - log2ns;
        static_for<KB - 1>([&](auto T) {
          constexpr int t = decltype(T)::value + 1;
          v[t] = mul_entry<KD, W, U, LN>(x[t], tw2 + ((a * (uint64_t)t) << sh2) * TwLayout<KD>::WORDS, m);
        });
      } else {
        const int shift = log2n - log2ns - LOGKB;
        static_for<KB - 1>([&](auto T) {
          constexpr int t = decltype(T)::value + 1;
          const uint64_t e = a * (uint64_t)t;
          const int rho = (int)(e >> log2ns);
          const uint64_t c = e & (ns - 1);
          const int rot = INV ? ((2 * KD - rho) & (2 * KD - 1)) : rho;
          v[t] = mul_twiddle<KD, W, U, LN>(x[t], tw + (c << shift) * TwLayout<KD>::WORDS, rot, l, m);
        });
      }
    } else {
      // per-group twiddles: staged through LDS from the raw-digit tables, the
      // next slot's digit fetched before this slot's product
      uint32_t* E = stg + (int)(threadIdx.x >> 6) * StageGeo<KD>::PER_WAVE + Gm::group(l) * StageGeo<KD>::WORDS;
      stage_init<KD>(E, m);
      if constexpr (T2) {
        const int sh2 = log2n - 2 * LOGKB - log2ns;
        uint64_t yn = twr2[(a << sh2) * KD + m];
        static_for<KB - 1>([&](auto T) {
          constexpr int t = decltype(T)::value + 1;
          const uint64_t y = yn;
          if constexpr (t + 1 < KB) yn = twr2[((a * (uint64_t)(t + 1)) << sh2) * KD + m];
          stage_entry<KD>(y, E, m);
          v[t] = mul_entry<KD, W, U, LN>(x[t], E, m);
        });
      } else {
        const int shift = log2n - log2ns - LOGKB;  // table stride N / (Ns K)
        uint64_t yn = twr1[((a & (ns - 1)) << shift) * KD + m];
        static_for<KB - 1>([&](auto T) {
          constexpr int t = decltype(T)::value + 1;
          const uint64_t e = a * (uint64_t)t;
          const int rho = (int)(e >> log2ns);
          const int rot = INV ? ((2 * KD - rho) & (2 * KD - 1)) : rho;
          const uint64_t y = yn;
          if constexpr (t + 1 < KB) yn = twr1[(((a * (uint64_t)(t + 1)) & (ns - 1)) << shift) * KD + m];
          stage_entry<KD>(y, E, m);
          v[t] = mul_twiddle<KD, W, U, LN>(x[t], E, rot, l, m);
        });
      }
    }
  }

  dft_base<KD, INV, LN, (LN && KD != 16 && !LAST) || (KD == 16 && UNIF)>(v, m);

  const uint64_t obase = (jj - a) * KB + a;
  static_for<KB>([&](auto T) {
    constexpr int t = decltype(T)::value;
    uint64_t d;
    if constexpr (LAST) {
      d = canonicalize<KD, W, U>(v[t], l, m);
    } else {
      d = seminorm<KD, W, U>(v[t], m);
    }
    if (active) out[(uint64_t)m * sd_out + (obase + (uint64_t)t * ns) * se_out] = d;
  });
}

// stg: 4 wavefronts' LDS staging areas (StageGeo<KD>::PER_WAVE words each).
template <int KD, int W, int U, bool INV, int MODE, bool LAST, bool UNIF, bool T2, bool BND = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, KD == 16 ? (UNIF ? 3 : 2) : 8))) void k_pass(
    const uint64_t* __restrict__ in, const uint64_t* __restrict__ in2, uint64_t se_in, uint64_t sd_in,
    uint64_t* __restrict__ out, uint64_t se_out, uint64_t sd_out, const uint32_t* __restrict__ tw,
    const uint32_t* __restrict__ tw2, const uint64_t* __restrict__ twr1, const uint64_t* __restrict__ twr2, int log2n,
    int log2ns, uint64_t ngroups, uint64_t nvec, uint64_t vin, uint64_t vout, int staged, uint64_t in_len) {
  __shared__ uint32_t stg[4 * StageGeo<KD>::PER_WAVE];
  pass_body<KD, W, U, INV, MODE, LAST, UNIF, T2, BND>(in, in2, se_in, sd_in, out, se_out, sd_out, tw, tw2, twr1, twr2,
                                                      log2n, log2ns, ngroups, nvec, vin, vout, staged, launch_vb(), stg,
                                                      in_len);
}

// ---------------------------------------------------------------------------
// one radix-K pass for k = 32 (K = 64): DFT_64 as DFT_8 x DFT_8 through LDS
// ---------------------------------------------------------------------------
// 64 lazy slots per lane do not fit in registers, so the base case is split
// once more by the same factorisation (section 4.1), now inside DFT_64 where
// every twiddle is a power of w_64 = r: with t = t1 + 8 t2 and u = u2 + 8 u1,
//   X[u2 + 8 u1] = sum_t1 r^(8 t1 u1) r^(t1 u2) sum_t2 x[t1 + 8 t2] r^(8 t2 u2).
// A workgroup of 4 wavefronts takes two groups j (one per half wavefront).
// Round A: wavefront w, for t1 = w and w + 4, loads slots t1 + 8 t2, applies
// the pass twiddle (as k_pass), runs DFT_8 over t2 (root r^8), multiplies
// output u2 by r^(t1 u2) and stores it, semi-normalised, to LDS.  Round B:
// for u2 = w and w + 4, DFT_8 over t1 and output u = u2 + 8 u1 goes to
// (j - a) K + a + u Ns.
// NTTM: the pass twiddles are multiplied with the FFT-based product of
// section 3.3 (mul_twiddle_ntt), their transforms read from spec (the table
// of w^j) and spec2 (of w^(K i)), instead of the schoolbook column product.
template <int KD, int W, int U, bool INV, int MODE, bool LAST, bool T2, bool NTTM>
__global__ __launch_bounds__(256) void k_pass_k32(const uint64_t* __restrict__ in, const uint64_t* __restrict__ in2,
                                                  uint64_t se_in, uint64_t sd_in, uint64_t* __restrict__ out,
                                                  uint64_t se_out, uint64_t sd_out, const uint32_t* __restrict__ tw,
                                                  const uint32_t* __restrict__ tw2, const uint64_t* __restrict__ spec,
                                                  const uint64_t* __restrict__ spec2, const uint64_t* __restrict__ ntb,
                                                  int log2n, int log2ns, uint64_t ngroups, uint64_t nvec, uint64_t vin,
                                                  uint64_t vout) {
  static_assert(KD == 32, "the split base case is built for k = 32");
  typedef Geo<KD> Gm;
  constexpr int KB = Gm::KB;
  constexpr int LOGKB = ilog2(KB);
  __shared__ uint64_t lds[KB * 64];  // [u2][t1][lane], 32 KiB
  const int l = Gm::lane();
  const int m = Gm::digit(l);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int log2nk = log2n - LOGKB;
  const uint64_t nk = ngroups;
  const uint64_t J = (uint64_t)blockIdx.x * 2 + (uint64_t)Gm::group(l);  // group over all vectors
  uint64_t vec = J >> log2nk;
  uint64_t j = J & (nk - 1);
  const bool active = vec < nvec;
  if (!active) {
    vec = 0;
    j = 0;
  }
  const uint64_t ns = 1ull << log2ns;
  const uint64_t a = j & (ns - 1);
  in += vec * vin;
  if constexpr (MODE == MODE_PRODUCT) in2 += vec * vin;
  out += vec * vout;

  // ---- round A
  static_for<2>([&](auto H) {
    const int t1 = w + 4 * decltype(H)::value;
    L96 v[8];
    static_for<8>([&](auto T) {
      constexpr int t2 = decltype(T)::value;
      const uint64_t t = (uint64_t)(t1 + 8 * t2);
      const uint64_t e = j + t * nk;
      const uint64_t x = in[(uint64_t)m * sd_in + e * se_in];
      slot_fence();
      if constexpr (MODE != MODE_PLAIN) {
        v[t2] = first_slot<KD, W, U, MODE>(x, in2 + e * se_in, tw, l, m);
      } else if constexpr (T2) {
        // w^(a t N / (K Ns)) = entry (a t) N / (K^2 Ns) of the w^(K i) table
        const int sh2 = log2n - 2 * LOGKB - log2ns;
        if constexpr (NTTM) {
          v[t2] = (log2ns == 0) ? l96(x) : mul_twiddle_ntt<KD, W, U>(x, spec2 + ((a * t) << sh2) * (3 * KD), ntb, 0, l, m);
        } else {
          v[t2] = (log2ns == 0) ? l96(x) : mul_entry<KD, W, U>(x, tw2 + ((a * t) << sh2) * TwLayout<KD>::WORDS, m);
        }
      } else {
        if (log2ns == 0) {
          v[t2] = l96(x);
        } else {
          const int shift = log2n - log2ns - LOGKB;
          const uint64_t at = a * t;
          const int rho = (int)(at >> log2ns);
          const uint64_t c = at & (ns - 1);
          const int rot = INV ? ((2 * KD - rho) & (2 * KD - 1)) : rho;
          if constexpr (NTTM) {
            v[t2] = mul_twiddle_ntt<KD, W, U>(x, spec + (c << shift) * (3 * KD), ntb, rot, l, m);
          } else {
            v[t2] = mul_twiddle<KD, W, U>(x, tw + (c << shift) * TwLayout<KD>::WORDS, rot, l, m);
          }
        }
      }
    });
    dft_pow2<KD, INV, 3>(v, m);
    static_for<8>([&](auto V) {
      constexpr int u2 = decltype(V)::value;
      const int e = (t1 * u2) & (2 * KD - 1);
      const L96 y = l96_mul_rpow<KD>(v[u2], INV ? ((2 * KD - e) & (2 * KD - 1)) : e, l, m);
      lds[(u2 * 8 + t1) * 64 + l] = seminorm<KD, W, U>(y, m);
    });
  });
  __syncthreads();

  // ---- round B
  const uint64_t obase = (j - a) * KB + a;
  static_for<2>([&](auto H) {
    const int u2 = w + 4 * decltype(H)::value;
    L96 v[8];
    static_for<8>([&](auto T) {
      constexpr int t1 = decltype(T)::value;
      v[t1] = l96(lds[(u2 * 8 + t1) * 64 + l]);
    });
    dft_pow2<KD, INV, 3>(v, m);
    static_for<8>([&](auto V) {
      constexpr int u1 = decltype(V)::value;
      const uint64_t u = (uint64_t)(u2 + 8 * u1);
      uint64_t d;
      if constexpr (LAST) {
        d = canonicalize<KD, W, U>(v[u1], l, m);
      } else {
        d = seminorm<KD, W, U>(v[u1], m);
      }
      if (active) out[(uint64_t)m * sd_out + (obase + u * ns) * se_out] = d;
    });
  });
}

// ---------------------------------------------------------------------------
// one radix-K pass for k = 64 (K = 128): DFT_128 as DFT_16 x DFT_8 through LDS
// ---------------------------------------------------------------------------
// The same split as k_pass_k32 with t = t1 + 16 t2 and u = u2 + 8 u1:
//   X[u2 + 8 u1] = sum_t1 r^(8 t1 u1) r^(t1 u2) sum_t2 x[t1 + 16 t2] r^(16 t2 u2).
// An element is a whole wavefront, so a 256-thread workgroup takes one group
// j.  Round A: wavefront w, for t1 = w, w + 4, w + 8, w + 12, loads slots
// t1 + 16 t2 (t2 < 8), applies the pass twiddles, DFT_8 over t2 (root r^16),
// multiplies output u2 by r^(t1 u2) and stores it to LDS (64 KiB).  Round B:
// for u2 = w and w + 4, DFT_16 over t1 (root r^8); output u2 + 8 u1 goes to
// (j - a) K + a + u Ns.
template <int KD, int W, int U, bool INV, int MODE, bool LAST, bool T2, bool NTTM>
__global__ __launch_bounds__(256) void k_pass_k64(const uint64_t* __restrict__ in, const uint64_t* __restrict__ in2,
                                                  uint64_t se_in, uint64_t sd_in, uint64_t* __restrict__ out,
                                                  uint64_t se_out, uint64_t sd_out, const uint32_t* __restrict__ tw,
                                                  const uint32_t* __restrict__ tw2, const uint64_t* __restrict__ spec,
                                                  const uint64_t* __restrict__ spec2, const uint64_t* __restrict__ ntb,
                                                  int log2n, int log2ns, uint64_t ngroups, uint64_t nvec, uint64_t vin,
                                                  uint64_t vout) {
  static_assert(KD == 64, "the split base case is built for k = 64");
  typedef Geo<KD> Gm;
  constexpr int KB = Gm::KB;
  constexpr int LOGKB = ilog2(KB);
  __shared__ uint64_t lds[KB * 64];  // [u2][t1][lane], 64 KiB
  const int l = Gm::lane();
  const int m = Gm::digit(l);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int log2nk = log2n - LOGKB;
  const uint64_t nk = ngroups;
  const uint64_t J = (uint64_t)blockIdx.x;  // group over all vectors (the grid covers them exactly)
  const uint64_t vec = J >> log2nk;
  const uint64_t j = J & (nk - 1);
  const uint64_t ns = 1ull << log2ns;
  const uint64_t a = j & (ns - 1);
  in += vec * vin;
  if constexpr (MODE == MODE_PRODUCT) in2 += vec * vin;
  out += vec * vout;

  // ---- round A (a run-time loop: four copies of 8 products are too much code)
#pragma unroll 1
  for (int h = 0; h < 4; ++h) {
    const int t1 = w + 4 * h;
    L96 v[8];
    static_for<8>([&](auto T) {
      constexpr int t2 = decltype(T)::value;
      const uint64_t t = (uint64_t)(t1 + 16 * t2);
      const uint64_t e = j + t * nk;
      const uint64_t x = in[(uint64_t)m * sd_in + e * se_in];
      slot_fence();
      if constexpr (MODE != MODE_PLAIN) {
        v[t2] = first_slot<KD, W, U, MODE>(x, in2 + e * se_in, tw, l, m);
      } else if constexpr (T2) {
        const int sh2 = log2n - 2 * LOGKB - log2ns;
        if constexpr (NTTM) {
          v[t2] = (log2ns == 0) ? l96(x) : mul_twiddle_ntt<KD, W, U>(x, spec2 + ((a * t) << sh2) * (3 * KD), ntb, 0, l, m);
        } else {
          v[t2] = (log2ns == 0) ? l96(x) : mul_entry<KD, W, U>(x, tw2 + ((a * t) << sh2) * TwLayout<KD>::WORDS, m);
        }
      } else {
        if (log2ns == 0) {
          v[t2] = l96(x);
        } else {
          const int shift = log2n - log2ns - LOGKB;
          const uint64_t at = a * t;
          const int rho = (int)(at >> log2ns);
          const uint64_t c = at & (ns - 1);
          const int rot = INV ? ((2 * KD - rho) & (2 * KD - 1)) : rho;
          if constexpr (NTTM) {
            v[t2] = mul_twiddle_ntt<KD, W, U>(x, spec + (c << shift) * (3 * KD), ntb, rot, l, m);
          } else {
            v[t2] = mul_twiddle<KD, W, U>(x, tw + (c << shift) * TwLayout<KD>::WORDS, rot, l, m);
          }
        }
      }
    });
    dft_pow2<KD, INV, 3>(v, m);
    static_for<8>([&](auto V) {
      constexpr int u2 = decltype(V)::value;
      const int e = (t1 * u2) & (2 * KD - 1);
      const L96 y = l96_mul_rpow<KD>(v[u2], INV ? ((2 * KD - e) & (2 * KD - 1)) : e, l, m);
      lds[(u2 * 16 + t1) * 64 + l] = seminorm<KD, W, U>(y, m);
    });
  }
  __syncthreads();

  // ---- round B
  const uint64_t obase = (j - a) * KB + a;
  static_for<2>([&](auto H) {
    const int u2 = w + 4 * decltype(H)::value;
    L96 v[16];
    static_for<16>([&](auto T) {
      constexpr int t1 = decltype(T)::value;
      v[t1] = l96(lds[(u2 * 16 + t1) * 64 + l]);
    });
    dft_pow2<KD, INV, 4>(v, m);
    static_for<16>([&](auto V) {
      constexpr int u1 = decltype(V)::value;
      const uint64_t u = (uint64_t)(u2 + 8 * u1);
      uint64_t d;
      if constexpr (LAST) {
        d = canonicalize<KD, W, U>(v[u1], l, m);
      } else {
        d = seminorm<KD, W, U>(v[u1], m);
      }
      out[(uint64_t)m * sd_out + (obase + u * ns) * se_out] = d;
    });
  });
}

// ---------------------------------------------------------------------------
// first pass of a transform of size N = R K^e, 1 < R = 2^LR < K
// ---------------------------------------------------------------------------
// Radix R with Ns = 1 (no twiddles): for every j < N/R the R elements
// x[j + t N/R] go through DFT_R at w^(N/R) = r^(K/R) and land at j R + t.
// The radix-K passes that follow run with Ns = R K^s (section 4.1: any
// factorisation N = N1 N2 with the base case at powers of r).  MODE_SCALE
// multiplies every element by the 1/N entry first (inverse transform).
template <int KD, int W, int U, bool INV, int MODE, int LR, bool BND = false>
__device__ __forceinline__ void pass_r_body(const uint64_t* __restrict__ in, const uint64_t* __restrict__ in2,
                                            uint64_t se_in, uint64_t sd_in, uint64_t* __restrict__ out,
                                            uint64_t se_out, uint64_t sd_out, const uint32_t* __restrict__ tw,
                                            int log2n, uint64_t nvec, uint64_t vin, uint64_t vout, VB vb,
                                            uint64_t in_len = ~0ull) {
  typedef Geo<KD> Gm;
  constexpr int R = 1 << LR;
  const int l = Gm::lane();
  const int m = Gm::digit(l);
  const uint64_t wave = vb.idx * (blockDim.x / 64) + (threadIdx.x >> 6);
  const uint64_t J = wave * Gm::G + Gm::group(l);
  const int log2nr = log2n - LR;  // groups per vector
  uint64_t vec = J >> log2nr;
  const bool active = vec < nvec;
  const uint64_t j = active ? (J & ((1ull << log2nr) - 1)) : 0;
  if (!active) vec = 0;
  in += vec * vin;
  if constexpr (MODE == MODE_PRODUCT) in2 += vec * vin;
  out += vec * vout;
  L96 v[R];
  static_for<R>([&](auto T) {
    constexpr int t = decltype(T)::value;
    const uint64_t i = j + ((uint64_t)t << log2nr);
    const uint64_t x = (!BND || i < in_len) ? in[(uint64_t)m * sd_in + i * se_in] : 0ull;
    if constexpr (MODE != MODE_PLAIN) {
      v[t] = first_slot<KD, W, U, MODE, (KD <= 16)>(x, in2 + (j + ((uint64_t)t << log2nr)) * se_in, tw, l, m);
    } else {
      v[t] = l96(x);
    }
  });
  dft_pow2<KD, INV, LR>(v, m);
  static_for<R>([&](auto T) {
    constexpr int t = decltype(T)::value;
    const uint64_t d = seminorm<KD, W, U>(v[t], m);
    if (active) out[(uint64_t)m * sd_out + (j * R + t) * se_out] = d;
  });
}

template <int KD, int W, int U, bool INV, int MODE, int LR, bool BND = false>
__global__ __launch_bounds__(256) void k_pass_r(const uint64_t* __restrict__ in, const uint64_t* __restrict__ in2,
                                                uint64_t se_in, uint64_t sd_in, uint64_t* __restrict__ out, uint64_t se_out, uint64_t sd_out,
                                                const uint32_t* __restrict__ tw, int log2n, uint64_t nvec,
                                                uint64_t vin, uint64_t vout, uint64_t in_len) {
  pass_r_body<KD, W, U, INV, MODE, LR, BND>(in, in2, se_in, sd_in, out, se_out, sd_out, tw, log2n, nvec, vin, vout,
                                            launch_vb(), in_len);
}

// ---------------------------------------------------------------------------
// two radix-K passes s, s+1 in one launch (a stage group of two)
// ---------------------------------------------------------------------------
// Block q of a vector (q < N/K^2): a = q mod Ns, c = q / Ns.  Its K^2
// elements are x[a + Ns c + (N/K^2) t2 + (N/K) t1], t1, t2 < K, and no other
// block reads or writes them in either pass.  Pass s: group t2 (slots t1,
// twiddles w_{K Ns}^(a t1), uniform over the block); DFT output t1' of group
// t2 is stored in LDS at (t1', t2).  Pass s+1 reads the transposed grid:
// group t1' (slots t2, twiddles w_{K^2 Ns}^((a + Ns t1') t2)) and writes
// output t2' to a + Ns t1' + K Ns t2' + K^2 Ns c -- the same element
// operations, in the same order, as the two passes run one after the other
// (section 4.1: the stride permutation L between the two tensor factors is
// the LDS transpose).  k = 8: two blocks per 256-thread workgroup; k = 16:
// one block (1024 elements, 130 KiB of LDS) per 512-thread workgroup, so one
// workgroup per CU.
template <int KD>
struct Span2Geo {
  static constexpr int KB = Geo<KD>::KB;
  static constexpr int WPB = KB / Geo<KD>::G;       // wavefronts per block
  static constexpr int BPW = WPB >= 4 ? 1 : 4 / WPB;  // blocks per workgroup
  static constexpr int WAVES = WPB * BPW;           // wavefronts per workgroup
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int ROW = KB * KD + 8;  // u64 words per LDS row, padded by 64 bytes
};

// T2B: the second pass is not the last one and takes its twiddles from the
// table of w^(K i); the first pass never is the last and always does.
// lds: SG::BPW * KB * SG::ROW words (the blocks' transposes); stg: the
// wavefronts' staging areas (SG::WAVES * StageGeo<KD>::PER_WAVE words).
template <int KD, int W, int U, bool INV, int MODE, bool LAST, bool T2B, bool BND = false>
__device__ __forceinline__ void pass2_body(const uint64_t* __restrict__ in, const uint64_t* __restrict__ in2,
                                           uint64_t se_in, uint64_t sd_in, uint64_t* __restrict__ out, uint64_t se_out,
                                           uint64_t sd_out, const uint32_t* __restrict__ tw0,
                                           const uint32_t* __restrict__ tw1, const uint32_t* __restrict__ tw2,
                                           const uint64_t* __restrict__ twr1, const uint64_t* __restrict__ twr2,
                                           int log2n, int log2ns, uint64_t nvec, uint64_t vin, uint64_t vout,
                                           int staged, VB vb, uint64_t* __restrict__ lds, uint32_t* __restrict__ stg,
                                           uint64_t in_len = ~0ull) {
  static_assert(KD == 8 || KD == 16, "the fused pass pair is built for k = 8 and 16");
  typedef Geo<KD> Gm;
  typedef Span2Geo<KD> SG;
  constexpr int KB = Gm::KB;
  constexpr int LOGKB = ilog2(KB);
  const int l = Gm::lane();
  const int m = Gm::digit(l);
  const int g = Gm::group(l);
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int bw = wv / SG::WPB, h = wv % SG::WPB;
  const int log2nb = log2n - 2 * LOGKB;  // blocks per vector
  uint64_t gq = xcd_block(se_in == 1 || se_out == 1, vb) * SG::BPW + bw;
  uint64_t vec = gq >> log2nb;
  const bool active = vec < nvec;
  if (!active) {
    gq = 0;
    vec = 0;
  }
  const uint64_t q = gq & ((1ull << log2nb) - 1);
  in += vec * vin;
  if constexpr (MODE == MODE_PRODUCT) in2 += vec * vin;
  out += vec * vout;
  const uint64_t ns = 1ull << log2ns;
  const uint64_t a = q & (ns - 1);  // uniform over the wavefront
  const uint64_t c = q >> log2ns;
  const uint64_t n1 = 1ull << (log2n - LOGKB);
  const uint64_t n2 = 1ull << log2nb;

  // ---- pass s: group t2, slots t1
  const uint64_t t2 = (uint64_t)(h * Gm::G + g);
  const uint64_t base = a + (c << log2ns) + t2 * n2;
  uint64_t x[KB];
  static_for<KB>([&](auto T) {
    constexpr int t = decltype(T)::value;
    const uint64_t i = base + (uint64_t)t * n1;
    x[t] = (!BND || i < in_len) ? in[(uint64_t)m * sd_in + i * se_in] : 0ull;
  });
  L96 v[KB];
  if constexpr (MODE != MODE_PLAIN) {
    static_for<KB>([&](auto T) {
      constexpr int t = decltype(T)::value;
      v[t] = first_slot<KD, W, U, MODE, true>(x[t], in2 + (base + (uint64_t)t * n1) * se_in, tw0, l, m);
    });
  } else {
    v[0] = l96(x[0]);
    if (a == 0) {
      static_for<KB - 1>([&](auto T) {
        constexpr int t = decltype(T)::value + 1;
        v[t] = l96(x[t]);
      });
    } else {
      // pass s is not the last radix-K pass: table of w^(K i), no rotation
      const int sh2 = log2n - 2 * LOGKB - log2ns;
      static_for<KB - 1>([&](auto T) {
        constexpr int t = decltype(T)::value + 1;
        v[t] = mul_entry_uniform<KD, W, U>(x[t], tw2 + ((a * (uint64_t)t) << sh2) * TwLayout<KD>::WORDS, m);
      });
    }
  }
  dft_base<KD, INV>(v, m);
  uint64_t* L = lds + bw * (KB * SG::ROW);
  static_for<KB>([&](auto T) {
    constexpr int t = decltype(T)::value;
    L[t * SG::ROW + (int)t2 * KD + m] = seminorm<KD, W, U>(v[t], m);
  });
  __syncthreads();

  // ---- pass s+1: group t1 = h G + g, slots t2
  const uint64_t t1 = (uint64_t)(h * Gm::G + g);
  static_for<KB>([&](auto T) {
    constexpr int t = decltype(T)::value;
    x[t] = L[(int)t1 * SG::ROW + t * KD + m];
  });
  const int log2ns1 = log2ns + LOGKB;
  const uint64_t ns1 = ns << LOGKB;
  const uint64_t a1 = a + (t1 << log2ns);
  v[0] = l96(x[0]);
  // per-group twiddles, staged through LDS from the raw-digit tables (or, for
  // small transforms, read whole by each lane from the limb tables)
  uint32_t* E = stg + wv * StageGeo<KD>::PER_WAVE + g * StageGeo<KD>::WORDS;
  if (!staged) {
    if constexpr (T2B) {
      const int sh2 = log2n - 2 * LOGKB - log2ns1;
      static_for<KB - 1>([&](auto T) {
        constexpr int t = decltype(T)::value + 1;
        v[t] = mul_entry<KD, W, U>(x[t], tw2 + ((a1 * (uint64_t)t) << sh2) * TwLayout<KD>::WORDS, m);
      });
    } else {
      const int shift1 = log2n - log2ns1 - LOGKB;
      static_for<KB - 1>([&](auto T) {
        constexpr int t = decltype(T)::value + 1;
        const uint64_t e = a1 * (uint64_t)t;
        const int rho = (int)(e >> log2ns1);
        const uint64_t cc = e & (ns1 - 1);
        const int rot = INV ? ((2 * KD - rho) & (2 * KD - 1)) : rho;
        v[t] = mul_twiddle<KD, W, U>(x[t], tw1 + (cc << shift1) * TwLayout<KD>::WORDS, rot, l, m);
      });
    }
  } else if constexpr (T2B) {
    stage_init<KD>(E, m);
    const int sh2 = log2n - 2 * LOGKB - log2ns1;
    uint64_t yn = twr2[(a1 << sh2) * KD + m];
    static_for<KB - 1>([&](auto T) {
      constexpr int t = decltype(T)::value + 1;
      const uint64_t y = yn;
      if constexpr (t + 1 < KB) yn = twr2[((a1 * (uint64_t)(t + 1)) << sh2) * KD + m];
      stage_entry<KD>(y, E, m);
      v[t] = mul_entry<KD, W, U>(x[t], E, m);
    });
  } else {
    stage_init<KD>(E, m);
    const int shift1 = log2n - log2ns1 - LOGKB;
    uint64_t yn = twr1[((a1 & (ns1 - 1)) << shift1) * KD + m];
    static_for<KB - 1>([&](auto T) {
      constexpr int t = decltype(T)::value + 1;
      const uint64_t e = a1 * (uint64_t)t;
      const int rho = (int)(e >> log2ns1);
      const int rot = INV ? ((2 * KD - rho) & (2 * KD - 1)) : rho;
      const uint64_t y = yn;
      if constexpr (t + 1 < KB) yn = twr1[(((a1 * (uint64_t)(t + 1)) & (ns1 - 1)) << shift1) * KD + m];
      stage_entry<KD>(y, E, m);
      v[t] = mul_twiddle<KD, W, U>(x[t], E, rot, l, m);
    });
  }
  dft_base<KD, INV>(v, m);
  const uint64_t obase = a + (t1 << log2ns) + (c << (log2ns + 2 * LOGKB));
  static_for<KB>([&](auto T) {
    constexpr int t = decltype(T)::value;
    uint64_t d;
    if constexpr (LAST) {
      d = canonicalize<KD, W, U>(v[t], l, m);
    } else {
      d = seminorm<KD, W, U>(v[t], m);
    }
    if (active) out[(uint64_t)m * sd_out + (obase + (uint64_t)t * ns1) * se_out] = d;
  });
}

template <int KD, int W, int U, bool INV, int MODE, bool LAST, bool T2B, bool BND = false>
__global__ __launch_bounds__(Span2Geo<KD>::THREADS) void k_pass2(const uint64_t* __restrict__ in, const uint64_t* __restrict__ in2,
                                               uint64_t se_in, uint64_t sd_in, uint64_t* __restrict__ out, uint64_t se_out, uint64_t sd_out,
                                               const uint32_t* __restrict__ tw0, const uint32_t* __restrict__ tw1,
                                               const uint32_t* __restrict__ tw2, const uint64_t* __restrict__ twr1,
                                               const uint64_t* __restrict__ twr2, int log2n, int log2ns, uint64_t nvec,
                                               uint64_t vin, uint64_t vout, int staged, uint64_t in_len) {
  typedef Span2Geo<KD> SG;
  __shared__ uint64_t lds[SG::BPW * SG::KB * SG::ROW];
  __shared__ uint32_t stg[SG::WAVES * StageGeo<KD>::PER_WAVE];
  pass2_body<KD, W, U, INV, MODE, LAST, T2B, BND>(in, in2, se_in, sd_in, out, se_out, sd_out, tw0, tw1, tw2, twr1,
                                                  twr2, log2n, log2ns, nvec, vin, vout, staged, launch_vb(), lds, stg,
                                                  in_len);
}

// The same pass pair with uniform twiddles in both halves ("wide"): a
// 1024-thread workgroup takes the 8 blocks q = a + Ns (8 cb + i), i < 8,
// which share a.  Pass s: wavefront w handles t2 = w, group g being block g
// (for s = 0 the 8 groups are consecutive elements, so digit-major loads
// coalesce).  Pass s+1: wavefront w handles t1' = w, group g being block g,
// so the twiddle base a + Ns t1' is the same for the whole wavefront.  Needs
// at least 8 blocks per twiddle base: N / (K^2 Ns) >= 8.
template <int KD>
struct Span2UGeo {
  static constexpr int KB = Geo<KD>::KB;
  static constexpr int NBLK = 8;                      // blocks per workgroup
  static constexpr int ROW = KB * KD;                 // u64 words per (block, t1) row
  static constexpr int BLK = KB * ROW + 8;            // words per block, padded by 64 bytes
  static constexpr int THREADS = 64 * NBLK * KB / Geo<KD>::G;
};

template <int KD, int W, int U, bool INV, int MODE, bool LAST, bool T2B, bool BND = false>
__global__ __launch_bounds__(1024) void k_pass2u(const uint64_t* __restrict__ in, const uint64_t* __restrict__ in2,
                                                 uint64_t se_in, uint64_t sd_in, uint64_t* __restrict__ out, uint64_t se_out, uint64_t sd_out,
                                                 const uint32_t* __restrict__ tw0, const uint32_t* __restrict__ tw1,
                                                 const uint32_t* __restrict__ tw2, int log2n, int log2ns, uint64_t nvec,
                                                 uint64_t vin, uint64_t vout, uint64_t in_len) {
  static_assert(KD == 8, "the fused pass pair is built for k = 8");
  typedef Geo<KD> Gm;
  typedef Span2UGeo<KD> SG;
  static_assert(SG::THREADS == 1024, "one 1024-thread workgroup per 8 blocks");
  constexpr int KB = Gm::KB;
  constexpr int LOGKB = ilog2(KB);
  __shared__ uint64_t lds[SG::NBLK * SG::BLK];
  const int l = Gm::lane();
  const int m = Gm::digit(l);
  const int g = Gm::group(l);
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int log2nb = log2n - 2 * LOGKB;      // blocks per vector
  const int log2wpv = log2nb - 3;            // workgroups per vector
  const uint64_t wg = xcd_block(se_in == 1 || se_out == 1);
  const uint64_t vec = wg >> log2wpv;
  const uint64_t r = wg & ((1ull << log2wpv) - 1);
  in += vec * vin;
  if constexpr (MODE == MODE_PRODUCT) in2 += vec * vin;
  out += vec * vout;
  const uint64_t ns = 1ull << log2ns;
  const uint64_t a = r & (ns - 1);         // uniform over the workgroup
  const uint64_t c0 = (r >> log2ns) << 3;  // first of the 8 blocks' c
  const uint64_t n1 = 1ull << (log2n - LOGKB);
  const uint64_t n2 = 1ull << log2nb;

  // ---- pass s: t2 = wv for the whole wavefront, group g = block g, slots t1
  const uint64_t t2 = (uint64_t)wv;
  const uint64_t base = a + ((c0 + (uint64_t)g) << log2ns) + t2 * n2;
  uint64_t x[KB];
  static_for<KB>([&](auto T) {
    constexpr int t = decltype(T)::value;
    const uint64_t i = base + (uint64_t)t * n1;
    x[t] = (!BND || i < in_len) ? in[(uint64_t)m * sd_in + i * se_in] : 0ull;
  });
  L96 v[KB];
  if constexpr (MODE != MODE_PLAIN) {
    static_for<KB>([&](auto T) {
      constexpr int t = decltype(T)::value;
      v[t] = first_slot<KD, W, U, MODE, true>(x[t], in2 + (base + (uint64_t)t * n1) * se_in, tw0, l, m);
    });
  } else {
    v[0] = l96(x[0]);
    if (a == 0) {
      static_for<KB - 1>([&](auto T) {
        constexpr int t = decltype(T)::value + 1;
        v[t] = l96(x[t]);
      });
    } else {
      // pass s is not the last radix-K pass: table of w^(K i), no rotation
      const int sh2 = log2n - 2 * LOGKB - log2ns;
      static_for<KB - 1>([&](auto T) {
        constexpr int t = decltype(T)::value + 1;
        v[t] = mul_entry_uniform<KD, W, U>(x[t], tw2 + ((a * (uint64_t)t) << sh2) * TwLayout<KD>::WORDS, m);
      });
    }
  }
  dft_base<KD, INV>(v, m);
  static_for<KB>([&](auto T) {
    constexpr int t = decltype(T)::value;
    lds[g * SG::BLK + t * SG::ROW + wv * KD + m] = seminorm<KD, W, U>(v[t], m);
  });
  __syncthreads();

  // ---- pass s+1: t1 = wv for the whole wavefront, group g = block g, slots t2
  const uint64_t t1 = (uint64_t)wv;
  static_for<KB>([&](auto T) {
    constexpr int t = decltype(T)::value;
    x[t] = lds[g * SG::BLK + wv * SG::ROW + t * KD + m];
  });
  const int log2ns1 = log2ns + LOGKB;
  const uint64_t ns1 = ns << LOGKB;
  const uint64_t a1 = a + (t1 << log2ns);  // uniform over the wavefront
  v[0] = l96(x[0]);
  if (a1 == 0) {
    static_for<KB - 1>([&](auto T) {
      constexpr int t = decltype(T)::value + 1;
      v[t] = l96(x[t]);
    });
  } else if constexpr (T2B) {
    const int sh2 = log2n - 2 * LOGKB - log2ns1;
    static_for<KB - 1>([&](auto T) {
      constexpr int t = decltype(T)::value + 1;
      v[t] = mul_entry_uniform<KD, W, U>(x[t], tw2 + ((a1 * (uint64_t)t) << sh2) * TwLayout<KD>::WORDS, m);
    });
  } else {
    const int shift1 = log2n - log2ns1 - LOGKB;
    static_for<KB - 1>([&](auto T) {
      constexpr int t = decltype(T)::value + 1;
      const uint64_t e = a1 * (uint64_t)t;
      const int rho = (int)(e >> log2ns1);
      const uint64_t cc = e & (ns1 - 1);
      const int rot = INV ? ((2 * KD - rho) & (2 * KD - 1)) : rho;
      v[t] = mul_twiddle_uniform<KD, W, U>(x[t], tw1 + (cc << shift1) * TwLayout<KD>::WORDS, rot, l, m);
    });
  }
  dft_base<KD, INV>(v, m);
  const uint64_t obase = a + (t1 << log2ns) + ((c0 + (uint64_t)g) << (log2ns + 2 * LOGKB));
  static_for<KB>([&](auto T) {
    constexpr int t = decltype(T)::value;
    uint64_t d;
    if constexpr (LAST) {
      d = canonicalize<KD, W, U>(v[t], l, m);
    } else {
      d = seminorm<KD, W, U>(v[t], m);
    }
    out[(uint64_t)m * sd_out + (obase + (uint64_t)t * ns1) * se_out] = d;
  });
}

// ---------------------------------------------------------------------------
// elementwise operations (one element per k lanes)
// ---------------------------------------------------------------------------
template <int KD, int W, int U, int OP>
__device__ __forceinline__ void elementwise_body(const uint64_t* __restrict__ x, uint64_t xse, uint64_t xsd,
                                                 const uint64_t* __restrict__ y, uint64_t yse, uint64_t ysd,
                                                 uint64_t* __restrict__ z, uint64_t zse, uint64_t zsd, uint64_t n,
                                                 int64_t s, const uint32_t* __restrict__ cst, VB vb) {
  typedef Geo<KD> Gm;
  const int l = Gm::lane();
  const int m = Gm::digit(l);
  const uint64_t e = (vb.idx * (blockDim.x / 64) + (threadIdx.x >> 6)) * Gm::G + Gm::group(l);
  const bool active = e < n;
  const uint64_t ee = active ? e : 0;
  L96 t;
  if constexpr (OP == GFP_OP_ADD || OP == GFP_OP_SUB) {
    const uint64_t xm = x[(uint64_t)m * xsd + ee * xse];
    const uint64_t ym = y[(uint64_t)m * ysd + ee * yse];
    t = (OP == GFP_OP_ADD) ? l96_add(l96(xm), l96(ym)) : l96_sub(l96(xm), l96(ym));
  } else if constexpr (OP == GFP_OP_MUL || OP == GFP_OP_MUL_SCALE) {
    const uint64_t xm = x[(uint64_t)m * xsd + ee * xse];
    t = mul_data_ptr<KD, W, U>(xm, y + ee * yse, ysd, l, m);
    if constexpr (OP == GFP_OP_MUL_SCALE) {
      const uint64_t sn = seminorm<KD, W, U>(t, m);
      t = mul_twiddle_pre<KD, W, U>(sn, cst, rot_lane<KD>(0, m), m);
    }
  } else if constexpr (OP == GFP_OP_MUL_NTT) {
    // the FFT-based product: each lane needs only its own digits
    const uint64_t xm = x[(uint64_t)m * xsd + ee * xse];
    const uint64_t ym = y[(uint64_t)m * ysd + ee * yse];
    t = mul_ntt<KD, W, U>(xm, ym, reinterpret_cast<const uint64_t*>(cst), l, m);
  } else {  // GFP_OP_MUL_CONST: x * c * r^s; GFP_OP_MUL_POW_R: the same with c = 1
    const RotLane<KD> rl = rot_lane<KD>((int)(((s % (2 * KD)) + 2 * KD) % (2 * KD)), m);
    const uint64_t xs = x[(uint64_t)rl.src * xsd + ee * xse];
    t = mul_twiddle_pre<KD, W, U>(xs, cst, rl, m);
  }
  const uint64_t d = canonicalize<KD, W, U>(t, l, m);
  if (active) z[(uint64_t)m * zsd + ee * zse] = d;
}

template <int KD, int W, int U, int OP>
__global__ __launch_bounds__(256) void k_elementwise(const uint64_t* __restrict__ x, uint64_t xse, uint64_t xsd,
                                                     const uint64_t* __restrict__ y, uint64_t yse, uint64_t ysd,
                                                     uint64_t* __restrict__ z, uint64_t zse, uint64_t zsd, uint64_t n,
                                                     int64_t s, const uint32_t* __restrict__ cst) {
  elementwise_body<KD, W, U, OP>(x, xse, xsd, y, yse, ysd, z, zse, zsd, n, s, cst, launch_vb());
}

// ---------------------------------------------------------------------------
// twiddle tables on the device (k <= 16)
// ---------------------------------------------------------------------------
// Entry j < cnt of the table of w^j from two small tables of raw digits:
// lo[i] = w^i (i < 2^log2b) and hi[i] = w^(i 2^log2b): w^j is their product,
// canonical, so it equals the value computed any other way digit for digit.
// Writes the raw digits (raw[j k + m]) and the entry layout read by the
// passes (tab + j WORDS: the 22/22/20-bit limbs of every digit, the suffix
// sums sum_{t >= i} y_t for i = 0..k as three words, zero padding).
template <int KD, int W, int U>
__global__ __launch_bounds__(256) void k_table_build(const uint64_t* __restrict__ lo, const uint64_t* __restrict__ hi,
                                                     int log2b, uint64_t cnt, uint32_t* __restrict__ tab,
                                                     uint64_t* __restrict__ raw) {
  typedef Geo<KD> Gm;
  static_assert(Gm::ROW, "elements inside one DPP row");
  const int l = Gm::lane();
  const int m = Gm::digit(l);
  const uint64_t e = ((uint64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6)) * Gm::G + Gm::group(l);
  const bool active = e < cnt;
  const uint64_t j = active ? e : 0;  // inactive groups compute entry 0 and store nothing
  const uint64_t xm = lo[(j & ((1ull << log2b) - 1)) * KD + m];
  const L96 t = mul_data_ptr<KD, W, U>(xm, hi + (j >> log2b) * KD, 1, l, m);
  const uint64_t d = canonicalize<KD, W, U>(t, l, m);
  uint32_t l0, l1, l2;
  split22(d, l0, l1, l2);
  // inclusive suffix sum sum_{t >= m} y_t (< 2^68) by doubling steps
  uint32_t s0 = (uint32_t)d, s1 = (uint32_t)(d >> 32), s2 = 0u;
  static_for<ilog2(KD)>([&](auto I) {
    constexpr int dd = 1 << decltype(I)::value;
    const uint32_t n0 = dig_up<KD, dd>(s0), n1 = dig_up<KD, dd>(s1), n2 = dig_up<KD, dd>(s2);
    unsigned c;
    s0 = __builtin_addc(s0, n0, 0u, &c);
    s1 = __builtin_addc(s1, n1, c, &c);
    s2 = s2 + n2 + c;
  });
  if (!active) return;
  raw[j * KD + m] = d;
  uint32_t* E = tab + j * TwLayout<KD>::WORDS;
  E[3 * m] = l0;
  E[3 * m + 1] = l1;
  E[3 * m + 2] = l2;
  uint32_t* suf = E + TwLayout<KD>::SUF + 3 * m;
  suf[0] = s0;
  suf[1] = s1;
  suf[2] = s2;
  if (m == KD - 1) {  // suffix(k) = 0 and the padding
    for (int w = TwLayout<KD>::SUF + 3 * KD; w < TwLayout<KD>::WORDS; ++w) E[w] = 0u;
  }
}

template <int KD, int W, int U>
hipError_t launch_table_build_t(const uint64_t* lo, const uint64_t* hi, int log2b, uint64_t cnt, uint32_t* tab,
                                uint64_t* raw, hipStream_t st) {
  if constexpr (KD > 16) {
    return hipErrorInvalidValue;
  } else {
    const uint64_t per_block = 4ull * Geo<KD>::G;  // 4 wavefronts of G entries
    const unsigned nb = (unsigned)((cnt + per_block - 1) / per_block);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL((k_table_build<KD, W, U>), dim3(nb), dim3(256), 0, st, lo, hi, log2b, cnt, tab, raw);
    return hipGetLastError();
  }
}

// ---------------------------------------------------------------------------
// one persistent launch for a batch of products (k <= 16)
// ---------------------------------------------------------------------------
// Copies with the descriptors in device memory, on one virtual block: vector
// v = block / tiles-per-vector, 256 words of it per block.
__device__ __forceinline__ void pad_dev_body(const CopyDesc* __restrict__ desc, uint64_t* __restrict__ work,
                                             uint64_t n, uint32_t k, VB vb) {
  const uint64_t per = (n * k + 255) / 256;
  const uint64_t v = vb.idx / per;
  const uint64_t t = (vb.idx - v * per) * 256 + threadIdx.x;
  if (t >= n * k) return;
  const uint64_t i = t / k;
  const uint32_t d = (uint32_t)(t - i * k);
  const CopyDesc cd = desc[v];
  work[v * n * k + t] = (i < cd.len) ? cd.src[(uint64_t)d * cd.ld + i] : 0ull;
}

// Unpad tile vb.idx: vector v = tile / per, per = tiles per vector; the
// tile transposes through LDS (ulds), and the trailing barrier lets the next
// tile reuse it.
template <int KD>
__device__ __forceinline__ void unpad_dev_body(const CopyDesc* __restrict__ desc, const uint64_t* __restrict__ work,
                                               uint64_t n, VB vb, uint64_t* __restrict__ ulds) {
  constexpr uint64_t E = kUnpadWords / KD;
  const uint64_t per = (n + E - 1) / E;
  const uint64_t v = vb.idx / per;
  const CopyDesc cd = desc[v];
  unpad_tile<KD>(cd, work + v * n * KD, vb.idx - v * per, ulds);
  __syncthreads();
}

template <int KD, int W, int U>
__device__ __forceinline__ void run_record(const PRec& R, uint64_t tile, uint32_t* __restrict__ stg,
                                           uint64_t* __restrict__ big) {
  const VB vb{tile, R.tiles};
  const uint64_t* in = reinterpret_cast<const uint64_t*>(R.in);
#define GFP_PBODY(INV, MODE, LAST, UNIF, T2)                                                                        \
  pass_body<KD, W, U, INV, MODE, LAST, UNIF, T2>(in, R.in2, R.se_in, R.sd_in, R.out, R.se_out, R.sd_out, R.tw, R.tw2, \
                                                 R.twr1, R.twr2, R.log2n, R.log2ns, R.ngroups, R.nvec, R.vin, R.vout, \
                                                 R.staged, vb, stg)
  switch (R.kind) {
    case PK_PAD:
      pad_dev_body(reinterpret_cast<const CopyDesc*>(R.in), R.out, R.ngroups, KD, vb);
      break;
    case PK_UNPAD:
      unpad_dev_body<KD>(reinterpret_cast<const CopyDesc*>(R.in), R.in2, R.ngroups, vb, big);
      break;
    case PK_MUL:
      elementwise_body<KD, W, U, GFP_OP_MUL>(in, KD, 1, R.in2, KD, 1, R.out, KD, 1, R.nvec, 0, nullptr, vb);
      break;
    case PK_PASS_FIRST: GFP_PBODY(false, MODE_PLAIN, false, false, false); break;
    case PK_PASS_MID: GFP_PBODY(false, MODE_PLAIN, false, true, true); break;
    case PK_PASS_IMID: GFP_PBODY(true, MODE_PLAIN, false, true, true); break;
    case PK_PASS_ILAST: GFP_PBODY(true, MODE_PLAIN, true, false, false); break;
    case PK_PASS_ISCALE: GFP_PBODY(true, MODE_SCALE, false, false, false); break;
    case PK_PASS_ISCALE_LAST: GFP_PBODY(true, MODE_SCALE, true, false, false); break;
    case PK_PASS_R_F:
    case PK_PASS_R_I: {
      const bool inv = R.kind == PK_PASS_R_I;
#define GFP_RBODY(LR)                                                                                              \
  if (inv) pass_r_body<KD, W, U, true, MODE_SCALE, LR>(in, R.in2, R.se_in, R.sd_in, R.out, R.se_out, R.sd_out, R.tw,  \
                                                       R.log2n, R.nvec, R.vin, R.vout, vb);                           \
  else pass_r_body<KD, W, U, false, MODE_PLAIN, LR>(in, R.in2, R.se_in, R.sd_in, R.out, R.se_out, R.sd_out, R.tw,     \
                                                    R.log2n, R.nvec, R.vin, R.vout, vb)
      if (R.lr == 1) {
        GFP_RBODY(1);
      } else if (R.lr == 2) {
        GFP_RBODY(2);
      } else if (R.lr == 3) {
        GFP_RBODY(3);
      } else if constexpr (KD >= 16) {
        if (R.lr == 4) {
          GFP_RBODY(4);
        }
      }
#undef GFP_RBODY
      break;
    }
#define GFP_P2BODY(INV, MODE, LAST, T2B)                                                                          \
  if constexpr (KD == 8) {                                                                                         \
    pass2_body<KD, W, U, INV, MODE, LAST, T2B>(in, R.in2, R.se_in, R.sd_in, R.out, R.se_out, R.sd_out, R.tw, R.tw1, \
                                               R.tw2, R.twr1, R.twr2, R.log2n, R.log2ns, R.nvec, R.vin, R.vout,     \
                                               R.staged, vb, big, stg);                                            \
    __syncthreads(); /* the next tile rewrites the transpose area */                                               \
  }
    case PK_PAIR_F_T2: GFP_P2BODY(false, MODE_PLAIN, false, true); break;
    case PK_PAIR_F: GFP_P2BODY(false, MODE_PLAIN, false, false); break;
    case PK_PAIR_I_T2: GFP_P2BODY(true, MODE_PLAIN, false, true); break;
    case PK_PAIR_I_LAST: GFP_P2BODY(true, MODE_PLAIN, true, false); break;
    case PK_PAIR_IS_T2: GFP_P2BODY(true, MODE_SCALE, false, true); break;
    case PK_PAIR_IS_LAST: GFP_P2BODY(true, MODE_SCALE, true, false); break;
#undef GFP_P2BODY
    default:
      break;
  }
#undef GFP_PBODY
}

// Grid-wide barrier between levels.  Each workgroup adds 1 to one of
// kSyncLines counters (one per 128-byte line, so the arrivals spread over
// memory channels instead of queueing on one address) after an agent-scope
// release fence; wavefront 0 then sums the counters (one per lane) until the
// total reaches gridDim.x (level + 1), and takes an agent-scope acquire
// fence.  The counters start at zero (written with the work list).  Measured
// on MI355X: 2-4x cheaper per level than the cooperative-groups grid barrier
// (768 workgroups: 27 against 53 us), the difference being the atomics on a
// single address.  Every workgroup is resident (cooperative launch), so every
// wait ends; the poll count is bounded all the same.
constexpr int kSyncLines = 64;
constexpr int kSyncStride = 32;  // uint32 words per counter line
__device__ __forceinline__ void level_barrier(uint32_t* __restrict__ sync, uint32_t target) {
  __syncthreads();  // every wavefront's stores are issued and complete to L2
  if (threadIdx.x == 0) {
    __threadfence();
    __hip_atomic_fetch_add(&sync[(blockIdx.x % kSyncLines) * kSyncStride], 1u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  }
  if (threadIdx.x < 64) {
    for (uint32_t poll = 0; poll < (1u << 26); ++poll) {
      uint32_t v = __hip_atomic_load(&sync[threadIdx.x * kSyncStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (v >= target) break;
      __builtin_amdgcn_s_sleep(1);
    }
    __threadfence();
  }
  __syncthreads();
}

// Every workgroup walks the tiles of a level (tile = blockIdx.x,
// blockIdx.x + gridDim.x, ...), the records of the level in tile order, then
// meets the others at the level barrier.  The LDS staging area is per
// wavefront, so tiles follow each other without a workgroup barrier.
// Registers: k = 8 at most 168 (three wavefronts per SIMD: at 128 the
// combined bodies spill), k = 16 at most 256 (two).
template <int KD, int W, int U>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KD == 16 ? 2 : 3, KD == 16 ? 2 : 3))) void k_batch_persistent(
    const PLevel* __restrict__ levels, uint32_t nlevels, const PRec* __restrict__ recs, uint32_t* __restrict__ sync) {
  static_assert(KD == 8 || KD == 16, "the persistent batch is built for k = 8 and 16");
  __shared__ uint32_t stg[4 * StageGeo<KD>::PER_WAVE];
  // the fused pairs' transposes (k = 8) or the unpad tiles
  constexpr int PAIR_WORDS = KD == 8 ? Span2Geo<KD>::BPW * Span2Geo<KD>::KB * Span2Geo<KD>::ROW : 0;
  constexpr int UNPAD_WORDS = kUnpadWords + kUnpadWords / KD;
  __shared__ uint64_t big[PAIR_WORDS > UNPAD_WORDS ? PAIR_WORDS : UNPAD_WORDS];
  for (uint32_t L = 0; L < nlevels; ++L) {
    const uint32_t r0 = levels[L].rec0, r1 = r0 + levels[L].nrec;
    const uint64_t tiles = levels[L].tiles;
    uint32_t r = r0;
    for (uint64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
      while (r + 1 < r1 && recs[r + 1].tile0 <= t) ++r;
      run_record<KD, W, U>(recs[r], t - recs[r].tile0, stg, big);
    }
    if (L + 1 < nlevels) level_barrier(sync, gridDim.x * (L + 1));
  }
}

template <int KD, int W, int U>
hipError_t launch_persistent_t(const PLevel* levels, uint32_t nlevels, const PRec* recs, uint32_t* sync,
                               uint32_t grid, hipStream_t st) {
  if constexpr (KD != 8 && KD != 16) {
    return hipErrorInvalidValue;
  } else {
    void* args[] = {(void*)&levels, (void*)&nlevels, (void*)&recs, (void*)&sync};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_batch_persistent<KD, W, U>), dim3(grid),
                                      dim3(256), args, 0, st);
  }
}

template <int KD, int W, int U>
int persistent_capacity_t(int* grid) {
  if constexpr (KD != 8 && KD != 16) {
    *grid = 0;
    return 0;
  } else {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_batch_persistent<KD, W, U>),
                                                     256, 0) != hipSuccess)
      return -1;
    *grid = per_cu * cus;
    return 0;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
inline unsigned blocks_for(uint64_t groups, int G) {
  const uint64_t per_block = 4ull * G;  // 4 wavefronts of 64 lanes per block
  return (unsigned)((groups + per_block - 1) / per_block);
}

template <int KD, int W, int U>
hipError_t launch_pass2_t(const PassArgs& p, hipStream_t st) {
  if constexpr (KD != 8 && KD != 16) {
    return hipErrorInvalidValue;
  } else {
    constexpr int LOGKB = ilog2(2 * KD);
    if (p.log2n < 2 * LOGKB || p.log2ns + 2 * LOGKB > p.log2n) return hipErrorInvalidValue;
    // the second pass takes the w^(K i) table unless it is the last pass
    const bool t2b = !p.last && p.log2n - 2 * LOGKB - (p.log2ns + LOGKB) >= 0;
    if (p.wide) {
      if constexpr (KD != 8) {
        return hipErrorInvalidValue;
      } else {
      // 8 blocks per workgroup: both halves with uniform twiddles
      if (p.log2n - 2 * LOGKB - p.log2ns < 3) return hipErrorInvalidValue;
      const uint64_t wgs = p.nvec << (p.log2n - 2 * LOGKB - 3);
#define GFP_LAUNCH2UB(INV, MODE, LAST, T2B, BND)                                                                  \
  hipLaunchKernelGGL((k_pass2u<KD, W, U, INV, MODE, LAST, T2B, BND>), dim3((unsigned)wgs),                          \
                     dim3(Span2UGeo<KD>::THREADS), 0, st, p.in, p.in2, p.se_in, p.sd_in, p.out, p.se_out, p.sd_out, \
                     p.tw, p.tw1, p.tw2, p.log2n, p.log2ns, p.nvec, p.vin, p.vout, p.in_len)
#define GFP_LAUNCH2U(INV, MODE, LAST, T2B) GFP_LAUNCH2UB(INV, MODE, LAST, T2B, false)
#define GFP_LAUNCH2U_T(INV, MODE)                   \
  if (p.last) GFP_LAUNCH2U(INV, MODE, true, false); \
  else if (t2b) GFP_LAUNCH2U(INV, MODE, false, true); \
  else GFP_LAUNCH2U(INV, MODE, false, false);
      if (p.in2) {
        GFP_LAUNCH2U_T(true, MODE_PRODUCT)
      } else if (p.scale) {
        GFP_LAUNCH2U_T(true, MODE_SCALE)
      } else if (p.inverse) {
        GFP_LAUNCH2U_T(true, MODE_PLAIN)
      } else if (p.in_len != ~0ull) {  // a product's first forward launch: the bounded variant
        if (p.last || !t2b) return hipErrorInvalidValue;
        GFP_LAUNCH2UB(false, MODE_PLAIN, false, true, true);
      } else {
        GFP_LAUNCH2U_T(false, MODE_PLAIN)
      }
#undef GFP_LAUNCH2U_T
#undef GFP_LAUNCH2U
#undef GFP_LAUNCH2UB
      return hipGetLastError();
      }
    }
    const uint64_t blocks = (p.nvec << (p.log2n - 2 * LOGKB));
    const unsigned nb = (unsigned)((blocks + Span2Geo<KD>::BPW - 1) / Span2Geo<KD>::BPW);
    if (nb == 0) return hipSuccess;
#define GFP_LAUNCH2B(INV, MODE, LAST, T2B, BND)                                                                    \
  hipLaunchKernelGGL((k_pass2<KD, W, U, INV, MODE, LAST, T2B, BND>), dim3(nb), dim3(Span2Geo<KD>::THREADS), 0, st,   \
                     p.in, p.in2, p.se_in, p.sd_in, p.out, p.se_out, p.sd_out, p.tw, p.tw1, p.tw2, p.twr1, p.twr2,    \
                     p.log2n, p.log2ns, p.nvec, p.vin, p.vout, (int)p.staged, p.in_len)
#define GFP_LAUNCH2(INV, MODE, LAST, T2B) GFP_LAUNCH2B(INV, MODE, LAST, T2B, false)
#define GFP_LAUNCH2_T(INV, MODE)                   \
  if (p.last) GFP_LAUNCH2(INV, MODE, true, false); \
  else if (t2b) GFP_LAUNCH2(INV, MODE, false, true); \
  else GFP_LAUNCH2(INV, MODE, false, false);
    if (p.in2) {
      GFP_LAUNCH2_T(true, MODE_PRODUCT)
    } else if (p.scale) {
      GFP_LAUNCH2_T(true, MODE_SCALE)
    } else if (p.inverse) {
      GFP_LAUNCH2_T(true, MODE_PLAIN)
    } else if (p.in_len != ~0ull) {  // a product's first forward launch: the bounded variant
      if (p.last) return hipErrorInvalidValue;
      if (t2b) GFP_LAUNCH2B(false, MODE_PLAIN, false, true, true);
      else GFP_LAUNCH2B(false, MODE_PLAIN, false, false, true);
    } else {
      GFP_LAUNCH2_T(false, MODE_PLAIN)
    }
#undef GFP_LAUNCH2_T
#undef GFP_LAUNCH2
#undef GFP_LAUNCH2B
    return hipGetLastError();
  }
}

template <int KD, int W, int U, int LR>
hipError_t launch_pass_r_lr(const PassArgs& p, hipStream_t st) {
  const unsigned nb = blocks_for(p.nvec << (p.log2n - LR), Geo<KD>::G);
  if (nb == 0) return hipSuccess;
#define GFP_LAUNCH_RB(INV, MODE, BND)                                                                          \
  hipLaunchKernelGGL((k_pass_r<KD, W, U, INV, MODE, LR, BND>), dim3(nb), dim3(256), 0, st, p.in, p.in2, p.se_in,   \
                     p.sd_in, p.out, p.se_out, p.sd_out, p.tw, p.log2n, p.nvec, p.vin, p.vout, p.in_len)
#define GFP_LAUNCH_R(INV, MODE) GFP_LAUNCH_RB(INV, MODE, false)
  if (p.in2) GFP_LAUNCH_R(true, MODE_PRODUCT);
  else if (p.scale) GFP_LAUNCH_R(true, MODE_SCALE);
  else if (p.inverse) GFP_LAUNCH_R(true, MODE_PLAIN);
  else if (p.in_len != ~0ull) GFP_LAUNCH_RB(false, MODE_PLAIN, true);  // a product's first forward launch
  else GFP_LAUNCH_R(false, MODE_PLAIN);
#undef GFP_LAUNCH_R
#undef GFP_LAUNCH_RB
  return hipGetLastError();
}

template <int KD, int W, int U>
hipError_t launch_pass_r_t(const PassArgs& p, hipStream_t st) {
  if (p.log2ns != 0 || p.last || p.log2n < p.radix_log2 + ilog2(2 * KD)) return hipErrorInvalidValue;
  switch (p.radix_log2) {
    case 1: return launch_pass_r_lr<KD, W, U, 1>(p, st);
    case 2: return launch_pass_r_lr<KD, W, U, 2>(p, st);
    case 3: return launch_pass_r_lr<KD, W, U, 3>(p, st);
    case 4:
      if constexpr (KD >= 16) return launch_pass_r_lr<KD, W, U, 4>(p, st);
      return hipErrorInvalidValue;
    case 5:
      if constexpr (KD >= 32) return launch_pass_r_lr<KD, W, U, 5>(p, st);
      return hipErrorInvalidValue;
    case 6:
      if constexpr (KD >= 64) return launch_pass_r_lr<KD, W, U, 6>(p, st);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <int KD, int W, int U>
hipError_t launch_pass_k32_t(const PassArgs& p, hipStream_t st) {
  constexpr int lk = ilog2(2 * KD);
  if (p.log2n < lk || p.log2ns + lk > p.log2n) return hipErrorInvalidValue;
  const uint64_t groups = p.ngroups * p.nvec;
  const unsigned nb = (unsigned)((groups + 1) / 2);  // two groups per workgroup
  if (nb == 0) return hipSuccess;
#define GFP_LAUNCH32(INV, MODE, LAST, T2, NTTM)                                                                    \
  hipLaunchKernelGGL((k_pass_k32<KD, W, U, INV, MODE, LAST, T2, NTTM>), dim3(nb), dim3(256), 0, st, p.in, p.in2,     \
                     p.se_in, p.sd_in, p.out, p.se_out, p.sd_out, p.tw, p.tw2, p.spec1, p.spec2, p.ntt, p.log2n,      \
                     p.log2ns, p.ngroups, p.nvec, p.vin, p.vout)
  const bool t2 = !p.last && p.log2n - 2 * lk - p.log2ns >= 0;
  // the scaled first launch of an inverse (a constant factor, MODE_SCALE or
  // MODE_PRODUCT) keeps the schoolbook product; plain passes need the tables
  if (p.ntt_mul && !p.in2 && !p.scale && (!p.spec1 || !p.ntt || (t2 && !p.spec2))) return hipErrorInvalidValue;
#define GFP_LAUNCH32_T(INV, MODE, NTTM)                  \
  if (p.last) GFP_LAUNCH32(INV, MODE, true, false, NTTM); \
  else if (t2) GFP_LAUNCH32(INV, MODE, false, true, NTTM); \
  else GFP_LAUNCH32(INV, MODE, false, false, NTTM);
  if (p.in2) {
    GFP_LAUNCH32_T(true, MODE_PRODUCT, false)
  } else if (p.scale) {
    GFP_LAUNCH32_T(true, MODE_SCALE, false)
  } else if (p.inverse) {
    if (p.ntt_mul) {
      GFP_LAUNCH32_T(true, MODE_PLAIN, true)
    } else {
      GFP_LAUNCH32_T(true, MODE_PLAIN, false)
    }
  } else {
    if (p.ntt_mul) {
      GFP_LAUNCH32_T(false, MODE_PLAIN, true)
    } else {
      GFP_LAUNCH32_T(false, MODE_PLAIN, false)
    }
  }
#undef GFP_LAUNCH32_T
#undef GFP_LAUNCH32
  return hipGetLastError();
}

template <int KD, int W, int U>
hipError_t launch_pass_k64_t(const PassArgs& p, hipStream_t st) {
  constexpr int lk = ilog2(2 * KD);
  if (p.log2n < lk || p.log2ns + lk > p.log2n) return hipErrorInvalidValue;
  const uint64_t nb = p.ngroups * p.nvec;  // one group per workgroup
  if (nb == 0) return hipSuccess;
  if (nb > 0xFFFFFFFFull) return hipErrorInvalidValue;
#define GFP_LAUNCH64(INV, MODE, LAST, T2, NTTM)                                                                     \
  hipLaunchKernelGGL((k_pass_k64<KD, W, U, INV, MODE, LAST, T2, NTTM>), dim3((unsigned)nb), dim3(256), 0, st, p.in,    \
                     p.in2, p.se_in, p.sd_in, p.out, p.se_out, p.sd_out, p.tw, p.tw2, p.spec1, p.spec2, p.ntt, p.log2n, \
                     p.log2ns, p.ngroups, p.nvec, p.vin, p.vout)
  const bool t2 = !p.last && p.log2n - 2 * lk - p.log2ns >= 0;
  // the scaled first launch of an inverse (a constant factor, MODE_SCALE or
  // MODE_PRODUCT) keeps the schoolbook product; plain passes need the tables
  if (p.ntt_mul && !p.in2 && !p.scale && (!p.spec1 || !p.ntt || (t2 && !p.spec2))) return hipErrorInvalidValue;
#define GFP_LAUNCH64_T(INV, MODE, NTTM)                  \
  if (p.last) GFP_LAUNCH64(INV, MODE, true, false, NTTM); \
  else if (t2) GFP_LAUNCH64(INV, MODE, false, true, NTTM); \
  else GFP_LAUNCH64(INV, MODE, false, false, NTTM);
  if (p.in2) {
    GFP_LAUNCH64_T(true, MODE_PRODUCT, false)
  } else if (p.scale) {
    GFP_LAUNCH64_T(true, MODE_SCALE, false)
  } else if (p.inverse) {
    if (p.ntt_mul) {
      GFP_LAUNCH64_T(true, MODE_PLAIN, true)
    } else {
      GFP_LAUNCH64_T(true, MODE_PLAIN, false)
    }
  } else {
    if (p.ntt_mul) {
      GFP_LAUNCH64_T(false, MODE_PLAIN, true)
    } else {
      GFP_LAUNCH64_T(false, MODE_PLAIN, false)
    }
  }
#undef GFP_LAUNCH64_T
#undef GFP_LAUNCH64
  return hipGetLastError();
}

template <int KD, int W, int U>
hipError_t launch_pass_t(const PassArgs& p, hipStream_t st) {
  if (p.in2 && (!p.scale || p.sd_in != 1 || (p.se_in & 1) || (p.vin & 1) || (reinterpret_cast<uintptr_t>(p.in2) & 15)))
    return hipErrorInvalidValue;  // the product operand is read 16 bytes at a time
  if (p.radix_log2 != 0) return launch_pass_r_t<KD, W, U>(p, st);
  if (p.span == 2) return launch_pass2_t<KD, W, U>(p, st);
  if (p.span != 1) return hipErrorInvalidValue;
  if constexpr (KD == 32) {
    return launch_pass_k32_t<KD, W, U>(p, st);
  } else if constexpr (KD == 64) {
    return launch_pass_k64_t<KD, W, U>(p, st);
  } else {
  const unsigned nb = blocks_for(p.ngroups * p.nvec, Geo<KD>::G);
  if (nb == 0) return hipSuccess;
#define GFP_LAUNCHB(INV, MODE, LAST, UNIF, T2, BND)                                                                 \
  hipLaunchKernelGGL((k_pass<KD, W, U, INV, MODE, LAST, UNIF, T2, BND>), dim3(nb), dim3(256), 0, st, p.in, p.in2,      \
                     p.se_in, p.sd_in, p.out, p.se_out, p.sd_out, p.tw, p.tw2, p.twr1, p.twr2, p.log2n, p.log2ns,      \
                     p.ngroups, p.nvec, p.vin, p.vout, (int)p.staged, p.in_len)
#define GFP_LAUNCH(INV, MODE, LAST, UNIF, T2) GFP_LAUNCHB(INV, MODE, LAST, UNIF, T2, false)
  // uniform twiddles when every base a has at least one wavefront of groups;
  // the w^(K i) table for every pass but the last
  const int lk = ilog2(2 * KD);
  const bool unif = p.log2ns > 0 && (p.log2n - lk - p.log2ns) >= ilog2(Geo<KD>::G);
  const bool t2 = !p.last && p.log2n - 2 * lk - p.log2ns >= 0;
#define GFP_LAUNCH_T(INV)                                                    \
  if (p.last) GFP_LAUNCH(INV, MODE_PLAIN, true, false, false);               \
  else if (unif && t2) GFP_LAUNCH(INV, MODE_PLAIN, false, true, true);       \
  else if (unif) GFP_LAUNCH(INV, MODE_PLAIN, false, true, false);            \
  else if (t2) GFP_LAUNCH(INV, MODE_PLAIN, false, false, true);              \
  else GFP_LAUNCH(INV, MODE_PLAIN, false, false, false);
  if (p.in2) {
    if (p.last) GFP_LAUNCH(true, MODE_PRODUCT, true, false, false);
    else GFP_LAUNCH(true, MODE_PRODUCT, false, false, false);
  } else if (p.scale) {
    if (p.last) GFP_LAUNCH(true, MODE_SCALE, true, false, false); else GFP_LAUNCH(true, MODE_SCALE, false, false, false);
  } else if (p.inverse) {
    GFP_LAUNCH_T(true)
  } else if (p.in_len != ~0ull) {  // a product's first forward launch (Ns = 1): the bounded variant
    if (p.last || unif) return hipErrorInvalidValue;
    if (t2) GFP_LAUNCHB(false, MODE_PLAIN, false, false, true, true);
    else GFP_LAUNCHB(false, MODE_PLAIN, false, false, false, true);
  } else {
    GFP_LAUNCH_T(false)
  }
#undef GFP_LAUNCH_T
#undef GFP_LAUNCH
#undef GFP_LAUNCHB
  return hipGetLastError();
  }
}

template <int KD, int W, int U>
hipError_t launch_elementwise_t(const EwArgs& a, hipStream_t st) {
  const unsigned nb = blocks_for(a.n, Geo<KD>::G);
  if (nb == 0) return hipSuccess;
#define GFP_LAUNCH_EW(OP)                                                                                        \
  hipLaunchKernelGGL((k_elementwise<KD, W, U, OP>), dim3(nb), dim3(256), 0, st, a.x, a.xse, a.xsd, a.y, a.yse, a.ysd, \
                     a.z, a.zse, a.zsd, a.n, a.s, a.cst)
  switch (a.op) {
    case GFP_OP_ADD: GFP_LAUNCH_EW(GFP_OP_ADD); break;
    case GFP_OP_SUB: GFP_LAUNCH_EW(GFP_OP_SUB); break;
    case GFP_OP_MUL: GFP_LAUNCH_EW(GFP_OP_MUL); break;
    case GFP_OP_MUL_POW_R: GFP_LAUNCH_EW(GFP_OP_MUL_POW_R); break;
    case GFP_OP_MUL_CONST: GFP_LAUNCH_EW(GFP_OP_MUL_CONST); break;
    case GFP_OP_MUL_SCALE: GFP_LAUNCH_EW(GFP_OP_MUL_SCALE); break;
    case GFP_OP_MUL_NTT: GFP_LAUNCH_EW(GFP_OP_MUL_NTT); break;
    default: return hipErrorInvalidValue;
  }
#undef GFP_LAUNCH_EW
  return hipGetLastError();
}

}  // namespace gfpk

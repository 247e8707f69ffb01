// Device arithmetic for Z/pZ, p = r^k + 1, r = 2^W + 2^U, on gfx950.
//
// Lane layout ("digit lanes").  A wavefront of 64 lanes is 4 DPP rows of 16
// lanes.  An element's k digits live in k lanes of one row: lane-in-row
// d * GPL + s holds digit d of the row's element s, GPL = 16 / k elements per
// row.  So k = 8 interleaves two elements per row and k = 16 uses one row per
// element.  Multiplying by r^i (section 2.3: a cyclic shift of the digits with
// the wrapped digits negated, since r^k = -1) is then a DPP row rotation by
// i * GPL lanes plus a per-lane sign, with no data leaving the row.  For
// k = 32 an element spans half a wavefront (lane (l & 32) | d holds digit d)
// and the rotations are ds_bpermute lane permutations within the half.
//
// Digits in flight are "lazy": a digit is any integer, the element being
// sum_d t_d r^d mod p (f_x(r) in the polynomial view of section 2).  Lazy
// digits are signed 96-bit (L96).  The base-case DFT adds and subtracts them
// without carries; a normalisation step later brings every digit back into
// 64 bits ("semi-normalised", [0, 2^64)) or to the canonical encoding of
// section 2 (digits < r, p - 1 written (r, 0, ..., 0)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace gfpk {

typedef unsigned __int128 u128;
typedef __int128 i128;

// ------------------------------------------------------------------------
// compile-time loops
// ------------------------------------------------------------------------
template <int I>
using IC = std::integral_constant<int, I>;

template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(IC<Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
constexpr int brev(int i, int bits) {
  int o = 0;
  for (int b = 0; b < bits; ++b) o |= ((i >> b) & 1) << (bits - 1 - b);
  return o;
}

// ------------------------------------------------------------------------
// lane geometry
// ------------------------------------------------------------------------
template <int KD>
struct Geo {
  static_assert(KD == 8 || KD == 16 || KD == 32 || KD == 64, "k must be 8, 16, 32 or 64");
  static constexpr bool ROW = KD <= 16;          // an element inside one DPP row
  static constexpr int GPL = ROW ? 16 / KD : 1;  // elements per DPP row (k <= 16)
  static constexpr int G = 64 / KD;              // elements per wavefront
  static constexpr int KB = 2 * KD;              // base-case DFT size K = 2k
  static constexpr int HI = 63 & ~(KD - 1);      // lane bits naming the element (k >= 32)
  __device__ static __forceinline__ int lane() { return (int)(threadIdx.x & 63); }
  __device__ static __forceinline__ int digit(int l) { return ROW ? (l & 15) / GPL : (l & (KD - 1)); }
  __device__ static __forceinline__ int group(int l) {
    return ROW ? (l >> 4) * GPL + (l & 15) % GPL : (l >> ilog2(KD));
  }
  // lane holding digit d of the same element as lane l
  __device__ static __forceinline__ int lane_of(int l, int d) {
    return ROW ? ((l & 0x30) | (d * GPL) | ((l & 15) % GPL)) : ((l & HI) | d);
  }
  // Shorter product tail (add_carried_q, undefined-old rotations, one SGPR
  // constant per shifted add): the default of the LN template parameter
  // below.  k = 16 keeps the longer forms by default (its fused pairs and
  // elementwise kernels); its single-pass kernels set LN = true themselves.
  static constexpr bool LEAN = KD != 16;
};

// DPP row rotate: lane i of a row takes the value of lane (i - N) mod 16.
template <int N>
__device__ __forceinline__ uint32_t row_ror(uint32_t v) {
  if constexpr ((N & 15) == 0) {
    return v;
  } else {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x120 + (N & 15), 0xF, 0xF, false);
  }
}

// row_ror for a result used as is: every lane of a rotation reads a valid
// lane, so the DPP "old" operand is never taken and is left undefined (no
// register to clear first).  row_ror keeps old = 0, which lets the compiler
// fold a rotation into the DPP form of the xor that follows it.
template <int N>
__device__ __forceinline__ uint32_t row_ror_u(uint32_t v) {
  if constexpr ((N & 15) == 0) {
    return v;
  } else {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x120 + (N & 15), 0xF, 0xF, false);
  }
}

// Digit rotation: the lane holding digit m of an element takes the value of
// the lane holding digit (m - N) mod k of the same element.
template <int KD, int N>
__device__ __forceinline__ uint32_t dig_rot(uint32_t v) {
  constexpr int n = N & (KD - 1);
  if constexpr (n == 0) {
    return v;
  } else if constexpr (Geo<KD>::ROW) {
    return row_ror<n * Geo<KD>::GPL>(v);
  } else if constexpr (KD == 64 && n == 1) {
    // one element spans the whole wavefront: a one-lane rotation is a single
    // DPP wave_ror:1 (lane i reads lane i - 1 mod 64), no LDS crossbar trip
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x13C, 0xF, 0xF, false);
  } else {
    const int l = (int)(threadIdx.x & 63);
    return (uint32_t)__builtin_amdgcn_ds_bpermute(((l & Geo<KD>::HI) | ((l - n) & (KD - 1))) << 2, (int)v);
  }
}

// dig_rot with the undefined-old forms (LN).
template <int KD, int N, bool LN = Geo<KD>::LEAN>
__device__ __forceinline__ uint32_t dig_rot_u(uint32_t v) {
  constexpr int n = N & (KD - 1);
  if constexpr (!LN || n == 0) {
    return dig_rot<KD, N>(v);
  } else if constexpr (Geo<KD>::ROW) {
    return row_ror_u<n * Geo<KD>::GPL>(v);
  } else if constexpr (KD == 64 && n == 1) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x13C, 0xF, 0xF, false);
  } else {
    return dig_rot<KD, N>(v);
  }
}

// ------------------------------------------------------------------------
// lazy digits
// ------------------------------------------------------------------------
struct L96 {
  uint64_t lo;
  int32_t hi;
};

__device__ __forceinline__ L96 l96(uint64_t x) { return L96{x, 0}; }
__device__ __forceinline__ L96 l96_add(L96 a, L96 b) {
  L96 c;
  c.lo = a.lo + b.lo;
  c.hi = a.hi + b.hi + (int32_t)(c.lo < a.lo);
  return c;
}
__device__ __forceinline__ L96 l96_sub(L96 a, L96 b) {
  L96 c;
  c.lo = a.lo - b.lo;
  c.hi = a.hi - b.hi - (int32_t)(a.lo < b.lo);
  return c;
}
__device__ __forceinline__ L96 l96_sel(bool c, L96 a, L96 b) { return L96{c ? a.lo : b.lo, c ? a.hi : b.hi}; }
template <int KD, int N, bool LN = Geo<KD>::LEAN>
__device__ __forceinline__ L96 l96_rot(L96 a) {
  uint32_t w0 = dig_rot_u<KD, N, LN>((uint32_t)a.lo), w1 = dig_rot_u<KD, N, LN>((uint32_t)(a.lo >> 32));
  uint32_t w2 = dig_rot_u<KD, N, LN>((uint32_t)a.hi);
  return L96{((uint64_t)w1 << 32) | w0, (int32_t)w2};
}
// a r^e for a run-time exponent 0 <= e < 2k (r^k = -1): lane m takes digit
// (m - e) mod k from the lane holding it, negated when it wrapped (m < e mod
// k) and once more when e >= k.
template <int KD>
__device__ __forceinline__ L96 l96_mul_rpow(L96 a, int e, int l, int m) {
  const int n = e & (KD - 1);
  const int src = Geo<KD>::lane_of(l, (m - n) & (KD - 1));
  const uint32_t w0 = (uint32_t)__shfl((int)(uint32_t)a.lo, src, 64);
  const uint32_t w1 = (uint32_t)__shfl((int)(uint32_t)(a.lo >> 32), src, 64);
  const uint32_t w2 = (uint32_t)__shfl((int)a.hi, src, 64);
  const L96 b{((uint64_t)w1 << 32) | w0, (int32_t)w2};
  const bool neg = (m < n) != ((e & KD) != 0);
  return neg ? l96_sub(L96{0, 0}, b) : b;
}
__device__ __forceinline__ L96 l96_from_i128(i128 v) { return L96{(uint64_t)v, (int32_t)(uint32_t)((u128)v >> 64)}; }
__device__ __forceinline__ i128 l96_to_i128(L96 a) { return ((i128)a.hi << 64) + (i128)a.lo; }

// ------------------------------------------------------------------------
// Radix-2 DIT base case DFT_K (K = 2k) at root r (or r^-1) on lazy digits.
//
// Section 4.3 builds DFT_K from DFT_2 = (x0 + x1, x0 - x1) and twiddles that
// are powers of r (the reduction formula for DFT_{2^n}).  Here: input slots
// in natural order are read in bit-reversed order, log2 K butterfly levels,
// output in natural order.  Butterfly (a, b) at exponent i: b' = b r^{+-i},
// outputs a + b', a - b'.  b r^i is the row rotation by i digits with the
// wrapped lanes (digit m < i) negated; the negation is folded into the
// butterfly: by swapping its two outputs in those lanes, or (CB) by adding
// the complement of the rotated word with a carry-in of 1.  CB is chosen per
// kernel: it pays where its rotations fold into DPP xors (the fused pairs,
// the k = 16 uniform-twiddle passes, k = 32, 64) and not in the k = 8 last
// pass or the k = 16 per-group passes.
// ------------------------------------------------------------------------
template <int KD, bool INV, int EXP, bool LN = Geo<KD>::LEAN, bool CB = Geo<KD>::LEAN>
__device__ __forceinline__ void bfly(L96& a, L96& b, int m) {
  if constexpr (EXP == 0) {
    L96 s = l96_add(a, b), d = l96_sub(a, b);
    a = s;
    b = d;
  } else {
    // forward: r^EXP = rotate by EXP, negate digits m < EXP.
    // inverse: r^-EXP = -r^(KD-EXP) = rotate by KD-EXP, negate digits m >= KD-EXP.
    constexpr int ROT = INV ? (KD - EXP) : EXP;
    const bool f = INV ? (m >= ROT) : (m < ROT);
    if constexpr (CB) {
      // in the negated lanes b' = ~bp + 1 = -bp: the complement rides on the
      // rotation (DPP xor) and the 1 enters as the carry of a + b' and the
      // borrow of a - b', so a + b' = a - bp and a - b' = a + bp (mod 2^96)
      const uint32_t M = f ? 0xFFFFFFFFu : 0u;
      const uint32_t b0 = dig_rot<KD, ROT>((uint32_t)b.lo) ^ M;
      const uint32_t b1 = dig_rot<KD, ROT>((uint32_t)(b.lo >> 32)) ^ M;
      const uint32_t b2 = dig_rot<KD, ROT>((uint32_t)b.hi) ^ M;
      const uint32_t a0 = (uint32_t)a.lo, a1 = (uint32_t)(a.lo >> 32), a2 = (uint32_t)a.hi;
      unsigned c, w;
      const uint32_t s0 = __builtin_addc(a0, b0, (unsigned)f, &c);
      const uint32_t s1 = __builtin_addc(a1, b1, c, &c);
      const uint32_t s2 = a2 + b2 + c;
      const uint32_t d0 = __builtin_subc(a0, b0, (unsigned)f, &w);
      const uint32_t d1 = __builtin_subc(a1, b1, w, &w);
      const uint32_t d2 = a2 - b2 - w;
      a = L96{((uint64_t)s1 << 32) | s0, (int32_t)s2};
      b = L96{((uint64_t)d1 << 32) | d0, (int32_t)d2};
    } else {
      L96 bp = l96_rot<KD, ROT, LN>(b);
      L96 s = l96_add(a, bp), d = l96_sub(a, bp);
      a = l96_sel(f, d, s);
      b = l96_sel(f, s, d);
    }
  }
}

// DFT_P, P = 2^LP <= K, at root r^(K/P) (a primitive P-th root of unity,
// since r has order K = 2k): the first LP levels of the same network.  At
// level half-size H the butterfly j uses (r^(K/P))^(j P/(2H)) = r^(j K/(2H)),
// the exponent DFT_K uses at that level.
template <int KD, bool INV, int LP, bool LN = Geo<KD>::LEAN, bool CB = Geo<KD>::LEAN>
__device__ __forceinline__ void dft_pow2(L96 (&v)[1 << LP], int m) {
  constexpr int KB = 2 * KD;
  constexpr int P = 1 << LP;
  static_assert(P >= 2 && P <= KB, "DFT size");
  L96 a[P];
  static_for<P>([&](auto I) {
    constexpr int i = decltype(I)::value;
    a[i] = v[brev(i, LP)];
  });
  static_for<LP>([&](auto S) {
    constexpr int H = 1 << decltype(S)::value;  // half size of this level
    static_for<P / 2>([&](auto B) {
      constexpr int blk = decltype(B)::value / H, j = decltype(B)::value % H;
      constexpr int i0 = blk * 2 * H + j;
      constexpr int e = j * (KB / (2 * H));  // exponent of r, 0 <= e < KD
      bfly<KD, INV, e, LN, CB>(a[i0], a[i0 + H], m);
    });
  });
  static_for<P>([&](auto I) {
    constexpr int i = decltype(I)::value;
    v[i] = a[i];
  });
}

template <int KD, bool INV, bool LN = Geo<KD>::LEAN, bool CB = Geo<KD>::LEAN>
__device__ __forceinline__ void dft_base(L96 (&v)[2 * KD], int m) {
  dft_pow2<KD, INV, ilog2(2 * KD), LN, CB>(v, m);
}

// ------------------------------------------------------------------------
// Product x * y in Z/pZ, one output column per lane (section 3.1.1).
//
// Column m of f_x f_y mod (R^k + 1) is u_m = sum_{i+j=m} x_i y_j -
// sum_{i+j=m+k} x_i y_j.  Lane m starts with x_m and, at step t, holds
// x_{m-t} (the digits travel one lane up per step, DPP row rotate); it
// multiplies by y_t.  A digit crossing from lane k-1 to lane 0 is a term of
// the negative sum; instead of negating it the lane stores its bitwise
// complement ~x = (2^64 - 1) - x, so every product stays unsigned, and the
// column is corrected afterwards by -(2^64 - 1) * S_m, S_m = the sum of the
// y_t met with complemented x.  An extra factor r^rho (twiddle rotation,
// section 4.1: w^(i N/K + j) = r^i w^j) is applied by starting lane m with
// x_{m - rho} under the same complement rule (the caller loads that digit).
//
// x is split into two 32-bit limbs and each y_t into three limbs of 22, 22
// and 20 bits, so every limb product is < 2^54 and k of them fit in a 64-bit
// accumulator: six v_mad_u64_u32 per digit pair, no carries.
//
// The column C (|C| < k r^2 + 2^132) is then gathered into 64-bit cells at
// 32-bit positions and folded three times with 2^64 = a r - b
// (a = 2^(64-W), b = 2^(64-W+U)) into C = Q r + T: T is this lane's lazy
// digit (|T| < 2^65) and Q (|Q| < 2^74) is carried to column m+1 (negated
// into column 0, r^k = -1).  The paper's (l, h, c) split of section 3.1.1 is
// the same idea with c carried two columns.
// ------------------------------------------------------------------------
// ------------------------------------------------------------------------
// word helpers for the fold
// ------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lo32(uint64_t x) { return (uint32_t)x; }
__device__ __forceinline__ uint32_t hi32(uint64_t x) { return (uint32_t)(x >> 32); }
// A constant the compiler cannot see through, so x * c + acc stays one
// v_mad_u64_u32 with the constant in an SGPR instead of a shift-and-mask.
__device__ __forceinline__ uint32_t sgpr_const(uint32_t c) {
  uint32_t v;
  asm("s_mov_b32 %0, %1" : "=s"(v) : "i"(c));
  return v;
}
// The same as a value of its own (ID tells the copies apart), so that the
// compiler cannot merge x*c + y*c into (x + y)*c: that 64-bit add of two
// zero-extended words costs more than the second v_mad_u64_u32.
template <int ID>
__device__ __forceinline__ uint32_t sgpr_const_n(uint32_t c) {
  uint32_t v;
  asm("s_mov_b32 %0, %1 ; %2" : "=s"(v) : "i"(c), "i"(ID));
  return v;
}
__device__ __forceinline__ uint64_t mad32(uint32_t x, uint32_t c, uint64_t acc) { return (uint64_t)x * c + acc; }
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, int sh) {  // (hi:lo) >> sh, 0 < sh < 32
  return __builtin_amdgcn_alignbit(hi, lo, sh);
}

// (o0..o3) = (l0, l1) - 2^SB (h0, h1, h2), as a signed 128-bit value
// truncated to 4 words (the caller knows the result fits).
template <int SB>
__device__ __forceinline__ void sub_shifted96(uint32_t l0, uint32_t l1, uint32_t h0, uint32_t h1, uint32_t h2,
                                              uint32_t& o0, uint32_t& o1, uint32_t& o2, uint32_t& o3) {
  unsigned b;
  if constexpr (SB >= 32) {
    constexpr int s = SB - 32;  // 2^SB H = (0, h0 << s, ...)
    const uint32_t w1 = s ? (h0 << s) : h0;
    const uint32_t w2 = s ? funnel(h1, h0, 32 - s) : h1;
    const uint32_t w3 = s ? funnel(h2, h1, 32 - s) : h2;
    o0 = l0;
    o1 = __builtin_subc(l1, w1, 0u, &b);
    o2 = __builtin_subc(0u, w2, b, &b);
    o3 = __builtin_subc(0u, w3, b, &b);
  } else {
    constexpr int s = SB;
    const uint32_t w0 = h0 << s;
    const uint32_t w1 = funnel(h1, h0, 32 - s);
    const uint32_t w2 = funnel(h2, h1, 32 - s);
    const uint32_t w3 = (uint32_t)((int32_t)h2 >> (32 - s));
    o0 = __builtin_subc(l0, w0, 0u, &b);
    o1 = __builtin_subc(l1, w1, b, &b);
    o2 = __builtin_subc(0u, w2, b, &b);
    o3 = __builtin_subc(0u, w3, b, &b);
  }
}

// (o0, o1, o2) = (l0, l1) - 2^SB (v2, v3) with (v2, v3) a signed 64-bit
// value; o2 is the signed high word (the result fits in 96 bits).
template <int SB>
__device__ __forceinline__ void sub_shifted64(uint32_t l0, uint32_t l1, uint32_t v2, uint32_t v3, uint32_t& o0,
                                              uint32_t& o1, uint32_t& o2) {
  unsigned b;
  if constexpr (SB >= 32) {
    constexpr int s = SB - 32;
    const uint32_t w1 = s ? (v2 << s) : v2;
    const uint32_t w2 = s ? funnel(v3, v2, 32 - s) : v3;
    o0 = l0;
    o1 = __builtin_subc(l1, w1, 0u, &b);
    o2 = __builtin_subc(0u, w2, b, &b);
  } else {
    constexpr int s = SB;
    const uint32_t w0 = v2 << s;
    const uint32_t w1 = funnel(v3, v2, 32 - s);
    const uint32_t w2 = (uint32_t)((int32_t)v3 >> (32 - s));
    o0 = __builtin_subc(l0, w0, 0u, &b);
    o1 = __builtin_subc(l1, w1, b, &b);
    o2 = __builtin_subc(0u, w2, b, &b);
  }
}

// (l0, l1) - 2^SB wh for a small signed wh, as a lazy digit.
template <int SB>
__device__ __forceinline__ L96 sub_shifted32(uint32_t l0, uint32_t l1, uint32_t wh) {
  unsigned b;
  uint32_t o0, o1, o2;
  if constexpr (SB >= 32) {
    constexpr int s = SB - 32;
    const uint32_t w1 = wh << s;
    const uint32_t w2 = s ? (uint32_t)((int32_t)wh >> (32 - s)) : (uint32_t)((int32_t)wh >> 31);
    o0 = l0;
    o1 = __builtin_subc(l1, w1, 0u, &b);
    o2 = __builtin_subc(0u, w2, b, &b);
  } else {
    constexpr int s = SB;
    const uint32_t w0 = wh << s;
    const uint32_t w1 = (uint32_t)((int32_t)wh >> (32 - s));
    const uint32_t w2 = (uint32_t)((int32_t)wh >> 31);
    o0 = __builtin_subc(l0, w0, 0u, &b);
    o1 = __builtin_subc(l1, w1, b, &b);
    o2 = __builtin_subc(0u, w2, b, &b);
  }
  return L96{((uint64_t)o1 << 32) | o0, (int32_t)o2};
}

// Radix shape: r = 2^W + 2^U for U > 0, r = 2^W - 2^|U| for U < 0.
template <int KD, int W, int U>
struct Field {
  static constexpr bool NEG = U < 0;
  static constexpr int UA = NEG ? -U : U;
  static constexpr uint64_t R = NEG ? (1ull << W) - (1ull << UA) : (1ull << W) + (1ull << UA);
  static constexpr int SA = 64 - W;      // 2^64 = 2^SA * r - 2^SB (U > 0)
  static constexpr int SB = 64 - W + U;
  // SPLIT: a fold with 2^64 = 2^SA r - 2^SB gains only W - U bits a round
  // (U close to W), or does not apply (U < 0).  Then r = 2^UA d with
  // d = 2^(W-UA) +- 1, and an integer t splits exactly as t = q r + rho,
  // rho = (t_h mod d) 2^UA + t_l in [0, r), where t_h = floor(t / 2^UA),
  // t_l = t mod 2^UA and q = floor(t_h / d).  Built for the k = 32 and
  // k = 64 primes of Table 1: r = 2^62 + 2^56 (d = 65) and r = 2^63 - 2^40
  // (d = 2^23 - 1).
  static constexpr bool SPLIT = NEG || U + 8 > W;
  // window of the remainder rho = t - (t >> W) r of a lazy digit: it lies in
  // (-OFF, 2^W + OFF); below 2 OFF it takes one more r, so that a carry of
  // up to 2^31 in either direction keeps the digit inside [0, 2^64)
  static constexpr uint64_t OFF = W >= 58 ? (1ull << 57) : (1ull << (W - 3));
  static_assert(W >= 56 && W <= 63 &&
                    ((U >= 8 && U + 8 <= W) || (W == 62 && U == 56) || (W == 63 && U == -40)),
                "unsupported radix shape");
};

// SPLIT division for r = 2^56 * 65.  65 is odd and 2^12 = 1 (mod 65), so
// n mod 65 is the sum of n's 12-bit chunks (words weighted by 2^32 = 61 and
// 2^64 = 16 mod 65) reduced once, and the quotient of the exact multiple
// n - (n mod 65) is its product with 65^-1 mod 2^96.
__device__ __forceinline__ uint32_t chunks12(uint32_t x) {
  return (x >> 24) + ((x >> 12) & 0xFFFu) + (x & 0xFFFu);
}

// C = (c0, c1, c2, c3, c4) signed 160-bit (c4 carries the sign), |C| < 2^133:
// C = Q r + T with 0 <= T < r.
__device__ __forceinline__ void split_qr160(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t c4,
                                            uint64_t& T, L96& Q) {
  // n = floor(C / 2^56) + 65 * 2^78, in [0, 2^86): three words
  const uint32_t n0 = __builtin_amdgcn_alignbit(c2, c1, 24);
  const uint32_t n1 = __builtin_amdgcn_alignbit(c3, c2, 24);
  const uint32_t n2 = __builtin_amdgcn_alignbit(c4, c3, 24) + (65u << 14);
  // n mod 65 from t < 2^20, t = n (mod 65); floor(t / 65) = t ceil(2^30 / 65) >> 30
  const uint32_t t = chunks12(n0) + 61u * chunks12(n1) + 16u * chunks12(n2);
  const uint32_t qt = (uint32_t)(((uint64_t)t * 16519105u) >> 30);
  const uint32_t rem = t - 65u * qt;
  // q' = (n - rem) / 65 = (n - rem) 65^-1 mod 2^96
  unsigned b;
  const uint32_t m0 = __builtin_subc(n0, rem, 0u, &b);
  const uint32_t m1 = __builtin_subc(n1, 0u, b, &b);
  const uint32_t m2 = n2 - b;
  constexpr uint32_t I0 = 0xC0FC0FC1u, I1 = 0x0FC0FC0Fu, I2 = 0xFC0FC0FCu;  // 65^-1 mod 2^96
  const uint64_t pa = (uint64_t)m0 * I0;
  const uint64_t pb = (uint64_t)m0 * I1 + (pa >> 32);
  const uint64_t pc = (uint64_t)m1 * I0 + (uint32_t)pb;
  const uint32_t q2 = (uint32_t)(pb >> 32) + (uint32_t)(pc >> 32) + m0 * I2 + m1 * I1 + m2 * I0;
  // Q = q' - 2^78
  Q.lo = ((uint64_t)(uint32_t)pc << 32) | (uint32_t)pa;
  Q.hi = (int32_t)(q2 - (1u << 14));
  T = ((uint64_t)((rem << 24) | (c1 & 0xFFFFFFu)) << 32) | c0;
}

// SPLIT division for r = 2^40 (2^23 - 1) (the k = 64 prime of Table 1).
// d = 2^23 - 1 is odd and 2^23 = 1 (mod d): n mod d is the sum of n's 23-bit
// chunks folded twice, and the quotient of the exact multiple n - (n mod d)
// is its product with d^-1 mod 2^96.  C as for split_qr160, |C| < 2^134.
__device__ __forceinline__ void split_qr160_m23(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t c4,
                                                uint64_t& T, L96& Q) {
  constexpr uint32_t D = (1u << 23) - 1, M23 = D;
  // n = floor(C / 2^40) + d 2^72, in [0, 2^96)
  const uint32_t n0 = __builtin_amdgcn_alignbit(c2, c1, 8);
  const uint32_t n1 = __builtin_amdgcn_alignbit(c3, c2, 8);
  const uint32_t n2 = __builtin_amdgcn_alignbit(c4, c3, 8) + (D << 8);
  uint32_t t = (n0 & M23) + (((n0 >> 23) | (n1 << 9)) & M23) + (((n1 >> 14) | (n2 << 18)) & M23) +
               ((n2 >> 5) & M23) + (n2 >> 28);
  t = (t & M23) + (t >> 23);
  t = (t & M23) + (t >> 23);
  const uint32_t rem = (t == D) ? 0u : t;
  unsigned b;
  const uint32_t m0 = __builtin_subc(n0, rem, 0u, &b);
  const uint32_t m1 = __builtin_subc(n1, 0u, b, &b);
  const uint32_t m2 = n2 - b;
  constexpr uint32_t I0 = 0xFF7FFFFFu, I1 = 0xFFFFBFFFu, I2 = 0xEFFFFFDFu;  // (2^23 - 1)^-1 mod 2^96
  const uint64_t pa = (uint64_t)m0 * I0;
  const uint64_t pb = (uint64_t)m0 * I1 + (pa >> 32);
  const uint64_t pc = (uint64_t)m1 * I0 + (uint32_t)pb;
  const uint32_t q2 = (uint32_t)(pb >> 32) + (uint32_t)(pc >> 32) + m0 * I2 + m1 * I1 + m2 * I0;
  // Q = q' - 2^72
  Q.lo = ((uint64_t)(uint32_t)pc << 32) | (uint32_t)pa;
  Q.hi = (int32_t)(q2 - (1u << 8));
  T = ((uint64_t)((rem << 8) | (c1 & 0xFFu)) << 32) | c0;
}

// t = q r + rho for a lazy digit, |t| < 2^84.  Non-SPLIT shapes: q = t >> W
// and rho = t - q r, true value in (-2^57, 2^W + 2^57).  SPLIT: exact,
// 0 <= rho < r (r = 2^56 65: t_h = t >> 56 has |t_h| < 2^28 and floor(n / 65)
// for n < 2^31 is n ceil(2^38 / 65) >> 38).
template <int KD, int W, int U>
__device__ __forceinline__ void qr_split(L96 t, int64_t& q, uint64_t& rho) {
  typedef Field<KD, W, U> F;
  if constexpr (F::NEG) {
    // t_h = t >> 40, |t_h| < 2^44; n = t_h + d 2^22 in [0, 2^46) = a 2^23 + b,
    // n = a d + (a + b) and a + b < 2^24 < 3 d
    const int64_t th = ((int64_t)t.hi << 24) + (int64_t)(t.lo >> 40);
    constexpr uint64_t D = (1ull << 23) - 1;
    const uint64_t n = (uint64_t)(th + (int64_t)(D << 22));
    const uint64_t a = n >> 23, c = a + (n & D);
    const uint64_t e = (uint64_t)(c >= D) + (uint64_t)(c >= 2 * D);
    q = (int64_t)(a + e) - (1ll << 22);
    rho = ((c - e * D) << 40) | (t.lo & ((1ull << 40) - 1));
  } else if constexpr (F::SPLIT) {
    const int32_t th = (int32_t)(((uint32_t)t.hi << 8) | (uint32_t)(t.lo >> 56));
    const uint32_t n = (uint32_t)(th + (65 << 23));
    const uint32_t qp = (uint32_t)(((uint64_t)n * 4228890877u) >> 38);
    const uint32_t rem = n - 65u * qp;
    q = (int64_t)(int32_t)qp - (1 << 23);
    rho = ((uint64_t)rem << 56) | (t.lo & ((1ull << 56) - 1));
  } else {
    q = ((int64_t)t.hi << (64 - W)) | (int64_t)(t.lo >> W);  // floor(t / 2^W)
    rho = (t.lo & ((1ull << W) - 1)) - ((uint64_t)q << U);
  }
}

// Limb form of y: yl[3t + c] = limb c of y_t.
template <int KD>
struct YLimbs {
  uint32_t l[3 * KD];
};

__device__ __forceinline__ void split22(uint64_t y, uint32_t& a, uint32_t& b, uint32_t& c) {
  a = (uint32_t)y & 0x3FFFFFu;
  b = (uint32_t)(y >> 22) & 0x3FFFFFu;
  c = (uint32_t)(y >> 44);
}

// Lane m's share of x * r^rot: which digit of x it starts with and whether
// that digit is complemented; the correction sum is the suffix sum of y from
// src + 1, or its complement in the total when `flip`.
template <int KD>
struct RotLane {
  int src;        // digit of x loaded into lane m: (m - rot) mod k
  uint32_t mask;  // all ones when the digit enters negated
  bool flip;      // same condition: S = total - suffix(src + 1)
};
template <int KD>
__device__ __forceinline__ RotLane<KD> rot_lane(int rot, int m) {
  const int rp = rot & (KD - 1);
  const bool neg = (m < rp) != ((rot & KD) != 0);
  RotLane<KD> r;
  r.src = (m - rp) & (KD - 1);
  r.mask = neg ? 0xFFFFFFFFu : 0u;
  r.flip = neg;
  return r;
}

// T + Q_{m-1} in lane m and T - Q_{k-1} in lane 0 (r^k = -1).  With LN the
// negation is ~Q + 1: the complement rides on the rotation (one DPP xor per
// word) and the +1 enters as the carry into the low word.
template <int KD, bool LN = Geo<KD>::LEAN>
__device__ __forceinline__ L96 add_carried_q(L96 T, L96 Q, int m) {
  if constexpr (LN) {
    const uint32_t wrap = (m == 0) ? 0xFFFFFFFFu : 0u;
    const uint32_t q0 = dig_rot<KD, 1>((uint32_t)Q.lo) ^ wrap;
    const uint32_t q1 = dig_rot<KD, 1>((uint32_t)(Q.lo >> 32)) ^ wrap;
    const uint32_t q2 = dig_rot<KD, 1>((uint32_t)Q.hi) ^ wrap;
    unsigned c;
    const uint32_t o0 = __builtin_addc((uint32_t)T.lo, q0, (unsigned)(m == 0), &c);
    const uint32_t o1 = __builtin_addc((uint32_t)(T.lo >> 32), q1, c, &c);
    const uint32_t o2 = (uint32_t)T.hi + q2 + c;
    return L96{((uint64_t)o1 << 32) | o0, (int32_t)o2};
  } else {
    const L96 nq = l96_sub(L96{0, 0}, Q);
    return l96_add(T, l96_rot<KD, 1>((m == KD - 1) ? nq : Q));
  }
}

// Column C = (l0, l1, h0, h1, h2) (signed 160-bit, h2 the top word) of lane
// m as C = Q r + T; returns the lazy digit T_m + Q_{m-1} (lane 0 takes
// -Q_{k-1}, since r^k = -1).
template <int KD, int W, int U, bool LN = Geo<KD>::LEAN>
__device__ __forceinline__ L96 column_tail(uint32_t l0, uint32_t l1, uint32_t h0, uint32_t h1, uint32_t h2, int m) {
  typedef Field<KD, W, U> F;
  if constexpr (F::SPLIT) {
    uint64_t T;
    L96 Qs;
    if constexpr (F::NEG) {
      split_qr160_m23(l0, l1, h0, h1, h2, T, Qs);
    } else {
      split_qr160(l0, l1, h0, h1, h2, T, Qs);
    }
    return add_carried_q<KD, LN>(l96(T), Qs, m);
  } else {
  constexpr int SA = F::SA, SB = F::SB;
  unsigned cy;
  // fold 1 (2^64 = a r - b): C = a H r + V, V = L - b H; keep V's low 64
  // bits (v0w, v1w) and Vh = V >> 64 (|Vh| < 2^45)
  uint32_t v0w, v1w, v2w, v3w;
  sub_shifted96<SB>(l0, l1, h0, h1, h2, v0w, v1w, v2w, v3w);
  // fold 2: V = a Vh r + W, W = Vl - b Vh; Wh = W >> 64 (|Wh| < 2^20)
  uint32_t w0w, w1w, w2w;
  sub_shifted64<SB>(v0w, v1w, v2w, v3w, w0w, w1w, w2w);
  // fold 3: T = Wl - b Wh, |T| < 2^65
  L96 Tm = sub_shifted32<SB>(w0w, w1w, w2w);
  // Q = a (H + Vh + Wh)
  const uint32_t vs = (uint32_t)((int32_t)v3w >> 31), ws = (uint32_t)((int32_t)w2w >> 31);
  uint32_t g0 = __builtin_addc(h0, v2w, 0u, &cy);
  uint32_t g1 = __builtin_addc(h1, v3w, cy, &cy);
  uint32_t g2 = h2 + vs + cy;
  g0 = __builtin_addc(g0, w2w, 0u, &cy);
  g1 = __builtin_addc(g1, ws, cy, &cy);
  g2 = g2 + ws + cy;
  L96 Q;
  Q.lo = ((uint64_t)g1 << 32 | g0) << SA;
  Q.hi = (int32_t)((g2 << SA) | (g1 >> (32 - SA)));
  return add_carried_q<KD, LN>(Tm, Q, m);
  }
}

// Core.  (v0, v1): the lane's starting x digit (rotated, complemented).
// yl(t, y0, y1, y2): the three limbs of y_t (t a compile-time constant for
// k <= 32, an int for k = 64).
// (s0, s1, s2): the correction sum S_m as three 32-bit words.
// Returns the lazy product digit T_m + Q_{m-1}.
template <int KD, int W, int U, bool LN = Geo<KD>::LEAN, class YL>
__device__ __forceinline__ L96 mul_core_y(uint32_t v0, uint32_t v1, YL&& yl, uint32_t s0, uint32_t s1, uint32_t s2,
                                          int m) {
  const uint32_t wrap = (m == 0) ? 0xFFFFFFFFu : 0u;
  uint64_t a00 = 0, a01 = 0, a02 = 0, a10 = 0, a11 = 0, a12 = 0;
  if constexpr (KD == 64) {
    // a run-time loop (yl takes a run-time t): 64 unrolled steps in every
    // product of a kernel make the code too large
#pragma unroll 4
    for (int t = 0; t < KD; ++t) {
      uint32_t y0, y1, y2;
      yl(t, y0, y1, y2);
      a00 += (uint64_t)v0 * y0;
      a01 += (uint64_t)v0 * y1;
      a02 += (uint64_t)v0 * y2;
      a10 += (uint64_t)v1 * y0;
      a11 += (uint64_t)v1 * y1;
      a12 += (uint64_t)v1 * y2;
      v0 = dig_rot<KD, 1>(v0) ^ wrap;
      v1 = dig_rot<KD, 1>(v1) ^ wrap;
    }
  } else {
    static_for<KD>([&](auto T) {
      constexpr int t = decltype(T)::value;
      uint32_t y0, y1, y2;
      yl(T, y0, y1, y2);
      a00 += (uint64_t)v0 * y0;
      a01 += (uint64_t)v0 * y1;
      a02 += (uint64_t)v0 * y2;
      a10 += (uint64_t)v1 * y0;
      a11 += (uint64_t)v1 * y1;
      a12 += (uint64_t)v1 * y2;
      if constexpr (t + 1 < KD) {
        v0 = dig_rot<KD, 1>(v0) ^ wrap;
        v1 = dig_rot<KD, 1>(v1) ^ wrap;
      }
    });
  }
  // Cells at 32-bit positions, C = c0 + c1 2^32 + c2 2^64 + c3 2^96 - S 2^64:
  // the accumulators sit at bit 0, 22, 44 (v0 limb) and 32, 54, 76 (v1 limb);
  // + S enters c0..c2.  Every shifted add is one v_mad_u64_u32 with a
  // power-of-two multiplier held in an SGPR.  c0, c1 < 2^59, c2 < 2^49,
  // c3 < 2^38.
  constexpr bool LEAN = LN;
  const uint32_t K22 = sgpr_const(1u << 22), K12 = sgpr_const(1u << 12), ONE = sgpr_const(1u);
  uint64_t c0 = mad32(lo32(a01), LEAN ? sgpr_const_n<0>(1u << 22) : K22, a00);
  c0 = mad32(s0, ONE, c0);
  uint64_t c1 = mad32(hi32(a01), LEAN ? sgpr_const_n<1>(1u << 22) : K22, a10);
  c1 = mad32(lo32(a02), LEAN ? sgpr_const_n<2>(1u << 12) : K12, c1);
  c1 = mad32(lo32(a11), LEAN ? sgpr_const_n<3>(1u << 22) : K22, c1);
  c1 = mad32(s1, ONE, c1);
  uint64_t c2 = mad32(hi32(a02), LEAN ? sgpr_const_n<4>(1u << 12) : K12, (uint64_t)s2);
  c2 = mad32(hi32(a11), LEAN ? sgpr_const_n<5>(1u << 22) : K22, c2);
  c2 = mad32(lo32(a12), LEAN ? sgpr_const_n<6>(1u << 12) : K12, c2);
  const uint64_t c3 = mad32(hi32(a12), LEAN ? sgpr_const_n<7>(1u << 12) : K12, 0ull);
  // C = L + H 2^64, L = (l0, l1), H = (h0, h1, h2) signed 96-bit, |H| < 2^71
  unsigned cy;
  const uint32_t l0 = lo32(c0);
  const uint32_t l1 = __builtin_addc(hi32(c0), lo32(c1), 0u, &cy);
  uint32_t h0 = __builtin_addc(lo32(c2), hi32(c1), cy, &cy);
  uint32_t h1 = __builtin_addc(hi32(c2), lo32(c3), cy, &cy);
  uint32_t h2 = hi32(c3) + cy;
  h0 = __builtin_subc(h0, s0, 0u, &cy);
  h1 = __builtin_subc(h1, s1, cy, &cy);
  h2 = h2 - s2 - cy;
  return column_tail<KD, W, U, LN>(l0, l1, h0, h1, h2, m);
}

template <int KD, int W, int U, bool LN = Geo<KD>::LEAN>
__device__ __forceinline__ L96 mul_core(uint32_t v0, uint32_t v1, const YLimbs<KD>& y, uint32_t s0, uint32_t s1,
                                        uint32_t s2, int m) {
  return mul_core_y<KD, W, U, LN>(
      v0, v1,
      [&](auto T, uint32_t& y0, uint32_t& y1, uint32_t& y2) {
        constexpr int t = decltype(T)::value;
        y0 = y.l[3 * t];
        y1 = y.l[3 * t + 1];
        y2 = y.l[3 * t + 2];
      },
      s0, s1, s2, m);
}

// Twiddle entry layout (u32 words): 3k limbs of the digits, then for
// i = 0..k the suffix sum sum_{t >= i} y_t as (lo, mid, hi) words
// (suffix(k) = 0), padded to a multiple of 4 words.
template <int KD>
struct TwLayout {
  static constexpr int LIMBS = 0;
  static constexpr int SUF = 3 * KD;
  static constexpr int WORDS = (6 * KD + 3 + 3) & ~3;
};

// S_m for lane m from a table entry: suffix(src + 1), or total - it.
template <int KD>
__device__ __forceinline__ void tw_correction(const uint32_t* __restrict__ tw, const RotLane<KD>& rl, uint32_t& s0,
                                              uint32_t& s1, uint32_t& s2) {
  const uint32_t* suf = tw + TwLayout<KD>::SUF;
  const int i = rl.src + 1;
  const uint64_t a = (uint64_t)suf[3 * i] | ((uint64_t)suf[3 * i + 1] << 32);
  const uint32_t ah = suf[3 * i + 2];
  const uint64_t t = (uint64_t)suf[0] | ((uint64_t)suf[1] << 32);
  const uint32_t th = suf[2];
  const uint64_t d = t - a;
  const uint32_t dh = th - ah - (uint32_t)(t < a);
  const uint64_t sl = rl.flip ? d : a;
  s0 = (uint32_t)sl;
  s1 = (uint32_t)(sl >> 32);
  s2 = rl.flip ? dh : ah;
}

template <int KD>
__device__ __forceinline__ void tw_limbs(const uint32_t* __restrict__ tw, YLimbs<KD>& y) {
  const uint4* lp = reinterpret_cast<const uint4*>(tw + TwLayout<KD>::LIMBS);
  static_for<3 * KD / 4>([&](auto I) {
    constexpr int i = decltype(I)::value;
    const uint4 q = lp[i];
    y.l[4 * i] = q.x;
    y.l[4 * i + 1] = q.y;
    y.l[4 * i + 2] = q.z;
    y.l[4 * i + 3] = q.w;
  });
}

// Keeps the loads of one slot's product from being hoisted above the
// previous slot's work (which only raises register pressure).
__device__ __forceinline__ void slot_fence() { asm volatile("" ::: "memory"); }

// k = 64: x * (table entry tw) for the lane's prepared x digit (v0, v1) and
// correction words.  An element is a whole wavefront, so the entry is
// wavefront-uniform; its 192 limbs are streamed through the column loop
// instead of held in registers.
template <int KD, int W, int U>
__device__ __forceinline__ L96 mul_tw_stream(uint32_t v0, uint32_t v1, const uint32_t* __restrict__ tw, uint32_t s0,
                                             uint32_t s1, uint32_t s2, int m) {
  return mul_core_y<KD, W, U>(
      v0, v1,
      [&](int t, uint32_t& y0, uint32_t& y1, uint32_t& y2) {
        y0 = tw[TwLayout<KD>::LIMBS + 3 * t];
        y1 = tw[TwLayout<KD>::LIMBS + 3 * t + 1];
        y2 = tw[TwLayout<KD>::LIMBS + 3 * t + 2];
      },
      s0, s1, s2, m);
}

// x * tw * r^rot where lane m already holds digit rl.src of x (xs).
template <int KD, int W, int U, bool LN = Geo<KD>::LEAN>
__device__ __forceinline__ L96 mul_twiddle_pre(uint64_t xs, const uint32_t* __restrict__ tw, const RotLane<KD>& rl,
                                               int m) {
  if constexpr (KD == 64) {
    uint32_t s0, s1, s2;
    tw_correction<KD>(tw, rl, s0, s1, s2);
    return mul_tw_stream<KD, W, U>((uint32_t)xs ^ rl.mask, (uint32_t)(xs >> 32) ^ rl.mask, tw, s0, s1, s2, m);
  } else {
    YLimbs<KD> y;
    tw_limbs<KD>(tw, y);
    uint32_t s0, s1, s2;
    tw_correction<KD>(tw, rl, s0, s1, s2);
    return mul_core<KD, W, U, LN>((uint32_t)xs ^ rl.mask, (uint32_t)(xs >> 32) ^ rl.mask, y, s0, s1, s2, m);
  }
}

// x * tw * r^rot where lane m holds digit m of x (the digit is fetched from
// the lane holding digit (m - rot) mod k with a cross-lane permute).
template <int KD, int W, int U, bool LN = Geo<KD>::LEAN>
__device__ __forceinline__ L96 mul_twiddle(uint64_t x, const uint32_t* __restrict__ tw, int rot, int l, int m) {
  const RotLane<KD> rl = rot_lane<KD>(rot, m);
  const int src = Geo<KD>::lane_of(l, rl.src);
  const uint32_t x0 = (uint32_t)__shfl((int)(uint32_t)x, src, 64);
  const uint32_t x1 = (uint32_t)__shfl((int)(uint32_t)(x >> 32), src, 64);
  return mul_twiddle_pre<KD, W, U, LN>(((uint64_t)x1 << 32) | x0, tw, rl, m);
}

// Same with a wavefront-uniform twiddle entry and rotation: the limbs are
// read with scalar loads (uniform address, read-only table) and stay in
// SGPRs; only the per-lane correction sum is a vector load.
template <int KD, int W, int U, bool LN = Geo<KD>::LEAN>
__device__ __forceinline__ L96 mul_twiddle_uniform(uint64_t x, const uint32_t* __restrict__ tw, int rot, int l,
                                                   int m) {
  const RotLane<KD> rl = rot_lane<KD>(rot, m);
  const int src = Geo<KD>::lane_of(l, rl.src);
  const uint32_t x0 = (uint32_t)__shfl((int)(uint32_t)x, src, 64) ^ rl.mask;
  const uint32_t x1 = (uint32_t)__shfl((int)(uint32_t)(x >> 32), src, 64) ^ rl.mask;
  if constexpr (KD == 64) {
    uint32_t s0, s1, s2;
    tw_correction<KD>(tw, rl, s0, s1, s2);
    return mul_tw_stream<KD, W, U>(x0, x1, tw, s0, s1, s2, m);
  } else {
    YLimbs<KD> y;
    static_for<3 * KD>([&](auto I) {
      constexpr int i = decltype(I)::value;
      y.l[i] = tw[TwLayout<KD>::LIMBS + i];
    });
    uint32_t s0, s1, s2;
    tw_correction<KD>(tw, rl, s0, s1, s2);
    return mul_core<KD, W, U, LN>(x0, x1, y, s0, s1, s2, m);
  }
}

// x * tw where lane m holds digit m of x (no rotation) and the table entry
// is wavefront-uniform: limbs through scalar loads, the lane's correction sum
// S_m = suffix(m + 1) through one vector load at a fixed per-lane offset.
template <int KD, int W, int U, bool LN = Geo<KD>::LEAN>
__device__ __forceinline__ L96 mul_entry_uniform(uint64_t x, const uint32_t* __restrict__ tw, int m) {
  slot_fence();
  if constexpr (KD == 64) {
    const uint32_t* suf = tw + TwLayout<KD>::SUF + 3 * (m + 1);
    return mul_tw_stream<KD, W, U>((uint32_t)x, (uint32_t)(x >> 32), tw, suf[0], suf[1], suf[2], m);
  } else {
    YLimbs<KD> y;
    static_for<3 * KD>([&](auto I) {
      constexpr int i = decltype(I)::value;
      y.l[i] = tw[TwLayout<KD>::LIMBS + i];
    });
    const uint32_t* suf = tw + TwLayout<KD>::SUF + 3 * (m + 1);
    return mul_core<KD, W, U, LN>((uint32_t)x, (uint32_t)(x >> 32), y, suf[0], suf[1], suf[2], m);
  }
}

// The same with a per-group entry (vector loads of the limbs).
template <int KD, int W, int U, bool LN = Geo<KD>::LEAN>
__device__ __forceinline__ L96 mul_entry(uint64_t x, const uint32_t* __restrict__ tw, int m) {
  slot_fence();
  if constexpr (KD == 64) {
    const uint32_t* suf = tw + TwLayout<KD>::SUF + 3 * (m + 1);
    return mul_tw_stream<KD, W, U>((uint32_t)x, (uint32_t)(x >> 32), tw, suf[0], suf[1], suf[2], m);
  } else {
    YLimbs<KD> y;
    tw_limbs<KD>(tw, y);
    const uint32_t* suf = tw + TwLayout<KD>::SUF + 3 * (m + 1);
    return mul_core<KD, W, U, LN>((uint32_t)x, (uint32_t)(x >> 32), y, suf[0], suf[1], suf[2], m);
  }
}

// ------------------------------------------------------------------------
// Per-group twiddles staged through LDS (k <= 16)
// ------------------------------------------------------------------------
// Where the groups of a wavefront take different twiddles (the last pass,
// the second pass of a fused pair), the product needs the whole entry of
// its group's twiddle in each of the group's k lanes.  Instead of every lane
// fetching the whole entry from memory (k times the bytes through the vector
// memory unit), lane m loads only digit m from a table of raw digits (one
// 8k-byte segment per group), splits it into limbs, forms the suffix sum
// sum_{t >= m} y_t by a scan across the element's lanes and writes both into
// its group's entry of a small LDS area in the twiddle-entry layout; the
// product then reads the entry from LDS (the group's lanes read the same
// words).  LDS operations of one wavefront take effect in issue order, so a
// group's own lanes see the entry right after the writes; the fences keep the
// compiler from moving the LDS accesses of consecutive slots across each
// other.

// Value of the lane holding digit m + D of the same element, 0 past digit
// k - 1 (a DPP row shift with zero fill; k <= 16).
template <int KD, int D>
__device__ __forceinline__ uint32_t dig_up(uint32_t v) {
  static_assert(Geo<KD>::ROW, "elements inside one DPP row");
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x100 + D * Geo<KD>::GPL, 0xF, 0xF, true);
}

// Words of the LDS staging area of one wavefront: one entry per group.
template <int KD>
struct StageGeo {
  static constexpr int WORDS = TwLayout<KD>::WORDS;
  static constexpr int PER_WAVE = Geo<KD>::G * WORDS;
};

// Once per kernel: suffix(k) = 0 in the group's entry (never written again).
template <int KD>
__device__ __forceinline__ void stage_init(uint32_t* __restrict__ e, int m) {
  if (m == KD - 1) {
    uint32_t* z = e + TwLayout<KD>::SUF + 3 * KD;
    z[0] = 0u;
    z[1] = 0u;
    z[2] = 0u;
  }
}

// Lane m holds y = digit m of its group's twiddle; writes the group's entry e.
template <int KD>
__device__ __forceinline__ void stage_entry(uint64_t y, uint32_t* __restrict__ e, int m) {
  uint32_t l0, l1, l2;
  split22(y, l0, l1, l2);
  // inclusive suffix sum sum_{t >= m} y_t (< 2^68) by doubling steps
  uint32_t s0 = (uint32_t)y, s1 = (uint32_t)(y >> 32), s2 = 0u;
  static_for<ilog2(KD)>([&](auto I) {
    constexpr int d = 1 << decltype(I)::value;
    const uint32_t n0 = dig_up<KD, d>(s0), n1 = dig_up<KD, d>(s1), n2 = dig_up<KD, d>(s2);
    unsigned c;
    s0 = __builtin_addc(s0, n0, 0u, &c);
    s1 = __builtin_addc(s1, n1, c, &c);
    s2 = s2 + n2 + c;
  });
  slot_fence();
  e[3 * m] = l0;
  e[3 * m + 1] = l1;
  e[3 * m + 2] = l2;
  uint32_t* suf = e + TwLayout<KD>::SUF + 3 * m;
  suf[0] = s0;
  suf[1] = s1;
  suf[2] = s2;
  slot_fence();
}

// x * y for two data elements: every lane of the element loads all of y's
// digits (same addresses across the element's lanes) and derives the limbs
// and its correction sum (rot = 0: S_m = sum_{t > m} y_t).
template <int KD, int W, int U>
__device__ __forceinline__ L96 mul_data(uint64_t x, const uint64_t (&yd)[KD], int m) {
  YLimbs<KD> y;
  uint64_t sl = 0;
  uint32_t sh = 0;
  static_for<KD>([&](auto T) {
    constexpr int t = decltype(T)::value;
    split22(yd[t], y.l[3 * t], y.l[3 * t + 1], y.l[3 * t + 2]);
    const uint64_t add = (t > m) ? yd[t] : 0ull;
    sl += add;
    sh += (uint32_t)(sl < add);
  });
  return mul_core<KD, W, U>((uint32_t)x, (uint32_t)(x >> 32), y, (uint32_t)sl, (uint32_t)(sl >> 32), sh, m);
}

// x * y for a data element whose digit t is y[t ys].  k <= 32 as mul_data.
// k = 64 (the element is the wavefront, so y's address is uniform): the
// digits are streamed and split as they are used, and S_m = total - (y_0 +
// ... + y_m) comes from an inclusive scan of the lanes' own digits.
template <int KD, int W, int U>
__device__ __forceinline__ L96 mul_data_ptr(uint64_t x, const uint64_t* __restrict__ y, uint64_t ys, int l, int m) {
  if constexpr (KD == 64) {
    uint64_t pl = y[(uint64_t)m * ys];
    uint32_t ph = 0;
    static_for<6>([&](auto I) {
      constexpr int d = 1 << decltype(I)::value;
      const uint32_t a0 = (uint32_t)__shfl_up((int)(uint32_t)pl, d, 64);
      const uint32_t a1 = (uint32_t)__shfl_up((int)(uint32_t)(pl >> 32), d, 64);
      const uint32_t a2 = (uint32_t)__shfl_up((int)ph, d, 64);
      if (m >= d) {
        const uint64_t add = ((uint64_t)a1 << 32) | a0;
        pl += add;
        ph += a2 + (uint32_t)(pl < add);
      }
    });
    const uint64_t tl = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(pl >> 32), 63, 64) << 32) |
                        (uint32_t)__shfl((int)(uint32_t)pl, 63, 64);
    const uint32_t th = (uint32_t)__shfl((int)ph, 63, 64);
    const uint64_t sl = tl - pl;
    const uint32_t sh = th - ph - (uint32_t)(tl < pl);
    (void)l;
    return mul_core_y<KD, W, U>(
        (uint32_t)x, (uint32_t)(x >> 32),
        [&](int t, uint32_t& y0, uint32_t& y1, uint32_t& y2) { split22(y[(uint64_t)t * ys], y0, y1, y2); },
        (uint32_t)sl, (uint32_t)(sl >> 32), sh, m);
  } else {
    (void)l;
    uint64_t yd[KD];
    static_for<KD>([&](auto T) {
      constexpr int t = decltype(T)::value;
      yd[t] = y[(uint64_t)t * ys];
    });
    return mul_data<KD, W, U>(x, yd, m);
  }
}

// ------------------------------------------------------------------------
// The FFT-based element product (section 3.3)
// ------------------------------------------------------------------------
// x y mod p through the negacyclic convolution of the digit vectors: for
// each of three word primes q (q < 2^62, 2k | q - 1) the columns u_m mod q
// are A' InverseDFT(DFT(A x) DFT(A y)) with A = (1, theta, ..., theta^(k-1)),
// theta a primitive 2k-th root mod q (the negacyclic convolution algorithm of
// section 3.3); the three residues give u_m exactly by the CRT (|u_m| <
// k 2^128 < q1 q2 q3 / 2, so three primes where the paper's two 61-bit primes
// bound k r^2 below 2^121), and u_m goes through the same fold into radix r
// as the schoolbook columns.  One lane per coefficient: the length-k DFTs
// are radix-2 butterflies between lanes (decimation in frequency forward,
// bit-reversed spectrum, decimation in time back).  Arithmetic mod q is
// Montgomery with 2^64; table constants are stored in Montgomery form.
//
// Table (u64 words, built on the host per field and device):
//   [0..2] q_i, [3..5] -q_i^-1 mod 2^64, [6] q1^-1 mod q2, [7] q1 mod q3,
//   [8] (q1 q2)^-1 mod q3 (the three in Montgomery form), [9..10] q1 q2,
//   [11..13] Q = q1 q2 q3, [14..16] (Q - 1) / 2, then per prime i at
//   NTT_HEAD + 3k i: theta^m (k), theta^-m k^-1 2^64 (k), w^j and w^-j
//   (k / 2 each), w = theta^2.
constexpr int NTT_HEAD = 20;

__device__ __forceinline__ uint64_t mont_mul(uint64_t a, uint64_t b, uint64_t q, uint64_t qn) {
  // a b < q 2^64; returns a b 2^-64 mod q in [0, q)
  const u128 t = (u128)a * b;
  const uint64_t mm = (uint64_t)t * qn;
  const u128 u = t + (u128)mm * q;  // < 2^65 q < 2^127, low 64 bits zero
  const uint64_t r = (uint64_t)(u >> 64);
  return r >= q ? r - q : r;
}
__device__ __forceinline__ uint64_t add_q(uint64_t a, uint64_t b, uint64_t q) {
  const uint64_t s = a + b;
  return s >= q ? s - q : s;
}
__device__ __forceinline__ uint64_t sub_q(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }

template <int KD>
__device__ __forceinline__ uint64_t lane_xchg(uint64_t v, int src) {
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, 64);
  const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, 64);
  return ((uint64_t)hi << 32) | lo;
}

// Forward length-k DFT across the element's lanes modulo q (decimation in
// frequency, natural order in, bit-reversed out): lane m holds v_m < q.
// Halves k/2, ..., 1: the upper lane of a pair takes (a - b) w^(j k / (2h)),
// the lower a + b.
template <int KD>
__device__ __forceinline__ uint64_t ntt_fwd_lanes(uint64_t v, const uint64_t* __restrict__ b, uint64_t q, uint64_t qn,
                                                  int l, int m) {
  constexpr int LK = ilog2(KD);
  static_for<LK>([&](auto S) {
    constexpr int h = KD >> (decltype(S)::value + 1);
    const int src = Geo<KD>::lane_of(l, m ^ h);
    const bool up = (m & h) != 0;
    const uint64_t w = b[2 * KD + (m & (h - 1)) * (KD / (2 * h))];
    const uint64_t pv = lane_xchg<KD>(v, src);
    v = up ? mont_mul(sub_q(pv, v, q), w, q, qn) : add_q(v, pv, q);
  });
  return v;
}

// The inverse (decimation in time, bit-reversed in, natural out, without
// the factor 1/k): halves 1, ..., k/2; the upper lane first takes b w^-j.
template <int KD>
__device__ __forceinline__ uint64_t ntt_inv_lanes(uint64_t v, const uint64_t* __restrict__ b, uint64_t q, uint64_t qn,
                                                  int l, int m) {
  constexpr int LK = ilog2(KD);
  static_for<LK>([&](auto S) {
    constexpr int h = 1 << decltype(S)::value;
    const int src = Geo<KD>::lane_of(l, m ^ h);
    const bool up = (m & h) != 0;
    const uint64_t w = b[2 * KD + KD / 2 + (m & (h - 1)) * (KD / (2 * h))];
    const uint64_t bw = up ? mont_mul(v, w, q, qn) : v;
    const uint64_t pv = lane_xchg<KD>(bw, src);
    v = up ? sub_q(pv, bw, q) : add_q(bw, pv, q);
  });
  return v;
}

// Column u_m from its three residues (Garner's CRT into (-Q/2, Q/2]), then
// the schoolbook product's fold into the lazy digit T_m + Q_{m-1}.
template <int KD, int W, int U>
__device__ __forceinline__ L96 ntt_crt_tail(const uint64_t (&u)[3], const uint64_t* __restrict__ tb, int m) {
  // CRT (Garner): u = v1 + q1 v2 + q1 q2 v3, then into (-Q/2, Q/2]
  const uint64_t q1 = tb[0], q2 = tb[1], q3 = tb[2];
  const uint64_t v1 = u[0];
  const uint64_t v1b = v1 >= q2 ? v1 - q2 : v1;
  const uint64_t v2 = mont_mul(sub_q(u[1], v1b, q2), tb[6], q2, tb[4]);
  const uint64_t v1c = v1 >= q3 ? v1 - q3 : v1;
  const uint64_t t3 = sub_q(sub_q(u[2], v1c, q3), mont_mul(v2, tb[7], q3, tb[5]), q3);
  const uint64_t v3 = mont_mul(t3, tb[8], q3, tb[5]);
  const u128 a = (u128)q1 * v2 + v1;                  // < 2^125
  const u128 blo = (u128)tb[9] * v3, bhi = (u128)tb[10] * v3;
  const u128 w0 = (u128)(uint64_t)a + (uint64_t)blo;
  const u128 w1 = (a >> 64) + (blo >> 64) + (uint64_t)bhi + (w0 >> 64);
  const uint64_t z0 = (uint64_t)w0, z1 = (uint64_t)w1;
  const uint64_t z2 = (uint64_t)(bhi >> 64) + (uint64_t)(w1 >> 64);
  // z > (Q - 1) / 2 ?  then z - Q (two's complement; the true value fits)
  const bool big = (z2 != tb[16]) ? (z2 > tb[16]) : (z1 != tb[15]) ? (z1 > tb[15]) : (z0 > tb[14]);
  uint64_t c0 = z0, c1 = z1, c2 = z2;
  if (big) {
    const u128 d0 = (u128)z0 - tb[11];
    const u128 d1 = (u128)z1 - tb[12] - (uint64_t)((d0 >> 64) != 0);
    c0 = (uint64_t)d0;
    c1 = (uint64_t)d1;
    c2 = z2 - tb[13] - (uint64_t)((d1 >> 64) != 0);
  }
  return column_tail<KD, W, U>((uint32_t)c0, (uint32_t)(c0 >> 32), (uint32_t)c1, (uint32_t)(c1 >> 32),
                               (uint32_t)c2, m);
}

template <int KD, int W, int U>
__device__ __forceinline__ L96 mul_ntt(uint64_t x, uint64_t y, const uint64_t* __restrict__ tb, int l, int m) {
  uint64_t u[3];
  static_for<3>([&](auto I) {
    constexpr int i = decltype(I)::value;
    const uint64_t q = tb[i], qn = tb[3 + i];
    const uint64_t* b = tb + NTT_HEAD + 3 * KD * i;
    // A x, A y (x, y < 2^64 and theta^m < q: the products stay below q 2^64)
    const uint64_t xv = ntt_fwd_lanes<KD>(mont_mul(x, b[m], q, qn), b, q, qn, l, m);
    const uint64_t yv = ntt_fwd_lanes<KD>(mont_mul(y, b[m], q, qn), b, q, qn, l, m);
    const uint64_t uv = ntt_inv_lanes<KD>(mont_mul(xv, yv, q, qn), b, q, qn, l, m);  // carries 2^-64
    // theta^-m / k, and the 2^64 of the pointwise product
    u[i] = mont_mul(uv, b[KD + m], q, qn);
  });
  return ntt_crt_tail<KD, W, U>(u, tb, m);
}

// The FFT-based product as a twiddle multiplier: x r^rot times a constant y
// whose three transforms are tabulated (spec[i k + m]: lane m's value of the
// forward transform of A y modulo prime i, as ntt_fwd_lanes leaves it), so
// only x is transformed.  xs: the lane's digit of x r^rot before its sign
// (digit (m - rot) mod k of x), neg: that digit enters negated (r^k = -1).
template <int KD, int W, int U>
__device__ __forceinline__ L96 mul_ntt_spec(uint64_t xs, bool neg, const uint64_t* __restrict__ spec,
                                            const uint64_t* __restrict__ tb, int l, int m) {
  uint64_t u[3];
  static_for<3>([&](auto I) {
    constexpr int i = decltype(I)::value;
    const uint64_t q = tb[i], qn = tb[3 + i];
    const uint64_t* b = tb + NTT_HEAD + 3 * KD * i;
    uint64_t xv = mont_mul(xs, b[m], q, qn);
    if (neg) xv = xv ? q - xv : 0ull;
    xv = ntt_fwd_lanes<KD>(xv, b, q, qn, l, m);
    const uint64_t uv = ntt_inv_lanes<KD>(mont_mul(xv, spec[i * KD + m], q, qn), b, q, qn, l, m);
    u[i] = mont_mul(uv, b[KD + m], q, qn);
  });
  return ntt_crt_tail<KD, W, U>(u, tb, m);
}

// x w r^rot with w's transforms tabulated (spec) and x's digits in place:
// lane m fetches digit (m - rot) mod k of x from the lane holding it.
template <int KD, int W, int U>
__device__ __forceinline__ L96 mul_twiddle_ntt(uint64_t x, const uint64_t* __restrict__ spec,
                                               const uint64_t* __restrict__ tb, int rot, int l, int m) {
  const RotLane<KD> rl = rot_lane<KD>(rot, m);
  const uint64_t xs = lane_xchg<KD>(x, Geo<KD>::lane_of(l, rl.src));
  return mul_ntt_spec<KD, W, U>(xs, rl.flip, spec, tb, l, m);
}

// ------------------------------------------------------------------------
// Normalisation
// ------------------------------------------------------------------------
// Semi-normalise a lazy digit (|t| < 2^84): digit' = rho + q_{m-1} in
// [0, 2^64), where t = q r + rho with rho in [OFF, 2^W + 2 OFF) and q passed
// one lane up (lane 0 takes -q_{k-1}, since r^k = -1).
template <int KD, int W, int U>
__device__ __forceinline__ uint64_t seminorm(L96 t, int m) {
  typedef Field<KD, W, U> F;
  int64_t q;
  uint64_t rho;  // true value in (-OFF, 2^W + OFF)
  qr_split<KD, W, U>(t, q, rho);
  const bool low = (rho + F::OFF) < 3 * F::OFF;  // rho < 2 OFF
  rho += low ? F::R : 0ull;
  q -= low ? 1 : 0;
  int32_t qi = (int32_t)q;
  int32_t qin = (int32_t)dig_rot<KD, 1>((uint32_t)qi);
  qin = (m == 0) ? -qin : qin;
  return rho + (uint64_t)(int64_t)qin;
}

// Exact canonical form (section 2 encoding).  All lanes of the wavefront must
// call this together (wavefront-uniform loops).  Groups with active == false
// take part in the lane exchanges but their result is meaningless.
template <int KD, int W, int U>
__device__ __forceinline__ uint64_t canonicalize(L96 t, int l, int m) {
  typedef Field<KD, W, U> F;
  // exact t = q r + rho, 0 <= rho < r
  int64_t q;
  uint64_t rho;  // true value in (-2^57, 2^W + 2^57)
  qr_split<KD, W, U>(t, q, rho);
  if constexpr (!F::SPLIT) {
    const uint64_t off = 1ull << 57;
    if (rho + off < off) {  // rho < 0
      rho += F::R;
      q -= 1;
    } else if (rho + off >= F::R + off) {  // rho >= r
      rho -= F::R;
      q += 1;
    }
  }
  // v_m = rho_m + q_{m-1}; v_0 = rho_0 - q_{k-1}.  Now X = sum v_m r^m exactly.
  int32_t qi = (int32_t)q;
  int32_t qin = (int32_t)dig_rot<KD, 1>((uint32_t)qi);
  qin = (m == 0) ? -qin : qin;
  uint64_t v = rho + (uint64_t)(int64_t)qin;  // true value in (-2^27, r + 2^27)
  const uint64_t NEG = 0ull - (1ull << 28);
  int top = 0;  // sum of carries out of digit k-1 (used in lane k-1)
  // ripple without wrap until every digit is in [0, r)
  for (int it = 0; it <= KD + 1; ++it) {
    const bool isneg = v >= NEG;
    const bool isbig = !isneg && v >= F::R;
    const int c = isneg ? -1 : (isbig ? 1 : 0);
    if (!__any(c != 0)) break;
    v = v - (uint64_t)(int64_t)c * F::R;
    int cin = (int)dig_rot<KD, 1>((uint32_t)c);
    if (m == 0) cin = 0;
    if (m == KD - 1) top += c;
    v += (uint64_t)(int64_t)cin;
  }
  // value = D - top, D = sum v_m r^m in [0, r^k)
  top = __shfl(top, Geo<KD>::lane_of(l, KD - 1), 64);
  if (__any(top != 0)) {
    if (m == 0) v -= (uint64_t)(int64_t)top;
    int top2 = 0;
    for (int it = 0; it <= KD + 1; ++it) {
      const bool isneg = v >= NEG;
      const bool isbig = !isneg && v >= F::R;
      const int c = isneg ? -1 : (isbig ? 1 : 0);
      if (!__any(c != 0)) break;
      v = v - (uint64_t)(int64_t)c * F::R;
      int cin = (int)dig_rot<KD, 1>((uint32_t)c);
      if (m == 0) cin = 0;
      if (m == KD - 1) top2 += c;
      v += (uint64_t)(int64_t)cin;
    }
    top2 = __shfl(top2, Geo<KD>::lane_of(l, KD - 1), 64);
    if (top2 != 0) v = (m == KD - 1) ? F::R : 0ull;  // the value is -1 = p - 1 = r^k
  }
  return v;
}

}  // namespace gfpk

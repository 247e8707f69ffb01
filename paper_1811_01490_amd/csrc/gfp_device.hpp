// Device arithmetic for Z/pZ, p = r^k + 1, r = 2^W + 2^U, on gfx950.
//
// Lane layout ("digit lanes").  A wavefront of 64 lanes is 4 DPP rows of 16
// lanes.  An element's k digits live in k lanes of one row: lane-in-row
// d * GPL + s holds digit d of the row's element s, GPL = 16 / k elements per
// row.  So k = 8 interleaves two elements per row and k = 16 uses one row per
// element.  Multiplying by r^i (section 2.3: a cyclic shift of the digits with
// the wrapped digits negated, since r^k = -1) is then a DPP row rotation by
// i * GPL lanes plus a per-lane sign, with no data leaving the row.
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
  static_assert(KD == 8 || KD == 16, "k must be 8 or 16");
  static constexpr int GPL = 16 / KD;  // elements per DPP row
  static constexpr int G = 64 / KD;    // elements per wavefront
  static constexpr int KB = 2 * KD;    // base-case DFT size K = 2k
  __device__ static __forceinline__ int lane() { return (int)(threadIdx.x & 63); }
  __device__ static __forceinline__ int digit(int l) { return (l & 15) / GPL; }
  __device__ static __forceinline__ int group(int l) { return (l >> 4) * GPL + (l & 15) % GPL; }
  // lane holding digit d of the same element as lane l
  __device__ static __forceinline__ int lane_of(int l, int d) { return (l & 0x30) | (d * GPL) | ((l & 15) % GPL); }
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
template <int N>
__device__ __forceinline__ L96 l96_ror(L96 a) {
  uint32_t w0 = row_ror<N>((uint32_t)a.lo), w1 = row_ror<N>((uint32_t)(a.lo >> 32));
  uint32_t w2 = row_ror<N>((uint32_t)a.hi);
  return L96{((uint64_t)w1 << 32) | w0, (int32_t)w2};
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
// butterfly by swapping its two outputs in those lanes.
// ------------------------------------------------------------------------
template <int KD, bool INV, int EXP>
__device__ __forceinline__ void bfly(L96& a, L96& b, int m) {
  constexpr int GPL = Geo<KD>::GPL;
  if constexpr (EXP == 0) {
    L96 s = l96_add(a, b), d = l96_sub(a, b);
    a = s;
    b = d;
  } else {
    // forward: r^EXP = rotate by EXP, negate digits m < EXP.
    // inverse: r^-EXP = -r^(KD-EXP) = rotate by KD-EXP, negate digits m >= KD-EXP.
    constexpr int ROT = INV ? (KD - EXP) : EXP;
    L96 bp = l96_ror<ROT * GPL>(b);
    bool f = INV ? (m >= ROT) : (m < ROT);
    L96 s = l96_add(a, bp), d = l96_sub(a, bp);
    a = l96_sel(f, d, s);
    b = l96_sel(f, s, d);
  }
}

template <int KD, bool INV>
__device__ __forceinline__ void dft_base(L96 (&v)[2 * KD], int m) {
  constexpr int KB = 2 * KD;
  constexpr int LG = ilog2(KB);
  L96 a[KB];
  static_for<KB>([&](auto I) {
    constexpr int i = decltype(I)::value;
    a[i] = v[brev(i, LG)];
  });
  static_for<LG>([&](auto S) {
    constexpr int H = 1 << decltype(S)::value;  // half size of this level
    static_for<KB / 2>([&](auto B) {
      constexpr int blk = decltype(B)::value / H, j = decltype(B)::value % H;
      constexpr int i0 = blk * 2 * H + j;
      constexpr int e = j * (KB / (2 * H));  // exponent of r, 0 <= e < KD
      bfly<KD, INV, e>(a[i0], a[i0 + H], m);
    });
  });
  static_for<KB>([&](auto I) {
    constexpr int i = decltype(I)::value;
    v[i] = a[i];
  });
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
// section 4.1: w^(i N/K + j) = r^i w^j) is applied by first gathering
// x_{m - rho} into lane m with the same complement rule.
//
// x is split into two 32-bit limbs and each y_t into three limbs of 22, 22
// and 20 bits, so every limb product is < 2^54 and k of them fit in a 64-bit
// accumulator: six v_mad_u64_u32 per digit pair, no carries.
//
// The column value (|u_m| < k r^2 plus the correction) is then folded with
// 2^64 = a r - b (a = 2^(64-W), b = 2^(64-W+U)): u = Q r + T with T a lazy
// digit (|T| < 2^66) and Q carried to column m+1 (negated into column 0).
// ------------------------------------------------------------------------
template <int KD, int W, int U>
struct Field {
  static constexpr uint64_t R = (1ull << W) + (1ull << U);
  static constexpr int SA = 64 - W;      // 2^64 = 2^SA * r - 2^SB
  static constexpr int SB = 64 - W + U;
  static_assert(W >= 56 && W <= 63 && U >= 8 && U + 8 <= W, "unsupported radix shape");
};

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

// Core: V = (v0, v1) is the lane's starting (possibly complemented) x digit,
// already rotated by rho.  S = (s_lo, s_hi) the correction sum for this lane.
// Returns the lazy product digit T_m + Q_{m-1}.
template <int KD, int W, int U>
__device__ __forceinline__ L96 mul_core(uint32_t v0, uint32_t v1, const YLimbs<KD>& y, uint64_t s_lo, uint32_t s_hi,
                                        int m) {
  constexpr int GPL = Geo<KD>::GPL;
  typedef Field<KD, W, U> F;
  const uint32_t wrap = (m == 0) ? 0xFFFFFFFFu : 0u;
  uint64_t a00 = 0, a01 = 0, a02 = 0, a10 = 0, a11 = 0, a12 = 0;
  static_for<KD>([&](auto T) {
    constexpr int t = decltype(T)::value;
    const uint32_t y0 = y.l[3 * t], y1 = y.l[3 * t + 1], y2 = y.l[3 * t + 2];
    a00 += (uint64_t)v0 * y0;
    a01 += (uint64_t)v0 * y1;
    a02 += (uint64_t)v0 * y2;
    a10 += (uint64_t)v1 * y0;
    a11 += (uint64_t)v1 * y1;
    a12 += (uint64_t)v1 * y2;
    if constexpr (t + 1 < KD) {
      v0 = row_ror<GPL>(v0) ^ wrap;
      v1 = row_ror<GPL>(v1) ^ wrap;
    }
  });
  // P0 = sum v0*y, P1 = sum v1*y (each < 2^102); column = P0 + P1 2^32 + S - S 2^64.
  const u128 P0 = (u128)a00 + ((u128)a01 << 22) + ((u128)a02 << 44);
  const u128 P1 = (u128)a10 + ((u128)a11 << 22) + ((u128)a12 << 44);
  const u128 S = ((u128)s_hi << 64) | s_lo;
  const u128 T2 = P0 + S + ((u128)(uint32_t)P1 << 32);
  const uint64_t L = (uint64_t)T2;
  const i128 H = (i128)(T2 >> 64) + (i128)(P1 >> 32) - (i128)S;  // column = L + H 2^64
  // fold three times with 2^64 = 2^SA r - 2^SB
  const i128 V = (i128)L - (H << F::SB);
  const i128 Vh = V >> 64;
  const uint64_t Vl = (uint64_t)V;
  const i128 W1 = (i128)Vl - (Vh << F::SB);
  const i128 W1h = W1 >> 64;
  const uint64_t W1l = (uint64_t)W1;
  const i128 Tm = (i128)W1l - (W1h << F::SB);  // |Tm| < 2^65
  const i128 Q = (H + Vh + W1h) << F::SA;       // |Q| < 2^75
  // Q_{m-1} into lane m; lane 0 takes -Q_{k-1}
  L96 q = l96_from_i128(Q);
  L96 qin = l96_ror<GPL>(q);
  L96 t = l96_from_i128(Tm);
  return (m == 0) ? l96_sub(t, qin) : l96_add(t, qin);
}

// Twiddle entry layout (u32 words): 3k limbs of the digits, then for
// i = 0..k-1 the suffix sum sum_{t >= i} y_t as (lo, mid, hi) words.
template <int KD>
struct TwLayout {
  static constexpr int LIMBS = 0;
  static constexpr int SUF = 3 * KD;
  static constexpr int WORDS = 6 * KD;
};

// x * tw * r^rot for a table twiddle; x is this lane's semi-normalised digit.
template <int KD, int W, int U>
__device__ __forceinline__ L96 mul_twiddle(uint64_t x, const uint32_t* __restrict__ tw, int rot, int l, int m) {
  typedef Geo<KD> Gm;
  const int rp = rot & (KD - 1);
  const bool sigma = (rot & KD) != 0;
  const int src = Gm::lane_of(l, (m - rp) & (KD - 1));
  uint32_t x0 = (uint32_t)__shfl((int)(uint32_t)x, src, 64);
  uint32_t x1 = (uint32_t)__shfl((int)(uint32_t)(x >> 32), src, 64);
  const uint32_t neg = ((m < rp) != sigma) ? 0xFFFFFFFFu : 0u;
  x0 ^= neg;
  x1 ^= neg;
  YLimbs<KD> y;
  const uint4* lp = reinterpret_cast<const uint4*>(tw + TwLayout<KD>::LIMBS);
  static_for<3 * KD / 4>([&](auto I) {
    constexpr int i = decltype(I)::value;
    uint4 q = lp[i];
    y.l[4 * i] = q.x;
    y.l[4 * i + 1] = q.y;
    y.l[4 * i + 2] = q.z;
    y.l[4 * i + 3] = q.w;
  });
  // correction set: suffix from idx = m - rp + 1 (wrapped into [1, k]), or its
  // complement when rp > m, complemented again when sigma
  int idx = m - rp + 1;
  if (idx <= 0) idx += KD;
  const bool flip = (rp > m) != sigma;
  const uint32_t* suf = tw + TwLayout<KD>::SUF;
  uint64_t s_lo = 0;
  uint32_t s_hi = 0;
  if (idx < KD) {
    s_lo = (uint64_t)suf[3 * idx] | ((uint64_t)suf[3 * idx + 1] << 32);
    s_hi = suf[3 * idx + 2];
  }
  if (flip) {
    const uint64_t t_lo = (uint64_t)suf[0] | ((uint64_t)suf[1] << 32);
    const uint32_t t_hi = suf[2];
    const u128 d = (((u128)t_hi << 64) | t_lo) - (((u128)s_hi << 64) | s_lo);
    s_lo = (uint64_t)d;
    s_hi = (uint32_t)(d >> 64);
  }
  return mul_core<KD, W, U>(x0, x1, y, s_lo, s_hi, m);
}

// x * y for two data elements: every lane of the element loads all of y's
// digits (same addresses across the element's lanes) and derives the limbs
// and its correction sum (rot = 0: S_m = sum_{t > m} y_t).
template <int KD, int W, int U>
__device__ __forceinline__ L96 mul_data(uint64_t x, const uint64_t (&yd)[KD], int m) {
  YLimbs<KD> y;
  u128 S = 0;
  static_for<KD>([&](auto T) {
    constexpr int t = decltype(T)::value;
    split22(yd[t], y.l[3 * t], y.l[3 * t + 1], y.l[3 * t + 2]);
    if (t > m) S += yd[t];
  });
  return mul_core<KD, W, U>((uint32_t)x, (uint32_t)(x >> 32), y, (uint64_t)S, (uint32_t)(S >> 64), m);
}

// ------------------------------------------------------------------------
// Normalisation
// ------------------------------------------------------------------------
// Semi-normalise a lazy digit (|t| < 2^84): digit' = rho + q_{m-1} in
// [0, 2^64), where t = q r + rho with rho in [2^57, 2^64 - 2^57) and q passed
// one lane up (lane 0 takes -q_{k-1}, since r^k = -1).
template <int KD, int W, int U>
__device__ __forceinline__ uint64_t seminorm(L96 t, int m) {
  constexpr int GPL = Geo<KD>::GPL;
  typedef Field<KD, W, U> F;
  int64_t q = ((int64_t)t.hi << (64 - W)) | (int64_t)(t.lo >> W);  // floor(t / 2^W)
  // rho = t - q 2^W - q 2^U, true value in (-2^57, 2^W + 2^57)
  uint64_t rho = (t.lo & ((1ull << W) - 1)) - ((uint64_t)q << U);
  const bool low = (rho + (1ull << 57)) < (3ull << 57);  // rho < 2^58
  rho += low ? F::R : 0ull;
  q -= low ? 1 : 0;
  int32_t qi = (int32_t)q;
  int32_t qin = (int32_t)row_ror<GPL>((uint32_t)qi);
  qin = (m == 0) ? -qin : qin;
  return rho + (uint64_t)(int64_t)qin;
}

// Exact canonical form (section 2 encoding).  All lanes of the wavefront must
// call this together (wavefront-uniform loops).  Groups with active == false
// take part in the lane exchanges but their result is meaningless.
template <int KD, int W, int U>
__device__ __forceinline__ uint64_t canonicalize(L96 t, int l, int m) {
  constexpr int GPL = Geo<KD>::GPL;
  typedef Field<KD, W, U> F;
  // exact t = q r + rho, 0 <= rho < r
  int64_t q = ((int64_t)t.hi << (64 - W)) | (int64_t)(t.lo >> W);
  uint64_t rho = (t.lo & ((1ull << W) - 1)) - ((uint64_t)q << U);  // true in (-2^57, 2^W + 2^57)
  const uint64_t off = 1ull << 57;
  if (rho + off < off) {  // rho < 0
    rho += F::R;
    q -= 1;
  } else if (rho + off >= F::R + off) {  // rho >= r
    rho -= F::R;
    q += 1;
  }
  // v_m = rho_m + q_{m-1}; v_0 = rho_0 - q_{k-1}.  Now X = sum v_m r^m exactly.
  int32_t qi = (int32_t)q;
  int32_t qin = (int32_t)row_ror<GPL>((uint32_t)qi);
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
    int cin = (int)row_ror<GPL>((uint32_t)c);
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
      int cin = (int)row_ror<GPL>((uint32_t)c);
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

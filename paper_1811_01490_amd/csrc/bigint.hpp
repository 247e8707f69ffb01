// Host-side multiprecision integers for field setup (prime check, roots of
// unity, twiddle tables).  Little-endian 64-bit limbs, schoolbook products,
// Montgomery multiplication modulo an odd modulus.  Setup only: nothing here
// runs per transform.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

namespace gfp {

typedef unsigned __int128 u128;

struct Big {
  std::vector<uint64_t> w;  // little endian, no trailing zero limbs

  Big() {}
  explicit Big(uint64_t v) { if (v) w.push_back(v); }
  void trim() { while (!w.empty() && w.back() == 0) w.pop_back(); }
  bool is_zero() const { return w.empty(); }
  size_t limbs() const { return w.size(); }
  uint64_t limb(size_t i) const { return i < w.size() ? w[i] : 0; }
  unsigned bits() const {
    if (w.empty()) return 0;
    return 64 * (unsigned)(w.size() - 1) + (64 - (unsigned)__builtin_clzll(w.back()));
  }
  bool bit(unsigned i) const { return (limb(i / 64) >> (i % 64)) & 1; }
};

inline int cmp(const Big& a, const Big& b) {
  if (a.w.size() != b.w.size()) return a.w.size() < b.w.size() ? -1 : 1;
  for (size_t i = a.w.size(); i-- > 0;)
    if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
  return 0;
}

inline Big add(const Big& a, const Big& b) {
  Big c;
  size_t n = std::max(a.w.size(), b.w.size());
  c.w.resize(n + 1);
  u128 carry = 0;
  for (size_t i = 0; i < n; ++i) {
    u128 s = (u128)a.limb(i) + b.limb(i) + carry;
    c.w[i] = (uint64_t)s;
    carry = s >> 64;
  }
  c.w[n] = (uint64_t)carry;
  c.trim();
  return c;
}

// a - b, requires a >= b
inline Big sub(const Big& a, const Big& b) {
  Big c;
  c.w.resize(a.w.size());
  uint64_t borrow = 0;
  for (size_t i = 0; i < a.w.size(); ++i) {
    u128 d = (u128)a.w[i] - b.limb(i) - borrow;
    c.w[i] = (uint64_t)d;
    borrow = (uint64_t)(d >> 64) ? 1 : 0;
  }
  c.trim();
  return c;
}

inline Big mul(const Big& a, const Big& b) {
  if (a.is_zero() || b.is_zero()) return Big();
  Big c;
  c.w.assign(a.w.size() + b.w.size(), 0);
  for (size_t i = 0; i < a.w.size(); ++i) {
    u128 carry = 0;
    for (size_t j = 0; j < b.w.size(); ++j) {
      u128 t = (u128)a.w[i] * b.w[j] + c.w[i + j] + carry;
      c.w[i + j] = (uint64_t)t;
      carry = t >> 64;
    }
    c.w[i + b.w.size()] = (uint64_t)carry;
  }
  c.trim();
  return c;
}

inline Big mul_small(const Big& a, uint64_t s) { return mul(a, Big(s)); }

inline Big shl(const Big& a, unsigned s) {
  if (a.is_zero()) return Big();
  Big c;
  unsigned ls = s / 64, bs = s % 64;
  c.w.assign(a.w.size() + ls + 1, 0);
  for (size_t i = 0; i < a.w.size(); ++i) {
    c.w[i + ls] |= a.w[i] << bs;
    if (bs) c.w[i + ls + 1] |= a.w[i] >> (64 - bs);
  }
  c.trim();
  return c;
}

inline Big shr(const Big& a, unsigned s) {
  Big c;
  unsigned ls = s / 64, bs = s % 64;
  if (ls >= a.w.size()) return c;
  c.w.assign(a.w.size() - ls, 0);
  for (size_t i = ls; i < a.w.size(); ++i) {
    c.w[i - ls] = a.w[i] >> bs;
    if (bs && i + 1 < a.w.size()) c.w[i - ls] |= a.w[i + 1] << (64 - bs);
  }
  c.trim();
  return c;
}

// Division by a single 64-bit limb; returns quotient, sets rem.
inline Big divmod_small(const Big& a, uint64_t d, uint64_t* rem) {
  Big q;
  q.w.assign(a.w.size(), 0);
  u128 r = 0;
  for (size_t i = a.w.size(); i-- > 0;) {
    u128 cur = (r << 64) | a.w[i];
    q.w[i] = (uint64_t)(cur / d);
    r = cur % d;
  }
  q.trim();
  *rem = (uint64_t)r;
  return q;
}

// Binary long division (setup only; sizes are a few thousand bits at most).
inline Big mod(const Big& a, const Big& m) {
  if (cmp(a, m) < 0) return a;
  Big r;
  for (unsigned i = a.bits(); i-- > 0;) {
    r = shl(r, 1);
    if (a.bit(i)) {
      if (r.w.empty()) r.w.push_back(1); else r.w[0] |= 1;
    }
    if (cmp(r, m) >= 0) r = sub(r, m);
  }
  return r;
}

inline Big divq(const Big& a, const Big& m) {  // floor(a / m)
  Big q, r;
  for (unsigned i = a.bits(); i-- > 0;) {
    r = shl(r, 1);
    if (a.bit(i)) {
      if (r.w.empty()) r.w.push_back(1); else r.w[0] |= 1;
    }
    q = shl(q, 1);
    if (cmp(r, m) >= 0) {
      r = sub(r, m);
      if (q.w.empty()) q.w.push_back(1); else q.w[0] |= 1;
    }
  }
  return q;
}

inline unsigned ctz(const Big& a) {
  for (size_t i = 0; i < a.w.size(); ++i)
    if (a.w[i]) return 64 * (unsigned)i + (unsigned)__builtin_ctzll(a.w[i]);
  return 0;
}

// Montgomery arithmetic modulo an odd m with R = 2^(64 L), L = limbs of m.
struct Mont {
  Big m;
  size_t L;
  uint64_t minv;  // -m^-1 mod 2^64
  Big r2;         // R^2 mod m
  Big one;        // R mod m

  explicit Mont(const Big& mod_) : m(mod_), L(mod_.w.size()) {
    uint64_t inv = 1;  // Newton iteration for m0^-1 mod 2^64
    for (int i = 0; i < 7; ++i) inv *= 2 - m.w[0] * inv;
    minv = (uint64_t)(0 - inv);
    Big R = shl(Big(1), 64 * (unsigned)L);
    one = mod(R, m);
    r2 = mod(mul(one, one), m);
  }
  // CIOS Montgomery product, inputs < m.
  Big mmul(const Big& a, const Big& b) const {
    std::vector<uint64_t> t(L + 2, 0);
    for (size_t i = 0; i < L; ++i) {
      u128 c = 0;
      uint64_t ai = a.limb(i);
      for (size_t j = 0; j < L; ++j) {
        u128 s = (u128)ai * b.limb(j) + t[j] + c;
        t[j] = (uint64_t)s;
        c = s >> 64;
      }
      u128 s = (u128)t[L] + c;
      t[L] = (uint64_t)s;
      t[L + 1] = (uint64_t)(s >> 64);
      uint64_t q = t[0] * minv;
      c = 0;
      for (size_t j = 0; j < L; ++j) {
        u128 s2 = (u128)q * m.w[j] + t[j] + c;
        t[j] = (uint64_t)s2;
        c = s2 >> 64;
      }
      s = (u128)t[L] + c;
      t[L] = (uint64_t)s;
      t[L + 1] += (uint64_t)(s >> 64);
      for (size_t j = 0; j <= L; ++j) t[j] = t[j + 1];
      t[L + 1] = 0;
    }
    Big r;
    r.w.assign(t.begin(), t.begin() + L + 1);
    r.trim();
    if (cmp(r, m) >= 0) r = sub(r, m);
    return r;
  }
  Big to(const Big& a) const { return mmul(mod(a, m), r2); }
  Big from(const Big& a) const { return mmul(a, Big(1)); }
  Big pow(const Big& base_m, const Big& e) const {  // base in Montgomery form
    Big acc = one;
    for (unsigned i = e.bits(); i-- > 0;) {
      acc = mmul(acc, acc);
      if (e.bit(i)) acc = mmul(acc, base_m);
    }
    return acc;
  }
};

// ---- Baillie-PSW probable-prime test ----------------------------------------
// A strong probable-prime test to base 2 followed by a strong Lucas test with
// Selfridge's parameters (D the first of 5, -7, 9, -11, ... with Jacobi
// symbol (D/n) = -1, P = 1, Q = (1 - D) / 4).  No composite is known to pass
// both.

// Jacobi symbol (D / n) for odd n > 0 and D = +-a, a odd and small.
inline int jacobi_small(bool negative, uint64_t a, const Big& n) {
  int t = 1;
  const uint64_t n4 = n.limb(0) & 3;
  if (negative && n4 == 3) t = -t;      // (-1 / n) = (-1)^((n - 1) / 2)
  if ((a & 3) == 3 && n4 == 3) t = -t;  // reciprocity: (a / n) = +-(n / a)
  uint64_t x;
  (void)divmod_small(n, a, &x);
  uint64_t y = a;
  while (x != 0) {  // (x / y), y odd
    while ((x & 1) == 0) {
      x >>= 1;
      const uint64_t y8 = y & 7;
      if (y8 == 3 || y8 == 5) t = -t;  // (2 / y)
    }
    std::swap(x, y);
    if ((x & 3) == 3 && (y & 3) == 3) t = -t;
    x %= y;
  }
  return y == 1 ? t : 0;
}

// floor(sqrt(a)) by Newton's iteration.
inline Big isqrt(const Big& a) {
  if (a.is_zero()) return a;
  Big x = shl(Big(1), (a.bits() + 1) / 2 + 1);
  for (;;) {
    Big y = shr(add(x, divq(a, x)), 1);
    if (cmp(y, x) >= 0) return x;
    x = y;
  }
}

inline bool strong_probable_prime_base2(const Big& n, const Mont& M) {
  const Big nm1 = sub(n, Big(1));
  const unsigned s = ctz(nm1);
  const Big minus_one = M.to(nm1);
  Big x = M.pow(M.to(Big(2)), shr(nm1, s));
  if (cmp(x, M.one) == 0 || cmp(x, minus_one) == 0) return true;
  for (unsigned i = 1; i < s; ++i) {
    x = M.mmul(x, x);
    if (cmp(x, minus_one) == 0) return true;
  }
  return false;
}

inline bool strong_lucas_probable_prime(const Big& n, const Mont& M) {
  // Selfridge: D = 5, -7, 9, -11, ...
  uint64_t a = 5;
  bool neg = false;
  for (;; a += 2, neg = !neg) {
    const int j = jacobi_small(neg, a, n);
    if (j == -1) break;
    if (j == 0 && cmp(n, Big(a)) != 0) return false;  // a shares a factor with n
    if (a == 61) {  // no D so far: rule out a perfect square, which has none
      const Big r = isqrt(n);
      if (cmp(mul(r, r), n) == 0) return false;
    }
  }
  auto neg_mod = [&](const Big& v) { return v.is_zero() ? v : sub(n, v); };
  auto addm = [&](const Big& x, const Big& y) {
    Big z = add(x, y);
    return cmp(z, n) >= 0 ? sub(z, n) : z;
  };
  auto subm = [&](const Big& x, const Big& y) { return cmp(x, y) >= 0 ? sub(x, y) : sub(add(x, n), y); };
  auto half = [&](const Big& x) { return (x.limb(0) & 1) ? shr(add(x, n), 1) : shr(x, 1); };
  // Montgomery forms (halving commutes with the factor R)
  const Big Dm = neg ? neg_mod(M.to(Big(a))) : M.to(Big(a));
  // Q = (1 - D) / 4: D = a gives -(a - 1) / 4, D = -a gives (a + 1) / 4
  const Big Qm = neg ? M.to(Big((a + 1) / 4)) : neg_mod(M.to(Big((a - 1) / 4)));
  const Big np1 = add(n, Big(1));
  const unsigned s = ctz(np1);
  const Big d = shr(np1, s);
  // U_1 = 1, V_1 = P = 1, Q^1; then the bits of d below the top one
  Big U = M.one, V = M.one, Qk = Qm;
  for (unsigned i = d.bits() - 1; i-- > 0;) {
    U = M.mmul(U, V);                               // U_2k = U_k V_k
    V = subm(M.mmul(V, V), addm(Qk, Qk));           // V_2k = V_k^2 - 2 Q^k
    Qk = M.mmul(Qk, Qk);
    if (d.bit(i)) {
      const Big U1 = half(addm(U, V));              // U_2k+1 = (P U + V) / 2
      const Big V1 = half(addm(M.mmul(Dm, U), V));  // V_2k+1 = (D U + P V) / 2
      U = U1;
      V = V1;
      Qk = M.mmul(Qk, Qm);
    }
  }
  if (U.is_zero() || V.is_zero()) return true;
  for (unsigned r = 1; r < s; ++r) {
    V = subm(M.mmul(V, V), addm(Qk, Qk));  // V_(d 2^r)
    if (V.is_zero()) return true;
    Qk = M.mmul(Qk, Qk);
  }
  return false;
}

// Baillie-PSW for odd n > 3.
inline bool bpsw(const Big& n) {
  static const uint64_t small[] = {3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47};
  for (uint64_t q : small) {
    uint64_t rem;
    (void)divmod_small(n, q, &rem);
    if (rem == 0) return cmp(n, Big(q)) == 0;
  }
  const Mont M(n);
  return strong_probable_prime_base2(n, M) && strong_lucas_probable_prime(n, M);
}

}  // namespace gfp

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

}  // namespace gfp

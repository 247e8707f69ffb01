// Multithreaded CPU transform over Z/pZ, p = r^k + 1 (oracle side; test and
// measurement infrastructure only).
//
// The timed CPU baseline: a textbook radix-2 decimation-in-time transform
// (bit reversal, then log2 n butterfly levels) with its own schoolbook
// multiprecision arithmetic modulo p, spread over std::thread workers level
// by level.  It computes the same values as the oracle's Python transform
// (Y_i = sum_j X_j w^(ij), section 1.1; the inverse is (1/n) times the
// transform at w^-1, section 3.3; the product of polynomials is the inverse
// transform of the pointwise product of the transforms, Alg. Fast
// Convolution of section 3.3) and is pinned against it by tests.  It uses
// none of the paper's radix-r tricks and none of the GPU library's code: an
// element is a plain binary integer of W 64-bit words, multiplied by the
// textbook word-serial Montgomery method (coarsely integrated operand
// scanning), so the timing is that of a generic big-prime-field transform.
//
// Interface: SoA digit vectors as the GPU library takes them (digit d of
// element i at v[d * n + i], radix r, canonical encoding of section 2),
// host memory, w given as its k canonical digits.  All functions return 0
// on success and -1 on bad arguments.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <thread>
#include <vector>

namespace {

typedef unsigned __int128 u128;

template <int W>
struct Mod {
  uint64_t p[W];
  uint64_t pinv;  // -p^-1 mod 2^64
  uint64_t r2[W];  // 2^(128 W) mod p
  uint64_t one[W];  // 2^(64 W) mod p (1 in Montgomery form)
};

template <int W>
bool geq(const uint64_t* a, const uint64_t* b) {
  for (int i = W - 1; i >= 0; --i)
    if (a[i] != b[i]) return a[i] > b[i];
  return true;
}

template <int W>
uint64_t sub_in(uint64_t* a, const uint64_t* b) {  // a -= b, returns the borrow
  uint64_t br = 0;
  for (int i = 0; i < W; ++i) {
    const u128 d = (u128)a[i] - b[i] - br;
    a[i] = (uint64_t)d;
    br = (uint64_t)(d >> 64) & 1;
  }
  return br;
}

template <int W>
uint64_t add_in(uint64_t* a, const uint64_t* b) {  // a += b, returns the carry
  uint64_t c = 0;
  for (int i = 0; i < W; ++i) {
    const u128 s = (u128)a[i] + b[i] + c;
    a[i] = (uint64_t)s;
    c = (uint64_t)(s >> 64);
  }
  return c;
}

template <int W>
void add_mod(uint64_t* out, const uint64_t* a, const uint64_t* b, const Mod<W>& M) {
  uint64_t t[W];
  memcpy(t, a, sizeof(t));
  const uint64_t c = add_in<W>(t, b);
  if (c || geq<W>(t, M.p)) sub_in<W>(t, M.p);
  memcpy(out, t, sizeof(t));
}

template <int W>
void sub_mod(uint64_t* out, const uint64_t* a, const uint64_t* b, const Mod<W>& M) {
  uint64_t t[W];
  memcpy(t, a, sizeof(t));
  if (sub_in<W>(t, b)) add_in<W>(t, M.p);
  memcpy(out, t, sizeof(t));
}

// a b 2^(-64 W) mod p for a, b < p (word-serial Montgomery multiplication)
template <int W>
void mont_mul(uint64_t* out, const uint64_t* a, const uint64_t* b, const Mod<W>& M) {
  uint64_t t[W + 2];
  memset(t, 0, sizeof(t));
  for (int i = 0; i < W; ++i) {
    uint64_t c = 0;
    for (int j = 0; j < W; ++j) {
      const u128 v = (u128)a[j] * b[i] + t[j] + c;
      t[j] = (uint64_t)v;
      c = (uint64_t)(v >> 64);
    }
    u128 v = (u128)t[W] + c;
    t[W] = (uint64_t)v;
    t[W + 1] = (uint64_t)(v >> 64);
    const uint64_t m = t[0] * M.pinv;
    v = (u128)m * M.p[0] + t[0];
    c = (uint64_t)(v >> 64);
    for (int j = 1; j < W; ++j) {
      v = (u128)m * M.p[j] + t[j] + c;
      t[j - 1] = (uint64_t)v;
      c = (uint64_t)(v >> 64);
    }
    v = (u128)t[W] + c;
    t[W - 1] = (uint64_t)v;
    t[W] = t[W + 1] + (uint64_t)(v >> 64);
  }
  if (t[W] || geq<W>(t, M.p)) sub_in<W>(t, M.p);
  memcpy(out, t, W * sizeof(uint64_t));
}

// binary value of a canonical radix-r digit vector: sum_d x_d r^d (< p)
template <int W>
void from_digits(uint64_t* v, const uint64_t* x, uint64_t n, uint64_t i, int k, uint64_t r) {
  uint64_t t[W + 1];
  memset(t, 0, sizeof(t));
  for (int d = k - 1; d >= 0; --d) {
    uint64_t c = x[(uint64_t)d * n + i];
    for (int j = 0; j <= W; ++j) {
      const u128 s = (u128)t[j] * r + c;
      t[j] = (uint64_t)s;
      c = (uint64_t)(s >> 64);
    }
  }
  memcpy(v, t, W * sizeof(uint64_t));
}

// canonical radix-r digits of v < p; p - 1 = r^k is written (0, ..., 0, r)
template <int W>
void to_digits(uint64_t* y, uint64_t n, uint64_t i, const uint64_t* v, int k, uint64_t r, const Mod<W>& M) {
  uint64_t pm1[W];
  memcpy(pm1, M.p, sizeof(pm1));
  pm1[0] -= 1;  // p is odd
  bool is_pm1 = true;
  for (int j = 0; j < W; ++j) is_pm1 = is_pm1 && v[j] == pm1[j];
  if (is_pm1) {
    for (int d = 0; d < k; ++d) y[(uint64_t)d * n + i] = (d == k - 1) ? r : 0;
    return;
  }
  uint64_t t[W];
  memcpy(t, v, sizeof(t));
  for (int d = 0; d < k; ++d) {
    uint64_t rem = 0;
    for (int j = W - 1; j >= 0; --j) {
      const u128 cur = ((u128)rem << 64) | t[j];
      t[j] = (uint64_t)(cur / r);
      rem = (uint64_t)(cur % r);
    }
    y[(uint64_t)d * n + i] = rem;
  }
}

template <int W>
bool setup(Mod<W>& M, int k, uint64_t r) {
  // p = r^k + 1 must fit in W words
  uint64_t t[W + 1];
  memset(t, 0, sizeof(t));
  t[0] = 1;
  for (int d = 0; d < k; ++d) {
    uint64_t c = 0;
    for (int j = 0; j <= W; ++j) {
      const u128 s = (u128)t[j] * r + c;
      t[j] = (uint64_t)s;
      c = (uint64_t)(s >> 64);
    }
    if (c) return false;
  }
  if (t[W]) return false;
  t[0] += 1;  // r^k is even: no carry
  memcpy(M.p, t, W * sizeof(uint64_t));
  // -p^-1 mod 2^64 by Newton's iteration (each step doubles the correct bits)
  uint64_t inv = 1;
  for (int it = 0; it < 7; ++it) inv *= 2 - M.p[0] * inv;
  M.pinv = 0 - inv;
  // 2^(64 W) mod p and 2^(128 W) mod p by doubling
  uint64_t x[W];
  memset(x, 0, sizeof(x));
  x[0] = 1;
  for (int b = 0; b < 128 * W; ++b) {
    const uint64_t top = x[W - 1] >> 63;
    for (int j = W - 1; j > 0; --j) x[j] = (x[j] << 1) | (x[j - 1] >> 63);
    x[0] <<= 1;
    if (top || geq<W>(x, M.p)) sub_in<W>(x, M.p);
    if (b == 64 * W - 1) memcpy(M.one, x, sizeof(x));
  }
  memcpy(M.r2, x, sizeof(x));
  return true;
}

template <class F>
void parallel_for(uint64_t count, int threads, F&& f) {
  const int nt = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)std::max(threads, 1), count));
  if (nt == 1) {
    f(0, count);
    return;
  }
  std::vector<std::thread> pool;
  const uint64_t chunk = (count + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const uint64_t lo = (uint64_t)t * chunk, hi = std::min(count, lo + chunk);
    if (lo < hi) pool.emplace_back([&f, lo, hi] { f(lo, hi); });
  }
  for (auto& th : pool) th.join();
}

// Powers w^j, j < n/2, in Montgomery form (w in Montgomery form): each
// worker starts its range at w^lo by square-and-multiply, then steps by w.
template <int W>
void powers(std::vector<uint64_t>& tw, uint64_t n, const uint64_t* w, const Mod<W>& M, int threads) {
  tw.assign((n / 2) * W, 0);
  parallel_for(n / 2, threads, [&](uint64_t lo, uint64_t hi) {
    uint64_t acc[W], base[W];
    memcpy(acc, M.one, sizeof(acc));
    memcpy(base, w, sizeof(base));
    for (uint64_t e = lo; e; e >>= 1) {
      if (e & 1) mont_mul<W>(acc, acc, base, M);
      mont_mul<W>(base, base, base, M);
    }
    memcpy(&tw[lo * W], acc, sizeof(acc));
    for (uint64_t j = lo + 1; j < hi; ++j) mont_mul<W>(&tw[j * W], &tw[(j - 1) * W], w, M);
  });
}

// In-place transform of n = 2^lg elements (Montgomery form); tw = powers of
// the root (see powers).
template <int W>
void ntt_mont(std::vector<uint64_t>& a, uint64_t n, const std::vector<uint64_t>& tw, const Mod<W>& M,
              int threads) {
  int lg = 0;
  while ((1ull << lg) < n) ++lg;
  // bit reversal
  parallel_for(n, threads, [&](uint64_t lo, uint64_t hi) {
    for (uint64_t i = lo; i < hi; ++i) {
      uint64_t j = 0;
      for (int b = 0; b < lg; ++b) j |= ((i >> b) & 1) << (lg - 1 - b);
      if (i < j)
        for (int q = 0; q < W; ++q) std::swap(a[i * W + q], a[j * W + q]);
    }
  });
  for (int lv = 0; lv < lg; ++lv) {
    const uint64_t h = 1ull << lv, stride = n / (2 * h);
    parallel_for(n / 2, threads, [&](uint64_t lo, uint64_t hi) {
      uint64_t v[W];
      for (uint64_t b = lo; b < hi; ++b) {
        const uint64_t grp = b / h, j = b % h;
        uint64_t* x0 = &a[(grp * 2 * h + j) * W];
        uint64_t* x1 = x0 + h * W;
        mont_mul<W>(v, x1, &tw[j * stride * W], M);
        sub_mod<W>(x1, x0, v, M);
        add_mod<W>(x0, x0, v, M);
      }
    });
  }
}

template <int W>
void load(std::vector<uint64_t>& a, const uint64_t* x, uint64_t lx, uint64_t n, int k, uint64_t r, const Mod<W>& M,
          int threads) {
  a.assign(n * W, 0);
  parallel_for(lx, threads, [&](uint64_t lo, uint64_t hi) {
    uint64_t v[W];
    for (uint64_t i = lo; i < hi; ++i) {
      from_digits<W>(v, x, lx, i, k, r);
      mont_mul<W>(&a[i * W], v, M.r2, M);
    }
  });
}

template <int W>
void store(uint64_t* y, uint64_t ly, const std::vector<uint64_t>& a, int k, uint64_t r, const Mod<W>& M,
           int threads) {
  uint64_t unit[W];
  memset(unit, 0, sizeof(unit));
  unit[0] = 1;
  parallel_for(ly, threads, [&](uint64_t lo, uint64_t hi) {
    uint64_t v[W];
    for (uint64_t i = lo; i < hi; ++i) {
      mont_mul<W>(v, &a[i * W], unit, M);
      to_digits<W>(y, ly, i, v, k, r, M);
    }
  });
}

// n^-1 in Montgomery form: n = 2^lg, so n^-1 = ((p + 1) / 2)^lg
template <int W>
void inv_n_mont(uint64_t* out, uint64_t n, const Mod<W>& M) {
  uint64_t half[W];
  memcpy(half, M.p, sizeof(half));
  half[0] += 1;  // p + 1 (p odd: no carry out of the low word would matter below)
  for (int j = 0; j < W; ++j) half[j] = (half[j] >> 1) | (j + 1 < W ? half[j + 1] << 63 : 0);
  uint64_t hm[W], acc[W];
  mont_mul<W>(hm, half, M.r2, M);
  memcpy(acc, M.one, sizeof(acc));
  for (uint64_t t = 1; t < n; t <<= 1) mont_mul<W>(acc, acc, hm, M);
  memcpy(out, acc, sizeof(acc));
}

template <int W>
int transform(int k, uint64_t r, uint64_t n, const uint64_t* x, uint64_t* y, const uint64_t* wd, int inverse,
              int threads) {
  Mod<W> M;
  if (!setup<W>(M, k, r)) return -1;
  std::vector<uint64_t> a, wv, tw;
  load<W>(wv, wd, 1, 1, k, r, M, 1);
  powers<W>(tw, n, &wv[0], M, threads);
  load<W>(a, x, n, n, k, r, M, threads);
  ntt_mont<W>(a, n, tw, M, threads);
  if (inverse) {
    uint64_t ni[W];
    inv_n_mont<W>(ni, n, M);
    parallel_for(n, threads, [&](uint64_t lo, uint64_t hi) {
      for (uint64_t i = lo; i < hi; ++i) mont_mul<W>(&a[i * W], &a[i * W], ni, M);
    });
  }
  store<W>(y, n, a, k, r, M, threads);
  return 0;
}

template <int W>
int polymul(int k, uint64_t r, uint64_t la, const uint64_t* a, uint64_t lb, const uint64_t* b, uint64_t* c,
            uint64_t n, const uint64_t* wd, const uint64_t* wid, int threads) {
  Mod<W> M;
  if (!setup<W>(M, k, r)) return -1;
  std::vector<uint64_t> A, B, wv, wiv, tw, twi;
  load<W>(wv, wd, 1, 1, k, r, M, 1);
  load<W>(wiv, wid, 1, 1, k, r, M, 1);
  powers<W>(tw, n, &wv[0], M, threads);
  powers<W>(twi, n, &wiv[0], M, threads);
  load<W>(A, a, la, n, k, r, M, threads);
  load<W>(B, b, lb, n, k, r, M, threads);
  ntt_mont<W>(A, n, tw, M, threads);
  ntt_mont<W>(B, n, tw, M, threads);
  uint64_t ni[W];
  inv_n_mont<W>(ni, n, M);
  parallel_for(n, threads, [&](uint64_t lo, uint64_t hi) {
    for (uint64_t i = lo; i < hi; ++i) {
      mont_mul<W>(&A[i * W], &A[i * W], &B[i * W], M);
      mont_mul<W>(&A[i * W], &A[i * W], ni, M);
    }
  });
  ntt_mont<W>(A, n, twi, M, threads);
  store<W>(c, la + lb - 1, A, k, r, M, threads);
  return 0;
}

int words_for(int k) { return k <= 8 ? 8 : k <= 16 ? 16 : k <= 32 ? 32 : k <= 64 ? 64 : 0; }

bool pow2(uint64_t n) { return n >= 2 && (n & (n - 1)) == 0; }

}  // namespace

extern "C" {

// y = transform of x (n elements) at w (k digits); inverse != 0: (1/n) times
// the transform at w (pass w^-1 for the inverse transform).
int cpu_ntt_transform(int k, uint64_t r, uint64_t n, const uint64_t* x, uint64_t* y, const uint64_t* w, int inverse,
                      int threads) {
  if (!x || !y || !w || !pow2(n) || r < 2) return -1;
  switch (words_for(k)) {
    case 8: return transform<8>(k, r, n, x, y, w, inverse, threads);
    case 16: return transform<16>(k, r, n, x, y, w, inverse, threads);
    case 32: return transform<32>(k, r, n, x, y, w, inverse, threads);
    case 64: return transform<64>(k, r, n, x, y, w, inverse, threads);
    default: return -1;
  }
}

// c (la + lb - 1 elements) = a b, through transforms of size n >= la + lb - 1
// at w (forward) and w_inv (inverse).
int cpu_ntt_polymul(int k, uint64_t r, uint64_t la, const uint64_t* a, uint64_t lb, const uint64_t* b, uint64_t* c,
                    uint64_t n, const uint64_t* w, const uint64_t* w_inv, int threads) {
  if (!a || !b || !c || !w || !w_inv || !pow2(n) || la == 0 || lb == 0 || la + lb - 1 > n || r < 2) return -1;
  switch (words_for(k)) {
    case 8: return polymul<8>(k, r, la, a, lb, b, c, n, w, w_inv, threads);
    case 16: return polymul<16>(k, r, la, a, lb, b, c, n, w, w_inv, threads);
    case 32: return polymul<32>(k, r, la, a, lb, b, c, n, w, w_inv, threads);
    case 64: return polymul<64>(k, r, la, a, lb, b, c, n, w, w_inv, threads);
    default: return -1;
  }
}

}  // extern "C"

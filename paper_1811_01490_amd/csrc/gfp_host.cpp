// Host side of libgfpfft: field setup (section 2), roots of unity (Alg. 1),
// twiddle tables, pass scheduling and the C ABI declared in include/gfp.h.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <map>
#include <string>
#include <tuple>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/gfp.h"
#include "bigint.hpp"
#include "gfp_internal.hpp"

using gfp::Big;
using gfp::Mont;

namespace {

const uint64_t kMaxLog2N = 25;
const size_t kMaxGraphs = 64;  // captured batched-product graphs kept per field

struct DevTables {
  uint32_t* fwd = nullptr;   // n/K entries: w^j
  uint32_t* inv = nullptr;   // n/K entries: w^-j
  uint32_t* fwd2 = nullptr;  // n/K entries: w^(K j) (n >= K^2)
  uint32_t* inv2 = nullptr;  // n/K entries: w^-(K j)
  uint32_t* ninv = nullptr;  // one entry: 1/n
  // k >= 32 and n > K: inv and inv2 times 1/n, so that the inverse's second
  // launch (a radix-K pass with Ns > 1: every slot is multiplied by a table
  // entry) also applies 1/n, instead of an extra product per element in the
  // first launch
  uint32_t* inv_s = nullptr;
  uint32_t* inv2_s = nullptr;
  // k <= 16: fwd, inv, fwd2, inv2 again as raw digits (k u64 per entry),
  // the form the per-group twiddle passes stage through LDS
  uint64_t* fwd_raw = nullptr;
  uint64_t* inv_raw = nullptr;
  uint64_t* fwd2_raw = nullptr;
  uint64_t* inv2_raw = nullptr;
  // k >= 32, built on the first transform that selects the FFT-based twiddle
  // product: the transforms of every entry of fwd, inv, fwd2, inv2, inv_s,
  // inv2_s (3k u64 per entry; see ntt_spectrum)
  uint64_t* fwd_spec = nullptr;
  uint64_t* inv_spec = nullptr;
  uint64_t* fwd2_spec = nullptr;
  uint64_t* inv2_spec = nullptr;
  uint64_t* inv_s_spec = nullptr;
  uint64_t* inv2_s_spec = nullptr;
};

void free_tables(DevTables& t) {
  (void)hipFree(t.fwd);
  (void)hipFree(t.inv);
  (void)hipFree(t.fwd2);
  (void)hipFree(t.inv2);
  (void)hipFree(t.ninv);
  (void)hipFree(t.inv_s);
  (void)hipFree(t.inv2_s);
  (void)hipFree(t.fwd_raw);
  (void)hipFree(t.inv_raw);
  (void)hipFree(t.fwd2_raw);
  (void)hipFree(t.inv2_raw);
  (void)hipFree(t.fwd_spec);
  (void)hipFree(t.inv_spec);
  (void)hipFree(t.fwd2_spec);
  (void)hipFree(t.inv2_spec);
  (void)hipFree(t.inv_s_spec);
  (void)hipFree(t.inv2_s_spec);
}

// Whether the inverse of size 2^log2n takes its 1/n from the scaled tables
// (see DevTables) rather than in its first launch.
bool scale_in_tables(const gfp_field* f, int log2n);

struct DevConsts {
  uint32_t* one = nullptr;  // one entry: 1
  uint64_t* ntt = nullptr;  // constants of the FFT-based element product
};

}  // namespace

struct gfp_field {
  uint32_t k = 0;
  uint64_t r = 0;
  int w = -1, u = 0;  // r = 2^w + 2^u (or 2^w - 2^-u for u < 0); w = -1: neither form
  bool gpu_shape = false;
  bool validate = false;  // GFP_VALIDATE set at create: check inputs are canonical
  bool host_tables = false;  // GFP_HOST_TABLES set at create: build every twiddle table on the host
  Big p, pm1;
  std::unique_ptr<Mont> mont;
  uint32_t log2max = 0;
  Big h_mont;       // smallest quadratic non-residue, Montgomery form
  uint64_t j1 = 0;  // Alg. 1's exponent (independent of n)
  std::mutex mu;
  std::map<std::pair<int, uint64_t>, DevTables> tables;
  std::map<int, DevConsts> consts;
  // batched products captured as graphs, keyed by the whole argument list
  // (descriptors, workspace, stream, device) and the plan generation, found
  // by a hash of it; at most kMaxGraphs, the least recently used evicted
  struct Graph {
    std::string key;
    hipGraphExec_t exec;
    hipEvent_t done;  // recorded after each launch of the graph
    uint64_t seq;     // last use
  };
  std::multimap<uint64_t, Graph> graphs;
  uint64_t graph_seq = 0;
  uint64_t plan_gen = 0;  // bumped by every plan change
  // stage groupings: (log2 n, batch class, layout) -> launch codes (1: one
  // pass, 2: fused pair, 3: wide fused pair), set by gfp_plan_set /
  // gfp_tune; keys without an entry use default_plan
  std::map<std::tuple<int, int, int>, std::vector<int>> plans;
  // side streams (default priority) for the size classes of a batched
  // product, per device, with their join events and the fork event
  struct Side {
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> joins;
    hipEvent_t fork = nullptr;
  };
  std::mutex side_mu;
  std::map<int, Side> side;
  // pinned staging of the persistent launch's work list, per device; `done`
  // is recorded behind the copy that last read it (guarded by stage_mu)
  struct Stage {
    void* host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
  };
  std::mutex stage_mu;
  std::map<int, Stage> stage;
};

namespace {

int log2_exact(uint64_t n) {
  if (n == 0 || (n & (n - 1))) return -1;
  return __builtin_ctzll(n);
}

bool scale_in_tables(const gfp_field* f, int log2n) {
  return f->k >= 32 && log2n > log2_exact(2ull * f->k);
}

// Per-group twiddles go through LDS from the raw-digit tables for transforms
// of at least 2^18 elements per vector times vectors (measured on MI355X: the
// k = 8 last pass at 2^20 67.5 -> 56.4 us), and are read whole by each lane
// from the limb tables below that, where the staging's longer chain per slot
// costs more than it saves (k = 16 at 2^15: 72.7 against 68.4 us).
bool staged_twiddles(const gfp_field* f, int log2n, uint64_t nvec) {
  return f->k <= 16 && (nvec << log2n) >= (1ull << 18);
}


// canonical radix-r digits of v (0 <= v < p)
void to_digits(const gfp_field* f, const Big& v, uint64_t* out) {
  if (gfp::cmp(v, f->pm1) == 0) {
    for (uint32_t d = 0; d < f->k; ++d) out[d] = 0;
    out[f->k - 1] = f->r;
    return;
  }
  Big cur = v;
  for (uint32_t d = 0; d < f->k; ++d) {
    uint64_t rem;
    cur = gfp::divmod_small(cur, f->r, &rem);
    out[d] = rem;
  }
}

// Twiddle-entry layout of the kernels: limbs (22, 22, 20 bits) of every
// digit, then the suffix sums sum_{t >= i} y_t, i = 0..k (the last is 0), as
// three 32-bit words each; padded to gfpk::tw_words(k) words.
void make_entry(uint32_t k, const uint64_t* y, uint32_t* e) {
  for (uint32_t t = 0; t < k; ++t) {
    e[3 * t] = (uint32_t)(y[t] & 0x3FFFFFu);
    e[3 * t + 1] = (uint32_t)((y[t] >> 22) & 0x3FFFFFu);
    e[3 * t + 2] = (uint32_t)(y[t] >> 44);
  }
  for (uint32_t i = 0; i <= k; ++i) {
    gfp::u128 s = 0;
    for (uint32_t t = i; t < k; ++t) s += y[t];
    e[3 * k + 3 * i] = (uint32_t)s;
    e[3 * k + 3 * i + 1] = (uint32_t)(s >> 32);
    e[3 * k + 3 * i + 2] = (uint32_t)(s >> 64);
  }
  for (int w = 6 * (int)k + 3; w < gfpk::tw_words((int)k); ++w) e[w] = 0;
}

// w_n in Montgomery form (Alg. 1 with g = h^((p-1)/n))
Big root_mont(const gfp_field* f, uint64_t n, bool inverse) {
  const int lg = log2_exact(n);
  Big e = gfp::mul_small(gfp::shr(f->pm1, (unsigned)lg), f->j1);  // j (p-1)/n
  if (inverse) {
    // w^-1 = w^(n-1)
    e = gfp::mul_small(e, n - 1);
  }
  return f->mont->pow(f->h_mont, e);
}

// host table of w^(sign j), j < cnt, in entry layout
// Entries scale w^j, j < cnt (wm = w and sm = scale in Montgomery form;
// sm == nullptr: scale 1).
// raw != nullptr: also the raw digits, k u64 per entry.
void build_table(const gfp_field* f, const Big& wm, uint64_t cnt, std::vector<uint32_t>& out,
                 const Big* sm = nullptr, std::vector<uint64_t>* raw = nullptr) {
  const int words = gfpk::tw_words((int)f->k);
  out.assign(cnt * words, 0);
  if (raw) raw->assign(cnt * f->k, 0);
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (cnt < 4096) nth = 1;
  const uint64_t chunk = (cnt + nth - 1) / nth;
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nth; ++t) {
    const uint64_t lo = t * chunk, hi = std::min(cnt, lo + chunk);
    if (lo >= hi) break;
    th.emplace_back([&, lo, hi]() {
      const Mont& M = *f->mont;
      Big acc = M.pow(wm, Big(lo));
      if (sm) acc = M.mmul(acc, *sm);
      std::vector<uint64_t> dg(f->k);
      for (uint64_t j = lo; j < hi; ++j) {
        to_digits(f, M.from(acc), dg.data());
        make_entry(f->k, dg.data(), &out[j * words]);
        if (raw) std::copy(dg.begin(), dg.end(), raw->begin() + j * f->k);
        acc = M.mmul(acc, wm);
      }
    });
  }
  for (auto& x : th) x.join();
}

int hip_status(hipError_t e) { return e == hipSuccess ? GFP_OK : (e == hipErrorOutOfMemory ? GFP_ENOMEM : GFP_EDEVICE); }

template <class T>
int upload(const std::vector<T>& host, T** dev) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, host.size() * sizeof(T));
  if (e != hipSuccess) return hip_status(e);
  // on the per-thread stream: no implicit wait for work on other streams
  e = hipMemcpyAsync(p, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice, hipStreamPerThread);
  if (e == hipSuccess) e = hipStreamSynchronize(hipStreamPerThread);
  if (e != hipSuccess) {
    (void)hipFree(p);
    return hip_status(e);
  }
  *dev = (T*)p;
  return GFP_OK;
}

// The table of w^j, j < cnt (a power of two), and its raw digits, built on the
// device (k <= 16): the host computes w^i for i < B = 2^ceil(lg cnt / 2) and
// w^(B i) for i < cnt / B (2 sqrt(cnt) powers instead of cnt), and
// k_table_build multiplies them.  Its products are canonical, so the tables
// equal the host-built ones digit for digit (measured: the first 2^20-point
// transform of a field 3.1 ms against 15.8 ms for k = 8, 7.1 against 27.5 ms
// for k = 16).
int build_table_dev(const gfp_field* f, const Big& wm, uint64_t cnt, uint32_t** tab, uint64_t** raw) {
  const int lg = log2_exact(cnt);
  if (lg < 0 || f->k > 16) return GFP_EINVAL;
  const Mont& M = *f->mont;
  const int lb = (lg + 1) / 2;
  const uint64_t B = 1ull << lb, H = cnt >> lb;
  std::vector<uint64_t> small((B + H) * f->k);
  Big acc = M.pow(wm, Big(0));
  for (uint64_t i = 0; i < B; ++i) {
    to_digits(f, M.from(acc), &small[i * f->k]);
    acc = M.mmul(acc, wm);
  }
  const Big wb = M.pow(wm, Big(B));
  acc = M.pow(wm, Big(0));
  for (uint64_t i = 0; i < H; ++i) {
    to_digits(f, M.from(acc), &small[(B + i) * f->k]);
    acc = M.mmul(acc, wb);
  }
  uint64_t* dsmall = nullptr;
  int rc = upload(small, &dsmall);
  if (rc != GFP_OK) return rc;
  void* t = nullptr;
  void* r = nullptr;
  hipError_t he = hipMalloc(&t, cnt * gfpk::tw_words((int)f->k) * sizeof(uint32_t));
  if (he == hipSuccess) he = hipMalloc(&r, cnt * f->k * sizeof(uint64_t));
  if (he == hipSuccess)
    he = gfpk::launch_table_build((int)f->k, f->w, f->u, dsmall, dsmall + B * f->k, lb, cnt, (uint32_t*)t,
                                  (uint64_t*)r, hipStreamPerThread);
  if (he == hipSuccess) he = hipStreamSynchronize(hipStreamPerThread);
  (void)hipFree(dsmall);
  if (he != hipSuccess) {
    if (t) (void)hipFree(t);
    if (r) (void)hipFree(r);
    return hip_status(he);
  }
  *tab = (uint32_t*)t;
  *raw = (uint64_t*)r;
  return GFP_OK;
}

// valid transform size: a power of two n >= K within the field and the build
// limit.  n = R K^e with R = 2^(log2n - e log2 K) < K: *e radix-K passes, preceded
// by one radix-R pass when R > 1.
int check_size(const gfp_field* f, uint64_t n, int* log2n, int* e) {
  const int lg = log2_exact(n);
  const int lk = log2_exact(2ull * f->k);
  if (lg < 0 || lg < lk) return GFP_EUNSUPPORTED;
  if ((uint64_t)lg > f->log2max || (uint64_t)lg > kMaxLog2N) return GFP_EUNSUPPORTED;
  *log2n = lg;
  *e = lg / lk;
  return GFP_OK;
}

// Tables are built and uploaded without the field lock held, so other
// threads keep launching meanwhile; two threads that build the same tables
// at once keep the first and free the second.
// build == false: only look the tables up (GFP_ENOTREADY when they are not
// on the device yet), never allocate.
int get_tables(gfp_field* f, uint64_t n, const DevTables** out, bool build = true) {
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return hip_status(he);
  auto key = std::make_pair(dev, n);
  {
    std::lock_guard<std::mutex> g(f->mu);
    auto it = f->tables.find(key);
    if (it != f->tables.end()) {
      *out = &it->second;
      return GFP_OK;
    }
  }
  if (!build) return GFP_ENOTREADY;
  const uint64_t cnt = n / (2ull * f->k);
  DevTables t;
  std::vector<uint32_t> host;
  std::vector<uint64_t> raw;
  std::vector<uint64_t>* rawp = f->k <= 16 ? &raw : nullptr;
  const Mont& M = *f->mont;
  const Big ninv_m = M.pow(M.to(Big(n)), gfp::sub(f->p, Big(2)));  // 1/n, Montgomery form
  // table of w^j (or w^(-j)) with its raw digits where the passes read them
  auto table = [&](const Big& wm, uint32_t** tab, uint64_t** rawt) -> int {
    if (rawp && !f->host_tables) return build_table_dev(f, wm, cnt, tab, rawt);
    build_table(f, wm, cnt, host, nullptr, rawp);
    int r2 = upload(host, tab);
    if (r2 == GFP_OK && rawp) r2 = upload(raw, rawt);
    return r2;
  };
  int rc = table(root_mont(f, n, false), &t.fwd, &t.fwd_raw);
  if (rc == GFP_OK) rc = table(root_mont(f, n, true), &t.inv, &t.inv_raw);
  // w^K = w_{n/K} (the roots are nested): twiddles of the passes before the last
  if (rc == GFP_OK && n >= 4ull * f->k * f->k) {
    rc = table(root_mont(f, n / (2ull * f->k), false), &t.fwd2, &t.fwd2_raw);
    if (rc == GFP_OK) rc = table(root_mont(f, n / (2ull * f->k), true), &t.inv2, &t.inv2_raw);
  }
  if (rc == GFP_OK && scale_in_tables(f, log2_exact(n))) {
    build_table(f, root_mont(f, n, true), cnt, host, &ninv_m);
    rc = upload(host, &t.inv_s);
    if (rc == GFP_OK && n >= 4ull * f->k * f->k) {
      build_table(f, root_mont(f, n / (2ull * f->k), true), cnt, host, &ninv_m);
      rc = upload(host, &t.inv2_s);
    }
  }
  if (rc == GFP_OK) {
    // 1/n = n^(p-2)
    Big ninv = M.from(ninv_m);
    std::vector<uint64_t> dg(f->k);
    to_digits(f, ninv, dg.data());
    host.assign(gfpk::tw_words((int)f->k), 0);
    make_entry(f->k, dg.data(), host.data());
    rc = upload(host, &t.ninv);
  }
  if (rc != GFP_OK) {
    free_tables(t);
    return rc;
  }
  std::lock_guard<std::mutex> g(f->mu);
  auto ins = f->tables.emplace(key, t);
  if (!ins.second) free_tables(t);
  *out = &ins.first->second;
  return GFP_OK;
}

int get_one(gfp_field* f, const uint32_t** out) {
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return hip_status(he);
  std::lock_guard<std::mutex> g(f->mu);
  auto it = f->consts.find(dev);
  if (it != f->consts.end() && it->second.one) {
    *out = it->second.one;
    return GFP_OK;
  }
  std::vector<uint64_t> dg(f->k, 0);
  dg[0] = 1;
  std::vector<uint32_t> host(gfpk::tw_words((int)f->k));
  make_entry(f->k, dg.data(), host.data());
  uint32_t* one = nullptr;
  int rc = upload(host, &one);
  if (rc != GFP_OK) return rc;
  f->consts[dev].one = one;
  *out = one;
  return GFP_OK;
}

// ---- constants of the FFT-based element product (section 3.3) ----------------
// Three word primes q < 2^62 with q = 1 (mod 128), so that every 2k <= 128
// divides q - 1; a primitive 2k-th root theta = g^((q-1)/2k) from the
// smallest quadratic non-residue g; Montgomery form with 2^64; CRT words.
// The layout is the one the device code reads (NTT_HEAD = 20 header words).
typedef unsigned __int128 u128h;
uint64_t mulm(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128h)a * b % q); }
uint64_t powm(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  for (a %= q; e; e >>= 1, a = mulm(a, a, q))
    if (e & 1) r = mulm(r, a, q);
  return r;
}
bool prime64(uint64_t n) {  // deterministic Miller-Rabin for n < 2^64
  if (n < 2) return false;
  for (uint64_t p : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull})
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int s = 0;
  while (!(d & 1)) d >>= 1, ++s;
  for (uint64_t a : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull}) {
    uint64_t x = powm(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < s && comp; ++i) {
      x = mulm(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}
// The three word primes of the FFT-based product (the largest q < 2^62 with
// q = 1 mod 128) and, for each, the primitive 2k-th root theta from its
// smallest quadratic non-residue.
void ntt_primes(uint32_t k, uint64_t q[3], uint64_t th[3]) {
  int found = 0;
  for (uint64_t c = (1ull << 62) - 127; found < 3; c -= 128)  // c = 1 (mod 128)
    if (prime64(c)) q[found++] = c;
  for (int i = 0; i < 3; ++i) {
    uint64_t g = 2;
    while (powm(g, (q[i] - 1) / 2, q[i]) != q[i] - 1) ++g;
    th[i] = powm(g, (q[i] - 1) / (2 * k), q[i]);
  }
}

// The transforms of a twiddle y as the FFT-based twiddle product reads them:
// for each prime, v_m = y_m theta^m mod q, then the device's forward
// transform (decimation in frequency over the lanes: for halves k/2, ..., 1,
// the pair (m, m + h) becomes (a + b, (a - b) w^(j k / (2h))), j = m mod h,
// w = theta^2); out[i k + m] = lane m's value.
void ntt_spectrum(uint32_t k, const uint64_t q[3], const uint64_t th[3], const uint64_t* y, uint64_t* out) {
  std::vector<uint64_t> v(k), wp(k / 2);
  for (int i = 0; i < 3; ++i) {
    const uint64_t qq = q[i], w = mulm(th[i], th[i], qq);
    uint64_t t = 1;
    for (uint32_t m = 0; m < k; ++m, t = mulm(t, th[i], qq)) v[m] = mulm(y[m] % qq, t, qq);
    wp[0] = 1;
    for (uint32_t j = 1; j < k / 2; ++j) wp[j] = mulm(wp[j - 1], w, qq);
    for (uint32_t h = k / 2; h >= 1; h /= 2) {
      for (uint32_t m = 0; m < k; ++m) {
        if (m & h) continue;
        const uint64_t a = v[m], b = v[m | h];
        v[m] = a + b >= qq ? a + b - qq : a + b;
        v[m | h] = mulm(a >= b ? a - b : a + qq - b, wp[(m & (h - 1)) * (k / (2 * h))], qq);
      }
    }
    std::copy(v.begin(), v.end(), out + (size_t)i * k);
  }
}

std::vector<uint64_t> ntt_constants(uint32_t k) {
  uint64_t q[3], thq[3];
  ntt_primes(k, q, thq);
  std::vector<uint64_t> t(20 + 9 * k, 0);
  auto mont = [](uint64_t a, uint64_t qq) { return (uint64_t)(((u128h)(a % qq) << 64) % qq); };
  for (int i = 0; i < 3; ++i) {
    const uint64_t qq = q[i];
    uint64_t inv = 1;  // q^-1 mod 2^64 by Newton iteration
    for (int it = 0; it < 7; ++it) inv *= 2 - qq * inv;
    t[i] = qq;
    t[3 + i] = 0 - inv;
    const uint64_t th = thq[i], thi = powm(th, qq - 2, qq);
    const uint64_t om = mulm(th, th, qq), omi = mulm(thi, thi, qq);
    const uint64_t kinv = powm(k, qq - 2, qq);
    const uint64_t r128 = mulm(mont(1, qq), mont(1, qq), qq);  // 2^128 mod q
    uint64_t* b = t.data() + 20 + 3 * k * i;
    for (uint32_t m = 0; m < k; ++m) {
      b[m] = mont(powm(th, m, qq), qq);
      b[k + m] = mulm(mulm(powm(thi, m, qq), kinv, qq), r128, qq);
    }
    for (uint32_t j = 0; j < k / 2; ++j) {
      b[2 * k + j] = mont(powm(om, j, qq), qq);
      b[2 * k + k / 2 + j] = mont(powm(omi, j, qq), qq);
    }
  }
  t[6] = mont(powm(q[0] % q[1], q[1] - 2, q[1]), q[1]);
  t[7] = mont(q[0] % q[2], q[2]);
  t[8] = mont(powm(mulm(q[0] % q[2], q[1] % q[2], q[2]), q[2] - 2, q[2]), q[2]);
  const u128h q12 = (u128h)q[0] * q[1];
  t[9] = (uint64_t)q12;
  t[10] = (uint64_t)(q12 >> 64);
  // Q = q12 q3 and (Q - 1) / 2, 192-bit
  const u128h lo = (u128h)t[9] * q[2], hi = (u128h)t[10] * q[2] + (uint64_t)(lo >> 64);
  t[11] = (uint64_t)lo;
  t[12] = (uint64_t)hi;
  t[13] = (uint64_t)(hi >> 64);
  const uint64_t m0 = t[11] - 1;  // Q is odd: Q - 1 has no borrow
  t[14] = (m0 >> 1) | (t[12] << 63);
  t[15] = (t[12] >> 1) | (t[13] << 63);
  t[16] = t[13] >> 1;
  return t;
}

int get_ntt(gfp_field* f, const uint64_t** out) {
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return hip_status(he);
  {
    std::lock_guard<std::mutex> g(f->mu);
    auto it = f->consts.find(dev);
    if (it != f->consts.end() && it->second.ntt) {
      *out = it->second.ntt;
      return GFP_OK;
    }
  }
  const std::vector<uint64_t> t = ntt_constants(f->k);
  void* p = nullptr;
  he = hipMalloc(&p, t.size() * 8);
  if (he != hipSuccess) return hip_status(he);
  he = hipMemcpyAsync(p, t.data(), t.size() * 8, hipMemcpyHostToDevice, hipStreamPerThread);
  if (he == hipSuccess) he = hipStreamSynchronize(hipStreamPerThread);
  if (he != hipSuccess) {
    (void)hipFree(p);
    return hip_status(he);
  }
  std::lock_guard<std::mutex> g(f->mu);
  DevConsts& c = f->consts[dev];
  if (c.ntt) {
    (void)hipFree(p);
  } else {
    c.ntt = (uint64_t*)p;
  }
  *out = c.ntt;
  return GFP_OK;
}

// Transforms of the entries w^j (scaled by sm), j < cnt, for the FFT-based
// twiddle product (3k u64 per entry).
void build_spec_table(const gfp_field* f, const Big& wm, uint64_t cnt, std::vector<uint64_t>& out,
                      const Big* sm = nullptr) {
  const uint32_t k = f->k;
  uint64_t q[3], th[3];
  ntt_primes(k, q, th);
  out.assign(cnt * 3 * k, 0);
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (cnt < 1024) nth = 1;
  const uint64_t chunk = (cnt + nth - 1) / nth;
  std::vector<std::thread> ths;
  for (unsigned t = 0; t < nth; ++t) {
    const uint64_t lo = t * chunk, hi = std::min(cnt, lo + chunk);
    if (lo >= hi) break;
    ths.emplace_back([&, lo, hi]() {
      const Mont& M = *f->mont;
      Big acc = M.pow(wm, Big(lo));
      if (sm) acc = M.mmul(acc, *sm);
      std::vector<uint64_t> dg(k);
      for (uint64_t j = lo; j < hi; ++j) {
        to_digits(f, M.from(acc), dg.data());
        ntt_spectrum(k, q, th, dg.data(), &out[j * 3 * k]);
        acc = M.mmul(acc, wm);
      }
    });
  }
  for (auto& x : ths) x.join();
}

// The tables of get_tables plus, for the FFT-based twiddle product (k >= 32),
// their transforms (built and uploaded on the first call for n on the
// device, without the field lock held).
int get_spec_tables(gfp_field* f, uint64_t n, const DevTables** out) {
  if (f->k < 32) return GFP_EUNSUPPORTED;
  int rc = get_tables(f, n, out);
  if (rc != GFP_OK) return rc;
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return hip_status(he);
  {
    std::lock_guard<std::mutex> g(f->mu);
    if ((*out)->fwd_spec) return GFP_OK;
  }
  const uint64_t cnt = n / (2ull * f->k);
  const Mont& M = *f->mont;
  const Big ninv_m = M.pow(M.to(Big(n)), gfp::sub(f->p, Big(2)));
  DevTables sp;
  std::vector<uint64_t> host;
  build_spec_table(f, root_mont(f, n, false), cnt, host);
  rc = upload(host, &sp.fwd_spec);
  if (rc == GFP_OK) {
    build_spec_table(f, root_mont(f, n, true), cnt, host);
    rc = upload(host, &sp.inv_spec);
  }
  if (rc == GFP_OK && n >= 4ull * f->k * f->k) {
    build_spec_table(f, root_mont(f, n / (2ull * f->k), false), cnt, host);
    rc = upload(host, &sp.fwd2_spec);
    if (rc == GFP_OK) {
      build_spec_table(f, root_mont(f, n / (2ull * f->k), true), cnt, host);
      rc = upload(host, &sp.inv2_spec);
    }
  }
  if (rc == GFP_OK && scale_in_tables(f, log2_exact(n))) {
    build_spec_table(f, root_mont(f, n, true), cnt, host, &ninv_m);
    rc = upload(host, &sp.inv_s_spec);
    if (rc == GFP_OK && n >= 4ull * f->k * f->k) {
      build_spec_table(f, root_mont(f, n / (2ull * f->k), true), cnt, host, &ninv_m);
      rc = upload(host, &sp.inv2_s_spec);
    }
  }
  if (rc != GFP_OK) {
    free_tables(sp);
    return rc;
  }
  std::lock_guard<std::mutex> g(f->mu);
  DevTables& t = f->tables[std::make_pair(dev, n)];
  if (t.fwd_spec) {  // another thread built them meanwhile
    free_tables(sp);
  } else {
    t.fwd_spec = sp.fwd_spec;
    t.inv_spec = sp.inv_spec;
    t.fwd2_spec = sp.fwd2_spec;
    t.inv2_spec = sp.inv2_spec;
    t.inv_s_spec = sp.inv_s_spec;
    t.inv2_s_spec = sp.inv2_s_spec;
  }
  *out = &t;
  return GFP_OK;
}

// Stream-ordered scratch when the caller passes no workspace.
struct Scratch {
  void* p = nullptr;
  hipStream_t st = nullptr;
  ~Scratch() {
    if (p) (void)hipFreeAsync(p, st);
  }
};

int get_workspace(void* ws, uint64_t ws_bytes, uint64_t need, hipStream_t st, Scratch& s, uint64_t** out) {
  if (ws) {
    if (ws_bytes < need) return GFP_EINVAL;
    *out = (uint64_t*)ws;
    return GFP_OK;
  }
  if (need == 0) {
    *out = nullptr;
    return GFP_OK;
  }
  hipError_t e = hipMallocAsync(&s.p, need, st);
  if (e != hipSuccess) return hip_status(e);
  s.st = st;
  *out = (uint64_t*)s.p;
  return GFP_OK;
}

// GFP_VALIDATE: GFP_EINVAL when any of the n elements of the digit-major
// vector x is not canonical (synchronises the stream).
int validate_input(const gfp_field* f, const uint64_t* x, uint64_t ld, uint64_t n, hipStream_t st) {
  if (!f->validate || n == 0) return GFP_OK;
  uint64_t bad = 0;
  const int rc = gfp_check_canonical(f, x, ld, n, st, &bad);
  if (rc != GFP_OK) return rc;
  return bad ? GFP_EINVAL : GFP_OK;
}

// Vector view for the pass scheduler: digit d of element i of vector v at
// base[v * vs + i * se + d * sd].
struct VecView {
  const uint64_t* p;
  uint64_t se, sd, vs;
};

// Run the e passes of nvec transforms of size n (log2n) from X to Y.
// Intermediate passes write element-major vectors (one element = k
// contiguous digits, so the strided element accesses of the following pass
// read whole 64- or 128-byte segments), alternating between W1 and W2 (each
// nvec * n elements); X is only read by pass 0.  `canonical`: the last pass
// writes the canonical encoding (else congruent digits in [0, 2^64)).  When
// Y aliases X and e == 1 the pass writes W1 and the result is copied.
// ---------------------------------------------------------------------------
// stage groupings (which passes share a launch)
// ---------------------------------------------------------------------------
// Batch class of a launch over nvec transforms: 0 (1), 1 (2..7), 2 (8..63), 3.
int batch_class(uint64_t nvec) { return nvec <= 1 ? 0 : nvec < 8 ? 1 : nvec < 64 ? 2 : 3; }

// Launch codes: 1 = one pass, 2 = two passes fused (two blocks per
// workgroup), 3 = two passes fused, eight blocks per workgroup ("wide").
// 4 = one pass whose twiddles are multiplied with the FFT-based product of
// section 3.3 (k >= 32).
enum { LC_ONE = 1, LC_PAIR = 2, LC_WIDE = 3, LC_NTT = 4 };
int code_passes(int c) { return (c == LC_ONE || c == LC_NTT) ? 1 : 2; }
char code_char(int c) { return c == LC_WIDE ? 'w' : c == LC_NTT ? 'n' : (char)('0' + c); }
int char_code(char c) {
  return c == '1' ? LC_ONE : c == '2' ? LC_PAIR : c == 'w' ? LC_WIDE : c == 'n' ? LC_NTT : 0;
}

// The plan covers the e radix-K passes (after the radix-R pass, if any).
bool plan_valid(const gfp_field* f, int log2n, int e, const std::vector<int>& plan) {
  const int lk = log2_exact(2ull * f->k);
  const int lr = log2n - e * lk;
  int s = 0;
  for (int c : plan) {
    if (c < LC_ONE || c > LC_NTT) return false;
    if (c == LC_NTT && f->k < 32) return false;
    if ((c == LC_PAIR || c == LC_WIDE) && !gfpk::span2_supported((int)f->k)) return false;
    if (c == LC_WIDE && !gfpk::wide_supported((int)f->k)) return false;
    if (s + code_passes(c) > e) return false;
    if (c == LC_WIDE && log2n - 2 * lk - lr - s * lk < 3) return false;  // 8 blocks per twiddle base
    s += code_passes(c);
  }
  return s == e;
}

std::string plan_text(const std::vector<int>& plan) {
  std::string t;
  for (int c : plan) t += code_char(c);
  return t;
}

// Untuned choice (k = 8), the fastest plans measured on MI355X for one
// transform (digit-major ends) and for the two forward transforms of a
// product (element-major); other k run one pass per launch.
std::vector<int> default_plan(const gfp_field* f, int log2n, int e, int layout) {
  std::vector<int> plan;
  if (f->k != 8) return std::vector<int>(e, LC_ONE);
  static const char* dm[] = {"", "1", "2", "12", "121", "w21"};
  static const char* em[] = {"", "1", "2", "12", "22", "w12"};
  if (e <= 5) {
    for (const char* c = (layout == GFP_LAYOUT_ELEMENT_MAJOR ? em : dm)[e]; *c; ++c) plan.push_back(char_code(*c));
    if (plan_valid(f, log2n, e, plan)) return plan;
    plan.clear();
  }
  int left = e;
  while (left > 0) {
    const int c = left >= 2 ? LC_PAIR : LC_ONE;
    plan.push_back(c);
    left -= code_passes(c);
  }
  return plan;
}

std::vector<int> plan_for(gfp_field* f, int log2n, int e, uint64_t nvec, int layout) {
  std::lock_guard<std::mutex> g(f->mu);
  auto it = f->plans.find(std::make_tuple(log2n, batch_class(nvec), layout));
  if (it != f->plans.end()) return it->second;
  return default_plan(f, log2n, e, layout);
}

// Launches of a transform: the radix-R pass (if any) and the plan's.
size_t launch_count(const gfp_field* f, int log2n, int e, const std::vector<int>& plan) {
  return plan.size() + (log2n != e * log2_exact(2ull * f->k) ? 1 : 0);
}

int view_layout(const VecView& X, const VecView& Y) {
  return (X.se == 1 || Y.se == 1) ? GFP_LAYOUT_DIGIT_MAJOR : GFP_LAYOUT_ELEMENT_MAJOR;
}

// While set (on this thread), run_transform_plan appends the pass arguments
// here instead of launching (the persistent batch turns them into records).
thread_local std::vector<gfpk::PassArgs>* t_record = nullptr;

// X2 (inverse only): the transform input is the pointwise product X X2, formed
// in the first launch (X2 has X's strides, element-major)
// in_len (k <= 16): elements of the input vectors at or past it are zero
// and the first launch does not read them.
int run_transform_plan(gfp_field* f, int log2n, int e, const std::vector<int>& plan, bool inverse, VecView X,
                       VecView Y, uint64_t nvec, bool canonical, uint64_t* W1, uint64_t* W2, hipStream_t st,
                       const uint64_t* X2 = nullptr, bool build_tables = true, uint64_t in_len = ~0ull) {
  const uint64_t n = 1ull << log2n;
  const uint64_t k = f->k;
  const DevTables* t = nullptr;
  int rc = get_tables(f, n, &t, build_tables);
  if (rc != GFP_OK) return rc;
  if (!plan_valid(f, log2n, e, plan)) return GFP_EINVAL;
  const uint64_t* ntt = nullptr;
  if (std::find(plan.begin(), plan.end(), (int)LC_NTT) != plan.end()) {
    if (build_tables) {
      rc = get_spec_tables(f, n, &t);
      if (rc == GFP_OK) rc = get_ntt(f, &ntt);
      if (rc != GFP_OK) return rc;
    } else {  // look up only: the transforms and constants must exist already
      int dev = 0;
      if (hipGetDevice(&dev) != hipSuccess) return GFP_EDEVICE;
      std::lock_guard<std::mutex> g(f->mu);
      auto it = f->consts.find(dev);
      if (!t->fwd_spec || it == f->consts.end() || !it->second.ntt) return GFP_ENOTREADY;
      ntt = it->second.ntt;
    }
  }
  const int lk = log2_exact(2ull * f->k);
  const int lr = log2n - e * lk;  // radix-R pass first when lr > 0
  // launch codes in order: 0 = the radix-R pass
  std::vector<int> codes;
  if (lr > 0) codes.push_back(0);
  codes.insert(codes.end(), plan.begin(), plan.end());
  const int nl = (int)codes.size();
  if (nl == 1 && X.p == Y.p) return GFP_EINVAL;  // a single launch cannot run in place
  const bool scale_tab = inverse && scale_in_tables(f, log2n);
  if (X2 && (!inverse || X.sd != 1 || scale_tab)) return GFP_EINVAL;
  VecView src = X;
  int s = 0;  // radix-K passes done
  for (int i = 0; i < nl; ++i) {
    VecView dst;
    if (i == nl - 1) {
      dst = Y;
    } else {
      dst.p = (((nl - 2 - i) % 2) == 0) ? W1 : W2;  // launch nl-2 -> W1, nl-3 -> W2, ...
      dst.se = k;
      dst.sd = 1;
      dst.vs = n * k;
    }
    gfpk::PassArgs p;
    p.in = src.p;
    p.se_in = src.se;
    p.sd_in = src.sd;
    p.out = const_cast<uint64_t*>(dst.p);
    p.se_out = dst.se;
    p.sd_out = dst.sd;
    p.log2n = log2n;
    p.ngroups = n >> lk;
    p.inverse = inverse;
    p.scale = inverse && i == 0 && !scale_tab;
    p.in2 = (i == 0) ? X2 : nullptr;
    p.in_len = (i == 0 && f->k <= 16) ? in_len : ~0ull;
    p.tw = p.scale ? t->ninv : (inverse ? t->inv : t->fwd);
    p.tw1 = inverse ? t->inv : t->fwd;
    p.tw2 = inverse ? t->inv2 : t->fwd2;
    p.twr1 = inverse ? t->inv_raw : t->fwd_raw;
    p.twr2 = inverse ? t->inv2_raw : t->fwd2_raw;
    p.staged = staged_twiddles(f, log2n, nvec);
    if (scale_tab && i == 1) {  // 1/n rides on this launch's twiddle tables
      p.tw = t->inv_s;
      p.tw2 = t->inv2_s;
    }
    if (codes[i] == LC_NTT) {
      p.ntt_mul = true;
      p.ntt = ntt;
      p.spec1 = (scale_tab && i == 1) ? t->inv_s_spec : (inverse ? t->inv_spec : t->fwd_spec);
      p.spec2 = (scale_tab && i == 1) ? t->inv2_s_spec : (inverse ? t->inv2_spec : t->fwd2_spec);
    }
    p.last = (i == nl - 1) && canonical;
    p.nvec = nvec;
    p.vin = src.vs;
    p.vout = dst.vs;
    if (codes[i] == 0) {
      p.log2ns = 0;
      p.radix_log2 = lr;
    } else {
      p.log2ns = lr + s * lk;
      p.span = code_passes(codes[i]);
      p.wide = codes[i] == LC_WIDE;
      s += p.span;
    }
    if (t_record) {
      t_record->push_back(p);
    } else {
      hipError_t he = gfpk::launch_pass((int)f->k, f->w, f->u, p, st);
      if (he != hipSuccess) return hip_status(he);
    }
    src = dst;
  }
  return GFP_OK;
}

int run_transform(gfp_field* f, int log2n, int e, bool inverse, VecView X, VecView Y, uint64_t nvec, bool canonical,
                  uint64_t* W1, uint64_t* W2, hipStream_t st, const uint64_t* X2 = nullptr,
                  uint64_t in_len = ~0ull) {
  return run_transform_plan(f, log2n, e, plan_for(f, log2n, e, nvec, view_layout(X, Y)), inverse, X, Y, nvec,
                            canonical, W1, W2, st, X2, true, in_len);
}

// no_alloc: ws is the static scratch (gfp_fft_noalloc); the tables must
// already exist, and nothing is allocated.
int transform_entry(const gfp_field* cf, uint64_t n, const uint64_t* x, uint64_t ldx, uint64_t* y, uint64_t ldy,
                    void* ws, uint64_t ws_bytes, void* stream, bool inverse, bool no_alloc = false) {
  gfp_field* f = const_cast<gfp_field*>(cf);
  if (!f || !x || !y) return GFP_EINVAL;
  if (!f->gpu_shape) return GFP_EUNSUPPORTED;
  int log2n, e;
  int rc = check_size(f, n, &log2n, &e);
  if (rc != GFP_OK) return rc;
  if (ldx < n || ldy < n) return GFP_EINVAL;
  if (x == y && ldx != ldy) return GFP_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const uint64_t need = 2ull * n * f->k * 8;
  if (no_alloc && (!ws || ws_bytes < need)) return GFP_EINVAL;
  if (!no_alloc) {
    rc = validate_input(f, x, ldx, n, st);
    if (rc != GFP_OK) return rc;
  }
  Scratch s;
  uint64_t* w = nullptr;
  rc = get_workspace(ws, ws_bytes, need, st, s, &w);
  if (rc != GFP_OK) return rc;
  VecView X{x, 1, ldx, 0}, Y{y, 1, ldy, 0};
  const std::vector<int> plan = plan_for(f, log2n, e, 1, GFP_LAYOUT_DIGIT_MAJOR);
  if (launch_count(f, log2n, e, plan) == 1 && x == y) {
    // one launch cannot run in place: transform into W2 (digit-major, ld n), copy back
    VecView T{w + n * f->k, 1, n, 0};
    rc = run_transform_plan(f, log2n, e, plan, inverse, X, T, 1, true, w, w, st, nullptr, !no_alloc);
    if (rc != GFP_OK) return rc;
    return hip_status(hipMemcpy2DAsync(y, ldy * 8, T.p, n * 8, n * 8, f->k, hipMemcpyDeviceToDevice, st));
  }
  return run_transform_plan(f, log2n, e, plan, inverse, X, Y, 1, true, w, w + n * f->k, st, nullptr, !no_alloc);
}

// ---------------------------------------------------------------------------
// polynomial products: one size class, a chunk of C requests
// ---------------------------------------------------------------------------
// Workspace per chunk: A (2C padded operands), F (2C transforms), W1, W2
// (2C each), all element-major vectors of n elements: 8 C n k words.
uint64_t chunk_words(uint64_t n, uint64_t k, uint64_t C) { return 8ull * C * n * k; }

struct PolyReq {
  const uint64_t* a;
  uint64_t la, lda;
  const uint64_t* b;
  uint64_t lb, ldb;
  uint64_t* c;
  uint64_t ldc;
};

// pad / unpad with descriptors passed by value (so graph capture keeps them)
// the first cols elements of each work vector (cols <= n)
int copy_in(gfp_field* f, const std::vector<gfpk::CopyDesc>& d, uint64_t* work, uint64_t n, uint64_t cols,
            hipStream_t st) {
  for (size_t i = 0; i < d.size(); i += gfpk::kCopyBatch) {
    const uint32_t cnt = (uint32_t)std::min<size_t>(gfpk::kCopyBatch, d.size() - i);
    hipError_t he = gfpk::launch_pad((int)f->k, d.data() + i, cnt, work + i * n * f->k, n, cols, st);
    if (he != hipSuccess) return hip_status(he);
  }
  return GFP_OK;
}

int copy_out(gfp_field* f, const std::vector<gfpk::CopyDesc>& d, const uint64_t* work, uint64_t n, hipStream_t st) {
  for (size_t i = 0; i < d.size(); i += gfpk::kCopyBatch) {
    const uint32_t cnt = (uint32_t)std::min<size_t>(gfpk::kCopyBatch, d.size() - i);
    uint64_t maxlen = 0;
    for (uint32_t j = 0; j < cnt; ++j) maxlen = std::max(maxlen, d[i + j].len);
    hipError_t he = gfpk::launch_unpad((int)f->k, d.data() + i, cnt, work + i * n * f->k, n, maxlen, st);
    if (he != hipSuccess) return hip_status(he);
  }
  return GFP_OK;
}

// Enqueue the products of C requests of transform size n = 2^log2n.
// Products over at least this many elements form the pointwise product in
// the first launch of the inverse transform (measured: 1-2% faster from
// 2^18 elements on, slower below, where that launch is latency bound).
constexpr uint64_t kFuseProductElems = 1ull << 18;

// dev_desc != nullptr: r is unused and the copies read their descriptors
// from device memory instead (dev_desc[0, 2C): the operands a then b,
// dev_desc[2C, 3C): the products), so the launches do not depend on the
// requests and a captured sequence serves any chunk of C requests.
int polymul_chunk(gfp_field* f, int log2n, int e, const PolyReq* r, uint64_t C, uint64_t* ws, hipStream_t st,
                  const gfpk::CopyDesc* dev_desc = nullptr) {
  const uint64_t n = 1ull << log2n, k = f->k;
  const uint64_t vw = n * k;  // words per vector
  uint64_t* A = ws;
  uint64_t* F = A + 2 * C * vw;
  uint64_t* W1 = F + 2 * C * vw;
  uint64_t* W2 = W1 + 2 * C * vw;
  std::vector<gfpk::CopyDesc> din, dout;
  // operand elements the forward transforms read: past the longest operand
  // everything is zero padding, which is neither written nor read (k <= 16;
  // with device descriptors the lengths are not known here)
  uint64_t cols = n;
  if (!dev_desc) {
    din.resize(2 * C);
    dout.resize(C);
    uint64_t longest = 0;
    for (uint64_t i = 0; i < C; ++i) {
      din[i] = gfpk::CopyDesc{r[i].a, nullptr, r[i].la, r[i].lda};
      din[C + i] = gfpk::CopyDesc{r[i].b, nullptr, r[i].lb, r[i].ldb};
      dout[i] = gfpk::CopyDesc{nullptr, r[i].c, r[i].la + r[i].lb - 1, r[i].ldc};
      longest = std::max(longest, std::max(r[i].la, r[i].lb));
    }
    // from 2^16 elements on (smaller products measured 1-2% slower with the
    // bounded first launch)
    if (k <= 16 && n >= (1ull << 16)) cols = std::min(n, longest);
  }
  auto copy_out_any = [&](const uint64_t* src) -> int {
    if (dev_desc) return hip_status(gfpk::launch_unpad_dev((int)k, dev_desc + 2 * C, (uint32_t)C, src, n, st));
    return copy_out(f, dout, src, n, st);
  };
  int rc = dev_desc ? hip_status(gfpk::launch_pad_dev((int)k, dev_desc, (uint32_t)(2 * C), A, n, st))
                    : copy_in(f, din, A, n, cols, st);
  // forward transforms of all 2C operands in one launch per pass; the last
  // pass leaves congruent (not canonical) digits for the pointwise product
  const VecView em{A, k, 1, vw}, fm{F, k, 1, vw};
  if (rc == GFP_OK) rc = run_transform(f, log2n, e, false, em, fm, 2 * C, false, W1, W2, st, nullptr, cols);
  if (rc != GFP_OK) return rc;
  if (C * n >= kFuseProductElems && !scale_in_tables(f, log2n)) {
    // inverse of the pointwise products F[i] F[C + i], formed in its first
    // launch, into A (free once the forward transforms are done)
    rc = run_transform(f, log2n, e, true, fm, em, C, true, W1, W2, st, F + C * vw);
    if (rc != GFP_OK) return rc;
    return copy_out_any(A);
  }
  // small chunks: the first inverse launch has too few groups to hide the
  // extra loads, so the product is a launch of its own (memory bound)
  gfpk::EwArgs ew;
  ew.op = GFP_OP_MUL;
  ew.x = F;
  ew.xse = k;
  ew.xsd = 1;
  ew.y = F + C * vw;
  ew.yse = k;
  ew.ysd = 1;
  ew.z = A;
  ew.zse = k;
  ew.zsd = 1;
  ew.n = C * n;  // C vectors back to back
  ew.s = 0;
  ew.cst = nullptr;
  hipError_t he = gfpk::launch_elementwise((int)k, f->w, f->u, ew, st);
  if (he != hipSuccess) return hip_status(he);
  rc = run_transform(f, log2n, e, true, em, fm, C, true, W1, W2, st);
  if (rc != GFP_OK) return rc;
  return copy_out_any(F);
}

int check_req(const gfp_field* f, const PolyReq& q) {
  if (!q.a || !q.b || !q.c || q.la == 0 || q.lb == 0) return GFP_EINVAL;
  if (q.lda < q.la || q.ldb < q.lb || q.ldc < q.la + q.lb - 1) return GFP_EINVAL;
  (void)f;
  return GFP_OK;
}

// Batched products: requests grouped by transform size; each group in
// chunks of at most `cap` requests whose workspace fits gfpk::kChunkBytes
// (or the whole group when smaller).

struct BatchPlan {
  struct Group {
    int log2n, e;
    std::vector<PolyReq> reqs;
    uint64_t cap;         // requests per chunk
    uint64_t ws_off = 0;  // its workspace region (words), used chunk after chunk
  };
  std::vector<Group> groups;  // ascending size
  uint64_t ws_words = 0;      // the regions of all groups, which run concurrently
  // Tail of the workspace, needed only by the persistent launch (tail_words
  // words from tail_off = ws_words): the work list of the
  // persistent launch (levels, records, copy descriptors, barrier counters).
  uint64_t tail_off = 0, tail_words = 0, nlevels = 0, nrecs = 0, ndesc = 0;
};

// Launches of one chunk in the persistent work list: pad, the forward
// passes, the pointwise product, the inverse passes, unpad.
uint64_t persist_levels_per_chunk(const gfp_field* f, int log2n, int e) {
  const int nl = e + (log2n != e * log2_exact(2ull * f->k) ? 1 : 0);
  return 2ull * nl + 3;
}
uint64_t align_words(uint64_t bytes) { return ((bytes + 255) & ~255ull) / 8; }

int plan_batch(gfp_field* f, uint32_t n, const gfp_polymul_desc* d, BatchPlan& plan) {
  if (!f || !d || n == 0) return GFP_EINVAL;
  if (!f->gpu_shape) return GFP_EUNSUPPORTED;
  std::map<int, size_t> index;
  for (uint32_t i = 0; i < n; ++i) {
    PolyReq q{d[i].a, d[i].la, d[i].ld_a, d[i].b, d[i].lb, d[i].ld_b, d[i].c, d[i].ld_c};
    int rc = check_req(f, q);
    if (rc != GFP_OK) return rc;
    uint64_t N;
    rc = gfp_polymul_size(f, q.la, q.lb, &N);
    if (rc != GFP_OK) return rc;
    int log2n, e;
    check_size(f, N, &log2n, &e);
    auto it = index.find(log2n);
    if (it == index.end()) {
      index[log2n] = plan.groups.size();
      plan.groups.push_back(BatchPlan::Group{log2n, e, {}, 0});
      it = index.find(log2n);
    }
    plan.groups[it->second].reqs.push_back(q);
  }
  std::sort(plan.groups.begin(), plan.groups.end(),
            [](const BatchPlan::Group& x, const BatchPlan::Group& y) { return x.log2n < y.log2n; });
  for (auto& g : plan.groups) {
    const uint64_t per = chunk_words(1ull << g.log2n, f->k, 1) * 8;
    g.cap = std::min<uint64_t>(g.reqs.size(), gfpk::chunk_cap(per));
    g.ws_off = plan.ws_words;
    plan.ws_words += chunk_words(1ull << g.log2n, f->k, g.cap);
    const uint64_t chunks = (g.reqs.size() + g.cap - 1) / g.cap;
    const uint64_t lv = chunks * persist_levels_per_chunk(f, g.log2n, g.e);
    plan.nlevels = std::max(plan.nlevels, lv);
    plan.nrecs += lv;
  }
  plan.ndesc = 3ull * n;
  plan.tail_off = plan.ws_words;
  plan.tail_words = align_words(plan.nlevels * sizeof(gfpk::PLevel)) + align_words(plan.nrecs * sizeof(gfpk::PRec)) +
                   align_words(plan.ndesc * sizeof(gfpk::CopyDesc)) + align_words(gfpk::kPersistSyncBytes);
  return GFP_OK;
}

int enqueue_group(gfp_field* f, const BatchPlan::Group& g, uint64_t* ws, hipStream_t st) {
  for (size_t i = 0; i < g.reqs.size(); i += g.cap) {
    const uint64_t C = std::min<uint64_t>(g.cap, g.reqs.size() - i);
    int rc = polymul_chunk(f, g.log2n, g.e, g.reqs.data() + i, C, ws + g.ws_off, st);
    if (rc != GFP_OK) return rc;
  }
  return GFP_OK;
}

// The size classes of a batch are independent: each runs on a side stream of
// its own, forked from `st` by an event and joined back into it, so that the
// small classes' launches overlap the large ones' instead of waiting behind
// them (under stream capture the forks become parallel graph branches).
int enqueue_batch(gfp_field* f, const BatchPlan& plan, uint64_t* ws, hipStream_t st) {
  if (plan.groups.size() == 1) return enqueue_group(f, plan.groups[0], ws, st);
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return hip_status(he);
  std::lock_guard<std::mutex> lk(f->side_mu);  // the side streams and events serve one enqueue at a time
  gfp_field::Side& sd = f->side[dev];
  while (sd.streams.size() < plan.groups.size()) {
    hipStream_t s2 = nullptr;
    hipEvent_t e2 = nullptr;
    he = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&e2, hipEventDisableTiming);
    if (he != hipSuccess) {
      if (s2) (void)hipStreamDestroy(s2);
      return hip_status(he);
    }
    sd.streams.push_back(s2);
    sd.joins.push_back(e2);
  }
  if (!sd.fork) {
    he = hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming);
    if (he != hipSuccess) return hip_status(he);
  }
  he = hipEventRecord(sd.fork, st);
  if (he != hipSuccess) return hip_status(he);
  int rc = GFP_OK;
  size_t forked = 0;
  for (size_t j = 0; j < plan.groups.size(); ++j) {
    he = hipStreamWaitEvent(sd.streams[j], sd.fork, 0);
    if (he != hipSuccess) {
      rc = hip_status(he);
      break;
    }
    ++forked;
    rc = enqueue_group(f, plan.groups[j], ws, sd.streams[j]);
    if (rc != GFP_OK) break;
  }
  // join every forked stream back, also after an error (a capture must end joined)
  for (size_t j = 0; j < forked; ++j) {
    he = hipEventRecord(sd.joins[j], sd.streams[j]);
    if (he == hipSuccess) he = hipStreamWaitEvent(st, sd.joins[j], 0);
    if (he != hipSuccess && rc == GFP_OK) rc = hip_status(he);
  }
  return rc;
}

// A record of the persistent work list for one pass launch.
int pass_record(const gfp_field* f, const gfpk::PassArgs& p, gfpk::PRec* r) {
  uint32_t kind = 0;
  uint64_t tiles = 0;
  if (!gfpk::persist_pass_kind((int)f->k, p, &kind, &tiles)) return GFP_EUNSUPPORTED;
  *r = gfpk::PRec{};
  r->kind = kind;
  r->log2n = p.log2n;
  r->log2ns = p.log2ns;
  r->lr = p.radix_log2;
  r->staged = p.staged ? 1 : 0;
  r->tiles = tiles;
  r->in = p.in;
  r->in2 = p.in2;
  r->se_in = p.se_in;
  r->sd_in = p.sd_in;
  r->out = p.out;
  r->se_out = p.se_out;
  r->sd_out = p.sd_out;
  r->tw = p.tw;
  r->tw1 = p.tw1;
  r->tw2 = p.tw2;
  r->twr1 = p.twr1;
  r->twr2 = p.twr2;
  r->ngroups = p.ngroups;
  r->nvec = p.nvec;
  r->vin = p.vin;
  r->vout = p.vout;
  return GFP_OK;
}

// Stage grouping of the persistent launch: k = 8 fuses pairs of passes (two
// blocks per 256-thread tile) from the first one on, leaving the last pass
// single (a fused last pair is slower, its twiddles being per group either
// way); e = 2 is one pair.  k = 16 runs single passes (its pairs need
// 512-thread workgroups).
std::vector<int> persist_plan(const gfp_field* f, int log2n, int e) {
  std::vector<int> plan;
  if (f->k != 8 || e < 2) return std::vector<int>(e, LC_ONE);
  if (e == 2) return std::vector<int>(1, LC_PAIR);
  int left = e;
  while (left >= 3) {
    plan.push_back(LC_PAIR);
    left -= 2;
  }
  while (left-- > 0) plan.push_back(LC_ONE);
  if (!plan_valid(f, log2n, e, plan)) return std::vector<int>(e, LC_ONE);
  return plan;
}

// The records of one chunk of C products of size 2^log2n (the launches of
// polymul_chunk with the persistent stage grouping and the pointwise product
// as a launch of its own), one per level, appended to seq.  dev_desc: its 3C copy
// descriptors in device memory (operands a, operands b, products).
int persist_chunk(gfp_field* f, int log2n, int e, uint64_t C, uint64_t* ws, const gfpk::CopyDesc* dev_desc,
                  std::vector<gfpk::PRec>& seq) {
  const uint64_t n = 1ull << log2n, k = f->k;
  const uint64_t vw = n * k;
  uint64_t* A = ws;
  uint64_t* F = A + 2 * C * vw;
  uint64_t* W1 = F + 2 * C * vw;
  uint64_t* W2 = W1 + 2 * C * vw;
  const uint64_t copy_tiles = (vw + 255) / 256;  // 256 words per tile
  const uint64_t ew_tiles = (C * n + 4 * (64 / k) - 1) / (4 * (64 / k));
  gfpk::PRec r{};
  r.kind = gfpk::PK_PAD;
  r.in = dev_desc;
  r.out = A;
  r.ngroups = n;
  r.nvec = 2 * C;
  r.tiles = 2 * C * copy_tiles;
  seq.push_back(r);
  const std::vector<int> plan = persist_plan(f, log2n, e);
  const VecView em{A, k, 1, vw}, fm{F, k, 1, vw};
  std::vector<gfpk::PassArgs> fwd, inv;
  t_record = &fwd;
  int rc = run_transform_plan(f, log2n, e, plan, false, em, fm, 2 * C, false, W1, W2, nullptr);
  if (rc == GFP_OK) {
    t_record = &inv;
    rc = run_transform_plan(f, log2n, e, plan, true, em, fm, C, true, W1, W2, nullptr);
  }
  t_record = nullptr;
  if (rc != GFP_OK) return rc;
  for (const auto& p : fwd) {
    rc = pass_record(f, p, &r);
    if (rc != GFP_OK) return rc;
    seq.push_back(r);
  }
  r = gfpk::PRec{};
  r.kind = gfpk::PK_MUL;
  r.in = F;
  r.in2 = F + C * vw;
  r.out = A;
  r.nvec = C * n;  // elements, C vectors back to back
  r.tiles = ew_tiles;
  seq.push_back(r);
  for (const auto& p : inv) {
    rc = pass_record(f, p, &r);
    if (rc != GFP_OK) return rc;
    seq.push_back(r);
  }
  r = gfpk::PRec{};
  r.kind = gfpk::PK_UNPAD;
  r.in = dev_desc + 2 * C;
  r.in2 = F;
  r.ngroups = n;
  r.nvec = C;
  const uint64_t e_tile = gfpk::kUnpadTileWords / k;  // elements per unpad tile
  r.tiles = C * ((n + e_tile - 1) / e_tile);
  seq.push_back(r);
  return GFP_OK;
}

// The whole batch as one cooperative launch over a work list (k <= 16): the
// chunks of each size class run level after level, the classes side by side
// (level j of every class in one grid-wide step).  The list and the zeroed
// barrier counters are copied into the workspace tail ahead of the launch,
// in stream order, from the field's pinned staging.
int enqueue_batch_persistent(gfp_field* f, const BatchPlan& plan, uint64_t* ws, hipStream_t st) {
  if (f->k > 16) return GFP_EUNSUPPORTED;
  int cap = 0;
  if (gfpk::persistent_capacity((int)f->k, f->w, f->u, &cap) != 0) return GFP_EDEVICE;
  if (cap <= 0) return GFP_EUNSUPPORTED;
  char* tail = reinterpret_cast<char*>(ws + plan.tail_off);
  const uint64_t lev_bytes = align_words(plan.nlevels * sizeof(gfpk::PLevel)) * 8;
  const uint64_t rec_bytes = align_words(plan.nrecs * sizeof(gfpk::PRec)) * 8;
  const uint64_t desc_bytes = align_words(plan.ndesc * sizeof(gfpk::CopyDesc)) * 8;
  const gfpk::CopyDesc* ddesc = reinterpret_cast<const gfpk::CopyDesc*>(tail + lev_bytes + rec_bytes);
  std::vector<gfpk::CopyDesc> descs;
  descs.reserve(plan.ndesc);
  std::vector<std::vector<gfpk::PRec>> levels(plan.nlevels);
  for (const auto& g : plan.groups) {
    uint64_t lvl = 0;
    for (size_t i = 0; i < g.reqs.size(); i += g.cap) {
      const uint64_t C = std::min<uint64_t>(g.cap, g.reqs.size() - i);
      const size_t d0 = descs.size();
      for (uint64_t j = 0; j < C; ++j) {
        const PolyReq& q = g.reqs[i + j];
        descs.push_back(gfpk::CopyDesc{q.a, nullptr, q.la, q.lda});
      }
      for (uint64_t j = 0; j < C; ++j) {
        const PolyReq& q = g.reqs[i + j];
        descs.push_back(gfpk::CopyDesc{q.b, nullptr, q.lb, q.ldb});
      }
      for (uint64_t j = 0; j < C; ++j) {
        const PolyReq& q = g.reqs[i + j];
        descs.push_back(gfpk::CopyDesc{nullptr, q.c, q.la + q.lb - 1, q.ldc});
      }
      std::vector<gfpk::PRec> seq;
      int rc = persist_chunk(f, g.log2n, g.e, C, ws + g.ws_off, ddesc + d0, seq);
      if (rc != GFP_OK) return rc;
      for (const auto& r : seq) {
        if (lvl >= levels.size()) return GFP_EINVAL;  // cannot happen: plan_batch counted them
        levels[lvl++].push_back(r);
      }
    }
  }
  std::vector<gfpk::PLevel> lv;
  std::vector<gfpk::PRec> recs;
  uint64_t most = 0;
  for (auto& L : levels) {
    if (L.empty()) continue;
    gfpk::PLevel pl{(uint32_t)recs.size(), (uint32_t)L.size(), 0};
    for (auto& r : L) {
      r.tile0 = pl.tiles;
      pl.tiles += r.tiles;
      recs.push_back(r);
    }
    most = std::max(most, pl.tiles);
    lv.push_back(pl);
  }
  if (lv.size() > plan.nlevels || recs.size() > plan.nrecs || descs.size() > plan.ndesc) return GFP_EINVAL;
  // the barrier counters (zeros) travel with the list
  std::vector<char> host(lev_bytes + rec_bytes + desc_bytes + gfpk::kPersistSyncBytes, 0);
  memcpy(host.data(), lv.data(), lv.size() * sizeof(gfpk::PLevel));
  memcpy(host.data() + lev_bytes, recs.data(), recs.size() * sizeof(gfpk::PRec));
  memcpy(host.data() + lev_bytes + rec_bytes, descs.data(), descs.size() * sizeof(gfpk::CopyDesc));
  // through pinned staging: wait until the previous copy from it is done,
  // refill it, copy in stream order and mark the copy
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return hip_status(he);
  {
    std::lock_guard<std::mutex> lk(f->stage_mu);
    gfp_field::Stage& sg = f->stage[dev];
    if (!sg.done) {
      he = hipEventCreateWithFlags(&sg.done, hipEventDisableTiming);
      if (he != hipSuccess) {
        sg.done = nullptr;
        return hip_status(he);
      }
    } else {
      he = hipEventSynchronize(sg.done);
      if (he != hipSuccess) return hip_status(he);
    }
    if (sg.bytes < host.size()) {
      if (sg.host) (void)hipHostFree(sg.host);
      sg.host = nullptr;
      sg.bytes = 0;
      he = hipHostMalloc(&sg.host, host.size(), hipHostMallocDefault);
      if (he != hipSuccess) {
        sg.host = nullptr;
        return hip_status(he);
      }
      sg.bytes = host.size();
    }
    memcpy(sg.host, host.data(), host.size());
    he = hipMemcpyAsync(tail, sg.host, host.size(), hipMemcpyHostToDevice, st);
    if (he == hipSuccess) he = hipEventRecord(sg.done, st);
    if (he != hipSuccess) return hip_status(he);
  }
  const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)cap, most);
  return hip_status(gfpk::launch_persistent(
      (int)f->k, f->w, f->u, reinterpret_cast<const gfpk::PLevel*>(tail), (uint32_t)lv.size(),
      reinterpret_cast<const gfpk::PRec*>(tail + lev_bytes),
      reinterpret_cast<uint32_t*>(tail + lev_bytes + rec_bytes + desc_bytes), grid, st));
}

uint64_t hash_bytes(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;  // FNV-1a
  return h;
}

}  // namespace

namespace gfpk {
int prepare_tables(const gfp_field* f, uint64_t n) {
  const DevTables* t = nullptr;
  return get_tables(const_cast<gfp_field*>(f), n, &t);
}

int transform_noalloc(const gfp_field* f, uint64_t n, int inverse, const uint64_t* x, uint64_t ldx, uint64_t* y,
                      uint64_t ldy, void* scratch, uint64_t scratch_bytes, void* stream) {
  return transform_entry(f, n, x, ldx, y, ldy, scratch, scratch_bytes, stream, inverse != 0, true);
}

uint64_t polymul_chunk_bytes(const gfp_field* f, uint64_t n, uint64_t C) { return chunk_words(n, f->k, C) * 8; }

int capture_polymul_chunk(const gfp_field* cf, uint64_t n, uint64_t C, uint64_t* ws, const CopyDesc* dev_desc,
                          hipStream_t st, hipGraphExec_t* out) {
  gfp_field* f = const_cast<gfp_field*>(cf);
  if (!f || !ws || !dev_desc || !out || C == 0 || !st) return GFP_EINVAL;
  if (!f->gpu_shape) return GFP_EUNSUPPORTED;
  int log2n, e;
  int rc = check_size(f, n, &log2n, &e);
  if (rc != GFP_OK) return rc;
  const DevTables* t = nullptr;
  rc = get_tables(f, n, &t);  // outside the capture: building them synchronises
  if (rc != GFP_OK) return rc;
  hipError_t he = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (he != hipSuccess) return hip_status(he);
  rc = polymul_chunk(f, log2n, e, nullptr, C, ws, st, dev_desc);
  hipGraph_t g = nullptr;
  he = hipStreamEndCapture(st, &g);
  if (rc != GFP_OK || he != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rc != GFP_OK ? rc : hip_status(he);
  }
  he = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return hip_status(he);
}
}  // namespace gfpk

extern "C" {

int gfp_field_create(uint32_t k, uint64_t r, gfp_field** out) {
  if (!out) return GFP_EINVAL;
  *out = nullptr;
  if (k < 2 || (k & (k - 1)) || k > 64 || r < 2 || (r & 1)) return GFP_EINVAL;
  gfp_field* f = new (std::nothrow) gfp_field();
  if (!f) return GFP_ENOMEM;
  f->k = k;
  f->r = r;
  const char* v = getenv("GFP_VALIDATE");
  f->validate = v && *v && strcmp(v, "0") != 0;
  const char* ht = getenv("GFP_HOST_TABLES");
  f->host_tables = ht && *ht && strcmp(ht, "0") != 0;
  // r = 2^w + 2^u (u > 0), or r = 2^w - 2^-u (u < 0) ?
  if (__builtin_popcountll(r) == 2) {
    f->u = __builtin_ctzll(r);
    f->w = 63 - __builtin_clzll(r);
  } else {
    const int lo = __builtin_ctzll(r);
    const unsigned __int128 up = (unsigned __int128)r + ((unsigned __int128)1 << lo);
    if ((up & (up - 1)) == 0 && up <= ((unsigned __int128)1 << 63)) {
      f->u = -lo;
      f->w = 63 - __builtin_clzll((uint64_t)up);
    }
  }
  f->gpu_shape = f->w >= 0 && gfpk::shape_supported((int)k, f->w, f->u);
  Big rk(1);
  for (uint32_t i = 0; i < k; ++i) rk = gfp::mul_small(rk, r);
  f->pm1 = rk;
  f->p = gfp::add(rk, Big(1));
  f->mont.reset(new Mont(f->p));
  if (!gfp::bpsw(f->p)) {
    delete f;
    return GFP_ENOTPRIME;
  }
  f->log2max = k * (uint32_t)__builtin_ctzll(r);  // v2(r^k)
  // smallest quadratic non-residue h (Euler's criterion)
  const Mont& M = *f->mont;
  Big half = gfp::shr(f->pm1, 1);
  Big minus_one = M.to(f->pm1);
  uint64_t h = 2;
  for (;; ++h) {
    Big x = M.pow(M.to(Big(h)), half);
    if (gfp::cmp(x, minus_one) == 0) break;
  }
  f->h_mont = M.to(Big(h));
  // Alg. 1: a = g^(n/2k) = h^((p-1)/2k) for every n; smallest j with a^j = r
  Big a = M.pow(f->h_mont, gfp::shr(f->pm1, (unsigned)__builtin_ctz(2 * k)));
  Big rm = M.to(Big(r));
  Big b = a;
  uint64_t j = 1;
  while (gfp::cmp(b, rm) != 0 && j <= 4 * k) {
    b = M.mmul(b, a);
    ++j;
  }
  if (j > 4 * k) {  // cannot happen for prime p: a and r are both primitive 2k-th roots
    delete f;
    return GFP_EINVAL;
  }
  f->j1 = j;
  *out = f;
  return GFP_OK;
}

int gfp_field_destroy(gfp_field* f) {
  if (!f) return GFP_OK;
  int dev = 0;
  (void)hipGetDevice(&dev);
  for (auto& kv : f->tables) {
    (void)hipSetDevice(kv.first.first);
    free_tables(kv.second);
  }
  for (auto& kv : f->consts) {
    (void)hipSetDevice(kv.first);
    (void)hipFree(kv.second.one);
    (void)hipFree(kv.second.ntt);
  }
  for (auto& kv : f->graphs) {
    (void)hipGraphExecDestroy(kv.second.exec);
    (void)hipEventDestroy(kv.second.done);
  }
  for (auto& kv : f->side) {
    (void)hipSetDevice(kv.first);
    for (hipStream_t s2 : kv.second.streams) (void)hipStreamDestroy(s2);
    for (hipEvent_t e2 : kv.second.joins) (void)hipEventDestroy(e2);
    if (kv.second.fork) (void)hipEventDestroy(kv.second.fork);
  }
  for (auto& kv : f->stage) {
    (void)hipSetDevice(kv.first);
    if (kv.second.done) {
      (void)hipEventSynchronize(kv.second.done);
      (void)hipEventDestroy(kv.second.done);
    }
    if (kv.second.host) (void)hipHostFree(kv.second.host);
  }
  if (!f->tables.empty() || !f->consts.empty() || !f->side.empty() || !f->stage.empty()) (void)hipSetDevice(dev);
  delete f;
  return GFP_OK;
}

int gfp_field_info(const gfp_field* f, uint32_t* k, uint64_t* r, uint32_t* log2_max_n) {
  if (!f) return GFP_EINVAL;
  if (k) *k = f->k;
  if (r) *r = f->r;
  if (log2_max_n) *log2_max_n = f->log2max;
  return GFP_OK;
}

int gfp_root_of_unity(const gfp_field* f, uint64_t n, int inverse, uint64_t* digits) {
  if (!f || !digits) return GFP_EINVAL;
  const int lg = log2_exact(n);
  if (lg < 0 || n < 2ull * f->k || (uint64_t)lg > f->log2max) return GFP_EINVAL;
  Big w = f->mont->from(root_mont(f, n, inverse != 0));
  to_digits(f, w, digits);
  return GFP_OK;
}

int gfp_fft_workspace_size(const gfp_field* f, uint64_t n, uint64_t* bytes) {
  if (!f || !bytes) return GFP_EINVAL;
  int log2n, e;
  int rc = check_size(f, n, &log2n, &e);
  if (rc != GFP_OK) return rc;
  *bytes = 2ull * n * f->k * 8;
  return GFP_OK;
}

int gfp_fft_forward(const gfp_field* f, uint64_t n, const uint64_t* x, uint64_t ld_x, uint64_t* y, uint64_t ld_y,
                    void* workspace, uint64_t ws_bytes, void* stream) {
  return transform_entry(f, n, x, ld_x, y, ld_y, workspace, ws_bytes, stream, false);
}

int gfp_fft_inverse(const gfp_field* f, uint64_t n, const uint64_t* x, uint64_t ld_x, uint64_t* y, uint64_t ld_y,
                    void* workspace, uint64_t ws_bytes, void* stream) {
  return transform_entry(f, n, x, ld_x, y, ld_y, workspace, ws_bytes, stream, true);
}

int gfp_fft_pass(const gfp_field* cf, uint64_t n, int s, int inverse, int flags, const uint64_t* x, uint64_t ld_x,
                 uint64_t* y, uint64_t ld_y, void* stream) {
  gfp_field* f = const_cast<gfp_field*>(cf);
  if (!f || !x || !y || x == y) return GFP_EINVAL;
  if (!f->gpu_shape) return GFP_EUNSUPPORTED;
  int log2n, e;
  int rc = check_size(f, n, &log2n, &e);
  if (rc != GFP_OK) return rc;
  const int lk = log2_exact(2ull * f->k);
  const int lr = log2n - e * lk;
  const int total = e + (lr > 0 ? 1 : 0);  // passes: the radix-R one first, if any
  if (s < 0 || s >= total || (flags & ~31)) return GFP_EINVAL;
  const bool radix_r = lr > 0 && s == 0;
  const int sk = s - (lr > 0 ? 1 : 0);  // index among the radix-K passes
  const bool wide = (flags & GFP_PASS_WIDE) != 0;
  const int span = (wide || (flags & GFP_PASS_PAIR)) ? 2 : 1;
  if (span == 2 && (radix_r || s + 1 >= total || !gfpk::span2_supported((int)f->k))) return GFP_EINVAL;
  if (wide && !gfpk::wide_supported((int)f->k)) return GFP_EINVAL;
  const bool nttm = (flags & GFP_PASS_NTT) != 0;
  if (nttm && (f->k < 32 || span != 1 || radix_r)) return GFP_EINVAL;
  if (wide && log2n - 2 * lk - lr - sk * lk < 3) return GFP_EINVAL;
  const bool in_em = (flags & GFP_PASS_IN_ELEMENT_MAJOR) != 0;
  const bool out_em = (flags & GFP_PASS_OUT_ELEMENT_MAJOR) != 0;
  if ((!in_em && ld_x < n) || (!out_em && ld_y < n)) return GFP_EINVAL;
  const DevTables* t = nullptr;
  rc = nttm ? get_spec_tables(f, n, &t) : get_tables(f, n, &t);
  if (rc != GFP_OK) return rc;
  gfpk::PassArgs p;
  if (nttm) {
    rc = get_ntt(f, &p.ntt);
    if (rc != GFP_OK) return rc;
  }
  p.in = x;
  p.se_in = in_em ? f->k : 1;
  p.sd_in = in_em ? 1 : ld_x;
  p.out = y;
  p.se_out = out_em ? f->k : 1;
  p.sd_out = out_em ? 1 : ld_y;
  p.log2n = log2n;
  p.log2ns = radix_r ? 0 : lr + sk * lk;
  p.radix_log2 = radix_r ? lr : 0;
  p.ngroups = n >> lk;
  p.inverse = inverse != 0;
  const bool scale_tab = p.inverse && scale_in_tables(f, log2n);
  p.scale = p.inverse && s == 0 && !scale_tab;
  p.tw = p.scale ? t->ninv : (p.inverse ? t->inv : t->fwd);
  p.tw1 = p.inverse ? t->inv : t->fwd;
  p.tw2 = p.inverse ? t->inv2 : t->fwd2;
  p.twr1 = p.inverse ? t->inv_raw : t->fwd_raw;
  p.twr2 = p.inverse ? t->inv2_raw : t->fwd2_raw;
  p.staged = staged_twiddles(f, log2n, 1);
  if (scale_tab && s == 1) {
    p.tw = t->inv_s;
    p.tw2 = t->inv2_s;
  }
  if (nttm) {
    p.ntt_mul = true;
    p.spec1 = (scale_tab && s == 1) ? t->inv_s_spec : (p.inverse ? t->inv_spec : t->fwd_spec);
    p.spec2 = (scale_tab && s == 1) ? t->inv2_s_spec : (p.inverse ? t->inv2_spec : t->fwd2_spec);
  }
  p.span = span;
  p.wide = wide;
  p.last = (s + span - 1 == total - 1);
  return hip_status(gfpk::launch_pass((int)f->k, f->w, f->u, p, (hipStream_t)stream));
}

int gfp_polymul_size(const gfp_field* f, uint64_t la, uint64_t lb, uint64_t* n) {
  if (!f || !n || la == 0 || lb == 0) return GFP_EINVAL;
  const uint64_t need = la + lb - 1;
  uint64_t N = 2ull * f->k;
  while (N < need) {
    if (N > (1ull << kMaxLog2N)) return GFP_EUNSUPPORTED;
    N *= 2;
  }
  int log2n, e;
  int rc = check_size(f, N, &log2n, &e);
  if (rc != GFP_OK) return rc;
  *n = N;
  return GFP_OK;
}

int gfp_polymul_workspace_size(const gfp_field* f, uint64_t la, uint64_t lb, uint64_t* bytes) {
  if (!bytes) return GFP_EINVAL;
  uint64_t N;
  int rc = gfp_polymul_size(f, la, lb, &N);
  if (rc != GFP_OK) return rc;
  *bytes = chunk_words(N, f->k, 1) * 8;
  return GFP_OK;
}

int gfp_polymul(const gfp_field* cf, const uint64_t* a, uint64_t la, uint64_t ld_a, const uint64_t* b, uint64_t lb,
                uint64_t ld_b, uint64_t* c, uint64_t ld_c, void* workspace, uint64_t ws_bytes, void* stream) {
  gfp_field* f = const_cast<gfp_field*>(cf);
  if (!f) return GFP_EINVAL;
  PolyReq q{a, la, ld_a, b, lb, ld_b, c, ld_c};
  int rc = check_req(f, q);
  if (rc != GFP_OK) return rc;
  if (!f->gpu_shape) return GFP_EUNSUPPORTED;
  uint64_t N;
  rc = gfp_polymul_size(f, la, lb, &N);
  if (rc != GFP_OK) return rc;
  int log2n, e;
  check_size(f, N, &log2n, &e);
  hipStream_t st = (hipStream_t)stream;
  rc = validate_input(f, a, ld_a, la, st);
  if (rc == GFP_OK) rc = validate_input(f, b, ld_b, lb, st);
  if (rc != GFP_OK) return rc;
  Scratch s;
  uint64_t* w = nullptr;
  rc = get_workspace(workspace, ws_bytes, chunk_words(N, f->k, 1) * 8, st, s, &w);
  if (rc != GFP_OK) return rc;
  return polymul_chunk(f, log2n, e, &q, 1, w, st);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// integer products (section 1: an integer product is a polynomial product
// evaluated at a power of two)
// ---------------------------------------------------------------------------
namespace {

struct BigintPlan {
  uint64_t b;   // chunk bits
  int ua;       // r = 2^ua d, d = 2^(w - ua) +- 1
  uint64_t d;
  uint64_t la, lb, lc, nw, N;
  int log2n, e;
  // workspace offsets in words
  uint64_t oA, oB, oC, oPoly, oE, oLo, oHi, oBytes;
  uint64_t words;
};

int plan_bigint(const gfp_field* f, uint64_t na, uint64_t nb, BigintPlan& p) {
  if (!f || na == 0 || nb == 0) return GFP_EINVAL;
  if (!f->gpu_shape) return GFP_EUNSUPPORTED;
  // r = 2^ua d with d = 2^(w - ua) + 1 (u > 0) or 2^(w - ua) - 1 (u < 0)
  p.ua = f->u < 0 ? -f->u : f->u;
  p.d = (1ull << (f->w - p.ua)) + (f->u < 0 ? -1ll : 1ll);
  // r > 2^we; the coefficients of the product, C_m < min(la, lb) 2^(2b) with
  // min(la, lb) <= 64 min(na, nb), must stay below p > r^k > 2^(k we)
  const uint64_t we = (uint64_t)(f->u < 0 ? f->w - 1 : f->w);
  uint64_t lg = 1;
  while ((1ull << lg) < 64 * std::min(na, nb)) ++lg;
  const int64_t room = (int64_t)(f->k * we) - 2 - (int64_t)lg;
  if (room < 2) return GFP_EUNSUPPORTED;
  p.b = std::min<uint64_t>((uint64_t)(room / 2), (uint64_t)gfpk::bigint_max_chunk_bits());
  if (2 * p.b + lg + 64 > 64 * gfpk::bigint_eval_words()) return GFP_EUNSUPPORTED;
  p.la = (64 * na + p.b - 1) / p.b;
  p.lb = (64 * nb + p.b - 1) / p.b;
  p.lc = p.la + p.lb - 1;
  p.nw = na + nb;
  int rc = gfp_polymul_size(f, p.la, p.lb, &p.N);
  if (rc != GFP_OK) return rc;
  check_size(f, p.N, &p.log2n, &p.e);
  const uint64_t k = f->k;
  p.oA = 0;
  p.oB = p.oA + k * p.la;
  p.oC = p.oB + k * p.lb;
  p.oPoly = p.oC + k * p.lc;
  p.oE = p.oPoly + chunk_words(p.N, k, 1);
  p.oLo = p.oE + p.lc * gfpk::bigint_eval_words();
  p.oHi = p.oLo + p.nw;
  p.oBytes = p.oHi + p.nw;  // flags (nw bytes), block aggregates and carries (2 bytes per block)
  const uint64_t nbk = gfpk::bigint_scan_blocks(p.nw);
  p.words = p.oBytes + (p.nw + 2 * nbk + 7) / 8;
  return GFP_OK;
}

}  // namespace

extern "C" {

int gfp_bigint_mul_workspace_size(const gfp_field* f, uint64_t na, uint64_t nb, uint64_t* bytes) {
  if (!bytes) return GFP_EINVAL;
  BigintPlan p;
  int rc = plan_bigint(f, na, nb, p);
  if (rc != GFP_OK) return rc;
  *bytes = p.words * 8;
  return GFP_OK;
}

int gfp_bigint_mul(const gfp_field* cf, const uint64_t* a, uint64_t na, const uint64_t* b, uint64_t nb, uint64_t* c,
                   void* workspace, uint64_t ws_bytes, void* stream) {
  gfp_field* f = const_cast<gfp_field*>(cf);
  if (!a || !b || !c) return GFP_EINVAL;
  BigintPlan p;
  int rc = plan_bigint(f, na, nb, p);
  if (rc != GFP_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  Scratch s;
  uint64_t* w = nullptr;
  rc = get_workspace(workspace, ws_bytes, p.words * 8, st, s, &w);
  if (rc != GFP_OK) return rc;
  const int k = (int)f->k;
  uint64_t* A = w + p.oA;
  uint64_t* B = w + p.oB;
  uint64_t* C = w + p.oC;
  hipError_t he = gfpk::launch_bigint_split(a, na, A, p.la, k, (int)p.b, p.ua, p.d, st);
  if (he == hipSuccess) he = gfpk::launch_bigint_split(b, nb, B, p.lb, k, (int)p.b, p.ua, p.d, st);
  if (he != hipSuccess) return hip_status(he);
  PolyReq q{A, p.la, p.la, B, p.lb, p.lb, C, p.lc};
  rc = polymul_chunk(f, p.log2n, p.e, &q, 1, w + p.oPoly, st);
  if (rc != GFP_OK) return rc;
  uint8_t* flags = (uint8_t*)(w + p.oBytes);
  uint8_t* agg = flags + p.nw;
  uint8_t* cin = agg + gfpk::bigint_scan_blocks(p.nw);
  he = gfpk::launch_bigint_combine(C, p.lc, k, (int)p.b, f->w, f->u, p.nw, w + p.oE, w + p.oLo, w + p.oHi, st);
  if (he == hipSuccess) he = gfpk::launch_bigint_carry(w + p.oLo, w + p.oHi, p.nw, c, flags, agg, cin, st);
  return hip_status(he);
}

}  // extern "C"

extern "C" {

int gfp_polymul_batched_workspace_size(const gfp_field* cf, uint32_t n, const gfp_polymul_desc* d, uint64_t* bytes) {
  if (!bytes) return GFP_EINVAL;
  BatchPlan plan;
  int rc = plan_batch(const_cast<gfp_field*>(cf), n, d, plan);
  if (rc != GFP_OK) return rc;
  *bytes = (plan.ws_words + plan.tail_words) * 8;  // enough for either path
  return GFP_OK;
}

int gfp_polymul_batched(const gfp_field* cf, uint32_t n, const gfp_polymul_desc* d, void* workspace, uint64_t ws_bytes,
                        int flags, void* stream) {
  gfp_field* f = const_cast<gfp_field*>(cf);
  if (flags & ~(GFP_BATCH_GRAPH | GFP_BATCH_PERSISTENT)) return GFP_EINVAL;
  if ((flags & GFP_BATCH_GRAPH) && (flags & GFP_BATCH_PERSISTENT)) return GFP_EINVAL;
  if ((flags & GFP_BATCH_PERSISTENT) && f && f->k > 16) return GFP_EUNSUPPORTED;
  BatchPlan plan;
  int rc = plan_batch(f, n, d, plan);
  if (rc != GFP_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  const bool graph = (flags & GFP_BATCH_GRAPH) != 0;
  if (graph && (!st || !workspace)) return GFP_EINVAL;
  for (uint32_t i = 0; f->validate && i < n; ++i) {
    rc = validate_input(f, d[i].a, d[i].ld_a, d[i].la, st);
    if (rc == GFP_OK) rc = validate_input(f, d[i].b, d[i].ld_b, d[i].lb, st);
    if (rc != GFP_OK) return rc;
  }
  // twiddle tables are uploaded synchronously: do it before any capture
  for (const auto& g : plan.groups) {
    const DevTables* t;
    rc = get_tables(f, 1ull << g.log2n, &t);
    if (rc != GFP_OK) return rc;
  }
  Scratch s;
  uint64_t* w = nullptr;
  const bool persistent = (flags & GFP_BATCH_PERSISTENT) != 0;
  rc = get_workspace(workspace, ws_bytes, (plan.ws_words + (persistent ? plan.tail_words : 0)) * 8, st, s, &w);
  if (rc != GFP_OK) return rc;
  if (flags & GFP_BATCH_PERSISTENT) return enqueue_batch_persistent(f, plan, w, st);
  if (!graph) return enqueue_batch(f, plan, w, st);

  int dev = 0;
  (void)hipGetDevice(&dev);
  std::string key;
  auto put = [&key](const void* p, size_t bytes) { key.append(reinterpret_cast<const char*>(p), bytes); };
  put(&n, sizeof(n));
  put(d, sizeof(gfp_polymul_desc) * n);
  put(&w, sizeof(w));
  put(&ws_bytes, sizeof(ws_bytes));
  put(&st, sizeof(st));
  put(&dev, sizeof(dev));
  uint64_t h = 0;
  // under f->mu: the cached graph for key, or nullptr
  auto find = [&]() -> gfp_field::Graph* {
    auto range = f->graphs.equal_range(h);
    for (auto it = range.first; it != range.second; ++it)
      if (it->second.key == key) return &it->second;
    return nullptr;
  };
  // under f->mu (so that an eviction cannot destroy the graph in between)
  auto launch = [&](gfp_field::Graph& g) -> int {
    g.seq = ++f->graph_seq;
    hipError_t he = hipGraphLaunch(g.exec, st);
    if (he == hipSuccess) he = hipEventRecord(g.done, st);
    return hip_status(he);
  };
  {
    std::lock_guard<std::mutex> lk(f->mu);
    put(&f->plan_gen, sizeof(f->plan_gen));  // a new plan means a new launch sequence
    h = hash_bytes(1469598103934665603ull, key.data(), key.size());
    if (gfp_field::Graph* g = find()) return launch(*g);
  }
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  {
    hipError_t he = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (he != hipSuccess) return hip_status(he);
    rc = enqueue_batch(f, plan, w, st);
    hipGraph_t g = nullptr;
    he = hipStreamEndCapture(st, &g);
    if (rc != GFP_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (he != hipSuccess) return hip_status(he);
    he = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (he != hipSuccess) {
      if (exec) (void)hipGraphExecDestroy(exec);
      return hip_status(he);
    }
  }
  gfp_field::Graph victim{std::string(), nullptr, nullptr, 0};
  {
    std::lock_guard<std::mutex> lk(f->mu);
    if (gfp_field::Graph* g = find()) {  // another thread captured the same list meanwhile
      (void)hipGraphExecDestroy(exec);
      (void)hipEventDestroy(done);
      return launch(*g);
    }
    if (f->graphs.size() >= kMaxGraphs) {
      auto old = f->graphs.begin();
      for (auto j = f->graphs.begin(); j != f->graphs.end(); ++j)
        if (j->second.seq < old->second.seq) old = j;
      victim = old->second;
      f->graphs.erase(old);
    }
    auto it = f->graphs.emplace(h, gfp_field::Graph{key, exec, done, 0});
    rc = launch(it->second);
  }
  if (victim.exec) {
    // out of the map, so no new launch; wait for its last one without the lock
    (void)hipEventSynchronize(victim.done);
    (void)hipGraphExecDestroy(victim.exec);
    (void)hipEventDestroy(victim.done);
  }
  return rc;
}

int gfp_elementwise(const gfp_field* cf, int op, const uint64_t* x, uint64_t ld_x, const uint64_t* y, uint64_t ld_y,
                    uint64_t* z, uint64_t ld_z, uint64_t n, int64_t s, const uint64_t* c_host, void* stream) {
  gfp_field* f = const_cast<gfp_field*>(cf);
  if (!f || !x || !z) return GFP_EINVAL;
  if (!f->gpu_shape) return GFP_EUNSUPPORTED;
  if (op < GFP_OP_ADD || op > GFP_OP_MUL_NTT) return GFP_EINVAL;
  const bool needs_y = (op == GFP_OP_ADD || op == GFP_OP_SUB || op == GFP_OP_MUL || op == GFP_OP_MUL_SCALE ||
                        op == GFP_OP_MUL_NTT);
  const bool needs_c = (op == GFP_OP_MUL_CONST || op == GFP_OP_MUL_SCALE);
  if (needs_y && !y) return GFP_EINVAL;
  if (needs_c && !c_host) return GFP_EINVAL;
  if (ld_x < n || ld_z < n || (needs_y && ld_y < n)) return GFP_EINVAL;
  if (n == 0) return GFP_OK;
  hipStream_t st = (hipStream_t)stream;
  int rc = validate_input(f, x, ld_x, n, st);
  if (rc == GFP_OK && needs_y) rc = validate_input(f, y, ld_y, n, st);
  if (rc != GFP_OK) return rc;
  const uint32_t* cst = nullptr;
  Scratch cs;
  if (needs_c) {
    // validate and stage the constant (stream-ordered, freed after use)
    std::vector<uint64_t> dg(c_host, c_host + f->k);
    bool canon = true;
    bool top_r = dg[f->k - 1] == f->r;
    for (uint32_t d = 0; d < f->k; ++d) {
      if (top_r ? (d + 1 < f->k && dg[d] != 0) : (dg[d] >= f->r)) canon = false;
    }
    if (!canon) return GFP_EINVAL;
    std::vector<uint32_t> host(gfpk::tw_words((int)f->k));
    make_entry(f->k, dg.data(), host.data());
    hipError_t he = hipMallocAsync(&cs.p, host.size() * 4, st);
    if (he != hipSuccess) return hip_status(he);
    cs.st = st;
    // the host vector must outlive the copy: copy synchronously with respect to the host
    he = hipMemcpyAsync(cs.p, host.data(), host.size() * 4, hipMemcpyHostToDevice, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return hip_status(he);
    cst = (const uint32_t*)cs.p;
  } else if (op == GFP_OP_MUL_POW_R) {
    int rc = get_one(f, &cst);
    if (rc != GFP_OK) return rc;
  } else if (op == GFP_OP_MUL_NTT) {
    const uint64_t* t = nullptr;
    int rc = get_ntt(f, &t);
    if (rc != GFP_OK) return rc;
    cst = reinterpret_cast<const uint32_t*>(t);
  }
  gfpk::EwArgs a;
  a.op = op;
  a.x = x;
  a.xse = 1;
  a.xsd = ld_x;
  a.y = needs_y ? y : x;
  a.yse = 1;
  a.ysd = needs_y ? ld_y : ld_x;
  a.z = z;
  a.zse = 1;
  a.zsd = ld_z;
  a.n = n;
  a.s = s;
  a.cst = cst;
  hipError_t he = gfpk::launch_elementwise((int)f->k, f->w, f->u, a, st);
  return hip_status(he);
}

int gfp_check_canonical(const gfp_field* f, const uint64_t* x, uint64_t ld_x, uint64_t n, void* stream,
                        uint64_t* bad) {
  if (!f || !bad || (n && !x) || ld_x < n) return GFP_EINVAL;
  *bad = 0;
  if (n == 0) return GFP_OK;
  hipStream_t st = (hipStream_t)stream;
  Scratch s;
  uint64_t* dev = nullptr;
  int rc = get_workspace(nullptr, 0, 8, st, s, &dev);
  if (rc != GFP_OK) return rc;
  hipError_t he = hipMemsetAsync(dev, 0, 8, st);
  if (he == hipSuccess) he = gfpk::launch_check_canonical(x, ld_x, n, (int)f->k, f->r, dev, st);
  if (he == hipSuccess) he = hipMemcpyAsync(bad, dev, 8, hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  return hip_status(he);
}

int gfp_plan_get(const gfp_field* cf, uint64_t n, uint64_t nvec, int layout, char* buf, uint32_t len) {
  gfp_field* f = const_cast<gfp_field*>(cf);
  if (!f || !buf || nvec == 0 || (layout != GFP_LAYOUT_DIGIT_MAJOR && layout != GFP_LAYOUT_ELEMENT_MAJOR))
    return GFP_EINVAL;
  int log2n, e;
  int rc = check_size(f, n, &log2n, &e);
  if (rc != GFP_OK) return rc;
  const std::string t = plan_text(plan_for(f, log2n, e, nvec, layout));
  if (len < t.size() + 1) return GFP_EINVAL;
  memcpy(buf, t.c_str(), t.size() + 1);
  return GFP_OK;
}

int gfp_plan_set(gfp_field* f, uint64_t n, uint64_t nvec, int layout, const char* text) {
  if (!f || nvec == 0 || (layout != GFP_LAYOUT_DIGIT_MAJOR && layout != GFP_LAYOUT_ELEMENT_MAJOR)) return GFP_EINVAL;
  int log2n, e;
  int rc = check_size(f, n, &log2n, &e);
  if (rc != GFP_OK) return rc;
  const auto key = std::make_tuple(log2n, batch_class(nvec), layout);
  if (!text || !*text) {
    std::lock_guard<std::mutex> g(f->mu);
    f->plans.erase(key);
    ++f->plan_gen;
    return GFP_OK;
  }
  std::vector<int> plan;
  for (const char* c = text; *c; ++c) {
    const int code = char_code(*c);
    if (!code) return GFP_EINVAL;
    plan.push_back(code);
  }
  if (!plan_valid(f, log2n, e, plan)) return GFP_EINVAL;
  std::lock_guard<std::mutex> g(f->mu);
  f->plans[key] = plan;
  ++f->plan_gen;
  return GFP_OK;
}

int gfp_tune(gfp_field* f, uint64_t n, uint64_t nvec, int layout, void* stream, char* best, uint32_t len,
             double* us) {
  if (!f || nvec == 0 || (layout != GFP_LAYOUT_DIGIT_MAJOR && layout != GFP_LAYOUT_ELEMENT_MAJOR)) return GFP_EINVAL;
  if (!f->gpu_shape) return GFP_EUNSUPPORTED;
  int log2n, e;
  int rc = check_size(f, n, &log2n, &e);
  if (rc != GFP_OK) return rc;
  const uint64_t words = nvec * n * f->k;
  if (words > (1ull << 30)) return GFP_EINVAL;  // 8 GiB per buffer
  // every sequence of launch codes the kernels support for this size
  std::vector<std::vector<int>> cands;
  std::vector<int> cur;
  std::function<void(int)> gen = [&](int s) {
    if (s == e) {
      if (plan_valid(f, log2n, e, cur)) cands.push_back(cur);
      return;
    }
    for (int c = LC_ONE; c <= LC_NTT; ++c) {
      if (s + code_passes(c) > e) continue;
      cur.push_back(c);
      gen(s + code_passes(c));
      cur.pop_back();
    }
  };
  gen(0);
  hipStream_t st = (hipStream_t)stream;
  const DevTables* t = nullptr;
  rc = get_tables(f, n, &t);
  if (rc != GFP_OK) return rc;
  uint64_t* buf = nullptr;
  if (hipMalloc((void**)&buf, 4 * words * 8) != hipSuccess) return GFP_ENOMEM;
  // canonical digits (every digit 0x5a5a5a5a5a5a5a5a < r) as input
  hipError_t he = hipMemsetD32Async(buf, 0x5a5a5a5au, 2 * words * 2, st);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (he == hipSuccess) he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  // digit-major: vector v's digit d at v n k + d n; element-major: v n k + i k + d
  const bool dm = layout == GFP_LAYOUT_DIGIT_MAJOR;
  const VecView X{buf, dm ? 1 : f->k, dm ? n : 1, n * f->k}, Y{buf + words, dm ? 1 : f->k, dm ? n : 1, n * f->k};
  uint64_t* W1 = buf + 2 * words;
  uint64_t* W2 = buf + 3 * words;
  double best_us = 0;
  std::vector<int> best_plan;
  for (const auto& plan : cands) {
    if (he != hipSuccess || rc != GFP_OK) break;
    for (int i = 0; i < 2 && rc == GFP_OK; ++i)
      rc = run_transform_plan(f, log2n, e, plan, false, X, Y, nvec, true, W1, W2, st);
    const int reps = 5;
    if (rc == GFP_OK) he = hipEventRecord(e0, st);
    for (int i = 0; i < reps && rc == GFP_OK && he == hipSuccess; ++i)
      rc = run_transform_plan(f, log2n, e, plan, false, X, Y, nvec, true, W1, W2, st);
    if (rc == GFP_OK && he == hipSuccess) he = hipEventRecord(e1, st);
    if (rc == GFP_OK && he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0;
    if (rc == GFP_OK && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    const double t_us = 1000.0 * ms / reps;
    if (rc == GFP_OK && he == hipSuccess && (best_plan.empty() || t_us < best_us)) {
      best_us = t_us;
      best_plan = plan;
    }
  }
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  if (rc != GFP_OK) return rc;
  if (he != hipSuccess) return hip_status(he);
  {
    std::lock_guard<std::mutex> g(f->mu);
    f->plans[std::make_tuple(log2n, batch_class(nvec), layout)] = best_plan;
    ++f->plan_gen;
  }
  if (us) *us = best_us;
  if (best) {
    const std::string t = plan_text(best_plan);
    if (len < t.size() + 1) return GFP_EINVAL;
    memcpy(best, t.c_str(), t.size() + 1);
  }
  return GFP_OK;
}

const char* gfp_strerror(int code) {
  switch (code) {
    case GFP_OK: return "ok";
    case GFP_EINVAL: return "invalid argument";
    case GFP_EUNSUPPORTED: return "unsupported field or size";
    case GFP_ENOMEM: return "out of memory";
    case GFP_EAGAIN: return "no capacity, try again";
    case GFP_EDEVICE: return "HIP device error";
    case GFP_ENOTPRIME: return "r^k + 1 is not a probable prime";
    case GFP_ECANCELED: return "request cancelled";
    case GFP_EPENDING: return "result not ready";
    case GFP_ENOTREADY: return "twiddle tables of this size not on the device yet";
    default: return "unknown error";
  }
}

}  // extern "C"

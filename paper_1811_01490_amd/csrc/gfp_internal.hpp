// Declarations shared by the host side (gfp_host.cpp) and the kernel
// launchers (gfp_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gfp.h"

namespace gfpk {

// Vector addressing: digit d of element i is at base[i * se + d * sd].
// Digit-major (the ABI's layout): se = 1, sd = ld.  Element-major (used
// between passes, one element = k contiguous digits): se = k, sd = 1.
struct PassArgs {
  const uint64_t* in;
  uint64_t se_in, sd_in;
  uint64_t* out;
  uint64_t se_out, sd_out;
  const uint32_t* tw;  // twiddle table (or the single scale entry when scale)
  int log2n;
  int log2ns;
  uint64_t ngroups;  // n / K
  bool inverse;
  bool scale;  // inverse pass 0: multiply every slot by tw[0] (1/n)
  bool last;   // canonical output
  uint64_t nvec = 1;  // transforms in this launch (same size)
  uint64_t vin = 0;   // u64 stride between the input vectors
  uint64_t vout = 0;  // u64 stride between the output vectors
  // span 2: passes log2ns / LOGK and the next one fused in one launch, the
  // stride permutation between them staged in LDS; tw1 is the table of the
  // second pass (tw the first pass's, or its scale entry), `last` applies
  // to the second pass.
  // radix_log2 > 0: the radix-R first pass (R = 2^radix_log2 < K, Ns = 1)
  // of a transform of size R K^e; span, wide and tw1 are then unused
  int radix_log2 = 0;
  int span = 1;
  bool wide = false;  // span 2 over 8 blocks per workgroup (needs N / (K^2 Ns) >= 8)
  const uint32_t* tw1 = nullptr;
  // table of w^(K i) (w^-(K i) for the inverse), i < N/K: the twiddles of
  // every radix-K pass but the last, without a rotation
  const uint32_t* tw2 = nullptr;
  // tw1 and tw2 as raw digits (k u64 per entry), k <= 16: the passes whose
  // groups take different twiddles stage them through LDS from these
  const uint64_t* twr1 = nullptr;
  const uint64_t* twr2 = nullptr;
  // per-group twiddles through the raw-digit tables and LDS (large
  // transforms) rather than whole limb-table entries read by every lane
  bool staged = false;
  // k >= 32, MODE_PLAIN passes: multiply the twiddles with the FFT-based
  // product (section 3.3) using their tabulated transforms (spec1 for the
  // table of tw, spec2 for tw2; 3k u64 per entry) and the constants ntt
  bool ntt_mul = false;
  const uint64_t* spec1 = nullptr;
  const uint64_t* spec2 = nullptr;
  const uint64_t* ntt = nullptr;
  // set with scale (inverse pass 0): the pass input is the pointwise product
  // in[i] in2[i] of two transforms; in2 has the strides of in and its digits
  // contiguous (sd_in 1), and the product is then multiplied by tw[0]
  const uint64_t* in2 = nullptr;
  // k <= 16, plain or scale passes: elements at or past in_len of each input
  // vector are zero and not read (the zero padding of a product's operands)
  uint64_t in_len = ~0ull;
};
// Whether two passes can share a launch for k (plan character '2'), and
// the wide variant over eight blocks per workgroup (plan character 'w').
bool span2_supported(int k);
bool wide_supported(int k);

struct EwArgs {
  int op;
  const uint64_t* x;
  uint64_t xse, xsd;
  const uint64_t* y;
  uint64_t yse, ysd;
  uint64_t* z;
  uint64_t zse, zsd;
  uint64_t n;
  int64_t s;
  const uint32_t* cst;  // one twiddle-layout entry (device)
};

// Copies between caller vectors (digit-major, ld) and padded element-major
// work vectors of n elements.  One descriptor per vector.
struct CopyDesc {
  const uint64_t* src;  // pad: caller vector; unpad: unused
  uint64_t* dst;        // unpad: caller vector; pad: unused
  uint64_t len;         // coefficients to copy (the rest of a padded vector is 0)
  uint64_t ld;          // caller row stride
};
// Descriptors travel as kernel arguments (by value, at most kCopyBatch per
// launch), so a captured graph holds its own copy of them.  Pad writes the
// first `cols` elements of each work vector (zeros past a descriptor's len);
// the rest stays unwritten, for a transform that reads at most cols
// elements (PassArgs::in_len).
constexpr uint32_t kCopyBatch = 48;
hipError_t launch_pad(int k, const CopyDesc* host_d, uint32_t nvec, uint64_t* work, uint64_t n, uint64_t cols,
                      hipStream_t st);
// maxlen: the largest len of the descriptors (at most n); k = 8, 16, 32, 64.
hipError_t launch_unpad(int k, const CopyDesc* host_d, uint32_t nvec, const uint64_t* work, uint64_t n,
                        uint64_t maxlen, hipStream_t st);
// The same with the descriptors in device memory (dev_desc[0, nvec), every
// len at most n).  Unpad moves tiles of kUnpadTileWords words (1024 / k
// elements) through LDS.
constexpr uint64_t kUnpadTileWords = 1024;
hipError_t launch_pad_dev(int k, const CopyDesc* dev_desc, uint32_t nvec, uint64_t* work, uint64_t n,
                          hipStream_t st);
hipError_t launch_unpad_dev(int k, const CopyDesc* dev_desc, uint32_t nvec, const uint64_t* work, uint64_t n,
                            hipStream_t st);

// integer products (gfp_bigint.hip)
hipError_t launch_bigint_split(const uint64_t* a, uint64_t na, uint64_t* A, uint64_t la, int k, int b, int ua,
                               uint64_t d, hipStream_t st);
hipError_t launch_bigint_combine(const uint64_t* C, uint64_t lc, int k, int b, int W, int U, uint64_t nw, uint64_t* E,
                                 uint64_t* lo, uint64_t* hi, hipStream_t st);
uint64_t bigint_eval_words();    // words per evaluated product coefficient
int bigint_max_chunk_bits();
uint64_t bigint_scan_blocks(uint64_t nw);
hipError_t launch_bigint_carry(const uint64_t* lo, const uint64_t* hi, uint64_t nw, uint64_t* c, uint8_t* flags,
                               uint8_t* agg, uint8_t* cin, hipStream_t st);

// count of non-canonical elements of a digit-major vector into *bad (device)
hipError_t launch_check_canonical(const uint64_t* x, uint64_t ld, uint64_t n, int k, uint64_t r, uint64_t* bad,
                                  hipStream_t st);

bool shape_supported(int k, int w, int u);
hipError_t launch_pass(int k, int w, int u, const PassArgs& p, hipStream_t st);
hipError_t launch_elementwise(int k, int w, int u, const EwArgs& a, hipStream_t st);

// ---- one persistent launch for a batch of products ---------------------------
// A batched product as one cooperative launch (k = 8 and 16): the launches
// the per-class path would make (pad, the single-pass transforms, the
// pointwise product, unpad) become records of a device work list grouped in
// levels; every workgroup walks the tiles (virtual blocks) of a level, then
// the grid synchronises before the next level.  Kinds of records:
enum PersistKind : uint32_t {
  PK_PAD = 0,          // copy-in: desc table `in` (CopyDesc), n = ngroups, nvec vectors into `out`
  PK_UNPAD = 1,        // copy-out: desc table `in`, n = ngroups, nvec vectors from `in2`
  PK_MUL = 2,          // elementwise product out = in * in2 over nvec elements (element-major)
  PK_PASS_FIRST = 3,   // k_pass <fwd, plain, not last, per group, w^j table> (first or last forward pass)
  PK_PASS_MID = 4,     // k_pass <fwd, plain, not last, uniform, w^(K i) table>
  PK_PASS_IMID = 5,    // k_pass <inv, plain, not last, uniform, w^(K i) table>
  PK_PASS_ILAST = 6,   // k_pass <inv, plain, last (canonical), per group>
  PK_PASS_ISCALE = 7,  // k_pass <inv, scale, not last>
  PK_PASS_ISCALE_LAST = 8,  // k_pass <inv, scale, last>
  PK_PASS_R_F = 9,     // k_pass_r <fwd, plain, radix 2^lr>
  PK_PASS_R_I = 10,    // k_pass_r <inv, scale, radix 2^lr>
  // fused pairs (k = 8, two blocks per tile): k_pass2 <inv, mode, last, T2B>
  PK_PAIR_F_T2 = 11,     // <fwd, plain, not last, second pass from the w^(K i) table>
  PK_PAIR_F = 12,        // <fwd, plain, not last, second pass the final one>
  PK_PAIR_I_T2 = 13,     // <inv, plain, not last, T2B>
  PK_PAIR_I_LAST = 14,   // <inv, plain, last>
  PK_PAIR_IS_T2 = 15,    // <inv, scale, not last, T2B>
  PK_PAIR_IS_LAST = 16,  // <inv, scale, last>
};

struct PRec {
  uint32_t kind;
  int32_t log2n, log2ns, lr;
  int32_t staged, pad0;
  uint64_t tile0;  // first tile of the record in its level
  uint64_t tiles;  // virtual blocks of the record
  const void* in;
  const uint64_t* in2;
  uint64_t se_in, sd_in;
  uint64_t* out;
  uint64_t se_out, sd_out;
  const uint32_t* tw;
  const uint32_t* tw1;  // fused pairs: the w^j table of the second pass
  const uint32_t* tw2;
  const uint64_t* twr1;
  const uint64_t* twr2;
  uint64_t ngroups, nvec, vin, vout;
};

struct PLevel {
  uint32_t rec0, nrec;  // records [rec0, rec0 + nrec)
  uint64_t tiles;       // total tiles of the level
};

// Kind and tile count of a pass launch (the variant launch_pass_t would
// pick) for k <= 16 single passes and k = 8 fused pairs; false if the
// persistent launch does not carry it (wide pairs, k = 16 pairs, k >= 32,
// the fused pointwise product).
inline bool persist_pass_kind(int k, const PassArgs& p, uint32_t* kind, uint64_t* tiles) {
  if (k > 16 || p.in2 || p.ntt_mul) return false;
  if (p.span == 2) {
    if (k != 8 || p.wide || p.radix_log2 != 0) return false;
    const int lk2 = 4;
    if (p.log2n < 2 * lk2 || p.log2ns + 2 * lk2 > p.log2n) return false;
    const bool t2b = !p.last && p.log2n - 2 * lk2 - (p.log2ns + lk2) >= 0;
    if (!p.inverse) {
      if (p.last) return false;  // forward transforms of a product stay non-canonical
      *kind = t2b ? PK_PAIR_F_T2 : PK_PAIR_F;
    } else if (p.scale) {
      if (p.last) *kind = PK_PAIR_IS_LAST;
      else if (t2b) *kind = PK_PAIR_IS_T2;
      else return false;
    } else {
      if (p.last) *kind = PK_PAIR_I_LAST;
      else if (t2b) *kind = PK_PAIR_I_T2;
      else return false;
    }
    *tiles = ((p.nvec << (p.log2n - 2 * lk2)) + 1) / 2;  // two K^2-element blocks per tile
    return true;
  }
  if (p.span != 1) return false;
  const int lk = k == 8 ? 4 : 5;
  const int lg = k == 8 ? 3 : 2;  // log2 of the element groups per wavefront
  const uint64_t groups_per_block = 4ull << lg;
  if (p.radix_log2 != 0) {
    if (p.last) return false;
    *kind = p.inverse ? PK_PASS_R_I : PK_PASS_R_F;
    if (p.inverse != p.scale) return false;  // the inverse's radix-R pass carries 1/n
    *tiles = ((p.nvec << (p.log2n - p.radix_log2)) + groups_per_block - 1) / groups_per_block;
    return true;
  }
  const bool unif = p.log2ns > 0 && (p.log2n - lk - p.log2ns) >= lg;
  const bool t2 = !p.last && p.log2n - 2 * lk - p.log2ns >= 0;
  if (p.scale) {
    *kind = p.last ? PK_PASS_ISCALE_LAST : PK_PASS_ISCALE;
  } else if (!p.inverse) {
    if (p.last) return false;  // forward transforms of a product stay non-canonical
    // not uniform: the first pass (Ns = 1, no twiddles, whichever table) or
    // the final one (per-group twiddles of the w^j table)
    if (unif && t2) *kind = PK_PASS_MID;
    else if (!unif && (p.log2ns == 0 || !t2)) *kind = PK_PASS_FIRST;
    else return false;
  } else {
    if (p.last) *kind = PK_PASS_ILAST;
    else if (unif && t2) *kind = PK_PASS_IMID;
    else return false;
  }
  *tiles = (p.ngroups * p.nvec + groups_per_block - 1) / groups_per_block;
  return true;
}

// Cooperative launch of the work list (levels, recs: device memory) for the
// radix shape (k, w, u); grid: workgroups (all resident at once); sync:
// kPersistSyncBytes of zeros (device memory) for the level barriers.
constexpr uint64_t kPersistSyncBytes = 64 * 128;
hipError_t launch_persistent(int k, int w, int u, const PLevel* levels, uint32_t nlevels, const PRec* recs,
                             uint32_t* sync, uint32_t grid, hipStream_t st);
// The table of w^j, j < cnt, on the device (k <= 16): lo[i] = w^i for
// i < 2^log2b, hi[i] = w^(i 2^log2b) for i < cnt / 2^log2b (raw digits,
// device); writes the entry-layout table tab and the raw-digit table raw.
hipError_t launch_table_build(int k, int w, int u, const uint64_t* lo, const uint64_t* hi, int log2b, uint64_t cnt,
                              uint32_t* tab, uint64_t* raw, hipStream_t st);
// Workgroups of that kernel that fit on the device at once (0 if the shape has none).
int persistent_capacity(int k, int w, int u, int* grid);

// Batched products run each transform size in chunks of requests whose
// workspace fits kChunkBytes (at least one request per chunk); the request
// loop sizes its batches with the same rule.
constexpr uint64_t kChunkBytes = 4ull << 30;
inline uint64_t chunk_cap(uint64_t per_request_bytes) {
  const uint64_t c = kChunkBytes / per_request_bytes;
  return c ? c : 1;
}

// words per twiddle-table entry (see TwLayout in gfp_device.hpp)
inline int tw_words(int k) { return (6 * k + 6) & ~3; }

// Builds (once per device and size) the twiddle tables of transforms of size
// n on the current device; a status code of gfp.h.
int prepare_tables(const gfp_field* f, uint64_t n);

// gfp_fft_forward / gfp_fft_inverse of size n with the two work vectors in
// `scratch` (scratch_bytes >= 2 n k 8, else GFP_EINVAL), taking the tables
// only if they are already on the device (else GFP_ENOTREADY): allocates
// nothing on the device.
int transform_noalloc(const gfp_field* f, uint64_t n, int inverse, const uint64_t* x, uint64_t ldx, uint64_t* y,
                      uint64_t ldy, void* scratch, uint64_t scratch_bytes, void* stream);

// Products of C requests of transform size n as a graph for the request
// loop: the launch sequence of one chunk of gfp_polymul_batched (pad, forward
// transforms, pointwise product, inverse transform, unpad) on workspace ws
// (polymul_chunk_bytes(f, n, C) bytes), captured on stream st with the copy
// descriptors read from dev_desc (3C entries: operands a, operands b,
// products; an entry with len 0 copies nothing), so that replaying it after
// rewriting dev_desc computes any C requests of that size.  The size's
// twiddle tables are built before the capture if needed.
uint64_t polymul_chunk_bytes(const gfp_field* f, uint64_t n, uint64_t C);
int capture_polymul_chunk(const gfp_field* f, uint64_t n, uint64_t C, uint64_t* ws, const CopyDesc* dev_desc,
                          hipStream_t st, hipGraphExec_t* out);

}  // namespace gfpk

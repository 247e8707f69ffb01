/*
 * gfp.h -- C ABI of libgfpfft: FFT and polynomial multiplication over Z/pZ
 * for a Generalized Fermat prime p = r^k + 1 on AMD MI355X (gfx950).
 *
 * The operations follow arXiv:1811.01490 ("Putting Furer Algorithm into
 * Practice with the BPAS Library"):
 *   - the field and the radix-r element encoding: section 2;
 *   - the primitive N-th root w with w^(N/2k) = r: section 2.1, Alg. 1;
 *   - the DFT at w, computed for N = R K^e, K = 2k, R = 2^j < K, with base
 *     case DFT_K at w^(N/K) = r and one DFT_R at w^(N/R) = r^(K/R): section
 *     1.1 (eq. CTCT), section 4.1 (eq. sixstepfft; any power of two N),
 *     section 4.3 (Alg. DFT_general);
 *   - the inverse transform (1/N) DFT at w^-1 and the product of two
 *     polynomials by forward transforms, a pointwise product and an inverse
 *     transform: section 3.3, Alg. Fast Convolution.
 *
 * Element encoding (section 2).  An element x of Z/pZ is k digits x_0..x_{k-1}
 * with x = sum_d x_d r^d, every digit in [0, r), except p - 1 which is written
 * x_{k-1} = r and all other digits 0.  This makes the encoding unique; every
 * output of the library is in this canonical form.
 *
 * Vector layout.  A vector of n elements is structure-of-arrays: digit d of
 * element i is the uint64_t at v[d * ld + i], ld >= n (row d is contiguous).
 *
 * Memory and streams.  Unless stated otherwise, vector pointers are device
 * pointers (HIP device memory of the current device) owned by the caller;
 * the library never frees them.  `stream` is a hipStream_t (NULL = the null
 * stream).  Transform calls only enqueue work on that stream and return; the
 * caller synchronises.  The library owns the field object, its host tables
 * and the per-device twiddle tables (uploaded on the first transform of a
 * size on a device, which synchronises that device once).
 *
 * Errors.  Every call returns GFP_OK or a GFP_E* code and never throws.
 * Invalid arguments are rejected before any work is enqueued.  Errors of
 * asynchronous device work surface as GFP_EDEVICE from a later call on the
 * stream or from the caller's own synchronisation.  Inputs are assumed
 * canonical; non-canonical digits give unspecified (but memory-safe) results.
 * Validation: when the environment variable GFP_VALIDATE is set (to anything
 * but "0") at gfp_field_create, the transform, product and elementwise calls
 * on that field first count non-canonical input elements on the device (as
 * gfp_check_canonical does, synchronising the stream) and return GFP_EINVAL
 * if there are any.  gfp_fft_noalloc, gfp_fft_pass, the integer products and
 * the request loop do not validate.
 * Twiddle tables: built once per (field, device, transform size) on first
 * use; for k <= 16 on the device (the host computes 2 sqrt(N/2k) powers of
 * the root, a kernel the rest), unless GFP_HOST_TABLES is set (to anything
 * but "0") at gfp_field_create, which builds them on the host as for k >= 32.
 * Both give the same tables digit for digit.  Either build uploads and
 * waits on the calling thread (gfp_server_submit included), so it can wait
 * behind other work on the GPU that shares its hardware queue.
 */
#ifndef GFP_H
#define GFP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GFP_OK 0
#define GFP_EINVAL 1       /* bad argument (null pointer, ld < n, size not allowed) */
#define GFP_EUNSUPPORTED 2 /* field or size outside what the library implements */
#define GFP_ENOMEM 3       /* device or host allocation failed */
#define GFP_EAGAIN 4       /* request loop: no capacity right now */
#define GFP_EDEVICE 5      /* HIP runtime error */
#define GFP_ENOTPRIME 6    /* r^k + 1 failed the probable-prime test */
#define GFP_ECANCELED 7    /* request loop: request cancelled at shutdown */
#define GFP_EPENDING 8     /* request loop: result not ready yet */
#define GFP_ENOTREADY 9    /* gfp_fft_noalloc: the size's twiddle tables are not on the device yet */

/* Elementwise operations (gfp_elementwise). */
#define GFP_OP_ADD 0       /* z = x + y */
#define GFP_OP_SUB 1       /* z = x - y */
#define GFP_OP_MUL 2       /* z = x * y */
#define GFP_OP_MUL_POW_R 3 /* z = x * r^s (section 2.3), y unused */
#define GFP_OP_MUL_CONST 4 /* z = x * c * r^s, c = host digits c_host */
#define GFP_OP_MUL_SCALE 5 /* z = x * y * c, c = host digits c_host */
#define GFP_OP_MUL_NTT 6   /* z = x * y by the FFT-based product (section 3.3) */

typedef struct gfp_field gfp_field;

/* Create the field Z/pZ, p = r^k + 1 (section 2).  Host-only; touches no GPU.
 * k must be a power of two and r even; the library runs transforms for
 * r = 2^w + 2^u with (k, w, u) in {(8, 63, 34), (8, 59, 16), (16, 62, 36),
 * (16, 58, 10), (32, 62, 56), (32, 56, 21)} and for r = 2^63 - 2^40 with
 * k = 64 (Table 1 and Table testprimes).  p is checked
 * with the Baillie-PSW probable-prime test (a strong test to base 2 and a
 * strong Lucas test with Selfridge's parameters).
 * Returns GFP_EINVAL (out == NULL, bad k/r), GFP_EUNSUPPORTED (shape not
 * compiled in), GFP_ENOTPRIME.  On success *out owns the field; release it
 * with gfp_field_destroy. */
int gfp_field_create(uint32_t k, uint64_t r, gfp_field** out);

/* Release a field and its device tables.  The caller must ensure no work
 * using the field is still running.  NULL is accepted. */
int gfp_field_destroy(gfp_field* f);

/* Field parameters.  log2_max_n: the largest e with 2^e | p - 1 (Table 1).
 * Any output pointer may be NULL. */
int gfp_field_info(const gfp_field* f, uint32_t* k, uint64_t* r, uint32_t* log2_max_n);

/* Primitive n-th root of unity w_n (section 2.1, Alg. 1): n a power of two,
 * 2k <= n <= 2^log2_max_n.  w_n^(n/2k) = r.  g in Alg. 1 is
 * h^((p-1)/n) for the smallest quadratic non-residue h, which makes the roots
 * nested: w_n = w_m^(m/n).  inverse != 0 returns w_n^-1.  digits: host array
 * of k uint64_t, canonical encoding.  Host-only. */
int gfp_root_of_unity(const gfp_field* f, uint64_t n, int inverse, uint64_t* digits);

/* Transform sizes: n a power of two, K = 2k <= n <= 2^log2_max_n and
 * n <= 2^25.  n = R K^e with R = 2^j < K runs a radix-R pass (DFT_R at
 * r^(K/R), no twiddles) before the e radix-K passes.
 * Workspace bytes needed by gfp_fft_forward / gfp_fft_inverse of size n. */
int gfp_fft_workspace_size(const gfp_field* f, uint64_t n, uint64_t* bytes);

/* Forward DFT at w_n: y_i = sum_j x_j w_n^(ij), natural order (section 1.1).
 * x: n elements (ld_x >= n), y: n elements (ld_y >= n), device memory.
 * x == y (same pointer and ld) is allowed.  Other overlap is not.
 * workspace: device memory of at least gfp_fft_workspace_size bytes, or NULL
 * to let the library take it from the stream-ordered allocator. */
int gfp_fft_forward(const gfp_field* f, uint64_t n, const uint64_t* x, uint64_t ld_x, uint64_t* y, uint64_t ld_y,
                    void* workspace, uint64_t ws_bytes, void* stream);

/* Inverse DFT including the 1/n factor: x_j = n^-1 sum_i y_i w_n^(-ij)
 * (section 3.3, Alg. Fast Convolution).  Same arguments as gfp_fft_forward. */
int gfp_fft_inverse(const gfp_field* f, uint64_t n, const uint64_t* x, uint64_t ld_x, uint64_t* y, uint64_t ld_y,
                    void* workspace, uint64_t ws_bytes, void* stream);

/* Layout flags of gfp_fft_pass.  Element-major: digit d of element i at
 * v[i * k + d] (ld ignored), the layout the transforms use between passes. */
#define GFP_PASS_IN_ELEMENT_MAJOR 1
#define GFP_PASS_OUT_ELEMENT_MAJOR 2
#define GFP_PASS_PAIR 4 /* passes s and s+1 in one launch, as plan character '2' */
#define GFP_PASS_WIDE 8 /* passes s and s+1 in one launch, as plan character 'w' */
#define GFP_PASS_NTT 16 /* k >= 32: twiddles multiplied by the FFT-based product, as plan character 'n' */

/* One pass (stage s) of the transform schedule used by gfp_fft_forward /
 * gfp_fft_inverse, n = R K^e.  The stages are s = 0..S-1 with S = e + 1 when
 * R > 1 (stage 0 is then the radix-R pass) and S = e otherwise.  A radix-K
 * stage with Ns = R K^(s') (s' its index among the radix-K stages): for
 * every j < n/K the K elements x[j + t n/K] are multiplied by the twiddles
 * w_L^(a t) (L = K Ns, a = j mod Ns; for the inverse the conjugate
 * twiddles), transformed by DFT_K at r (r^-1) and written to
 * y[(j - a) K + a + t Ns] (section 1.1, eq. CTCT; section 4.1).  The radix-R
 * stage does the same with K replaced by R, Ns = 1 and DFT_R at r^(K/R).
 * Stage 0 of the inverse also multiplies by 1/n; for k >= 32 and n > K,
 * stage 1 does instead, through twiddle tables scaled by 1/n.  Running s = 0..S-1 with
 * y of one pass as x of the next is the full transform.  Outputs of
 * s < S-1 are not canonical: every digit is in [0, 2^64) and the value is
 * congruent mod p (the next pass accepts this); s = S-1 writes the
 * canonical encoding.  x and y must not overlap.  flags: GFP_PASS_* layout
 * bits (0 = both digit-major).  gfp_fft_forward runs stage 0 digit-major to
 * element-major, the middle stages element-major, the last stage
 * element-major to digit-major.  With GFP_PASS_PAIR or GFP_PASS_WIDE the
 * launch runs radix-K stages s and s+1 (s + 1 < S; PAIR: k = 8 or 16; WIDE:
 * k = 8 and n / (K^2 Ns) >= 8), exactly as that character of a plan does.  For
 * instrumentation and custom schedules. */
int gfp_fft_pass(const gfp_field* f, uint64_t n, int s, int inverse, int flags, const uint64_t* x, uint64_t ld_x,
                 uint64_t* y, uint64_t ld_y, void* stream);

/* Transform size used by gfp_polymul for la + lb - 1 output coefficients:
 * the smallest power of two >= la + lb - 1 (and >= K). */
int gfp_polymul_size(const gfp_field* f, uint64_t la, uint64_t lb, uint64_t* n);

/* Workspace bytes for gfp_polymul(la, lb). */
int gfp_polymul_workspace_size(const gfp_field* f, uint64_t la, uint64_t lb, uint64_t* bytes);

/* Product c = a * b of polynomials over Z/pZ (section 3.3, Alg. Fast
 * Convolution with zero padding so the cyclic product does not wrap):
 * c_m = sum_{i+j=m} a_i b_j, m < la + lb - 1.  a: la coefficients (ld_a >= la),
 * b: lb coefficients (ld_b >= lb), c: la + lb - 1 coefficients
 * (ld_c >= la + lb - 1), device memory, c must not overlap a or b.
 * la, lb >= 1.  Workspace as for the transforms. */
int gfp_polymul(const gfp_field* f, const uint64_t* a, uint64_t la, uint64_t ld_a, const uint64_t* b, uint64_t lb,
                uint64_t ld_b, uint64_t* c, uint64_t ld_c, void* workspace, uint64_t ws_bytes, void* stream);

/* One request of a batched product: c = a * b as in gfp_polymul. */
typedef struct gfp_polymul_desc {
  const uint64_t* a;
  uint64_t la, ld_a;
  const uint64_t* b;
  uint64_t lb, ld_b;
  uint64_t* c;
  uint64_t ld_c;
} gfp_polymul_desc;

/* gfp_polymul_batched flags */
#define GFP_BATCH_GRAPH 1      /* capture the launches into a hipGraph, cache it per argument list, replay it */
#define GFP_BATCH_PERSISTENT 2 /* k <= 16: the whole batch as one cooperative launch over a device work list */

/* Workspace bytes gfp_polymul_batched needs for this request list, with
 * either flag.  Without GFP_BATCH_PERSISTENT the call needs less: the sum of
 * the size classes' chunk workspaces (8 C N k words for a chunk of C requests
 * of transform size N), without the work-list tail (its levels, records,
 * three 32-byte copy descriptors per request and 8 KiB of counters). */
int gfp_polymul_batched_workspace_size(const gfp_field* f, uint32_t n, const gfp_polymul_desc* d, uint64_t* bytes);

/* n independent products (section 3.3, Alg. Fast Convolution), each exactly
 * as gfp_polymul, of mixed sizes.  d: host array of n descriptors (device
 * pointers inside, caller-owned).  Requests are grouped by transform size;
 * each group runs as one launch per pass over all its operands (in chunks
 * bounded by the workspace), so the number of launches does not grow with
 * n.  workspace: device memory of gfp_polymul_batched_workspace_size bytes
 * (required with GFP_BATCH_GRAPH), or NULL for a stream-ordered allocation.
 * flags & GFP_BATCH_GRAPH: the launch sequence is captured into a hipGraph
 * on the first call with this exact argument list (descriptors, workspace,
 * stream) and plans, and replayed on later calls; stream must not be NULL.
 * A field keeps at most 64 such graphs; capturing another evicts the least
 * recently used one, after waiting (outside the field's lock) for an event
 * recorded behind its last launch.
 * flags & GFP_BATCH_PERSISTENT (k = 8 and 16 only, else GFP_EUNSUPPORTED;
 * not with GFP_BATCH_GRAPH): one cooperative launch walks a work list of
 * (launch, tile) items, grouped in levels separated by grid-wide barriers:
 * pad, each pass of the forward transforms, the pointwise product, each
 * pass of the inverse, unpad; the size classes share every level.  The list
 * is written into the workspace tail by a stream-ordered copy before the
 * launch, so one launch serves any number of size classes.  Results
 * do not depend on the batch composition (bit-identical to gfp_polymul).
 * Errors: GFP_EINVAL (bad descriptor, n == 0, NULL stream with
 * GFP_BATCH_GRAPH, workspace too small), GFP_EUNSUPPORTED, GFP_EDEVICE. */
int gfp_polymul_batched(const gfp_field* f, uint32_t n, const gfp_polymul_desc* d, void* workspace, uint64_t ws_bytes,
                        int flags, void* stream);

/* Elementwise z = op(x, y) on n elements (section 2: addition, subtraction,
 * multiplication by a power of r, multiplication).  x, y, z device vectors
 * (y unused for GFP_OP_MUL_POW_R and GFP_OP_MUL_CONST); z may equal x or y.
 * s: the exponent for GFP_OP_MUL_POW_R / GFP_OP_MUL_CONST (any integer,
 * taken mod 2k).  c_host: k host digits of the constant c for
 * GFP_OP_MUL_CONST and GFP_OP_MUL_SCALE, else ignored.  GFP_OP_MUL and
 * GFP_OP_MUL_NTT give the same products by two algorithms: the schoolbook
 * column product the transforms use, and the FFT-based multiplication of
 * section 3.3 (negacyclic convolutions modulo three word primes, CRT). */
int gfp_elementwise(const gfp_field* f, int op, const uint64_t* x, uint64_t ld_x, const uint64_t* y, uint64_t ld_y,
                    uint64_t* z, uint64_t ld_z, uint64_t n, int64_t s, const uint64_t* c_host, void* stream);

/* ---- Integer products ---------------------------------------------------------
 *
 * c = a * b for non-negative integers of na and nb 64-bit words (device
 * memory, little-endian; c has na + nb words and must not overlap a or b):
 * the application the paper starts from (section 1) -- an integer is a
 * polynomial evaluated at a power of two, so the product is a polynomial
 * product over Z/pZ (section 3.3, Alg. Fast Convolution) followed by the
 * evaluation.  The integers are cut into b-bit coefficients, b as large as
 * the field allows (the product's coefficients, below min(la, lb) 2^(2b),
 * must stay below p: b = min(448, (k W' - 2 - ceil(log2(64 min(na, nb)))) / 2)
 * with r > 2^W'), each converted to k radix-r digits on the device; the
 * canonical digits of the product's coefficients give them exactly; they
 * are converted back to binary, added at their bit offsets and the carries
 * resolved by a carry-lookahead scan, all on the device.  Sizes:
 * la + lb - 1 coefficients (la = ceil(64 na / b)) within the transform limit.
 * Workspace: gfp_bigint_mul_workspace_size bytes, or NULL. */
int gfp_bigint_mul_workspace_size(const gfp_field* f, uint64_t na, uint64_t nb, uint64_t* bytes);
int gfp_bigint_mul(const gfp_field* f, const uint64_t* a, uint64_t na, const uint64_t* b, uint64_t nb, uint64_t* c,
                   void* workspace, uint64_t ws_bytes, void* stream);

/* ---- Stage groupings and the autotuner -------------------------------------
 *
 * A transform of size n = R K^e runs as a sequence of launches: the radix-R
 * pass alone (when R > 1), then the e radix-K passes, each launch covering
 * one radix-K pass or (k = 8, 16) two consecutive passes fused in one launch,
 * with the stride permutation between them (section 4.1, eq. sixstepfft)
 * staged through LDS so the intermediate never goes to HBM.  A plan is a
 * string with one character per launch: '1' one pass, '2' two fused passes
 * (K^2-element blocks, two per workgroup for k = 8, one for k = 16; the
 * second pass reads its twiddles per element group), 'w' (k = 8) two fused
 * passes over eight blocks per workgroup (wavefront-uniform twiddles in both
 * passes; needs n / (K^2 R K^s) >= 8 at its first radix-K pass s), and for
 * k = 32, 64 'n': one pass whose twiddle products use the FFT-based
 * multiplication of section 3.3 (negacyclic transforms of the digits modulo
 * three word primes and the CRT) with the twiddles' transforms tabulated
 * (built on the first such transform of a size on a device), instead of the
 * schoolbook column product; the results are identical.  The plan covers the radix-K passes only.
 * Example: "1211" for e = 5.  Plans are kept per
 * (n, batch class, layout): the batch class is the number of same-size
 * transforms one launch covers (1, 2-7, 8-63, 64 and more: gfp_polymul runs
 * 2 forward and 1 inverse, gfp_polymul_batched 2C and C); the layout is that
 * of the transform's ends (digit-major for gfp_fft_forward/inverse,
 * element-major inside the products).  Keys without a plan use a built-in
 * default.  Results never depend on the plan.  Plans live in the field
 * object; a caller that wants them to persist stores the strings. */
#define GFP_LAYOUT_DIGIT_MAJOR 0
#define GFP_LAYOUT_ELEMENT_MAJOR 1

/* The plan in use for nvec transforms of size n with the given layout, as a
 * NUL-terminated string in buf (len >= e + 1). */
int gfp_plan_get(const gfp_field* f, uint64_t n, uint64_t nvec, int layout, char* buf, uint32_t len);

/* Set the plan for (n, batch class of nvec, layout); plan NULL or "" restores
 * the default.  GFP_EINVAL for an unknown character, passes that do not sum
 * to e, a fused pair for a k without one, or 'w' where it does not fit. */
int gfp_plan_set(gfp_field* f, uint64_t n, uint64_t nvec, int layout, const char* plan);

/* Autotuner: times every valid plan on nvec forward transforms of size n with
 * the given layout, on `stream`, and keeps the fastest for (n, batch class,
 * layout).  Allocates and frees its own device buffers (4 nvec n k words, at
 * most 8 GiB each) and synchronises the stream; must not be called during
 * stream capture.  best: the chosen plan (len >= e + 1) or NULL; us: its mean
 * time in microseconds or NULL. */
int gfp_tune(gfp_field* f, uint64_t n, uint64_t nvec, int layout, void* stream, char* best, uint32_t len, double* us);

/* ---- Request loop (serving) ------------------------------------------------
 *
 * A server takes polynomial-product requests (section 3.3, Alg. Fast
 * Convolution, exactly as gfp_polymul) of any size and any of the compiled
 * fields as they arrive, and runs them in batches on the GPU with continuous
 * batching: it owns `slots` HIP streams, each with its own share of the
 * workspace budget; a slot that is free takes the requests waiting at that
 * moment (first come, first served, up to max_batch, as long as their
 * transform workspace fits the slot's share) and runs them as one
 * gfp_polymul_batched call per (field, transform size) class, smallest first;
 * each class is done as soon as its own work is.  Requests that arrive while
 * slots are busy wait until a slot frees, and batches of different slots run
 * concurrently on the device.  An express slot (express_log2n) serves only
 * small requests, taken from anywhere in the queue in arrival order.  Batches run as replayed hipGraphs (see
 * gfp_server_config.flags).  Each result is bit-identical to gfp_polymul of
 * the same request alone: the arithmetic is exact and does not depend on the
 * batch.  All calls are thread-safe, except that gfp_server_destroy must not
 * overlap any other call on the same server.  Timestamps are CLOCK_MONOTONIC
 * nanoseconds (comparable with the host clock of the caller). */
typedef struct gfp_server gfp_server;

typedef struct gfp_server_config {
  uint64_t workspace_bytes; /* device memory budget for transform workspace, split evenly over the slots */
  uint32_t slots;           /* batches in flight at once (0 = 2) */
  uint32_t max_batch;       /* requests per batch (0 = 256) */
  uint32_t max_pending;     /* submitted, not yet admitted requests before submit returns GFP_EAGAIN (0 = 65536) */
  uint32_t max_wait_us;     /* a free slot waits up to this long for more requests before launching (0 = launch at once) */
  int32_t device;           /* HIP device ordinal, -1 = the current device */
  uint32_t express_log2n;   /* 0, or: the last slot only takes requests of transform size <= 2^express_log2n
                               (needs slots >= 2) */
  uint32_t flags;           /* GFP_SERVER_* bits */
} gfp_server_config;

/* gfp_server_config.flags.  By default each slot runs a chunk of C requests
 * of one (field, transform size) class as a hipGraph: the chunk's launch
 * sequence (as in gfp_polymul_batched) is captured per (field, size, C) and
 * slot, the second time that shape occurs (the first time it runs eagerly),
 * with the copy descriptors read from a small device table of the slot, and
 * replayed for every later chunk of that shape after the new descriptors are
 * copied into the table.  C is rounded up to a power of two where the
 * chunk's work is small (C n <= 2^17 elements; the extra entries copy
 * nothing).  With GFP_SERVER_EAGER the launches are enqueued one by one
 * instead. */
#define GFP_SERVER_EAGER 1

typedef struct gfp_request {
  const gfp_field* field; /* must outlive the request */
  const uint64_t* a;      /* device, la coefficients, row stride ld_a */
  uint64_t la, ld_a;
  const uint64_t* b;
  uint64_t lb, ld_b;
  uint64_t* c;            /* device, la + lb - 1 coefficients, row stride ld_c; written when the request is done */
  uint64_t ld_c;
  void* ready_event;      /* hipEvent_t the batch waits for before reading a and b (recorded by the caller after
                             writing them), or NULL: the operands are ready when submit is called */
} gfp_request;

typedef struct gfp_result {
  int32_t status;       /* GFP_OK, or the error of this request (GFP_EDEVICE, GFP_ECANCELED, ...) */
  uint32_t batch_size;  /* requests in the batch that carried it */
  uint64_t batch_id;    /* 1, 2, ... in launch order */
  uint64_t t_submit_ns; /* submit returned the ticket */
  uint64_t t_admit_ns;  /* taken into a batch */
  uint64_t t_launch_ns; /* its batch started enqueueing */
  uint64_t t_done_ns;   /* its batch finished on the device */
} gfp_result;

typedef struct gfp_server_stats {
  uint64_t submitted, completed, rejected; /* rejected: submit calls that returned GFP_EAGAIN */
  uint64_t batches;
  uint64_t max_batch_size;
  uint64_t max_batch_workspace;            /* largest workspace a batch needed, bytes */
  uint64_t overlapped_batches;             /* batches launched while another slot's batch was in flight */
  uint64_t slot_bytes;                     /* workspace per slot */
  uint64_t graph_launches;                 /* chunks run by replaying a captured graph */
  uint64_t graph_captures;                 /* chunk graphs captured (a shape's second occurrence) */
} gfp_server_stats;

/* Start a server on cfg->device: allocates the workspace (cfg->workspace_bytes),
 * a copy-descriptor table per slot (96 max_batch bytes, rounded up to 256)
 * and pinned host staging for the descriptors (192 max_batch bytes per
 * slot), and creates the slot streams and threads.  Errors: GFP_EINVAL
 * (NULL argument, slots > 64, max_batch > 65535, workspace_bytes / slots
 * under 256 bytes, express_log2n > 40 or with fewer than 2 slots, unknown
 * flags), GFP_ENOMEM, GFP_EDEVICE. */
int gfp_server_create(const gfp_server_config* cfg, gfp_server** out);

/* Queue one request; returns at once with a ticket (1, 2, ...), except that
 * the first request of a transform size not yet used with this field on the
 * server's device builds that size's twiddle tables first, on the caller's
 * thread.  The request is copied; the buffers it names stay the caller's and
 * must not be touched until the ticket is done.  Errors: GFP_EINVAL (bad
 * pointers or lengths), GFP_EUNSUPPORTED (field or size), GFP_ENOMEM (its
 * workspace exceeds one slot's share, so it could never run, or no device
 * memory for the tables), GFP_EAGAIN (max_pending requests are waiting; try
 * again later), GFP_ECANCELED (the server is shutting down), GFP_EDEVICE. */
int gfp_server_submit(gfp_server* s, const gfp_request* req, uint64_t* ticket);

/* If the request is done, write its result, forget the ticket and return
 * GFP_OK (the output is then complete and visible to every stream); else
 * GFP_EPENDING.  GFP_EINVAL for an unknown ticket. */
int gfp_server_poll(gfp_server* s, uint64_t ticket, gfp_result* out);

/* As gfp_server_poll, but blocks until the request is done or timeout_us
 * microseconds passed (timeout_us < 0: no limit); GFP_EPENDING on time-out. */
int gfp_server_wait(gfp_server* s, uint64_t ticket, int64_t timeout_us, gfp_result* out);

/* Block until every submitted request is done (results stay available). */
int gfp_server_drain(gfp_server* s);

/* Counters since create. */
int gfp_server_get_stats(gfp_server* s, gfp_server_stats* out);

/* Stop the server: requests not yet admitted are cancelled (GFP_ECANCELED),
 * admitted ones run to completion; then the threads, streams and workspace
 * are released and every ticket becomes invalid.  NULL is accepted. */
int gfp_server_destroy(gfp_server* s);

/* ---- Transforms that allocate nothing ----------------------------------------
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * gfp_fft_noalloc is gfp_fft_forward (inverse == 0) or gfp_fft_inverse
 * (inverse != 0) with the same arguments and bit-identical results, except
 * that the workspace is not an argument: the two work vectors come from a
 * static device array of GFP_STATIC_SCRATCH_BYTES bytes that the library
 * holds on every device it runs on until the process ends.  The call makes
 * no device allocation and frees nothing.
 *   - Size limit: 2 n k 8 <= GFP_STATIC_SCRATCH_BYTES, i.e. n <= 2^18 for
 *     k = 8, 2^17 for k = 16, 2^16 for k = 32, 2^15 for k = 64; larger n
 *     returns GFP_EINVAL before any work is enqueued.
 *   - The twiddle tables of size n must already be on the current device
 *     (built by any earlier gfp_fft_forward, gfp_fft_inverse, gfp_polymul or
 *     gfp_tune of that size there); otherwise GFP_ENOTREADY.
 *   - Every call on one device uses that device's single array, and the
 *     array keeps the last call's contents (it needs no clearing: a call
 *     reads only words it wrote first).  Calls that overlap in time on one
 *     device -- two streams, or two host threads -- race on it and give wrong
 *     results; run them on one stream.
 *   - The first call on a device resolves the array's device address
 *     (hipGetSymbolAddress; no allocation).
 * Other errors as gfp_fft_forward. */
#define GFP_STATIC_SCRATCH_BYTES (32ull << 20)
int gfp_fft_noalloc(const gfp_field* f, uint64_t n, int inverse, const uint64_t* x, uint64_t ld_x, uint64_t* y,
                    uint64_t ld_y, void* stream);

/* Input validation (the library assumes canonical inputs and does not check
 * them on the hot path).  Counts the elements of the digit-major vector x
 * (n elements, ld_x >= n, device memory) whose digits are not the canonical
 * encoding of section 2 (every digit below r, or p - 1 as (0, ..., 0, r)),
 * into the host *bad.  Synchronises the stream; not for stream capture. */
int gfp_check_canonical(const gfp_field* f, const uint64_t* x, uint64_t ld_x, uint64_t n, void* stream, uint64_t* bad);

/* Static description of an error code. */
const char* gfp_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* GFP_H */

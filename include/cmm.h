/*
 * cmm.h -- compressed matrix multiplication on one MI355X (gfx950).
 *
 * C interface to the sketch of a matrix product from R. Pagh, "Compressed
 * Matrix Multiplication".  For d independent repetitions t the library
 * computes the length-b count sketch of AB
 *
 *     c_t[u] = sum over (i,j) with (h1_t(i) + h2_t(j)) mod b = u
 *              of s1_t(i) s2_t(j) (AB)_ij                       (Section 2.2)
 *
 * without forming AB: every outer product a_k b_k of eq. (1) is count-
 * sketched on both sides, the two sketches are multiplied as polynomials
 * modulo x^b - 1 through the FFT, and the products are summed over k before
 * one inverse FFT per repetition (Figure 1, COMPRESSEDPRODUCT).  Entries are
 * decoded as the median over t of s1_t(i) s2_t(j) c_t[(h1_t(i)+h2_t(j)) mod b]
 * (Figure 1, DECOMPRESS) and the largest ones are selected.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every function returns an int status: CMM_OK (0) or a negative CMM_E*
 *   code.  No exception crosses the interface.  cmm_strerror() names a code;
 *   cmm_last_error() gives the message of the context's last failure.
 * - Matrix operands are caller-owned DEVICE pointers, read only, and must
 *   stay valid until the call returns (or, with CMM_ASYNC, until the context
 *   stream has passed the call).  They are laid out in the single-pass order
 *   of Section 2.2: A (n1 x m) column-major, i.e. A[i,k] at A[k*lda + i]
 *   with lda >= n1; B (m x n3) row-major, B[k,j] at B[k*ldb + j] with
 *   ldb >= n3.  For a sample covariance product A = X^T, B = X, both are the
 *   m-by-n observation matrix X (one row per sample, Section 3.2).
 * - Work is ordered on the context's HIP stream.  Calls return after the
 *   stream has finished unless CMM_ASYNC is passed.
 * - Hashing (Section 2.2, polynomial hash functions): g(x) = (a x + c) mod
 *   (2^61 - 1); h = g mod b; s = +1 if g is even, -1 if odd; one (a, c) pair
 *   per repetition and per function h1, s1, h2, s2 (in that order).  With a
 *   seed the pairs come from the SplitMix64 stream of the seed: outputs
 *   z_{8t+2f+1}, z_{8t+2f+2} give a = 1 + z mod (2^61-2), c = z' mod (2^61-1).
 * - b must be a power of two in [16, 2^20]; 1 <= d <= 63.  The transform
 *   splits b = R * C with C <= 2^13 (two C-point buffers in LDS) and
 *   R <= 256 (its row-weight table and 16-bit row field), which caps the
 *   design at 2^21; 2^20 is the largest length the test suite runs.
 * - fp8 scales are per hashed index (scaleA[n1], scaleB[n3]): one float per
 *   column of each stored k-major array, multiplied into every value of
 *   that index before it is hashed.
 * - Values must be finite and of float32-friendly size.  Each column a_k
 *   and row b_k is count-sketched and transformed in float32 (its fold into
 *   the transform rows is 30-bit fixed point relative to its largest
 *   |value|), and the products of two spectra are float32; the k-sum and
 *   the inverse transform are float64.  So max|a_k| * max|b_k| * n1 * n3
 *   must stay below about 1e37, and a column or row whose largest |value|
 *   is nonzero but below about 1e-29 lies outside the range of its
 *   fixed-point scale, and its fold is then meaningless (its terms would be
 *   below float32's range in the products anyway).  Errors are relative to
 *   the largest sketch entries.
 * - Objects are library-owned: free sketches with cmm_sketch_free() before
 *   destroying their context with cmm_ctx_destroy().
 * - A context and its sketches are used by one host thread at a time (the
 *   context holds a buffer cache and small pinned staging buffers); threads
 *   that work concurrently each create their own context, which may share
 *   the device and run on their own streams.
 */
#ifndef CMM_H
#define CMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define CMM_OK            0
#define CMM_EINVAL       -1  /* an argument is out of its documented range */
#define CMM_ENOMEM       -2  /* device memory could not be allocated */
#define CMM_EHIP         -3  /* a HIP runtime call or kernel launch failed */
#define CMM_EUNSUPPORTED -4  /* valid request outside what the library handles */
#define CMM_ESTATE       -5  /* object in the wrong state (freed, mismatched) */

/* element types of the stored operands */
#define CMM_F32       0      /* IEEE binary32 */
#define CMM_BF16      1      /* bfloat16 bits (uint16) */
#define CMM_FP8_E4M3  2      /* OCP e4m3fn bits (uint8) times a per-column scale */

/* flags of cmm_sketch_product_ex */
#define CMM_SUBTRACT_DIAG 1u /* sketch AB with its diagonal zeroed (n1 == n3) */
#define CMM_ASYNC         2u /* do not wait for the stream before returning */
#define CMM_AUTOTUNE      4u /* cmm_batch_create: tune size classes not yet tuned */

/* candidate domains of cmm_topk */
#define CMM_TOPK_ALL        0 /* every (i, j) */
#define CMM_TOPK_UPPER      1 /* i < j only (symmetric products) */
#define CMM_TOPK_PER_COLUMN 2 /* the K largest of every column j, n3*K results */

typedef struct cmm_ctx cmm_ctx;
typedef struct cmm_sketch cmm_sketch;
typedef struct cmm_batch cmm_batch;

/* One product of a batch: the arguments of cmm_sketch_product_ex with a
 * seed (A, B device pointers in the layouts above; flags 0 or
 * CMM_SUBTRACT_DIAG). */
typedef struct cmm_problem {
  const void* A;
  int64_t lda;
  const void* B;
  int64_t ldb;
  int64_t n1, m, n3;
  int64_t b;
  int32_t d;
  int32_t dtype;
  const float* scaleA;
  const float* scaleB;
  uint64_t seed;
  uint32_t flags;
  uint32_t reserved;   /* must be 0 */
} cmm_problem;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device` whose work is ordered on
 * `hip_stream` (a hipStream_t; NULL = the device's null stream).  The
 * context owns a cache of device buffers reused across calls. */
int cmm_ctx_create(int device, void* hip_stream, cmm_ctx** out);

/* Switch the context to another stream; waits for the old one first. */
int cmm_ctx_set_stream(cmm_ctx* ctx, void* hip_stream);

/* Workspace limit of one product, in bytes (0 restores the default, half of
 * the device memory).  A product is a sum of m outer products (eq. (1)) and
 * its sketch is linear in them (Section 2.2), so a product whose workspace
 * (count sketches of every k, k-split partial spectra, layout tables) would
 * exceed the limit runs as consecutive k-slabs, each as long as the limit
 * allows (at least one k), whose float64 sketches are added.  The result
 * equals the unsplit product's up to float rounding.  Applies to
 * cmm_sketch_product, _ex, _tables, _sparse and cmm_estimate_nnz; batches,
 * the autotuner and cmm_find_significant keep whole products.
 * Errors: CMM_EINVAL for a negative limit or an invalid context. */
int cmm_ctx_set_workspace_limit(cmm_ctx* ctx, int64_t bytes);

/* Wait for the stream, release every cached buffer and the context. */
int cmm_ctx_destroy(cmm_ctx* ctx);

const char* cmm_strerror(int code);
const char* cmm_last_error(const cmm_ctx* ctx);

/* Kernel timing: while enabled, the library records a pair of HIP events on
 * the context stream around every launch of the named kernels and sums
 * their durations.  `name` is one of "hash", "layout", "countsketch",
 * "fft_mac", "ifft", "decode", "frobenius" (cmm_frobenius_bound), "nnz"
 * (every product of cmm_estimate_nnz), "extract"
 * (the masked sketches, decoding and vote of cmm_find_significant), or
 * "batch" (a whole graph replay of
 * cmm_batch_run; the kernels inside a graph are not timed one by one).
 * Reading waits for the stream. */
int cmm_ctx_profile(cmm_ctx* ctx, int enable);
int cmm_ctx_profile_read(cmm_ctx* ctx, const char* name, double* total_ms, int64_t* launches);

/* Bytes the named kernels move to and from device memory by design, summed
 * over the launches timed since profiling was enabled.  Only "countsketch"
 * is recorded: the stored operands (and fp8 scales) read once, and the
 * count-sketch positions written (the layout's padded segments, W * lseg
 * per side, repetition and k) plus one column maximum per side, repetition
 * and k.  Recorded for synchronous dense products (not for CMM_ASYNC,
 * sparse operands or batches); the segment lengths are read back after the
 * product, outside its kernels.  Unknown names read 0. */
int cmm_ctx_profile_bytes(cmm_ctx* ctx, const char* name, double* read_bytes, double* written_bytes);

/* HBM stream measurement, for comparing a kernel with what plain streams of
 * the same shape reach on this device: `reps` timed launches (after one
 * untimed) of a kernel that reads read_bytes (16-byte loads) and writes
 * write_bytes (16-byte stores, streaming non-temporal ones when
 * `nontemporal`), in r = write_bytes / read_bytes contiguous output planes
 * per input element when both are non-zero.  Sizes are multiples of 16 and
 * write_bytes a multiple of read_bytes when both are set (CMM_EINVAL
 * otherwise).  Allocates and frees its buffers.  *ms_per_launch receives
 * the HIP-event time per launch on the context stream. */
int cmm_stream_probe(cmm_ctx* ctx, int64_t read_bytes, int64_t write_bytes, int32_t nontemporal,
                     int32_t reps, double* ms_per_launch);

/* ---- the sketch (COMPRESSEDPRODUCT, Figure 1) ------------------------- */

/* Square float32 form: A (n x n, column-major, lda = n), B (n x n,
 * row-major, ldb = n), b buckets, d repetitions, hash seed.  On success
 * *out holds the sketch c[d][b] on the device. */
int cmm_sketch_product(cmm_ctx* ctx, const float* A, const float* B, int64_t n,
                       int64_t b, int32_t d, uint64_t seed, cmm_sketch** out);

/* General form.  `dtype` is CMM_F32, CMM_BF16 or CMM_FP8_E4M3; for fp8,
 * scaleA (n1 floats, device) scales A's row i and scaleB (n3 floats,
 * device) scales B's column j (the stored arrays' column scales); NULL means
 * 1.  `hash_params` (host, d*4*2 uint64 (a, c) pairs in the order h1, s1,
 * h2, s2, with 1 <= a < 2^61-1 and c < 2^61-1) replaces the seed-derived
 * parameters when non-NULL.  `flags` combines CMM_SUBTRACT_DIAG (requires
 * n1 == n3; subtracts s1(i)s2(i)(AB)_ii from bucket (h1(i)+h2(i)) mod b,
 * giving the sketch of the product with a zero diagonal, Section 3.2) and
 * CMM_ASYNC.  Sizes: n1, n3 <= 65535 (CMM_EUNSUPPORTED above; rows of up to
 * 24576 elements are staged in LDS, longer ones are read from global
 * memory), m <= 2^30, b a power of two in [16, 2^20], 1 <= d <= 63
 * (CMM_EINVAL otherwise). */
int cmm_sketch_product_ex(cmm_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                          int64_t n1, int64_t m, int64_t n3, int32_t dtype,
                          const float* scaleA, const float* scaleB, int64_t b, int32_t d,
                          uint64_t seed, const uint64_t* hash_params, uint32_t flags,
                          cmm_sketch** out);

/* Same product with explicit hash tables instead of hash functions (host
 * arrays: h1[d*n1] in [0,b), s1[d*n1] in {-1,+1}, h2[d*n3], s2[d*n3]).
 * Meant for tests that need a chosen splitting function, e.g. an injective
 * one that turns the sketch into the plain product. */
int cmm_sketch_product_tables(cmm_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                              int64_t n1, int64_t m, int64_t n3, int32_t dtype,
                              const float* scaleA, const float* scaleB, int64_t b, int32_t d,
                              const int32_t* h1, const int8_t* s1, const int32_t* h2,
                              const int8_t* s2, uint32_t flags, cmm_sketch** out);

/* Sparse operands (Corollary 8: the count sketches cost O(N) for N
 * non-zeros): A by columns (column k of A: row indices a_idx[e] and values
 * a_val[e] for e in [a_ptr[k], a_ptr[k+1])) and B by rows (row k of B:
 * column indices b_idx[e], values b_val[e], e in [b_ptr[k], b_ptr[k+1])).
 * All device arrays; a_ptr and b_ptr have m + 1 entries starting at 0;
 * indices lie in [0, n1) resp. [0, n3) and are distinct within a column
 * (row); values are float32.  The result equals cmm_sketch_product_ex on
 * the dense matrices (same hashing, same sketch; it is the same computation
 * from the staged row on).  Offsets and index ranges are checked on the
 * device first (CMM_EINVAL); repeated indices are not detected.  An operand
 * without entries may pass NULL index and value arrays.  flags:
 * CMM_SUBTRACT_DIAG (n1 == n3), CMM_ASYNC.  n1, n3 <= 24576 (every row is
 * staged in LDS; CMM_EUNSUPPORTED above). */
int cmm_sketch_product_sparse(cmm_ctx* ctx, const int64_t* a_ptr, const int32_t* a_idx,
                              const float* a_val, const int64_t* b_ptr, const int32_t* b_idx,
                              const float* b_val, int64_t n1, int64_t m, int64_t n3, int64_t b,
                              int32_t d, uint64_t seed, uint32_t flags, cmm_sketch** out);

/* Allocation-free form of cmm_sketch_product_ex, for callers that cannot
 * allocate: code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc.  It computes the same sketch with the same kernels and
 * writes c[d][b] (row-major float64) to the caller's DEVICE buffer c_out;
 * it returns no handle.  It calls no hipMalloc/hipFree and no allocating
 * library routine, creates no event, and does not wait for the stream: the
 * result is ready when the context stream has passed the call.  All
 * workspace (hash tables, bucket layout, count sketches, partial spectra,
 * twiddles, hash parameters) lives in one device array of 256 MiB that the
 * library holds on every device it runs on until the process ends; a
 * product that needs more returns CMM_EUNSUPPORTED (call
 * cmm_sketch_product_ex instead).  Every call on a device shares that
 * device's array and leaves its contents behind (each call initialises what
 * it reads), so calls that overlap on one device -- on two streams, or
 * from two threads -- race and must be ordered by the caller.  The hash
 * parameters come from `seed` (computed on the device by the rule above);
 * flags: 0 or CMM_SUBTRACT_DIAG (n1 == n3).  Other arguments and errors as
 * in cmm_sketch_product_ex. */
int cmm_sketch_product_noalloc(cmm_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                               int64_t n1, int64_t m, int64_t n3, int32_t dtype,
                               const float* scaleA, const float* scaleB, int64_t b, int32_t d,
                               uint64_t seed, uint32_t flags, double* c_out);

int cmm_sketch_free(cmm_sketch* sk);

/* Dimensions of a sketch (any output pointer may be NULL). */
int cmm_sketch_info(const cmm_sketch* sk, int64_t* n1, int64_t* m, int64_t* n3,
                    int64_t* b, int32_t* d);

/* Copy c[t][u] (row-major d x b, float64) to `dst`, `count` = d*b; dst is a
 * device pointer when dst_on_device != 0, else host memory. */
int cmm_sketch_copy_c(const cmm_sketch* sk, double* dst, int64_t count, int32_t dst_on_device);

/* Host copies of the hash parameters (d*4*2 uint64) and of repetition t's
 * hash tables (h1[n1], s1[n1], h2[n3], s2[n3]; any pointer may be NULL). */
int cmm_sketch_hash_params(const cmm_sketch* sk, uint64_t* ac);
int cmm_sketch_hashes(const cmm_sketch* sk, int32_t t, int32_t* h1, int8_t* s1,
                      int32_t* h2, int8_t* s2);

/* Linear updates of a sketch (Section 3.2 and eq. (1)): subtract the
 * diagonal diag[0..len) (device float64, len <= min(n1, n3)) from every
 * repetition; add another sketch of the same (hash parameters, b, d, n1,
 * n3), e.g. one taken over a different range of k.  CMM_ESTATE if they do
 * not match. */
int cmm_sketch_subtract_diagonal(cmm_sketch* sk, const double* diag, int64_t len);
int cmm_sketch_merge(cmm_sketch* dst, const cmm_sketch* src);

/* ---- many products in one launch --------------------------------------- */

/* A batch is a set of independent sketch products (COMPRESSEDPRODUCT,
 * Figure 1, once per problem, each with its own n1, m, n3, b, d, dtype and
 * seed) recorded once into one HIP graph.  Creation validates every problem,
 * computes each problem's bucket layout from its hash functions (which fix
 * it), allocates the sketches and a workspace per concurrent branch of the
 * graph (problems are spread over up to four branches, longest first), and
 * captures every kernel of every product; it runs nothing but the layout
 * pass.  The operand pointers are recorded: each replay reads the current
 * contents of the same buffers, which must stay allocated while the batch
 * lives.  With CMM_AUTOTUNE, size classes the context has no tuning for are
 * tuned first (cmm_autotune).  count in [1, 4096]. */
int cmm_batch_create(cmm_ctx* ctx, const cmm_problem* probs, int32_t count, uint32_t flags,
                     cmm_batch** out);

/* Replay the whole batch as one graph launch on the context stream; waits
 * for it unless flags has CMM_ASYNC.  Replays of one batch are ordered on
 * that stream and give identical sketches for identical operands. */
int cmm_batch_run(cmm_batch* batch, uint32_t flags);

/* The sketch of problem `index`, owned by the batch and rewritten by every
 * replay; cmm_sketch_free() on it returns CMM_ESTATE. */
int cmm_batch_sketch(cmm_batch* batch, int32_t index, cmm_sketch** out);

/* cmm_topk of every product of the batch, on the context stream, with
 * K[q] for product q (an array of the batch's count) and one `mode` for all.
 * Product q's results start at offset sum over p < q of K[p] (K[p]*n3 of
 * product p for CMM_TOPK_PER_COLUMN) in the host arrays out_i, out_j and
 * out_val, which hold the total.  Results equal those of cmm_topk on each
 * product's sketch; each decoding phase is issued for all products before
 * its one host wait (DECOMPRESS, Figure 1; the selection itself is this
 * library's, see cmm_topk).  Errors as cmm_topk's, checked for every product
 * before any work starts, except CMM_EUNSUPPORTED for more than 4096 tied
 * estimates, which can come after earlier products' work. */
int cmm_batch_topk(cmm_batch* batch, const int32_t* K, int32_t mode, int64_t* out_i, int64_t* out_j,
                   float* out_val);

/* Wait for the context stream and release the graph, the workspace and the
 * batch's sketches. */
int cmm_batch_free(cmm_batch* batch);

/* One-shot form: create a batch of `count` problems, run it once, hand the
 * sketches to the caller (outs[count], each freed with cmm_sketch_free()) and
 * release the rest. */
int cmm_sketch_product_batched(cmm_ctx* ctx, const cmm_problem* probs, int32_t count,
                               cmm_sketch** outs);

/* ---- tuning ------------------------------------------------------------ */

/* The geometry of a product is (log2c, kmax, cs_blocks): the FFT row length
 * C = 2^log2c of the four-step transform of length b = R*C (log2c in
 * [4, 13], capped at log2 b), the largest number of k per spectral block
 * (kmax in [1, 128]) and the number of count-sketch blocks over k
 * (cs_blocks >= 1).  Tuning entries are keyed by size class: log2 b, the
 * ceilings of log2 n1, log2 m, log2 n3, d and dtype.
 *
 * cmm_autotune times every candidate geometry of the class of (n1, m, n3,
 * b, d, dtype) on synthetic operands on the context stream, stores the
 * fastest for the class and returns it (tuning[3], may be NULL) with its
 * time (best_ms, may be NULL).  Products whose class has an entry use it;
 * others use the built-in default.  cmm_tuning_get returns the geometry a
 * product of these sizes would use; cmm_tuning_set stores one.  Save/load
 * write and read the entries as a JSON array (one object per class, tagged
 * with the device's architecture name; entries of another architecture are
 * skipped on load).  cmm_ctx_create loads the file named by the environment
 * variable CMM_TUNE_CACHE when it is set and exists. */
int cmm_autotune(cmm_ctx* ctx, int64_t n1, int64_t m, int64_t n3, int64_t b, int32_t d,
                 int32_t dtype, int32_t* tuning, double* best_ms);
int cmm_tuning_get(const cmm_ctx* ctx, int64_t n1, int64_t m, int64_t n3, int64_t b, int32_t d,
                   int32_t dtype, int32_t* tuning);
int cmm_tuning_set(cmm_ctx* ctx, int64_t n1, int64_t m, int64_t n3, int64_t b, int32_t d,
                   int32_t dtype, const int32_t* tuning);
int cmm_tuning_save(const cmm_ctx* ctx, const char* path);
int cmm_tuning_load(cmm_ctx* ctx, const char* path);

/* ---- Frobenius-norm bound (Section 5.2) -------------------------------- */

/* Upper bound on ||AB||_F^2 from AMS sketches (Section 2.1): for every
 * repetition t, X_t = sum_ij s1_t(i) s2_t(j) (AB)_ij, computed without AB as
 * sum_k (sum_i s1_t(i) A_ik)(sum_j s2_t(j) B_kj).  s1_t and s2_t are 4-wise
 * independent: the parity of a degree-3 polynomial (a0 + a1 x + a2 x^2 +
 * a3 x^3) mod (2^61 - 1), s = +1 if even, with a_c = z mod (2^61 - 1) for
 * z = output 1024 + 8t + 4f + c + 1 of the seed's SplitMix64 stream (f = 0
 * for s1, 1 for s2).  X_t^2 is unbiased for ||AB||_F^2 with variance at most
 * 8 (||AB||_F^2)^2; *bound = 32 * median_t X_t^2 (Section 5.2).  Operands,
 * dtype and scales as in cmm_sketch_product_ex; flags: CMM_SUBTRACT_DIAG
 * (the bound for AB with its diagonal zeroed, n1 == n3) and CMM_ASYNC (then
 * X and bound must be NULL).  X (host, d values) and bound (host) may be
 * NULL.  Sums are float64.  1 <= d <= 63. */
int cmm_frobenius_bound(cmm_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                        int64_t n1, int64_t m, int64_t n3, int32_t dtype, const float* scaleA,
                        const float* scaleB, int32_t d, uint64_t seed, uint32_t flags, double* X,
                        double* bound);

/* Host copies of the sign tables of cmm_frobenius_bound (s1[d*n1],
 * s2[d*n3] in {-1,+1}; either may be NULL), for the bit-exact check. */
int cmm_frobenius_signs(cmm_ctx* ctx, int64_t n1, int64_t n3, int32_t d, uint64_t seed,
                        int8_t* s1, int8_t* s2);

/* ---- number of non-zeros (Section 5.1) --------------------------------- */

/* Doubling search for an upper bound on the number of non-zero entries of
 * AB: the operands are scaled by random diagonal matrices D1 (rows of A)
 * and D2 (columns of B), entries uniform in [1, 2) drawn from the seed's
 * SplitMix64 stream at outputs 2^40 + i + 1 and 2^41 + j + 1 (so sums of
 * non-zero entries do not cancel), and D1 A B D2 is sketched at b = 16, 32,
 * ..., 2^20 with the hash functions of `seed`.  The search stops at the
 * first b for which at least 4b/5 buckets are zero for all d hash functions
 * (a bucket is zero when |c_t[u]| <= zero_rel * max_u |c_t[u]|; the float32
 * sketch is never exactly 0); *b_out = that b, an upper bound on nnz(AB)
 * with probability 1 - (3/4)^d and at most about 10 nnz(AB), or -1 if no
 * b <= 2^20 qualifies.  zeros (host, d values, may be NULL) receives the
 * zero counts of the last b tried.  Operands as in cmm_sketch_product_ex;
 * flags: CMM_SUBTRACT_DIAG (count the product with a zero diagonal). */
int cmm_estimate_nnz(cmm_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                     int64_t n1, int64_t m, int64_t n3, int32_t dtype, const float* scaleA,
                     const float* scaleB, int32_t d, uint64_t seed, uint32_t flags, double zero_rel,
                     int64_t* b_out, int64_t* zeros);

/* ---- sublinear extraction (Section 4, Figure 3) ----------------------- */

/* FINDSIGNIFICANTENTRIES(delta): positions (i, j) of significant entries of
 * AB.  Besides the sketch of AB, the library computes with the same hash
 * functions the sketches of the submatrix products of eq. (3),
 * (I_{E_r} A) B for the 63 bits of the row code and A (B I_{E_r}) for the
 * 63 bits of the column code.  E is the binary BCH code of length 63 with
 * designed distance 23 (16 information bits; any 11 bit errors are
 * corrected): index x is the systematic codeword of message x + 1, so
 * n1, n3 <= 65535.  (The paper names an expander code; any code that
 * corrects a constant fraction of errors serves, and this one corrects
 * 11/63 of them.)  For every repetition t and bucket k the two 63-bit strings
 * [|p^(t,r)[k]| > delta/2] are decoded (syndromes, Berlekamp-Massey, Chien
 * search); a string that does not decode, or decodes to message 0 (a bucket
 * without a significant entry thresholds to weight <= 11), gives nothing.
 * Positions decoded in at least d/2 repetitions are returned, sorted by
 * i*n3 + j, at most `cap` of them in out_i/out_j (host arrays), with
 * *out_count the full number (call again with a larger cap if it exceeds
 * cap).  Operands, dtype, scales, b, d, seed as in cmm_sketch_product_ex;
 * flags: CMM_SUBTRACT_DIAG (the product with a zero diagonal).  main_out,
 * if non-NULL, receives the sketch of AB itself (for DECOMPRESS of the
 * returned positions); free it with cmm_sketch_free().  The work is
 * 2 * 63 + 1 sketch products (Section 4: a factor O(lg n) more time for
 * compression). */
int cmm_find_significant(cmm_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                         int64_t n1, int64_t m, int64_t n3, int32_t dtype, const float* scaleA,
                         const float* scaleB, int64_t b, int32_t d, uint64_t seed, uint32_t flags,
                         double delta, int64_t cap, int64_t* out_i, int64_t* out_j,
                         int64_t* out_count, cmm_sketch** main_out);

/* ---- decoding (DECOMPRESS, Figure 1) ---------------------------------- */

/* Estimate of (AB)_ij: median over t of s1_t(i) s2_t(j) c_t[(h1_t(i) +
 * h2_t(j)) mod b]; for even d the mean of the two middle values.  Result in
 * host memory. */
int cmm_estimate(const cmm_sketch* sk, int64_t i, int64_t j, double* out);

/* Batched estimates of q pairs (device arrays i[q], j[q]; device out[q]). */
int cmm_estimate_batch(const cmm_sketch* sk, const int64_t* i, const int64_t* j, int64_t q,
                       float* out);

/* The K estimates of largest magnitude in the candidate domain `mode`,
 * ordered by |C_ij| descending and then by linear index i*n3 + j ascending
 * (ties between equal magnitudes therefore resolve to the smaller index).
 * Outputs are host arrays of K entries (n3*K for CMM_TOPK_PER_COLUMN, column
 * j's results at [j*K, (j+1)*K)).  The estimates are decoded on the device
 * and never stored as a whole matrix.
 * Limits (CMM_EUNSUPPORTED): for CMM_TOPK_ALL and CMM_TOPK_UPPER, K <= 2048
 * (the last ranking sorts at most 4096 candidates in one block's LDS) and
 * at most 4096 estimates may tie at the K-th magnitude (ties are common
 * only with d = 1, where every entry of a bucket has the same magnitude).
 * Section 4's goal of the b/kappa largest entries exceeds 2048 at b >= 2^16
 * with kappa <= 32; that extraction is cmm_find_significant, which has no
 * such cap.  CMM_TOPK_PER_COLUMN takes any K up to n1. */
int cmm_topk(const cmm_sketch* sk, int32_t K, int32_t mode, int64_t* out_i, int64_t* out_j,
             float* out_val);

#ifdef __cplusplus
}
#endif

#endif /* CMM_H */

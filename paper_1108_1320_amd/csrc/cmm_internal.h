// Internal declarations of the cmm HIP library (not part of the C ABI).
//
// Data layout in HBM for one product AB (A n1 x m column-major, B m x n3
// row-major; "side" 0 hashes the rows i of A with (h1, s1), side 1 the
// columns j of B with (h2, s2)):
//
//   hs[side][t][x]        int32  (h(x) << 1) | (s(x) == -1)
//   cnt[side][t][u]       int32  members of bucket u (u < b)
//   pos[side][t][u]       int32  layout position of non-empty bucket u, -1 if empty
//   ent[side][t][p]       uint32 FFT fold entry of position p: 8 (u div T) << 16 | 8 fold_slot(u)
//                                (padding: an own slot of the segment's wave, weight index 0)
//   tab[side][t][p]       uint32 first member | sign << 31 | more-members << 30
//   SA[side][t][k][p]     float  count sketch of column k (side 0) / row k (side 1)
//   colmax[side][t][k]    float  max |SA[side][t][k][.]| (fixed-point scale of the fold)
//   Ppart[t][ks][f1][f2]  float2 partial spectral sums of one k-split (<= 128 k)
//   c64[t][u], c32[t][u]  the sketch
//
// Layout positions: the fused FFT kernel works on C-point rows with T = C/16
// threads; the thread that owns slot r (r = u mod C) is r mod T, and the
// wave that owns it is (u mod T) / G with G = min(T, 64).  Each of the
// W = T / G waves gets one segment of Lcap positions holding the non-empty
// buckets it owns (increasing u), padded to a multiple of 64 (lseg[side][t]).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define CMM_P61 0x1FFFFFFFFFFFFFFFull
#define CMM_PAD_TAB 0xFFFFFFFFu
#define CMM_TAB_NEG 0x80000000u
#define CMM_TAB_MORE 0x40000000u
#define CMM_TAB_IDX 0x3FFFFFFFu

namespace cmm {

// LDS index swizzle of the FFT kernel's C-point buffers: xor the low 4 bits
// with bits 4..7 (a bijection on [0, C)).
__host__ __device__ __forceinline__ int fft_swizzle(int i) { return i ^ ((i >> 4) & 15); }

// (a x + c) mod (2^61 - 1) for a, c < 2^61 - 1 and x < 2^32, exact: the
// 93-bit product is folded with 2^61 = 1 (mod p).  One step of Horner's rule
// for longer polynomials.
__device__ __forceinline__ uint64_t cw_hash61(uint64_t a, uint64_t x, uint64_t c) {
  uint64_t lo = a * x;
  uint64_t hi = __umul64hi(a, x);           // < 2^29 since a < 2^61, x < 2^32
  uint64_t s = lo + c;
  hi += (s < lo) ? 1ull : 0ull;
  // v = hi 2^64 + s and 2^64 = 8 (mod p): fold both words into 61-bit digits
  uint64_t r = (s & CMM_P61) + (s >> 61) + (hi << 3);
  r = (r & CMM_P61) + (r >> 61);
  if (r >= CMM_P61) r -= CMM_P61;
  return r;
}

// Output k (k >= 1) of SplitMix64 seeded with `seed` (Steele, Lea, Flood
// 2014): the counter seed + k * gamma mixed by two xor-shift-multiply rounds.
__device__ __forceinline__ uint64_t splitmix64_dev(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// OCP e4m3fn code (low 8 bits of v) to float32: bias 7, no infinities,
// S.1111.111 is NaN, subnormals m * 2^-9.
__device__ __forceinline__ float e4m3fn_to_f32(uint32_t v) {
  uint32_t sign = (v & 0x80u) << 24;
  uint32_t e = (v >> 3) & 0xFu, mnt = v & 7u;
  float mag;
  if (e == 0) mag = (float)mnt * 0x1p-9f;
  else if (e == 15 && mnt == 7) mag = __uint_as_float(0x7FC00000u);
  else mag = __uint_as_float(((e + 120u) << 23) | (mnt << 20));
  return __uint_as_float(__float_as_uint(mag) | sign);
}

// Element `off` of a stored operand as float32 (0: f32, 1: bf16 bits,
// 2: e4m3fn code; the fp8 column scale is applied by the caller).
template <int DT> __device__ __forceinline__ float load_deq(const void* X, int64_t off) {
  if constexpr (DT == 0) return ((const float*)X)[off];
  else if constexpr (DT == 1) return __uint_as_float((uint32_t)((const uint16_t*)X)[off] << 16);
  else return e4m3fn_to_f32(((const uint8_t*)X)[off]);
}

// Fold entry of bucket u for an FFT row of length C = 1 << log2c, as two
// byte offsets of 8-byte LDS elements: bits 0..15 hold 8 * (swizzled slot of
// u mod C) (C <= 8192), bits 16..31 hold 8 * (weight index u >> log2(C/16)),
// an index below 16 R <= 4096 for at most 256 rows.
__host__ __device__ __forceinline__ uint32_t fold_entry(uint32_t u, int log2c) {
  return ((u >> (log2c - 4)) << 19) |
         ((uint32_t)fft_swizzle((int)(u & ((1u << log2c) - 1))) << 3);
}

// Fold entry of padding position r of layout segment w (G lanes per
// segment): the first own slot of the lane that folds position r (lane
// r mod G), with weight index 0.  The count sketch stores 0 at padding
// positions, so folding one adds 0 to a slot of the folding lane itself
// (distinct lanes, distinct LDS addresses).
__host__ __device__ __forceinline__ uint32_t pad_entry(int w, int G, int r) {
  return (uint32_t)fft_swizzle(w * G + r % G) << 3;
}

// Fold entry of bucket u for the row pair {0, R/2} (C = 2^log2c): the LDS
// byte offset of its slot s = (u mod 2C) div 2 (swizzled), with the parity
// of u in bit 0 (0: the real part of the slot, 1: the imaginary part).  The
// offset is a multiple of 8 below 8C <= 2^16, so the entry fits 16 bits.
// Padding positions use pad_entry's value (parity 0, value 0).
__host__ __device__ __forceinline__ uint16_t pair_entry(uint32_t u, int log2c) {
  const uint32_t s = (u & ((2u << log2c) - 1u)) >> 1;
  return (uint16_t)(((uint32_t)fft_swizzle((int)s) << 3) | (u & 1u));
}

constexpr int kMaxLog2C = 13;          // FFT row length C <= 8192
// Hashed dimensions n1, n3: rows up to kMaxStagedDim floats are staged in LDS
// by the count-sketch kernel (sparse operands always are); dense rows up to
// kMaxHashedDim are read from global memory instead.  n1 * n3 < 2^32 keeps
// every top-K histogram count inside uint32.
constexpr int kMaxStagedDim = 24576;
constexpr int kMaxHashedDim = 65535;
// per-column top-K keeps a column's keys in LDS up to this many rows and
// recomputes them each round above it
constexpr int kMaxColumnKeys = 40704;   // 159 KB of keys + the static shared words
constexpr int kTopkCap = 4096;         // candidates sorted by the final top-K pass
constexpr int kMaxKPerBlock = 128;     // k per FFT block (float32 partial sums)

// Element type codes of a stored operand: 0 f32, 1 bf16, 2 fp8 e4m3fn, and
// 3 sparse f32 (row k's entries at sptr[k] .. sptr[k+1] of sidx / X).
constexpr int kSparseF32 = 3;

struct SideDesc {
  const void* X;        // stored operand (k-major rows of length n); sparse: the values
  int64_t ld;           // row stride in elements (dense)
  const int64_t* sptr = nullptr;   // sparse: row offsets [m + 1]
  const int32_t* sidx = nullptr;   // sparse: index of each entry in [0, n)
  const float* scale;   // per-element-position scale (fp8) or nullptr
  int n;                // hashed dimension (n1 or n3)
  int32_t* hs;          // [d][n]
  int32_t* cnt;         // [d][b]
  int32_t* pos;         // [d][b]
  uint32_t* ent;        // [d][Lrow] fold entries of the rows (fold_entry)
  uint16_t* entp;       // [d][Lrow] fold entries of the row pair (pair_entry)
  uint32_t* tab;        // [d][Lrow]
  int32_t* cntp;        // [d][Lrow]
  int32_t* moff;        // [d][Lrow]
  int32_t* fill;        // [d][Lrow]
  int32_t* perm;        // [d][n]
  int32_t* segcount;    // [d][W]
  int32_t* lseg;        // [d]
  float* SA;            // [d][m][Lrow]
  float* colmax;        // [d][m] max |SA| of each sketched column / row
  int Lcap;             // positions per segment
  int Lrow;             // W * Lcap
};

// Launch-shape choices of one product (picked by the autotuner or defaults):
// FFT row length 2^log2c (its radix sequence: 2^(log2c mod 4) then 16s),
// at most kmax values of k per FFT block (the float32 partial-sum length),
// and the number of countsketch blocks.  The defaults are the autotuner's
// choice for the covariance and transform workloads with n = 4096..16384
// measured on gfx950.
struct Tuning {
  int log2c = 12;
  int kmax = 32;
  int cs_blocks = 4096;
};

struct Geometry {
  int64_t b;
  int log2b;
  int d;
  int m;
  int log2c;            // FFT row length C = 1 << log2c
  int T;                // threads of the FFT kernel = C / 16
  int G;                // lanes per segment class group = min(T, 64)
  int W;                // segments = T / G
  int R;                // rows of the four-step split = b / C
  int rows;             // computed rows (R/2 + 1, or 1 when R == 1)
  int rblocks;          // FFT blocks per (repetition, k-split): R/2 (rows 0
                        // and R/2 share one), or 1 when R == 1
  int KS;               // k-splits of the FFT kernel
  int cs_blocks;        // countsketch blocks
};

// ---- kernel launchers (stream-ordered, return hipError_t) ----
hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s);
hipError_t launch_twiddles(double2* tw64, float2* tw32, int64_t b, hipStream_t s);
hipError_t launch_params_from_seed(uint64_t seed, int d, uint64_t* out, hipStream_t s);
hipError_t launch_hash(const uint64_t* params_dev, int side, const Geometry& g, SideDesc& sd,
                       hipStream_t s);
hipError_t launch_count(const Geometry& g, SideDesc& sd, hipStream_t s);
hipError_t launch_layout(const Geometry& g, SideDesc& sd, int32_t* overflow, hipStream_t s);
hipError_t prepare_countsketch();
hipError_t prepare_fft_mac();
hipError_t prepare_decode();
hipError_t launch_countsketch(int dtype, const Geometry& g, SideDesc& sd, hipStream_t s);
// A second stream and two events with which the row-pair kernel of the
// spectral step runs beside the row kernel (a fork from and a join back to
// the launching stream).
struct Overlap {
  hipStream_t aux = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
hipError_t launch_fft_mac(const Geometry& g, const SideDesc& a, const SideDesc& bside,
                          const float2* tw32, float2* Ppart, hipStream_t s,
                          const Overlap* ov = nullptr);
hipError_t launch_ifft(const Geometry& g, const float2* Ppart, double2* work0, double2* work1,
                       const double2* tw64, double* c64, hipStream_t s);
hipError_t launch_diag(int dtype, const SideDesc& a, const SideDesc& bside, int m, int n,
                       double* partial, int kchunks, double* diag, hipStream_t s);
// tmp: device scratch of at least 16 * d * b bytes (the inverse FFT's work
// buffer after the inverse FFT)
hipError_t launch_sub_diag(const Geometry& g, const int32_t* hs1, const int32_t* hs2, int n1,
                           int n3, const double* diag, int len, double* c64, void* tmp,
                           hipStream_t s);
hipError_t launch_to_f32(const double* c64, float* c32, int64_t count, hipStream_t s);
hipError_t launch_add_f64(double* dst, const double* src, int64_t count, hipStream_t s);
hipError_t launch_ams_signs(const uint64_t* params, int d, int side, int n, uint64_t* mask,
                            hipStream_t s);
hipError_t launch_ams_rows(int dtype, const void* X, int64_t ld, const float* scale, int n, int m,
                           int d, const uint64_t* mask, double* out, hipStream_t s);
hipError_t launch_ams_final(const double* u, const double* v, int m, int d, const uint64_t* mask1,
                            const uint64_t* mask2, const double* diag, int ndiag, double* X,
                            hipStream_t s);
// The extraction's code: codewords of messages x + 1 (x < n) of the
// length-63 BCH code with generator g (bit mask of degree 47), masks of bit
// r, and the decode of every (t, k) into a key i * n3 + j or -1.
hipError_t launch_code_words(int n, uint64_t g, uint64_t* cw, hipStream_t s);
hipError_t launch_code_mask(int n, int r, const uint64_t* cw, const float* scale, float* out,
                            hipStream_t s);
hipError_t launch_code_mask_diag(int n, int r, const uint64_t* cw, const double* diag, double* out,
                                 hipStream_t s);
hipError_t launch_extract_decode(const float* c, int d, int64_t b, int n1, int n3, float half_delta,
                                 int64_t* keys, hipStream_t s);
hipError_t launch_vote(const int64_t* keys, int64_t nkeys, unsigned long long* tkeys,
                       uint32_t* tcnt, int64_t tsize, int d, int64_t* out, uint32_t* count,
                       int64_t cap, hipStream_t s);
hipError_t launch_sparse_check(const int64_t* ptr, const int32_t* idx, int m, int n, int64_t nnz,
                               int32_t* bad, hipStream_t s);
hipError_t prepare_sparse();
hipError_t launch_nnz_weights(uint64_t seed, uint64_t offset, int n, const float* scale, float* out,
                              hipStream_t s);
hipError_t launch_nnz_zeros(const double* c, int d, int64_t b, double rel, int64_t* zeros,
                            hipStream_t s);
hipError_t launch_fill_random(void* X, int64_t count, int dtype, uint64_t seed, hipStream_t s);
hipError_t launch_stream_probe(const void* src, void* dst, float* sink, int64_t read_bytes,
                               int64_t write_bytes, bool nt, hipStream_t s);

struct DecodeDesc {
  const int32_t* hs1;   // [d][n1]
  const int32_t* hs2;   // [d][n3]
  const float* c32;     // [d][b]
  int n1, n3, d;
  uint32_t mask;        // b - 1
  int64_t b;
};

struct TopkCand {
  uint32_t key;         // float bits of |estimate|
  int32_t i, j;
  float val;
};

hipError_t launch_estimate(const DecodeDesc& dd, const int64_t* qi, const int64_t* qj, int64_t q,
                           float* out, hipStream_t s);
// screen: optional bitmap of launch_screen_bits at the same threshold (only
// read when cand is given, i.e. in the collecting pass).
hipError_t launch_topk_hist(const DecodeDesc& dd, int mode, int tile_stride, uint32_t prefix,
                            int prefix_shift, int digit_shift, uint32_t digit_mask, uint32_t* hist,
                            uint32_t thresh, TopkCand* cand, uint32_t* count, int cap,
                            hipStream_t s, const uint32_t* screen = nullptr, int screen_log2w = 0);
// Rows of the screening bitmap (d - ceil(d/2) + 1), its log2 width per row
// for (d, b) (0: no screen), and the kernel that builds it for a threshold.
int screen_nf(int d);
int screen_log2w(int d, int64_t b);
hipError_t launch_screen_bits(const DecodeDesc& dd, uint32_t thresh, int log2w, uint32_t* bits,
                              hipStream_t s);
hipError_t launch_topk_filter(const TopkCand* in, const uint32_t* in_count, int in_cap,
                              uint32_t thresh, TopkCand* out, uint32_t* out_count, int out_cap,
                              hipStream_t s);
hipError_t launch_topk_collect(const DecodeDesc& dd, int mode, uint32_t thresh, TopkCand* cand,
                               uint32_t* count, int cap, hipStream_t s);
hipError_t launch_topk_final(const TopkCand* cand, const uint32_t* count, int cap, int K, int n3,
                             int64_t* oi, int64_t* oj, float* ov, hipStream_t s);
hipError_t launch_topk_column(const DecodeDesc& dd, int K, int64_t* oi, float* ov, hipStream_t s);

}  // namespace cmm

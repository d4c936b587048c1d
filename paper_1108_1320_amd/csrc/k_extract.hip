// Sublinear extraction of significant entries (Section 4, Figure 3).
//
// The sketches of the submatrix products of eq. (3) -- (I_{E_r} A) B and
// A (B I_{E_r}), same hash functions -- are ordinary sketch products whose
// operand rows (columns) are weighted by bit r of a code E of the index.
// E is the binary BCH code of length 63 with designed distance 23 (16
// information bits, corrects any 11 errors): index x is the systematic
// codeword of message x + 1, with the message in bits 47..62 and the
// parity (message * x^47 mod g) in bits 0..46.  For every repetition t and
// bucket k, the magnitudes of the 63 row-code and 63 column-code sketches
// at k are compared with Delta/2; each 63-bit string is decoded (syndromes
// in GF(2^6), Berlekamp-Massey, Chien search) and a position (i, j) is
// produced when both decode to a non-zero message.  Positions decoded in at
// least d/2 repetitions are kept (a multiset held in a hash table).
#include "cmm_internal.h"

namespace cmm {

constexpr int kCodeLen = 63;     // bits of the code of one index
constexpr int kCodeT = 11;       // errors it corrects
constexpr int kCodePar = 47;     // parity bits (degree of the generator)

// (msg * x^47) mod g over GF(2), g of degree 47 (bit masks)
__host__ __device__ __forceinline__ uint64_t bch_parity(uint64_t msg, uint64_t g) {
  uint64_t r = msg << kCodePar;
  for (int bit = kCodePar + 15; bit >= kCodePar; --bit)
    if ((r >> bit) & 1) r ^= g << (bit - kCodePar);
  return r;
}

// cw[x] = codeword of message x + 1 (63 bits)
__global__ void k_code_words(int n, uint64_t g, uint64_t* __restrict__ cw) {
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
    const uint64_t msg = (uint64_t)(x + 1);
    cw[x] = (msg << kCodePar) | bch_parity(msg, g);
  }
}

// out[x] = E(x)_r * (scale ? scale[x] : 1)
__global__ void k_code_mask(int n, int r, const uint64_t* __restrict__ cw,
                            const float* __restrict__ scale, float* __restrict__ out) {
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x)
    out[x] = ((cw[x] >> r) & 1) ? (scale ? scale[x] : 1.0f) : 0.0f;
}

// out[i] = E(i)_r * diag[i]: the diagonal of the masked product
__global__ void k_code_mask_diag(int n, int r, const uint64_t* __restrict__ cw,
                                 const double* __restrict__ diag, double* __restrict__ out) {
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x)
    out[x] = ((cw[x] >> r) & 1) ? diag[x] : 0.0;
}

// GF(2^6) with the primitive polynomial x^6 + x + 1: exp over two periods
// (so log a + log b indexes it directly) and log, in LDS.
struct Gf64 {
  uint8_t exp[128];
  uint8_t log[64];
};

__device__ __forceinline__ int gf_mul(const Gf64& f, int a, int b) {
  return (a == 0 || b == 0) ? 0 : f.exp[f.log[a] + f.log[b]];
}

// The message of the codeword within distance 11 of w, or -1 when the
// decoder finds none.
__device__ int bch_decode(const Gf64& f, uint64_t w) {
  // syndromes S_j = w(alpha^j), j = 1 .. 22; S_2j = S_j^2 for a binary word
  int S[2 * kCodeT + 1];
#pragma unroll
  for (int j = 0; j <= 2 * kCodeT; ++j) S[j] = 0;
  for (uint64_t bits = w; bits; bits &= bits - 1) {
    const int p = __builtin_ctzll(bits);
#pragma unroll
    for (int j = 1; j <= 2 * kCodeT; j += 2) S[j] ^= f.exp[(j * p) % 63];
  }
  bool zero = true;
#pragma unroll
  for (int j = 1; j <= 2 * kCodeT; ++j) {
    if (j % 2 == 0) S[j] = gf_mul(f, S[j / 2], S[j / 2]);
    zero = zero && S[j] == 0;
  }
  if (zero) return (int)(w >> kCodePar);
  // Berlekamp-Massey: shortest linear recurrence sigma generating S_1..S_22
  int sig[kCodeT + 2], prv[kCodeT + 2];
#pragma unroll
  for (int i = 0; i < kCodeT + 2; ++i) { sig[i] = 0; prv[i] = 0; }
  sig[0] = 1; prv[0] = 1;
  int L = 0, m = 1, bprev = 1;
#pragma unroll
  for (int n = 0; n < 2 * kCodeT; ++n) {
    int disc = S[n + 1];
#pragma unroll
    for (int i = 1; i <= kCodeT + 1; ++i)
      if (i <= n && i <= L) disc ^= gf_mul(f, sig[i], S[n + 1 - i]);
    if (disc == 0) { ++m; continue; }
    const int coef = gf_mul(f, disc, f.exp[(63 - f.log[bprev]) % 63]);
    int nxt[kCodeT + 2];
#pragma unroll
    for (int i = 0; i < kCodeT + 2; ++i) nxt[i] = sig[i];
    // nxt += coef * x^m * prv (terms above degree kCodeT + 1 mean failure)
    bool over = false;
#pragma unroll
    for (int i = 0; i < kCodeT + 2; ++i) {
      if (prv[i] == 0) continue;
      const int dst = i + m;
      if (dst < kCodeT + 2) nxt[dst] ^= gf_mul(f, coef, prv[i]);
      else over = true;
    }
    if (over) return -1;
    if (2 * L <= n) {
#pragma unroll
      for (int i = 0; i < kCodeT + 2; ++i) prv[i] = sig[i];
      L = n + 1 - L; bprev = disc; m = 1;
    } else {
      ++m;
    }
#pragma unroll
    for (int i = 0; i < kCodeT + 2; ++i) sig[i] = nxt[i];
  }
  if (L > kCodeT) return -1;
  // Chien search: position p is in error when sigma(alpha^-p) = 0
  int roots = 0;
  uint64_t fix = 0;
  for (int p = 0; p < kCodeLen; ++p) {
    int acc = 0;
#pragma unroll
    for (int i = 0; i <= kCodeT; ++i)
      if (i <= L && sig[i]) acc ^= f.exp[(f.log[sig[i]] + (63 - p) * i) % 63];
    if (acc == 0) { ++roots; fix |= 1ull << p; }
  }
  if (roots != L) return -1;
  return (int)((w ^ fix) >> kCodePar);
}

// One thread per (t, k): key = i * n3 + j, or -1 when either string does not
// decode to a non-zero message inside the index range.  c holds the 63
// row-code sketches then the 63 column-code ones, each [t][k] float32.  A
// string of weight at most 11 lies within distance 11 of the zero codeword
// (message 0) and is skipped without decoding.
__global__ __launch_bounds__(256) void k_extract_decode(const float* __restrict__ c, int d, int64_t b,
                                                        int n1, int n3, float half_delta,
                                                        int64_t* __restrict__ keys) {
  __shared__ Gf64 f;
  if (threadIdx.x == 0) {
    int v = 1;
    for (int i = 0; i < 63; ++i) {
      f.exp[i] = f.exp[i + 63] = (uint8_t)v;
      f.log[v] = (uint8_t)i;
      v <<= 1;
      if (v & 64) v ^= 0x43;
    }
    f.exp[126] = f.exp[127] = 0;
    f.log[0] = 0;
  }
  __syncthreads();
  const int64_t total = (int64_t)d * b;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    uint64_t wr = 0, wc = 0;
    for (int r = 0; r < kCodeLen; ++r) {
      wr |= (uint64_t)(fabsf(c[(int64_t)r * total + idx]) > half_delta) << r;
      wc |= (uint64_t)(fabsf(c[(int64_t)(kCodeLen + r) * total + idx]) > half_delta) << r;
    }
    int64_t key = -1;
    if (__popcll(wr) > kCodeT && __popcll(wc) > kCodeT) {
      const int mi = bch_decode(f, wr);
      const int mj = mi > 0 ? bch_decode(f, wc) : -1;
      if (mi > 0 && mj > 0 && mi - 1 < n1 && mj - 1 < n3) key = (int64_t)(mi - 1) * n3 + (mj - 1);
    }
    keys[idx] = key;
  }
}

constexpr unsigned long long kEmptyKey = ~0ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Multiset insertion: open addressing with linear probing; the table holds
// at least twice as many slots as keys, so every probe sequence ends.
__global__ void k_vote_insert(const int64_t* __restrict__ keys, int64_t nkeys,
                              unsigned long long* __restrict__ tkeys, uint32_t* __restrict__ tcnt,
                              uint64_t tmask) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < nkeys;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t key = keys[idx];
    if (key < 0) continue;
    uint64_t h = mix64((uint64_t)key) & tmask;
    for (uint64_t probe = 0; probe <= tmask; ++probe) {
      const unsigned long long prev = atomicCAS(&tkeys[h], kEmptyKey, (unsigned long long)key);
      if (prev == kEmptyKey || prev == (unsigned long long)key) {
        atomicAdd(&tcnt[h], 1u);
        break;
      }
      h = (h + 1) & tmask;
    }
  }
}

// Keep the positions inserted at least d/2 times.
__global__ void k_vote_collect(const unsigned long long* __restrict__ tkeys,
                               const uint32_t* __restrict__ tcnt, int64_t size, int d,
                               int64_t* __restrict__ out, uint32_t* __restrict__ count, int64_t cap) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < size;
       s += (int64_t)gridDim.x * blockDim.x) {
    if (tkeys[s] != kEmptyKey && 2u * tcnt[s] >= (uint32_t)d) {
      const uint32_t slot = atomicAdd(count, 1u);
      if ((int64_t)slot < cap) out[slot] = (int64_t)tkeys[s];
    }
  }
}

static unsigned grid_n(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return (unsigned)g;
}

hipError_t launch_code_words(int n, uint64_t g, uint64_t* cw, hipStream_t s) {
  hipLaunchKernelGGL(k_code_words, dim3(grid_n(n)), dim3(256), 0, s, n, g, cw);
  return hipGetLastError();
}

hipError_t launch_code_mask(int n, int r, const uint64_t* cw, const float* scale, float* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_code_mask, dim3(grid_n(n)), dim3(256), 0, s, n, r, cw, scale, out);
  return hipGetLastError();
}

hipError_t launch_code_mask_diag(int n, int r, const uint64_t* cw, const double* diag, double* out,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_code_mask_diag, dim3(grid_n(n)), dim3(256), 0, s, n, r, cw, diag, out);
  return hipGetLastError();
}

hipError_t launch_extract_decode(const float* c, int d, int64_t b, int n1, int n3, float half_delta,
                                 int64_t* keys, hipStream_t s) {
  hipLaunchKernelGGL(k_extract_decode, dim3(grid_n((int64_t)d * b)), dim3(256), 0, s, c, d, b, n1,
                     n3, half_delta, keys);
  return hipGetLastError();
}

hipError_t launch_vote(const int64_t* keys, int64_t nkeys, unsigned long long* tkeys,
                       uint32_t* tcnt, int64_t tsize, int d, int64_t* out, uint32_t* count,
                       int64_t cap, hipStream_t s) {
  hipLaunchKernelGGL(k_vote_insert, dim3(grid_n(nkeys)), dim3(256), 0, s, keys, nkeys, tkeys, tcnt,
                     (uint64_t)(tsize - 1));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vote_collect, dim3(grid_n(tsize)), dim3(256), 0, s, tkeys, tcnt, tsize, d,
                     out, count, cap);
  return hipGetLastError();
}

}  // namespace cmm

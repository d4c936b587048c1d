// Sublinear extraction of significant entries (Section 4, Figure 3).
//
// The sketches of the submatrix products of eq. (3) -- (I_{E_r} A) B and
// A (B I_{E_r}), same hash functions -- are ordinary sketch products whose
// operand rows (columns) are weighted by bit r of a code E of the index.
// The code is the complement code E(x) = bits(x) || not bits(x) over L
// information bits.  For every repetition t and bucket k, the magnitudes of
// the 2 L1 row-code and 2 L3 column-code sketches at k are compared with
// Delta/2 and the resulting bit string is decoded into a position (i, j)
// (or rejected when a bit pair is not complementary); positions decoded in
// at least d/2 repetitions are kept (a multiset held in a hash table).
#include "cmm_internal.h"

namespace cmm {

__device__ __forceinline__ int code_bit(int64_t x, int L, int r) {
  return r < L ? (int)((x >> r) & 1) : 1 - (int)((x >> (r - L)) & 1);
}

// out[x] = E(x)_r * (scale ? scale[x] : 1)
__global__ void k_code_mask(int n, int L, int r, const float* __restrict__ scale,
                            float* __restrict__ out) {
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x)
    out[x] = code_bit(x, L, r) ? (scale ? scale[x] : 1.0f) : 0.0f;
}

// out[i] = E(i)_r * diag[i]: the diagonal of the masked product
__global__ void k_code_mask_diag(int n, int L, int r, const double* __restrict__ diag,
                                 double* __restrict__ out) {
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x)
    out[x] = code_bit(x, L, r) ? diag[x] : 0.0;
}

// One thread per (t, k): key = i * n3 + j, or -1 when DECODE fails.
// c holds the row-code sketches (2 L1 of them) then the column-code ones
// (2 L3), each [t][k] float32.
__global__ void k_extract_decode(const float* __restrict__ c, int d, int64_t b, int L1, int L3,
                                 int n1, int n3, float half_delta, int64_t* __restrict__ keys) {
  const int64_t total = (int64_t)d * b;
  const int64_t stride = total;   // one sketch is d * b values
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    bool ok = true;
    int64_t i = 0, j = 0;
    for (int q = 0; q < L1 && ok; ++q) {
      const bool hi = fabsf(c[(int64_t)q * stride + idx]) > half_delta;
      const bool lo = fabsf(c[(int64_t)(q + L1) * stride + idx]) > half_delta;
      ok = hi != lo;
      i |= (int64_t)hi << q;
    }
    const float* cc = c + (int64_t)2 * L1 * stride;
    for (int q = 0; q < L3 && ok; ++q) {
      const bool hi = fabsf(cc[(int64_t)q * stride + idx]) > half_delta;
      const bool lo = fabsf(cc[(int64_t)(q + L3) * stride + idx]) > half_delta;
      ok = hi != lo;
      j |= (int64_t)hi << q;
    }
    keys[idx] = (ok && i < n1 && j < n3) ? i * n3 + j : -1;
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

hipError_t launch_code_mask(int n, int L, int r, const float* scale, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_code_mask, dim3(grid_n(n)), dim3(256), 0, s, n, L, r, scale, out);
  return hipGetLastError();
}

hipError_t launch_code_mask_diag(int n, int L, int r, const double* diag, double* out,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_code_mask_diag, dim3(grid_n(n)), dim3(256), 0, s, n, L, r, diag, out);
  return hipGetLastError();
}

hipError_t launch_extract_decode(const float* c, int d, int64_t b, int L1, int L3, int n1, int n3,
                                 float half_delta, int64_t* keys, hipStream_t s) {
  hipLaunchKernelGGL(k_extract_decode, dim3(grid_n((int64_t)d * b)), dim3(256), 0, s, c, d, b, L1,
                     L3, n1, n3, half_delta, keys);
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

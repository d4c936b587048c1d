// Number of non-zeros of AB by doubling search (Section 5.1): the operands
// are scaled by random diagonal matrices (so a sum of non-zero entries of
// D1 A B D2 vanishes with probability 0, by the Schwartz-Zippel argument of
// the paper), sketched at b = 16, 32, ..., and the search stops at the
// first b for which at least 4b/5 buckets are zero for every hash function.
#include "cmm_internal.h"

namespace cmm {

// out[x] = float(1 + (z_{offset + x + 1} >> 11) 2^-53) * (scale ? scale[x] : 1)
__global__ void k_nnz_weights(uint64_t seed, uint64_t offset, int n, const float* __restrict__ scale,
                              float* __restrict__ out) {
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
    const double u = (double)(splitmix64_dev(seed, offset + (uint64_t)x + 1) >> 11) * 0x1p-53;
    const float w = (float)(1.0 + u);
    out[x] = scale ? w * scale[x] : w;
  }
}

// One block per repetition: zeros[t] = #{u : |c_t[u]| <= rel * max_u |c_t[u]|}.
__global__ __launch_bounds__(256) void k_nnz_zeros(const double* __restrict__ c, int64_t b,
                                                   double rel, int64_t* __restrict__ zeros) {
  __shared__ double smax[4];
  __shared__ unsigned long long scnt[4];
  const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double* ct = c + (int64_t)t * b;
  double mx = 0.0;
  for (int64_t u = tid; u < b; u += 256) mx = fmax(mx, fabs(ct[u]));
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) smax[wv] = mx;
  __syncthreads();
  mx = fmax(fmax(smax[0], smax[1]), fmax(smax[2], smax[3]));
  const double thr = rel * mx;
  unsigned long long cnt = 0;
  for (int64_t u = tid; u < b; u += 256) cnt += fabs(ct[u]) <= thr ? 1ull : 0ull;
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
  if (lane == 0) scnt[wv] = cnt;
  __syncthreads();
  if (tid == 0) zeros[t] = (int64_t)(scnt[0] + scnt[1] + scnt[2] + scnt[3]);
}

hipError_t launch_nnz_weights(uint64_t seed, uint64_t offset, int n, const float* scale, float* out,
                              hipStream_t s) {
  int blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_nnz_weights, dim3(blocks), dim3(256), 0, s, seed, offset, n, scale, out);
  return hipGetLastError();
}

hipError_t launch_nnz_zeros(const double* c, int d, int64_t b, double rel, int64_t* zeros,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_nnz_zeros, dim3(d), dim3(256), 0, s, c, b, rel, zeros);
  return hipGetLastError();
}

}  // namespace cmm

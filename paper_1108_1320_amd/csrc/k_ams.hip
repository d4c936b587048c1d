// Upper bound on the Frobenius norm of AB (Section 5.2) from AMS sketches
// (Section 2.1).  For every repetition t the AMS sketch of the weighted set
// AB with product signs s(i,j) = s1_t(i) s2_t(j) is a sum over the outer
// products of eq. (1), and the sketch of one outer product is the product of
// the two vectors' sketches:
//
//   X_t = sum_k u_t[k] v_t[k],   u_t[k] = sum_i s1_t(i) A_ik,
//                                v_t[k] = sum_j s2_t(j) B_kj.
//
// u and v are two sign-weighted row sums over the stored operands (one read
// of A and one of B for all repetitions); the signs come from degree-3
// polynomials mod 2^61 - 1 (a 4-wise independent family, as Section 5.2
// asks).  Sums are float64.
#include "cmm_internal.h"

namespace cmm {

// Sign masks: bit t of mask[x] is set when s_t(x) = -1, i.e. when the
// polynomial value a0 + a1 x + a2 x^2 + a3 x^3 (mod 2^61 - 1) is odd.
// params: [t][f][c] with f = 0 for s1, 1 for s2, c the power of x.
__global__ void k_ams_signs(const uint64_t* __restrict__ params, int d, int side, int n,
                            uint64_t* __restrict__ mask) {
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
    uint64_t m = 0;
    for (int t = 0; t < d; ++t) {
      const uint64_t* a = params + ((int64_t)t * 2 + side) * 4;
      // Horner: ((a3 x + a2) x + a1) x + a0
      uint64_t g = cw_hash61(a[3], (uint64_t)x, a[2]);
      g = cw_hash61(g, (uint64_t)x, a[1]);
      g = cw_hash61(g, (uint64_t)x, a[0]);
      m |= (g & 1ull) << t;
    }
    mask[x] = m;
  }
}

constexpr int kAmsThreads = 256;
constexpr int kAmsReps = 8;   // repetitions summed per sweep over a row

// One wave per row k of a stored operand (row k of A's storage holds
// A[., k]; row k of B holds B[k, .]): out[t][k] = sum_x s_t(x) X[k, x] for
// every repetition, eight repetitions per sweep (the row stays in cache),
// reduced across the wave with shuffles only.
template <int DT>
__global__ __launch_bounds__(kAmsThreads) void k_ams_rows(const void* __restrict__ X, int64_t ld,
                                                          const float* __restrict__ scale, int n,
                                                          int m, int d,
                                                          const uint64_t* __restrict__ mask,
                                                          double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int waves = gridDim.x * (kAmsThreads / 64);
  for (int k = blockIdx.x * (kAmsThreads / 64) + (threadIdx.x >> 6); k < m; k += waves) {
    for (int t0 = 0; t0 < d; t0 += kAmsReps) {
      double acc[kAmsReps];
#pragma unroll
      for (int q = 0; q < kAmsReps; ++q) acc[q] = 0.0;
      for (int x = lane; x < n; x += 64) {
        float v = load_deq<DT>(X, (int64_t)k * ld + x);
        if (scale) v *= scale[x];
        const double dv = (double)v;
        const uint64_t mk = mask[x] >> t0;
#pragma unroll
        for (int q = 0; q < kAmsReps; ++q) acc[q] += ((mk >> q) & 1ull) ? -dv : dv;
      }
#pragma unroll
      for (int q = 0; q < kAmsReps; ++q)
        for (int off = 32; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off, 64);
#pragma unroll
      for (int q = 0; q < kAmsReps; ++q)
        if (lane == q && t0 + q < d) out[(int64_t)(t0 + q) * m + k] = acc[q];
    }
  }
}

// One block per repetition: X_t = sum_k u_t[k] v_t[k], minus
// sum_i s1_t(i) s2_t(i) diag[i] when the diagonal is removed (the sketch of
// the product with a zero diagonal; the sketch is linear).
__global__ __launch_bounds__(kAmsThreads) void k_ams_final(const double* __restrict__ u,
                                                           const double* __restrict__ v, int m,
                                                           const uint64_t* __restrict__ mask1,
                                                           const uint64_t* __restrict__ mask2,
                                                           const double* __restrict__ diag,
                                                           int ndiag, double* __restrict__ X) {
  __shared__ double red[kAmsThreads / 64];
  const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double a = 0.0;
  for (int k = tid; k < m; k += kAmsThreads) a += u[(int64_t)t * m + k] * v[(int64_t)t * m + k];
  if (diag) {
    for (int i = tid; i < ndiag; i += kAmsThreads) {
      const bool neg = (((mask1[i] ^ mask2[i]) >> t) & 1ull) != 0;
      a -= neg ? -diag[i] : diag[i];
    }
  }
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
  if (lane == 0) red[wv] = a;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < kAmsThreads / 64; ++w) s += red[w];
    X[t] = s;
  }
}

hipError_t launch_ams_signs(const uint64_t* params, int d, int side, int n, uint64_t* mask,
                            hipStream_t s) {
  int blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_ams_signs, dim3(blocks), dim3(256), 0, s, params, d, side, n, mask);
  return hipGetLastError();
}

hipError_t launch_ams_rows(int dtype, const void* X, int64_t ld, const float* scale, int n, int m,
                           int d, const uint64_t* mask, double* out, hipStream_t s) {
  const int per = kAmsThreads / 64;
  int blocks = (m + per - 1) / per;
  if (blocks > 8192) blocks = 8192;
  if (dtype == 0)
    hipLaunchKernelGGL(k_ams_rows<0>, dim3(blocks), dim3(kAmsThreads), 0, s, X, ld, scale, n, m, d, mask, out);
  else if (dtype == 1)
    hipLaunchKernelGGL(k_ams_rows<1>, dim3(blocks), dim3(kAmsThreads), 0, s, X, ld, scale, n, m, d, mask, out);
  else
    hipLaunchKernelGGL(k_ams_rows<2>, dim3(blocks), dim3(kAmsThreads), 0, s, X, ld, scale, n, m, d, mask, out);
  return hipGetLastError();
}

hipError_t launch_ams_final(const double* u, const double* v, int m, int d, const uint64_t* mask1,
                            const uint64_t* mask2, const double* diag, int ndiag, double* X,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_ams_final, dim3(d), dim3(kAmsThreads), 0, s, u, v, m, mask1, mask2, diag,
                     ndiag, X);
  return hipGetLastError();
}

}  // namespace cmm

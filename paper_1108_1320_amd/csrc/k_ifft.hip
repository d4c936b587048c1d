// Inverse transform of the accumulated spectrum (Figure 1: c_t is the
// inverse DFT of the summed spectrum P_t), the diagonal correction of
// Section 3.2, and small linear helpers.  Everything here is float64.
//
// The FFT kernel leaves, per k-split, rows f1 in [0, R/2] of the spectrum
// (frequency f = f1 + R f2).  The reduction sums the k-splits in a fixed
// order.  The inverse DFT runs as global-memory Stockham passes (radix 16
// with one smaller first pass): the first reads the full length-b spectrum
// through Hermitian symmetry, for f1 > R/2
// P[f1 + R f2] = conj P[(R - f1) + R (C - 1 - f2)], and the last writes
// c_t[u] = Re(.)/b.
#include "cmm_internal.h"
#include "cmm_dft.h"

#include <algorithm>

namespace cmm {

// Psum[t][f1][f2] = sum over ks of Ppart[t][ks][f1][f2], each element's sum
// in increasing ks.  A thread sums two neighbouring elements (16-byte loads;
// C is even) with eight k-splits' loads issued ahead of their adds.
__global__ void k_reduce_splits(const float2* __restrict__ Ppart, int KS, int rows, int C,
                                int d, double2* __restrict__ Psum) {
  const int64_t per_t = (int64_t)rows * C;
  const int64_t pairs = per_t / 2;
  const int64_t total = (int64_t)d * pairs;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(idx / pairs);
    const int64_t rest = 2 * (idx - (int64_t)t * pairs);
    const float4* src = reinterpret_cast<const float4*>(Ppart + (int64_t)t * KS * per_t + rest);
    const int64_t stride = per_t / 2;   // one k-split, in float4
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int ks = 0;
    for (; ks + 8 <= KS; ks += 8) {
      float4 v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = src[(int64_t)(ks + q) * stride];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        s0 += (double)v[q].x; s1 += (double)v[q].y; s2 += (double)v[q].z; s3 += (double)v[q].w;
      }
    }
    for (; ks < KS; ++ks) {
      const float4 v = src[(int64_t)ks * stride];
      s0 += (double)v.x; s1 += (double)v.y; s2 += (double)v.z; s3 += (double)v.w;
    }
    double2* dst = Psum + (int64_t)t * per_t + rest;
    dst[0] = make_double2(s0, s1);
    dst[1] = make_double2(s2, s3);
  }
}

// Spectrum value P_t[f] from the k-split sums: rows f1 <= R/2 are stored,
// the others are the conjugates of their Hermitian mirrors.
__device__ __forceinline__ double2 assembled(const double2* __restrict__ Psum, int t, int64_t f,
                                             int R, int rows, int C) {
  int f1 = (int)(f & (R - 1));
  int64_t f2 = f / R;
  bool cj = false;
  if (R > 1 && 2 * f1 > R) { f1 = R - f1; f2 = C - 1 - f2; cj = true; }
  double2 v = Psum[((int64_t)t * rows + f1) * C + f2];
  if (cj) v.y = -v.y;
  return v;
}

struct IfftEnds {
  const double2* Psum;   // FIRST: read the spectrum from the k-split sums
  int R, rows, C;
  double* c;             // LAST: write Re(.) / b as the sketch
  double inv_b;
};

// One inverse Stockham pass of radix RS over every repetition:
// out[(jb/Ns) Ns RS + jb mod Ns + r Ns] = IDFT_RS( in[jb + r b/RS] conj(w) ).
// The first pass reads the assembled spectrum, the last writes the real
// sketch c_t[u] = Re(x_t[u]) / b.
template <int RS, bool FIRST, bool LAST>
__global__ void k_ifft_pass(const double2* __restrict__ in, double2* __restrict__ out,
                            const double2* __restrict__ tw, int64_t b, int d, int64_t Ns,
                            IfftEnds ends) {
  const int64_t nb = b / RS;
  const int64_t total = (int64_t)d * nb;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(idx / nb);
    const int64_t jb = idx - (int64_t)t * nb;
    const double2* src = in + (int64_t)t * b;
    const int64_t jm = jb % Ns;
    const int64_t step = b / (Ns * RS);
    double2 x[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      // inverse = conj(DFT(conj(x) * w)), with twiddle w^(jm r)
      double2 v = FIRST ? assembled(ends.Psum, t, jb + (int64_t)r * nb, ends.R, ends.rows, ends.C)
                        : src[jb + (int64_t)r * nb];
      v = cconj(v);
      if (r > 0 && jm > 0) v = cmul(v, tw[(jm * r * step) & (b - 1)]);
      x[r] = v;
    }
    dft<RS>(x);
    const int64_t base = (jb / Ns) * Ns * RS + jm;
    if constexpr (LAST) {
      double* c = ends.c + (int64_t)t * b;
#pragma unroll
      for (int r = 0; r < RS; ++r) c[base + (int64_t)r * Ns] = x[r].x * ends.inv_b;
    } else {
      double2* dst = out + (int64_t)t * b;
#pragma unroll
      for (int r = 0; r < RS; ++r) dst[base + (int64_t)r * Ns] = cconj(x[r]);
    }
  }
}

static inline unsigned grid_for(int64_t n, int64_t cap = 16384) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

hipError_t launch_ifft(const Geometry& g, const float2* Ppart, double2* work0, double2* work1,
                       const double2* tw64, double* c64, hipStream_t s) {
  const int C = 1 << g.log2c;
  const int64_t nsum = (int64_t)g.d * g.rows * C / 2;   // element pairs
  // Psum lives in work1 (size d*b >= d*rows*C)
  hipLaunchKernelGGL(k_reduce_splits, dim3(grid_for(nsum)), dim3(256), 0, s, Ppart, g.KS,
                     g.rows, C, g.d, work1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the first pass reads Psum; the passes then alternate work0 / work1
  IfftEnds ends{work1, g.R, g.rows, C, c64, 1.0 / (double)g.b};
  double2* src = work1;   // unused by the first pass
  double2* dst = work0;
  int64_t Ns = 1;
  const int rem = g.log2b % 4;
  const int passes = g.log2b / 4 + (rem ? 1 : 0);
  for (int p = 0; p < passes; ++p) {
    const int rs = (p == 0 && rem) ? (1 << rem) : 16;
    const int64_t nthreads = (int64_t)g.d * (g.b / rs);
    // one wave per block: d * b / 16 butterflies are only a few hundred
    // waves, which then spread over every CU instead of a quarter of them
    const dim3 grid((unsigned)std::min<int64_t>((nthreads + 63) / 64, 65536));
    const bool first = p == 0, last = p == passes - 1;
#define CMM_IF(RS_, F_, L_) hipLaunchKernelGGL((k_ifft_pass<RS_, F_, L_>), grid, dim3(64), 0, s, src, dst, tw64, g.b, g.d, Ns, ends)
#define CMM_IF_RS(RS_) \
    if (first && last) CMM_IF(RS_, true, true); \
    else if (first) CMM_IF(RS_, true, false); \
    else if (last) CMM_IF(RS_, false, true); \
    else CMM_IF(RS_, false, false);
    switch (rs) {
      case 2: CMM_IF_RS(2) break;
      case 4: CMM_IF_RS(4) break;
      case 8: CMM_IF_RS(8) break;
      default: CMM_IF_RS(16) break;
    }
#undef CMM_IF_RS
#undef CMM_IF
    if ((e = hipGetLastError()) != hipSuccess) return e;
    Ns *= rs;
    // the first pass read Psum (work1) and wrote work0; then ping-pong
    if (first) { src = work0; dst = work1; }
    else { double2* tmpb = src; src = dst; dst = tmpb; }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- diagonal


// partial[kc][i] = sum over k in chunk kc of A[i,k] B[k,i] (float64)
template <int DT>
__global__ void k_diag_partial(const void* A, int64_t lda, const float* sA, const void* B,
                               int64_t ldb, const float* sB, int m, int n, int kchunks,
                               double* __restrict__ partial) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int kc = blockIdx.y;
  if (i >= n) return;
  const int k0 = (int)((int64_t)m * kc / kchunks), k1 = (int)((int64_t)m * (kc + 1) / kchunks);
  // the operand values are float32(decoded element * scale), as in the sketch
  const float fa = sA ? sA[i] : 1.0f, fb = sB ? sB[i] : 1.0f;
  double acc = 0.0;
  for (int k = k0; k < k1; ++k)
    acc += (double)(load_deq<DT>(A, (int64_t)k * lda + i) * fa) *
           (double)(load_deq<DT>(B, (int64_t)k * ldb + i) * fb);
  partial[(int64_t)kc * n + i] = acc;
}

// Sum of the k-chunk partials of entry i: eight independent running sums
// (chunk kc goes to sum kc mod 8) keep eight loads in flight, and are added
// in a fixed order, so the result does not depend on timing.
__global__ __launch_bounds__(64) void k_diag_reduce(const double* __restrict__ partial, int n,
                                                    int kchunks, double* __restrict__ diag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int kc = 0;
  for (; kc + 8 <= kchunks; kc += 8) {
#pragma unroll
    for (int q = 0; q < 8; ++q) s[q] += partial[(int64_t)(kc + q) * n + i];
  }
  for (int q = 0; kc + q < kchunks; ++q) s[q] += partial[(int64_t)(kc + q) * n + i];
  diag[i] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// partial[kc][j] = sum over k in chunk kc of A[j,k] B[k,j] for sparse A (by
// columns k) and B (by rows k): block kc takes its k one after the other,
// stages column k of A in LDS (zeroed, then scattered) and adds the float64
// products with the entries of row k of B into its own partial row.  Within
// one k the entries of row k of B have distinct columns, so no two threads
// touch one j; successive k are separated by block barriers.  The partial
// rows are then summed in a fixed order (k_diag_reduce), so the diagonal
// does not depend on scheduling.
__global__ void k_diag_sparse(const int64_t* __restrict__ aptr, const int32_t* __restrict__ aidx,
                              const float* __restrict__ aval, const int64_t* __restrict__ bptr,
                              const int32_t* __restrict__ bidx, const float* __restrict__ bval,
                              int m, int n, int kchunks, double* __restrict__ partial) {
  extern __shared__ float col[];
  const int kc = blockIdx.x;
  double* pr = partial + (int64_t)kc * n;
  for (int x = threadIdx.x; x < n; x += blockDim.x) pr[x] = 0.0;
  const int k0 = (int)((int64_t)m * kc / kchunks), k1 = (int)((int64_t)m * (kc + 1) / kchunks);
  for (int k = k0; k < k1; ++k) {
    for (int x = threadIdx.x; x < n; x += blockDim.x) col[x] = 0.0f;
    __syncthreads();
    for (int64_t e = aptr[k] + threadIdx.x; e < aptr[k + 1]; e += blockDim.x) col[aidx[e]] = aval[e];
    __syncthreads();
    for (int64_t e = bptr[k] + threadIdx.x; e < bptr[k + 1]; e += blockDim.x) {
      const int j = bidx[e];
      if (j < n && col[j] != 0.0f) pr[j] += (double)col[j] * (double)bval[e];
    }
    __syncthreads();
  }
}

// Sparse operand check: offsets non-decreasing from 0, every index in [0, n).
__global__ void k_sparse_check(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                               int m, int n, int32_t* __restrict__ bad) {
  const int64_t nnz = ptr[m];
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < (int64_t)m + nnz;
       q += (int64_t)gridDim.x * blockDim.x) {
    if (q < m) {
      if (ptr[q] > ptr[q + 1] || (q == 0 && ptr[0] != 0)) *bad = 1;
    } else {
      const int32_t v = idx[q - m];
      if (v < 0 || v >= n) *bad = 1;
    }
  }
}

hipError_t launch_sparse_check(const int64_t* ptr, const int32_t* idx, int m, int n, int64_t nnz,
                               int32_t* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_sparse_check, dim3(grid_for((int64_t)m + nnz)), dim3(256), 0, s, ptr, idx, m,
                     n, bad);
  return hipGetLastError();
}

hipError_t prepare_sparse() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_diag_sparse),
                             hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
}

hipError_t launch_diag(int dtype, const SideDesc& a, const SideDesc& bs, int m, int n,
                       double* partial, int kchunks, double* diag, hipStream_t s) {
  if (dtype == kSparseF32) {
    hipLaunchKernelGGL(k_diag_sparse, dim3(kchunks), dim3(256), (size_t)n * sizeof(float), s,
                       a.sptr, a.sidx, (const float*)a.X, bs.sptr, bs.sidx, (const float*)bs.X, m, n,
                       kchunks, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag_reduce, dim3((n + 63) / 64), dim3(64), 0, s, partial, n, kchunks, diag);
    return hipGetLastError();
  }
  dim3 grid((n + 255) / 256, kchunks);
  if (dtype == 0)
    hipLaunchKernelGGL(k_diag_partial<0>, grid, dim3(256), 0, s, a.X, a.ld, a.scale, bs.X, bs.ld, bs.scale, m, n, kchunks, partial);
  else if (dtype == 1)
    hipLaunchKernelGGL(k_diag_partial<1>, grid, dim3(256), 0, s, a.X, a.ld, a.scale, bs.X, bs.ld, bs.scale, m, n, kchunks, partial);
  else
    hipLaunchKernelGGL(k_diag_partial<2>, grid, dim3(256), 0, s, a.X, a.ld, a.scale, bs.X, bs.ld, bs.scale, m, n, kchunks, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_diag_reduce, dim3((n + 63) / 64), dim3(64), 0, s, partial, n, kchunks, diag);
  return hipGetLastError();
}

// c_t[(h1(i) + h2(i)) mod b] -= s1(i) s2(i) diag[i] for i < len, the same
// for every run: several i can share a bucket, so their contributions are
// summed exactly in 64-bit fixed point (integer sums do not depend on the
// order of the adds) and one thread per touched bucket, that of its
// smallest i, applies the sum.  The shift s keeps len * max|diag| * 2^s
// below 2^62; each contribution is rounded to a multiple of 2^-s, an error
// below len * max|diag| * 2^-63.  tmp holds acc[d * b] (int64), owner[d * b]
// (int32) and the shift (int32): at least 16 d b bytes.
__global__ __launch_bounds__(1024) void k_diag_shift(const double* __restrict__ diag, int len,
                                                     int* __restrict__ shift) {
  __shared__ double wmax[16];
  double mx = 0.0;
  for (int i = threadIdx.x; i < len; i += blockDim.x) mx = fmax(mx, fabs(diag[i]));
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) mx = fmax(mx, wmax[w]);
    int e = 0;
    (void)frexp(mx, &e);                 // mx < 2^e
    int l = 0;
    while ((1 << l) < len) ++l;          // len <= 2^l
    *shift = mx > 0.0 ? 62 - e - l : 0;
  }
}

__device__ __forceinline__ int64_t diag_bucket(const int32_t* hs1, const int32_t* hs2, int n1, int n3,
                                               int t, int i, int64_t b, bool* neg) {
  const int32_t a = hs1[(int64_t)t * n1 + i], c = hs2[(int64_t)t * n3 + i];
  *neg = ((a ^ c) & 1) != 0;      // s1(i) s2(i) = -1
  return (int64_t)t * b + ((int64_t)((a >> 1) + (c >> 1)) & (b - 1));
}

__global__ void k_sub_diag_init(const int32_t* __restrict__ hs1, const int32_t* __restrict__ hs2,
                                int n1, int n3, int len, int d, int64_t b,
                                long long* __restrict__ acc, int* __restrict__ owner) {
  const int64_t total = (int64_t)d * len;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(idx / len), i = (int)(idx - (int64_t)t * len);
    bool neg;
    const int64_t u = diag_bucket(hs1, hs2, n1, n3, t, i, b, &neg);
    acc[u] = 0;
    owner[u] = 0x7FFFFFFF;
  }
}

__global__ void k_sub_diag_add(const int32_t* __restrict__ hs1, const int32_t* __restrict__ hs2,
                               int n1, int n3, const double* __restrict__ diag, int len, int d,
                               int64_t b, const int* __restrict__ shift, long long* __restrict__ acc,
                               int* __restrict__ owner) {
  const int64_t total = (int64_t)d * len;
  const int sh = *shift;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(idx / len), i = (int)(idx - (int64_t)t * len);
    bool neg;
    const int64_t u = diag_bucket(hs1, hs2, n1, n3, t, i, b, &neg);
    const double v = neg ? diag[i] : -diag[i];    // the amount added to c_t[u]
    const long long q = __double2ll_rn(ldexp(v, sh));
    atomicAdd(reinterpret_cast<unsigned long long*>(&acc[u]), (unsigned long long)q);
    atomicMin(&owner[u], i);
  }
}

__global__ void k_sub_diag_apply(const int32_t* __restrict__ hs1, const int32_t* __restrict__ hs2,
                                 int n1, int n3, int len, int d, int64_t b,
                                 const int* __restrict__ shift, const long long* __restrict__ acc,
                                 const int* __restrict__ owner, double* __restrict__ c64) {
  const int64_t total = (int64_t)d * len;
  const int sh = *shift;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(idx / len), i = (int)(idx - (int64_t)t * len);
    bool neg;
    const int64_t u = diag_bucket(hs1, hs2, n1, n3, t, i, b, &neg);
    if (owner[u] == i) c64[u] += ldexp((double)acc[u], -sh);
  }
}

hipError_t launch_sub_diag(const Geometry& g, const int32_t* hs1, const int32_t* hs2, int n1,
                           int n3, const double* diag, int len, double* c64, void* tmp,
                           hipStream_t s) {
  const int64_t db = (int64_t)g.d * g.b;
  long long* acc = static_cast<long long*>(tmp);
  int* owner = reinterpret_cast<int*>(acc + db);
  int* shift = owner + db;
  const unsigned grid = grid_for((int64_t)g.d * len);
  hipLaunchKernelGGL(k_diag_shift, dim3(1), dim3(1024), 0, s, diag, len, shift);
  hipLaunchKernelGGL(k_sub_diag_init, dim3(grid), dim3(256), 0, s, hs1, hs2, n1, n3, len, g.d, g.b, acc, owner);
  hipLaunchKernelGGL(k_sub_diag_add, dim3(grid), dim3(256), 0, s, hs1, hs2, n1, n3, diag, len, g.d,
                     g.b, shift, acc, owner);
  hipLaunchKernelGGL(k_sub_diag_apply, dim3(grid), dim3(256), 0, s, hs1, hs2, n1, n3, len, g.d, g.b,
                     shift, acc, owner, c64);
  return hipGetLastError();
}

__global__ void k_to_f32(const double* __restrict__ c64, float* __restrict__ c32, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    c32[i] = (float)c64[i];
}

hipError_t launch_to_f32(const double* c64, float* c32, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f32, dim3(grid_for(count)), dim3(256), 0, s, c64, c32, count);
  return hipGetLastError();
}

__global__ void k_add_f64(double* __restrict__ dst, const double* __restrict__ src, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] += src[i];
}

hipError_t launch_add_f64(double* dst, const double* src, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_add_f64, dim3(grid_for(count)), dim3(256), 0, s, dst, src, count);
  return hipGetLastError();
}

}  // namespace cmm

namespace cmm {

// Deterministic pseudo-random operand values for the autotuner's trial
// products (SplitMix64 of the element index): uniform in [-1, 1) for f32,
// its bf16 rounding, or fp8 codes of magnitude < 448.
__global__ void k_fill_random(void* X, int64_t count, int dtype, uint64_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const float u = (float)(z >> 40) * 0x1p-23f - 1.0f;
    if (dtype == 0) ((float*)X)[i] = u;
    else if (dtype == 1) ((uint16_t*)X)[i] = (uint16_t)(__float_as_uint(u) >> 16);
    else ((uint8_t*)X)[i] = (uint8_t)((z & 0x7E) | ((z >> 8) & 0x80));
  }
}

hipError_t launch_fill_random(void* X, int64_t count, int dtype, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_random, dim3(grid_for(count)), dim3(256), 0, s, X, count, dtype, seed);
  return hipGetLastError();
}

}  // namespace cmm

// COUNT SKETCH of every column a_k of A and row b_k of B (the polynomials
// p_{a_k}^{h1,s1} and p_{b_k}^{h2,s2} of Section 2.2 / Figure 1), for all d
// repetitions from one read of each input row.
//
// The stored operands are k-major (Section 2.2's single-pass order), so the
// vector to sketch for a given k is one contiguous row of n elements.  A
// block stages that row in LDS (dequantising bf16 / fp8 and applying the
// per-position scale; rows longer than the 24576 floats LDS staging holds
// are read element by element from global memory, where they stay in L2),
// then, for every repetition, writes the row's sketch
// in the bucket layout of the FFT kernel: position p holds the signed sum of
// the row entries of the bucket placed there.  Members of a bucket are summed
// in increasing index order, so the result does not depend on scheduling.
// The kernel streams its input once and writes d compact sketches; it is
// bound by HBM bandwidth.
#include "cmm_internal.h"

#include <algorithm>

namespace cmm {


template <int DT> struct Elem;
template <> struct Elem<0> {      // f32
  typedef float S; typedef float4 V4;
  static __device__ __forceinline__ float one(S s) { return s; }
  static __device__ __forceinline__ void four(V4 v, float* o) { o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w; }
};
template <> struct Elem<1> {      // bf16 bits
  typedef uint16_t S; typedef uint2 V4;
  static __device__ __forceinline__ float one(S s) { return __uint_as_float((uint32_t)s << 16); }
  static __device__ __forceinline__ void four(V4 v, float* o) {
    o[0] = __uint_as_float(v.x << 16); o[1] = __uint_as_float(v.x & 0xFFFF0000u);
    o[2] = __uint_as_float(v.y << 16); o[3] = __uint_as_float(v.y & 0xFFFF0000u);
  }
};
template <> struct Elem<2> {      // fp8 e4m3fn bits
  typedef uint8_t S; typedef uint32_t V4;
  static __device__ __forceinline__ float one(S s) { return e4m3fn_to_f32(s); }
  static __device__ __forceinline__ void four(V4 v, float* o) {
    o[0] = e4m3fn_to_f32(v & 0xFF); o[1] = e4m3fn_to_f32((v >> 8) & 0xFF);
    o[2] = e4m3fn_to_f32((v >> 16) & 0xFF); o[3] = e4m3fn_to_f32(v >> 24);
  }
};

// grid.x = k-blocks; block = 512 threads; dynamic LDS = n floats.
// Positions are handled four at a time (16-byte table reads and stores; the
// layout's segments are multiples of 64 positions, so a group of four never
// straddles two segments).  The per-column max |value| is kept per thread and
// merged through an LDS integer max (float bits of non-negative values order
// like the integers), one barrier per row.
constexpr int kCsThreads = 512;

template <int DT, bool STAGED>
__global__ __launch_bounds__(kCsThreads) void k_countsketch(SideDesc sd, int d, int m, int W, int kblock) {
  static_assert(STAGED || DT != kSparseF32, "sparse rows are always staged");
  extern __shared__ float row[];
  __shared__ uint32_t smax[2][64];
  typedef Elem<DT == kSparseF32 ? 0 : DT> E;
  typedef typename E::S S;
  const int tid = threadIdx.x;
  const int n = sd.n;
  const int k0 = blockIdx.x * kblock;
  const int k1 = min(m, k0 + kblock);
  const S* X = (const S*)sd.X;
  const bool scale16 = sd.scale == nullptr || (uintptr_t)sd.scale % 16 == 0;
  if (tid < 128) smax[tid >> 6][tid & 63] = 0u;
  int par = 0;
  for (int k = k0; k < k1; ++k, par ^= 1) {
    const S* xr = DT == kSparseF32 ? X : X + (int64_t)k * sd.ld;
    // value of row element x (dequantised and scaled)
    auto val = [&](int x) -> float {
      if constexpr (STAGED) return row[x];
      else return E::one(xr[x]) * (sd.scale ? sd.scale[x] : 1.0f);
    };
    if constexpr (!STAGED) {
      // nothing to stage
    } else if constexpr (DT == kSparseF32) {
      // sparse row: zero the staged row, then scatter the row's entries
      for (int x = tid; x < n; x += kCsThreads) row[x] = 0.0f;
      __syncthreads();
      const int64_t e1 = sd.sptr[k + 1];
      for (int64_t e = sd.sptr[k] + tid; e < e1; e += kCsThreads) row[sd.sidx[e]] = X[e];
      __syncthreads();
    } else {
    // the row's first `head` elements are staged one by one, the body four at
    // a time from an address aligned to four elements, then the tail
    const int head = min(n, (int)((4 - ((uintptr_t)xr / sizeof(S)) % 4) % 4));
    const int n4 = (n - head) >> 2;
    const typename E::V4* xv = (const typename E::V4*)(xr + head);
    if (head == 0 && scale16) {
      for (int q = tid; q < n4; q += kCsThreads) {
        float o[4];
        E::four(xv[q], o);
        if (sd.scale) {
          const float4 sc = ((const float4*)sd.scale)[q];
          o[0] *= sc.x; o[1] *= sc.y; o[2] *= sc.z; o[3] *= sc.w;
        }
        *(float4*)&row[4 * q] = make_float4(o[0], o[1], o[2], o[3]);
      }
    } else {
      for (int q = tid; q < n4; q += kCsThreads) {
        float o[4];
        E::four(xv[q], o);
        const int x = head + 4 * q;
#pragma unroll
        for (int i = 0; i < 4; ++i) row[x + i] = o[i] * (sd.scale ? sd.scale[x + i] : 1.0f);
      }
    }
    if (tid < head) row[tid] = E::one(xr[tid]) * (sd.scale ? sd.scale[tid] : 1.0f);
    for (int x = head + 4 * n4 + tid; x < n; x += kCsThreads)
      row[x] = E::one(xr[x]) * (sd.scale ? sd.scale[x] : 1.0f);
    __syncthreads();
    }
    for (int t = 0; t < d; ++t) {
      const int L = sd.lseg[t];
      const int L4 = L >> 2;
      const int total4 = W * L4;
      const uint32_t* tab = sd.tab + (int64_t)t * sd.Lrow;
      float* out = sd.SA + ((int64_t)t * m + k) * sd.Lrow;
      float amax = 0.0f;
      // groups of four positions, UQ per thread at a time: their table reads
      // are issued together, so several are in flight before the gathers
      // and stores that depend on them
      constexpr int UQ = 3;
      for (int base = tid; base < total4; base += UQ * kCsThreads) {
        uint4 e4s[UQ];
        int ps[UQ];
#pragma unroll
        for (int u = 0; u < UQ; ++u) {
          const int idx = base + u * kCsThreads;
          const int w = idx / L4;
          ps[u] = w * sd.Lcap + 4 * (idx - w * L4);
          if (idx < total4) e4s[u] = *(const uint4*)&tab[ps[u]];
        }
#pragma unroll
        for (int u = 0; u < UQ; ++u) {
          if (base + u * kCsThreads >= total4) break;
          const int p = ps[u];
          const uint32_t ev[4] = {e4s[u].x, e4s[u].y, e4s[u].z, e4s[u].w};
          float v[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const uint32_t e = ev[q];
            float x = 0.0f;
            if (e != CMM_PAD_TAB) {
              x = val((int)(e & CMM_TAB_IDX));
              if (e & CMM_TAB_NEG) x = -x;
              if (e & CMM_TAB_MORE) {
                const int64_t tp = (int64_t)t * sd.Lrow + p + q;
                const int c = sd.cntp[tp];
                const int32_t* mem = sd.perm + (int64_t)t * n + sd.moff[tp];
                const int32_t* hs = sd.hs + (int64_t)t * n;
                for (int a = 1; a < c; ++a) {
                  const int xm = mem[a];
                  const float y = val(xm);
                  x += (hs[xm] & 1) ? -y : y;
                }
              }
            }
            v[q] = x;
            amax = fmaxf(amax, fabsf(x));
          }
          // streaming store: the sketches are several times larger than the
          // caches and are read back only by the spectral kernel
          typedef float v4f __attribute__((ext_vector_type(4)));
          __builtin_nontemporal_store(v4f{v[0], v[1], v[2], v[3]}, reinterpret_cast<v4f*>(&out[p]));
        }
      }
      for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off, 64));
      if ((tid & 63) == 0) atomicMax(&smax[par][t], __float_as_uint(amax));   // d <= 63
    }
    __syncthreads();
    if (tid < d) {
      sd.colmax[(int64_t)tid * m + k] = __uint_as_float(smax[par][tid]);
      smax[par][tid] = 0u;   // free for row k+2 (the next row uses the other half)
    }
  }
}

hipError_t launch_countsketch(int dtype, const Geometry& g, SideDesc& sd, hipStream_t s) {
  int kblock = (int)((int64_t)g.m / std::max(1, g.cs_blocks));
  if (kblock < 1) kblock = 1;
  const int blocks = (g.m + kblock - 1) / kblock;
  const bool staged = sd.n <= kMaxStagedDim;
  if (!staged && dtype == kSparseF32) return hipErrorInvalidValue;
  const size_t lds = staged ? (size_t)sd.n * sizeof(float) : 0;
#define CMM_CS(DT, ST) \
  hipLaunchKernelGGL((k_countsketch<DT, ST>), dim3(blocks), dim3(kCsThreads), lds, s, sd, g.d, g.m, g.W, kblock)
  if (dtype == 0) { if (staged) CMM_CS(0, true); else CMM_CS(0, false); }
  else if (dtype == 1) { if (staged) CMM_CS(1, true); else CMM_CS(1, false); }
  else if (dtype == 2) { if (staged) CMM_CS(2, true); else CMM_CS(2, false); }
  else CMM_CS(kSparseF32, true);
#undef CMM_CS
  return hipGetLastError();
}

// Raise the dynamic LDS limit of every instantiation to the 96 KB a staged
// row of up to 24576 floats needs (done once per context, outside any graph
// capture).
hipError_t prepare_countsketch() {
  const void* fns[] = {reinterpret_cast<const void*>(&k_countsketch<0, true>),
                       reinterpret_cast<const void*>(&k_countsketch<1, true>),
                       reinterpret_cast<const void*>(&k_countsketch<2, true>),
                       reinterpret_cast<const void*>(&k_countsketch<kSparseF32, true>)};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace cmm

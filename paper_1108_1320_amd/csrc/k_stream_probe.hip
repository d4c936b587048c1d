// Plain HBM streams for measuring what this GPU sustains for the access
// patterns of the count-sketch kernel: reads only, writes only, and reads
// with r times as many bytes written (r = 1 is a copy).  Writes go either
// through ordinary or streaming (non-temporal) 16-byte stores, the latter
// being what the count sketch uses for its output.  Each launch touches
// every byte once; the caller times a series of launches.
#include "cmm_internal.h"

namespace cmm {

typedef float v4f __attribute__((ext_vector_type(4)));

// Read n4 float4 values, four loads in flight per thread; one float per
// block keeps the loads live.
__global__ __launch_bounds__(256) void k_stream_read(const v4f* __restrict__ src, int64_t n4,
                                                     float* __restrict__ sink) {
  float acc = 0.0f;
  const int64_t step = (int64_t)gridDim.x * blockDim.x * 4;
  for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x * 4 + threadIdx.x; i0 < n4; i0 += step) {
    v4f v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = i0 + (int64_t)u * blockDim.x;
      v[u] = i < n4 ? src[i] : v4f{0.0f, 0.0f, 0.0f, 0.0f};
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0 && acc == 12345.678f) sink[blockIdx.x] = acc;   // practically never
}

// Write n4 float4 values (no reads); each thread issues four stores per
// iteration, a block-width apart, so several stores are in flight.
template <bool NT>
__global__ __launch_bounds__(256) void k_stream_write(v4f* __restrict__ dst, int64_t n4, float val) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x * 4;
  for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x * 4 + threadIdx.x; i0 < n4; i0 += step) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = i0 + (int64_t)u * blockDim.x;
      if (i < n4) {
        const v4f v = {val, val + 1.0f, val + 2.0f, (float)i};
        if constexpr (NT) __builtin_nontemporal_store(v, dst + i);
        else dst[i] = v;
      }
    }
  }
}

// Read float4 q of src and write it, scaled, to float4 q of each of r
// planes of dst (plane p starts at p * n4): each store instruction covers a
// contiguous span, as the count sketch's per-repetition output planes do.
template <bool NT>
__global__ __launch_bounds__(256) void k_stream_mixed(const v4f* __restrict__ src, int64_t n4, int r,
                                                      v4f* __restrict__ dst) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x * 2;
  for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x * 2 + threadIdx.x; i0 < n4; i0 += step) {
    const int64_t i1 = i0 + blockDim.x;
    const v4f v0 = src[i0];
    const v4f v1 = i1 < n4 ? src[i1] : v4f{0.0f, 0.0f, 0.0f, 0.0f};
    for (int p = 0; p < r; ++p) {
      const v4f w0 = v0 * (float)(p + 1), w1 = v1 * (float)(p + 1);
      if constexpr (NT) {
        __builtin_nontemporal_store(w0, dst + (int64_t)p * n4 + i0);
        if (i1 < n4) __builtin_nontemporal_store(w1, dst + (int64_t)p * n4 + i1);
      } else {
        dst[(int64_t)p * n4 + i0] = w0;
        if (i1 < n4) dst[(int64_t)p * n4 + i1] = w1;
      }
    }
  }
}

hipError_t launch_stream_probe(const void* src, void* dst, float* sink, int64_t read_bytes,
                               int64_t write_bytes, bool nt, hipStream_t s) {
  const int blocks = 256 * 8;    // 8 blocks of 4 waves per CU
  if (write_bytes == 0) {
    hipLaunchKernelGGL(k_stream_read, dim3(blocks), dim3(256), 0, s, (const v4f*)src, read_bytes / 16, sink);
  } else if (read_bytes == 0) {
    if (nt) hipLaunchKernelGGL(k_stream_write<true>, dim3(blocks), dim3(256), 0, s, (v4f*)dst, write_bytes / 16, 1.0f);
    else hipLaunchKernelGGL(k_stream_write<false>, dim3(blocks), dim3(256), 0, s, (v4f*)dst, write_bytes / 16, 1.0f);
  } else {
    const int r = (int)(write_bytes / read_bytes);
    if (nt) hipLaunchKernelGGL(k_stream_mixed<true>, dim3(blocks), dim3(256), 0, s, (const v4f*)src, read_bytes / 16, r, (v4f*)dst);
    else hipLaunchKernelGGL(k_stream_mixed<false>, dim3(blocks), dim3(256), 0, s, (const v4f*)src, read_bytes / 16, r, (v4f*)dst);
  }
  return hipGetLastError();
}

}  // namespace cmm

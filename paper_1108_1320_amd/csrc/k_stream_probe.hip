// Plain HBM streams for measuring what this GPU sustains for the access
// patterns of the count-sketch kernel: reads only, writes only, and reads
// with r times as many bytes written (r = 1 is a copy).  Writes go either
// through ordinary or streaming (non-temporal) 16-byte stores, the latter
// being what the count sketch uses for its output.  Each launch touches
// every byte once; the caller times a series of launches.
#include "cmm_internal.h"

namespace cmm {

typedef float v4f __attribute__((ext_vector_type(4)));

// Read n4 float4 values; one float per block keeps the loads live.
__global__ __launch_bounds__(256) void k_stream_read(const v4f* __restrict__ src, int64_t n4,
                                                     float* __restrict__ sink) {
  float acc = 0.0f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4;
       i += (int64_t)gridDim.x * blockDim.x) {
    const v4f v = src[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0 && acc == 12345.678f) sink[blockIdx.x] = acc;   // practically never
}

// Write n4 float4 values (no reads).
template <bool NT>
__global__ __launch_bounds__(256) void k_stream_write(v4f* __restrict__ dst, int64_t n4, float val) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4;
       i += (int64_t)gridDim.x * blockDim.x) {
    const v4f v = {val, val + 1.0f, val + 2.0f, (float)i};
    if constexpr (NT) __builtin_nontemporal_store(v, dst + i);
    else dst[i] = v;
  }
}

// Read float4 q of src and write it, scaled, to float4 q of each of r
// planes of dst (plane p starts at p * n4): each store instruction covers a
// contiguous span, as the count sketch's per-repetition output planes do.
template <bool NT>
__global__ __launch_bounds__(256) void k_stream_mixed(const v4f* __restrict__ src, int64_t n4, int r,
                                                      v4f* __restrict__ dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4;
       i += (int64_t)gridDim.x * blockDim.x) {
    const v4f v = src[i];
    for (int p = 0; p < r; ++p) {
      const v4f w = v * (float)(p + 1);
      if constexpr (NT) __builtin_nontemporal_store(w, dst + (int64_t)p * n4 + i);
      else dst[(int64_t)p * n4 + i] = w;
    }
  }
}

hipError_t launch_stream_probe(const void* src, void* dst, float* sink, int64_t read_bytes,
                               int64_t write_bytes, bool nt, hipStream_t s) {
  const int blocks = 256 * 16;   // 16 blocks of 4 waves per CU
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

// Hashing (Section 2.2, polynomial hash functions) and the bucket layout the
// count-sketch and FFT kernels share.
//
// g(x) = (a x + c) mod (2^61 - 1) is evaluated exactly: the 93-bit product
// a*x comes from a 64x64 multiply (low word and __umul64hi) and is reduced
// with the Mersenne identity 2^61 = 1 (mod 2^61 - 1).  h = g mod b is the
// low bits of g (b a power of two); the sign is -1 when g is odd.
#include "cmm_internal.h"

namespace cmm {


__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

// omega_b^x = exp(-2 pi i x / b) in float64 (argument 2x/b is exact), and its
// float32 rounding.
__global__ void k_twiddles(double2* tw64, float2* tw32, int64_t b) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < b;
       x += (int64_t)gridDim.x * blockDim.x) {
    double a = 2.0 * (double)x / (double)b;
    double cs = cospi(a), sn = sinpi(a);
    tw64[x] = make_double2(cs, -sn);
    tw32[x] = make_float2((float)cs, (float)-sn);
  }
}

hipError_t launch_twiddles(double2* tw64, float2* tw32, int64_t b, hipStream_t s) {
  int64_t blocks = (b + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_twiddles, dim3((unsigned)blocks), dim3(256), 0, s, tw64, tw32, b);
  return hipGetLastError();
}

// Hash parameters of every repetition t and function f (h1, s1, h2, s2)
// from the SplitMix64 stream of `seed`, by the rule the host uses: thread
// q = 4t + f reads outputs z_{2q+1}, z_{2q+2} and writes
// a = 1 + z mod (2^61 - 2), c = z' mod (2^61 - 1) to out[2q], out[2q+1].
__global__ void k_params_from_seed(uint64_t seed, int d, uint64_t* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 4 * d) return;
  const uint64_t za = splitmix64_dev(seed, 2 * (uint64_t)q + 1);
  const uint64_t zc = splitmix64_dev(seed, 2 * (uint64_t)q + 2);
  out[2 * q] = 1 + za % (CMM_P61 - 1);
  out[2 * q + 1] = zc % CMM_P61;
}

hipError_t launch_params_from_seed(uint64_t seed, int d, uint64_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_params_from_seed, dim3((4 * d + 255) / 256), dim3(256), 0, s, seed, d, out);
  return hipGetLastError();
}

// hs[t][x] = (h(x) << 1) | (s(x) == -1) for x < n, every repetition t.
__global__ void k_hash(const uint64_t* __restrict__ params, int side, int d, int n,
                       uint64_t bmask, int32_t* __restrict__ hs) {
  const int64_t total = (int64_t)d * n;
  const int fh = side == 0 ? 0 : 2;   // h1,s1 for side 0; h2,s2 for side 1
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int t = (int)(idx / n);
    uint64_t x = (uint64_t)(idx - (int64_t)t * n);
    const uint64_t* pr = params + (size_t)t * 8;
    uint64_t gh = cw_hash61(pr[2 * fh], x, pr[2 * fh + 1]);
    uint64_t gs = cw_hash61(pr[2 * fh + 2], x, pr[2 * fh + 3]);
    hs[idx] = (int32_t)(((gh & bmask) << 1) | (gs & 1ull));
  }
}

hipError_t launch_hash(const uint64_t* params_dev, int side, const Geometry& g, SideDesc& sd,
                       hipStream_t s) {
  int64_t total = (int64_t)g.d * sd.n;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_hash, dim3((unsigned)blocks), dim3(256), 0, s, params_dev, side, g.d,
                     sd.n, (uint64_t)(g.b - 1), sd.hs);
  return hipGetLastError();
}

__global__ void k_count(const int32_t* __restrict__ hs, int d, int n, int64_t b,
                        int32_t* __restrict__ cnt) {
  const int64_t total = (int64_t)d * n;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int t = (int)(idx / n);
    int u = hs[idx] >> 1;
    atomicAdd(&cnt[(int64_t)t * b + u], 1);
  }
}

hipError_t launch_count(const Geometry& g, SideDesc& sd, hipStream_t s) {
  hipError_t e = launch_fill_i32(sd.cnt, (int64_t)g.d * g.b, 0, s);
  if (e != hipSuccess) return e;
  int64_t total = (int64_t)g.d * sd.n;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_count, dim3((unsigned)blocks), dim3(256), 0, s, sd.hs, g.d, sd.n, g.b,
                     sd.cnt);
  return hipGetLastError();
}

// One block per (segment w, repetition t): rank the non-empty buckets of the
// segment in increasing u and give each its layout position.
__global__ __launch_bounds__(1024) void k_segment_rank(const int32_t* __restrict__ cnt,
                                                       int64_t b, int log2c, int T, int G, int W, int Lcap,
                                                       int Lrow, int32_t* __restrict__ pos,
                                                       uint32_t* __restrict__ ent,
                                                       uint16_t* __restrict__ entp,
                                                       int32_t* __restrict__ cntp,
                                                       int32_t* __restrict__ segcount,
                                                       int32_t* __restrict__ overflow) {
  const int w = blockIdx.x, t = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  __shared__ int wave_tot[16];
  __shared__ int wave_pre[16];
  const int64_t nseg = b / W;
  const int32_t* cnt_t = cnt + (int64_t)t * b;
  int32_t* pos_t = pos + (int64_t)t * b;
  uint32_t* ent_t = ent + (int64_t)t * Lrow + (int64_t)w * Lcap;
  uint16_t* entp_t = entp + (int64_t)t * Lrow + (int64_t)w * Lcap;
  int32_t* cntp_t = cntp + (int64_t)t * Lrow + (int64_t)w * Lcap;
  int base = 0;
  for (int64_t e0 = 0; e0 < nseg; e0 += 1024) {
    int64_t e = e0 + tid;
    bool valid = e < nseg;
    int64_t u = (e / G) * T + (int64_t)w * G + (e % G);
    int c = valid ? cnt_t[u] : 0;
    bool occ = c > 0;
    uint64_t bal = __ballot(occ);
    int lrank = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wave_tot[wv] = __popcll(bal);
    __syncthreads();
    if (tid == 0) {
      int acc = 0;
      for (int i = 0; i < 16; ++i) { wave_pre[i] = acc; acc += wave_tot[i]; }
      wave_tot[0] = acc;   // block total
    }
    __syncthreads();
    int rank = base + wave_pre[wv] + lrank;
    if (valid) {
      if (occ && rank < Lcap) {
        pos_t[u] = w * Lcap + rank;
        ent_t[rank] = fold_entry((uint32_t)u, log2c);
        entp_t[rank] = pair_entry((uint32_t)u, log2c);
        cntp_t[rank] = c;
      } else {
        pos_t[u] = -1;
        if (occ) atomicExch(overflow, 1);
      }
    }
    int tot = wave_tot[0];
    __syncthreads();
    base += tot;
  }
  if (tid == 0) segcount[t * W + w] = base;
}

// The same ranking with one block per (chunk of 1024 segment entries,
// segment w, repetition t): a block first counts the non-empty buckets of
// the earlier chunks of its segment (its base rank), so all chunks rank at
// once.  Used while a segment has at most kRankChunks chunks (the recount
// grows with the square of their number).
constexpr int kRankChunks = 32;

__global__ __launch_bounds__(1024) void k_segment_rank_chunks(const int32_t* __restrict__ cnt,
                                                              int64_t b, int log2c, int T, int G, int W,
                                                              int Lcap, int Lrow, int32_t* __restrict__ pos,
                                                              uint32_t* __restrict__ ent,
                                                              uint16_t* __restrict__ entp,
                                                              int32_t* __restrict__ cntp,
                                                              int32_t* __restrict__ segcount,
                                                              int32_t* __restrict__ overflow) {
  const int chunk = blockIdx.x, w = blockIdx.y, t = blockIdx.z;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  __shared__ int wave_tot[16];
  __shared__ int wave_pre[16];
  const int64_t nseg = b / W;
  const int32_t* cnt_t = cnt + (int64_t)t * b;
  auto bucket = [&](int64_t e) { return (e / G) * T + (int64_t)w * G + (e % G); };
  // base rank: non-empty buckets of the segment before this chunk
  int before = 0;
  for (int64_t e = tid; e < (int64_t)chunk * 1024; e += 1024) before += cnt_t[bucket(e)] > 0;
  for (int off = 32; off > 0; off >>= 1) before += __shfl_xor(before, off, 64);
  if (lane == 0) wave_tot[wv] = before;
  __syncthreads();
  int base = 0;
  for (int i = 0; i < 16; ++i) base += wave_tot[i];
  __syncthreads();
  // rank within the chunk, as k_segment_rank does for one chunk
  const int64_t e = (int64_t)chunk * 1024 + tid;
  const bool valid = e < nseg;
  const int64_t u = bucket(e);
  const int c = valid ? cnt_t[u] : 0;
  const bool occ = c > 0;
  const uint64_t bal = __ballot(occ);
  const int lrank = __popcll(bal & ((1ull << lane) - 1ull));
  if (lane == 0) wave_tot[wv] = __popcll(bal);
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int i = 0; i < 16; ++i) { wave_pre[i] = acc; acc += wave_tot[i]; }
    wave_tot[0] = acc;
  }
  __syncthreads();
  const int rank = base + wave_pre[wv] + lrank;
  int32_t* pos_t = pos + (int64_t)t * b;
  uint32_t* ent_t = ent + (int64_t)t * Lrow + (int64_t)w * Lcap;
  uint16_t* entp_t = entp + (int64_t)t * Lrow + (int64_t)w * Lcap;
  int32_t* cntp_t = cntp + (int64_t)t * Lrow + (int64_t)w * Lcap;
  if (valid) {
    if (occ && rank < Lcap) {
      pos_t[u] = w * Lcap + rank;
      ent_t[rank] = fold_entry((uint32_t)u, log2c);
        entp_t[rank] = pair_entry((uint32_t)u, log2c);
      cntp_t[rank] = c;
    } else {
      pos_t[u] = -1;
      if (occ) atomicExch(overflow, 1);
    }
  }
  if (tid == 0 && (int64_t)(chunk + 1) * 1024 >= nseg) segcount[t * W + w] = base + wave_tot[0];
}

// One block per repetition: segment padding, per-position member offsets.
__global__ __launch_bounds__(1024) void k_layout_finish(int W, int G, int Lcap, int Lrow,
                                                        const int32_t* __restrict__ segcount,
                                                        int32_t* __restrict__ lseg,
                                                        uint32_t* __restrict__ ent,
                                                        uint16_t* __restrict__ entp,
                                                        uint32_t* __restrict__ tab,
                                                        int32_t* __restrict__ cntp,
                                                        int32_t* __restrict__ moff) {
  const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  __shared__ int s_l;
  __shared__ int wave_tot[16];
  __shared__ int wave_pre[16];
  if (tid == 0) {
    int mx = 0;
    for (int w = 0; w < W; ++w) mx = max(mx, min(segcount[t * W + w], Lcap));
    int l = (mx + 63) & ~63;
    s_l = min(l, Lcap);
    lseg[t] = s_l;
  }
  __syncthreads();
  const int L = s_l;
  uint32_t* ent_t = ent + (int64_t)t * Lrow;
  uint16_t* entp_t = entp + (int64_t)t * Lrow;
  uint32_t* tab_t = tab + (int64_t)t * Lrow;
  int32_t* cntp_t = cntp + (int64_t)t * Lrow;
  int32_t* moff_t = moff + (int64_t)t * Lrow;
  int base = 0;
  for (int w = 0; w < W; ++w) {
    int sc = min(segcount[t * W + w], Lcap);
    for (int r = sc + tid; r < L; r += blockDim.x) {
      ent_t[w * Lcap + r] = pad_entry(w, G, r);
      entp_t[w * Lcap + r] = (uint16_t)pad_entry(w, G, r);
      tab_t[w * Lcap + r] = CMM_PAD_TAB;
      cntp_t[w * Lcap + r] = 0;
    }
    for (int r0 = 0; r0 < sc; r0 += 1024) {
      int r = r0 + tid;
      int c = r < sc ? cntp_t[w * Lcap + r] : 0;
      // inclusive scan of c within the wave
      int v = c;
      for (int off = 1; off < 64; off <<= 1) {
        int y = __shfl_up(v, off, 64);
        if (lane >= off) v += y;
      }
      if (lane == 63) wave_tot[wv] = v;
      __syncthreads();
      if (tid == 0) {
        int acc = 0;
        for (int i = 0; i < 16; ++i) { wave_pre[i] = acc; acc += wave_tot[i]; }
        wave_tot[0] = acc;
      }
      __syncthreads();
      if (r < sc) moff_t[w * Lcap + r] = base + wave_pre[wv] + v - c;
      int tot = wave_tot[0];
      __syncthreads();
      base += tot;
    }
  }
}

// Scatter every element into its bucket's member list (order fixed later).
__global__ void k_place(const int32_t* __restrict__ hs, int d, int n, int64_t b, int Lrow,
                        const int32_t* __restrict__ pos, const int32_t* __restrict__ moff,
                        int32_t* __restrict__ fill, int32_t* __restrict__ perm) {
  const int64_t total = (int64_t)d * n;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int t = (int)(idx / n);
    int x = (int)(idx - (int64_t)t * n);
    int u = hs[idx] >> 1;
    int p = pos[(int64_t)t * b + u];
    if (p < 0) continue;   // overflowed layout; the call is retried
    int slot = atomicAdd(&fill[(int64_t)t * Lrow + p], 1);
    perm[(int64_t)t * n + moff[(int64_t)t * Lrow + p] + slot] = x;
  }
}

// Sort each bucket's members by index (deterministic summation order) and
// write the count-sketch gather table.
__global__ void k_build_tab(const int32_t* __restrict__ hs, int d, int n, int W, int Lcap,
                            int Lrow, const int32_t* __restrict__ segcount,
                            const int32_t* __restrict__ cntp, const int32_t* __restrict__ moff,
                            int32_t* __restrict__ perm, uint32_t* __restrict__ tab) {
  const int64_t total = (int64_t)d * Lrow;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int t = (int)(idx / Lrow);
    int p = (int)(idx - (int64_t)t * Lrow);
    int w = p / Lcap, r = p - w * Lcap;
    if (r >= min(segcount[t * W + w], Lcap)) continue;
    int c = cntp[idx];
    int32_t* mem = perm + (int64_t)t * n + moff[idx];
    for (int a = 1; a < c; ++a) {          // insertion sort, buckets are short
      int v = mem[a], q = a - 1;
      while (q >= 0 && mem[q] > v) { mem[q + 1] = mem[q]; --q; }
      mem[q + 1] = v;
    }
    int first = mem[0];
    uint32_t neg = (uint32_t)(hs[(int64_t)t * n + first] & 1);
    tab[idx] = (uint32_t)first | (neg << 31) | (c > 1 ? CMM_TAB_MORE : 0u);
  }
}

hipError_t launch_layout(const Geometry& g, SideDesc& sd, int32_t* overflow, hipStream_t s) {
  hipError_t e;
  const int64_t nchunks = (g.b / g.W + 1023) / 1024;
  if (nchunks <= kRankChunks)
    hipLaunchKernelGGL(k_segment_rank_chunks, dim3((unsigned)nchunks, g.W, g.d), dim3(1024), 0, s, sd.cnt,
                       g.b, g.log2c, g.T, g.G, g.W, sd.Lcap, sd.Lrow, sd.pos, sd.ent, sd.entp, sd.cntp,
                       sd.segcount, overflow);
  else
    hipLaunchKernelGGL(k_segment_rank, dim3(g.W, g.d), dim3(1024), 0, s, sd.cnt, g.b, g.log2c, g.T, g.G,
                       g.W, sd.Lcap, sd.Lrow, sd.pos, sd.ent, sd.entp, sd.cntp, sd.segcount, overflow);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_layout_finish, dim3(g.d), dim3(1024), 0, s, g.W, g.G, sd.Lcap, sd.Lrow,
                     sd.segcount, sd.lseg, sd.ent, sd.entp, sd.tab, sd.cntp, sd.moff);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_fill_i32(sd.fill, (int64_t)g.d * sd.Lrow, 0, s)) != hipSuccess) return e;
  int64_t total = (int64_t)g.d * sd.n;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_place, dim3((unsigned)blocks), dim3(256), 0, s, sd.hs, g.d, sd.n, g.b,
                     sd.Lrow, sd.pos, sd.moff, sd.fill, sd.perm);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int64_t total2 = (int64_t)g.d * sd.Lrow;
  int64_t blocks2 = (total2 + 255) / 256;
  if (blocks2 > 8192) blocks2 = 8192;
  hipLaunchKernelGGL(k_build_tab, dim3((unsigned)blocks2), dim3(256), 0, s, sd.hs, g.d, sd.n,
                     g.W, sd.Lcap, sd.Lrow, sd.segcount, sd.cntp, sd.moff, sd.perm, sd.tab);
  return hipGetLastError();
}

}  // namespace cmm

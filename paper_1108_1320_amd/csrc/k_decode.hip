// Decoding (Figure 1, DECOMPRESS): X_t = s1_t(i) s2_t(j) c_t[(h1_t(i) +
// h2_t(j)) mod b], estimate = median over the d repetitions (Section 3.3),
// and selection of the estimates of largest magnitude without storing the
// n1-by-n3 estimate matrix (the product stays implicit, Section 2.2).
//
// Global top-K works on the 32-bit key |estimate| (float bits are ordered
// like the values for non-negative floats) in passes that re-decode the
// candidate domain: a histogram of the key's top 12 bits locates the bin of
// the K-th largest key, further 12- and 7-bit digit passes refine it if the
// bin is crowded, one pass collects every candidate at or above the
// threshold, and a single block sorts them by (key desc, i*n3+j asc).
#include "cmm_internal.h"

namespace cmm {

template <int D>
__device__ __forceinline__ float estimate(const DecodeDesc& dd, const int32_t* a1, const int32_t* a2,
                                          int dr) {
  // a1[t] = hs1[t][i], a2[t] = hs2[t][j]
  if constexpr (D > 0) {
    float x[D];
#pragma unroll
    for (int t = 0; t < D; ++t) {
      const uint32_t u = (uint32_t)((a1[t] >> 1) + (a2[t] >> 1)) & dd.mask;
      const float v = dd.c32[(int64_t)t * dd.b + u];
      x[t] = ((a1[t] ^ a2[t]) & 1) ? -v : v;
    }
    // odd-even transposition sort, D rounds
#pragma unroll
    for (int r = 0; r < D; ++r) {
#pragma unroll
      for (int q = (r & 1); q + 1 < D; q += 2) {
        const float lo = fminf(x[q], x[q + 1]), hi = fmaxf(x[q], x[q + 1]);
        x[q] = lo; x[q + 1] = hi;
      }
    }
    if constexpr (D & 1) return x[(D - 1) / 2];
    else return 0.5f * (x[D / 2 - 1] + x[D / 2]);
  } else {
    float x[64];
    for (int t = 0; t < dr; ++t) {
      const uint32_t u = (uint32_t)((a1[t] >> 1) + (a2[t] >> 1)) & dd.mask;
      const float v = dd.c32[(int64_t)t * dd.b + u];
      const float y = ((a1[t] ^ a2[t]) & 1) ? -v : v;
      int q = t - 1;
      while (q >= 0 && x[q] > y) { x[q + 1] = x[q]; --q; }
      x[q + 1] = y;
    }
    return (dr & 1) ? x[(dr - 1) / 2] : 0.5f * (x[dr / 2 - 1] + x[dr / 2]);
  }
}

// The estimate of (i, j) if its magnitude can reach T, else NaN.  |median| >= T
// needs at least ceil(d/2) of the d signed values >= T or at least as many
// <= -T (for even d the larger middle value must reach T), so the values are
// gathered one repetition at a time and the gathering stops once neither
// count can get there; a surviving candidate's estimate is computed exactly
// as estimate() does.
template <int D>
__device__ __forceinline__ float estimate_above(const DecodeDesc& dd, const int32_t* a1,
                                                const int32_t* a2, float T) {
  static_assert(D > 0, "fixed d only");
  constexpr int need = (D + 1) / 2;
  float x[D];
  int hi = 0, lo = 0;
#pragma unroll
  for (int t = 0; t < D; ++t) {
    const uint32_t u = (uint32_t)((a1[t] >> 1) + (a2[t] >> 1)) & dd.mask;
    const float v = dd.c32[(int64_t)t * dd.b + u];
    x[t] = ((a1[t] ^ a2[t]) & 1) ? -v : v;
    hi += x[t] >= T;
    lo += x[t] <= -T;
    const int left = D - 1 - t;
    if (hi + left < need && lo + left < need) return __uint_as_float(0x7FC00000u);
  }
#pragma unroll
  for (int r = 0; r < D; ++r) {
#pragma unroll
    for (int q = (r & 1); q + 1 < D; q += 2) {
      const float l = fminf(x[q], x[q + 1]), h = fmaxf(x[q], x[q + 1]);
      x[q] = l; x[q + 1] = h;
    }
  }
  if constexpr (D & 1) return x[(D - 1) / 2];
  else return 0.5f * (x[D / 2 - 1] + x[D / 2]);
}

template <int D> struct HashVec {
  int32_t v[D > 0 ? D : 64];
};

template <int D>
__device__ __forceinline__ void load_hash(HashVec<D>& h, const int32_t* hs, int n, int x, int dr) {
  if constexpr (D > 0) {
#pragma unroll
    for (int t = 0; t < D; ++t) h.v[t] = hs[(int64_t)t * n + x];
  } else {
    for (int t = 0; t < dr; ++t) h.v[t] = hs[(int64_t)t * n + x];
  }
}

// ---------------------------------------------------------------- batch

template <int D>
__global__ void k_estimate(DecodeDesc dd, const int64_t* __restrict__ qi,
                           const int64_t* __restrict__ qj, int64_t q, float* __restrict__ out) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < q;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = qi[idx], j = qj[idx];
    if (i < 0 || j < 0 || i >= dd.n1 || j >= dd.n3) { out[idx] = __uint_as_float(0x7FC00000u); continue; }
    HashVec<D> h1, h2;
    load_hash<D>(h1, dd.hs1, dd.n1, (int)i, dd.d);
    load_hash<D>(h2, dd.hs2, dd.n3, (int)j, dd.d);
    out[idx] = estimate<D>(dd, h1.v, h2.v, dd.d);
  }
}

// ------------------------------------------------------------- top-K passes
// Tile: 16 rows i (uniform in the block) x 256 columns j (one per thread).
constexpr int kTI = 16;

__device__ __forceinline__ bool in_domain(int mode, int i, int j, int n1, int n3) {
  return i < n1 && j < n3 && (mode != 1 || i < j);
}

// Screening bitmap for a key threshold (Section 3.3: |median| >= T needs
// ceil(d/2) of the d values to reach T in magnitude).  Bit (u mod W) of row t
// is set when some bucket u' = u (mod W) of repetition t has |c_t[u']| >= T;
// rows t < nf, W = 2^log2w (a power of two dividing b, at least 64).  A
// candidate whose first nf = d - ceil(d/2) + 1 buckets all have clear bits
// cannot reach T (at most d - nf values could), so the pass skips it without
// touching c; folding several buckets into one bit only lets more candidates
// through to the exact test.
__global__ void k_screen_bits(DecodeDesc dd, int nf, int log2w, uint32_t thresh,
                              uint32_t* __restrict__ bits) {
  const int64_t W = (int64_t)1 << log2w;
  const int64_t total = (int64_t)nf * W;   // a multiple of 64
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(idx >> log2w);
    const int64_t u0 = idx & (W - 1);
    bool big = false;
    for (int64_t u = u0; u < dd.b; u += W)
      big |= (__float_as_uint(dd.c32[(int64_t)t * dd.b + u]) & 0x7FFFFFFFu) >= thresh;
    const unsigned long long m = __ballot(big);
    if ((threadIdx.x & 63) == 0) {
      bits[idx >> 5] = (uint32_t)m;
      bits[(idx >> 5) + 1] = (uint32_t)(m >> 32);
    }
  }
}

// Histogram of one key digit over the candidates whose key matches
// `prefix` under `pmask`, over every tile_stride-th tile of 16 rows (1 = the
// whole domain).  With COLLECT, only candidates with key >= thresh are
// counted, and they are also appended to `cand` (at most `cap`; `count`
// keeps counting past it).
template <int D, bool COLLECT>
__global__ __launch_bounds__(256) void k_topk_hist(DecodeDesc dd, int mode, int tile_stride,
                                                   uint32_t pmask, uint32_t prefix, int dshift,
                                                   uint32_t dmask, uint32_t* __restrict__ hist,
                                                   uint32_t thresh, TopkCand* __restrict__ cand,
                                                   uint32_t* __restrict__ count, int cap,
                                                   const uint32_t* __restrict__ screen, int log2w) {
  __shared__ uint32_t h[4096];
  extern __shared__ uint32_t sbits[];   // the screening bitmap (COLLECT with a screen)
  constexpr int kNeed = (D + 1) / 2;
  constexpr int kNF = D - kNeed + 1;
  const int tid = threadIdx.x;
  const int j = blockIdx.x * 256 + tid;
  const int i0 = blockIdx.y * tile_stride * kTI;
  if (mode == 1 && i0 >= (int)(blockIdx.x * 256 + 255)) return;   // tile below the diagonal
  for (int q = tid; q < 4096; q += 256) h[q] = 0;
  const bool scr = COLLECT && D > 0 && screen != nullptr;
  const uint32_t wmask = ((uint32_t)1 << log2w) - 1u;
  const int wrow = scr ? (1 << log2w) >> 5 : 0;   // words per repetition
  if (scr)
    for (int q = tid; q < kNF * wrow; q += 256) sbits[q] = screen[q];
  __syncthreads();
  if (j < dd.n3) {
    HashVec<D> h2;
    load_hash<D>(h2, dd.hs2, dd.n3, j, dd.d);
    for (int ii = 0; ii < kTI; ++ii) {
      const int i = i0 + ii;
      if (!in_domain(mode, i, j, dd.n1, dd.n3)) continue;
      HashVec<D> h1;
      load_hash<D>(h1, dd.hs1, dd.n1, i, dd.d);
      float est;
      if constexpr (COLLECT && D > 0) {
        if (scr) {
          int big = 0;
#pragma unroll
          for (int t = 0; t < kNF; ++t) {
            const uint32_t u = (uint32_t)((h1.v[t] >> 1) + (h2.v[t] >> 1)) & wmask;
            big += (sbits[t * wrow + (u >> 5)] >> (u & 31)) & 1u;
          }
          if (big + (D - kNF) < kNeed) continue;   // cannot reach the threshold
        }
        est = estimate_above<D>(dd, h1.v, h2.v, __uint_as_float(thresh));
        if (est != est) continue;   // cannot reach the threshold
      } else {
        est = estimate<D>(dd, h1.v, h2.v, dd.d);
      }
      const uint32_t key = __float_as_uint(fabsf(est));
      if constexpr (COLLECT) {
        // only keys >= thresh are counted (and kept): the bulk of the
        // distribution, far below it, never touches the histogram
        if (key >= thresh) {
          if ((key & pmask) == prefix) atomicAdd(&h[(key >> dshift) & dmask], 1u);
          const uint32_t slot = atomicAdd(count, 1u);
          if (slot < (uint32_t)cap) {
            TopkCand c; c.key = key; c.i = i; c.j = j; c.val = est;
            cand[slot] = c;
          }
        }
      } else {
        if ((key & pmask) == prefix) atomicAdd(&h[(key >> dshift) & dmask], 1u);
      }
    }
  }
  __syncthreads();
  for (int q = tid; q < 4096; q += 256)
    if (h[q]) atomicAdd(&hist[q], h[q]);
}

// Keep the candidates with key >= thresh (order not kept).
__global__ void k_topk_filter(const TopkCand* __restrict__ in, const uint32_t* __restrict__ in_count,
                              int in_cap, uint32_t thresh, TopkCand* __restrict__ out,
                              uint32_t* __restrict__ out_count, int out_cap) {
  const uint32_t c = *in_count;
  const int n = (int)(c < (uint32_t)in_cap ? c : (uint32_t)in_cap);
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const TopkCand e = in[q];
    if (e.key >= thresh) {
      const uint32_t slot = atomicAdd(out_count, 1u);
      if (slot < (uint32_t)out_cap) out[slot] = e;
    }
  }
}

template <int D>
__global__ __launch_bounds__(256) void k_topk_collect(DecodeDesc dd, int mode, uint32_t thresh,
                                                      TopkCand* __restrict__ cand,
                                                      uint32_t* __restrict__ count, int cap) {
  const int tid = threadIdx.x;
  const int j = blockIdx.x * 256 + tid;
  const int i0 = blockIdx.y * kTI;
  if (mode == 1 && i0 >= (int)(blockIdx.x * 256 + 255)) return;
  if (j >= dd.n3) return;
  HashVec<D> h2;
  load_hash<D>(h2, dd.hs2, dd.n3, j, dd.d);
  for (int ii = 0; ii < kTI; ++ii) {
    const int i = i0 + ii;
    if (!in_domain(mode, i, j, dd.n1, dd.n3)) continue;
    HashVec<D> h1;
    load_hash<D>(h1, dd.hs1, dd.n1, i, dd.d);
    const float est = estimate<D>(dd, h1.v, h2.v, dd.d);
    const uint32_t key = __float_as_uint(fabsf(est));
    if (key >= thresh) {
      const uint32_t slot = atomicAdd(count, 1u);
      if (slot < (uint32_t)cap) {
        TopkCand c; c.key = key; c.i = i; c.j = j; c.val = est;
        cand[slot] = c;
      }
    }
  }
}

__device__ __forceinline__ bool later(const TopkCand& a, const TopkCand& b, int n3) {
  // true if a sorts after b: smaller key, or equal key and larger i*n3+j
  if (a.key != b.key) return a.key < b.key;
  return (int64_t)a.i * n3 + a.j > (int64_t)b.i * n3 + b.j;
}

__global__ __launch_bounds__(1024) void k_topk_final(const TopkCand* __restrict__ cand,
                                                     const uint32_t* __restrict__ count, int cap,
                                                     int K, int n3, int64_t* __restrict__ oi,
                                                     int64_t* __restrict__ oj,
                                                     float* __restrict__ ov) {
  __shared__ TopkCand s[kTopkCap];
  const int tid = threadIdx.x;
  const uint32_t cnt = *count;
  const int n = (int)(cnt < (uint32_t)cap ? cnt : (uint32_t)cap);
  int N2 = 1;
  while (N2 < n) N2 <<= 1;
  for (int q = tid; q < N2; q += 1024) {
    if (q < n) s[q] = cand[q];
    else { TopkCand z; z.key = 0; z.i = 0x7FFFFFFF; z.j = 0x7FFFFFFF; z.val = 0.f; s[q] = z; }
  }
  for (int size = 2; size <= N2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int q = tid; q < N2; q += 1024) {
        const int l = q ^ stride;
        if (l > q) {
          const TopkCand a = s[q], b = s[l];
          const bool up = (q & size) == 0;
          if (up ? later(a, b, n3) : later(b, a, n3)) { s[q] = b; s[l] = a; }
        }
      }
    }
  }
  __syncthreads();
  for (int r = tid; r < K; r += 1024) {
    if (r < n) { oi[r] = s[r].i; oj[r] = s[r].j; ov[r] = s[r].val; }
    else { oi[r] = -1; oj[r] = -1; ov[r] = 0.f; }
  }
}

// ---------------------------------------------------------------- per column

// One block per column j; K rounds, each picking the best (|estimate|, then
// smaller i) strictly below the previous pick.  STORE keeps the column's
// keys in LDS (n1 <= kMaxColumnKeys); otherwise every round decodes the
// column again.
constexpr int kColList = 256;   // survivors listed by the per-column sampled path
// dynamic LDS of the stored per-column kernel: the keys, then (when it fits)
// the survivor list
constexpr size_t kColumnLds = (size_t)kMaxColumnKeys * 4;

template <int D, bool STORE>
__global__ __launch_bounds__(256) void k_topk_column(DecodeDesc dd, int K, int64_t* __restrict__ oi,
                                                     float* __restrict__ ov, bool list) {
  extern __shared__ uint32_t keys[];
  __shared__ unsigned long long wbest[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int j = blockIdx.x;
  HashVec<D> h2;
  load_hash<D>(h2, dd.hs2, dd.n3, j, dd.d);
  auto key = [&](int i) -> uint32_t {
    HashVec<D> h1;
    load_hash<D>(h1, dd.hs1, dd.n1, i, dd.d);
    return __float_as_uint(fabsf(estimate<D>(dd, h1.v, h2.v, dd.d)));
  };
  // the best key strictly below `last` over keys[0 .. cnt) (block-wide)
  auto best_below = [&](int cnt, unsigned long long last) -> unsigned long long {
    unsigned long long best = 0ull;
    for (int i = tid; i < cnt; i += 256) {
      const unsigned long long p = ((unsigned long long)keys[i] << 32) | (uint32_t)(0xFFFFFFFFu - (uint32_t)i);
      if (p < last && p > best) best = p;
    }
    for (int off = 32; off > 0; off >>= 1) {
      const unsigned long long o = __shfl_xor(best, off, 64);
      best = o > best ? o : best;
    }
    if (lane == 0) wbest[wv] = best;
    __syncthreads();
    best = wbest[0];
    for (int q = 1; q < 4; ++q) best = wbest[q] > best ? wbest[q] : best;
    __syncthreads();
    return best;
  };
  if constexpr (STORE) {
    bool exact = true;
    if constexpr (D > 0) {
      if (dd.n1 >= 1024) {
        // threshold from every 16th row: the r-th largest sampled key with
        // r = ceil(K/16) + 2 leaves about 16 r >= K + 32 rows above it; the
        // full pass then stops decoding a row as soon as its median cannot
        // reach the threshold (estimate_above), and keeps key 0 for it
        const int ns = (dd.n1 + 15) / 16;
        for (int q = tid; q < ns; q += 256) keys[q] = key(16 * q);
        __syncthreads();
        const int rr = min(ns, (K + 15) / 16 + 2);
        unsigned long long lastp = ~0ull;
        for (int r = 0; r < rr; ++r) lastp = best_below(ns, lastp);
        const uint32_t T = (uint32_t)(lastp >> 32);
        // rows reaching T, with their estimates, in arrival order (in the
        // dynamic LDS after the keys when the launch made room: list = true)
        __shared__ int survivors;
        uint32_t* skey = keys + dd.n1;
        int* srow = reinterpret_cast<int*>(skey + kColList);
        float* sval = reinterpret_cast<float*>(srow + kColList);
        const int cap = list ? kColList : 0;
        if (tid == 0) survivors = 0;
        __syncthreads();
        for (int i = tid; i < dd.n1; i += 256) {
          HashVec<D> h1;
          load_hash<D>(h1, dd.hs1, dd.n1, i, dd.d);
          const float e = estimate_above<D>(dd, h1.v, h2.v, __uint_as_float(T));
          const bool keep = e == e && __float_as_uint(fabsf(e)) >= T;
          keys[i] = keep ? __float_as_uint(fabsf(e)) : 0u;
          if (keep) {
            const int slot = atomicAdd(&survivors, 1);
            if (slot < cap) { skey[slot] = __float_as_uint(fabsf(e)); srow[slot] = i; sval[slot] = e; }
          }
        }
        __syncthreads();
        const int S = survivors;
        // exact when at least K rows reach T: every row left at key 0 lies
        // below all of them
        exact = S < K;
        if (!exact && S <= cap) {
          // the K largest survivors by (key desc, row asc): each survivor's
          // rank is the number of survivors ahead of it
          for (int a = tid; a < S; a += 256) {
            const uint32_t ka = skey[a];
            const int ia = srow[a];
            int rank = 0;
            for (int c = 0; c < S; ++c) rank += (skey[c] > ka) || (skey[c] == ka && srow[c] < ia);
            if (rank < K) {
              oi[(int64_t)j * K + rank] = ia;
              ov[(int64_t)j * K + rank] = sval[a];
            }
          }
          return;
        }
      }
    }
    if (exact) {
      for (int i = tid; i < dd.n1; i += 256) keys[i] = key(i);
      __syncthreads();
    }
  }
  unsigned long long last = ~0ull;
  for (int r = 0; r < K; ++r) {
    // packed (key, ~i): larger is better; pick the best strictly below `last`
    unsigned long long best = 0ull;
    for (int i = tid; i < dd.n1; i += 256) {
      const uint32_t kv = STORE ? keys[i] : key(i);
      const unsigned long long p = ((unsigned long long)kv << 32) | (uint32_t)(0xFFFFFFFFu - (uint32_t)i);
      if (p < last && p > best) best = p;
    }
    for (int off = 32; off > 0; off >>= 1) {
      const unsigned long long o = __shfl_xor(best, off, 64);
      best = o > best ? o : best;
    }
    if (lane == 0) wbest[wv] = best;
    __syncthreads();
    best = wbest[0];
    for (int q = 1; q < 4; ++q) best = wbest[q] > best ? wbest[q] : best;
    __syncthreads();
    last = best;
    if (tid == 0) {
      const int i = (int)(0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFull));
      HashVec<D> h1;
      load_hash<D>(h1, dd.hs1, dd.n1, i, dd.d);
      oi[(int64_t)j * K + r] = i;
      ov[(int64_t)j * K + r] = estimate<D>(dd, h1.v, h2.v, dd.d);
    }
  }
}

// ---------------------------------------------------------------- launchers

#define CMM_DISPATCH_D(d, MACRO)                                                   \
  switch (d) {                                                                     \
    case 1: MACRO(1); break;  case 2: MACRO(2); break;  case 3: MACRO(3); break;   \
    case 4: MACRO(4); break;  case 5: MACRO(5); break;  case 6: MACRO(6); break;   \
    case 7: MACRO(7); break;  case 8: MACRO(8); break;  case 9: MACRO(9); break;   \
    case 10: MACRO(10); break; case 11: MACRO(11); break; case 12: MACRO(12); break; \
    case 13: MACRO(13); break; case 14: MACRO(14); break; case 15: MACRO(15); break; \
    default: MACRO(0); break;                                                      \
  }

static inline unsigned grid1(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > 16384) g = 16384;
  return (unsigned)g;
}

hipError_t launch_estimate(const DecodeDesc& dd, const int64_t* qi, const int64_t* qj, int64_t q,
                           float* out, hipStream_t s) {
  if (q <= 0) return hipSuccess;
#define CMM_EST(DV) hipLaunchKernelGGL(k_estimate<DV>, dim3(grid1(q)), dim3(256), 0, s, dd, qi, qj, q, out)
  CMM_DISPATCH_D(dd.d, CMM_EST)
#undef CMM_EST
  return hipGetLastError();
}

hipError_t launch_topk_hist(const DecodeDesc& dd, int mode, int tile_stride, uint32_t prefix,
                            int prefix_shift, int digit_shift, uint32_t digit_mask, uint32_t* hist,
                            uint32_t thresh, TopkCand* cand, uint32_t* count, int cap,
                            hipStream_t s, const uint32_t* screen, int screen_log2w) {
  const uint32_t pmask = prefix_shift >= 32 ? 0u : ~((1u << prefix_shift) - 1u);
  const int tiles = (dd.n1 + kTI - 1) / kTI;
  dim3 grid((dd.n3 + 255) / 256, (tiles + tile_stride - 1) / tile_stride);
  if (cand) {
    const size_t slds = screen ? (size_t)screen_nf(dd.d) * ((size_t)1 << screen_log2w) / 8 : 0;
#define CMM_H(DV) hipLaunchKernelGGL((k_topk_hist<DV, true>), grid, dim3(256), slds, s, dd, mode, tile_stride, pmask, prefix & pmask, digit_shift, digit_mask, hist, thresh, cand, count, cap, screen, screen_log2w)
    CMM_DISPATCH_D(dd.d, CMM_H)
#undef CMM_H
  } else {
#define CMM_H(DV) hipLaunchKernelGGL((k_topk_hist<DV, false>), grid, dim3(256), 0, s, dd, mode, tile_stride, pmask, prefix & pmask, digit_shift, digit_mask, hist, 0u, (TopkCand*)nullptr, (uint32_t*)nullptr, 0, (const uint32_t*)nullptr, 0)
    CMM_DISPATCH_D(dd.d, CMM_H)
#undef CMM_H
  }
  return hipGetLastError();
}

int screen_nf(int d) { return d - (d + 1) / 2 + 1; }

int screen_log2w(int d, int64_t b) {
  // the bitmap of screen_nf(d) rows stays within 32 KB of LDS
  if (d < 1 || d > 15 || b < 4096) return 0;
  int lw = 0;
  while (((int64_t)1 << (lw + 1)) <= b && ((int64_t)screen_nf(d) << (lw + 1)) <= 8 * 32768) ++lw;
  return lw >= 6 ? lw : 0;
}

hipError_t launch_screen_bits(const DecodeDesc& dd, uint32_t thresh, int log2w, uint32_t* bits,
                              hipStream_t s) {
  const int64_t total = (int64_t)screen_nf(dd.d) << log2w;
  const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_screen_bits, dim3(grid), dim3(256), 0, s, dd, screen_nf(dd.d), log2w, thresh, bits);
  return hipGetLastError();
}

hipError_t launch_topk_filter(const TopkCand* in, const uint32_t* in_count, int in_cap,
                              uint32_t thresh, TopkCand* out, uint32_t* out_count, int out_cap,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_topk_filter, dim3(grid1(in_cap)), dim3(256), 0, s, in, in_count, in_cap,
                     thresh, out, out_count, out_cap);
  return hipGetLastError();
}

hipError_t launch_topk_collect(const DecodeDesc& dd, int mode, uint32_t thresh, TopkCand* cand,
                               uint32_t* count, int cap, hipStream_t s) {
  dim3 grid((dd.n3 + 255) / 256, (dd.n1 + kTI - 1) / kTI);
#define CMM_C(DV) hipLaunchKernelGGL(k_topk_collect<DV>, grid, dim3(256), 0, s, dd, mode, thresh, cand, count, cap)
  CMM_DISPATCH_D(dd.d, CMM_C)
#undef CMM_C
  return hipGetLastError();
}

hipError_t launch_topk_final(const TopkCand* cand, const uint32_t* count, int cap, int K, int n3,
                             int64_t* oi, int64_t* oj, float* ov, hipStream_t s) {
  hipLaunchKernelGGL(k_topk_final, dim3(1), dim3(1024), 0, s, cand, count, cap, K, n3, oi, oj, ov);
  return hipGetLastError();
}

hipError_t launch_topk_column(const DecodeDesc& dd, int K, int64_t* oi, float* ov, hipStream_t s) {
  const bool store = dd.n1 <= kMaxColumnKeys;
  // the survivor list follows the keys when both fit in the 160 KB
  const size_t keys = (size_t)dd.n1 * sizeof(uint32_t);
  const size_t list_bytes = (size_t)kColList * (sizeof(uint32_t) + sizeof(int) + sizeof(float));
  const bool list = store && keys + list_bytes <= kColumnLds;
  const size_t lds = store ? keys + (list ? list_bytes : 0) : 0;
#define CMM_K(DV)                                                                              \
  if (store) hipLaunchKernelGGL((k_topk_column<DV, true>), dim3(dd.n3), dim3(256), lds, s, dd, K, oi, ov, list); \
  else hipLaunchKernelGGL((k_topk_column<DV, false>), dim3(dd.n3), dim3(256), 0, s, dd, K, oi, ov, false)
  CMM_DISPATCH_D(dd.d, CMM_K)
#undef CMM_K
  return hipGetLastError();
}

// Raise the dynamic LDS limit of the stored per-column top-K to its 160 KB
// of keys (done once per context, outside any graph capture).
hipError_t prepare_decode() {
#define CMM_P(DV)                                                                          \
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_topk_column<DV, true>),          \
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)kColumnLds);     \
  if (e != hipSuccess) return e;
  hipError_t e = hipSuccess;
  CMM_P(0) CMM_P(1) CMM_P(2) CMM_P(3) CMM_P(4) CMM_P(5) CMM_P(6) CMM_P(7) CMM_P(8)
  CMM_P(9) CMM_P(10) CMM_P(11) CMM_P(12) CMM_P(13) CMM_P(14) CMM_P(15)
#undef CMM_P
  return hipSuccess;
}

}  // namespace cmm

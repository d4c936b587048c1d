// Fused forward FFT and spectral multiply-accumulate (Figure 1: FFT of pa
// and pb, pointwise product, sum over k; Section 2.2: the pointwise product
// of the two Fourier representations is the Fourier representation of the
// count sketch of the outer product).
//
// The length-b transform of a count-sketch vector x (at most n non-zero
// coefficients) is split four-step style, b = R * C:
//
//   X[f1 + R f2] = DFT_C( z_f1 )[f2],
//   z_f1[r]      = w_b^(f1 r) * sum_q x[r + C q] w_R^(f1 q)   (r < C, q < R)
//
// so every "row" f1 is a weighted fold of the sketch's non-zero entries into
// C slots followed by one C-point FFT in LDS.  x is real, so rows
// f1 in [0, R/2] carry the whole spectrum (X[b - f] = conj X[f]).  One
// block owns one (repetition t, row f1, range of at most 128 k): for each k
// it folds the column sketch of A and the row sketch of B, transforms both,
// multiplies them bin by bin and adds the products into float32
// accumulators held in registers; the per-block partial sums are added in
// float64 afterwards.  The n-by-b spectra are never stored.
//
// FFT: Stockham autosort, T = C/16 threads with 16 complex values each; the
// first stage has radix 2^(log2 C mod 4) (if not zero) and the rest radix
// 16, with LDS exchanges (xor-swizzled) between stages.  Thread j starts
// with slots j + T v and ends with frequencies j + T v.
//
// Fold: the slots of thread j are exactly the buckets u with u mod T = j.
// The bucket layout hands every wave only buckets whose slots belong to its
// own lanes, so a wave's LDS atomics never touch another wave's slots; the
// sums are exact integer (fixed-point) sums, independent of their order.
#include "cmm_internal.h"
#include "cmm_dft.h"
#include <algorithm>
#include <cmath>

namespace cmm {

// LDS index swizzle: xor the low 4 bits with bits 4..7.  Rows of 16
// consecutive complex values stay rows (stage reads at j + T v are
// conflict-free) and the stride-16 writes of the first radix-16 stage spread
// over all banks.
__device__ __forceinline__ int sw(int i) { return fft_swizzle(i); }

// LDS address of slot j + T q (the own positions of thread j).  For T a
// multiple of 256 the swizzle leaves the T q part alone, so the address is
// one base plus an immediate offset.
template <int T> __device__ __forceinline__ int own(int jbase, int j, int q) {
  if constexpr (T % 256 == 0) return jbase + T * q;
  else return sw(j + T * q);
}

struct FftArgs {
  const float* SA0; const float* SA1;
  const uint32_t* ent0; const uint32_t* ent1;
  const uint16_t* entp0; const uint16_t* entp1;   // the row pair's entries
  const int32_t* lseg0; const int32_t* lseg1;
  const float* cmax0; const float* cmax1;
  int Lcap0, Lcap1, Lrow0, Lrow1;
  const float2* tw;        // omega_b^x for x < b
  float2* Ppart;
  int64_t b;
  int R, rows, nrow, roff, d, m, KS;
};

// LDS element at byte offset `off` (fold entries and stage writes carry byte
// offsets).
template <typename V> __device__ __forceinline__ V& at_byte(V* base, uint32_t off) {
  return *reinterpret_cast<V*>(reinterpret_cast<char*>(base) + off);
}
template <typename V> __device__ __forceinline__ const V& at_byte(const V* base, uint32_t off) {
  return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + off);
}

constexpr int ipow16(int e) { return e <= 0 ? 1 : 16 * ipow16(e - 1); }

template <int L> struct FftShape {
  static constexpr int C = 1 << L;
  static constexpr int T = C / 16;
  static constexpr int E = L % 4;
  static constexpr int S = L / 4 + (E ? 1 : 0);
  static constexpr int G = T < 64 ? T : 64;
  // fold entries per lane and batch.  At L = 12, 17 entries per lane hold a
  // whole wave segment of up to 1088 entries (n = b/16 gives segments of
  // about 1000 +- 32), so no fetch waits after the transform.  L = 13 has 8
  // waves, half the entries each.
  static constexpr int U = L == 12 ? 17 : (L == 13 ? 4 : 8);
  static constexpr int span(int s) { return s == 0 ? 1 : (E ? (1 << E) : 16) * ipow16(s - 1); }
  static constexpr int radix(int s) { return (s == 0 && E) ? (1 << E) : 16; }
  // At L = 12 the one middle stage takes its 15 twiddles from registers
  // (like the last stage); other row lengths read those of their middle
  // stages 1 .. S-2 from an LDS table, stage s from tmoff(s) on, 15 *
  // span(s) entries (shorter rows run their fold batch and transform in
  // fewer registers, but 30 more would spill there).
  static constexpr bool kRegMid = L == 12;
  static constexpr int tmoff(int s) { return s <= 1 ? 0 : tmoff(s - 1) + 15 * span(s - 1); }
  static constexpr int NMID = (S >= 3 && !kRegMid) ? tmoff(S - 1) : 0;
};

// LDS (address space 3) views of the dynamic shared array: 32-bit byte
// addresses, so that an address formed by xor is used as it is.  The
// spectral kernels declare no static shared memory (prepare_fft_mac checks
// it), so the dynamic array starts at address 0, and the two transform
// buffers at 0 and 8C bytes: multiples of 2048 bytes for the row lengths
// whose stages write through xor-formed addresses (256 and 4096 points),
// and the xors touch bits 3..10 only.
typedef __attribute__((address_space(3))) unsigned long long lds_u64;
__device__ __forceinline__ uint32_t lds_addr(const float2* p) {
  return (uint32_t)(uintptr_t)(const lds_u64*)p;
}
__device__ __forceinline__ void lds_store(uint32_t addr, float2 v) {
  *(lds_u64*)(uintptr_t)addr = __builtin_bit_cast(unsigned long long, v);
}

// LDS address of the write of output r in stages 0 and 1 of a radix-16
// row: position sw(16 j + r) for stage 0 and sw(256 (j / 16) + (j mod 16) +
// 16 r) for stage 1.  The swizzle only mixes bits 4..7 into bits 0..3, so
// both are one base per thread xor a multiple of r: 8 r and 136 r.  The base
// (with the buffer's own address) is made opaque so that it is formed once
// per stage instead of 16 addresses being held in registers across the loop.
template <int s> __device__ __forceinline__ uint32_t stage_write_base(const float2* buf, int j) {
  uint32_t A = lds_addr(buf) + (uint32_t)(s == 0 ? 128 * j + 8 * (j & 15) : 2048 * (j >> 4) + 8 * (j & 15));
  asm volatile("" : "+v"(A));
  return A;
}

template <int L, int s> struct Stage {
  // tl: last-stage twiddles and tm1: middle-stage twiddles (registers; tm1
  // at L = 12 only); tm: middle-stage table in LDS (other row lengths),
  // tm[(r - 1) * Ns + (j mod Ns)] = omega_{16 Ns}^((j mod Ns) r).  With
  // kPre every input of stage 0 is first multiplied by pre.
  template <bool kPre>
  static __device__ __forceinline__ void run(float2* v, float2* P0, float2* P1,
                                             const float2 (&tl)[15], const float2 (&tm1)[15],
                                             const float2* tm, int j, float2 pre) {
    typedef FftShape<L> F;
    constexpr int Rs = F::radix(s);
    constexpr int BPT = 16 / Rs;
    constexpr int Ns = F::span(s);
    float2* bin = (s % 2 == 0) ? P0 : P1;
    float2* bout = (s % 2 == 0) ? P1 : P0;
    if constexpr (s > 0) {
      // radix 16; the twiddles of inputs 1..15 enter the first butterflies
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = bin[own<F::T>(sw(j), j, q)];
      if constexpr (s == F::S - 1) {
        dft16_tw(v, tl);
      } else if constexpr (F::kRegMid) {
        dft16_tw(v, tm1);
      } else {
        // table twiddles are multiplied in as they arrive (fewer registers)
        const int jm = j % Ns;
        const float2* tms = tm + F::tmoff(s);
#pragma unroll
        for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], tms[(r - 1) * Ns + jm]);
        dft16(v);
      }
    } else if constexpr (Rs == 16) {
      if constexpr (kPre) dft16_scaled(v, pre);
      else dft16(v);
    } else {
      if constexpr (kPre) {
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = cmul(v[q], pre);
      }
#pragma unroll
      for (int mi = 0; mi < BPT; ++mi) {
        float2 x[Rs];
#pragma unroll
        for (int r = 0; r < Rs; ++r) x[r] = v[mi + r * BPT];
        dft<Rs>(x);
#pragma unroll
        for (int r = 0; r < Rs; ++r) v[mi + r * BPT] = x[r];
      }
    }
    if constexpr (s < F::S - 1) {
      if constexpr (s == 0 && F::S % 2 == 0) __syncthreads();
      if constexpr (Rs == 16 && (s == 0 || Ns == 16)) {
        const uint32_t A = stage_write_base<s>(bout, j);
        constexpr uint32_t K = s == 0 ? 8 : 136;
#pragma unroll
        for (int r = 0; r < 16; ++r) lds_store(A ^ (K * (uint32_t)r), v[r]);
      } else {
#pragma unroll
        for (int mi = 0; mi < BPT; ++mi) {
          const int jb = j + F::T * mi;
          const int base = (jb / Ns) * Ns * Rs + (jb % Ns);
#pragma unroll
          for (int r = 0; r < Rs; ++r) bout[sw(base + r * Ns)] = v[mi + r * BPT];
        }
      }
      __syncthreads();
      Stage<L, s + 1>::template run<false>(v, P0, P1, tl, tm1, tm, j, pre);
    }
  }
};

// Entries of the fold are fetched U per lane at a time; the first batch of
// the next (side, k) is issued before the current transform so its latency
// hides behind the FFT.
template <int U> struct Batch {
  float v[U];
  uint32_t u[U];
};

// Past the segment's end a lane gets value 0 and its own first slot.  A
// batch wholly inside the segment (a wave-uniform test) is loaded without
// per-entry tests.
template <int G, int kU, typename E>
__device__ __forceinline__ void fetch(Batch<kU>& bt, const float* sa, const E* en, int ls,
                                      int lane, int first, uint32_t own_off) {
  if ((first + kU) * G <= ls) {
#pragma unroll
    for (int i = 0; i < kU; ++i) {
      const int it = lane + G * (first + i);
      bt.v[i] = sa[it];
      bt.u[i] = en[it];
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < kU; ++i) {
    const int it = lane + G * (first + i);
    if (it < ls) { bt.v[i] = sa[it]; bt.u[i] = en[it]; }
    else { bt.v[i] = 0.0f; bt.u[i] = own_off; }
  }
}

// Fold weight of entry u in row f1: omega_b^(f1 r) omega_R^(f1 q) with
// r = u mod C, q = u div C equals omega_b^(f1 j) * omega_16R^(f1 v) with
// j = u mod T (the owning thread) and v = u div T; the first factor is
// common to all slots of thread j and applied once per slot after the fold,
// the second comes from the block's 16R-entry table wf[v] = omega_16R^(f1 v).
//
// The fold adds in fixed point with LDS integer atomics (float LDS atomics
// are an order of magnitude slower, and integer sums do not depend on the
// order of the adds).  A slot gathers at most R buckets and |w| = 1, so with
// the column's max |value| cmax the slot sums stay below R cmax; values are
// scaled by 2^(30 - e) with R cmax < 2^e and converted to int32 by
// truncation toward zero, so each folded value loses less than one unit
// 2^(e - 30) <= 2 R cmax 2^-30 (frexp puts 2^e in (R cmax, 2 R cmax]).  The real and
// imaginary parts travel packed in one 64-bit add, im * 2^32 + re: the sum
// is exact modulo 2^64 and both 32-bit sums are recovered from it because
// each stays inside int32.
__device__ __forceinline__ unsigned long long pack2(int re, int im) {
  return (unsigned long long)(((long long)im << 32) + (long long)re);
}
// p = im * 2^32 + re with re signed: the high word is im - [re < 0].
__device__ __forceinline__ int2 unpack2(unsigned long long p) {
  const uint32_t lo = (uint32_t)p, hi = (uint32_t)(p >> 32);
  return make_int2((int)lo, (int)(hi + (lo >> 31)));
}

// omega_32^q = exp(-2 pi i q / 32) for q < 16 (cos, sin of q pi / 16)
constexpr float kW32[16][2] = {
    {1.0f, 0.0f}, {0.98078528040323043f, -0.19509032201612825f},
    {0.92387953251128674f, -0.38268343236508978f}, {0.83146961230254524f, -0.55557023301960218f},
    {0.70710678118654757f, -0.70710678118654746f}, {0.55557023301960229f, -0.83146961230254524f},
    {0.38268343236508984f, -0.92387953251128674f}, {0.19509032201612833f, -0.98078528040323043f},
    {0.0f, -1.0f}, {-0.19509032201612819f, -0.98078528040323043f},
    {-0.38268343236508973f, -0.92387953251128674f}, {-0.55557023301960196f, -0.83146961230254546f},
    {-0.70710678118654746f, -0.70710678118654757f}, {-0.83146961230254535f, -0.55557023301960218f},
    {-0.92387953251128674f, -0.38268343236508989f}, {-0.98078528040323043f, -0.19509032201612861f},
};

// Fold modes: the single row of R == 1 (unit weights), a weighted row f1
// in [1, R/2), and the row pair {0, R/2} (see below).
enum { kFoldRow0 = 0, kFoldRow = 1, kFoldPair = 2 };

// Row pair {0, R/2}.  Row 0 holds the spectrum at multiples of R and row R/2
// at odd multiples of R/2; both are the length-2C DFT of the real sequence
// p[r'] = sum of x[u] over u = r' (mod 2C), at even and odd frequencies.
// That DFT comes from one C-point complex FFT of z[s] = p[2s] + i p[2s+1]:
// with Z = FFT(z) and Zm[f] = Z[(C - f) mod C],
//   P[f]     = (Z[f] + conj Zm[f]) / 2 + omega_2C^f (Z[f] - conj Zm[f]) / (2i),
//   P[C]     = Re Z[0] - Im Z[0],
// and P[2C - f] = conj P[f].  Bucket u folds with weight 1 into slot
// s = (u mod 2C) div 2, real part for even u mod 2C and imaginary part for
// odd.  The layout stores, for each bucket, that slot's LDS offset and the
// parity of u (pair_entry), so the pair fold reads its target directly.
// Slot s belongs to thread s mod T, in general not in the wave of the
// entry, so this fold is bracketed by block barriers.

// The batch is folded in groups of 4 entries (the last group may be
// shorter): a group that lies wholly past the segment is skipped by a
// wave-uniform test; inside a group there is no branch, so the weight reads
// issue together.  Padding entries carry value 0 and an own slot of the
// wave.
template <int kU, int MODE, int kG>
__device__ __forceinline__ void fold_group(const Batch<kU>& bt, int g0, unsigned long long* Z,
                                           const float2* wf, float scale) {
  const int gn = kU - g0 < kG ? kU - g0 : kG;
  float2 w[kG];
  if constexpr (MODE == kFoldRow) {
#pragma unroll
    for (int i = 0; i < kG; ++i)
      if (i < gn) w[i] = at_byte(wf, bt.u[g0 + i] >> 16);
  }
#pragma unroll
  for (int i = 0; i < kG; ++i) {
    if (i >= gn) break;
    const uint32_t e = bt.u[g0 + i];
    const uint32_t off = e & 0xFFFFu;
    // |value * scale| < 2^30: float32 keeps 24 bits, so values near the top
    // have no fraction and truncation only touches the smallest ones
    const float sv = bt.v[g0 + i] * scale;
    if constexpr (MODE == kFoldRow0) {
      atomicAdd(&at_byte(Z, off), (unsigned long long)(long long)(int)sv);
    } else if constexpr (MODE == kFoldRow) {
      atomicAdd(&at_byte(Z, off), pack2((int)(sv * w[i].x), (int)(sv * w[i].y)));
    } else {
      // pair entry: the slot's byte offset, the real/imaginary choice in bit 0
      const unsigned long long add = (unsigned long long)(long long)(int)sv;
      atomicAdd(&at_byte(Z, e & ~7u), add << ((e & 1u) << 5));
    }
  }
}

template <int G, int kU, int MODE, int kG>
__device__ __forceinline__ void fold(const Batch<kU>& bt, unsigned long long* Z,
                                     const float2* wf, float scale, int ls, int first) {
#pragma unroll
  for (int g0 = 0; g0 < kU; g0 += kG) {
    if ((first + g0) * G >= ls) break;
    fold_group<kU, MODE, kG>(bt, g0, Z, wf, scale);
  }
}

// Entries g0 .. g0+3 (fewer in the last group) of batch `first` into the
// same positions of `bt`; `whole`: the batch lies wholly inside the segment.
template <int G, int kU, int kG, typename E>
__device__ __forceinline__ void fetch_group(Batch<kU>& bt, int g0, const float* sa,
                                            const E* en, int ls, int lane, int first,
                                            uint32_t own_off, bool whole) {
  const int gn = kU - g0 < kG ? kU - g0 : kG;
#pragma unroll
  for (int i = 0; i < kG; ++i) {
    if (i >= gn) break;
    const int it = lane + G * (first + g0 + i);
    if (whole || it < ls) { bt.v[g0 + i] = sa[it]; bt.u[g0 + i] = en[it]; }
    else { bt.v[g0 + i] = 0.0f; bt.u[g0 + i] = own_off; }
  }
}

// The whole segment, batch by batch; batch `a` (kU entries per lane) was
// fetched during the previous transform.  Callers raise the wave's priority
// for the fold and the next fetch: two waves share a SIMD, and a fold
// (latency-bound: weight reads, LDS atomics, global loads) then issues ahead
// of the other wave's transform (issue-bound) and overlaps with it, instead
// of waiting behind it.  While a batch is folded, each
// group's registers are refilled with the same group of the next batch
// right after the group is folded, so the next batch's loads are in flight
// behind the rest of the folding, with no second buffer.
template <int G, int kU, int MODE, int kG, typename E>
__device__ __forceinline__ void fold_all(Batch<kU>& a, unsigned long long* Z, const float2* wf,
                                         float scale, const float* sa, const E* en, int ls,
                                         int lane, uint32_t own_off) {
  for (int first = 0;; first += kU) {
    const int next = first + kU;
    if (next * G < ls) {
      // every group of this batch lies inside the segment
      const bool whole = (next + kU) * G <= ls;
#pragma unroll
      for (int g0 = 0; g0 < kU; g0 += kG) {
        fold_group<kU, MODE, kG>(a, g0, Z, wf, scale);
        fetch_group<G, kU, kG>(a, g0, sa, en, ls, lane, next, own_off, whole);
      }
    } else {
      fold<G, kU, MODE, kG>(a, Z, wf, scale, ls, first);
      break;
    }
  }
}

// One block per (repetition t, k-split ks): the row pair {0, R/2} (R > 1;
// see the fold modes above).  A kernel of its own, launched beside the row
// kernel, so that each keeps its own register allocation.
template <int L, int kG>
__global__ __launch_bounds__(FftShape<L>::T, 2) void k_fft_mac_pair(FftArgs a) {
  typedef FftShape<L> F;
  const int logical = blockIdx.x;
  const int ks = logical % a.KS;
  const int t = logical / a.KS;
  constexpr int C = F::C, T = F::T, G = F::G, kU = F::U;
  extern __shared__ float2 lds[];
  float2* P0 = lds;
  float2* P1 = lds + C;
  float2* tm = lds + 2 * C;
  const int j = threadIdx.x;
  const int lane = j % G, wv = j / G;
  const int R = a.R;
  const uint64_t bm = (uint64_t)(a.b - 1);
  const int kb = (int)((int64_t)a.m * ks / a.KS);
  const int ke = (int)((int64_t)a.m * (ks + 1) / a.KS);
  const float2 sj = a.tw[((uint64_t)j * (uint64_t)(R >> 1)) & bm];   // omega_2C^j
  const int jbase = sw(j);
  // last-stage twiddles omega_C^((j mod Ns) r), Ns = span(S-1)
  float2 tl[15];
  if constexpr (F::S >= 2) {
    constexpr int Ns = F::span(F::S - 1);
#pragma unroll
    for (int r = 1; r < 16; ++r)
      tl[r - 1] = a.tw[(int64_t)((j % Ns) * r) * (C / (16 * Ns)) * R];
  }
  // middle-stage twiddles omega_{16 Ns}^((j mod Ns) r), Ns = span(1):
  // registers at L = 12, the LDS table for the other row lengths
  float2 tm1[15];
  if constexpr (F::kRegMid) {
    constexpr int Ns = F::span(1);
#pragma unroll
    for (int r = 1; r < 16; ++r) tm1[r - 1] = a.tw[(int64_t)((j % Ns) * r) * (C / (16 * Ns)) * R];
  }
#pragma unroll
  for (int s = 1; s < F::S - 1 && !F::kRegMid; ++s) {
    const int Ns = F::span(s);
    for (int e = j; e < 15 * Ns; e += T) {
      const int r = e / Ns + 1, jm = e % Ns;
      tm[F::tmoff(s) + e] = a.tw[(int64_t)(jm * r) * (C / (16 * Ns)) * R];
    }
  }
  unsigned long long* Z = reinterpret_cast<unsigned long long*>(P0);
  // LDS position of the mirror frequency of j + 15 T when T is a multiple
  // of 256 (the swizzle then only touches the part below T)
  const int mirror_base = sw((T - j) & (T - 1)) + (j == 0 ? T : 0);
  // the first fold adds into other waves' slots: clear before the barrier
#pragma unroll
  for (int q = 0; q < 16; ++q) Z[own<T>(jbase, j, q)] = 0ull;
  __syncthreads();

  float2 acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = make_float2(0.f, 0.f);
  const float* sa0 = a.SA0 + (int64_t)t * a.m * a.Lrow0 + wv * a.Lcap0;
  const float* sa1 = a.SA1 + (int64_t)t * a.m * a.Lrow1 + wv * a.Lcap1;
  const uint16_t* en0 = a.entp0 + (int64_t)t * a.Lrow0 + wv * a.Lcap0;
  const uint16_t* en1 = a.entp1 + (int64_t)t * a.Lrow1 + wv * a.Lcap1;
  const int ls0 = a.lseg0[t], ls1 = a.lseg1[t];
  const float* cm0 = a.cmax0 + (int64_t)t * a.m;
  const float* cm1 = a.cmax1 + (int64_t)t * a.m;
  const uint32_t own_off = (uint32_t)jbase * 8u;   // a pair entry too (parity 0)
  Batch<kU> bt;
  if (kb < ke) fetch<G, kU>(bt, sa0 + (int64_t)kb * a.Lrow0, en0, ls0, lane, 0, own_off);
  const float2* wf = nullptr;   // unused by the pair fold
  float accn = 0.0f;   // 4 P_A[C] P_B[C] summed (thread 0's is used)
  for (int k = kb; k < ke; ++k) {
    float2 X[16];
    float xn = 0.0f;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const float* sa = side == 0 ? sa0 + (int64_t)k * a.Lrow0 : sa1 + (int64_t)k * a.Lrow1;
      const uint16_t* en = side == 0 ? en0 : en1;
      const int ls = side == 0 ? ls0 : ls1;
      // a slot of the pair gathers at most R/2 buckets: the bound of the
      // rows holds
      int ex;
      const float bound = (float)R * (side == 0 ? cm0[k] : cm1[k]);
      (void)frexpf(bound, &ex);
      const float scale = bound > 0.0f ? ldexpf(1.0f, 30 - ex) : 0.0f;
      const float inv = bound > 0.0f ? ldexpf(1.0f, ex - 30) : 0.0f;
      __builtin_amdgcn_s_setprio(1);
      fold_all<G, kU, kFoldPair, kG>(bt, Z, wf, scale, sa, en, ls, lane, own_off);
      if (side == 0) fetch<G, kU>(bt, sa1 + (int64_t)k * a.Lrow1, en1, ls1, lane, 0, own_off);
      else if (k + 1 < ke) fetch<G, kU>(bt, sa0 + (int64_t)(k + 1) * a.Lrow0, en0, ls0, lane, 0, own_off);
      __builtin_amdgcn_s_setprio(0);
      __syncthreads();   // every wave's adds are in
      float2 v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int2 zi = unpack2(Z[own<T>(jbase, j, q)]);
        v[q] = make_float2((float)zi.x * inv, (float)zi.y * inv);
      }
      Stage<L, 0>::template run<false>(v, P0, P1, tl, tm1, tm, j, make_float2(0.f, 0.f));
      // No thread touches this thread's own positions after the last
      // stage's barrier: clear the Z slots for the next fold and pass the
      // spectrum through P1 to the threads holding the mirror frequencies.
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        Z[own<T>(jbase, j, q)] = 0ull;
        P1[own<T>(jbase, j, q)] = v[q];
      }
      __syncthreads();
      const float nyq = 2.0f * (v[0].x - v[0].y);   // 2 P[C] at thread 0
      // the 16 twiddles below are loop-invariant; kept opaque so that they
      // are formed here rather than held in registers across the loop
      float2 sjk = sj;
      int mb = mirror_base;
      asm volatile("" : "+v"(sjk.x), "+v"(sjk.y), "+v"(mb));
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        float2 zm;
        if constexpr (T % 256 == 0) {
          // mirror of j + T q: (T - j) + T (15 - q) for j > 0 and
          // T (16 - q) mod C for j = 0, i.e. mb + T (15 - q), which wraps
          // to 0 only for j = q = 0
          zm = q == 0 ? P1[(mb + T * 15) & (C - 1)] : P1[mb + T * (15 - q)];
        } else {
          zm = P1[sw((C - (j + T * q)) & (C - 1))];
        }
        const float2 ev = make_float2(v[q].x + zm.x, v[q].y - zm.y);   // Z + conj Zm
        const float2 od = make_float2(v[q].y + zm.y, zm.x - v[q].x);   // -i (Z - conj Zm)
        // omega_2C^f = omega_2C^j omega_32^q
        const float2 w = cmul(sjk, make_float2(kW32[q][0], kW32[q][1]));
        const float2 p2 = cadd(ev, cmul(w, od));                         // 2 P[f]
        if (side == 0) {
          X[q] = p2;
        } else {
          acc[q].x = fmaf(X[q].x, p2.x, fmaf(-X[q].y, p2.y, acc[q].x));
          acc[q].y = fmaf(X[q].x, p2.y, fmaf(X[q].y, p2.x, acc[q].y));
        }
      }
      if (side == 0) xn = nyq;
      else accn = fmaf(xn, nyq, accn);
    }
  }
  // acc holds 4 sum P_A P_B at 2C-frequencies f = j + T q < C, accn at C.
  // Row 0 position g is frequency 2g and row R/2 position g is 2g + 1;
  // those at or above C are conjugates of 2C minus them.
  __syncthreads();   // the last mirror reads are done
#pragma unroll
  for (int q = 0; q < 16; ++q) P1[own<T>(jbase, j, q)] = acc[q];
  if (j == 0) P0[0] = make_float2(accn, 0.0f);
  __syncthreads();
  float2* out0 = a.Ppart + ((int64_t)t * a.KS + ks) * a.rows * C;
  float2* outh = out0 + (int64_t)(R >> 1) * C;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int g = j + T * q;
    float2 r0, rh;
    if (2 * g < C) r0 = P1[sw(2 * g)];
    else if (2 * g == C) r0 = P0[0];
    else r0 = cconj(P1[sw(2 * (C - g))]);
    if (2 * g + 1 < C) rh = P1[sw(2 * g + 1)];
    else rh = cconj(P1[sw(2 * (C - 1 - g) + 1)]);
    out0[g] = make_float2(0.25f * r0.x, 0.25f * r0.y);
    outh[g] = make_float2(0.25f * rh.x, 0.25f * rh.y);
  }
}

// nrow blocks per (repetition, k-split): rows f1 = roff .. roff + nrow - 1,
// i.e. 1 .. R/2 - 1 when R > 1 (the pair kernel computes rows 0 and R/2)
// and row 0 alone when R == 1.
template <int L, int kG, bool kRow0>
__global__ __launch_bounds__(FftShape<L>::T, 2) void k_fft_mac(FftArgs a) {
  typedef FftShape<L> F;
  constexpr int C = F::C, T = F::T, G = F::G, kU = F::U;
  extern __shared__ float2 lds[];
  float2* P0 = lds;
  float2* P1 = lds + C;
  float2* tm = lds + 2 * C;
  float2* wf = tm + F::NMID;         // omega_16R^(f1 v), v < 16 R
  static_assert(F::S <= 4, "at most two middle stages");

  // Tile order (t, ks, f1), row fastest.  Workgroups are dealt to the eight
  // XCDs in turn, so the rows of one (repetition, k-range), which read the
  // same sketches, run on different XCDs at about the same time.  Grouping
  // them on one XCD so that they share its L2 cuts the reads beyond L2
  // sixfold but makes this kernel 2.5-5 % slower at 4096-point rows.
  const int logical = blockIdx.x;
  const int f1 = logical % a.nrow + a.roff;
  const int tmp = logical / a.nrow;
  const int ks = tmp % a.KS;
  const int t = tmp / a.KS;
  const int j = threadIdx.x;
  const int lane = j % G, wv = j / G;
  const int R = a.R;
  const uint64_t bm = (uint64_t)(a.b - 1);
  const int kb = (int)((int64_t)a.m * ks / a.KS);
  const int ke = (int)((int64_t)a.m * (ks + 1) / a.KS);

  const int m16 = 16 * R - 1;
  for (int q = j; q < 16 * R; q += T) wf[q] = a.tw[(int64_t)((f1 * q) & m16) * T];
  const float2 sj = a.tw[((uint64_t)f1 * (uint64_t)j) & bm];   // omega_b^(f1 j)
  const int jbase = sw(j);
  // last-stage twiddles omega_C^((j mod Ns) r), Ns = span(S-1)
  float2 tl[15];
  if constexpr (F::S >= 2) {
    constexpr int Ns = F::span(F::S - 1);
#pragma unroll
    for (int r = 1; r < 16; ++r)
      tl[r - 1] = a.tw[(int64_t)((j % Ns) * r) * (C / (16 * Ns)) * R];
  }
  // middle-stage twiddles omega_{16 Ns}^((j mod Ns) r), Ns = span(1):
  // registers at L = 12, the LDS table for the other row lengths
  float2 tm1[15];
  if constexpr (F::kRegMid) {
    constexpr int Ns = F::span(1);
#pragma unroll
    for (int r = 1; r < 16; ++r) tm1[r - 1] = a.tw[(int64_t)((j % Ns) * r) * (C / (16 * Ns)) * R];
  }
#pragma unroll
  for (int s = 1; s < F::S - 1 && !F::kRegMid; ++s) {
    const int Ns = F::span(s);
    for (int e = j; e < 15 * Ns; e += T) {
      const int r = e / Ns + 1, jm = e % Ns;
      tm[F::tmoff(s) + e] = a.tw[(int64_t)(jm * r) * (C / (16 * Ns)) * R];
    }
  }
  __syncthreads();

  float2 acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = make_float2(0.f, 0.f);

  const float* sa0 = a.SA0 + (int64_t)t * a.m * a.Lrow0 + wv * a.Lcap0;
  const float* sa1 = a.SA1 + (int64_t)t * a.m * a.Lrow1 + wv * a.Lcap1;
  const uint32_t* en0 = a.ent0 + (int64_t)t * a.Lrow0 + wv * a.Lcap0;
  const uint32_t* en1 = a.ent1 + (int64_t)t * a.Lrow1 + wv * a.Lcap1;
  const int ls0 = a.lseg0[t], ls1 = a.lseg1[t];
  const float* cm0 = a.cmax0 + (int64_t)t * a.m;
  const float* cm1 = a.cmax1 + (int64_t)t * a.m;
  unsigned long long* Z = reinterpret_cast<unsigned long long*>(P0);

  const uint32_t own_off = (uint32_t)jbase * 8u;
  Batch<kU> bt;
  if (kb < ke) fetch<G, kU>(bt, sa0 + (int64_t)kb * a.Lrow0, en0, ls0, lane, 0, own_off);


  for (int k = kb; k < ke; ++k) {
    float2 X[16];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const float* sa = side == 0 ? sa0 + (int64_t)k * a.Lrow0 : sa1 + (int64_t)k * a.Lrow1;
      const uint32_t* en = side == 0 ? en0 : en1;
      const int ls = side == 0 ? ls0 : ls1;
      // fixed-point scale 2^(30 - e) with R * cmax < 2^e
      int ex;
      const float bound = (float)R * (side == 0 ? cm0[k] : cm1[k]);
      (void)frexpf(bound, &ex);
      const float scale = bound > 0.0f ? ldexpf(1.0f, 30 - ex) : 0.0f;
      const float inv = bound > 0.0f ? ldexpf(1.0f, ex - 30) : 0.0f;
      float2 v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) Z[own<T>(jbase, j, q)] = 0ull;
      __builtin_amdgcn_wave_barrier();
      // the fold and the fetch run at raised wave priority (see fold_all)
      __builtin_amdgcn_s_setprio(1);
      if constexpr (kRow0) fold_all<G, kU, kFoldRow0, kG>(bt, Z, wf, scale, sa, en, ls, lane, own_off);
      else fold_all<G, kU, kFoldRow, kG>(bt, Z, wf, scale, sa, en, ls, lane, own_off);
      // first batch of the next (side, k), in flight during the transform
      if (side == 0) fetch<G, kU>(bt, sa1 + (int64_t)k * a.Lrow1, en1, ls1, lane, 0, own_off);
      else if (k + 1 < ke) fetch<G, kU>(bt, sa0 + (int64_t)(k + 1) * a.Lrow0, en0, ls0, lane, 0, own_off);
      __builtin_amdgcn_s_setprio(0);
      __builtin_amdgcn_wave_barrier();
      // the slot factor omega_b^(f1 j) (1 in row 0) and the fixed-point unit
      // multiply every input of stage 0
      const float2 pre = !kRow0 ? make_float2(sj.x * inv, sj.y * inv) : make_float2(inv, 0.0f);
      if constexpr (!kRow0) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int2 zi = unpack2(Z[own<T>(jbase, j, q)]);
          v[q] = make_float2((float)zi.x, (float)zi.y);
        }
      } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int re = (int)(uint32_t)(Z[own<T>(jbase, j, q)] & 0xFFFFFFFFull);
          v[q] = make_float2((float)re, 0.0f);
        }
      }
      Stage<L, 0>::template run<true>(v, P0, P1, tl, tm1, tm, j, pre);
      if (side == 0) {
#pragma unroll
        for (int q = 0; q < 16; ++q) X[q] = v[q];
      } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          acc[q].x = fmaf(X[q].x, v[q].x, fmaf(-X[q].y, v[q].y, acc[q].x));
          acc[q].y = fmaf(X[q].x, v[q].y, fmaf(X[q].y, v[q].x, acc[q].y));
        }
      }
    }
  }
  float2* out = a.Ppart + (((int64_t)t * a.KS + ks) * a.rows + f1) * C;
#pragma unroll
  for (int q = 0; q < 16; ++q) out[j + T * q] = acc[q];
}

// The pair kernel has one block per (repetition, k-split), an eighth of the
// work at R = 16; alone it would leave most of the chip idle for its last
// blocks, so with `ov` it runs on the second stream beside the row kernel.
template <int L, int kG>
static hipError_t launch_LG(FftArgs a, const Geometry& g, hipStream_t s, const Overlap* ov) {
  typedef FftShape<L> F;
  const size_t lds = (size_t)(2 * F::C + F::NMID + 16 * a.R) * sizeof(float2);
  hipError_t e = hipSuccess;
  const bool fork = ov && g.R > 1;
  if (fork) {
    if ((e = hipEventRecord(ov->fork, s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(ov->aux, ov->fork, 0)) != hipSuccess) return e;
  }
  if (g.R > 1) {
    hipLaunchKernelGGL((k_fft_mac_pair<L, kG>), dim3(g.d * g.KS), dim3(F::T), lds, fork ? ov->aux : s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (fork && (e = hipEventRecord(ov->join, ov->aux)) != hipSuccess) return e;
  a.nrow = g.R > 1 ? g.R / 2 - 1 : 1;
  a.roff = g.R > 1 ? 1 : 0;
  if (a.nrow > 0) {
    const int nwg = g.d * g.KS * a.nrow;
    if (g.R > 1) hipLaunchKernelGGL((k_fft_mac<L, kG, false>), dim3(nwg), dim3(F::T), lds, s, a);
    else hipLaunchKernelGGL((k_fft_mac<L, 4, true>), dim3(nwg), dim3(F::T), lds, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (fork) e = hipStreamWaitEvent(s, ov->join, 0);
  return e;
}

// Fold group size: 8 entries when a wave's segment is expected to take
// well over one batch of U entries per lane (more refetched entries in
// flight per group then pay), else 4 (one batch, or a short second one,
// where groups of 8 would fold more padding).  Both measured at 4096-point
// rows.  The expected segment length is the expected number of non-empty
// buckets of the fuller side over the W segments of a repetition.
template <int L>
static hipError_t launch_L(FftArgs a, const Geometry& g, int64_t n_max, hipStream_t s, const Overlap* ov) {
  typedef FftShape<L> F;
  const double nb = (double)g.b * -std::expm1((double)n_max * std::log1p(-1.0 / (double)g.b));
  const bool several = nb / g.W > 1.5 * F::U * F::G;
  return several ? launch_LG<L, 8>(a, g, s, ov) : launch_LG<L, 4>(a, g, s, ov);
}

hipError_t launch_fft_mac(const Geometry& g, const SideDesc& sa, const SideDesc& sb,
                          const float2* tw32, float2* Ppart, hipStream_t s, const Overlap* ov) {
  FftArgs a;
  a.SA0 = sa.SA; a.SA1 = sb.SA;
  a.ent0 = sa.ent; a.ent1 = sb.ent;
  a.entp0 = sa.entp; a.entp1 = sb.entp;
  a.lseg0 = sa.lseg; a.lseg1 = sb.lseg;
  a.cmax0 = sa.colmax; a.cmax1 = sb.colmax;
  a.Lcap0 = sa.Lcap; a.Lcap1 = sb.Lcap; a.Lrow0 = sa.Lrow; a.Lrow1 = sb.Lrow;
  a.tw = tw32; a.Ppart = Ppart; a.b = g.b;
  a.R = g.R; a.rows = g.rows; a.d = g.d; a.m = g.m; a.KS = g.KS;
  a.nrow = 1; a.roff = 0;
  const int64_t n_max = std::max<int64_t>(sa.n, sb.n);
  switch (g.log2c) {
    case 4: return launch_L<4>(a, g, n_max, s, ov);
    case 5: return launch_L<5>(a, g, n_max, s, ov);
    case 6: return launch_L<6>(a, g, n_max, s, ov);
    case 7: return launch_L<7>(a, g, n_max, s, ov);
    case 8: return launch_L<8>(a, g, n_max, s, ov);
    case 9: return launch_L<9>(a, g, n_max, s, ov);
    case 10: return launch_L<10>(a, g, n_max, s, ov);
    case 11: return launch_L<11>(a, g, n_max, s, ov);
    case 12: return launch_L<12>(a, g, n_max, s, ov);
    case 13: return launch_L<13>(a, g, n_max, s, ov);
    default: return hipErrorInvalidValue;
  }
}

// Raise the dynamic LDS limit of every row length to 160 KB (done once per
// context, outside any graph capture).
hipError_t prepare_fft_mac() {
#define CMM_FNS(K, ...) \
  reinterpret_cast<const void*>(&K<4, __VA_ARGS__>), reinterpret_cast<const void*>(&K<5, __VA_ARGS__>), \
  reinterpret_cast<const void*>(&K<6, __VA_ARGS__>), reinterpret_cast<const void*>(&K<7, __VA_ARGS__>), \
  reinterpret_cast<const void*>(&K<8, __VA_ARGS__>), reinterpret_cast<const void*>(&K<9, __VA_ARGS__>), \
  reinterpret_cast<const void*>(&K<10, __VA_ARGS__>), reinterpret_cast<const void*>(&K<11, __VA_ARGS__>), \
  reinterpret_cast<const void*>(&K<12, __VA_ARGS__>), reinterpret_cast<const void*>(&K<13, __VA_ARGS__>)
  const void* fns[] = {CMM_FNS(k_fft_mac, 4, false), CMM_FNS(k_fft_mac, 4, true), CMM_FNS(k_fft_mac, 8, false),
                       CMM_FNS(k_fft_mac_pair, 4), CMM_FNS(k_fft_mac_pair, 8)};
#undef CMM_FNS
  for (const void* f : fns) {
    // the stage-write addressing needs the dynamic array at address 0
    hipFuncAttributes at;
    hipError_t e = hipFuncGetAttributes(&at, f);
    if (e != hipSuccess) return e;
    if (at.sharedSizeBytes != 0) return hipErrorInvalidDeviceFunction;
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace cmm

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
// block owns one (repetition t, row f1, range of k): for each k it folds the
// column sketch of A and the row sketch of B, transforms both, multiplies
// them bin by bin and adds the products into float64 accumulators held in
// registers.  The n-by-b spectra are never stored.
//
// FFT: Stockham autosort, T = C/16 threads with 16 complex values each; the
// first stage has radix 2^(log2 C mod 4) (if not zero) and the rest radix
// 16, with LDS exchanges (padded by one element per 16) between stages.
// Thread j starts with slots j + T v and ends with frequencies j + T v.
//
// Fold: the slots of thread j are exactly the buckets u with u mod T = j.
// The bucket layout hands every wave only buckets whose slots belong to its
// own lanes, so a wave's LDS float atomics never race with another wave's
// and the wave's in-order LDS queue makes the fold's summation order fixed.
#include "cmm_internal.h"
#include "cmm_dft.h"

namespace cmm {

__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }

struct FftArgs {
  const float* SA0; const float* SA1;
  const uint32_t* ent0; const uint32_t* ent1;
  const int32_t* lseg0; const int32_t* lseg1;
  int Lcap0, Lcap1, Lrow0, Lrow1;
  const float2* tw;        // omega_b^x for x < b
  double2* Ppart;
  int64_t b;
  int R, rows, d, m, KS, nwg, remap;
};

constexpr int ipow16(int e) { return e <= 0 ? 1 : 16 * ipow16(e - 1); }

template <int L> struct FftShape {
  static constexpr int C = 1 << L;
  static constexpr int T = C / 16;
  static constexpr int E = L % 4;
  static constexpr int S = L / 4 + (E ? 1 : 0);
  static constexpr int G = T < 64 ? T : 64;
  static constexpr int BUF = C + C / 16;
  static constexpr int NTW = S > 1 ? S - 1 : 1;
  // span of stage s (product of the earlier radices)
  static constexpr int span(int s) { return s == 0 ? 1 : (E ? (1 << E) : 16) * ipow16(s - 1); }
  static constexpr int radix(int s) { return (s == 0 && E) ? (1 << E) : 16; }
};

template <int L, int s> struct Stage {
  static __device__ __forceinline__ void run(float2* v, float2* P0, float2* P1,
                                             const float2 (&tw)[FftShape<L>::NTW][15], int j) {
    typedef FftShape<L> F;
    constexpr int Rs = F::radix(s);
    constexpr int BPT = 16 / Rs;
    constexpr int Ns = F::span(s);
    float2* bin = (s % 2 == 0) ? P0 : P1;
    float2* bout = (s % 2 == 0) ? P1 : P0;
    if constexpr (s > 0) {
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = bin[pidx(j + F::T * q)];
#pragma unroll
      for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], tw[s - 1][r - 1]);
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
    if constexpr (s < F::S - 1) {
      if constexpr (s == 0 && F::S % 2 == 0) __syncthreads();
#pragma unroll
      for (int mi = 0; mi < BPT; ++mi) {
        const int jb = j + F::T * mi;
        const int base = (jb / Ns) * Ns * Rs + (jb % Ns);
#pragma unroll
        for (int r = 0; r < Rs; ++r) bout[pidx(base + r * Ns)] = v[mi + r * BPT];
      }
      __syncthreads();
      Stage<L, s + 1>::run(v, P0, P1, tw, j);
    }
  }
};

template <int L>
__global__ __launch_bounds__(FftShape<L>::T) void k_fft_mac(FftArgs a) {
  typedef FftShape<L> F;
  constexpr int C = F::C, T = F::T, G = F::G;
  extern __shared__ float2 lds[];
  float2* P0 = lds;
  float2* P1 = lds + F::BUF;
  float2* wr = lds + 2 * F::BUF;

  const int bid = blockIdx.x;
  const int logical = a.remap ? (bid & 7) * (a.nwg >> 3) + (bid >> 3) : bid;
  const int f1 = logical % a.rows;
  const int tmp = logical / a.rows;
  const int ks = tmp % a.KS;
  const int t = tmp / a.KS;
  const int j = threadIdx.x;
  const int lane = j % G, wv = j / G;
  const int R = a.R;
  const uint64_t bm = (uint64_t)(a.b - 1);
  const int kb = (int)((int64_t)a.m * ks / a.KS);
  const int ke = (int)((int64_t)a.m * (ks + 1) / a.KS);

  for (int q = j; q < R; q += T) wr[q] = a.tw[(int64_t)q * C];
  float2 st[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) st[q] = a.tw[((uint64_t)f1 * (uint64_t)(j + T * q)) & bm];
  float2 tw[F::NTW][15];
#pragma unroll
  for (int s = 1; s < F::S; ++s) {
    const int Ns = F::span(s);
#pragma unroll
    for (int r = 1; r < 16; ++r)
      tw[s - 1][r - 1] = a.tw[(int64_t)((j % Ns) * r) * (C / (16 * Ns)) * R];
  }
  __syncthreads();

  double2 acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = make_double2(0.0, 0.0);
  const bool realw = (f1 == 0) || (2 * f1 == R);

  for (int k = kb; k < ke; ++k) {
    float2 X[16];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const float* sa = (side == 0 ? a.SA0 : a.SA1) +
                        ((int64_t)t * a.m + k) * (side == 0 ? a.Lrow0 : a.Lrow1) +
                        wv * (side == 0 ? a.Lcap0 : a.Lcap1);
      const uint32_t* en = (side == 0 ? a.ent0 : a.ent1) +
                           (int64_t)t * (side == 0 ? a.Lrow0 : a.Lrow1) +
                           wv * (side == 0 ? a.Lcap0 : a.Lcap1);
      const int ls = (side == 0 ? a.lseg0 : a.lseg1)[t];
      float2 v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) P0[pidx(j + T * q)] = make_float2(0.f, 0.f);
      __builtin_amdgcn_wave_barrier();
      if (realw) {
        for (int it = lane; it < ls; it += G) {
          float val = sa[it];
          const uint32_t u = en[it] & 0x7FFFFFFFu;
          if (f1 != 0 && ((u >> L) & 1u)) val = -val;
          atomicAdd(&P0[pidx((int)(u & (C - 1)))].x, val);
        }
      } else {
        for (int it = lane; it < ls; it += G) {
          const float val = sa[it];
          const uint32_t u = en[it] & 0x7FFFFFFFu;
          const float2 w = wr[(f1 * (int)(u >> L)) & (R - 1)];
          float2* dst = &P0[pidx((int)(u & (C - 1)))];
          atomicAdd(&dst->x, val * w.x);
          atomicAdd(&dst->y, val * w.y);
        }
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = P0[pidx(j + T * q)];
      if (f1 != 0) {
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = cmul(v[q], st[q]);
      }
      Stage<L, 0>::run(v, P0, P1, tw, j);
      if (side == 0) {
#pragma unroll
        for (int q = 0; q < 16; ++q) X[q] = v[q];
      } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          acc[q].x += (double)(X[q].x * v[q].x - X[q].y * v[q].y);
          acc[q].y += (double)(X[q].x * v[q].y + X[q].y * v[q].x);
        }
      }
    }
  }
  double2* out = a.Ppart + (((int64_t)t * a.KS + ks) * a.rows + f1) * C;
#pragma unroll
  for (int q = 0; q < 16; ++q) out[j + T * q] = acc[q];
}

template <int L>
static hipError_t launch_L(const FftArgs& a, hipStream_t s) {
  typedef FftShape<L> F;
  const size_t lds = (size_t)(2 * F::BUF + a.R) * sizeof(float2);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_mac<L>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_fft_mac<L>, dim3(a.nwg), dim3(F::T), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_fft_mac(const Geometry& g, const SideDesc& sa, const SideDesc& sb,
                          const float2* tw32, double2* Ppart, hipStream_t s) {
  FftArgs a;
  a.SA0 = sa.SA; a.SA1 = sb.SA;
  a.ent0 = sa.ent; a.ent1 = sb.ent;
  a.lseg0 = sa.lseg; a.lseg1 = sb.lseg;
  a.Lcap0 = sa.Lcap; a.Lcap1 = sb.Lcap; a.Lrow0 = sa.Lrow; a.Lrow1 = sb.Lrow;
  a.tw = tw32; a.Ppart = Ppart; a.b = g.b;
  a.R = g.R; a.rows = g.rows; a.d = g.d; a.m = g.m; a.KS = g.KS;
  a.nwg = g.d * g.KS * g.rows;
  a.remap = (a.nwg % 8 == 0) ? 1 : 0;
  switch (g.log2c) {
    case 4: return launch_L<4>(a, s);
    case 5: return launch_L<5>(a, s);
    case 6: return launch_L<6>(a, s);
    case 7: return launch_L<7>(a, s);
    case 8: return launch_L<8>(a, s);
    case 9: return launch_L<9>(a, s);
    case 10: return launch_L<10>(a, s);
    case 11: return launch_L<11>(a, s);
    case 12: return launch_L<12>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cmm

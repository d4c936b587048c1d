// Small in-register DFTs (natural order in and out, forward sign
// exp(-2 pi i n k / R)) for float2 and double2.  R = 16 and R = 8 are split
// Cooley-Tukey style into 4x4 and 2x4 with the inner twiddles
// exp(-2 pi i n1 k2 / R) applied between the layers.
#pragma once

#include <hip/hip_runtime.h>

namespace cmm {

template <typename V> struct Scal;
template <> struct Scal<float2> { typedef float T; };
template <> struct Scal<double2> { typedef double T; };

template <typename V> __host__ __device__ __forceinline__ V cx(typename Scal<V>::T a, typename Scal<V>::T b) {
  V r; r.x = a; r.y = b; return r;
}
template <typename V> __host__ __device__ __forceinline__ V cadd(V a, V b) { return cx<V>(a.x + b.x, a.y + b.y); }
template <typename V> __host__ __device__ __forceinline__ V csub(V a, V b) { return cx<V>(a.x - b.x, a.y - b.y); }
template <typename V> __host__ __device__ __forceinline__ V cmul(V a, V b) {
  return cx<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename V> __host__ __device__ __forceinline__ V cconj(V a) { return cx<V>(a.x, -a.y); }
// -i * a
template <typename V> __host__ __device__ __forceinline__ V cmul_mi(V a) { return cx<V>(a.y, -a.x); }

template <typename V> __host__ __device__ __forceinline__ void dft2(V& a, V& b) {
  V t = a; a = cadd(t, b); b = csub(t, b);
}

template <typename V> __host__ __device__ __forceinline__ void dft4(V& x0, V& x1, V& x2, V& x3) {
  V t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3), t3 = cmul_mi(csub(x1, x3));
  x0 = cadd(t0, t2); x2 = csub(t0, t2); x1 = cadd(t1, t3); x3 = csub(t1, t3);
}

// cos/sin of 2 pi k / 16
#define CMM_C1 0.92387953251128675613
#define CMM_S1 0.38268343236508977173
#define CMM_R2 0.70710678118654752440

// x[n], n = n1 + 2 n2 -> y[k2 + 4 k1]
template <typename V> __host__ __device__ __forceinline__ void dft8(V* x) {
  typedef typename Scal<V>::T S;
  dft4(x[0], x[2], x[4], x[6]);
  dft4(x[1], x[3], x[5], x[7]);
  // z[1][k2] *= w8^k2
  x[3] = cmul(x[3], cx<V>((S)CMM_R2, (S)-CMM_R2));
  x[5] = cmul_mi(x[5]);
  x[7] = cmul(x[7], cx<V>((S)-CMM_R2, (S)-CMM_R2));
  V y[8];
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    V a = x[2 * k2], b = x[2 * k2 + 1];
    y[k2] = cadd(a, b);
    y[k2 + 4] = csub(a, b);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = y[k];
}

// x[n], n = n1 + 4 n2 -> y[k2 + 4 k1]
template <typename V> __host__ __device__ __forceinline__ void dft16(V* x) {
  typedef typename Scal<V>::T S;
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) dft4(x[n1], x[n1 + 4], x[n1 + 8], x[n1 + 12]);
  // now x[n1 + 4 k2] = z[n1][k2]; twiddle by w16^(n1 k2)
  const V w1 = cx<V>((S)CMM_C1, (S)-CMM_S1), w2 = cx<V>((S)CMM_R2, (S)-CMM_R2),
          w3 = cx<V>((S)CMM_S1, (S)-CMM_C1), w6 = cx<V>((S)-CMM_R2, (S)-CMM_R2),
          w9 = cx<V>((S)-CMM_C1, (S)CMM_S1);
  x[5] = cmul(x[5], w1);  x[9] = cmul(x[9], w2);  x[13] = cmul(x[13], w3);
  x[6] = cmul(x[6], w2);  x[10] = cmul_mi(x[10]); x[14] = cmul(x[14], w6);
  x[7] = cmul(x[7], w3);  x[11] = cmul(x[11], w6); x[15] = cmul(x[15], w9);
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) dft4(x[4 * k2], x[4 * k2 + 1], x[4 * k2 + 2], x[4 * k2 + 3]);
  // x[4 k2 + k1] = y[k2 + 4 k1]
  V y[16];
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2)
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) y[k2 + 4 * k1] = x[4 * k2 + k1];
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = y[k];
}

// Fused forms for the radix-16 stages that multiply their inputs first.  A
// product u q that enters a butterfly is folded into it: a = p + u q costs
// four fused multiply-adds, and the other output p - u q is taken as 2 p - a
// (two more), where a separate product and two additions would take eight.
// The second output carries the rounding error of a, an error of the same
// size as the one of the product it replaces.

// p + u q
template <typename V> __host__ __device__ __forceinline__ V cfma(V p, V u, V q) {
  return cx<V>(fma(u.x, q.x, fma(-u.y, q.y, p.x)), fma(u.x, q.y, fma(u.y, q.x, p.y)));
}
// 2 p - a
template <typename V> __host__ __device__ __forceinline__ V ctwice_minus(V p, V a) {
  typedef typename Scal<V>::T S;
  return cx<V>(fma((S)2, p.x, -a.x), fma((S)2, p.y, -a.y));
}

// dft4 of (x0, u1 x1, u2 x2, u3 x3)
template <typename V>
__host__ __device__ __forceinline__ void dft4_tw(V& x0, V& x1, V& x2, V& x3, V u1, V u2, V u3) {
  const V a = cfma(x0, u2, x2), b = ctwice_minus(x0, a);
  const V c1 = cmul(x1, u1);
  const V c = cfma(c1, u3, x3), d = cmul_mi(ctwice_minus(c1, c));
  x0 = cadd(a, c); x2 = csub(a, c); x1 = cadd(b, d); x3 = csub(b, d);
}

// Second layer of dft16 with the inner twiddles w16^(n1 k2) folded in, then
// the output order y[k2 + 4 k1] (see dft16).
template <typename V> __host__ __device__ __forceinline__ void dft16_layer2(V* x) {
  typedef typename Scal<V>::T S;
  const V w1 = cx<V>((S)CMM_C1, (S)-CMM_S1), w2 = cx<V>((S)CMM_R2, (S)-CMM_R2),
          w3 = cx<V>((S)CMM_S1, (S)-CMM_C1), w6 = cx<V>((S)-CMM_R2, (S)-CMM_R2),
          w9 = cx<V>((S)-CMM_C1, (S)CMM_S1);
  dft4(x[0], x[1], x[2], x[3]);
  dft4_tw(x[4], x[5], x[6], x[7], w1, w2, w3);
  {
    // k2 = 2: twiddles 1, w2, -i, w6
    const V m = cmul_mi(x[10]);
    const V a = cadd(x[8], m), b = csub(x[8], m);
    const V c1 = cmul(x[9], w2);
    const V c = cfma(c1, w6, x[11]), d = cmul_mi(ctwice_minus(c1, c));
    x[8] = cadd(a, c); x[10] = csub(a, c); x[9] = cadd(b, d); x[11] = csub(b, d);
  }
  dft4_tw(x[12], x[13], x[14], x[15], w3, w6, w9);
  V y[16];
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2)
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) y[k2 + 4 * k1] = x[4 * k2 + k1];
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = y[k];
}

// dft16 of (x[0], u[0] x[1], ..., u[14] x[15])
template <typename V> __host__ __device__ __forceinline__ void dft16_tw(V* x, const V (&u)[15]) {
  dft4_tw(x[0], x[4], x[8], x[12], u[3], u[7], u[11]);
#pragma unroll
  for (int n1 = 1; n1 < 4; ++n1) {
    x[n1] = cmul(x[n1], u[n1 - 1]);
    dft4_tw(x[n1], x[n1 + 4], x[n1 + 8], x[n1 + 12], u[n1 + 3], u[n1 + 7], u[n1 + 11]);
  }
  dft16_layer2(x);
}

// dft16 of (s x[0], ..., s x[15])
template <typename V> __host__ __device__ __forceinline__ void dft16_scaled(V* x, V s) {
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    x[n1] = cmul(x[n1], s);
    dft4_tw(x[n1], x[n1 + 4], x[n1 + 8], x[n1 + 12], s, s, s);
  }
  dft16_layer2(x);
}

template <int R, typename V> __host__ __device__ __forceinline__ void dft(V* x) {
  if constexpr (R == 2) dft2(x[0], x[1]);
  else if constexpr (R == 4) dft4(x[0], x[1], x[2], x[3]);
  else if constexpr (R == 8) dft8(x);
  else dft16(x);
}

}  // namespace cmm

// Host build of the radix-16 helpers of cmm_dft.h (plain, with input
// twiddles folded into the butterflies, with a common input factor), for
// the CPU test test_dft_host.py: reads N cases of 16 complex inputs, 15
// twiddles and one factor (float32) from stdin, writes the three transforms
// of every case (float32) to stdout.
#include "cmm_dft.h"

#include <cstdio>
#include <vector>

int main() {
  int n = 0;
  if (std::fread(&n, sizeof(int), 1, stdin) != 1 || n <= 0) return 2;
  std::vector<float> in((size_t)n * (32 + 30 + 2));
  if (std::fread(in.data(), sizeof(float), in.size(), stdin) != in.size()) return 2;
  std::vector<float> out((size_t)n * 96);
  for (int c = 0; c < n; ++c) {
    const float* p = in.data() + (size_t)c * 64;
    float2 x[16], y[16], z[16], u[15];
    for (int k = 0; k < 16; ++k) x[k] = y[k] = z[k] = make_float2(p[2 * k], p[2 * k + 1]);
    for (int k = 0; k < 15; ++k) u[k] = make_float2(p[32 + 2 * k], p[33 + 2 * k]);
    const float2 s = make_float2(p[62], p[63]);
    cmm::dft<16>(x);
    cmm::dft16_tw(y, u);
    cmm::dft16_scaled(z, s);
    float* o = out.data() + (size_t)c * 96;
    for (int k = 0; k < 16; ++k) {
      o[2 * k] = x[k].x; o[2 * k + 1] = x[k].y;
      o[32 + 2 * k] = y[k].x; o[33 + 2 * k] = y[k].y;
      o[64 + 2 * k] = z[k].x; o[65 + 2 * k] = z[k].y;
    }
  }
  return std::fwrite(out.data(), sizeof(float), out.size(), stdout) == out.size() ? 0 : 3;
}

// C interface of the cmm library: argument checking, device memory,
// ordering of the kernels of one sketch product on the context stream.
#include "cmm.h"
#include "cmm_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

namespace {

constexpr uint32_t kCtxMagic = 0xC3A70001u;
constexpr uint32_t kSketchMagic = 0xC3A75001u;
constexpr uint32_t kDeadMagic = 0xDEADDEADu;

struct Pending {
  std::string name;
  hipEvent_t a, b;
};

}  // namespace

struct cmm_ctx {
  uint32_t magic = kCtxMagic;
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  std::multimap<size_t, void*> free_blocks;
  std::map<void*, size_t> sizes;
  std::map<int64_t, std::pair<double2*, float2*>> twiddles;
  bool prof = false;
  std::vector<Pending> pending;
  std::map<std::string, std::pair<double, int64_t>> prof_acc;
  uint32_t* pinned_u32 = nullptr;   // small pinned host scratch
};

struct cmm_sketch {
  uint32_t magic = kSketchMagic;
  cmm_ctx* ctx = nullptr;
  int64_t n1 = 0, m = 0, n3 = 0, b = 0;
  int d = 0;
  int log2b = 0;
  bool has_params = false;
  std::vector<uint64_t> params;   // d * 8
  int32_t* hs1 = nullptr;
  int32_t* hs2 = nullptr;
  double* c64 = nullptr;
  float* c32 = nullptr;
};

namespace {

int fail(cmm_ctx* c, int code, const std::string& msg) {
  if (c) c->last_error = msg;
  return code;
}

#define CMM_HIP(ctx, expr)                                                          \
  do {                                                                              \
    hipError_t e__ = (expr);                                                        \
    if (e__ != hipSuccess)                                                          \
      return fail((ctx), CMM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e__)); \
  } while (0)

bool valid_ctx(const cmm_ctx* c) { return c && c->magic == kCtxMagic; }
bool valid_sketch(const cmm_sketch* s) { return s && s->magic == kSketchMagic && valid_ctx(s->ctx); }

// ---- caching device allocator (stream-ordered reuse on the context stream)
void* dalloc(cmm_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 4095) & ~(size_t)4095;
  auto it = c->free_blocks.lower_bound(bytes);
  if (it != c->free_blocks.end() && it->first <= bytes * 2) {
    void* p = it->second;
    c->free_blocks.erase(it);
    return p;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    // give cached blocks back and retry once
    hipStreamSynchronize(c->stream);
    for (auto& kv : c->free_blocks) { c->sizes.erase(kv.second); hipFree(kv.second); }
    c->free_blocks.clear();
    if (hipMalloc(&p, bytes) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
  }
  c->sizes[p] = bytes;
  return p;
}

void dfree(cmm_ctx* c, void* p) {
  if (!p) return;
  auto it = c->sizes.find(p);
  if (it == c->sizes.end()) return;
  c->free_blocks.emplace(it->second, p);
}

struct Scope {
  cmm_ctx* c;
  const char* name;
  hipEvent_t a = nullptr, b = nullptr;
  Scope(cmm_ctx* cc, const char* nm) : c(cc), name(nm) {
    if (c->prof && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
      hipEventRecord(a, c->stream);
    else { a = b = nullptr; }
  }
  ~Scope() {
    if (a && b) {
      hipEventRecord(b, c->stream);
      c->pending.push_back({name, a, b});
    }
  }
};

void drain_profile(cmm_ctx* c) {
  hipStreamSynchronize(c->stream);
  for (auto& p : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      auto& acc = c->prof_acc[p.name];
      acc.first += ms;
      acc.second += 1;
    }
    hipEventDestroy(p.a);
    hipEventDestroy(p.b);
  }
  c->pending.clear();
}

// SplitMix64 (Steele, Lea, Flood 2014): output k of seed s mixes s + k*gamma.
uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void params_from_seed(uint64_t seed, int d, std::vector<uint64_t>& out) {
  out.resize((size_t)d * 8);
  for (int t = 0; t < d; ++t)
    for (int f = 0; f < 4; ++f) {
      uint64_t za = splitmix64_at(seed, (uint64_t)(8 * t + 2 * f + 1));
      uint64_t zc = splitmix64_at(seed, (uint64_t)(8 * t + 2 * f + 2));
      out[(size_t)t * 8 + 2 * f] = 1 + za % (CMM_P61 - 1);
      out[(size_t)t * 8 + 2 * f + 1] = zc % CMM_P61;
    }
}

int ilog2(int64_t v) { int l = 0; while ((int64_t(1) << l) < v) ++l; return l; }
bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int get_twiddles(cmm_ctx* c, int64_t b, double2** t64, float2** t32) {
  auto it = c->twiddles.find(b);
  if (it != c->twiddles.end()) { *t64 = it->second.first; *t32 = it->second.second; return CMM_OK; }
  double2* a = nullptr; float2* f = nullptr;
  CMM_HIP(c, hipMalloc(&a, sizeof(double2) * b));
  CMM_HIP(c, hipMalloc(&f, sizeof(float2) * b));
  CMM_HIP(c, cmm::launch_twiddles(a, f, b, c->stream));
  c->twiddles[b] = {a, f};
  *t64 = a; *t32 = f;
  return CMM_OK;
}

cmm::Geometry make_geometry(int64_t b, int d, int64_t m) {
  cmm::Geometry g;
  g.b = b; g.log2b = ilog2(b); g.d = d; g.m = (int)m;
  // FFT row length: 4096 measured fastest on the b = 2^16 covariance product;
  // 8192 (fewer rows, one block per CU) is kept for tuning (CMM_LOG2C).
  int lc = 12;
  if (const char* ev = std::getenv("CMM_LOG2C")) lc = std::max(4, std::min(cmm::kMaxLog2C, std::atoi(ev)));
  g.log2c = std::min(g.log2b, lc);
  const int C = 1 << g.log2c;
  g.T = C / 16;
  g.G = std::min(g.T, 64);
  g.W = g.T / g.G;
  g.R = (int)(b / C);
  g.rows = g.R > 1 ? g.R / 2 + 1 : 1;
  const int64_t base = (int64_t)d * g.rows;
  int64_t ks = std::max<int64_t>(1, (2048 + base - 1) / base);
  ks = std::max<int64_t>(ks, (m + cmm::kMaxKPerBlock - 1) / cmm::kMaxKPerBlock);
  ks = std::min<int64_t>(ks, m);
  while (ks < m && (base * ks) % 8 != 0) ++ks;
  g.KS = (int)std::max<int64_t>(1, ks);
  return g;
}

// Upper bound on the non-empty buckets of one layout segment.
int layout_cap(int64_t n, int64_t b, int W, bool safe) {
  const int64_t hard = std::min<int64_t>(n, b / W);
  if (safe) return (int)((hard + 63) & ~63LL);
  const double nb = (double)b * (1.0 - std::exp((double)n * std::log1p(-1.0 / (double)b)));
  const double mu = nb / W;
  int64_t cap = (int64_t)std::ceil(mu + 8.0 * std::sqrt(mu) + 64.0);
  cap = std::min<int64_t>(cap, hard);
  return (int)((cap + 63) & ~63LL);
}

struct Work {
  cmm_ctx* c;
  std::vector<void*> blocks;
  explicit Work(cmm_ctx* cc) : c(cc) {}
  template <typename T> T* get(size_t count) {
    void* p = dalloc(c, count * sizeof(T));
    if (p) blocks.push_back(p);
    return (T*)p;
  }
  ~Work() { for (void* p : blocks) dfree(c, p); }
};

int check_operands(cmm_ctx* c, const void* A, int64_t lda, const void* B, int64_t ldb, int64_t n1,
                   int64_t m, int64_t n3, int32_t dtype, int64_t b, int32_t d) {
  if (!A || !B) return fail(c, CMM_EINVAL, "A and B must be device pointers");
  if (n1 <= 0 || m <= 0 || n3 <= 0) return fail(c, CMM_EINVAL, "n1, m, n3 must be positive");
  if (n1 > (1 << 29) || n3 > (1 << 29) || m > (1 << 30))
    return fail(c, CMM_EUNSUPPORTED, "dimensions too large");
  if (lda < n1 || ldb < n3) return fail(c, CMM_EINVAL, "lda < n1 or ldb < n3");
  if (dtype < CMM_F32 || dtype > CMM_FP8_E4M3) return fail(c, CMM_EINVAL, "unknown dtype");
  if (!is_pow2(b) || b < 16 || b > (1 << 20)) return fail(c, CMM_EINVAL, "b must be a power of two in [16, 2^20]");
  if (d < 1 || d > 63) return fail(c, CMM_EINVAL, "d must be in [1, 63]");
  if (std::max(n1, n3) * (int64_t)sizeof(float) > 96 * 1024)
    return fail(c, CMM_EUNSUPPORTED, "hashed dimension above 24576 (count-sketch row staging)");
  return CMM_OK;
}

int run_product(cmm_ctx* c, cmm_sketch* sk, const void* A, int64_t lda, const void* B, int64_t ldb,
                int32_t dtype, const float* scaleA, const float* scaleB, uint32_t flags,
                bool safe_layout, bool* overflowed) {
  hipStream_t s = c->stream;
  cmm::Geometry g = make_geometry(sk->b, sk->d, sk->m);
  const int C = 1 << g.log2c;
  Work w(c);
  cmm::SideDesc side[2];
  const int64_t nn[2] = {sk->n1, sk->n3};
  const void* X[2] = {A, B};
  const int64_t ld[2] = {lda, ldb};
  const float* sc[2] = {scaleA, scaleB};
  int32_t* hsv[2] = {sk->hs1, sk->hs2};
  const bool async = flags & CMM_ASYNC;
  for (int q = 0; q < 2; ++q) {
    cmm::SideDesc& sd = side[q];
    sd.X = X[q]; sd.ld = ld[q]; sd.scale = sc[q]; sd.n = (int)nn[q];
    sd.hs = hsv[q];
    sd.Lcap = layout_cap(nn[q], g.b, g.W, safe_layout || async);
    sd.Lrow = g.W * sd.Lcap;
    sd.cnt = w.get<int32_t>((size_t)g.d * g.b);
    sd.pos = w.get<int32_t>((size_t)g.d * g.b);
    sd.ent = w.get<uint32_t>((size_t)g.d * sd.Lrow);
    sd.tab = w.get<uint32_t>((size_t)g.d * sd.Lrow);
    sd.cntp = w.get<int32_t>((size_t)g.d * sd.Lrow);
    sd.moff = w.get<int32_t>((size_t)g.d * sd.Lrow);
    sd.fill = w.get<int32_t>((size_t)g.d * sd.Lrow);
    sd.perm = w.get<int32_t>((size_t)g.d * sd.n);
    sd.segcount = w.get<int32_t>((size_t)g.d * g.W);
    sd.lseg = w.get<int32_t>((size_t)g.d);
    sd.SA = w.get<float>((size_t)g.d * g.m * sd.Lrow);
    sd.colmax = w.get<float>((size_t)g.d * g.m);
    if (!sd.colmax || !sd.cnt || !sd.pos || !sd.ent || !sd.tab || !sd.cntp || !sd.moff || !sd.fill || !sd.perm ||
        !sd.segcount || !sd.lseg || !sd.SA)
      return fail(c, CMM_ENOMEM, "workspace allocation failed");
  }
  float2* Ppart = w.get<float2>((size_t)g.d * g.KS * g.rows * C);
  double2* work0 = w.get<double2>((size_t)g.d * g.b);
  double2* work1 = w.get<double2>((size_t)g.d * g.b);
  int32_t* oflow = w.get<int32_t>(1);
  uint64_t* pdev = sk->has_params ? w.get<uint64_t>((size_t)g.d * 8) : nullptr;
  if (!Ppart || !work0 || !work1 || !oflow || (sk->has_params && !pdev))
    return fail(c, CMM_ENOMEM, "workspace allocation failed");
  double2* tw64; float2* tw32;
  int rc = get_twiddles(c, g.b, &tw64, &tw32);
  if (rc) return rc;

  CMM_HIP(c, cmm::launch_fill_i32(oflow, 1, 0, s));
  {
    Scope sc_(c, "hash");
    if (sk->has_params) {
      CMM_HIP(c, hipMemcpyAsync(pdev, sk->params.data(), sizeof(uint64_t) * g.d * 8,
                                hipMemcpyHostToDevice, s));
      for (int q = 0; q < 2; ++q) CMM_HIP(c, cmm::launch_hash(pdev, q, g, side[q], s));
    }
    for (int q = 0; q < 2; ++q) CMM_HIP(c, cmm::launch_count(g, side[q], s));
  }
  {
    Scope sc_(c, "layout");
    for (int q = 0; q < 2; ++q) CMM_HIP(c, cmm::launch_layout(g, side[q], oflow, s));
  }
  {
    Scope sc_(c, "countsketch");
    for (int q = 0; q < 2; ++q) CMM_HIP(c, cmm::launch_countsketch(dtype, g, side[q], s));
  }
  {
    Scope sc_(c, "fft_mac");
    CMM_HIP(c, cmm::launch_fft_mac(g, side[0], side[1], tw32, Ppart, s));
  }
  {
    Scope sc_(c, "ifft");
    CMM_HIP(c, cmm::launch_ifft(g, Ppart, work0, work1, tw64, sk->c64, s));
    if (flags & CMM_SUBTRACT_DIAG) {
      const int n = (int)sk->n1;
      const int kch = (int)std::max<int64_t>(1, std::min<int64_t>(sk->m, 1 + 4096 / ((n + 255) / 256)));
      double* partial = w.get<double>((size_t)kch * n);
      double* diag = w.get<double>((size_t)n);
      if (!partial || !diag) return fail(c, CMM_ENOMEM, "workspace allocation failed");
      CMM_HIP(c, cmm::launch_diag(dtype, side[0], side[1], g.m, n, partial, kch, diag, s));
      CMM_HIP(c, cmm::launch_sub_diag(g, sk->hs1, sk->hs2, (int)sk->n1, (int)sk->n3, diag, n,
                                      sk->c64, s));
    }
    CMM_HIP(c, cmm::launch_to_f32(sk->c64, sk->c32, (int64_t)g.d * g.b, s));
  }
  *overflowed = false;
  if (!async) {
    CMM_HIP(c, hipMemcpyAsync(c->pinned_u32, oflow, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    CMM_HIP(c, hipStreamSynchronize(s));
    *overflowed = c->pinned_u32[0] != 0;
  }
  return CMM_OK;
}

int product_common(cmm_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                   int64_t n1, int64_t m, int64_t n3, int32_t dtype, const float* scaleA,
                   const float* scaleB, int64_t b, int32_t d, uint64_t seed,
                   const uint64_t* hash_params, const int32_t* th1, const int8_t* ts1,
                   const int32_t* th2, const int8_t* ts2, uint32_t flags, cmm_sketch** out) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  if (!out) return fail(ctx, CMM_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_operands(ctx, A, lda, B, ldb, n1, m, n3, dtype, b, d);
  if (rc) return rc;
  if ((flags & CMM_SUBTRACT_DIAG) && n1 != n3)
    return fail(ctx, CMM_EINVAL, "CMM_SUBTRACT_DIAG needs n1 == n3");
  if (flags & ~(CMM_SUBTRACT_DIAG | CMM_ASYNC)) return fail(ctx, CMM_EINVAL, "unknown flag");
  if (dtype != CMM_FP8_E4M3 && (scaleA || scaleB))
    return fail(ctx, CMM_EINVAL, "scales are only taken with CMM_FP8_E4M3");
  hipError_t e0 = hipSetDevice(ctx->device);
  if (e0 != hipSuccess) return fail(ctx, CMM_EHIP, "hipSetDevice failed");

  cmm_sketch* sk = new cmm_sketch();
  sk->ctx = ctx; sk->n1 = n1; sk->m = m; sk->n3 = n3; sk->b = b; sk->d = d;
  sk->log2b = ilog2(b);
  std::vector<int32_t> hsh1, hsh2;
  if (th1) {
    if (!ts1 || !th2 || !ts2) { delete sk; return fail(ctx, CMM_EINVAL, "all four tables are needed"); }
    hsh1.resize((size_t)d * n1); hsh2.resize((size_t)d * n3);
    for (size_t x = 0; x < hsh1.size(); ++x) {
      if (th1[x] < 0 || th1[x] >= b || (ts1[x] != 1 && ts1[x] != -1)) { delete sk; return fail(ctx, CMM_EINVAL, "bad h1/s1 table entry"); }
      hsh1[x] = (th1[x] << 1) | (ts1[x] < 0 ? 1 : 0);
    }
    for (size_t x = 0; x < hsh2.size(); ++x) {
      if (th2[x] < 0 || th2[x] >= b || (ts2[x] != 1 && ts2[x] != -1)) { delete sk; return fail(ctx, CMM_EINVAL, "bad h2/s2 table entry"); }
      hsh2[x] = (th2[x] << 1) | (ts2[x] < 0 ? 1 : 0);
    }
  } else {
    sk->has_params = true;
    if (hash_params) {
      sk->params.assign(hash_params, hash_params + (size_t)d * 8);
      for (int q = 0; q < d * 4; ++q)
        if (sk->params[2 * q] == 0 || sk->params[2 * q] >= CMM_P61 || sk->params[2 * q + 1] >= CMM_P61) {
          delete sk; return fail(ctx, CMM_EINVAL, "hash parameters out of range");
        }
    } else {
      params_from_seed(seed, d, sk->params);
    }
  }
  sk->hs1 = (int32_t*)dalloc(ctx, sizeof(int32_t) * d * n1);
  sk->hs2 = (int32_t*)dalloc(ctx, sizeof(int32_t) * d * n3);
  sk->c64 = (double*)dalloc(ctx, sizeof(double) * d * b);
  sk->c32 = (float*)dalloc(ctx, sizeof(float) * d * b);
  if (!sk->hs1 || !sk->hs2 || !sk->c64 || !sk->c32) {
    dfree(ctx, sk->hs1); dfree(ctx, sk->hs2); dfree(ctx, sk->c64); dfree(ctx, sk->c32);
    delete sk;
    return fail(ctx, CMM_ENOMEM, "sketch allocation failed");
  }
  if (th1) {
    hipError_t e1 = hipMemcpyAsync(sk->hs1, hsh1.data(), sizeof(int32_t) * hsh1.size(), hipMemcpyHostToDevice, ctx->stream);
    hipError_t e2 = hipMemcpyAsync(sk->hs2, hsh2.data(), sizeof(int32_t) * hsh2.size(), hipMemcpyHostToDevice, ctx->stream);
    hipError_t e3 = hipStreamSynchronize(ctx->stream);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) { cmm_sketch_free(sk); return fail(ctx, CMM_EHIP, "table upload failed"); }
  }
  bool over = false;
  rc = run_product(ctx, sk, A, lda, B, ldb, dtype, scaleA, scaleB, flags, false, &over);
  if (rc == CMM_OK && over)
    rc = run_product(ctx, sk, A, lda, B, ldb, dtype, scaleA, scaleB, flags, true, &over);
  if (rc != CMM_OK) { cmm_sketch_free(sk); return rc; }
  *out = sk;
  return CMM_OK;
}

cmm::DecodeDesc decode_desc(const cmm_sketch* sk) {
  cmm::DecodeDesc dd;
  dd.hs1 = sk->hs1; dd.hs2 = sk->hs2; dd.c32 = sk->c32;
  dd.n1 = (int)sk->n1; dd.n3 = (int)sk->n3; dd.d = sk->d;
  dd.mask = (uint32_t)(sk->b - 1); dd.b = sk->b;
  return dd;
}

}  // namespace

// =========================================================================
extern "C" {

const char* cmm_strerror(int code) {
  switch (code) {
    case CMM_OK: return "ok";
    case CMM_EINVAL: return "invalid argument";
    case CMM_ENOMEM: return "out of device memory";
    case CMM_EHIP: return "HIP runtime error";
    case CMM_EUNSUPPORTED: return "unsupported request";
    case CMM_ESTATE: return "object in wrong state";
    default: return "unknown status";
  }
}

const char* cmm_last_error(const cmm_ctx* ctx) {
  if (!valid_ctx(ctx)) return "invalid context";
  return ctx->last_error.c_str();
}

int cmm_ctx_create(int device, void* hip_stream, cmm_ctx** out) {
  if (!out) return CMM_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) { (void)hipGetLastError(); return CMM_EHIP; }
  if (device < 0 || device >= n) return CMM_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return CMM_EHIP;
  cmm_ctx* c = new cmm_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (hipHostMalloc((void**)&c->pinned_u32, 64 * sizeof(uint32_t)) != hipSuccess) {
    delete c;
    return CMM_ENOMEM;
  }
  *out = c;
  return CMM_OK;
}

int cmm_ctx_set_stream(cmm_ctx* ctx, void* hip_stream) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  CMM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  ctx->stream = (hipStream_t)hip_stream;
  return CMM_OK;
}

int cmm_ctx_destroy(cmm_ctx* ctx) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  for (auto& p : ctx->pending) { hipEventDestroy(p.a); hipEventDestroy(p.b); }
  for (auto& kv : ctx->sizes) hipFree(kv.first);
  for (auto& kv : ctx->twiddles) { hipFree(kv.second.first); hipFree(kv.second.second); }
  if (ctx->pinned_u32) hipHostFree(ctx->pinned_u32);
  ctx->magic = kDeadMagic;
  delete ctx;
  return CMM_OK;
}

int cmm_ctx_profile(cmm_ctx* ctx, int enable) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  drain_profile(ctx);
  ctx->prof = enable != 0;
  ctx->prof_acc.clear();
  return CMM_OK;
}

int cmm_ctx_profile_read(cmm_ctx* ctx, const char* name, double* total_ms, int64_t* launches) {
  if (!valid_ctx(ctx) || !name) return CMM_EINVAL;
  drain_profile(ctx);
  auto it = ctx->prof_acc.find(name);
  if (total_ms) *total_ms = it == ctx->prof_acc.end() ? 0.0 : it->second.first;
  if (launches) *launches = it == ctx->prof_acc.end() ? 0 : it->second.second;
  return CMM_OK;
}

int cmm_sketch_product(cmm_ctx* ctx, const float* A, const float* B, int64_t n, int64_t b,
                       int32_t d, uint64_t seed, cmm_sketch** out) {
  return product_common(ctx, A, n, B, n, n, n, n, CMM_F32, nullptr, nullptr, b, d, seed, nullptr,
                        nullptr, nullptr, nullptr, nullptr, 0, out);
}

int cmm_sketch_product_ex(cmm_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                          int64_t n1, int64_t m, int64_t n3, int32_t dtype, const float* scaleA,
                          const float* scaleB, int64_t b, int32_t d, uint64_t seed,
                          const uint64_t* hash_params, uint32_t flags, cmm_sketch** out) {
  return product_common(ctx, A, lda, B, ldb, n1, m, n3, dtype, scaleA, scaleB, b, d, seed,
                        hash_params, nullptr, nullptr, nullptr, nullptr, flags, out);
}

int cmm_sketch_product_tables(cmm_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                              int64_t n1, int64_t m, int64_t n3, int32_t dtype,
                              const float* scaleA, const float* scaleB, int64_t b, int32_t d,
                              const int32_t* h1, const int8_t* s1, const int32_t* h2,
                              const int8_t* s2, uint32_t flags, cmm_sketch** out) {
  if (valid_ctx(ctx) && (!h1 || !s1 || !h2 || !s2)) return fail(ctx, CMM_EINVAL, "tables are NULL");
  return product_common(ctx, A, lda, B, ldb, n1, m, n3, dtype, scaleA, scaleB, b, d, 0, nullptr,
                        h1, s1, h2, s2, flags, out);
}

int cmm_sketch_free(cmm_sketch* sk) {
  if (!valid_sketch(sk)) return CMM_EINVAL;
  cmm_ctx* c = sk->ctx;
  dfree(c, sk->hs1); dfree(c, sk->hs2); dfree(c, sk->c64); dfree(c, sk->c32);
  sk->magic = kDeadMagic;
  delete sk;
  return CMM_OK;
}

int cmm_sketch_info(const cmm_sketch* sk, int64_t* n1, int64_t* m, int64_t* n3, int64_t* b,
                    int32_t* d) {
  if (!valid_sketch(sk)) return CMM_EINVAL;
  if (n1) *n1 = sk->n1;
  if (m) *m = sk->m;
  if (n3) *n3 = sk->n3;
  if (b) *b = sk->b;
  if (d) *d = sk->d;
  return CMM_OK;
}

int cmm_sketch_copy_c(const cmm_sketch* sk, double* dst, int64_t count, int32_t dst_on_device) {
  if (!valid_sketch(sk)) return CMM_EINVAL;
  cmm_ctx* c = sk->ctx;
  if (!dst || count != sk->d * sk->b) return fail(c, CMM_EINVAL, "dst NULL or count != d*b");
  CMM_HIP(c, hipMemcpyAsync(dst, sk->c64, sizeof(double) * count,
                            dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                            c->stream));
  CMM_HIP(c, hipStreamSynchronize(c->stream));
  return CMM_OK;
}

int cmm_sketch_hash_params(const cmm_sketch* sk, uint64_t* ac) {
  if (!valid_sketch(sk)) return CMM_EINVAL;
  if (!ac) return fail(sk->ctx, CMM_EINVAL, "ac is NULL");
  if (!sk->has_params) return fail(sk->ctx, CMM_ESTATE, "sketch was built from explicit tables");
  std::memcpy(ac, sk->params.data(), sizeof(uint64_t) * sk->params.size());
  return CMM_OK;
}

int cmm_sketch_hashes(const cmm_sketch* sk, int32_t t, int32_t* h1, int8_t* s1, int32_t* h2,
                      int8_t* s2) {
  if (!valid_sketch(sk)) return CMM_EINVAL;
  cmm_ctx* c = sk->ctx;
  if (t < 0 || t >= sk->d) return fail(c, CMM_EINVAL, "t out of range");
  std::vector<int32_t> a((size_t)sk->n1), b2((size_t)sk->n3);
  CMM_HIP(c, hipMemcpyAsync(a.data(), sk->hs1 + (size_t)t * sk->n1, sizeof(int32_t) * sk->n1, hipMemcpyDeviceToHost, c->stream));
  CMM_HIP(c, hipMemcpyAsync(b2.data(), sk->hs2 + (size_t)t * sk->n3, sizeof(int32_t) * sk->n3, hipMemcpyDeviceToHost, c->stream));
  CMM_HIP(c, hipStreamSynchronize(c->stream));
  for (int64_t x = 0; x < sk->n1; ++x) {
    if (h1) h1[x] = a[x] >> 1;
    if (s1) s1[x] = (a[x] & 1) ? -1 : 1;
  }
  for (int64_t x = 0; x < sk->n3; ++x) {
    if (h2) h2[x] = b2[x] >> 1;
    if (s2) s2[x] = (b2[x] & 1) ? -1 : 1;
  }
  return CMM_OK;
}

int cmm_sketch_subtract_diagonal(cmm_sketch* sk, const double* diag, int64_t len) {
  if (!valid_sketch(sk)) return CMM_EINVAL;
  cmm_ctx* c = sk->ctx;
  if (!diag || len < 0 || len > std::min(sk->n1, sk->n3)) return fail(c, CMM_EINVAL, "bad diag");
  if (len == 0) return CMM_OK;
  cmm::Geometry g = make_geometry(sk->b, sk->d, sk->m);
  CMM_HIP(c, cmm::launch_sub_diag(g, sk->hs1, sk->hs2, (int)sk->n1, (int)sk->n3, diag, (int)len, sk->c64, c->stream));
  CMM_HIP(c, cmm::launch_to_f32(sk->c64, sk->c32, sk->d * sk->b, c->stream));
  CMM_HIP(c, hipStreamSynchronize(c->stream));
  return CMM_OK;
}

int cmm_sketch_merge(cmm_sketch* dst, const cmm_sketch* src) {
  if (!valid_sketch(dst) || !valid_sketch(src)) return CMM_EINVAL;
  cmm_ctx* c = dst->ctx;
  if (dst->b != src->b || dst->d != src->d || dst->n1 != src->n1 || dst->n3 != src->n3 ||
      dst->has_params != src->has_params || !dst->has_params || dst->params != src->params)
    return fail(c, CMM_ESTATE, "sketches differ in hash functions or shape");
  CMM_HIP(c, hipStreamSynchronize(src->ctx->stream));
  CMM_HIP(c, cmm::launch_add_f64(dst->c64, src->c64, dst->d * dst->b, c->stream));
  CMM_HIP(c, cmm::launch_to_f32(dst->c64, dst->c32, dst->d * dst->b, c->stream));
  CMM_HIP(c, hipStreamSynchronize(c->stream));
  return CMM_OK;
}

int cmm_estimate(const cmm_sketch* sk, int64_t i, int64_t j, double* out) {
  if (!valid_sketch(sk)) return CMM_EINVAL;
  cmm_ctx* c = sk->ctx;
  if (!out || i < 0 || j < 0 || i >= sk->n1 || j >= sk->n3) return fail(c, CMM_EINVAL, "index out of range");
  // the d hash words and sketch entries, read back, median on the host
  std::vector<double> x((size_t)sk->d);
  for (int t = 0; t < sk->d; ++t) {
    int32_t a = 0, b2 = 0;
    CMM_HIP(c, hipMemcpyAsync(&a, sk->hs1 + (size_t)t * sk->n1 + i, 4, hipMemcpyDeviceToHost, c->stream));
    CMM_HIP(c, hipMemcpyAsync(&b2, sk->hs2 + (size_t)t * sk->n3 + j, 4, hipMemcpyDeviceToHost, c->stream));
    CMM_HIP(c, hipStreamSynchronize(c->stream));
    const int64_t u = ((int64_t)(a >> 1) + (b2 >> 1)) & (sk->b - 1);
    double v = 0.0;
    CMM_HIP(c, hipMemcpyAsync(&v, sk->c64 + (size_t)t * sk->b + u, 8, hipMemcpyDeviceToHost, c->stream));
    CMM_HIP(c, hipStreamSynchronize(c->stream));
    x[t] = ((a ^ b2) & 1) ? -v : v;
  }
  std::sort(x.begin(), x.end());
  const int dd = sk->d;
  *out = (dd & 1) ? x[(dd - 1) / 2] : 0.5 * (x[dd / 2 - 1] + x[dd / 2]);
  return CMM_OK;
}

int cmm_estimate_batch(const cmm_sketch* sk, const int64_t* i, const int64_t* j, int64_t q,
                       float* out) {
  if (!valid_sketch(sk)) return CMM_EINVAL;
  cmm_ctx* c = sk->ctx;
  if (q < 0 || (q > 0 && (!i || !j || !out))) return fail(c, CMM_EINVAL, "bad batch arguments");
  {
    Scope sc_(c, "decode");
    CMM_HIP(c, cmm::launch_estimate(decode_desc(sk), i, j, q, out, c->stream));
  }
  CMM_HIP(c, hipStreamSynchronize(c->stream));
  return CMM_OK;
}

int cmm_topk(const cmm_sketch* sk, int32_t K, int32_t mode, int64_t* out_i, int64_t* out_j,
             float* out_val) {
  if (!valid_sketch(sk)) return CMM_EINVAL;
  cmm_ctx* c = sk->ctx;
  if (!out_i || !out_j || !out_val) return fail(c, CMM_EINVAL, "output arrays are NULL");
  if (K < 1) return fail(c, CMM_EINVAL, "K < 1");
  hipStream_t s = c->stream;
  const cmm::DecodeDesc dd = decode_desc(sk);
  Work w(c);
  if (mode == CMM_TOPK_PER_COLUMN) {
    if (K > sk->n1) return fail(c, CMM_EINVAL, "K larger than a column");
    if (sk->n1 * 4 > 64 * 1024) return fail(c, CMM_EUNSUPPORTED, "per-column top-K needs n1 <= 16384");
    const size_t tot = (size_t)K * sk->n3;
    int64_t* oi = w.get<int64_t>(tot);
    float* ov = w.get<float>(tot);
    if (!oi || !ov) return fail(c, CMM_ENOMEM, "workspace allocation failed");
    {
      Scope sc_(c, "decode");
      CMM_HIP(c, cmm::launch_topk_column(dd, K, oi, ov, s));
    }
    CMM_HIP(c, hipMemcpyAsync(out_i, oi, sizeof(int64_t) * tot, hipMemcpyDeviceToHost, s));
    CMM_HIP(c, hipMemcpyAsync(out_val, ov, sizeof(float) * tot, hipMemcpyDeviceToHost, s));
    CMM_HIP(c, hipStreamSynchronize(s));
    for (int64_t jj = 0; jj < sk->n3; ++jj)
      for (int r = 0; r < K; ++r) out_j[jj * K + r] = jj;
    return CMM_OK;
  }
  if (mode != CMM_TOPK_ALL && mode != CMM_TOPK_UPPER) return fail(c, CMM_EINVAL, "unknown mode");
  const int64_t domain = mode == CMM_TOPK_ALL
                             ? sk->n1 * sk->n3
                             : [&] { int64_t t = 0; for (int64_t i = 0; i < sk->n1; ++i) t += std::max<int64_t>(0, sk->n3 - i - 1); return t; }();
  if (K > domain) return fail(c, CMM_EINVAL, "K larger than the candidate domain");
  if (K > cmm::kTopkCap / 2) return fail(c, CMM_EUNSUPPORTED, "K above 2048");
  uint32_t* hist = w.get<uint32_t>(4096);
  uint32_t* count = w.get<uint32_t>(1);
  cmm::TopkCand* cand = w.get<cmm::TopkCand>(cmm::kTopkCap);
  int64_t* oi = w.get<int64_t>(K);
  int64_t* oj = w.get<int64_t>(K);
  float* ov = w.get<float>(K);
  if (!hist || !count || !cand || !oi || !oj || !ov) return fail(c, CMM_ENOMEM, "workspace allocation failed");
  std::vector<uint32_t> h(4096);
  // digit passes: bits [30:19], [18:7], [6:0]
  const int dshift[3] = {19, 7, 0};
  const uint32_t dmask[3] = {0xFFF, 0xFFF, 0x7F};
  uint32_t prefix = 0;
  int pshift = 32;
  int64_t above = 0;
  int64_t need = K;
  uint32_t thresh = 0;
  bool done = false;
  {
    Scope sc_(c, "decode");
    for (int level = 0; level < 3 && !done; ++level) {
      CMM_HIP(c, cmm::launch_fill_i32((int32_t*)hist, 4096, 0, s));
      CMM_HIP(c, cmm::launch_topk_hist(dd, mode, prefix, pshift, dshift[level], dmask[level], hist, s));
      CMM_HIP(c, hipMemcpyAsync(h.data(), hist, 4096 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      CMM_HIP(c, hipStreamSynchronize(s));
      int64_t cum = 0;
      int bin = -1;
      for (int q = (int)dmask[level]; q >= 0; --q) {
        if (cum + h[q] >= need) { bin = q; break; }
        cum += h[q];
      }
      if (bin < 0) return fail(c, CMM_EHIP, "top-K histogram lost entries");
      prefix |= (uint32_t)bin << dshift[level];
      const int64_t total = above + cum + h[bin];
      if (total <= cmm::kTopkCap) { thresh = prefix; done = true; break; }
      above += cum;
      need -= cum;
      pshift = dshift[level];
    }
    if (!done) return fail(c, CMM_EUNSUPPORTED, "more than 4096 estimates tie at the K-th magnitude");
    CMM_HIP(c, cmm::launch_fill_i32((int32_t*)count, 1, 0, s));
    CMM_HIP(c, cmm::launch_topk_collect(dd, mode, thresh, cand, count, cmm::kTopkCap, s));
    CMM_HIP(c, cmm::launch_topk_final(cand, count, cmm::kTopkCap, K, (int)sk->n3, oi, oj, ov, s));
  }
  CMM_HIP(c, hipMemcpyAsync(out_i, oi, sizeof(int64_t) * K, hipMemcpyDeviceToHost, s));
  CMM_HIP(c, hipMemcpyAsync(out_j, oj, sizeof(int64_t) * K, hipMemcpyDeviceToHost, s));
  CMM_HIP(c, hipMemcpyAsync(out_val, ov, sizeof(float) * K, hipMemcpyDeviceToHost, s));
  CMM_HIP(c, hipStreamSynchronize(s));
  return CMM_OK;
}

}  // extern "C"

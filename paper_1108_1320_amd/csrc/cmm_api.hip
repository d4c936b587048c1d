// C interface of the cmm library: argument checking, device memory,
// ordering of the kernels of one sketch product on the context stream.
#include "cmm.h"
#include "cmm_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

namespace {

constexpr uint32_t kCtxMagic = 0xC3A70001u;
constexpr uint32_t kSketchMagic = 0xC3A75001u;
constexpr uint32_t kBatchMagic = 0xC3A7B001u;
constexpr uint32_t kDeadMagic = 0xDEADDEADu;

struct Pending {
  std::string name;
  hipEvent_t a, b;
};

// Tuning key of a product: sizes rounded to powers of two.
struct TuneKey {
  int log2b, ln1, lm, ln3, d, dtype;
  bool operator<(const TuneKey& o) const {
    return std::tie(log2b, ln1, lm, ln3, d, dtype) < std::tie(o.log2b, o.ln1, o.lm, o.ln3, o.d, o.dtype);
  }
};

struct TuneEntry {
  cmm::Tuning tu;
  double ms = 0.0;
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
  std::vector<hipEvent_t> event_pool;   // timing events reused across scopes
  std::map<std::string, std::pair<double, double>> prof_bytes;   // read, written
  uint32_t* pinned_u32 = nullptr;   // small pinned host scratch
  char* pinned = nullptr;           // pinned staging of downloads (pinned_cap bytes)
  size_t pinned_cap = 0;
  std::map<TuneKey, TuneEntry> tuning;
  std::string arch;
  int64_t ws_limit = 0;     // workspace limit of one product in bytes (0: ws_default)
  int64_t ws_default = 0;   // half the device memory
  cmm::Overlap ov;          // second stream of the spectral step
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
  cmm_batch* owner = nullptr;     // set while the sketch belongs to a batch
};

namespace {

void destroy_overlap(cmm::Overlap& ov) {
  if (ov.aux) { hipStreamSynchronize(ov.aux); hipStreamDestroy(ov.aux); }
  if (ov.fork) hipEventDestroy(ov.fork);
  if (ov.join) hipEventDestroy(ov.join);
  ov = cmm::Overlap();
}

// The second stream for a spectral step on stream `s`: the context's, for
// work on the context stream that is not being captured into a graph (the
// pair kernel then runs on `s` itself, before the row kernel).
const cmm::Overlap* overlap_for(cmm_ctx* c, hipStream_t s) {
  if (s != c->stream) return nullptr;
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
  return st == hipStreamCaptureStatusNone ? &c->ov : nullptr;
}

int fail(cmm_ctx* c, int code, const std::string& msg) {
  if (c) c->last_error = msg;
  return code;
}

constexpr size_t kPinnedBytes = 256 * 1024;   // initial pinned staging
constexpr size_t kPinnedMax = 64u << 20;       // the staging grows up to this

#define CMM_HIP(ctx, expr)                                                          \
  do {                                                                              \
    hipError_t e__ = (expr);                                                        \
    if (e__ != hipSuccess)                                                          \
      return fail((ctx), CMM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e__)); \
  } while (0)

struct Download {
  void* dst;
  const void* src;
  size_t bytes;
};

// Device-to-host copies on stream `s`, then a wait.  A pageable destination
// makes the runtime stage the copy through a blit kernel; copies that fit
// together go through the context's pinned buffer instead (plain DMA) and
// are moved to their destinations on the host.
int download(cmm_ctx* c, hipStream_t s, std::initializer_list<Download> list);
int download_n(cmm_ctx* c, hipStream_t s, const Download* list, size_t n);

bool valid_ctx(const cmm_ctx* c) { return c && c->magic == kCtxMagic; }
bool valid_sketch(const cmm_sketch* s) { return s && s->magic == kSketchMagic && valid_ctx(s->ctx); }

// ---- device scratch of the allocation-free product (cmm_sketch_product_noalloc)
//
// One array per device, held from the library's load until the process
// ends.  Host code never passes `scratch` itself to a kernel or a copy (in
// host code it names a host-side stand-in): the device address comes from
// hipGetSymbolAddress, taken once per device with that device current when
// a context is created there, and kept in g_scratch_dev.
constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
void* g_scratch_dev[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of `scratch` on `device` (the current device); looked up
// once per device.
void bind_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices || g_scratch_dev[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    g_scratch_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
    return;
  }
  g_scratch_dev[device] = p;
}

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

// A timing event from the context's pool (created on first use).
hipEvent_t take_event(cmm_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
  return e;
}

struct Scope {
  cmm_ctx* c;
  const char* name;
  hipEvent_t a = nullptr, b = nullptr;
  Scope(cmm_ctx* cc, const char* nm) : c(cc), name(nm) {
    if (!c->prof) return;
    a = take_event(c);
    b = take_event(c);
    if (a && b) {
      hipEventRecord(a, c->stream);
    } else {
      if (a) c->event_pool.push_back(a);
      if (b) c->event_pool.push_back(b);
      a = b = nullptr;
    }
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
    c->event_pool.push_back(p.a);
    c->event_pool.push_back(p.b);
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

// Coefficients (a0..a3) of the degree-3 sign polynomials of the Frobenius
// bound: [t][f][c] = z_{1024 + 8t + 4f + c + 1} mod p, f = 0 for s1, 1 for s2.
void ams_params_from_seed(uint64_t seed, int d, std::vector<uint64_t>& out) {
  out.resize((size_t)d * 8);
  for (int t = 0; t < d; ++t)
    for (int f = 0; f < 2; ++f)
      for (int c = 0; c < 4; ++c)
        out[(size_t)t * 8 + f * 4 + c] =
            splitmix64_at(seed, (uint64_t)(1024 + 8 * t + 4 * f + c + 1)) % CMM_P61;
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

cmm::Tuning default_tuning(int64_t b) {
  cmm::Tuning t;
  // 4096-point rows measured fastest on b = 2^16 (8192-point rows: fewer
  // rows but one block per CU); CMM_LOG2C overrides for experiments
  t.log2c = 12;
  if (const char* ev = std::getenv("CMM_LOG2C")) t.log2c = std::atoi(ev);
  t.log2c = std::max(4, std::min(cmm::kMaxLog2C, t.log2c));
  (void)b;
  return t;
}

cmm::Geometry make_geometry(int64_t b, int d, int64_t m, const cmm::Tuning& tu) {
  cmm::Geometry g;
  g.b = b; g.log2b = ilog2(b); g.d = d; g.m = (int)m;
  // at most 256 rows (R = b / C): the fold-weight table of 16 R entries
  // stays in LDS and a bucket's row index fits the 16-bit field of its entry
  g.log2c = std::min(g.log2b, std::max(tu.log2c, g.log2b - 8));
  const int C = 1 << g.log2c;
  g.T = C / 16;
  g.G = std::min(g.T, 64);
  g.W = g.T / g.G;
  g.R = (int)(b / C);
  g.rows = g.R > 1 ? g.R / 2 + 1 : 1;
  g.rblocks = g.R > 1 ? g.R / 2 : 1;
  const int64_t base = (int64_t)d * g.rblocks;
  const int kmax = std::max(1, std::min(tu.kmax, cmm::kMaxKPerBlock));
  // k-splits: at least 2048 spectral blocks per product (four rounds of the
  // chip's 512 block slots), at most kmax k per block, at least one k each
  int64_t ks = std::max<int64_t>(1, (2048 + base - 1) / base);
  ks = std::max<int64_t>(ks, (m + kmax - 1) / kmax);
  ks = std::min<int64_t>(ks, m);
  g.KS = (int)std::max<int64_t>(1, ks);
  g.cs_blocks = std::max(1, tu.cs_blocks);
  return g;
}

cmm::Tuning lookup_tuning(const cmm_ctx* c, int64_t n1, int64_t m, int64_t n3, int64_t b, int d,
                          int dtype);

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

// Element counts of every workspace buffer of one product.
enum WsBuf { W_CNT0, W_POS0, W_ENT0, W_TAB0, W_CNTP0, W_MOFF0, W_FILL0, W_PERM0, W_SEG0, W_LSEG0,
             W_SA0, W_CMAX0, W_ENTP0, W_CNT1, W_POS1, W_ENT1, W_TAB1, W_CNTP1, W_MOFF1, W_FILL1, W_PERM1,
             W_SEG1, W_LSEG1, W_SA1, W_CMAX1, W_ENTP1, W_PPART, W_WORK0, W_WORK1, W_OFLOW, W_PARTIAL,
             W_DIAG, W_COUNT };
constexpr size_t kElemSize[W_COUNT] = {4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 2, 4, 4, 4, 4, 4, 4, 4,
                                       4, 4, 4, 4, 4, 2, 8, 16, 16, 4, 8, 8};
static_assert(kElemSize[W_COUNT - 1] != 0 && W_CNT1 - W_CNT0 == W_PPART - W_CNT1,
              "one element size per workspace buffer, the same buffers for both sides");

struct WsSpec {
  size_t count[W_COUNT] = {};
  int Lcap[2] = {0, 0};
  int kch = 1;
};

WsSpec ws_spec(const cmm::Geometry& g, int64_t n1, int64_t n3, bool safe, uint32_t flags) {
  WsSpec w;
  const int64_t nn[2] = {n1, n3};
  for (int q = 0; q < 2; ++q) {
    const int o = q * (W_CNT1 - W_CNT0);
    w.Lcap[q] = layout_cap(nn[q], g.b, g.W, safe);
    const size_t Lrow = (size_t)g.W * w.Lcap[q];
    w.count[W_CNT0 + o] = (size_t)g.d * g.b;
    w.count[W_POS0 + o] = (size_t)g.d * g.b;
    w.count[W_ENT0 + o] = w.count[W_TAB0 + o] = w.count[W_CNTP0 + o] = (size_t)g.d * Lrow;
    w.count[W_ENTP0 + o] = (size_t)g.d * Lrow;
    w.count[W_MOFF0 + o] = w.count[W_FILL0 + o] = (size_t)g.d * Lrow;
    w.count[W_PERM0 + o] = (size_t)g.d * nn[q];
    w.count[W_SEG0 + o] = (size_t)g.d * g.W;
    w.count[W_LSEG0 + o] = (size_t)g.d;
    w.count[W_SA0 + o] = (size_t)g.d * g.m * Lrow;
    w.count[W_CMAX0 + o] = (size_t)g.d * g.m;
  }
  w.count[W_PPART] = (size_t)g.d * g.KS * g.rows * ((size_t)1 << g.log2c);
  w.count[W_WORK0] = w.count[W_WORK1] = (size_t)g.d * g.b;
  w.count[W_OFLOW] = 1;
  if (flags & CMM_SUBTRACT_DIAG) {
    const int n = (int)n1;
    w.kch = (int)std::max<int64_t>(1, std::min<int64_t>(g.m, 1 + 4096 / ((n + 255) / 256)));
    w.count[W_PARTIAL] = (size_t)w.kch * n;
    w.count[W_DIAG] = (size_t)n;
  }
  return w;
}

struct WsPtrs {
  void* p[W_COUNT] = {};
};

// Allocate every buffer of `spec` (sizes only) from the context cache.
int ws_alloc(cmm_ctx* c, const WsSpec& spec, WsPtrs& ptr, std::vector<void*>& owned) {
  for (int i = 0; i < W_COUNT; ++i) {
    if (spec.count[i] == 0) continue;
    void* q = dalloc(c, spec.count[i] * kElemSize[i]);
    if (!q) return fail(c, CMM_ENOMEM, "workspace allocation failed");
    owned.push_back(q);
    ptr.p[i] = q;
  }
  return CMM_OK;
}

void ws_release(cmm_ctx* c, std::vector<void*>& owned) {
  for (void* q : owned) dfree(c, q);
  owned.clear();
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
  if (std::max(n1, n3) > cmm::kMaxHashedDim)
    return fail(c, CMM_EUNSUPPORTED, "hashed dimension above 65535");
  return CMM_OK;
}

struct Operands {
  const void* A; int64_t lda; const void* B; int64_t ldb;
  int32_t dtype; const float* scaleA; const float* scaleB; uint32_t flags;
  // sparse operands (dtype kSparseF32): A by columns, B by rows
  const int64_t* aptr = nullptr; const int32_t* aidx = nullptr;
  const int64_t* bptr = nullptr; const int32_t* bidx = nullptr;
};

// Side descriptors of a product over the buffers `ptr` (which may be larger
// than this product needs, e.g. a workspace shared by a batch).
void bind_sides(const cmm::Geometry& g, const cmm_sketch* sk, const Operands& op,
                const WsSpec& spec, const WsPtrs& ptr, cmm::SideDesc side[2]) {
  const int64_t nn[2] = {sk->n1, sk->n3};
  const void* X[2] = {op.A, op.B};
  const int64_t ld[2] = {op.lda, op.ldb};
  const float* sc[2] = {op.scaleA, op.scaleB};
  int32_t* hsv[2] = {sk->hs1, sk->hs2};
  for (int q = 0; q < 2; ++q) {
    const int o = q * (W_CNT1 - W_CNT0);
    cmm::SideDesc& sd = side[q];
    sd.X = X[q]; sd.ld = ld[q]; sd.scale = sc[q]; sd.n = (int)nn[q]; sd.hs = hsv[q];
    sd.sptr = q == 0 ? op.aptr : op.bptr;
    sd.sidx = q == 0 ? op.aidx : op.bidx;
    sd.Lcap = spec.Lcap[q];
    sd.Lrow = g.W * sd.Lcap;
    sd.cnt = (int32_t*)ptr.p[W_CNT0 + o];
    sd.pos = (int32_t*)ptr.p[W_POS0 + o];
    sd.ent = (uint32_t*)ptr.p[W_ENT0 + o];
    sd.entp = (uint16_t*)ptr.p[W_ENTP0 + o];
    sd.tab = (uint32_t*)ptr.p[W_TAB0 + o];
    sd.cntp = (int32_t*)ptr.p[W_CNTP0 + o];
    sd.moff = (int32_t*)ptr.p[W_MOFF0 + o];
    sd.fill = (int32_t*)ptr.p[W_FILL0 + o];
    sd.perm = (int32_t*)ptr.p[W_PERM0 + o];
    sd.segcount = (int32_t*)ptr.p[W_SEG0 + o];
    sd.lseg = (int32_t*)ptr.p[W_LSEG0 + o];
    sd.SA = (float*)ptr.p[W_SA0 + o];
    sd.colmax = (float*)ptr.p[W_CMAX0 + o];
  }
}

// Hash tables (when `pdev` holds parameters), bucket counts and the bucket
// layout of both sides; `oflow` is set when a layout segment overflows.
int enqueue_layout(cmm_ctx* c, const cmm::Geometry& g, cmm::SideDesc side[2],
                   const uint64_t* pdev, int32_t* oflow, hipStream_t s) {
  CMM_HIP(c, cmm::launch_fill_i32(oflow, 1, 0, s));
  {
    Scope sc_(c, "hash");
    if (pdev)
      for (int q = 0; q < 2; ++q) CMM_HIP(c, cmm::launch_hash(pdev, q, g, side[q], s));
    for (int q = 0; q < 2; ++q) CMM_HIP(c, cmm::launch_count(g, side[q], s));
  }
  {
    Scope sc_(c, "layout");
    for (int q = 0; q < 2; ++q) CMM_HIP(c, cmm::launch_layout(g, side[q], oflow, s));
  }
  return CMM_OK;
}

// Every kernel of one sketch product, in stream order, on stream `s`: no
// allocation, no host synchronisation, no host-to-device copy (hash
// parameters are already at `pdev`), so the sequence can be captured.
// Grow the pinned staging buffer to `bytes` (at most kPinnedMax; the old
// buffer is idle between calls, every download waits before returning).
bool ensure_pinned(cmm_ctx* c, size_t bytes) {
  if (c->pinned && bytes <= c->pinned_cap) return true;
  if (bytes > kPinnedMax) return false;
  char* p = nullptr;
  if (hipHostMalloc((void**)&p, bytes) != hipSuccess) { (void)hipGetLastError(); return false; }
  if (c->pinned) hipHostFree(c->pinned);
  c->pinned = p;
  c->pinned_cap = bytes;
  return true;
}

int download_n(cmm_ctx* c, hipStream_t s, const Download* list, size_t n) {
  size_t total = 0;
  for (size_t q = 0; q < n; ++q) total += (list[q].bytes + 255) & ~(size_t)255;
  const bool staged = ensure_pinned(c, total);
  size_t off = 0;
  for (size_t q = 0; q < n; ++q) {
    const Download& x = list[q];
    if (x.bytes == 0) continue;
    void* to = staged ? (void*)(c->pinned + off) : x.dst;
    CMM_HIP(c, hipMemcpyAsync(to, x.src, x.bytes, hipMemcpyDeviceToHost, s));
    off += (x.bytes + 255) & ~(size_t)255;
  }
  CMM_HIP(c, hipStreamSynchronize(s));
  if (staged) {
    off = 0;
    for (size_t q = 0; q < n; ++q) {
      const Download& x = list[q];
      if (x.bytes == 0) continue;
      std::memcpy(x.dst, c->pinned + off, x.bytes);
      off += (x.bytes + 255) & ~(size_t)255;
    }
  }
  return CMM_OK;
}

int download(cmm_ctx* c, hipStream_t s, std::initializer_list<Download> list) {
  return download_n(c, s, list.begin(), list.size());
}

// All kernels of one product on stream `s`.  The float64 sketch goes to
// `c_out` (the sketch's own when null); `finish` also writes its float32 copy.
int enqueue_product(cmm_ctx* c, cmm_sketch* sk, const Operands& op, const cmm::Geometry& g,
                    const WsSpec& spec, const WsPtrs& ptr, const uint64_t* pdev, hipStream_t s,
                    double* c_out = nullptr, bool finish = true, double2* tw64_in = nullptr,
                    float2* tw32_in = nullptr) {
  double* c64 = c_out ? c_out : sk->c64;
  cmm::SideDesc side[2];
  bind_sides(g, sk, op, spec, ptr, side);
  double2* tw64 = tw64_in; float2* tw32 = tw32_in;
  int rc = tw64 && tw32 ? CMM_OK : get_twiddles(c, g.b, &tw64, &tw32);
  if (rc) return rc;
  rc = enqueue_layout(c, g, side, pdev, (int32_t*)ptr.p[W_OFLOW], s);
  if (rc) return rc;
  {
    Scope sc_(c, "countsketch");
    for (int q = 0; q < 2; ++q) CMM_HIP(c, cmm::launch_countsketch(op.dtype, g, side[q], s));
  }
  {
    Scope sc_(c, "fft_mac");
    CMM_HIP(c, cmm::launch_fft_mac(g, side[0], side[1], tw32, (float2*)ptr.p[W_PPART], s,
                                   overlap_for(c, s)));
  }
  {
    Scope sc_(c, "ifft");
    CMM_HIP(c, cmm::launch_ifft(g, (float2*)ptr.p[W_PPART], (double2*)ptr.p[W_WORK0],
                                (double2*)ptr.p[W_WORK1], tw64, c64, s));
    if (op.flags & CMM_SUBTRACT_DIAG) {
      const int n = (int)sk->n1;
      CMM_HIP(c, cmm::launch_diag(op.dtype, side[0], side[1], g.m, n, (double*)ptr.p[W_PARTIAL],
                                  spec.kch, (double*)ptr.p[W_DIAG], s));
      CMM_HIP(c, cmm::launch_sub_diag(g, sk->hs1, sk->hs2, (int)sk->n1, (int)sk->n3,
                                      (double*)ptr.p[W_DIAG], n, c64, ptr.p[W_WORK0], s));
    }
    if (finish) CMM_HIP(c, cmm::launch_to_f32(sk->c64, sk->c32, (int64_t)g.d * g.b, s));
  }
  return CMM_OK;
}

size_t spec_bytes(const WsSpec& spec) {
  size_t t = 0;
  for (int i = 0; i < W_COUNT; ++i) t += spec.count[i] * kElemSize[i];
  return t;
}

// Longest k-slab whose workspace stays within the context's limit (all of
// m when the whole product fits; at least one k).  The workspace grows with
// the slab length (count sketches, column maxima, k-split partials), so the
// search is a bisection over the length.
int64_t slab_length(const cmm_ctx* c, const cmm_sketch* sk, const cmm::Tuning& tu, bool safe,
                    uint32_t flags) {
  const int64_t limit = c->ws_limit > 0 ? c->ws_limit : c->ws_default;
  auto bytes = [&](int64_t mk) {
    return (int64_t)spec_bytes(ws_spec(make_geometry(sk->b, sk->d, mk, tu), sk->n1, sk->n3, safe, flags));
  };
  if (limit <= 0 || bytes(sk->m) <= limit) return sk->m;
  int64_t lo = 1, hi = sk->m;   // bytes(lo) may exceed the limit: one k is the least
  while (hi - lo > 1) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (bytes(mid) <= limit) lo = mid; else hi = mid;
  }
  return lo;
}

// Operands of the k-slab starting at k0: rows k0.. of both stored operands.
Operands slab_operands(const Operands& op, int64_t k0) {
  Operands o = op;
  if (op.dtype == cmm::kSparseF32) {
    o.aptr = op.aptr + k0;
    o.bptr = op.bptr + k0;
    return o;
  }
  const int64_t esz = op.dtype == CMM_F32 ? 4 : (op.dtype == CMM_BF16 ? 2 : 1);
  o.A = (const char*)op.A + k0 * op.lda * esz;
  o.B = (const char*)op.B + k0 * op.ldb * esz;
  return o;
}

// Bytes the count-sketch launches of a finished dense product moved by
// design, added to the "countsketch" byte record of the context: the stored
// operands (and fp8 scales) read once, and, per side, repetition and k, the
// W * lseg positions of the layout written (padding included) plus one
// column maximum.  Needs the layout's segment lengths from the device.
int account_countsketch(cmm_ctx* c, const cmm_sketch* sk, const Operands& op,
                        const cmm::Geometry& g, const WsPtrs& ptr, hipStream_t s) {
  std::vector<int32_t> l0((size_t)sk->d), l1((size_t)sk->d);
  const size_t nb = sizeof(int32_t) * sk->d;
  int rc = download(c, s, {{l0.data(), ptr.p[W_LSEG0], nb}, {l1.data(), ptr.p[W_LSEG1], nb}});
  if (rc) return rc;
  const double esz = op.dtype == CMM_F32 ? 4.0 : (op.dtype == CMM_BF16 ? 2.0 : 1.0);
  double rd = esz * (double)sk->m * (double)(sk->n1 + sk->n3);
  if (op.scaleA) rd += 4.0 * (double)sk->n1;
  if (op.scaleB) rd += 4.0 * (double)sk->n3;
  double wr = 0.0;
  for (int t = 0; t < sk->d; ++t) wr += 4.0 * (double)sk->m * g.W * (double)(l0[t] + l1[t]);
  wr += 4.0 * 2.0 * (double)sk->d * (double)sk->m;
  auto& acc = c->prof_bytes["countsketch"];
  acc.first += rd;
  acc.second += wr;
  return CMM_OK;
}

// One product on the context stream with a workspace from the cache.
// A product whose workspace would exceed the context's limit runs as
// consecutive k-slabs: the sketch of AB is the sum of the sketches of the
// slabs' partial products (eq. (1); the sketch is linear), added in float64.
int run_product(cmm_ctx* c, cmm_sketch* sk, const Operands& op, const cmm::Tuning& tu,
                bool safe_layout, bool* overflowed) {
  hipStream_t s = c->stream;
  const bool async = op.flags & CMM_ASYNC;
  const bool safe = safe_layout || async;
  const int64_t slab = slab_length(c, sk, tu, safe, op.flags);
  const cmm::Geometry g = make_geometry(sk->b, sk->d, slab, tu);
  const WsSpec spec = ws_spec(g, sk->n1, sk->n3, safe, op.flags);
  WsPtrs ptr;
  std::vector<void*> owned;
  uint64_t* pdev = nullptr;
  double* csum = nullptr;
  int rc = ws_alloc(c, spec, ptr, owned);
  if (rc == CMM_OK && slab < sk->m) {
    csum = (double*)dalloc(c, sizeof(double) * sk->d * sk->b);
    if (!csum) rc = fail(c, CMM_ENOMEM, "workspace allocation failed");
    else owned.push_back(csum);
  }
  if (rc == CMM_OK && sk->has_params) {
    pdev = (uint64_t*)dalloc(c, sizeof(uint64_t) * sk->d * 8);
    if (!pdev) rc = fail(c, CMM_ENOMEM, "workspace allocation failed");
    else owned.push_back(pdev);
  }
  if (rc == CMM_OK && pdev) {
    hipError_t e = hipMemcpyAsync(pdev, sk->params.data(), sizeof(uint64_t) * sk->d * 8,
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) rc = fail(c, CMM_EHIP, "parameter upload failed");
  }
  if (rc == CMM_OK && slab >= sk->m) rc = enqueue_product(c, sk, op, g, spec, ptr, pdev, s);
  // later slabs are shorter or equal: their workspace fits in the first's
  for (int64_t k0 = 0; rc == CMM_OK && slab < sk->m && k0 < sk->m; k0 += slab) {
    const cmm::Geometry gk = make_geometry(sk->b, sk->d, std::min(slab, sk->m - k0), tu);
    const WsSpec sk_spec = ws_spec(gk, sk->n1, sk->n3, safe, op.flags);
    rc = enqueue_product(c, sk, slab_operands(op, k0), gk, sk_spec, ptr, pdev, s,
                         k0 == 0 ? sk->c64 : csum, false);
    if (rc == CMM_OK && k0 > 0 &&
        cmm::launch_add_f64(sk->c64, csum, (int64_t)sk->d * sk->b, s) != hipSuccess)
      rc = fail(c, CMM_EHIP, "slab sum launch failed");
    if (rc == CMM_OK && k0 + slab >= sk->m &&
        cmm::launch_to_f32(sk->c64, sk->c32, (int64_t)sk->d * sk->b, s) != hipSuccess)
      rc = fail(c, CMM_EHIP, "float32 copy launch failed");
  }
  *overflowed = false;
  if (rc == CMM_OK && !async) {
    hipError_t e1 = hipMemcpyAsync(c->pinned_u32, ptr.p[W_OFLOW], sizeof(int32_t),
                                   hipMemcpyDeviceToHost, s);
    hipError_t e2 = hipStreamSynchronize(s);
    if (e1 != hipSuccess || e2 != hipSuccess) rc = fail(c, CMM_EHIP, "stream synchronisation failed");
    else *overflowed = c->pinned_u32[0] != 0;
  }
  if (rc == CMM_OK && !async && c->prof && op.dtype != cmm::kSparseF32)
    rc = account_countsketch(c, sk, op, g, ptr, s);
  ws_release(c, owned);   // stream-ordered reuse: later work on this stream follows
  return rc;
}

// Device buffers of a sketch whose sizes are set (frees what it got on failure).
bool alloc_sketch(cmm_sketch* sk) {
  cmm_ctx* c = sk->ctx;
  sk->hs1 = (int32_t*)dalloc(c, sizeof(int32_t) * sk->d * sk->n1);
  sk->hs2 = (int32_t*)dalloc(c, sizeof(int32_t) * sk->d * sk->n3);
  sk->c64 = (double*)dalloc(c, sizeof(double) * sk->d * sk->b);
  sk->c32 = (float*)dalloc(c, sizeof(float) * sk->d * sk->b);
  if (sk->hs1 && sk->hs2 && sk->c64 && sk->c32) return true;
  dfree(c, sk->hs1); dfree(c, sk->hs2); dfree(c, sk->c64); dfree(c, sk->c32);
  sk->hs1 = sk->hs2 = nullptr; sk->c64 = nullptr; sk->c32 = nullptr;
  return false;
}

void release_sketch(cmm_sketch* sk) {
  cmm_ctx* c = sk->ctx;
  dfree(c, sk->hs1); dfree(c, sk->hs2); dfree(c, sk->c64); dfree(c, sk->c32);
  sk->magic = kDeadMagic;
  delete sk;
}

int product_common(cmm_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                   int64_t n1, int64_t m, int64_t n3, int32_t dtype, const float* scaleA,
                   const float* scaleB, int64_t b, int32_t d, uint64_t seed,
                   const uint64_t* hash_params, const int32_t* th1, const int8_t* ts1,
                   const int32_t* th2, const int8_t* ts2, uint32_t flags, cmm_sketch** out,
                   const Operands* sparse = nullptr) {
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
  if (!alloc_sketch(sk)) {
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
  Operands op{A, lda, B, ldb, dtype, scaleA, scaleB, flags};
  if (sparse) {
    op.dtype = cmm::kSparseF32;
    op.aptr = sparse->aptr; op.aidx = sparse->aidx; op.bptr = sparse->bptr; op.bidx = sparse->bidx;
  }
  const cmm::Tuning tu = lookup_tuning(ctx, n1, m, n3, b, d, dtype);
  rc = run_product(ctx, sk, op, tu, false, &over);
  if (rc == CMM_OK && over) rc = run_product(ctx, sk, op, tu, true, &over);
  if (rc != CMM_OK) { cmm_sketch_free(sk); return rc; }
  *out = sk;
  return CMM_OK;
}

TuneKey tune_key(int64_t n1, int64_t m, int64_t n3, int64_t b, int d, int dtype) {
  return TuneKey{ilog2(b), ilog2(n1), ilog2(m), ilog2(n3), d, dtype};
}

cmm::Tuning lookup_tuning(const cmm_ctx* c, int64_t n1, int64_t m, int64_t n3, int64_t b, int d,
                          int dtype) {
  auto it = c->tuning.find(tune_key(n1, m, n3, b, d, dtype));
  return it != c->tuning.end() ? it->second.tu : default_tuning(b);
}

bool valid_tuning(const cmm::Tuning& t) {
  return t.log2c >= 4 && t.log2c <= cmm::kMaxLog2C && t.kmax >= 1 && t.kmax <= cmm::kMaxKPerBlock &&
         t.cs_blocks >= 1 && t.cs_blocks <= (1 << 20);
}

int check_dims(cmm_ctx* c, int64_t n1, int64_t m, int64_t n3, int64_t b, int32_t d, int32_t dtype) {
  static const char dummy = 0;
  return check_operands(c, &dummy, n1, &dummy, n3, n1, m, n3, dtype, b, d);
}

// Mean time of one product under tuning `tu` on the synthetic operands of
// `sk` (5 back-to-back runs after a warm-up run on the context stream).
// With `cs_only` the timed runs are the two count-sketch launches alone, 10
// pairs after the warm-up product has built the layout they read: the
// number of count-sketch blocks changes nothing else, and its effect is a
// few per cent of a product, below the noise of whole-product timing.
int time_candidate(cmm_ctx* c, cmm_sketch* sk, const Operands& op, const cmm::Tuning& tu,
                   const uint64_t* pdev, hipEvent_t ev0, hipEvent_t ev1, double* ms,
                   bool cs_only = false) {
  hipStream_t s = c->stream;
  const cmm::Geometry g = make_geometry(sk->b, sk->d, sk->m, tu);
  for (int attempt = 0; attempt < 2; ++attempt) {
    const WsSpec spec = ws_spec(g, sk->n1, sk->n3, attempt == 1, op.flags);
    WsPtrs ptr;
    std::vector<void*> owned;
    int rc = ws_alloc(c, spec, ptr, owned);
    if (rc == CMM_OK) rc = enqueue_product(c, sk, op, g, spec, ptr, pdev, s);
    if (rc == CMM_OK && hipMemcpyAsync(c->pinned_u32, ptr.p[W_OFLOW], sizeof(int32_t),
                                       hipMemcpyDeviceToHost, s) != hipSuccess)
      rc = fail(c, CMM_EHIP, "overflow flag copy failed");
    if (rc == CMM_OK && hipStreamSynchronize(s) != hipSuccess)
      rc = fail(c, CMM_EHIP, "stream synchronisation failed");
    if (rc == CMM_OK && c->pinned_u32[0] != 0 && attempt == 0) { ws_release(c, owned); continue; }
    const int reps = cs_only ? 10 : 5;
    cmm::SideDesc side[2];
    if (cs_only) bind_sides(g, sk, op, spec, ptr, side);
    if (rc == CMM_OK && hipEventRecord(ev0, s) != hipSuccess) rc = fail(c, CMM_EHIP, "event record failed");
    for (int r = 0; r < reps && rc == CMM_OK; ++r) {
      if (!cs_only) { rc = enqueue_product(c, sk, op, g, spec, ptr, pdev, s); continue; }
      for (int q = 0; q < 2 && rc == CMM_OK; ++q)
        if (cmm::launch_countsketch(op.dtype, g, side[q], s) != hipSuccess)
          rc = fail(c, CMM_EHIP, "countsketch launch failed");
    }
    if (rc == CMM_OK && hipEventRecord(ev1, s) != hipSuccess) rc = fail(c, CMM_EHIP, "event record failed");
    if (rc == CMM_OK && hipEventSynchronize(ev1) != hipSuccess) rc = fail(c, CMM_EHIP, "event wait failed");
    float t = 0.f;
    if (rc == CMM_OK && hipEventElapsedTime(&t, ev0, ev1) != hipSuccess) rc = fail(c, CMM_EHIP, "event time failed");
    if (rc == CMM_OK) *ms = t / reps;
    (void)hipStreamSynchronize(s);
    ws_release(c, owned);
    return rc;
  }
  return fail(c, CMM_EHIP, "layout overflow with the safe layout");
}

// Coordinate search over the geometry of one size class: the FFT row
// length first, then the number of k per spectral block (both timed as
// whole products), then the number of count-sketch blocks (timed on the
// count-sketch launches alone), starting from the built-in default;
// candidates that give the same launch shapes as one already timed are
// skipped, and a candidate replaces the incumbent only when at least 3 %
// faster.  The recorded time is that of a whole product with the result.
int autotune_class(cmm_ctx* c, int64_t n1, int64_t m, int64_t n3, int64_t b, int d, int dtype,
                   TuneEntry* best) {
  hipStream_t s = c->stream;
  const size_t esz = dtype == CMM_F32 ? 4 : (dtype == CMM_BF16 ? 2 : 1);
  Work w(c);
  void* A = w.get<uint8_t>(esz * n1 * m);
  void* B = w.get<uint8_t>(esz * m * n3);
  uint64_t* pdev = w.get<uint64_t>((size_t)d * 8);
  if (!A || !B || !pdev) return fail(c, CMM_ENOMEM, "autotune operand allocation failed");
  CMM_HIP(c, cmm::launch_fill_random(A, n1 * m, dtype, 0x243F6A8885A308D3ull, s));
  CMM_HIP(c, cmm::launch_fill_random(B, m * n3, dtype, 0x13198A2E03707344ull, s));
  cmm_sketch* sk = new cmm_sketch();
  sk->ctx = c; sk->n1 = n1; sk->m = m; sk->n3 = n3; sk->b = b; sk->d = d; sk->log2b = ilog2(b);
  sk->has_params = true;
  params_from_seed(0xA4093822299F31D0ull, d, sk->params);
  if (!alloc_sketch(sk)) { delete sk; return fail(c, CMM_ENOMEM, "autotune sketch allocation failed"); }
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int rc = CMM_OK;
  if (hipMemcpyAsync(pdev, sk->params.data(), sizeof(uint64_t) * d * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess)
    rc = fail(c, CMM_EHIP, "autotune set-up failed");
  const bool prof = c->prof;
  c->prof = false;
  const Operands op{A, n1, B, n3, dtype, nullptr, nullptr, 0};
  cmm::Tuning cur = default_tuning(b);
  double cur_ms = 0.0;
  // the class's first timing also pays for clocks still ramping up after an
  // idle GPU; it is taken twice and the second kept, so that a candidate has
  // to beat the default at the same clocks
  for (int pass = 0; pass < 2 && rc == CMM_OK; ++pass)
    rc = time_candidate(c, sk, op, cur, pdev, ev0, ev1, &cur_ms);
  auto shape = [&](const cmm::Tuning& t) {
    const cmm::Geometry g = make_geometry(b, d, m, t);
    const int kb = std::max<int>(1, (int)(m / g.cs_blocks));
    return std::make_tuple(g.log2c, g.KS, (int)((m + kb - 1) / kb));
  };
  std::vector<std::tuple<int, int, int>> seen{shape(cur)};
  for (int axis = 0; axis < 3 && rc == CMM_OK; ++axis) {
    const std::vector<int> vals = axis == 0 ? std::vector<int>{10, 11, 12, 13}
                                : axis == 1 ? std::vector<int>{32, 48, 64, 128}
                                            : std::vector<int>{512, 1024, 2048, 4096};
    const bool cs_only = axis == 2;
    const cmm::Tuning base = cur;
    double base_ms = cur_ms;
    if (cs_only) rc = time_candidate(c, sk, op, base, pdev, ev0, ev1, &base_ms, true);
    for (int v : vals) {
      if (rc != CMM_OK) break;
      cmm::Tuning t = base;
      (axis == 0 ? t.log2c : axis == 1 ? t.kmax : t.cs_blocks) = v;
      const auto sh = shape(t);
      if (std::find(seen.begin(), seen.end(), sh) != seen.end()) continue;
      seen.push_back(sh);
      double ms = 0.0;
      rc = time_candidate(c, sk, op, t, pdev, ev0, ev1, &ms, cs_only);
      if (rc != CMM_OK) break;
      // a candidate must be clearly faster than the incumbent (timing noise
      // between runs is a few per cent)
      if (ms < 0.97 * base_ms) { cur = t; base_ms = ms; if (!cs_only) cur_ms = ms; }
    }
    if (rc == CMM_OK && cs_only && cur.cs_blocks != base.cs_blocks)
      rc = time_candidate(c, sk, op, cur, pdev, ev0, ev1, &cur_ms);
  }
  c->prof = prof;
  (void)hipStreamSynchronize(s);
  if (ev0) hipEventDestroy(ev0);
  if (ev1) hipEventDestroy(ev1);
  release_sketch(sk);
  if (rc == CMM_OK) { best->tu = cur; best->ms = cur_ms; }
  return rc;
}

const char* device_arch(cmm_ctx* c) {
  if (c->arch.empty()) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
      std::string a = prop.gcnArchName;
      c->arch = a.substr(0, a.find(':'));
    } else {
      c->arch = "unknown";
    }
  }
  return c->arch.c_str();
}

int load_tuning(cmm_ctx* c, const char* path, bool missing_ok) {
  FILE* f = std::fopen(path, "r");
  if (!f) return missing_ok ? CMM_OK : fail(c, CMM_EINVAL, std::string("cannot open ") + path);
  const std::string arch = device_arch(c);
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    char a[64] = {0};
    TuneKey k;
    TuneEntry e;
    const int got = std::sscanf(line,
        " {\"arch\": \"%63[^\"]\", \"log2b\": %d, \"ln1\": %d, \"lm\": %d, \"ln3\": %d, \"d\": %d, "
        "\"dtype\": %d, \"log2c\": %d, \"kmax\": %d, \"cs_blocks\": %d, \"ms\": %lf}",
        a, &k.log2b, &k.ln1, &k.lm, &k.ln3, &k.d, &k.dtype, &e.tu.log2c, &e.tu.kmax,
        &e.tu.cs_blocks, &e.ms);
    if (got != 11 || arch != a || !valid_tuning(e.tu)) continue;
    c->tuning[k] = e;
  }
  std::fclose(f);
  return CMM_OK;
}

}  // namespace

// A set of products recorded into one HIP graph.
struct cmm_batch {
  static constexpr int kMaxBranches = 4;
  uint32_t magic = kBatchMagic;
  cmm_ctx* ctx = nullptr;
  std::vector<cmm_sketch*> sk;
  std::vector<void*> owned;   // workspaces and hash parameters (context cache blocks)
  int nbranch = 0;
  hipStream_t streams[kMaxBranches] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kMaxBranches] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

bool valid_batch(const cmm_batch* b) { return b && b->magic == kBatchMagic && valid_ctx(b->ctx); }

// Release everything of a batch; its sketches are deleted too unless
// `keep_sketches`, which hands them over as ordinary sketches.
void destroy_batch(cmm_batch* bt, bool keep_sketches) {
  cmm_ctx* c = bt->ctx;
  (void)hipStreamSynchronize(c->stream);
  if (bt->exec) hipGraphExecDestroy(bt->exec);
  if (bt->graph) hipGraphDestroy(bt->graph);
  for (int q = 0; q < cmm_batch::kMaxBranches; ++q) {
    if (bt->streams[q]) { (void)hipStreamSynchronize(bt->streams[q]); hipStreamDestroy(bt->streams[q]); }
    if (bt->join[q]) hipEventDestroy(bt->join[q]);
  }
  if (bt->fork) hipEventDestroy(bt->fork);
  for (void* p : bt->owned) dfree(c, p);
  for (cmm_sketch* sk : bt->sk) {
    if (keep_sketches) sk->owner = nullptr;
    else release_sketch(sk);
  }
  bt->magic = kDeadMagic;
  delete bt;
}

struct BatchItem {
  cmm::Geometry g;
  WsSpec spec;
  Operands op;
  const uint64_t* pdev = nullptr;
  double cost = 0.0;
  int branch = 0;
};

// Relative cost of a product for spreading a batch over graph branches:
// spectral work (a C-point FFT per row, per k and side) plus the fold and
// count-sketch work over the hashed entries.
double product_cost(const cmm::Geometry& g, int64_t n1, int64_t n3) {
  const double C = (double)(1 << g.log2c);
  return (double)g.d * g.m * (2.0 * g.rblocks * C * g.log2c + 8.0 * (n1 + n3));
}

int build_batch(cmm_ctx* c, const cmm_problem* pr, int count, uint32_t flags, cmm_batch* bt) {
  hipStream_t s = c->stream;
  std::vector<BatchItem> it(count);
  // sketches, hash parameters, geometry, twiddle tables
  for (int i = 0; i < count; ++i) {
    const cmm_problem& p = pr[i];
    cmm_sketch* sk = new cmm_sketch();
    sk->ctx = c; sk->n1 = p.n1; sk->m = p.m; sk->n3 = p.n3; sk->b = p.b; sk->d = p.d;
    sk->log2b = ilog2(p.b);
    sk->has_params = true;
    params_from_seed(p.seed, p.d, sk->params);
    if (!alloc_sketch(sk)) { delete sk; return fail(c, CMM_ENOMEM, "sketch allocation failed"); }
    sk->owner = bt;
    bt->sk.push_back(sk);
    uint64_t* pdev = (uint64_t*)dalloc(c, sizeof(uint64_t) * p.d * 8);
    if (!pdev) return fail(c, CMM_ENOMEM, "parameter buffer allocation failed");
    bt->owned.push_back(pdev);
    CMM_HIP(c, hipMemcpyAsync(pdev, sk->params.data(), sizeof(uint64_t) * p.d * 8,
                              hipMemcpyHostToDevice, s));
    if ((flags & CMM_AUTOTUNE) && !c->tuning.count(tune_key(p.n1, p.m, p.n3, p.b, p.d, p.dtype))) {
      // tune the class on its largest problem (the one that costs most)
      const TuneKey key = tune_key(p.n1, p.m, p.n3, p.b, p.d, p.dtype);
      const cmm_problem* big = &p;
      for (int q = i + 1; q < count; ++q) {
        const cmm_problem& o = pr[q];
        if (tune_key(o.n1, o.m, o.n3, o.b, o.d, o.dtype) < key || key < tune_key(o.n1, o.m, o.n3, o.b, o.d, o.dtype))
          continue;
        if ((double)o.n1 * o.m * o.n3 > (double)big->n1 * big->m * big->n3) big = &o;
      }
      TuneEntry e;
      int rc = autotune_class(c, big->n1, big->m, big->n3, big->b, big->d, big->dtype, &e);
      if (rc) return rc;
      c->tuning[key] = e;
    }
    it[i].g = make_geometry(p.b, p.d, p.m, lookup_tuning(c, p.n1, p.m, p.n3, p.b, p.d, p.dtype));
    it[i].op = Operands{p.A, p.lda, p.B, p.ldb, p.dtype, p.scaleA, p.scaleB, p.flags};
    it[i].pdev = pdev;
    it[i].cost = product_cost(it[i].g, p.n1, p.n3);
    double2* t64; float2* t32;
    int rc = get_twiddles(c, p.b, &t64, &t32);
    if (rc) return rc;
  }
  // bucket layouts: the hash functions fix them, so one layout pass per
  // problem decides whether the compact segment capacity holds for good
  for (int i = 0; i < count; ++i) {
    BatchItem& x = it[i];
    WsSpec probe = ws_spec(x.g, pr[i].n1, pr[i].n3, false, 0);
    for (int k : {W_SA0, W_SA1, W_CMAX0, W_CMAX1, W_PPART, W_WORK0, W_WORK1}) probe.count[k] = 0;
    WsPtrs ptr;
    std::vector<void*> owned;
    int rc = ws_alloc(c, probe, ptr, owned);
    cmm::SideDesc side[2];
    if (rc == CMM_OK) {
      bind_sides(x.g, bt->sk[i], x.op, probe, ptr, side);
      rc = enqueue_layout(c, x.g, side, x.pdev, (int32_t*)ptr.p[W_OFLOW], s);
    }
    if (rc == CMM_OK && (hipMemcpyAsync(c->pinned_u32, ptr.p[W_OFLOW], sizeof(int32_t),
                                        hipMemcpyDeviceToHost, s) != hipSuccess ||
                         hipStreamSynchronize(s) != hipSuccess))
      rc = fail(c, CMM_EHIP, "layout pass failed");
    ws_release(c, owned);
    if (rc) return rc;
    x.spec = ws_spec(x.g, pr[i].n1, pr[i].n3, c->pinned_u32[0] != 0, pr[i].flags);
  }
  // longest product first onto the least loaded branch
  bt->nbranch = std::min(count, (int)cmm_batch::kMaxBranches);
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b2) { return it[a].cost > it[b2].cost; });
  std::vector<double> load(bt->nbranch, 0.0);
  for (int i : order) {
    const int br = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    it[i].branch = br;
    load[br] += it[i].cost;
  }
  // one workspace per branch, each buffer as large as its largest user
  std::vector<WsPtrs> ws(bt->nbranch);
  for (int br = 0; br < bt->nbranch; ++br) {
    WsSpec mx;
    for (int i = 0; i < count; ++i)
      if (it[i].branch == br)
        for (int k = 0; k < W_COUNT; ++k) mx.count[k] = std::max(mx.count[k], it[i].spec.count[k]);
    int rc = ws_alloc(c, mx, ws[br], bt->owned);
    if (rc) return rc;
  }
  for (int br = 0; br < bt->nbranch; ++br) {
    CMM_HIP(c, hipStreamCreateWithFlags(&bt->streams[br], hipStreamNonBlocking));
    CMM_HIP(c, hipEventCreateWithFlags(&bt->join[br], hipEventDisableTiming));
  }
  CMM_HIP(c, hipEventCreateWithFlags(&bt->fork, hipEventDisableTiming));
  CMM_HIP(c, hipStreamSynchronize(s));
  // capture: branch 0 forks the others and joins them at the end
  hipStream_t s0 = bt->streams[0];
  const bool prof = c->prof;
  c->prof = false;
  int rc = CMM_OK;
  if (hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    c->prof = prof;
    return fail(c, CMM_EHIP, "hipStreamBeginCapture failed");
  }
  if (hipEventRecord(bt->fork, s0) != hipSuccess) rc = fail(c, CMM_EHIP, "fork record failed");
  for (int br = 1; br < bt->nbranch && rc == CMM_OK; ++br)
    if (hipStreamWaitEvent(bt->streams[br], bt->fork, 0) != hipSuccess)
      rc = fail(c, CMM_EHIP, "fork wait failed");
  for (int i : order) {
    if (rc) break;
    rc = enqueue_product(c, bt->sk[i], it[i].op, it[i].g, it[i].spec, ws[it[i].branch],
                         it[i].pdev, bt->streams[it[i].branch]);
  }
  for (int br = 1; br < bt->nbranch; ++br) {
    (void)hipEventRecord(bt->join[br], bt->streams[br]);
    (void)hipStreamWaitEvent(s0, bt->join[br], 0);
  }
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(s0, &graph);
  c->prof = prof;
  bt->graph = graph;
  if (rc) return rc;
  if (ec != hipSuccess || !graph) return fail(c, CMM_EHIP, std::string("graph capture failed: ") + hipGetErrorString(ec));
  CMM_HIP(c, hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0));
  return CMM_OK;
}

cmm::DecodeDesc decode_desc(const cmm_sketch* sk) {
  cmm::DecodeDesc dd;
  dd.hs1 = sk->hs1; dd.hs2 = sk->hs2; dd.c32 = sk->c32;
  dd.n1 = (int)sk->n1; dd.n3 = (int)sk->n3; dd.d = sk->d;
  dd.mask = (uint32_t)(sk->b - 1); dd.b = sk->b;
  return dd;
}

// One request of topk_many: a sketch, its K and host destinations.
struct TopkJob {
  const cmm_sketch* sk;
  int32_t K;
  int64_t* out_i;
  int64_t* out_j;
  float* out_val;
};

// Top-K (cmm_topk's semantics) of several sketches of context `c`, on its
// stream.  Each phase is issued for every sketch before the single host wait
// it needs, so n sketches cost the round trips of one; a sketch whose fast
// path does not settle runs the digit passes with waits of its own.
int topk_many(cmm_ctx* c, int mode, const std::vector<TopkJob>& jobs) {
  if (mode != CMM_TOPK_ALL && mode != CMM_TOPK_UPPER && mode != CMM_TOPK_PER_COLUMN)
    return fail(c, CMM_EINVAL, "unknown mode");
  const size_t n = jobs.size();
  std::vector<int64_t> domain(n, 0);
  for (size_t q = 0; q < n; ++q) {
    const TopkJob& jb = jobs[q];
    const cmm_sketch* sk = jb.sk;
    if (!jb.out_i || !jb.out_j || !jb.out_val) return fail(c, CMM_EINVAL, "output arrays are NULL");
    if (jb.K < 1) return fail(c, CMM_EINVAL, "K < 1");
    if (mode == CMM_TOPK_PER_COLUMN) {
      if (jb.K > sk->n1) return fail(c, CMM_EINVAL, "K larger than a column");
      continue;
    }
    int64_t dom = sk->n1 * sk->n3;
    if (mode == CMM_TOPK_UPPER) {
      dom = 0;
      for (int64_t i = 0; i < sk->n1; ++i) dom += std::max<int64_t>(0, sk->n3 - i - 1);
    }
    domain[q] = dom;
    if (jb.K > dom) return fail(c, CMM_EINVAL, "K larger than the candidate domain");
    if (jb.K > cmm::kTopkCap / 2) return fail(c, CMM_EUNSUPPORTED, "K above 2048");
  }
  hipStream_t s = c->stream;
  Work w(c);
  std::vector<Download> dl;
  if (mode == CMM_TOPK_PER_COLUMN) {
    {
      Scope sc_(c, "decode");
      for (size_t q = 0; q < n; ++q) {
        const TopkJob& jb = jobs[q];
        const size_t tot = (size_t)jb.K * jb.sk->n3;
        int64_t* oi = w.get<int64_t>(tot);
        float* ov = w.get<float>(tot);
        if (!oi || !ov) return fail(c, CMM_ENOMEM, "workspace allocation failed");
        CMM_HIP(c, cmm::launch_topk_column(decode_desc(jb.sk), jb.K, oi, ov, s));
        dl.push_back({jb.out_i, oi, sizeof(int64_t) * tot});
        dl.push_back({jb.out_val, ov, sizeof(float) * tot});
      }
    }
    const int rc = download_n(c, s, dl.data(), dl.size());
    if (rc) return rc;
    for (const TopkJob& jb : jobs)
      for (int64_t jj = 0; jj < jb.sk->n3; ++jj)
        for (int r = 0; r < jb.K; ++r) jb.out_j[jj * jb.K + r] = jj;
    return CMM_OK;
  }
  constexpr int kWide = 16384;   // candidates kept by the fused histogram + collect pass
  struct State {
    cmm::DecodeDesc dd;
    int tiles = 0, b0 = -1;
    bool done = false;
    uint32_t* hist = nullptr;
    uint32_t* count = nullptr;
    cmm::TopkCand* wide = nullptr;
    cmm::TopkCand* cand = nullptr;
    int64_t* oi = nullptr;
    int64_t* oj = nullptr;
    float* ov = nullptr;
    int log2w = 0;                 // screening bitmap width (0: none)
    uint32_t* bits = nullptr;
    std::vector<uint32_t> h;
  };
  std::vector<State> st(n);
  for (size_t q = 0; q < n; ++q) {
    State& x = st[q];
    const TopkJob& jb = jobs[q];
    x.dd = decode_desc(jb.sk);
    x.tiles = (int)((jb.sk->n1 + 15) / 16);
    x.hist = w.get<uint32_t>(4096);
    x.count = w.get<uint32_t>(2);
    x.wide = w.get<cmm::TopkCand>(kWide);
    x.cand = w.get<cmm::TopkCand>(cmm::kTopkCap);
    x.oi = w.get<int64_t>(jb.K);
    x.oj = w.get<int64_t>(jb.K);
    x.ov = w.get<float>(jb.K);
    x.log2w = cmm::screen_log2w(x.dd.d, x.dd.b);
    if (x.log2w > 0) x.bits = w.get<uint32_t>((size_t)cmm::screen_nf(x.dd.d) << (x.log2w - 5));
    if (!x.hist || !x.count || !x.wide || !x.cand || !x.oi || !x.oj || !x.ov || (x.log2w > 0 && !x.bits))
      return fail(c, CMM_ENOMEM, "workspace allocation failed");
    x.h.assign(4096, 0u);
  }
  {
    Scope sc_(c, "decode");
    // Fast path: a pass over every 16th row tile estimates a threshold T0
    // above which about 2K + 64 estimates lie; one full pass then builds the
    // exact histogram of the top 12 key bits of the keys >= T0 and keeps
    // those candidates.  The histogram shows whether T0 is at or below the
    // K-th key and whether the kept set is complete; otherwise the
    // digit-by-digit passes below run.
    dl.clear();
    for (State& x : st) {
      if (x.tiles < 64) continue;
      CMM_HIP(c, cmm::launch_fill_i32((int32_t*)x.hist, 4096, 0, s));
      CMM_HIP(c, cmm::launch_topk_hist(x.dd, mode, 16, 0, 32, 19, 0xFFF, x.hist, 0, nullptr, nullptr, 0, s));
      dl.push_back({x.h.data(), x.hist, 4096 * sizeof(uint32_t)});
    }
    if (!dl.empty()) { const int rc_ = download_n(c, s, dl.data(), dl.size()); if (rc_) return rc_; }
    dl.clear();
    for (size_t q = 0; q < n; ++q) {
      State& x = st[q];
      if (x.tiles < 64) continue;
      int64_t sampled = 0;
      for (uint32_t v : x.h) sampled += v;
      if (sampled <= 0) continue;
      const double want = (2.0 * jobs[q].K + 64.0) * (double)sampled / (double)domain[q];
      int64_t cum = 0;
      for (int b = 4095; b >= 0; --b) {
        cum += x.h[b];
        if (cum >= 8 && (double)cum >= want) { x.b0 = b; break; }
      }
      if (x.b0 < 0) continue;
      const uint32_t T0 = (uint32_t)x.b0 << 19;
      CMM_HIP(c, cmm::launch_fill_i32((int32_t*)x.hist, 4096, 0, s));
      CMM_HIP(c, cmm::launch_fill_i32((int32_t*)x.count, 2, 0, s));
      if (x.log2w > 0) CMM_HIP(c, cmm::launch_screen_bits(x.dd, T0, x.log2w, x.bits, s));
      CMM_HIP(c, cmm::launch_topk_hist(x.dd, mode, 1, 0, 32, 19, 0xFFF, x.hist, T0, x.wide, x.count, kWide, s,
                                       x.bits, x.log2w));
      dl.push_back({x.h.data(), x.hist, 4096 * sizeof(uint32_t)});
    }
    if (!dl.empty()) { const int rc_ = download_n(c, s, dl.data(), dl.size()); if (rc_) return rc_; }
    for (size_t q = 0; q < n; ++q) {
      State& x = st[q];
      if (x.b0 < 0) continue;
      const int K = jobs[q].K;
      // h counts only keys >= T0 (bins b0 and up): exact there
      int64_t n0 = 0;
      for (int b = x.b0; b < 4096; ++b) n0 += x.h[b];
      if (n0 < K || n0 > kWide) continue;
      int64_t cum = 0;
      int bk = 4095;
      for (; bk >= 0; --bk) { cum += x.h[bk]; if (cum >= K) break; }
      if (n0 <= cmm::kTopkCap) {
        CMM_HIP(c, cmm::launch_topk_final(x.wide, x.count, cmm::kTopkCap, K, x.dd.n3, x.oi, x.oj, x.ov, s));
        x.done = true;
      } else if (cum <= cmm::kTopkCap) {
        CMM_HIP(c, cmm::launch_topk_filter(x.wide, x.count, kWide, (uint32_t)bk << 19, x.cand, x.count + 1,
                                           cmm::kTopkCap, s));
        CMM_HIP(c, cmm::launch_topk_final(x.cand, x.count + 1, cmm::kTopkCap, K, x.dd.n3, x.oi, x.oj, x.ov, s));
        x.done = true;
      }
    }
    for (size_t q = 0; q < n; ++q) {
      State& x = st[q];
      if (x.done) continue;
      // digit passes: bits [30:19], [18:7], [6:0]
      const int dshift[3] = {19, 7, 0};
      const uint32_t dmask[3] = {0xFFF, 0xFFF, 0x7F};
      uint32_t prefix = 0;
      int pshift = 32;
      int64_t above = 0;
      int64_t need = jobs[q].K;
      uint32_t thresh = 0;
      bool found = false;
      for (int level = 0; level < 3 && !found; ++level) {
        CMM_HIP(c, cmm::launch_fill_i32((int32_t*)x.hist, 4096, 0, s));
        CMM_HIP(c, cmm::launch_topk_hist(x.dd, mode, 1, prefix, pshift, dshift[level], dmask[level], x.hist,
                                         0, nullptr, nullptr, 0, s));
        { const int rc_ = download(c, s, {{x.h.data(), x.hist, 4096 * sizeof(uint32_t)}}); if (rc_) return rc_; }
        int64_t cum = 0;
        int bin = -1;
        for (int b = (int)dmask[level]; b >= 0; --b) {
          if (cum + x.h[b] >= need) { bin = b; break; }
          cum += x.h[b];
        }
        if (bin < 0) return fail(c, CMM_EHIP, "top-K histogram lost entries");
        prefix |= (uint32_t)bin << dshift[level];
        const int64_t total = above + cum + x.h[bin];
        if (total <= cmm::kTopkCap) { thresh = prefix; found = true; break; }
        above += cum;
        need -= cum;
        pshift = dshift[level];
      }
      if (!found) return fail(c, CMM_EUNSUPPORTED, "more than 4096 estimates tie at the K-th magnitude");
      CMM_HIP(c, cmm::launch_fill_i32((int32_t*)x.count, 1, 0, s));
      CMM_HIP(c, cmm::launch_topk_collect(x.dd, mode, thresh, x.cand, x.count, cmm::kTopkCap, s));
      CMM_HIP(c, cmm::launch_topk_final(x.cand, x.count, cmm::kTopkCap, jobs[q].K, x.dd.n3, x.oi, x.oj, x.ov, s));
    }
  }
  dl.clear();
  for (size_t q = 0; q < n; ++q) {
    const TopkJob& jb = jobs[q];
    dl.push_back({jb.out_i, st[q].oi, sizeof(int64_t) * jb.K});
    dl.push_back({jb.out_j, st[q].oj, sizeof(int64_t) * jb.K});
    dl.push_back({jb.out_val, st[q].ov, sizeof(float) * jb.K});
  }
  return download_n(c, s, dl.data(), dl.size());
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
  if (hipHostMalloc((void**)&c->pinned_u32, 64 * sizeof(uint32_t)) != hipSuccess ||
      hipHostMalloc((void**)&c->pinned, kPinnedBytes) != hipSuccess) {
    if (c->pinned_u32) hipHostFree(c->pinned_u32);
    delete c;
    return CMM_ENOMEM;
  }
  c->pinned_cap = kPinnedBytes;
  size_t mem_free = 0, mem_total = 0;
  c->ws_default = hipMemGetInfo(&mem_free, &mem_total) == hipSuccess && mem_total > 0
                      ? (int64_t)(mem_total / 2) : (int64_t)64 << 30;
  if (cmm::prepare_countsketch() != hipSuccess || cmm::prepare_fft_mac() != hipSuccess ||
      cmm::prepare_sparse() != hipSuccess || cmm::prepare_decode() != hipSuccess ||
      hipStreamCreateWithFlags(&c->ov.aux, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ov.fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ov.join, hipEventDisableTiming) != hipSuccess) {
    destroy_overlap(c->ov);
    hipHostFree(c->pinned_u32);
    hipHostFree(c->pinned);
    delete c;
    return CMM_EHIP;
  }
  if (const char* path = std::getenv("CMM_TUNE_CACHE")) load_tuning(c, path, true);
  bind_scratch(device);   // device is current here
  *out = c;
  return CMM_OK;
}

int cmm_ctx_set_workspace_limit(cmm_ctx* ctx, int64_t bytes) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  if (bytes < 0) return fail(ctx, CMM_EINVAL, "workspace limit must be >= 0");
  ctx->ws_limit = bytes;
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
  destroy_overlap(ctx->ov);
  for (auto& p : ctx->pending) { hipEventDestroy(p.a); hipEventDestroy(p.b); }
  for (hipEvent_t e : ctx->event_pool) hipEventDestroy(e);
  for (auto& kv : ctx->sizes) hipFree(kv.first);
  for (auto& kv : ctx->twiddles) { hipFree(kv.second.first); hipFree(kv.second.second); }
  if (ctx->pinned_u32) hipHostFree(ctx->pinned_u32);
  if (ctx->pinned) hipHostFree(ctx->pinned);
  ctx->magic = kDeadMagic;
  delete ctx;
  return CMM_OK;
}

int cmm_ctx_profile(cmm_ctx* ctx, int enable) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  drain_profile(ctx);
  ctx->prof = enable != 0;
  ctx->prof_acc.clear();
  ctx->prof_bytes.clear();
  return CMM_OK;
}

int cmm_ctx_profile_bytes(cmm_ctx* ctx, const char* name, double* read_bytes, double* written_bytes) {
  if (!valid_ctx(ctx) || !name) return CMM_EINVAL;
  auto it = ctx->prof_bytes.find(name);
  if (read_bytes) *read_bytes = it == ctx->prof_bytes.end() ? 0.0 : it->second.first;
  if (written_bytes) *written_bytes = it == ctx->prof_bytes.end() ? 0.0 : it->second.second;
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

int cmm_stream_probe(cmm_ctx* ctx, int64_t read_bytes, int64_t write_bytes, int32_t nontemporal,
                     int32_t reps, double* ms_per_launch) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  if (read_bytes < 0 || write_bytes < 0 || (read_bytes == 0 && write_bytes == 0) ||
      read_bytes % 16 || write_bytes % 16 || reps < 1 || !ms_per_launch ||
      (read_bytes > 0 && write_bytes > 0 && write_bytes % read_bytes))
    return fail(ctx, CMM_EINVAL, "stream probe: sizes must be multiples of 16, write a multiple of read");
  CMM_HIP(ctx, hipSetDevice(ctx->device));
  void* src = nullptr;
  void* dst = nullptr;
  float* sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = CMM_OK;
  if ((read_bytes && hipMalloc(&src, (size_t)read_bytes) != hipSuccess) ||
      (write_bytes && hipMalloc(&dst, (size_t)write_bytes) != hipSuccess) ||
      hipMalloc((void**)&sink, 4096 * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    rc = fail(ctx, CMM_ENOMEM, "stream probe buffers");
  }
  if (rc == CMM_OK && src && hipMemsetAsync(src, 0, (size_t)read_bytes, ctx->stream) != hipSuccess)
    rc = fail(ctx, CMM_EHIP, "stream probe fill");
  if (rc == CMM_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = fail(ctx, CMM_EHIP, "stream probe events");
  const bool nt = nontemporal != 0;
  // one untimed launch, then `reps` timed ones
  if (rc == CMM_OK && cmm::launch_stream_probe(src, dst, sink, read_bytes, write_bytes, nt, ctx->stream) != hipSuccess)
    rc = fail(ctx, CMM_EHIP, "stream probe launch");
  if (rc == CMM_OK && hipEventRecord(e0, ctx->stream) != hipSuccess) rc = fail(ctx, CMM_EHIP, "event");
  for (int r = 0; rc == CMM_OK && r < reps; ++r)
    if (cmm::launch_stream_probe(src, dst, sink, read_bytes, write_bytes, nt, ctx->stream) != hipSuccess)
      rc = fail(ctx, CMM_EHIP, "stream probe launch");
  if (rc == CMM_OK && hipEventRecord(e1, ctx->stream) != hipSuccess) rc = fail(ctx, CMM_EHIP, "event");
  float ms = 0.0f;
  if (rc == CMM_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = fail(ctx, CMM_EHIP, "stream probe timing");
  if (rc == CMM_OK) *ms_per_launch = ms / reps;
  hipStreamSynchronize(ctx->stream);
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (src) hipFree(src);
  if (dst) hipFree(dst);
  if (sink) hipFree(sink);
  return rc;
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

int cmm_sketch_product_noalloc(cmm_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                               int64_t n1, int64_t m, int64_t n3, int32_t dtype,
                               const float* scaleA, const float* scaleB, int64_t b, int32_t d,
                               uint64_t seed, uint32_t flags, double* c_out) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  int rc = check_operands(ctx, A, lda, B, ldb, n1, m, n3, dtype, b, d);
  if (rc) return rc;
  if (!c_out) return fail(ctx, CMM_EINVAL, "c_out is NULL");
  if (flags & ~CMM_SUBTRACT_DIAG) return fail(ctx, CMM_EINVAL, "only CMM_SUBTRACT_DIAG is taken");
  if ((flags & CMM_SUBTRACT_DIAG) && n1 != n3)
    return fail(ctx, CMM_EINVAL, "CMM_SUBTRACT_DIAG needs n1 == n3");
  if (dtype != CMM_FP8_E4M3 && (scaleA || scaleB))
    return fail(ctx, CMM_EINVAL, "scales are only taken with CMM_FP8_E4M3");
  CMM_HIP(ctx, hipSetDevice(ctx->device));
  void* base = ctx->device < kMaxDevices ? g_scratch_dev[ctx->device] : nullptr;
  if (!base) {
    const hipError_t e = ctx->device < kMaxDevices ? g_scratch_err[ctx->device] : hipErrorInvalidDevice;
    return fail(ctx, CMM_EHIP, std::string("device scratch unavailable: ") + hipGetErrorString(e));
  }
  // the layout takes its safe segment capacity (no overflow, so no host wait)
  const cmm::Tuning tu = lookup_tuning(ctx, n1, m, n3, b, d, dtype);
  const cmm::Geometry g = make_geometry(b, d, m, tu);
  const WsSpec spec = ws_spec(g, n1, n3, true, flags);
  // carve every buffer from the scratch array at 256-byte boundaries
  size_t off = 0;
  auto carve = [&](size_t bytes) -> size_t {
    const size_t at = off;
    off += (bytes + 255) & ~(size_t)255;
    return at;
  };
  size_t at[W_COUNT] = {};
  for (int i = 0; i < W_COUNT; ++i) at[i] = carve(spec.count[i] * kElemSize[i]);
  const size_t at_hs1 = carve(sizeof(int32_t) * (size_t)d * n1);
  const size_t at_hs2 = carve(sizeof(int32_t) * (size_t)d * n3);
  const size_t at_par = carve(sizeof(uint64_t) * (size_t)d * 8);
  const size_t at_tw64 = carve(sizeof(double2) * (size_t)b);
  const size_t at_tw32 = carve(sizeof(float2) * (size_t)b);
  if (off > kScratchBytes)
    return fail(ctx, CMM_EUNSUPPORTED,
                "the allocation-free product needs " + std::to_string(off) + " bytes of device scratch; it holds " +
                    std::to_string(kScratchBytes) + " (use cmm_sketch_product_ex)");
  unsigned char* p = static_cast<unsigned char*>(base);
  WsPtrs ptr;
  for (int i = 0; i < W_COUNT; ++i) ptr.p[i] = spec.count[i] ? (void*)(p + at[i]) : nullptr;
  cmm_sketch sk;   // a view: tables in the scratch, the result in c_out
  sk.ctx = ctx; sk.n1 = n1; sk.m = m; sk.n3 = n3; sk.b = b; sk.d = d; sk.log2b = ilog2(b);
  sk.hs1 = (int32_t*)(p + at_hs1);
  sk.hs2 = (int32_t*)(p + at_hs2);
  sk.c64 = c_out;
  uint64_t* pdev = (uint64_t*)(p + at_par);
  double2* tw64 = (double2*)(p + at_tw64);
  float2* tw32 = (float2*)(p + at_tw32);
  const bool prof = ctx->prof;
  ctx->prof = false;   // no timing events: nothing is created here
  if (cmm::launch_params_from_seed(seed, d, pdev, ctx->stream) != hipSuccess ||
      cmm::launch_twiddles(tw64, tw32, b, ctx->stream) != hipSuccess)
    rc = fail(ctx, CMM_EHIP, "parameter or twiddle launch failed");
  const Operands op{A, lda, B, ldb, dtype, scaleA, scaleB, flags | CMM_ASYNC};
  if (rc == CMM_OK) rc = enqueue_product(ctx, &sk, op, g, spec, ptr, pdev, ctx->stream, c_out, false, tw64, tw32);
  ctx->prof = prof;
  sk.magic = kDeadMagic;
  return rc;
}

int cmm_sketch_free(cmm_sketch* sk) {
  if (!valid_sketch(sk)) return CMM_EINVAL;
  if (sk->owner) return fail(sk->ctx, CMM_ESTATE, "the sketch belongs to a batch");
  release_sketch(sk);
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
  cmm::Geometry g = make_geometry(sk->b, sk->d, sk->m, cmm::Tuning());
  Work w(c);
  void* tmp = w.get<double2>((size_t)sk->d * sk->b);
  if (!tmp) return fail(c, CMM_ENOMEM, "workspace allocation failed");
  CMM_HIP(c, cmm::launch_sub_diag(g, sk->hs1, sk->hs2, (int)sk->n1, (int)sk->n3, diag, (int)len, sk->c64,
                                  tmp, c->stream));
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
    int rc = download(c, c->stream, {{&a, sk->hs1 + (size_t)t * sk->n1 + i, 4},
                                     {&b2, sk->hs2 + (size_t)t * sk->n3 + j, 4}});
    if (rc) return rc;
    const int64_t u = ((int64_t)(a >> 1) + (b2 >> 1)) & (sk->b - 1);
    double v = 0.0;
    rc = download(c, c->stream, {{&v, sk->c64 + (size_t)t * sk->b + u, 8}});
    if (rc) return rc;
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
  return topk_many(sk->ctx, mode, {TopkJob{sk, K, out_i, out_j, out_val}});
}

int cmm_batch_create(cmm_ctx* ctx, const cmm_problem* probs, int32_t count, uint32_t flags,
                     cmm_batch** out) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  if (!out) return fail(ctx, CMM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!probs) return fail(ctx, CMM_EINVAL, "probs is NULL");
  if (count < 1 || count > 4096) return fail(ctx, CMM_EINVAL, "count must be in [1, 4096]");
  if (flags & ~CMM_AUTOTUNE) return fail(ctx, CMM_EINVAL, "unknown flag");
  for (int i = 0; i < count; ++i) {
    const cmm_problem& p = probs[i];
    int rc = check_operands(ctx, p.A, p.lda, p.B, p.ldb, p.n1, p.m, p.n3, p.dtype, p.b, p.d);
    if (rc) return fail(ctx, rc, "problem " + std::to_string(i) + ": " + ctx->last_error);
    if (p.flags & ~CMM_SUBTRACT_DIAG)
      return fail(ctx, CMM_EINVAL, "problem " + std::to_string(i) + ": unknown flag");
    if (p.reserved != 0) return fail(ctx, CMM_EINVAL, "problem " + std::to_string(i) + ": reserved field set");
    if ((p.flags & CMM_SUBTRACT_DIAG) && p.n1 != p.n3)
      return fail(ctx, CMM_EINVAL, "problem " + std::to_string(i) + ": CMM_SUBTRACT_DIAG needs n1 == n3");
    if (p.dtype != CMM_FP8_E4M3 && (p.scaleA || p.scaleB))
      return fail(ctx, CMM_EINVAL, "problem " + std::to_string(i) + ": scales are only taken with CMM_FP8_E4M3");
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, CMM_EHIP, "hipSetDevice failed");
  cmm_batch* bt = new cmm_batch();
  bt->ctx = ctx;
  int rc = build_batch(ctx, probs, count, flags, bt);
  if (rc) {
    const std::string msg = ctx->last_error;
    destroy_batch(bt, false);
    ctx->last_error = msg;
    return rc;
  }
  *out = bt;
  return CMM_OK;
}

int cmm_batch_run(cmm_batch* batch, uint32_t flags) {
  if (!valid_batch(batch)) return CMM_EINVAL;
  cmm_ctx* c = batch->ctx;
  if (flags & ~CMM_ASYNC) return fail(c, CMM_EINVAL, "unknown flag");
  CMM_HIP(c, hipSetDevice(c->device));
  {
    Scope sc_(c, "batch");
    CMM_HIP(c, hipGraphLaunch(batch->exec, c->stream));
  }
  if (!(flags & CMM_ASYNC)) CMM_HIP(c, hipStreamSynchronize(c->stream));
  return CMM_OK;
}

int cmm_batch_sketch(cmm_batch* batch, int32_t index, cmm_sketch** out) {
  if (!valid_batch(batch)) return CMM_EINVAL;
  if (!out) return fail(batch->ctx, CMM_EINVAL, "out is NULL");
  if (index < 0 || index >= (int32_t)batch->sk.size()) return fail(batch->ctx, CMM_EINVAL, "index out of range");
  *out = batch->sk[index];
  return CMM_OK;
}

int cmm_batch_topk(cmm_batch* batch, const int32_t* K, int32_t mode, int64_t* out_i, int64_t* out_j,
                   float* out_val) {
  if (!valid_batch(batch)) return CMM_EINVAL;
  cmm_ctx* c = batch->ctx;
  if (!K || !out_i || !out_j || !out_val) return fail(c, CMM_EINVAL, "K or an output array is NULL");
  CMM_HIP(c, hipSetDevice(c->device));
  // the workspace of a group is about 0.35 MB per product
  constexpr size_t kGroup = 256;
  std::vector<TopkJob> jobs;
  int64_t off = 0;
  for (size_t q = 0; q < batch->sk.size(); ++q) {
    const cmm_sketch* sk = batch->sk[q];
    if (K[q] < 1) return fail(c, CMM_EINVAL, "K < 1");
    jobs.push_back(TopkJob{sk, K[q], out_i + off, out_j + off, out_val + off});
    off += mode == CMM_TOPK_PER_COLUMN ? (int64_t)K[q] * sk->n3 : (int64_t)K[q];
  }
  for (size_t g = 0; g < jobs.size(); g += kGroup) {
    const std::vector<TopkJob> part(jobs.begin() + g, jobs.begin() + std::min(jobs.size(), g + kGroup));
    const int rc = topk_many(c, mode, part);
    if (rc) return rc;
  }
  return CMM_OK;
}

int cmm_batch_free(cmm_batch* batch) {
  if (!valid_batch(batch)) return CMM_EINVAL;
  destroy_batch(batch, false);
  return CMM_OK;
}

int cmm_sketch_product_batched(cmm_ctx* ctx, const cmm_problem* probs, int32_t count,
                               cmm_sketch** outs) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  if (!outs) return fail(ctx, CMM_EINVAL, "outs is NULL");
  cmm_batch* bt = nullptr;
  int rc = cmm_batch_create(ctx, probs, count, 0, &bt);
  if (rc) return rc;
  rc = cmm_batch_run(bt, 0);
  if (rc) { const std::string msg = ctx->last_error; destroy_batch(bt, false); ctx->last_error = msg; return rc; }
  for (int i = 0; i < count; ++i) outs[i] = bt->sk[i];
  destroy_batch(bt, true);
  return CMM_OK;
}

int cmm_autotune(cmm_ctx* ctx, int64_t n1, int64_t m, int64_t n3, int64_t b, int32_t d,
                 int32_t dtype, int32_t* tuning, double* best_ms) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  int rc = check_dims(ctx, n1, m, n3, b, d, dtype);
  if (rc) return rc;
  CMM_HIP(ctx, hipSetDevice(ctx->device));
  TuneEntry e;
  rc = autotune_class(ctx, n1, m, n3, b, d, dtype, &e);
  if (rc) return rc;
  ctx->tuning[tune_key(n1, m, n3, b, d, dtype)] = e;
  if (tuning) { tuning[0] = e.tu.log2c; tuning[1] = e.tu.kmax; tuning[2] = e.tu.cs_blocks; }
  if (best_ms) *best_ms = e.ms;
  return CMM_OK;
}

int cmm_tuning_get(const cmm_ctx* ctx, int64_t n1, int64_t m, int64_t n3, int64_t b, int32_t d,
                   int32_t dtype, int32_t* tuning) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  cmm_ctx* c = const_cast<cmm_ctx*>(ctx);
  if (!tuning) return fail(c, CMM_EINVAL, "tuning is NULL");
  int rc = check_dims(c, n1, m, n3, b, d, dtype);
  if (rc) return rc;
  const cmm::Geometry g = make_geometry(b, d, m, lookup_tuning(ctx, n1, m, n3, b, d, dtype));
  const cmm::Tuning t = lookup_tuning(ctx, n1, m, n3, b, d, dtype);
  tuning[0] = g.log2c; tuning[1] = t.kmax; tuning[2] = g.cs_blocks;
  return CMM_OK;
}

int cmm_tuning_set(cmm_ctx* ctx, int64_t n1, int64_t m, int64_t n3, int64_t b, int32_t d,
                   int32_t dtype, const int32_t* tuning) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  if (!tuning) return fail(ctx, CMM_EINVAL, "tuning is NULL");
  int rc = check_dims(ctx, n1, m, n3, b, d, dtype);
  if (rc) return rc;
  TuneEntry e;
  e.tu.log2c = tuning[0]; e.tu.kmax = tuning[1]; e.tu.cs_blocks = tuning[2];
  if (!valid_tuning(e.tu)) return fail(ctx, CMM_EINVAL, "tuning out of range");
  ctx->tuning[tune_key(n1, m, n3, b, d, dtype)] = e;
  return CMM_OK;
}

int cmm_tuning_save(const cmm_ctx* ctx, const char* path) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  cmm_ctx* c = const_cast<cmm_ctx*>(ctx);
  if (!path) return fail(c, CMM_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(c, CMM_EINVAL, std::string("cannot write ") + path);
  const std::string arch = device_arch(c);
  std::fprintf(f, "[\n");
  size_t q = 0;
  for (const auto& kv : c->tuning) {
    const TuneKey& k = kv.first;
    const TuneEntry& e = kv.second;
    std::fprintf(f,
                 " {\"arch\": \"%s\", \"log2b\": %d, \"ln1\": %d, \"lm\": %d, \"ln3\": %d, \"d\": %d, "
                 "\"dtype\": %d, \"log2c\": %d, \"kmax\": %d, \"cs_blocks\": %d, \"ms\": %.6f}%s\n",
                 arch.c_str(), k.log2b, k.ln1, k.lm, k.ln3, k.d, k.dtype, e.tu.log2c, e.tu.kmax,
                 e.tu.cs_blocks, e.ms, ++q < c->tuning.size() ? "," : "");
  }
  std::fprintf(f, "]\n");
  const bool ok = std::fclose(f) == 0;
  return ok ? CMM_OK : fail(c, CMM_EINVAL, std::string("cannot write ") + path);
}

int cmm_tuning_load(cmm_ctx* ctx, const char* path) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  if (!path) return fail(ctx, CMM_EINVAL, "path is NULL");
  return load_tuning(ctx, path, false);
}

int cmm_frobenius_signs(cmm_ctx* ctx, int64_t n1, int64_t n3, int32_t d, uint64_t seed,
                        int8_t* s1, int8_t* s2) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  if (n1 <= 0 || n3 <= 0 || n1 > (1 << 29) || n3 > (1 << 29)) return fail(ctx, CMM_EINVAL, "n1, n3 out of range");
  if (d < 1 || d > 63) return fail(ctx, CMM_EINVAL, "d must be in [1, 63]");
  CMM_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  std::vector<uint64_t> pr;
  ams_params_from_seed(seed, d, pr);
  Work w(ctx);
  uint64_t* pdev = w.get<uint64_t>(pr.size());
  uint64_t* m1 = w.get<uint64_t>((size_t)n1);
  uint64_t* m2 = w.get<uint64_t>((size_t)n3);
  if (!pdev || !m1 || !m2) return fail(ctx, CMM_ENOMEM, "workspace allocation failed");
  CMM_HIP(ctx, hipMemcpyAsync(pdev, pr.data(), sizeof(uint64_t) * pr.size(), hipMemcpyHostToDevice, s));
  CMM_HIP(ctx, cmm::launch_ams_signs(pdev, d, 0, (int)n1, m1, s));
  CMM_HIP(ctx, cmm::launch_ams_signs(pdev, d, 1, (int)n3, m2, s));
  std::vector<uint64_t> h1((size_t)n1), h2((size_t)n3);
  CMM_HIP(ctx, hipMemcpyAsync(h1.data(), m1, sizeof(uint64_t) * n1, hipMemcpyDeviceToHost, s));
  CMM_HIP(ctx, hipMemcpyAsync(h2.data(), m2, sizeof(uint64_t) * n3, hipMemcpyDeviceToHost, s));
  CMM_HIP(ctx, hipStreamSynchronize(s));
  for (int t = 0; t < d; ++t) {
    if (s1) for (int64_t x = 0; x < n1; ++x) s1[(int64_t)t * n1 + x] = ((h1[x] >> t) & 1) ? -1 : 1;
    if (s2) for (int64_t x = 0; x < n3; ++x) s2[(int64_t)t * n3 + x] = ((h2[x] >> t) & 1) ? -1 : 1;
  }
  return CMM_OK;
}

int cmm_frobenius_bound(cmm_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                        int64_t n1, int64_t m, int64_t n3, int32_t dtype, const float* scaleA,
                        const float* scaleB, int32_t d, uint64_t seed, uint32_t flags, double* X,
                        double* bound) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  int rc = check_operands(ctx, A, lda, B, ldb, n1, m, n3, dtype, 16, d);
  if (rc) return rc;
  if (flags & ~(CMM_SUBTRACT_DIAG | CMM_ASYNC)) return fail(ctx, CMM_EINVAL, "unknown flag");
  if ((flags & CMM_ASYNC) && (X || bound)) return fail(ctx, CMM_EINVAL, "CMM_ASYNC returns no values");
  if ((flags & CMM_SUBTRACT_DIAG) && n1 != n3) return fail(ctx, CMM_EINVAL, "CMM_SUBTRACT_DIAG needs n1 == n3");
  if (dtype != CMM_FP8_E4M3 && (scaleA || scaleB))
    return fail(ctx, CMM_EINVAL, "scales are only taken with CMM_FP8_E4M3");
  CMM_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  std::vector<uint64_t> pr;
  ams_params_from_seed(seed, d, pr);
  Work w(ctx);
  uint64_t* pdev = w.get<uint64_t>(pr.size());
  uint64_t* m1 = w.get<uint64_t>((size_t)n1);
  uint64_t* m2 = w.get<uint64_t>((size_t)n3);
  double* u = w.get<double>((size_t)d * m);
  double* v = w.get<double>((size_t)d * m);
  double* Xd = w.get<double>((size_t)d);
  if (!pdev || !m1 || !m2 || !u || !v || !Xd) return fail(ctx, CMM_ENOMEM, "workspace allocation failed");
  double* diag = nullptr;
  double* partial = nullptr;
  int kch = 1;
  if (flags & CMM_SUBTRACT_DIAG) {
    const int n = (int)n1;
    kch = (int)std::max<int64_t>(1, std::min<int64_t>(m, 1 + 4096 / ((n + 255) / 256)));
    diag = w.get<double>((size_t)n);
    partial = w.get<double>((size_t)kch * n);
    if (!diag || !partial) return fail(ctx, CMM_ENOMEM, "workspace allocation failed");
  }
  CMM_HIP(ctx, hipMemcpyAsync(pdev, pr.data(), sizeof(uint64_t) * pr.size(), hipMemcpyHostToDevice, s));
  {
    Scope sc_(ctx, "frobenius");
    CMM_HIP(ctx, cmm::launch_ams_signs(pdev, d, 0, (int)n1, m1, s));
    CMM_HIP(ctx, cmm::launch_ams_signs(pdev, d, 1, (int)n3, m2, s));
    CMM_HIP(ctx, cmm::launch_ams_rows(dtype, A, lda, scaleA, (int)n1, (int)m, d, m1, u, s));
    CMM_HIP(ctx, cmm::launch_ams_rows(dtype, B, ldb, scaleB, (int)n3, (int)m, d, m2, v, s));
    if (diag) {
      cmm::SideDesc sa, sb;
      sa.X = A; sa.ld = lda; sa.scale = scaleA; sa.n = (int)n1;
      sb.X = B; sb.ld = ldb; sb.scale = scaleB; sb.n = (int)n3;
      CMM_HIP(ctx, cmm::launch_diag(dtype, sa, sb, (int)m, (int)n1, partial, kch, diag, s));
    }
    CMM_HIP(ctx, cmm::launch_ams_final(u, v, (int)m, d, m1, m2, diag, (int)n1, Xd, s));
  }
  if (flags & CMM_ASYNC) return CMM_OK;
  std::vector<double> xh((size_t)d);
  CMM_HIP(ctx, hipMemcpyAsync(xh.data(), Xd, sizeof(double) * d, hipMemcpyDeviceToHost, s));
  CMM_HIP(ctx, hipStreamSynchronize(s));
  if (X) std::copy(xh.begin(), xh.end(), X);
  if (bound) {
    std::vector<double> sq(xh.size());
    for (size_t t = 0; t < xh.size(); ++t) sq[t] = xh[t] * xh[t];
    std::sort(sq.begin(), sq.end());
    const size_t h = sq.size() / 2;
    const double med = (sq.size() & 1) ? sq[h] : 0.5 * (sq[h - 1] + sq[h]);
    *bound = 32.0 * med;
  }
  return CMM_OK;
}

// The extraction's code (Section 4): the binary BCH code of length 63 with
// designed distance 23.  Its generator is the product of (x - alpha^j) over
// the union of the cyclotomic cosets (j, 2j, 4j, ... mod 63) of j = 1 .. 22,
// computed in GF(2^6) (primitive polynomial x^6 + x + 1); the coefficients
// of that product lie in GF(2).  Returned as a bit mask (bit i = x^i,
// degree 47).
constexpr int kExtractCodeLen = 63;

uint64_t bch_generator() {
  int ex[63], lg[64];
  int v = 1;
  for (int i = 0; i < 63; ++i) {
    ex[i] = v; lg[v] = i;
    v <<= 1;
    if (v & 64) v ^= 0x43;
  }
  auto mul = [&](int a, int b) { return (a == 0 || b == 0) ? 0 : ex[(lg[a] + lg[b]) % 63]; };
  bool root[63] = {};
  for (int j = 1; j <= 22; ++j)
    for (int c = j % 63; !root[c]; c = (2 * c) % 63) root[c] = true;
  int poly[64] = {1};   // GF(64) coefficients, lowest degree first
  int deg = 0;
  for (int c = 0; c < 63; ++c) {
    if (!root[c]) continue;
    for (int i = deg + 1; i >= 1; --i) poly[i] = poly[i - 1] ^ mul(poly[i], ex[c]);
    poly[0] = mul(poly[0], ex[c]);
    ++deg;
  }
  uint64_t g = 0;
  for (int i = 0; i <= deg; ++i) g |= (uint64_t)(poly[i] & 1) << i;
  return g;
}

int cmm_find_significant(cmm_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                         int64_t n1, int64_t m, int64_t n3, int32_t dtype, const float* scaleA,
                         const float* scaleB, int64_t b, int32_t d, uint64_t seed, uint32_t flags,
                         double delta, int64_t cap, int64_t* out_i, int64_t* out_j,
                         int64_t* out_count, cmm_sketch** main_out) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  if (main_out) *main_out = nullptr;
  if (!out_count) return fail(ctx, CMM_EINVAL, "out_count is NULL");
  *out_count = 0;
  if (cap < 0 || (cap > 0 && (!out_i || !out_j))) return fail(ctx, CMM_EINVAL, "bad output arrays");
  if (!(delta > 0.0) || !std::isfinite(delta)) return fail(ctx, CMM_EINVAL, "delta must be positive");
  int rc = check_operands(ctx, A, lda, B, ldb, n1, m, n3, dtype, b, d);
  if (rc) return rc;
  if (flags & ~CMM_SUBTRACT_DIAG) return fail(ctx, CMM_EINVAL, "unknown flag");
  if ((flags & CMM_SUBTRACT_DIAG) && n1 != n3) return fail(ctx, CMM_EINVAL, "CMM_SUBTRACT_DIAG needs n1 == n3");
  if (dtype != CMM_FP8_E4M3 && (scaleA || scaleB))
    return fail(ctx, CMM_EINVAL, "scales are only taken with CMM_FP8_E4M3");
  CMM_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const int ell = kExtractCodeLen;   // bits of the code of one index (both sides)
  const int64_t db = (int64_t)d * b;

  cmm_sketch* sk = new cmm_sketch();
  sk->ctx = ctx; sk->n1 = n1; sk->m = m; sk->n3 = n3; sk->b = b; sk->d = d; sk->log2b = ilog2(b);
  sk->has_params = true;
  params_from_seed(seed, d, sk->params);
  if (!alloc_sketch(sk)) { delete sk; return fail(ctx, CMM_ENOMEM, "sketch allocation failed"); }
  const Operands op{A, lda, B, ldb, dtype, scaleA, scaleB, flags & CMM_SUBTRACT_DIAG};
  const cmm::Geometry g = make_geometry(b, d, m, lookup_tuning(ctx, n1, m, n3, b, d, dtype));
  int64_t tsize = 1;
  while (tsize < 2 * db) tsize <<= 1;
  std::vector<int64_t> found;
  uint32_t nfound = 0;
  {
    Work w(ctx);
    float* cr = w.get<float>((size_t)2 * ell * db);
    uint64_t* cw1 = w.get<uint64_t>((size_t)n1);
    uint64_t* cw3 = w.get<uint64_t>((size_t)n3);
    double* ctmp = w.get<double>((size_t)db);
    float* mask = w.get<float>((size_t)std::max(n1, n3));
    double* diagm = (flags & CMM_SUBTRACT_DIAG) ? w.get<double>((size_t)n1) : nullptr;
    int64_t* keys = w.get<int64_t>((size_t)db);
    unsigned long long* tkeys = w.get<unsigned long long>((size_t)tsize);
    uint32_t* tcnt = w.get<uint32_t>((size_t)tsize);
    int64_t* outk = w.get<int64_t>((size_t)std::max<int64_t>(cap, 1));
    uint32_t* cnt = w.get<uint32_t>(1);
    uint64_t* pdev = w.get<uint64_t>((size_t)d * 8);
    if (!cr || !cw1 || !cw3 || !ctmp || !mask || ((flags & CMM_SUBTRACT_DIAG) && !diagm) || !keys ||
        !tkeys || !tcnt || !outk || !cnt || !pdev) {
      release_sketch(sk);
      return fail(ctx, CMM_ENOMEM, "workspace allocation failed");
    }
    rc = CMM_OK;
    if (hipMemcpyAsync(pdev, sk->params.data(), sizeof(uint64_t) * d * 8, hipMemcpyHostToDevice, s) != hipSuccess)
      rc = fail(ctx, CMM_EHIP, "parameter upload failed");
    const uint64_t gen = bch_generator();
    if (rc == CMM_OK && (cmm::launch_code_words((int)n1, gen, cw1, s) != hipSuccess ||
                         cmm::launch_code_words((int)n3, gen, cw3, s) != hipSuccess))
      rc = fail(ctx, CMM_EHIP, "code word launch failed");
    // the sketch of AB itself, keeping its workspace (layout, both count sketches)
    WsSpec spec;
    WsPtrs ptr;
    std::vector<void*> owned;
    for (int attempt = 0; attempt < 2 && rc == CMM_OK; ++attempt) {
      spec = ws_spec(g, n1, n3, attempt == 1, op.flags);
      ptr = WsPtrs();
      rc = ws_alloc(ctx, spec, ptr, owned);
      if (rc == CMM_OK) rc = enqueue_product(ctx, sk, op, g, spec, ptr, pdev, s);
      if (rc == CMM_OK && (hipMemcpyAsync(ctx->pinned_u32, ptr.p[W_OFLOW], sizeof(int32_t),
                                          hipMemcpyDeviceToHost, s) != hipSuccess ||
                           hipStreamSynchronize(s) != hipSuccess))
        rc = fail(ctx, CMM_EHIP, "stream synchronisation failed");
      if (rc == CMM_OK && ctx->pinned_u32[0] != 0 && attempt == 0) { ws_release(ctx, owned); continue; }
      break;
    }
    double2* tw64 = nullptr; float2* tw32 = nullptr;
    if (rc == CMM_OK) rc = get_twiddles(ctx, b, &tw64, &tw32);
    if (rc == CMM_OK) {
      cmm::SideDesc side[2];
      bind_sides(g, sk, op, spec, ptr, side);
      const int64_t nn[2] = {n1, n3};
      const uint64_t* cws[2] = {cw1, cw3};
      const float* scl[2] = {scaleA, scaleB};
      // the sketch of the product with side q's index weighted by code bit r
      auto masked = [&](int q, int r, int64_t slot) -> int {
        CMM_HIP(ctx, cmm::launch_code_mask((int)nn[q], r, cws[q], scl[q], mask, s));
        side[q].scale = mask;
        CMM_HIP(ctx, cmm::launch_countsketch(dtype, g, side[q], s));
        CMM_HIP(ctx, cmm::launch_fft_mac(g, side[0], side[1], tw32, (float2*)ptr.p[W_PPART], s,
                                         overlap_for(ctx, s)));
        CMM_HIP(ctx, cmm::launch_ifft(g, (float2*)ptr.p[W_PPART], (double2*)ptr.p[W_WORK0],
                                      (double2*)ptr.p[W_WORK1], tw64, ctmp, s));
        if (diagm) {
          CMM_HIP(ctx, cmm::launch_code_mask_diag((int)n1, r, cws[q], (const double*)ptr.p[W_DIAG], diagm, s));
          CMM_HIP(ctx, cmm::launch_sub_diag(g, sk->hs1, sk->hs2, (int)n1, (int)n3, diagm, (int)n1, ctmp,
                                            ptr.p[W_WORK0], s));
        }
        CMM_HIP(ctx, cmm::launch_to_f32(ctmp, cr + slot * db, db, s));
        return CMM_OK;
      };
      Scope sc_(ctx, "extract");
      // column-code sketches, then the row-code ones (B's sketch restored)
      for (int r = 0; r < ell && rc == CMM_OK; ++r) rc = masked(1, r, ell + r);
      if (rc == CMM_OK) {
        side[1].scale = scaleB;
        if (cmm::launch_countsketch(dtype, g, side[1], s) != hipSuccess) rc = fail(ctx, CMM_EHIP, "countsketch launch failed");
      }
      for (int r = 0; r < ell && rc == CMM_OK; ++r) rc = masked(0, r, r);
      if (rc == CMM_OK) {
        hipError_t e = cmm::launch_extract_decode(cr, d, b, (int)n1, (int)n3, (float)(0.5 * delta), keys, s);
        if (e == hipSuccess) e = cmm::launch_fill_i32((int32_t*)tkeys, 2 * tsize, -1, s);
        if (e == hipSuccess) e = cmm::launch_fill_i32((int32_t*)tcnt, tsize, 0, s);
        if (e == hipSuccess) e = cmm::launch_fill_i32((int32_t*)cnt, 1, 0, s);
        if (e == hipSuccess) e = cmm::launch_vote(keys, db, tkeys, tcnt, tsize, d, outk, cnt, cap, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&nfound, cnt, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = fail(ctx, CMM_EHIP, std::string("extraction failed: ") + hipGetErrorString(e));
      }
      if (rc == CMM_OK && nfound > 0 && cap > 0) {
        found.resize((size_t)std::min<int64_t>(nfound, cap));
        if (hipMemcpy(found.data(), outk, sizeof(int64_t) * found.size(), hipMemcpyDeviceToHost) != hipSuccess)
          rc = fail(ctx, CMM_EHIP, "result copy failed");
      }
    }
    (void)hipStreamSynchronize(s);
    ws_release(ctx, owned);
  }
  if (rc != CMM_OK) { release_sketch(sk); return rc; }
  std::sort(found.begin(), found.end());
  for (size_t q = 0; q < found.size(); ++q) { out_i[q] = found[q] / n3; out_j[q] = found[q] % n3; }
  *out_count = nfound;
  if (main_out) *main_out = sk;
  else release_sketch(sk);
  return CMM_OK;
}

int cmm_sketch_product_sparse(cmm_ctx* ctx, const int64_t* a_ptr, const int32_t* a_idx,
                              const float* a_val, const int64_t* b_ptr, const int32_t* b_idx,
                              const float* b_val, int64_t n1, int64_t m, int64_t n3, int64_t b,
                              int32_t d, uint64_t seed, uint32_t flags, cmm_sketch** out) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  if (!out) return fail(ctx, CMM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!a_ptr || !b_ptr) return fail(ctx, CMM_EINVAL, "sparse offsets must be device pointers");
  if (m <= 0 || m > (1 << 30)) return fail(ctx, CMM_EINVAL, "m out of range");
  if (std::max(n1, n3) > cmm::kMaxStagedDim)
    return fail(ctx, CMM_EUNSUPPORTED, "sparse operands: hashed dimension above 24576 (rows are staged in LDS)");
  CMM_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  {
    // offsets from 0, non-decreasing; every index inside its dimension
    Work w(ctx);
    int32_t* bad = w.get<int32_t>(1);
    if (!bad) return fail(ctx, CMM_ENOMEM, "workspace allocation failed");
    int64_t nnz[2] = {0, 0};
    CMM_HIP(ctx, hipMemcpyAsync(&nnz[0], a_ptr + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CMM_HIP(ctx, hipMemcpyAsync(&nnz[1], b_ptr + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CMM_HIP(ctx, hipStreamSynchronize(s));
    if (nnz[0] < 0 || nnz[1] < 0) return fail(ctx, CMM_EINVAL, "negative entry count");
    if ((nnz[0] > 0 && (!a_idx || !a_val)) || (nnz[1] > 0 && (!b_idx || !b_val)))
      return fail(ctx, CMM_EINVAL, "sparse indices and values must be device pointers");
    CMM_HIP(ctx, cmm::launch_fill_i32(bad, 1, 0, s));
    if (n1 > 0 && n3 > 0) {
      CMM_HIP(ctx, cmm::launch_sparse_check(a_ptr, a_idx, (int)m, (int)n1, nnz[0], bad, s));
      CMM_HIP(ctx, cmm::launch_sparse_check(b_ptr, b_idx, (int)m, (int)n3, nnz[1], bad, s));
    }
    int32_t hbad = 0;
    CMM_HIP(ctx, hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    CMM_HIP(ctx, hipStreamSynchronize(s));
    if (hbad) return fail(ctx, CMM_EINVAL, "sparse offsets decrease or an index is out of range");
  }
  Operands sp{a_val, n1, b_val, n3, CMM_F32, nullptr, nullptr, flags};
  sp.aptr = a_ptr; sp.aidx = a_idx; sp.bptr = b_ptr; sp.bidx = b_idx;
  // an operand without entries may have NULL index and value arrays (never
  // read); the offsets stand in for the value pointer in the generic checks
  const void* av = a_val ? (const void*)a_val : (const void*)a_ptr;
  const void* bv = b_val ? (const void*)b_val : (const void*)b_ptr;
  return product_common(ctx, av, n1, bv, n3, n1, m, n3, CMM_F32, nullptr, nullptr, b, d, seed,
                        nullptr, nullptr, nullptr, nullptr, nullptr, flags, out, &sp);
}

int cmm_estimate_nnz(cmm_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                     int64_t n1, int64_t m, int64_t n3, int32_t dtype, const float* scaleA,
                     const float* scaleB, int32_t d, uint64_t seed, uint32_t flags, double zero_rel,
                     int64_t* b_out, int64_t* zeros) {
  if (!valid_ctx(ctx)) return CMM_EINVAL;
  if (!b_out) return fail(ctx, CMM_EINVAL, "b_out is NULL");
  *b_out = -1;
  int rc = check_operands(ctx, A, lda, B, ldb, n1, m, n3, dtype, 16, d);
  if (rc) return rc;
  if (flags & ~CMM_SUBTRACT_DIAG) return fail(ctx, CMM_EINVAL, "unknown flag");
  if ((flags & CMM_SUBTRACT_DIAG) && n1 != n3) return fail(ctx, CMM_EINVAL, "CMM_SUBTRACT_DIAG needs n1 == n3");
  if (dtype != CMM_FP8_E4M3 && (scaleA || scaleB))
    return fail(ctx, CMM_EINVAL, "scales are only taken with CMM_FP8_E4M3");
  if (!(zero_rel >= 0.0) || !(zero_rel < 1.0)) return fail(ctx, CMM_EINVAL, "zero_rel must be in [0, 1)");
  CMM_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  Work w(ctx);
  float* w1 = w.get<float>((size_t)n1);
  float* w2 = w.get<float>((size_t)n3);
  int64_t* zdev = w.get<int64_t>((size_t)d);
  if (!w1 || !w2 || !zdev) return fail(ctx, CMM_ENOMEM, "workspace allocation failed");
  // D1, D2: entries in [1, 2) from the seed's SplitMix64 stream at 2^40 and
  // 2^41 (times the fp8 column scales)
  CMM_HIP(ctx, cmm::launch_nnz_weights(seed, 1ull << 40, (int)n1, scaleA, w1, s));
  CMM_HIP(ctx, cmm::launch_nnz_weights(seed, 1ull << 41, (int)n3, scaleB, w2, s));
  const Operands op{A, lda, B, ldb, dtype, w1, w2, flags & CMM_SUBTRACT_DIAG};
  std::vector<int64_t> zh((size_t)d);
  for (int64_t b = 16; b <= (1 << 20); b *= 2) {
    cmm_sketch* sk = new cmm_sketch();
    sk->ctx = ctx; sk->n1 = n1; sk->m = m; sk->n3 = n3; sk->b = b; sk->d = d; sk->log2b = ilog2(b);
    sk->has_params = true;
    params_from_seed(seed, d, sk->params);
    if (!alloc_sketch(sk)) { delete sk; return fail(ctx, CMM_ENOMEM, "sketch allocation failed"); }
    bool over = false;
    const cmm::Tuning tu = lookup_tuning(ctx, n1, m, n3, b, d, dtype);
    {
      Scope sc_(ctx, "nnz");
      rc = run_product(ctx, sk, op, tu, false, &over);
      if (rc == CMM_OK && over) rc = run_product(ctx, sk, op, tu, true, &over);
      if (rc == CMM_OK && cmm::launch_nnz_zeros(sk->c64, d, b, zero_rel, zdev, s) != hipSuccess)
        rc = fail(ctx, CMM_EHIP, "zero count launch failed");
    }
    if (rc == CMM_OK && (hipMemcpyAsync(zh.data(), zdev, sizeof(int64_t) * d, hipMemcpyDeviceToHost, s) != hipSuccess ||
                         hipStreamSynchronize(s) != hipSuccess))
      rc = fail(ctx, CMM_EHIP, "zero count copy failed");
    release_sketch(sk);
    if (rc) return rc;
    if (zeros) std::copy(zh.begin(), zh.end(), zeros);
    bool done = true;
    for (int t = 0; t < d; ++t) done = done && 5 * zh[t] >= 4 * b;
    if (done) { *b_out = b; return CMM_OK; }
  }
  return CMM_OK;
}

}  // extern "C"

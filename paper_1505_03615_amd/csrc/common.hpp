// Internal infrastructure of the camfe HIP library: error reporting, device
// arrays, the context, and small device helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "camfe.h"

namespace camfe {

typedef unsigned long long u64;

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
  camfe_status code;
  Error(camfe_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// Records msg as the calling thread's last error and, when the failing call
// has reached its context (camfe_ctx_s::use_device), as that context's.
void set_last_error(const std::string& msg);

// Scratch of camfe_apply_noalloc: a file-scope device array of
// 2 * NOALLOC_BLOCK doubles (16 MiB) per device, held until the process ends.
constexpr size_t NOALLOC_BLOCK = size_t(1) << 20;
// context reached by the entry point running on this thread (or null)
camfe_ctx current_ctx();
void set_current_ctx(camfe_ctx ctx);

#define CAMFE_HIP(call)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::camfe::Error(e_ == hipErrorOutOfMemory ? CAMFE_ENOMEM : CAMFE_EDEVICE,      \
                           std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)

#define CAMFE_REQUIRE(cond, code, msg) \
  do {                                 \
    if (!(cond)) throw ::camfe::Error((code), (msg)); \
  } while (0)

// Runs f, mapping exceptions to status codes and the thread's last error.
// An entry point called from inside another keeps the outer call's context.
template <class Fn>
camfe_status guarded(Fn&& f) {
  struct Scope {
    camfe_ctx saved;
    Scope() : saved(current_ctx()) { set_current_ctx(nullptr); }
    ~Scope() { set_current_ctx(saved); }
  } scope;
  try {
    f();
    return CAMFE_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return CAMFE_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return CAMFE_EDEVICE;
  }
}

// ------------------------------------------------------ device memory cache
// Device memory of the library comes from a cache of blocks keyed by device,
// stream and size class (pool.hip).  A freed block goes back to the list of
// the stream it was allocated for and is handed out again only for that
// stream, so stream order puts every earlier use of the block ahead of the
// next one.  The stream is the one of the context whose entry point is
// running (set by camfe_ctx_s::use_device); streams are attached by
// camfe_ctx_create and detached (their blocks freed) by camfe_ctx_destroy.
// Blocks of a detached stream, and blocks beyond a quarter of the device's
// memory, are freed at once.
struct PoolBlock {
  size_t cls = 0;           // size class in bytes
  int dev = 0;
  hipStream_t st = nullptr;
};
void* pool_alloc(size_t bytes, PoolBlock* b);
void pool_free(void* p, const PoolBlock& b);
void pool_attach_stream(int dev, hipStream_t st);
void pool_detach_stream(int dev, hipStream_t st);   // the stream must be idle
void set_current_stream(hipStream_t st);             // of the calling thread

// ----------------------------------------------------------- device arrays
template <class T>
struct DArr {
  T* p = nullptr;
  size_t n = 0;
  PoolBlock blk;
  DArr() = default;
  explicit DArr(size_t count) { alloc(count); }
  DArr(const DArr&) = delete;
  DArr& operator=(const DArr&) = delete;
  DArr(DArr&& o) noexcept : p(o.p), n(o.n), blk(o.blk) { o.p = nullptr; o.n = 0; }
  DArr& operator=(DArr&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; blk = o.blk; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DArr() { release(); }
  void alloc(size_t count) {
    release();
    if (count) p = (T*)pool_alloc(count * sizeof(T), &blk);
    n = count;
  }
  void release() {
    if (p) pool_free(p, blk);
    p = nullptr;
    n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
};

// ------------------------------------------------------ kernel timing
// Opt-in measurement: launches of the hot kernels are bracketed with HIP
// events on the launching stream; totals are resolved when read.  Each
// launch also records its algorithmic work (bytes that the method must move,
// or flops of the dense contractions).
enum KernelId { KT_GS = 0, KT_RESIDUAL, KT_SPMV, KT_RESTRICT, KT_PROLONG, KT_COARSE, KT_ASSEMBLE,
                KT_PAIRS, KT_UF_LINK, KT_SUPPORT_SORT, KT_CG_VEC, KT_COUNT };
inline const char* kernel_name(int k) {
  static const char* n[] = {"gs_colour", "residual", "spmv_dot", "restrict", "prolong", "coarse_solve",
                            "assemble", "pairs", "uf_link", "support_sort", "cg_vector"};
  return n[k];
}
struct KernelTimer {
  bool on = false;
  struct Rec { int k; hipEvent_t a, b; double work; };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  double total_ms[KT_COUNT] = {0};
  double work[KT_COUNT] = {0};
  long long count[KT_COUNT] = {0};
  hipEvent_t get() {
    if (pool.empty()) {
      hipEvent_t e;
      CAMFE_HIP(hipEventCreate(&e));
      return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  void begin(int k, hipStream_t s, double w) {
    Rec r{k, get(), get(), w};
    CAMFE_HIP(hipEventRecord(r.a, s));
    pending.push_back(r);
  }
  void end(hipStream_t s) { CAMFE_HIP(hipEventRecord(pending.back().b, s)); }
  void resolve() {
    for (Rec& r : pending) {
      CAMFE_HIP(hipEventSynchronize(r.b));
      float ms = 0;
      CAMFE_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      total_ms[r.k] += ms;
      work[r.k] += r.work;
      count[r.k] += 1;
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  void reset() {
    resolve();
    for (int i = 0; i < KT_COUNT; ++i) { total_ms[i] = 0; work[i] = 0; count[i] = 0; }
  }
  ~KernelTimer() {
    for (auto& r : pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// ---------------------------------------------------------------- context
}  // namespace camfe

struct camfe_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  camfe::DArr<unsigned char> scratch;  // reused temporary storage (sort/scan)
  camfe::DArr<unsigned char> scratch2;
  int* d_flag = nullptr;               // device error flag
  camfe::KernelTimer timer;
  double* noalloc_scratch = nullptr;   // this device's scratch of camfe_apply_noalloc (never freed)
  std::mutex err_mu;                   // guards last_error
  std::string last_error;              // last failed call that reached this context
  unsigned char* scratch_bytes(size_t b) {
    if (scratch.n < b) scratch.alloc(b + (b >> 2) + 256);
    return scratch.p;
  }
  unsigned char* scratch2_bytes(size_t b) {
    if (scratch2.n < b) scratch2.alloc(b + (b >> 2) + 256);
    return scratch2.p;
  }
  void sync() { CAMFE_HIP(hipStreamSynchronize(stream)); }
  void use_device() {
    camfe::set_current_ctx(this);
    CAMFE_HIP(hipSetDevice(device));
    camfe::set_current_stream(stream);
  }
};

namespace camfe {

// copies between host/device memory of any kind (unified addressing)
// Copies complete before returning, so host sources may be temporaries.
template <class T>
void copy_in(camfe_ctx ctx, T* dst, const T* src, size_t count) {
  if (!count) return;
  CAMFE_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDefault, ctx->stream));
  CAMFE_HIP(hipStreamSynchronize(ctx->stream));
}
template <class T>
void copy_out(camfe_ctx ctx, T* dst, const T* src, size_t count) {
  if (!count) return;
  CAMFE_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDefault, ctx->stream));
  CAMFE_HIP(hipStreamSynchronize(ctx->stream));
}
template <class T>
T read_scalar(camfe_ctx ctx, const T* dptr) {
  T v;
  CAMFE_HIP(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, ctx->stream));
  ctx->sync();
  return v;
}
template <class T>
void zero(camfe_ctx ctx, T* p, size_t count) {
  if (count) CAMFE_HIP(hipMemsetAsync(p, 0, count * sizeof(T), ctx->stream));
}

inline void check_launch() { CAMFE_HIP(hipGetLastError()); }

// launch with optional event timing; `work` = algorithmic bytes or flops
#define CAMFE_TIMED(ctx, KID, WORK, ...)                                             \
  do {                                                                               \
    const bool t_on_ = (ctx)->timer.on;                                              \
    if (t_on_) (ctx)->timer.begin((KID), (ctx)->stream, (double)(WORK));             \
    hipLaunchKernelGGL(__VA_ARGS__);                                                 \
    if (t_on_) (ctx)->timer.end((ctx)->stream);                                      \
  } while (0)

inline unsigned grid_for(size_t n, unsigned block) {
  size_t g = (n + block - 1) / block;
  if (g == 0) g = 1;
  if (g > 0x7fffffffULL) g = 0x7fffffff;
  return (unsigned)g;
}

// ------------------------------------------------- primitives (prim.hip)
// Radix sorts of 64- or 32-bit keys on bits [0, end_bit) (sort_pairs: [begin_bit,
// end_bit)); stable.  Temporary storage comes from the context.  In-place on
// (keys[, vals]).
void sort_keys(camfe_ctx ctx, u64* keys, size_t n, int end_bit);
void sort_keys_u32(camfe_ctx ctx, uint32_t* keys, size_t n, int end_bit);
void sort_pairs(camfe_ctx ctx, u64* keys, uint32_t* vals, size_t n, int end_bit, int begin_bit = 0);
void sort_pairs_u32(camfe_ctx ctx, uint32_t* keys, uint32_t* vals, size_t n, int end_bit);
// exclusive prefix sums (out may alias in); returns nothing (total = last in + last out)
void exclusive_scan(camfe_ctx ctx, const int* in, int* out, size_t n);
void exclusive_scan64(camfe_ctx ctx, const long long* in, long long* out, size_t n);
// sum reduction into a device scalar
void reduce_sum64(camfe_ctx ctx, const long long* in, long long* out, size_t n);

// ------------------------------------------------------- device helpers
__host__ __device__ inline u64 spread3(u64 x) {
  x &= 0x1fffffULL;
  x = (x | (x << 32)) & 0x1f00000000ffffULL;
  x = (x | (x << 16)) & 0x1f0000ff0000ffULL;
  x = (x | (x << 8)) & 0x100f00f00f00f00fULL;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ULL;
  x = (x | (x << 2)) & 0x1249249249249249ULL;
  return x;
}
__host__ __device__ inline u64 compact3(u64 x) {
  x &= 0x1249249249249249ULL;
  x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ULL;
  x = (x ^ (x >> 4)) & 0x100f00f00f00f00fULL;
  x = (x ^ (x >> 8)) & 0x1f0000ff0000ffULL;
  x = (x ^ (x >> 16)) & 0x1f00000000ffffULL;
  x = (x ^ (x >> 32)) & 0x1fffffULL;
  return x;
}
__host__ __device__ inline u64 morton(u64 x, u64 y, u64 z) {
  return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}
__host__ __device__ inline void demorton(u64 k, long long c[3]) {
  c[0] = (long long)compact3(k);
  c[1] = (long long)compact3(k >> 1);
  c[2] = (long long)compact3(k >> 2);
}

constexpr int TRI_BITS = 24;
constexpr u64 TRI_MASK = (1ULL << TRI_BITS) - 1;

}  // namespace camfe

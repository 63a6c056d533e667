// Building blocks of the hierarchy build and the solver set-up: a stable
// least-significant-digit radix sort, prefix sums and a sum reduction,
// written for 64-wide wavefronts.
//
// Radix sort, one pass per 8-bit digit:
//   1. k_radix_hist: every tile of STILE keys counts its digits; the counts
//      land digit-major, counts[d * tiles + tile].
//   2. an exclusive scan of that array gives, for every (digit, tile), the
//      output position of the tile's first key with that digit.
//   3. k_radix_scatter: every wave ranks its keys among the equal digits of
//      the wave (eight ballots give the lanes that share a digit) against
//      wave-private running counters in LDS, the waves' counts are combined
//      per digit, the tile is reordered by digit in LDS and written out, so
//      that keys of one digit leave a tile as one contiguous run.
// A tile is eight waves, each with a contiguous eighth, so the order within a
// tile (wave, then step, then lane) is the input order: the sort is stable.
#include "common.hpp"

namespace camfe {

namespace {

// scans and reductions
constexpr int PB = 256;             // threads per block (four waves)
constexpr int PW = PB / 64;         // waves per block
constexpr int PI = 8;               // values per thread
constexpr int TILE = PB * PI;       // values per tile
// radix sort
constexpr int SB = 512;             // threads per block (eight waves)
constexpr int SW = SB / 64;         // waves per block
constexpr int SI = 8;               // keys per thread
constexpr int STILE = SB * SI;      // keys per tile
constexpr int WTILE = STILE / SW;   // keys per wave
constexpr int RBITS = 8;            // bits per digit
constexpr int RD = 1 << RBITS;      // digits
static_assert(SB >= RD && SB % RD == 0, "every digit has a thread in the per-tile digit scan");

__device__ inline unsigned long long lanes_below() {
  return (1ULL << __lane_id()) - 1ULL;
}

// lanes of the wave whose valid key has digit d (0 for an invalid lane)
__device__ inline unsigned long long same_digit(unsigned d, bool valid) {
  unsigned long long m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < RBITS; ++b) {
    const bool bit = (d >> b) & 1u;
    const unsigned long long v = __ballot(bit);
    m &= bit ? v : ~v;
  }
  return valid ? m : 0ULL;
}

template <class T>
__device__ inline T wave_inclusive_sum(T x) {
  const int lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  return x;
}

// exclusive sum over the block of one value per thread; `part` holds
// blockDim.x / 64 entries; `total` receives the block's sum
template <class T>
__device__ inline T block_exclusive_sum(T v, T* part, T& total) {
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const T inc = wave_inclusive_sum(v);
  if (__lane_id() == 63) part[w] = inc;
  __syncthreads();
  T before = 0, all = 0;
  for (int i = 0; i < nw; ++i) {
    const T p = part[i];
    if (i < w) before += p;
    all += p;
  }
  __syncthreads();   // part is reused by the caller's next call
  total = all;
  return before + inc - v;
}

template <class K>
__global__ __launch_bounds__(SB) void k_radix_hist(const K* __restrict__ keys, long long n, int shift,
                                                   unsigned dmask, int* __restrict__ counts, int tiles) {
  __shared__ int h[RD];
  if (threadIdx.x < RD) h[threadIdx.x] = 0;
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long base = (long long)blockIdx.x * STILE + (long long)w * WTILE + lane;
  K key[SI];
#pragma unroll
  for (int k = 0; k < SI; ++k) {
    const long long i = base + 64LL * k;
    key[k] = i < n ? keys[i] : K(0);
  }
#pragma unroll
  for (int k = 0; k < SI; ++k) {
    const bool valid = base + 64LL * k < n;
    const unsigned d = (unsigned)(key[k] >> shift) & dmask;
    const unsigned long long m = same_digit(d, valid);
    if (valid && (m & lanes_below()) == 0ULL) atomicAdd(&h[d], (int)__popcll(m));
  }
  __syncthreads();
  if (threadIdx.x < RD) counts[(size_t)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

template <class K, bool VALS>
__global__ __launch_bounds__(SB) void k_radix_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                      K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                      long long n, int shift, unsigned dmask,
                                                      const int* __restrict__ offs, int tiles) {
  __shared__ K sk[STILE];
  __shared__ uint32_t sv[VALS ? STILE : 1];
  __shared__ int run[SW][RD];     // per wave: keys of each digit ranked so far, then the wave's prefix
  __shared__ int tstart[RD];      // first position of each digit within the reordered tile
  __shared__ int gshift[RD];      // output position of the tile's digit-d run, minus tstart[d]
  __shared__ int part[SW];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const long long tile0 = (long long)blockIdx.x * STILE;
  const long long base = tile0 + (long long)w * WTILE + lane;
  K key[SI];
  uint32_t val[SI];
  int rank[SI];
#pragma unroll
  for (int k = 0; k < SI; ++k) {
    const long long i = base + 64LL * k;
    key[k] = i < n ? kin[i] : K(0);
    if (VALS) val[k] = i < n ? vin[i] : 0u;
  }
  for (int i = t; i < SW * RD; i += SB) (&run[0][0])[i] = 0;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < SI; ++k) {
    const bool valid = base + 64LL * k < n;
    const unsigned d = (unsigned)(key[k] >> shift) & dmask;
    const unsigned long long m = same_digit(d, valid);
    int r = 0;
    if (valid) {
      // every lane reads the counter before the group's first lane advances it
      // (one wave: the LDS read and the later write stay in program order)
      const int before = run[w][d];
      const unsigned long long below = m & lanes_below();
      r = before + (int)__popcll(below);
      if (below == 0ULL) run[w][d] = before + (int)__popcll(m);
    }
    rank[k] = r;
  }
  __syncthreads();
  {
    // threads below RD own one digit each; the others add zeros to the scan
    const int d = t;
    int s = 0;
    if (d < RD) {
#pragma unroll
      for (int ww = 0; ww < SW; ++ww) {
        const int c = run[ww][d];
        run[ww][d] = s;
        s += c;
      }
    }
    int total;
    const int ex = block_exclusive_sum(s, part, total);
    if (d < RD) {
      tstart[d] = ex;
      gshift[d] = offs[(size_t)d * tiles + blockIdx.x] - ex;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < SI; ++k) {
    if (base + 64LL * k < n) {
      const unsigned d = (unsigned)(key[k] >> shift) & dmask;
      const int pos = tstart[d] + run[w][d] + rank[k];
      sk[pos] = key[k];
      if (VALS) sv[pos] = val[k];
    }
  }
  __syncthreads();
  const long long rem = n - tile0;
  const int cnt = rem < STILE ? (int)rem : STILE;
  for (int p = t; p < cnt; p += SB) {
    const K kk = sk[p];
    const unsigned d = (unsigned)(kk >> shift) & dmask;
    const long long o = (long long)gshift[d] + p;
    kout[o] = kk;
    if (VALS) vout[o] = sv[p];
  }
}

// ---------------------------------------------------------------- scans
// tile sums: one partial per TILE consecutive values
template <class T>
__global__ __launch_bounds__(PB) void k_tile_sums(const T* __restrict__ in, long long n, T* __restrict__ part_out) {
  __shared__ T part[PW];
  const long long tile0 = (long long)blockIdx.x * TILE;
  T s = 0;
#pragma unroll
  for (int k = 0; k < PI; ++k) {
    const long long i = tile0 + (long long)k * PB + threadIdx.x;
    if (i < n) s += in[i];
  }
  T total;
  (void)block_exclusive_sum(s, part, total);
  if (threadIdx.x == 0) part_out[blockIdx.x] = total;
}

// exclusive scan, in place, of m partials by one block (chunks of blockDim.x)
template <class T>
__global__ __launch_bounds__(1024) void k_scan_partials(T* __restrict__ p, long long m) {
  __shared__ T part[16];
  T carry = 0;
  for (long long c = 0; c < m; c += blockDim.x) {
    const long long i = c + threadIdx.x;
    const T v = i < m ? p[i] : T(0);
    T total;
    const T ex = block_exclusive_sum(v, part, total);
    if (i < m) p[i] = carry + ex;
    carry += total;
  }
}

// exclusive scan of each tile, offset by its scanned partial (nullptr: one tile)
template <class T>
__global__ __launch_bounds__(PB) void k_scan_tiles(const T* in, T* out, long long n, const T* __restrict__ tile_off) {
  __shared__ T part[PW];
  const long long tile0 = (long long)blockIdx.x * TILE;
  T carry = tile_off ? tile_off[blockIdx.x] : T(0);
  for (int k = 0; k < PI; ++k) {
    const long long i = tile0 + (long long)k * PB + threadIdx.x;
    const T v = i < n ? in[i] : T(0);
    T total;
    const T ex = block_exclusive_sum(v, part, total);
    if (i < n) out[i] = carry + ex;
    carry += total;
  }
}

// sum of m partials by one block into *out
template <class T>
__global__ __launch_bounds__(1024) void k_sum_partials(const T* __restrict__ p, long long m, T* __restrict__ out) {
  __shared__ T part[16];
  T s = 0;
  for (long long i = threadIdx.x; i < m; i += blockDim.x) s += p[i];
  T total;
  (void)block_exclusive_sum(s, part, total);
  if (threadIdx.x == 0) *out = total;
}

inline size_t tiles_of(size_t n) { return (n + TILE - 1) / TILE; }
inline size_t sort_tiles_of(size_t n) { return (n + STILE - 1) / STILE; }
inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// exclusive scan with caller-provided room for tiles_of(n) partials
template <class T>
void scan_with(camfe_ctx ctx, const T* in, T* out, size_t n, T* partials) {
  if (n == 0) return;
  const size_t tl = tiles_of(n);
  if (tl == 1) {
    hipLaunchKernelGGL(k_scan_tiles<T>, dim3(1), dim3(PB), 0, ctx->stream, in, out, (long long)n, (const T*)nullptr);
    check_launch();
    return;
  }
  hipLaunchKernelGGL(k_tile_sums<T>, dim3((unsigned)tl), dim3(PB), 0, ctx->stream, in, (long long)n, partials);
  hipLaunchKernelGGL(k_scan_partials<T>, dim3(1), dim3(1024), 0, ctx->stream, partials, (long long)tl);
  hipLaunchKernelGGL(k_scan_tiles<T>, dim3((unsigned)tl), dim3(PB), 0, ctx->stream, in, out, (long long)n,
                     (const T*)partials);
  check_launch();
}

template <class K, bool VALS>
void radix_sort(camfe_ctx ctx, K* keys, uint32_t* vals, size_t n, int end_bit, int begin_bit = 0) {
  CAMFE_REQUIRE(begin_bit >= 0, CAMFE_EINVAL, "radix sort begin bit below 0");
  if (n < 2 || end_bit <= begin_bit) return;
  CAMFE_REQUIRE(n < (size_t(1) << 31), CAMFE_EINVAL, "radix sort of 2^31 keys or more");
  CAMFE_REQUIRE(end_bit <= (int)(8 * sizeof(K)), CAMFE_EINVAL, "radix sort end bit beyond the key");
  const size_t tl = sort_tiles_of(n);
  const size_t ncount = tl * RD;
  // scratch: digit counts, then the partials of their scan
  unsigned char* s1 = ctx->scratch_bytes(align256(ncount * sizeof(int)) + align256(tiles_of(ncount) * sizeof(int)));
  int* counts = (int*)s1;
  int* partials = (int*)(s1 + align256(ncount * sizeof(int)));
  // scratch2: the other key (and value) buffer
  unsigned char* s2 = ctx->scratch2_bytes(align256(n * sizeof(K)) + (VALS ? align256(n * sizeof(uint32_t)) : 0));
  K* kalt = (K*)s2;
  uint32_t* valt = VALS ? (uint32_t*)(s2 + align256(n * sizeof(K))) : nullptr;
  K* ksrc = keys;
  K* kdst = kalt;
  uint32_t* vsrc = vals;
  uint32_t* vdst = valt;
  int passes = 0;
  for (int shift = begin_bit; shift < end_bit; shift += RBITS, ++passes) {
    const int bits = end_bit - shift < RBITS ? end_bit - shift : RBITS;
    const unsigned dmask = (1u << bits) - 1u;
    hipLaunchKernelGGL(k_radix_hist<K>, dim3((unsigned)tl), dim3(SB), 0, ctx->stream, (const K*)ksrc, (long long)n,
                       shift, dmask, counts, (int)tl);
    check_launch();
    scan_with<int>(ctx, counts, counts, ncount, partials);
    hipLaunchKernelGGL((k_radix_scatter<K, VALS>), dim3((unsigned)tl), dim3(SB), 0, ctx->stream, (const K*)ksrc,
                       (const uint32_t*)vsrc, kdst, vdst, (long long)n, shift, dmask, (const int*)counts, (int)tl);
    check_launch();
    K* tk = ksrc; ksrc = kdst; kdst = tk;
    uint32_t* tv = vsrc; vsrc = vdst; vdst = tv;
  }
  if (passes & 1) {
    copy_in(ctx, keys, ksrc, n);
    if (VALS) copy_in(ctx, vals, vsrc, n);
  }
}

}  // namespace

void sort_keys_u32(camfe_ctx ctx, uint32_t* keys, size_t n, int end_bit) {
  radix_sort<uint32_t, false>(ctx, keys, nullptr, n, end_bit);
}

void sort_keys(camfe_ctx ctx, u64* keys, size_t n, int end_bit) {
  radix_sort<u64, false>(ctx, keys, nullptr, n, end_bit);
}

void sort_pairs(camfe_ctx ctx, u64* keys, uint32_t* vals, size_t n, int end_bit, int begin_bit) {
  radix_sort<u64, true>(ctx, keys, vals, n, end_bit, begin_bit);
}

void sort_pairs_u32(camfe_ctx ctx, uint32_t* keys, uint32_t* vals, size_t n, int end_bit) {
  radix_sort<uint32_t, true>(ctx, keys, vals, n, end_bit);
}

void exclusive_scan(camfe_ctx ctx, const int* in, int* out, size_t n) {
  if (n == 0) return;
  int* partials = (int*)ctx->scratch_bytes(tiles_of(n) * sizeof(int));
  scan_with<int>(ctx, in, out, n, partials);
}

void exclusive_scan64(camfe_ctx ctx, const long long* in, long long* out, size_t n) {
  if (n == 0) return;
  long long* partials = (long long*)ctx->scratch_bytes(tiles_of(n) * sizeof(long long));
  scan_with<long long>(ctx, in, out, n, partials);
}

void reduce_sum64(camfe_ctx ctx, const long long* in, long long* out, size_t n) {
  if (n == 0) {
    hipLaunchKernelGGL(k_sum_partials<long long>, dim3(1), dim3(1024), 0, ctx->stream, in, 0LL, out);
    check_launch();
    return;
  }
  const size_t tl = tiles_of(n);
  long long* partials = (long long*)ctx->scratch_bytes(tl * sizeof(long long));
  hipLaunchKernelGGL(k_tile_sums<long long>, dim3((unsigned)tl), dim3(PB), 0, ctx->stream, in, (long long)n, partials);
  hipLaunchKernelGGL(k_sum_partials<long long>, dim3(1), dim3(1024), 0, ctx->stream, (const long long*)partials,
                     (long long)tl, out);
  check_launch();
}

}  // namespace camfe

camfe_status camfe_radix_sort(camfe_ctx ctx, void* keys, int key_bytes, uint32_t* vals, int64_t n, int end_bit) {
  using namespace camfe;
  return guarded([&] {
    CAMFE_REQUIRE(ctx, CAMFE_EINVAL, "null context");
    set_current_ctx(ctx);
    CAMFE_REQUIRE(n >= 0 && n < (int64_t(1) << 31), CAMFE_EINVAL, "n outside [0, 2^31)");
    CAMFE_REQUIRE(key_bytes == 4 || key_bytes == 8, CAMFE_EINVAL, "key_bytes must be 4 or 8");
    CAMFE_REQUIRE(end_bit >= 0 && end_bit <= 8 * key_bytes, CAMFE_EINVAL, "end_bit outside [0, 8 key_bytes]");
    CAMFE_REQUIRE(keys || n == 0, CAMFE_EINVAL, "null keys");
    ctx->use_device();
    if (key_bytes == 8) {
      if (vals) sort_pairs(ctx, (u64*)keys, vals, (size_t)n, end_bit);
      else sort_keys(ctx, (u64*)keys, (size_t)n, end_bit);
    } else {
      if (vals) sort_pairs_u32(ctx, (uint32_t*)keys, vals, (size_t)n, end_bit);
      else sort_keys_u32(ctx, (uint32_t*)keys, (size_t)n, end_bit);
    }
    ctx->sync();
  });
}

camfe_status camfe_exclusive_sum(camfe_ctx ctx, const void* in, void* out, int64_t n, int elem_bytes) {
  using namespace camfe;
  return guarded([&] {
    CAMFE_REQUIRE(ctx, CAMFE_EINVAL, "null context");
    set_current_ctx(ctx);
    CAMFE_REQUIRE(n >= 0, CAMFE_EINVAL, "negative n");
    CAMFE_REQUIRE(elem_bytes == 4 || elem_bytes == 8, CAMFE_EINVAL, "elem_bytes must be 4 or 8");
    CAMFE_REQUIRE((in && out) || n == 0, CAMFE_EINVAL, "null pointer");
    ctx->use_device();
    if (elem_bytes == 8) exclusive_scan64(ctx, (const long long*)in, (long long*)out, (size_t)n);
    else exclusive_scan(ctx, (const int*)in, (int*)out, (size_t)n);
    ctx->sync();
  });
}

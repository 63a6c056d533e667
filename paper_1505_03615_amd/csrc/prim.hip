// Library primitives used as building blocks: stable radix sort, prefix sums
// and reductions (rocPRIM through hipCUB).  Kept in one translation unit so
// the heavy template instantiation compiles once.
#include <hipcub/hipcub.hpp>

#include "common.hpp"

namespace camfe {

void sort_keys(camfe_ctx ctx, u64* keys, size_t n, int end_bit) {
  if (n < 2) return;
  u64* alt = (u64*)ctx->scratch2_bytes(n * sizeof(u64));
  hipcub::DoubleBuffer<u64> db(keys, alt);
  size_t tb = 0;
  CAMFE_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, tb, db, (int)n, 0, end_bit, ctx->stream));
  void* tmp = ctx->scratch_bytes(tb);
  CAMFE_HIP(hipcub::DeviceRadixSort::SortKeys(tmp, tb, db, (int)n, 0, end_bit, ctx->stream));
  if (db.Current() != keys) copy_in(ctx, keys, db.Current(), n);
}

void sort_pairs(camfe_ctx ctx, u64* keys, uint32_t* vals, size_t n, int end_bit) {
  if (n < 2) return;
  unsigned char* s2 = ctx->scratch2_bytes(n * (sizeof(u64) + sizeof(uint32_t)) + 256);
  u64* kalt = (u64*)s2;
  uint32_t* valt = (uint32_t*)(s2 + ((n * sizeof(u64) + 255) & ~size_t(255)));
  hipcub::DoubleBuffer<u64> dk(keys, kalt);
  hipcub::DoubleBuffer<uint32_t> dv(vals, valt);
  size_t tb = 0;
  CAMFE_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, dk, dv, (int)n, 0, end_bit, ctx->stream));
  void* tmp = ctx->scratch_bytes(tb);
  CAMFE_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, dk, dv, (int)n, 0, end_bit, ctx->stream));
  if (dk.Current() != keys) copy_in(ctx, keys, dk.Current(), n);
  if (dv.Current() != vals) copy_in(ctx, vals, dv.Current(), n);
}

void sort_pairs_u32(camfe_ctx ctx, uint32_t* keys, uint32_t* vals, size_t n, int end_bit) {
  if (n < 2) return;
  unsigned char* s2 = ctx->scratch2_bytes(2 * n * sizeof(uint32_t) + 256);
  uint32_t* kalt = (uint32_t*)s2;
  uint32_t* valt = (uint32_t*)(s2 + ((n * sizeof(uint32_t) + 255) & ~size_t(255)));
  hipcub::DoubleBuffer<uint32_t> dk(keys, kalt);
  hipcub::DoubleBuffer<uint32_t> dv(vals, valt);
  size_t tb = 0;
  CAMFE_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, dk, dv, (int)n, 0, end_bit, ctx->stream));
  void* tmp = ctx->scratch_bytes(tb);
  CAMFE_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, dk, dv, (int)n, 0, end_bit, ctx->stream));
  if (dk.Current() != keys) copy_in(ctx, keys, dk.Current(), n);
  if (dv.Current() != vals) copy_in(ctx, vals, dv.Current(), n);
}

void exclusive_scan(camfe_ctx ctx, const int* in, int* out, size_t n) {
  if (n == 0) return;
  size_t tb = 0;
  CAMFE_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, in, out, (int)n, ctx->stream));
  void* tmp = ctx->scratch_bytes(tb);
  CAMFE_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, in, out, (int)n, ctx->stream));
}

void exclusive_scan64(camfe_ctx ctx, const long long* in, long long* out, size_t n) {
  if (n == 0) return;
  size_t tb = 0;
  CAMFE_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, in, out, (int)n, ctx->stream));
  void* tmp = ctx->scratch_bytes(tb);
  CAMFE_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, in, out, (int)n, ctx->stream));
}

void reduce_sum64(camfe_ctx ctx, const long long* in, long long* out, size_t n) {
  size_t tb = 0;
  CAMFE_HIP(hipcub::DeviceReduce::Sum(nullptr, tb, in, out, (int)n, ctx->stream));
  void* tmp = ctx->scratch_bytes(tb);
  CAMFE_HIP(hipcub::DeviceReduce::Sum(tmp, tb, in, out, (int)n, ctx->stream));
}

}  // namespace camfe

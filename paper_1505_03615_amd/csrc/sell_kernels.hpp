// SELL-64 sweep kernels of the V-cycle and of CG: multicolour Gauss-Seidel
// (also SOR with per-row weights), weighted Jacobi, residual, and SpMV with
// per-block dot products, with the slice helpers they share.  Included by
// solve.hip only (the definitions land in its anonymous namespace); bench.py
// keys its recorded HBM traffic of the colour sweep to this file's contents.
#pragma once

#include "solver.hpp"

namespace camfe {
namespace {

// XCD-aware slice order: consecutive workgroups go to different XCDs, so
// give each XCD a contiguous range of slices (neighbouring rows share x).
__device__ inline long long xcd_block(long long b, long long nb) {
  const long long X = 8;
  if (nb < X) return b;
  long long per = nb / X, rem = nb % X;
  long long x = b % X, i = b / X;
  long long base = x * per + min(x, rem);
  long long lim = per + (x < rem ? 1 : 0);
  return i < lim ? base + i : b;   // remainder blocks keep their index
}

// Each 64-row slice is processed by SW wavefronts: wavefront w takes the
// slice's entry columns j = w, w + SW, ... (each load instruction still reads
// one contiguous 64-entry segment), first issuing all of its value/column
// loads, then the gathers of x; partial row sums meet in LDS.  This gives a
// colour pass of n/8 rows enough memory-level parallelism to hide latency.
// Each slice's metadata is one int4 {first entry, end entry, first row, rows
// | flags}, a single scalar load per workgroup.
//
// Columns come in two forms.  A slice flagged C16 (degree 1) stores per
// entry a 16-bit code, colour << 13 | offset, and per slice one base per
// colour (rows are numbered colour by colour, so a slice's neighbours of one
// colour lie close together in that colour's range): column = base[colour] +
// offset.  A slice whose neighbours of some colour span 8192 rows or more
// (where the Morton order jumps) keeps 32-bit columns.  Both forms hold the
// same columns in the same positions, so a row's sum is the same either way.
constexpr int SW = 8;          // wavefronts per slice (default tile)
constexpr int MU = 4;          // entries per lane issued together (default tile)
constexpr int C16 = 0x100;     // slice record flag (in .w above the row count): 16-bit column codes
constexpr int C16_BITS = 13;   // offset bits of a code; the colour takes the 3 above
__host__ __device__ inline int slice_rows(const int4& m) { return m.w & 0xFF; }

// Tiles of the colour sweep that the autotuner chooses from per level
// (camfe_system_autotune): {wavefronts per slice, entries per lane issued
// together}.  Index 0 is the default of every other SELL kernel.
// Tiles 5 and 6 give each wavefront one pass over a row of up to 32 entries
// with fewer wavefronts per slice, so that more slices (and their chains of
// dependent loads) are in flight per CU.
constexpr int NTILE = 7;
__host__ __device__ constexpr int tile_sw(int t) {
  return (t == 1 || t == 5) ? 4 : (t == 3 || t == 4) ? 16 : t == 6 ? 2 : 8;
}
__host__ __device__ constexpr int tile_mu(int t) { return (t == 2 || t == 3) ? 2 : t == 5 ? 8 : t == 6 ? 16 : 4; }

template <class T, int K, int SWV = SW, int MUV = MU>
__device__ inline void slice_row_dot(const int4& m, long long s, int lane, int sub, const int* scol,
                                     const uint16_t* scol16, const int* sbase, const T* sval, const T* x,
                                     T acc[K]) {
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0;
  // lanes past the slice's last row load its padding (value 0, a valid
  // column) rather than wait for the row count before their first load
  const int w = (m.y - m.x) / SL;
  const long long base = m.x + lane;
  if (m.w & C16) {
    // the slice's eight bases are uniform: scalar loads, then a per-lane
    // select by the code's colour (entries past the end decode to base[0],
    // a valid row)
    const int* sb = sbase + s * 8;
    int b[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) b[k] = sb[k];
    for (int j0 = sub; j0 < w; j0 += SWV * MUV) {
      T a[MUV];
      int c[MUV];
#pragma unroll
      for (int u = 0; u < MUV; ++u) {
        const int j = j0 + SWV * u;
        a[u] = j < w ? sval[base + (long long)j * SL] : (T)0;
        const int v = j < w ? (int)scol16[base + (long long)j * SL] : 0;
        const int col = v >> C16_BITS;
        int bb = b[0];
#pragma unroll
        for (int k = 1; k < 8; ++k) bb = col == k ? b[k] : bb;
        c[u] = bb + (v & ((1 << C16_BITS) - 1));
      }
#pragma unroll
      for (int u = 0; u < MUV; ++u)
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] = fma(a[u], x[(long long)c[u] * K + q], acc[q]);
    }
    return;
  }
  for (int j0 = sub; j0 < w; j0 += SWV * MUV) {
    T a[MUV];
    int c[MUV];
#pragma unroll
    for (int u = 0; u < MUV; ++u) {
      const int j = j0 + SWV * u;
      a[u] = j < w ? sval[base + (long long)j * SL] : (T)0;
      c[u] = j < w ? scol[base + (long long)j * SL] : 0;
    }
#pragma unroll
    for (int u = 0; u < MUV; ++u)
#pragma unroll
      for (int q = 0; q < K; ++q) acc[q] = fma(a[u], x[(long long)c[u] * K + q], acc[q]);
  }
}

// sum of the SWV partial sums of each row (valid in wavefront 0 after return)
template <class T, int K, int SWV = SW>
__device__ inline void slice_reduce(T (*red)[K][SL], int lane, int sub, T acc[K]) {
#pragma unroll
  for (int q = 0; q < K; ++q) red[sub][q][lane] = acc[q];
  __syncthreads();
  if (sub == 0) {
#pragma unroll
    for (int q = 0; q < K; ++q) {
      T s = red[0][q][lane];
#pragma unroll
      for (int w = 1; w < SWV; ++w) s += red[w][q][lane];
      acc[q] = s;
    }
  }
}

template <class T, int K, int TILE = 0>
__global__ __launch_bounds__(SL * tile_sw(TILE)) void k_gs(const int4* meta, int s_begin, int s_end, const int* scol,
                                                           const uint16_t* scol16, const int* sbase, const T* sval,
                                                           const T* invd, const T* b, T* x) {
  constexpr int SWV = tile_sw(TILE), MUV = tile_mu(TILE);
  __shared__ T red[SWV][K][SL];
  const int sub = threadIdx.x / SL, lane = threadIdx.x % SL;
  const long long s = s_begin + xcd_block(blockIdx.x, s_end - s_begin);
  const int4 m = meta[s];
  const bool active = lane < slice_rows(m);
  // the writing wavefront fetches b_i, x_i and the weight first, so that these
  // loads overlap the row's dot product instead of following it (no other row
  // of this colour writes x_i)
  const bool writer = sub == 0 && active;
  long long i = 0;
  T di = 0, bi[K], xi[K];
  if (writer) {
    i = m.z + lane;
    di = invd[i];
#pragma unroll
    for (int q = 0; q < K; ++q) {
      bi[q] = b[i * K + q];
      xi[q] = x[i * K + q];
    }
  }
  T acc[K];
  slice_row_dot<T, K, SWV, MUV>(m, s, lane, sub, scol, scol16, sbase, sval, x, acc);
  slice_reduce<T, K, SWV>(red, lane, sub, acc);
  if (writer) {
#pragma unroll
    for (int q = 0; q < K; ++q) x[i * K + q] = xi[q] + (bi[q] - acc[q]) * di;
  }
}

// weighted Jacobi over all slices: x_out = x_in + w_i (b - A x_in), w_i = omega_i / A_ii
template <class T, int K>
__global__ __launch_bounds__(SL * SW) void k_jacobi(const int4* meta, int ns, const int* scol, const uint16_t* scol16,
                                                    const int* sbase, const T* sval, const T* winvd, const T* b,
                                                    const T* x_in, T* x_out) {
  __shared__ T red[SW][K][SL];
  const int sub = threadIdx.x / SL, lane = threadIdx.x % SL;
  const long long s = xcd_block(blockIdx.x, ns);
  const int4 m = meta[s];
  const bool active = lane < slice_rows(m);
  const bool writer = sub == 0 && active;
  long long i = 0;
  T w = 0, bi[K], xi[K];
  if (writer) {   // fetched before the dot product (see k_gs)
    i = m.z + lane;
    w = winvd[i];
#pragma unroll
    for (int q = 0; q < K; ++q) {
      bi[q] = b[i * K + q];
      xi[q] = x_in[i * K + q];
    }
  }
  T acc[K];
  slice_row_dot<T, K>(m, s, lane, sub, scol, scol16, sbase, sval, x_in, acc);
  slice_reduce<T, K>(red, lane, sub, acc);
  if (writer) {
#pragma unroll
    for (int q = 0; q < K; ++q) x_out[i * K + q] = xi[q] + (bi[q] - acc[q]) * w;
  }
}

// r = b - A x over all slices; with nrm != null also accumulate ||r||^2 per column
template <class T, class TR, int K>
__global__ __launch_bounds__(SL * SW) void k_residual(const int4* meta, int ns, const int* scol,
                                                      const uint16_t* scol16, const int* sbase, const T* sval,
                                                      const TR* b, const T* x, TR* r, double* nrm) {
  __shared__ T red[SW][K][SL];
  const int sub = threadIdx.x / SL, lane = threadIdx.x % SL;
  const long long s = xcd_block(blockIdx.x, ns);
  const int4 m = meta[s];
  const bool active = lane < slice_rows(m);
  long long i = 0;
  TR bi[K];
  if (sub == 0 && active) {   // fetched before the dot product (see k_gs)
    i = m.z + lane;
#pragma unroll
    for (int q = 0; q < K; ++q) bi[q] = b[i * K + q];
  }
  T acc[K];
  slice_row_dot<T, K>(m, s, lane, sub, scol, scol16, sbase, sval, x, acc);
  slice_reduce<T, K>(red, lane, sub, acc);
  if (sub != 0) return;
  double loc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) loc[q] = 0.0;
  if (active) {
#pragma unroll
    for (int q = 0; q < K; ++q) {
      TR v = bi[q] - (TR)acc[q];
      r[(long long)i * K + q] = v;
      loc[q] = (double)v * (double)v;
    }
  }
  if (nrm) {   // per-block partial sums of ||r||^2, reduced by k_finalize
#pragma unroll
    for (int q = 0; q < K; ++q) {
      double v = loc[q];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (lane == 0) nrm[(long long)blockIdx.x * K + q] = v;
    }
  }
}

// y = A p (FP64) and pq += p . y per column
template <int K>
__global__ __launch_bounds__(SL * SW) void k_spmv_dot(const int4* meta, int ns, const int* scol,
                                                      const uint16_t* scol16, const int* sbase,
                                                      const double* sval, const double* p, double* y, double* dot) {
  __shared__ double red[SW][K][SL];
  const int sub = threadIdx.x / SL, lane = threadIdx.x % SL;
  const long long s = xcd_block(blockIdx.x, ns);
  const int4 m = meta[s];
  const bool active = lane < slice_rows(m);
  double acc[K];
  slice_row_dot<double, K>(m, s, lane, sub, scol, scol16, sbase, sval, p, acc);
  slice_reduce<double, K>(red, lane, sub, acc);
  if (sub != 0) return;
  double loc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) loc[q] = 0.0;
  if (active) {
    const int i = m.z + lane;
#pragma unroll
    for (int q = 0; q < K; ++q) {
      y[(long long)i * K + q] = acc[q];
      loc[q] = acc[q] * p[(long long)i * K + q];
    }
  }
#pragma unroll
  for (int q = 0; q < K; ++q) {   // per-block partial of p . Ap
    double v = loc[q];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) dot[(long long)blockIdx.x * K + q] = v;
  }
}

}  // namespace
}  // namespace camfe

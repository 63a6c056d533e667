// Cell-block Schwarz smoother (not in the paper; an alternative to its
// Gauss-Seidel smoother, Section 5.2, for the trilinear space): the sweep's
// block product x += omega sum_B w_B R_B^T A_B^-1 R_B r.  Included by
// solve.hip only.
//
// A block holds the functions of one occupied cell (its 8 corners, one
// function per component met in the cell), with the symmetric inverse of its
// unit-diagonal-scaled matrix stored as its packed upper triangle (W (W + 1)
// / 2 values, row by row; rows past the block's functions are zero), its
// weight w_B and the row scales s_i = 1 / sqrt(A_ii): A_B^-1 r_B = s (inverse
// (s r)).  A workgroup stages the packed inverses of its blocks in LDS with
// coalesced loads; a group of W lanes of a wavefront takes one block: lane i
// loads s_i r_i of the block's function i, the group's values meet through
// shuffles, lane i forms its entry of the product from row i of the inverse
// and adds it, times omega w_B s_i, to x_i with an atomic add (a function
// sits in up to eight blocks).  A row with s_i = 0 (zero mass; in FP32 also a
// diagonal whose reciprocal has no FP32 value) takes no part.
#pragma once

#include "solver.hpp"

namespace camfe {
namespace {

// Blocks [b_begin, b_end).  ATOMIC: blocks of the range may share functions
// (atomic adds); otherwise the range is one cell colour (cells whose
// coordinates have the same parities share no corner, hence no function),
// and x is updated with plain adds, one launch per colour.
template <class T, int K, int W, bool ATOMIC>
__global__ __launch_bounds__(256) void k_block_apply(long long b_begin, long long b_end, const int* idx, const T* inv,
                                                     const T* weight, const T* scale, const T* r, T omega, T* x) {
  constexpr int NP = W * (W + 1) / 2, G = 256 / W;
  __shared__ T sm[G * NP];
  const long long b0 = b_begin + blockIdx.x * (long long)G;   // the grid covers the range: b0 < b_end
  const long long nload = (b_end - b0 < G ? b_end - b0 : G) * NP;
  for (int e = threadIdx.x; e < G * NP; e += 256) sm[e] = e < nload ? inv[b0 * NP + e] : (T)0;
  __syncthreads();
  const int grp = threadIdx.x / W, i = threadIdx.x % W;
  const long long b = b0 + grp;
  const bool ok = b < b_end;
  const int f = ok ? idx[b * W + i] : -1;
  const T sf = f >= 0 ? scale[f] : (T)0;
  T rv[K], u[K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    rv[q] = f >= 0 ? sf * r[(long long)f * K + q] : (T)0;
    u[q] = 0;
  }
  const T* A = sm + grp * NP;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    const T a = A[i <= j ? bpk<W>(i, j) : bpk<W>(j, i)];   // entry (i, j) of the symmetric inverse
#pragma unroll
    for (int q = 0; q < K; ++q) u[q] = fma(a, __shfl(rv[q], j, W), u[q]);
  }
  if (f >= 0 && sf != (T)0) {
    const T w = omega * weight[b] * sf;
#pragma unroll
    for (int q = 0; q < K; ++q) {
      if (ATOMIC) atomicAdd(&x[(long long)f * K + q], w * u[q]);
      else x[(long long)f * K + q] += w * u[q];
    }
  }
}

}  // namespace
}  // namespace camfe

// Set-up of the cell-block Schwarz smoother (trilinear space only; not in the
// paper, whose smoother is Gauss-Seidel, Section 5.2).
//
// At every depth of a solver state, one block per occupied cell: the
// functions whose support contains the cell and whose component holds one of
// the cell's triangles, i.e. for each of the cell's (cell, triangle) pairs the
// function at each of the cell's 8 corners labelled by that triangle
// (pair_rows).  Functions of zero computed mass are left out.  A cell with
// more than BLOCK_CAP functions (many separate pieces of surface in one
// cell, at coarse split depths) gives one single-function block per function
// instead.  A block's weight is 1 / (the largest number of blocks holding one
// of its functions).  Each block's inverse is D^-1/2 (D^-1/2 A_B D^-1/2 + eps I)^-1
// D^-1/2 with the state's coarse_eps (the coarsest solve's treatment of
// exactly dependent functions): the middle factor is computed in FP64 by a
// Cholesky factorisation and kept in FP64 and FP32 as its packed upper
// triangle, the outer D^-1/2 as one scale per row applied by the sweep.  The
// damping of the weighted block sum is chosen per depth at set-up (solve.hip,
// estimate_block_damping): the weights alone do not make a sweep contract.
//
// Deduplication per cell: the functions at one corner are a contiguous range
// of the canonical numbering (one per component, cfirst of the corner's
// support), so each corner keeps a 64-bit mask of the components met (a
// corner of more than 64 components is scanned pair by pair instead).
#include <algorithm>
#include <vector>

#include "solver.hpp"

namespace camfe {
namespace {

constexpr int BLK = 256;
constexpr int BLOCK_CAP = 16;

// first pair of each cell (pairs sorted by cell key), ncells + 1 entries
__global__ void k_cell_flags(const u64* pairs, long long n, int* flag) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  flag[i] = (i == 0 || (pairs[i] >> TRI_BITS) != (pairs[i - 1] >> TRI_BITS)) ? 1 : 0;
}
__global__ void k_cell_start(const int* flag, const int* pos, long long n, long long ncell, int* cstart) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n && flag[i]) cstart[pos[i]] = (int)i;
  if (i == 0) cstart[ncell] = (int)n;
}

// the canonical range of functions at each corner of a cell
__device__ inline void corner_ranges(u64 cell, const u64* ckey, int ncorn, const int* cfirst, int first[8],
                                     int count[8]) {
  long long c[3];
  demorton(cell, c);
  for (int j = 0; j < 8; ++j) {
    const u64 k = morton((u64)(c[0] + (j & 1)), (u64)(c[1] + ((j >> 1) & 1)), (u64)(c[2] + (j >> 2)));
    int lo = 0, hi = ncorn;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (ckey[mid] < k) lo = mid + 1;
      else hi = mid;
    }
    const bool found = lo < ncorn && ckey[lo] == k;
    first[j] = found ? cfirst[lo] : 0;
    count[j] = found ? cfirst[lo + 1] - cfirst[lo] : 0;
  }
}

// Calls emit(internal row) once for each function of the cell's block
// candidate list (functions of zero mass left out), corner by corner, in a
// fixed order.  A corner's components met in the cell are a 64-bit mask when
// the corner has at most 64 components; a corner with more (many separate
// pieces of surface, at coarse depths) is deduplicated by scanning the
// cell's earlier pairs.  err bit 1: a pair's function outside its corner.
template <class Emit>
__device__ inline void cell_functions(long long cell_i, const u64* pairs, const int* cstart, const int* pair_rows,
                                      const u64* ckey, int ncorn, const int* cfirst, const int* iperm,
                                      const double* invd, int* err, Emit emit) {
  int first[8], count[8];
  corner_ranges(pairs[cstart[cell_i]] >> TRI_BITS, ckey, ncorn, cfirst, first, count);
  const int p0 = cstart[cell_i], p1 = cstart[cell_i + 1];
  for (int j = 0; j < 8; ++j) {
    if (count[j] <= 64) {
      unsigned long long mask = 0;
      for (int p = p0; p < p1; ++p) {
        const int l = pair_rows[(long long)p * 8 + j] - first[j];
        if (l < 0 || l >= count[j]) { atomicOr(err, 1); continue; }
        mask |= 1ULL << l;
      }
      while (mask) {
        const int l = __ffsll(mask) - 1;
        mask &= mask - 1;
        const int r = iperm[first[j] + l];
        if (invd[r] != 0.0) emit(r);
      }
    } else {
      for (int p = p0; p < p1; ++p) {
        const int f = pair_rows[(long long)p * 8 + j];
        bool seen = false;
        for (int q = p0; q < p && !seen; ++q) seen = pair_rows[(long long)q * 8 + j] == f;
        if (seen) continue;
        const int r = iperm[f];
        if (invd[r] != 0.0) emit(r);
      }
    }
  }
}

__global__ void k_block_count(long long ncell, const u64* pairs, const int* cstart, const int* pair_rows,
                              const u64* ckey, int ncorn, const int* cfirst, const int* iperm, const double* invd,
                              int* cnt8, int* cnt16, int* err) {
  const long long c = blockIdx.x * (long long)BLK + threadIdx.x;
  if (c >= ncell) return;
  int m = 0;
  cell_functions(c, pairs, cstart, pair_rows, ckey, ncorn, cfirst, iperm, invd, err, [&](int) { ++m; });
  cnt8[c] = (m >= 1 && m <= 8) ? 1 : (m > BLOCK_CAP ? m : 0);
  cnt16[c] = (m > 8 && m <= BLOCK_CAP) ? 1 : 0;
}

__global__ void k_block_fill(long long ncell, const u64* pairs, const int* cstart, const int* pair_rows,
                             const u64* ckey, int ncorn, const int* cfirst, const int* iperm, const double* invd,
                             const int* off8, const int* off16, const int* cnt8, const int* cnt16, int* idx8,
                             int* idx16, int* err) {
  const long long c = blockIdx.x * (long long)BLK + threadIdx.x;
  if (c >= ncell) return;
  int* out;
  int W, stride, m;
  if (cnt16[c]) { out = idx16 + (long long)off16[c] * 16; W = 16; stride = 1; m = BLOCK_CAP; }
  else if (cnt8[c] == 1) { out = idx8 + (long long)off8[c] * 8; W = 8; stride = 1; m = 8; }
  else if (cnt8[c] > 1) { out = idx8 + (long long)off8[c] * 8; W = 8; stride = 8; m = cnt8[c]; }   // single-function blocks
  else return;
  int w = 0;
  cell_functions(c, pairs, cstart, pair_rows, ckey, ncorn, cfirst, iperm, invd, err, [&](int r) {
    if (w >= m) { atomicOr(err, 4); return; }   // the count pass saw fewer
    out[w * stride] = r;
    if (stride > 1)
      for (int z = 1; z < 8; ++z) out[w * stride + z] = -1;
    ++w;
  });
  if (stride == 1)
    for (; w < W; ++w) out[w] = -1;
}

// colour of each occupied cell: the parities of its coordinates
__global__ void k_cell_colour(long long ncell, const u64* pairs, const int* cstart, int* colour) {
  const long long c = blockIdx.x * (long long)BLK + threadIdx.x;
  if (c >= ncell) return;
  long long x[3];
  demorton(pairs[cstart[c]] >> TRI_BITS, x);
  colour[c] = (int)((x[0] & 1) + 2 * (x[1] & 1) + 4 * (x[2] & 1));
}
__global__ void k_colour_mask(long long ncell, const int* colour, int k, const int* cnt, int* out) {
  const long long c = blockIdx.x * (long long)BLK + threadIdx.x;
  if (c > ncell) return;
  out[c] = (c < ncell && colour[c] == k) ? cnt[c] : 0;
}
__global__ void k_colour_offsets(long long ncell, const int* colour, int k, const int* pre, long long base, int* off) {
  const long long c = blockIdx.x * (long long)BLK + threadIdx.x;
  if (c < ncell && colour[c] == k) off[c] = (int)(base + pre[c]);
}

// block offsets of every cell, colour by colour (cell order within a
// colour); bc receives the colour ranges, and the total is returned
long long colour_major_offsets(camfe_ctx ctx, long long nc, const int* colour, const int* cnt, int* off,
                               long long bc[9]) {
  DArr<int> masked(nc + 1), pre(nc + 1);
  long long base = 0;
  for (int k = 0; k < 8; ++k) {
    bc[k] = base;
    hipLaunchKernelGGL(k_colour_mask, grid_for(nc + 1, BLK), BLK, 0, ctx->stream, nc, colour, k, cnt, masked.p);
    exclusive_scan(ctx, masked.p, pre.p, (size_t)nc + 1);
    hipLaunchKernelGGL(k_colour_offsets, grid_for(nc, BLK), BLK, 0, ctx->stream, nc, colour, k, (const int*)pre.p,
                       base, off);
    check_launch();
    base += read_scalar(ctx, pre.p + nc);
  }
  bc[8] = base;
  return base;
}

// entry (r, c) of A = M + t L (canonical CSR, ascending columns)
__device__ inline double a_entry(const int* ptr, const int* col, const double* M, const double* L, double t, int r,
                                 int c) {
  int lo = ptr[r], hi = ptr[r + 1];
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (col[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  return (lo < ptr[r + 1] && col[lo] == c) ? M[lo] + t * L[lo] : 0.0;
}

// Inverse of the unit-diagonal-scaled block plus eps I (its entries are at
// most 1 / eps in size); the scaling s_i = 1 / sqrt(A_ii) is applied by the
// sweep, on both sides, so no entry of the size of 1 / A_ii of a
// rounding-sliver function is ever formed
template <int W>
__global__ void k_block_invert(long long nb, const int* idx, const int* perm, const int* ptr, const int* col,
                               const double* M, const double* L, double t, double eps, double* inv64, float* inv32,
                               int* mult, int* err) {
  const long long b = blockIdx.x * (long long)BLK + threadIdx.x;
  if (b >= nb) return;
  int f[W], m = 0;
  for (int i = 0; i < W; ++i) {
    const int r = idx[b * W + i];
    if (r >= 0) f[m++] = r;
  }
  double a[W * W], sc[W];
  for (int i = 0; i < m; ++i) sc[i] = 1.0 / sqrt(a_entry(ptr, col, M, L, t, perm[f[i]], perm[f[i]]));
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j)
      a[i * W + j] = a_entry(ptr, col, M, L, t, perm[f[i]], perm[f[j]]) * sc[i] * sc[j] + (i == j ? eps : 0.0);
  // Cholesky (lower triangle in place)
  for (int j = 0; j < m; ++j) {
    double d = a[j * W + j];
    for (int k = 0; k < j; ++k) d -= a[j * W + k] * a[j * W + k];
    if (!(d > 0.0)) { atomicOr(err, 2); d = 1.0; }
    d = sqrt(d);
    a[j * W + j] = d;
    for (int i = j + 1; i < m; ++i) {
      double s = a[i * W + j];
      for (int k = 0; k < j; ++k) s -= a[i * W + k] * a[j * W + k];
      a[i * W + j] = s / d;
    }
  }
  constexpr int NP = W * (W + 1) / 2;
  double* o64 = inv64 + b * (long long)NP;
  float* o32 = inv32 + b * (long long)NP;
  for (int i = 0; i < NP; ++i) { o64[i] = 0.0; o32[i] = 0.0f; }
  for (int j = 0; j < m; ++j) {
    double e[W];
    for (int i = 0; i < m; ++i) e[i] = i == j ? 1.0 : 0.0;
    for (int i = 0; i < m; ++i) {   // L y = e
      double s = e[i];
      for (int k = 0; k < i; ++k) s -= a[i * W + k] * e[k];
      e[i] = s / a[i * W + i];
    }
    for (int i = m - 1; i >= 0; --i) {   // L^T z = y
      double s = e[i];
      for (int k = i + 1; k < m; ++k) s -= a[k * W + i] * e[k];
      e[i] = s / a[i * W + i];
    }
    for (int i = 0; i <= j; ++i) {   // rows up to j of column j: the packed upper triangle
      o64[bpk<W>(i, j)] = e[i];
      o32[bpk<W>(i, j)] = (float)e[i];
    }
  }
  for (int i = 0; i < m; ++i) atomicAdd(&mult[f[i]], 1);
}

// s_i = 1 / sqrt(A_ii) per row (0 for a row of zero mass; in FP32 also 0
// where 1 / A_ii has no FP32 value, the rows the FP32 sweeps skip)
__global__ void k_block_scale(const double* invd, long long n, double* s64, float* s32) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  const double v = invd[i] > 0.0 ? sqrt(invd[i]) : 0.0;
  s64[i] = v;
  s32[i] = invd[i] > 0.0 && invd[i] < 3.0e38 ? (float)v : 0.0f;
}

// weight of each block: 1 / (the largest number of blocks holding one of
// its functions), so that the weights of the blocks holding any function sum
// to at most 1 and a sweep is an A-norm contraction
template <int W>
__global__ void k_block_weight(long long nb, const int* idx, const int* mult, double* w64, float* w32) {
  const long long b = blockIdx.x * (long long)BLK + threadIdx.x;
  if (b >= nb) return;
  int mx = 1;
  for (int i = 0; i < W; ++i) {
    const int r = idx[b * W + i];
    if (r >= 0) mx = max(mx, mult[r]);
  }
  w64[b] = 1.0 / mx;
  w32[b] = (float)(1.0 / mx);
}

void build_level(camfe_sys s, SolverState* S, int d) {
  camfe_ctx ctx = S->ctx;
  hipStream_t st = ctx->stream;
  const HLevel& H = s->h->lev[d];
  const SLevel& SL_ = s->lev[d];
  GLevel& G = S->lev[d];
  const long long np = (long long)H.npairs, nc = (long long)H.ncells, n = (long long)G.n;
  DArr<int> err(1);
  zero(ctx, err.p, 1);
  DArr<int> flag(std::max(np, 1LL)), pos(std::max(np, 1LL)), cstart(nc + 1);
  hipLaunchKernelGGL(k_cell_flags, grid_for(np, BLK), BLK, 0, st, H.pairs.p, np, flag.p);
  exclusive_scan(ctx, flag.p, pos.p, (size_t)np);
  hipLaunchKernelGGL(k_cell_start, grid_for(np, BLK), BLK, 0, st, flag.p, pos.p, np, nc, cstart.p);
  DArr<int> cnt8(nc + 1), cnt16(nc + 1), off8(nc + 1), off16(nc + 1);
  zero(ctx, cnt8.p, nc + 1);
  zero(ctx, cnt16.p, nc + 1);
  hipLaunchKernelGGL(k_block_count, grid_for(nc, BLK), BLK, 0, st, nc, H.pairs.p, cstart.p, H.pair_rows.p,
                     H.ckey.p, (int)H.ncorn, H.cfirst.p, G.iperm.p, G.invd64.p, cnt8.p, cnt16.p, err.p);
  check_launch();
  DArr<int> colour(std::max(nc, 1LL));
  hipLaunchKernelGGL(k_cell_colour, grid_for(nc, BLK), BLK, 0, st, nc, H.pairs.p, cstart.p, colour.p);
  G.nb8 = colour_major_offsets(ctx, nc, colour.p, cnt8.p, off8.p, G.bc8);
  G.nb16 = colour_major_offsets(ctx, nc, colour.p, cnt16.p, off16.p, G.bc16);
  G.bidx8.alloc(std::max(G.nb8, 1LL) * 8);
  G.bidx16.alloc(std::max(G.nb16, 1LL) * 16);
  hipLaunchKernelGGL(k_block_fill, grid_for(nc, BLK), BLK, 0, st, nc, H.pairs.p, cstart.p, H.pair_rows.p, H.ckey.p,
                     (int)H.ncorn, H.cfirst.p, G.iperm.p, G.invd64.p, off8.p, off16.p, cnt8.p, cnt16.p, G.bidx8.p,
                     G.bidx16.p, err.p);
  G.binv8_64.alloc(std::max(G.nb8, 1LL) * 36);
  G.binv8_32.alloc(std::max(G.nb8, 1LL) * 36);
  G.binv16_64.alloc(std::max(G.nb16, 1LL) * 136);
  G.binv16_32.alloc(std::max(G.nb16, 1LL) * 136);
  DArr<int> mult(n);
  zero(ctx, mult.p, n);
  if (G.nb8)
    hipLaunchKernelGGL(k_block_invert<8>, grid_for(G.nb8, BLK), BLK, 0, st, G.nb8, G.bidx8.p, G.perm.p,
                       SL_.ptr.p, SL_.col.p, SL_.M.p, SL_.L.p, S->t, S->coarse_eps, G.binv8_64.p, G.binv8_32.p,
                       mult.p, err.p);
  if (G.nb16)
    hipLaunchKernelGGL(k_block_invert<16>, grid_for(G.nb16, BLK), BLK, 0, st, G.nb16, G.bidx16.p, G.perm.p,
                       SL_.ptr.p, SL_.col.p, SL_.M.p, SL_.L.p, S->t, S->coarse_eps, G.binv16_64.p, G.binv16_32.p,
                       mult.p, err.p);
  G.bs64.alloc(n);
  G.bs32.alloc(n);
  hipLaunchKernelGGL(k_block_scale, grid_for(n, BLK), BLK, 0, st, G.invd64.p, n, G.bs64.p, G.bs32.p);
  G.bw8_64.alloc(std::max(G.nb8, 1LL));
  G.bw8_32.alloc(std::max(G.nb8, 1LL));
  G.bw16_64.alloc(std::max(G.nb16, 1LL));
  G.bw16_32.alloc(std::max(G.nb16, 1LL));
  if (G.nb8)
    hipLaunchKernelGGL(k_block_weight<8>, grid_for(G.nb8, BLK), BLK, 0, st, G.nb8, G.bidx8.p, mult.p, G.bw8_64.p,
                       G.bw8_32.p);
  if (G.nb16)
    hipLaunchKernelGGL(k_block_weight<16>, grid_for(G.nb16, BLK), BLK, 0, st, G.nb16, G.bidx16.p, mult.p,
                       G.bw16_64.p, G.bw16_32.p);
  check_launch();
  const int e = read_scalar(ctx, err.p);
  CAMFE_REQUIRE(!(e & 5), CAMFE_EDEVICE, "cell blocks: inconsistent (cell, triangle) functions");
  CAMFE_REQUIRE(!(e & 2), CAMFE_ESINGULAR, "cell blocks: a block matrix is not positive definite");
}

}  // namespace

void build_cell_blocks(camfe_sys s, SolverState* S) {
  CAMFE_REQUIRE(s->h->degree == 1, CAMFE_EINVAL, "the cell-block smoother is defined for degree 1");
  CAMFE_REQUIRE(!S->batch, CAMFE_EINVAL, "the batched solver takes Gauss-Seidel only");
  // (a coarsest depth solved directly needs no smoother)
  for (int d = S->direct ? S->d0 + 1 : S->d0; d <= S->D; ++d) build_level(s, S, d);
  S->ctx->sync();
  S->blocks_ready = true;
}

}  // namespace camfe

// Multigrid solver on the GPU (Sections 3.2, 4.3, 5.2; discussion of 5.3).
//
// Layout per depth: functions renumbered colour by colour (a colour class
// never couples with itself, so a colour sweep is a parallel Gauss-Seidel
// step), the matrix A = M + t L packed as SELL-64 (slices of 64 consecutive
// rows, column-major inside a slice, one lane per row: every entry load of a
// wavefront is one contiguous 512 B (FP64) or 256 B (FP32) segment).
// Transfers: P (fine rows gather at most 8 coarse parents) and R = P^T
// (coarse rows gather their fine children), both explicit CSR so that
// restriction needs no atomics.  Coarsest depth: dense inverse of the
// unit-diagonal-scaled matrix plus eps * Id, applied as a matrix-vector product.
//
// V-cycle: nu_pre forward colour sweeps, residual, restriction, recursion
// with zero start, prolongation-add, nu_post reverse colour sweeps; symmetric,
// hence usable as a CG preconditioner.  Precision 1 runs the whole V-cycle in
// FP32 while CG recurrences, the residual and the coarsest solve stay FP64.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <functional>
#include <string>
#include <map>

#include <type_traits>

#include "solver.hpp"
#include "sell_kernels.hpp"
#include "block_kernels.hpp"
#include <climits>

namespace camfe {

namespace {
constexpr int BLK = SBLK;
constexpr int SORT_MIN_ROWS = 1 << 19;  // default: rows of a colour from which its rows are sorted by length
constexpr int SORT_WINDOW = 1024;      // rows per sorted window (16 slices)
}  // namespace

void destroy_solver(SolverState* s) { delete s; }

namespace {

// --------------------------------------------------------------- kernels
__global__ void k_colour(const u64* fkey, long long n, int degree, uint32_t* colour, uint32_t* idx) {
  long long f = blockIdx.x * (long long)BLK + threadIdx.x;
  if (f >= n) return;
  long long c[3];
  demorton(fkey[f], c);
  uint32_t col = degree == 1 ? (uint32_t)((c[0] & 1) + 2 * (c[1] & 1) + 4 * (c[2] & 1))
                             : (uint32_t)((c[0] % 3) + 3 * (c[1] % 3) + 9 * (c[2] % 3));
  colour[f] = col;
  idx[f] = (uint32_t)f;
}
__global__ void k_iperm(const uint32_t* perm, long long n, int* iperm, int* permi) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  iperm[perm[i]] = (int)i;
  permi[i] = (int)perm[i];
}
// sort keys that order the rows of each colour window by decreasing row length
// (colours outside mask keep their order): window index << 8 | (255 - length)
__global__ void k_window_keys(const int* perm, const int* ptr, long long n, const int* coff, const int* wbase,
                              int ncol, int mask, uint32_t* key, uint32_t* val) {
  const long long r = blockIdx.x * (long long)BLK + threadIdx.x;
  if (r >= n) return;
  int c = 0;
  while (c + 1 < ncol && r >= coff[c + 1]) ++c;
  const int f = perm[r];
  const int len = ptr[f + 1] - ptr[f];
  const uint32_t lk = ((mask >> c) & 1) ? 255u - (uint32_t)min(len, 255) : 0u;
  key[r] = ((uint32_t)(wbase[c] + (int)((r - coff[c]) / SORT_WINDOW)) << 8) | lk;
  val[r] = (uint32_t)f;
}
__global__ void k_slice_width(const int* ptr, const int* perm, const int* row0, const int* rows, long long ns,
                              int* width) {
  long long s = blockIdx.x * (long long)BLK + threadIdx.x;
  if (s >= ns) return;
  int w = 0;
  for (int l = 0; l < rows[s]; ++l) {
    int f = perm[row0[s] + l];
    w = max(w, ptr[f + 1] - ptr[f]);
  }
  width[s] = w * SL;
}
// v as FP32, or 0 where it has no finite FP32 value
__device__ inline float f32_or_zero(double v) { return fabs(v) < 3.0e38 ? (float)v : 0.0f; }

// pack A = M + t L of internal row i into its slice (valid lanes only)
__global__ void k_sell_fill(const int* ptr, const int* col, const double* M, const double* L, double t,
                            const int* perm, const int* iperm, const int* sl_ptr, const int* row0, const int* rows,
                            long long ns, int* scol, double* sval, float* sval32, double* invd, float* invd32) {
  long long g = blockIdx.x * (long long)BLK + threadIdx.x;
  long long s = g / SL;
  int lane = (int)(g - s * SL);
  if (s >= ns || lane >= rows[s]) return;
  const int width = (sl_ptr[s + 1] - sl_ptr[s]) / SL;
  const int i = row0[s] + lane;
  const int f = perm[i];
  const int b = ptr[f];
  const int len = ptr[f + 1] - b;
  double diag = 0.0;
  for (int j = 0; j < width; ++j) {
    long long o = sl_ptr[s] + (long long)j * SL + lane;
    if (j < len) {
      double a = M[b + j] + t * L[b + j];
      int c = col[b + j];
      scol[o] = iperm[c];
      sval[o] = a;
      sval32[o] = (float)a;
      if (c == f) diag = a;
    } else {
      scol[o] = i;
      sval[o] = 0.0;
      sval32[o] = 0.0f;
    }
  }
  // a function of zero computed mass has an empty row: nothing to relax; a
  // diagonal so small that 1 / A_ii has no FP32 value (rounding slivers) makes
  // the row numerically empty in single precision, and the FP32 sweeps skip it
  invd[i] = diag != 0.0 ? 1.0 / diag : 0.0;
  invd32[i] = diag != 0.0 ? f32_or_zero(1.0 / diag) : 0.0f;
}
__global__ void k_sell_pad(const int* sl_ptr, const int* row0, const int* rows, long long ns, int* scol,
                           double* sval, float* sval32) {
  long long g = blockIdx.x * (long long)BLK + threadIdx.x;
  long long s = g / SL;
  int lane = (int)(g - s * SL);
  if (s >= ns || lane < rows[s]) return;
  const int width = (sl_ptr[s + 1] - sl_ptr[s]) / SL;
  for (int j = 0; j < width; ++j) {
    long long o = sl_ptr[s] + (long long)j * SL + lane;
    scol[o] = row0[s];
    sval[o] = 0.0;
    sval32[o] = 0.0f;
  }
}

// 16-bit column codes of one slice, one wavefront per slice (degree 1: 8
// colours).  The smallest and largest column of each colour among the
// slice's entries (padding included) meet by shuffles; when every colour
// spans fewer than 2^C16_BITS rows the slice gets its codes colour << 13 |
// (column - base), its eight bases (a colour it lacks takes the slice's first
// row, so that the padding lanes' code 0 still decodes to a valid row) and
// the C16 flag, and `count` one more.
struct ColourStarts { int c[9]; };
__device__ inline int colour_of_row(const ColourStarts& co, int r) {
  int c = 0;
#pragma unroll
  for (int k = 1; k < 8; ++k) c += r >= co.c[k] ? 1 : 0;
  return c;
}
__global__ __launch_bounds__(64) void k_sell_compact(long long ns, ColourStarts co, const int* scol, int4* meta,
                                                     int* sbase, uint16_t* scol16, unsigned long long* count) {
  const long long s = blockIdx.x;
  if (s >= ns) return;
  const int lane = threadIdx.x;
  const int4 m = meta[s];
  const int w = (m.y - m.x) / SL;
  int lo[8], hi[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) { lo[k] = INT_MAX; hi[k] = INT_MIN; }
  for (int j = 0; j < w; ++j) {
    const int col = scol[m.x + lane + (long long)j * SL];
    const int c = colour_of_row(co, col);
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (c == k) { lo[k] = min(lo[k], col); hi[k] = max(hi[k], col); }
  }
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    for (int o = 32; o > 0; o >>= 1) {
      lo[k] = min(lo[k], __shfl_xor(lo[k], o));
      hi[k] = max(hi[k], __shfl_xor(hi[k], o));
    }
    if (hi[k] >= lo[k] && hi[k] - lo[k] >= (1 << C16_BITS)) ok = false;
    if (hi[k] < lo[k]) lo[k] = m.z;
  }
  if (!ok) return;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (lane == k) sbase[s * 8 + k] = lo[k];
  for (int j = 0; j < w; ++j) {
    const long long e = m.x + lane + (long long)j * SL;
    const int col = scol[e];
    const int c = colour_of_row(co, col);
    int b = lo[0];
#pragma unroll
    for (int k = 1; k < 8; ++k) b = c == k ? lo[k] : b;
    scol16[e] = (uint16_t)((c << C16_BITS) | (col - b));
  }
  if (lane == 0) {
    meta[s].w = m.w | C16;
    atomicAdd(count, 1ULL);
  }
}

// transfer matrices in internal numbering
__global__ void k_p_count(const int* Pptr, const int* permf, long long nf, int* cnt) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= nf) return;
  int f = permf[i];
  cnt[i] = Pptr[f + 1] - Pptr[f];
}
__global__ void k_p_fill(const int* Pptr, const int* Pcol, const double* Pw, const int* permf, const int* ipermc,
                         long long nf, const int* optr, int* ocol, double* ow, float* ow32, uint32_t* rkey,
                         uint32_t* rval) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= nf) return;
  int f = permf[i];
  int o = optr[i];
  for (int e = Pptr[f]; e < Pptr[f + 1]; ++e, ++o) {
    ocol[o] = ipermc[Pcol[e]];
    ow[o] = Pw[e];
    ow32[o] = (float)Pw[e];
    rkey[o] = (uint32_t)ocol[o];
    rval[o] = (uint32_t)o;
  }
}
__global__ void k_r_fill(const uint32_t* rkey, const uint32_t* rval, long long nnz, const int* prow_of,
                         const double* pw, int* rcol, double* rw, float* rw32) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= nnz) return;
  uint32_t e = rval[i];
  rcol[i] = prow_of[e];
  rw[i] = pw[e];
  rw32[i] = (float)pw[e];
}
__global__ void k_row_of_entry(const int* ptr, long long n, int* row_of) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  for (int e = ptr[i]; e < ptr[i + 1]; ++e) row_of[e] = (int)i;
}
__global__ void k_ptr_from_sorted(const uint32_t* key, long long nnz, long long n, int* ptr) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= nnz) return;
  long long v = key[i];
  long long pv = i == 0 ? -1 : (long long)key[i - 1];
  for (long long w = pv + 1; w <= v; ++w) ptr[w] = (int)i;
  if (i == nnz - 1)
    for (long long w = v + 1; w <= n; ++w) ptr[w] = (int)nnz;
}

// coarsest: dense scaled matrix (internal order), Cholesky, inverse
__global__ void k_dense_scaled(const int* ptr, const int* col, const double* M, const double* L, double t,
                               const int* perm, const int* iperm, long long n, double eps, double* A) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  int f = perm[i];
  double di = 0.0;
  for (int e = ptr[f]; e < ptr[f + 1]; ++e)
    if (col[e] == f) di = M[e] + t * L[e];
  if (di > 0.0)
    for (int e = ptr[f]; e < ptr[f + 1]; ++e) {
      int c = col[e];
      double dc = 0.0;
      for (int q = ptr[c]; q < ptr[c + 1]; ++q)
        if (col[q] == c) dc = M[q] + t * L[q];
      if (dc > 0.0) A[i * n + iperm[c]] = (M[e] + t * L[e]) / sqrt(di * dc);
    }
  // zero-mass functions get an identity row (their right-hand side is 0)
  A[i * n + i] = (di > 0.0 ? A[i * n + i] : 1.0) + eps;
}
__global__ void k_inv_sqrt_diag(int n, double* s, const double* diagsrc) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) s[i] = diagsrc[i] > 0.0 ? 1.0 / sqrt(diagsrc[i]) : 0.0;
}
__global__ void k_diag_of(const int* ptr, const int* col, const double* M, const double* L, double t,
                          const int* perm, long long n, double* dg) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  int f = perm[i];
  double v = 0.0;
  for (int e = ptr[f]; e < ptr[f + 1]; ++e)
    if (col[e] == f) v = M[e] + t * L[e];
  dg[i] = v;
}

// ------------------------------------------------------ V-cycle kernels
// Batched solves gate the row-parallel kernels by member: with gate != null a
// workgroup whose rows belong to a member m with act[m] == 0 (every column of
// it converged) returns at once.  A member's rows are padded to whole
// BLK-row blocks, so each block has one member (gate[block]); its slices are
// emptied in the gated slice records instead (k_gate_meta).
__device__ inline bool gated_off(const int* gate, const int* act, long long blk) {
  return gate && !act[gate[blk]];
}

// b_c = R r_f (coarse rows gather their fine children, 8 lanes per row) and
// x_c = 0 for the recursion (gate: member of each BLK-row block of the coarse level)
constexpr int RL = 8;
template <class T, int K>
__global__ void k_restrict(const int* Rptr, const int* Rcol, const T* Rw, long long nc, const T* rf, T* bc, T* xc,
                           const T* dinv, long long n0c, const int* gate, const int* act) {
  if (gated_off(gate, act, blockIdx.x * (long long)(BLK / RL) / BLK)) return;
  const long long g = blockIdx.x * (long long)BLK + threadIdx.x;
  const long long i = g / RL;
  const int sub = (int)(g % RL);
  T acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0;
  if (i < nc)
    for (int e = Rptr[i] + sub; e < Rptr[i + 1]; e += RL) {
      const T w = Rw[e];
      const int c = Rcol[e];
#pragma unroll
      for (int q = 0; q < K; ++q) acc[q] = fma(w, rf[(long long)c * K + q], acc[q]);
    }
#pragma unroll
  for (int q = 0; q < K; ++q)
    for (int o = RL / 2; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o);
  if (i < nc && sub < K) {
    // lane `sub` writes column `sub`
    T v = acc[0];
#pragma unroll
    for (int q = 1; q < K; ++q) if (sub == q) v = acc[q];
    bc[i * K + sub] = v;
    // x_c starts at zero; with dinv, the first sweep's colour-0 rows (the
    // first n0c) are relaxed here: from x = 0, Gauss-Seidel gives b_i * dinv_i
    xc[i * K + sub] = (dinv && i < n0c) ? v * dinv[i] : (T)0;
  }
}

// x_f += P x_c (gate: member of each BLK-row block of the fine level)
template <class T, int K>
__global__ void k_prolong(const int* Pptr, const int* Pcol, const T* Pw, long long nf, const T* xc, T* xf,
                          const int* gate, const int* act) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= nf || gated_off(gate, act, blockIdx.x)) return;
  T acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0;
  for (int e = Pptr[i]; e < Pptr[i + 1]; ++e) {
    const T w = Pw[e];
    const int c = Pcol[e];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = fma(w, xc[(long long)c * K + q], acc[q]);
  }
#pragma unroll
  for (int q = 0; q < K; ++q) xf[i * K + q] += acc[q];
}

// x = Ainv b at the coarsest depth, one wavefront per row; the inverse is
// FP64 in both precisions (in FP32 the regularised inverse of a singular
// coarsest matrix would lose everything but its null-space term)
template <class T, int K>
__global__ void k_coarse(const double* Ainv, int n, const T* b, T* x) {
  long long wave = (blockIdx.x * (long long)BLK + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (wave >= n) return;
  double acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0.0;
  // unrolled so that several row loads are in flight per lane (the sums
  // keep their order)
#pragma unroll 8
  for (int j = lane; j < n; j += 64) {
    const double a = (double)Ainv[wave * n + j];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] += a * (double)b[(long long)j * K + q];
  }
#pragma unroll
  for (int q = 0; q < K; ++q) {
    double v = acc[q];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) x[wave * K + q] = (T)v;
  }
}

// batched coarse solves: x = Ainv_j b on the rows of every mesh j whose
// coarsest depth is this level (one wavefront per row; member j of the
// batch is cbmem[j], skipped once it stopped iterating)
template <class T, int K>
__global__ void k_coarse_b(int nm, const int* rowoff, const int* cum, const long long* aoff, const double* ainv,
                           const T* b, T* x, const int* cbmem, const int* act) {
  long long wave = (blockIdx.x * (long long)BLK + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (wave >= cum[nm]) return;
  int j = 0;
  while (cum[j + 1] <= wave) ++j;
  if (!act[cbmem[j]]) return;
  const int n = cum[j + 1] - cum[j];
  const long long lr = wave - cum[j];
  const double* A = ainv + aoff[j];
  const long long r0 = rowoff[j];
  double acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0.0;
#pragma unroll 8
  for (int c = lane; c < n; c += 64) {   // unrolled as in k_coarse
    const double a = (double)A[lr * n + c];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] += a * (double)b[(r0 + c) * K + q];
  }
#pragma unroll
  for (int q = 0; q < K; ++q) {
    double v = acc[q];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) x[(r0 + lr) * K + q] = (T)v;
  }
}

// reference launches for camfe_measure_kernel: an empty kernel on the colour
// sweep's grid, and a plain copy of 16-byte elements
__global__ __launch_bounds__(SL * SW) void k_nop() {}
__global__ void k_copy16(const double2* __restrict__ src, double2* __restrict__ dst, long long n) {
  const long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

template <class T>
__global__ void k_fill(T* p, long long n, T v) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n) p[i] = v;
}
template <class A, class B>
__global__ void k_convert(const A* in, long long n, B* out) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n) out[i] = (B)in[i];
}

// ------------------------------------------------------- CG kernels
// sum of a block's per-thread values (BLK threads); result valid in thread 0
__device__ inline double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < BLK / 64; ++i) s += sh[i];
  return s;
}

// per-block partials of a . b per column
template <int K>
__global__ __launch_bounds__(BLK) void k_dot(long long n, const double* a, const double* b, double* part) {
  __shared__ double sh[BLK / 64];
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    const double s = block_sum(i < n ? a[i * K + c] * b[i * K + c] : 0.0, sh);
    if (threadIdx.x == 0) part[(long long)blockIdx.x * K + c] = s;
  }
}
// out[c] = sum of nb per-block partials (one block of 1024 threads)
template <int K>
__global__ __launch_bounds__(1024) void k_finalize(const double* part, int nb, double* out) {
  __shared__ double sh[16];
  for (int c = 0; c < K; ++c) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += 1024) v += part[(long long)b * K + c];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int w = 0; w < 16; ++w) s += sh[w];
      out[c] = s;
    }
    __syncthreads();
  }
}
// p = z + beta p per column
template <int K>
__global__ void k_cg_direction(long long n, const double* beta, const double* z, double* p) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int c = 0; c < K; ++c) p[i * K + c] = z[i * K + c] + beta[c] * p[i * K + c];
}

// The CG step's vector work around the V-cycle, fused with the V-cycle's
// start and end.  MODE 0 (FP64 cycle): the update also zeroes z, the cycle's
// initial guess.  MODE 1 (FP32 cycle): the update also writes b32 = r and
// zeroes x32, and the dot product converts the cycle's x32 into z.  With row
// weights (dinv64 / dinv32), the first n0c rows (colour 0) also take the first
// pre-sweep's relaxation from the zero guess, b_i * dinv_i.
// alpha = rz / pq; x += alpha p; r -= alpha q; per-block partials of r.r
template <int K, int MODE>
__global__ __launch_bounds__(BLK) void k_cg_update_v(long long n, const double* sc, double* x, double* r,
                                                     const double* p, const double* q, double* part, double* z,
                                                     float* b32, float* x32, const double* dinv64,
                                                     const float* dinv32, long long n0c) {
  __shared__ double sh[BLK / 64];
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    const double rz = sc[c], pq = sc[K + c];
    const double al = (pq != 0.0 && rz != 0.0) ? rz / pq : 0.0;
    double loc = 0.0;
    if (i < n) {
      x[i * K + c] += al * p[i * K + c];
      double v = r[i * K + c] - al * q[i * K + c];
      r[i * K + c] = v;
      loc = v * v;
      if (MODE == 0) {
        z[i * K + c] = (dinv64 && i < n0c) ? v * dinv64[i] : 0.0;
      } else {
        const float v32 = (float)v;
        b32[i * K + c] = v32;
        x32[i * K + c] = (dinv32 && i < n0c) ? v32 * dinv32[i] : 0.0f;
      }
    }
    const double s = block_sum(loc, sh);
    if (threadIdx.x == 0) part[(long long)blockIdx.x * K + c] = s;
  }
}
// per-block partials of r . z (MODE 1: z = x32 converted first)
template <int K, int MODE>
__global__ __launch_bounds__(BLK) void k_dot_rz(long long n, const double* r, double* z, const float* x32,
                                                double* part) {
  __shared__ double sh[BLK / 64];
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    double v = 0.0;
    if (i < n) {
      double zz;
      if (MODE == 0) {
        zz = z[i * K + c];
      } else {
        zz = (double)x32[i * K + c];
        z[i * K + c] = zz;
      }
      v = r[i * K + c] * zz;
    }
    const double s = block_sum(v, sh);
    if (threadIdx.x == 0) part[(long long)blockIdx.x * K + c] = s;
  }
}
// one block: rr = sum of part_rr, rz_new = sum of part_rz; beta = rz_new / rz;
// sc: rz[K] pq[K] rr[K] rz_new[K] bb[K] beta[K]; rz <- rz_new
template <int K>
__global__ __launch_bounds__(1024) void k_finalize_cg(const double* part_rz, const double* part_rr, int nb,
                                                      double* sc) {
  __shared__ double sh[16];
  for (int c = 0; c < 2 * K; ++c) {
    const double* part = c < K ? part_rr : part_rz;
    const int q = c % K;
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += 1024) v += part[(long long)b * K + q];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int w = 0; w < 16; ++w) s += sh[w];
      if (c < K) {
        sc[2 * K + q] = s;
      } else {
        const double old = sc[q];
        sc[3 * K + q] = s;
        sc[5 * K + q] = old != 0.0 ? s / old : 0.0;
        sc[q] = s;
      }
    }
    __syncthreads();
  }
}
template <int K>
__global__ void k_axpy_inplace(long long n, double* x, const double* y) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n * K) x[i] += y[i];
}

// --------------------------------------------- batched CG (per-mesh scalars)
// Scalars of mesh m live at sc[m * SCS + ...]: rz[K] pq[K] rr[K] rz_new[K]
// bb[K] act[K] (act = 1 while the column still iterates, 0 once frozen).
constexpr int SCS = 8 * KMAXS;

// a member still iterates while one of its columns does
template <int K>
__device__ inline bool live_member(const double* sc) {
  bool on = false;
#pragma unroll
  for (int c = 0; c < K; ++c) on = on || sc[5 * K + c] != 0.0;
  return on;
}

// per-block partials of a . b per column; blocks of members with act 0 give zero
template <int K>
__global__ __launch_bounds__(BLK) void k_dot_b(long long n, const int* bmesh, const int* act, const double* a,
                                               const double* b, double* part) {
  __shared__ double sh[BLK / 64];
  if (!act[bmesh[blockIdx.x]]) {
    if (threadIdx.x < K) part[(long long)blockIdx.x * K + threadIdx.x] = 0.0;
    return;
  }
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    const double v = i < n ? a[i * K + c] * b[i * K + c] : 0.0;
    const double s = block_sum(v, sh);
    if (threadIdx.x == 0) part[(long long)blockIdx.x * K + c] = s;
  }
}

// out[m * SCS + off + c] = sum of the partials of mesh m's blocks
template <int K>
__global__ __launch_bounds__(BLK) void k_finalize_seg(const double* part, const int* bstart, double* out, int off) {
  __shared__ double sh[BLK / 64];
  const int m = blockIdx.x;
  const int b0 = bstart[m], b1 = bstart[m + 1];
  for (int c = 0; c < K; ++c) {
    double v = 0.0;
    for (int b = b0 + threadIdx.x; b < b1; b += BLK) v += part[(long long)b * K + c];
    const double s = block_sum(v, sh);
    if (threadIdx.x == 0) out[(long long)m * SCS + off + c] = s;
    __syncthreads();
  }
}
template <int K>
__global__ __launch_bounds__(BLK) void k_cg_update_b(long long n, const int* bmesh, const double* scall, double* x,
                                                     double* r, const double* p, const double* q, double* part) {
  __shared__ double sh[BLK / 64];
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  const double* sc = scall + (long long)bmesh[blockIdx.x] * SCS;
  if (!live_member<K>(sc)) {   // every column frozen: x and r stay, the partials are zero
    if (threadIdx.x < K) part[(long long)blockIdx.x * K + threadIdx.x] = 0.0;
    return;
  }
#pragma unroll
  for (int c = 0; c < K; ++c) {
    const double rz = sc[c], pq = sc[K + c];
    const double al = (sc[5 * K + c] != 0.0 && pq != 0.0 && rz != 0.0) ? rz / pq : 0.0;
    double loc = 0.0;
    if (i < n) {
      x[i * K + c] += al * p[i * K + c];
      double v = r[i * K + c] - al * q[i * K + c];
      r[i * K + c] = v;
      loc = v * v;
    }
    const double s = block_sum(loc, sh);
    if (threadIdx.x == 0) part[(long long)blockIdx.x * K + c] = s;
  }
}
template <int K>
__global__ void k_cg_direction_b(long long n, const int* bmesh, const double* scall, const double* z, double* p) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  const double* sc = scall + (long long)bmesh[blockIdx.x] * SCS;
  if (!live_member<K>(sc)) return;   // p of a frozen member is never used again
#pragma unroll
  for (int c = 0; c < K; ++c) {
    const double be = (sc[5 * K + c] != 0.0 && sc[c] != 0.0) ? sc[3 * K + c] / sc[c] : 0.0;
    p[i * K + c] = z[i * K + c] + be * p[i * K + c];
  }
}
template <int K>
__global__ void k_copy_rz_b(int nm, double* scall) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nm * K) return;
  double* sc = scall + (long long)(i / K) * SCS;
  sc[i % K] = sc[3 * K + i % K];
}

// gated slice records: the slices of members that stopped iterating become
// empty (no entries, no rows), so the SELL kernels skip them unchanged
__global__ void k_gate_meta(long long ns, const int4* all, const int* slmem, const int* act, int4* out) {
  const long long s = blockIdx.x * (long long)BLK + threadIdx.x;
  if (s >= ns) return;
  const int4 m = all[s];
  out[s] = act[slmem[s]] ? m : make_int4(m.x, m.x, m.z, 0);
}

// canonical column-major n x k block (columns c0..c0+K) <-> internal row-major n x K
template <int K>
__global__ void k_gather_in(const double* src, long long n, int c0, int kk, const int* iperm, double* dst) {
  long long f = blockIdx.x * (long long)BLK + threadIdx.x;
  if (f >= n) return;
  int i = iperm[f];
#pragma unroll
  for (int q = 0; q < K; ++q) dst[(long long)i * K + q] = (c0 + q < kk) ? src[(long long)(c0 + q) * n + f] : 0.0;
}
template <int K>
__global__ void k_scatter_out(const double* src, long long n, int c0, int kk, const int* iperm, double* dst) {
  long long f = blockIdx.x * (long long)BLK + threadIdx.x;
  if (f >= n) return;
  int i = iperm[f];
#pragma unroll
  for (int q = 0; q < K; ++q)
    if (c0 + q < kk) dst[(long long)(c0 + q) * n + f] = src[(long long)i * K + q];
}

// ------------------------------------------------------------ host side
// per-slice metadata packed for one scalar load in the sweep kernels
void pack_meta(camfe_ctx ctx, GLevel& G, const std::vector<int>& ptr, const std::vector<int>& row0,
               const std::vector<int>& rows) {
  std::vector<int4> m(std::max<size_t>(G.nslices, 1), make_int4(0, 0, 0, 0));
  for (size_t i = 0; i < G.nslices; ++i) m[i] = make_int4(ptr[i], ptr[i + 1], row0[i], rows[i]);
  G.sl_meta.alloc(m.size());
  copy_in(ctx, G.sl_meta.p, m.data(), m.size());
}

// Colour-sweep tile of a depth that the autotuner has not seen, by its rows
// per colour (degree 1; measured on the depth-11 knot and sphere and their
// coarser depths): large colours take one pass of 8 entries per lane with 4
// wavefronts per slice (more slices in flight per CU), mid-sized ones 4 x 4
// or the 8 x 4 default, small ones 16 wavefronts of 2 entries (latency of a
// short launch).
int default_tile(int degree, size_t rows_per_colour) {
  if (degree != 1) return 0;
  if (rows_per_colour >= (size_t)1 << 19) return 5;
  if (rows_per_colour >= (size_t)1 << 17) return 1;
  if (rows_per_colour >= (size_t)1 << 15) return 0;
  return 3;
}

void setup_level(camfe_sys s, SolverState* st, int d) {
  camfe_hier h = s->h;
  camfe_ctx ctx = h->ctx;
  const HLevel& H = h->lev[d];
  const SLevel& S = s->lev[d];
  GLevel& G = st->lev[d];
  G.d = d;
  G.n = S.n;
  G.ncol = h->degree == 1 ? 8 : 27;
  const size_t n = G.n;
  G.tile = (size_t)d < s->tiles.size() ? std::max(0, s->tiles[d]) : default_tile(h->degree, n / G.ncol);
  unsigned g = grid_for(n, BLK);
  // colour order (stable: canonical order inside a colour)
  DArr<uint32_t> colour(n), idx(n);
  hipLaunchKernelGGL(k_colour, g, BLK, 0, ctx->stream, H.fkey.p, (long long)n, h->degree, colour.p, idx.p);
  check_launch();
  sort_pairs_u32(ctx, colour.p, idx.p, n, 5);
  G.perm.alloc(n);
  G.iperm.alloc(n);
  hipLaunchKernelGGL(k_iperm, g, BLK, 0, ctx->stream, idx.p, (long long)n, G.iperm.p, G.perm.p);
  check_launch();
  std::vector<uint32_t> hcol(n);
  copy_out(ctx, hcol.data(), colour.p, n);
  ctx->sync();
  G.coff.assign(G.ncol + 1, 0);
  for (size_t i = 0; i < n; ++i) G.coff[hcol[i] + 1]++;
  for (int c = 0; c < G.ncol; ++c) G.coff[c + 1] += G.coff[c];
  // Large colours: rows sorted by decreasing length inside windows of
  // SORT_WINDOW rows, so that a slice's rows have similar lengths and the
  // SELL padding shrinks (about 1.45x -> 1.03x of the nonzeros).  Rows of
  // one colour are independent, so the order changes no row's arithmetic;
  // small colours keep the canonical order, whose neighbouring rows share
  // more of the cache lines their x gathers touch (latency dominates there).
  {
    std::vector<int> wbase(G.ncol + 1, 0);
    int mask = 0;
    const long long sort_min = s->sell_sort_min_rows > 0 ? s->sell_sort_min_rows : SORT_MIN_ROWS;
    for (int c = 0; c < G.ncol; ++c) {
      const int nc = G.coff[c + 1] - G.coff[c];
      wbase[c + 1] = wbase[c] + (nc + SORT_WINDOW - 1) / SORT_WINDOW;
      if (nc >= sort_min) mask |= 1 << c;
    }
    if (mask) {
      DArr<int> dco(G.ncol + 1), dwb(G.ncol + 1);
      copy_in(ctx, dco.p, G.coff.data(), G.ncol + 1);
      copy_in(ctx, dwb.p, wbase.data(), G.ncol + 1);
      DArr<uint32_t> key(n), val(n);
      hipLaunchKernelGGL(k_window_keys, g, BLK, 0, ctx->stream, (const int*)G.perm.p, S.ptr.p, (long long)n, dco.p,
                         dwb.p, G.ncol, mask, key.p, val.p);
      check_launch();
      int bits = 8;
      while ((1LL << (bits - 8)) <= wbase[G.ncol]) ++bits;
      sort_pairs_u32(ctx, key.p, val.p, n, bits);
      hipLaunchKernelGGL(k_iperm, g, BLK, 0, ctx->stream, (const uint32_t*)val.p, (long long)n, G.iperm.p, G.perm.p);
      check_launch();
    }
  }
  // slices: per colour, runs of 64 rows
  G.cslice.assign(G.ncol + 1, 0);
  std::vector<int> row0, rows;
  for (int c = 0; c < G.ncol; ++c) {
    G.cslice[c] = (int)row0.size();
    for (int r = G.coff[c]; r < G.coff[c + 1]; r += SL) {
      row0.push_back(r);
      rows.push_back(std::min(SL, G.coff[c + 1] - r));
    }
  }
  G.cslice[G.ncol] = (int)row0.size();
  {
    std::vector<int> hptr(n + 1), hperm(n);
    copy_out(ctx, hptr.data(), S.ptr.p, n + 1);
    copy_out(ctx, hperm.data(), G.perm.p, n);
    G.cnnz.assign(G.ncol, 0);
    for (int c = 0; c < G.ncol; ++c)
      for (int r = G.coff[c]; r < G.coff[c + 1]; ++r) G.cnnz[c] += hptr[hperm[r] + 1] - hptr[hperm[r]];
    G.nnz = hptr[n];
  }
  G.nslices = row0.size();
  G.sl_row0.alloc(G.nslices);
  G.sl_rows.alloc(G.nslices);
  copy_in(ctx, G.sl_row0.p, row0.data(), G.nslices);
  copy_in(ctx, G.sl_rows.p, rows.data(), G.nslices);
  DArr<int> width(G.nslices);
  G.sl_ptr.alloc(G.nslices + 1);
  hipLaunchKernelGGL(k_slice_width, grid_for(G.nslices, BLK), BLK, 0, ctx->stream, S.ptr.p, G.perm.p,
                     G.sl_row0.p, G.sl_rows.p, (long long)G.nslices, width.p);
  check_launch();
  std::vector<int> hw(G.nslices), hp(G.nslices + 1, 0);
  copy_out(ctx, hw.data(), width.p, G.nslices);
  ctx->sync();
  for (size_t i = 0; i < G.nslices; ++i) hp[i + 1] = hp[i] + hw[i];
  G.snnz = (size_t)hp[G.nslices];
  copy_in(ctx, G.sl_ptr.p, hp.data(), G.nslices + 1);
  pack_meta(ctx, G, hp, row0, rows);
  G.scol.alloc(G.snnz);
  G.sval64.alloc(G.snnz);
  G.sval32.alloc(G.snnz);
  G.invd64.alloc(n);
  G.invd32.alloc(n);
  const long long threads = (long long)G.nslices * SL;
  hipLaunchKernelGGL(k_sell_pad, grid_for(threads, BLK), BLK, 0, ctx->stream, G.sl_ptr.p, G.sl_row0.p, G.sl_rows.p,
                     (long long)G.nslices, G.scol.p, G.sval64.p, G.sval32.p);
  hipLaunchKernelGGL(k_sell_fill, grid_for(threads, BLK), BLK, 0, ctx->stream, S.ptr.p, S.col.p, S.M.p, S.L.p,
                     st->t, G.perm.p, G.iperm.p, G.sl_ptr.p, G.sl_row0.p, G.sl_rows.p, (long long)G.nslices,
                     G.scol.p, G.sval64.p, G.sval32.p, G.invd64.p, G.invd32.p);
  check_launch();
  G.ns16 = 0;
  if (G.ncol == 8 && s->sell_compact && G.nslices) {
    ColourStarts co;
    for (int c = 0; c <= 8; ++c) co.c[c] = G.coff[c];
    G.scol16.alloc(G.snnz);
    G.sbase.alloc(G.nslices * 8);
    DArr<unsigned long long> cnt(1);
    zero(ctx, cnt.p, 1);
    hipLaunchKernelGGL(k_sell_compact, (unsigned)G.nslices, 64, 0, ctx->stream, (long long)G.nslices, co,
                       (const int*)G.scol.p, G.sl_meta.p, G.sbase.p, G.scol16.p, cnt.p);
    check_launch();
    G.ns16 = (long long)read_scalar(ctx, cnt.p);
  }
  G.x64.alloc(n * KMAXS); G.b64.alloc(n * KMAXS); G.r64.alloc(n * KMAXS); G.t64.alloc(n * KMAXS);
  G.x32.alloc(n * KMAXS); G.b32.alloc(n * KMAXS); G.r32.alloc(n * KMAXS); G.t32.alloc(n * KMAXS);
}

// transfers between depth d (fine) and d-1 in internal numbering
void setup_transfer(camfe_sys s, SolverState* st, int d) {
  camfe_hier h = s->h;
  camfe_ctx ctx = h->ctx;
  const HLevel& H = h->lev[d];
  GLevel& Fg = st->lev[d];
  GLevel& Cg = st->lev[d - 1];
  const size_t nf = Fg.n, nc = Cg.n, nnz = H.pnnz;
  Fg.pnnz = (long long)nnz;
  unsigned g = grid_for(nf, BLK);
  DArr<int> cnt(nf);
  Fg.Pptr.alloc(nf + 1);
  hipLaunchKernelGGL(k_p_count, g, BLK, 0, ctx->stream, H.P_ptr.p, Fg.perm.p, (long long)nf, cnt.p);
  exclusive_scan(ctx, cnt.p, Fg.Pptr.p, nf);
  int tot = (int)nnz;
  copy_in(ctx, Fg.Pptr.p + nf, &tot, 1);
  Fg.Pcol.alloc(nnz);
  Fg.Pw64.alloc(nnz);
  Fg.Pw32.alloc(nnz);
  DArr<uint32_t> rkey(nnz), rval(nnz);
  hipLaunchKernelGGL(k_p_fill, g, BLK, 0, ctx->stream, H.P_ptr.p, H.P_col.p, H.P_w.p, Fg.perm.p, Cg.iperm.p,
                     (long long)nf, Fg.Pptr.p, Fg.Pcol.p, Fg.Pw64.p, Fg.Pw32.p, rkey.p, rval.p);
  check_launch();
  DArr<int> row_of(nnz);
  hipLaunchKernelGGL(k_row_of_entry, g, BLK, 0, ctx->stream, Fg.Pptr.p, (long long)nf, row_of.p);
  int bits = 1;
  while ((1ULL << bits) <= nc) ++bits;
  sort_pairs_u32(ctx, rkey.p, rval.p, nnz, bits);
  Fg.Rptr.alloc(nc + 1);
  Fg.Rcol.alloc(nnz);
  Fg.Rw64.alloc(nnz);
  Fg.Rw32.alloc(nnz);
  hipLaunchKernelGGL(k_ptr_from_sorted, grid_for(nnz, BLK), BLK, 0, ctx->stream, rkey.p, (long long)nnz,
                     (long long)nc, Fg.Rptr.p);
  hipLaunchKernelGGL(k_r_fill, grid_for(nnz, BLK), BLK, 0, ctx->stream, rkey.p, rval.p, (long long)nnz, row_of.p,
                     Fg.Pw64.p, Fg.Rcol.p, Fg.Rw64.p, Fg.Rw32.p);
  check_launch();
}

void setup_coarsest(camfe_sys s, SolverState* st) {
  camfe_hier h = s->h;
  camfe_ctx ctx = h->ctx;
  const int d = h->d0;
  const SLevel& S = s->lev[d];
  GLevel& G = st->lev[d];
  st->direct = h->max_coarse > 0 && (long long)G.n <= h->max_coarse;
  if (!st->direct) return;
  const int n = (int)G.n;
  st->n0 = n;
  DArr<double> A((size_t)n * n), dg(n), sv(n);
  zero(ctx, A.p, A.n);
  hipLaunchKernelGGL(k_dense_scaled, grid_for(n, BLK), BLK, 0, ctx->stream, S.ptr.p, S.col.p, S.M.p, S.L.p, st->t,
                     G.perm.p, G.iperm.p, (long long)n, st->coarse_eps, A.p);
  hipLaunchKernelGGL(k_diag_of, grid_for(n, BLK), BLK, 0, ctx->stream, S.ptr.p, S.col.p, S.M.p, S.L.p, st->t,
                     G.perm.p, (long long)n, dg.p);
  hipLaunchKernelGGL(k_inv_sqrt_diag, grid_for(n, BLK), BLK, 0, ctx->stream, n, sv.p, (const double*)dg.p);
  check_launch();
  if (st->Ainv64.n != (size_t)n * n)   // kept in place on refresh: captured graphs hold its address
    st->Ainv64.alloc((size_t)n * n);
  // Ainv = D^-1/2 (D^-1/2 A D^-1/2 + eps I)^-1 D^-1/2
  spd_inverse_scaled(ctx, A.p, n, sv.p, st->Ainv64.p);
}

SolverState* setup(camfe_sys s, double t, int precision, double coarse_eps) {
  camfe_hier h = s->h;
  camfe_ctx ctx = h->ctx;
  auto t0 = std::chrono::steady_clock::now();
  std::unique_ptr<SolverState> st(new SolverState());
  st->ctx = ctx;
  st->t = t;
  st->precision = precision;
  st->coarse_eps = coarse_eps;
  st->D = h->D;
  st->d0 = h->d0;
  st->lev.resize(h->D + 1);
  for (int d = h->d0; d <= h->D; ++d) setup_level(s, st.get(), d);
  for (int d = h->d0 + 1; d <= h->D; ++d) setup_transfer(s, st.get(), d);
  setup_coarsest(s, st.get());
  const size_t n = st->lev[h->D].n * KMAXS;
  st->X.alloc(n); st->R.alloc(n); st->Z.alloc(n); st->P.alloc(n); st->Q.alloc(n); st->B.alloc(n);
  st->sc.alloc(8 * KMAXS);
  {
    const GLevel& F = st->lev[h->D];
    const size_t nb = std::max(F.nslices, (F.n + BLK - 1) / BLK) + 1;
    st->part.alloc(nb * KMAXS);
    st->part2.alloc(nb * KMAXS);
  }
  ctx->sync();
  st->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return st.release();
}

template <class T>
struct Vec {
  static T* x(GLevel& g);
  static T* b(GLevel& g);
  static T* r(GLevel& g);
};
template <>
double* Vec<double>::x(GLevel& g) { return g.x64.p; }
template <>
double* Vec<double>::b(GLevel& g) { return g.b64.p; }
template <>
double* Vec<double>::r(GLevel& g) { return g.r64.p; }
template <>
float* Vec<float>::x(GLevel& g) { return g.x32.p; }
template <>
float* Vec<float>::b(GLevel& g) { return g.b32.p; }
template <>
float* Vec<float>::r(GLevel& g) { return g.r32.p; }

template <class T>
const T* sval_of(const GLevel& g);
template <>
const double* sval_of<double>(const GLevel& g) { return g.sval64.p; }
template <>
const float* sval_of<float>(const GLevel& g) { return g.sval32.p; }
template <class T>
const T* invd_of(const GLevel& g);
template <>
const double* invd_of<double>(const GLevel& g) { return g.invd64.p; }
template <>
const float* invd_of<float>(const GLevel& g) { return g.invd32.p; }
template <class T>
const T* pw_of(const GLevel& g);
template <>
const double* pw_of<double>(const GLevel& g) { return g.Pw64.p; }
template <>
const float* pw_of<float>(const GLevel& g) { return g.Pw32.p; }
template <class T>
const T* rw_of(const GLevel& g);
template <>
const double* rw_of<double>(const GLevel& g) { return g.Rw64.p; }
template <>
const float* rw_of<float>(const GLevel& g) { return g.Rw32.p; }


// algorithmic bytes of one matrix pass over rows with z nonzeros: matrix
// values plus read b, read x, write x (or r)
template <class T, int K>
double pass_bytes(long long z, long long rows) {
  return (double)z * sizeof(T) + 3.0 * (double)rows * K * sizeof(T);
}

// one multicolour sweep x_i += w_i (b_i - (A x)_i) with w = dinv (1 / A_ii for
// Gauss-Seidel, omega_i / A_ii for SOR)
template <class T, int K, int TILE>
void gs_colour(camfe_ctx ctx, GLevel& G, int c, const T* b, T* x, const T* dinv) {
  const int s0 = G.cslice[c], s1 = G.cslice[c + 1];
  CAMFE_TIMED(ctx, KT_GS, (pass_bytes<T, K>(G.cnnz[c], G.coff[c + 1] - G.coff[c])), (k_gs<T, K, TILE>),
              (unsigned)(s1 - s0), SL * tile_sw(TILE), 0, ctx->stream, G.sl_meta.p, s0, s1, G.scol.p, G.scol16.p, G.sbase.p,
              sval_of<T>(G), dinv, b, x);
}

// tile: the level's choice (G.tile) unless given
template <class T, int K>
void gs_sweep(camfe_ctx ctx, GLevel& G, const T* b, T* x, bool forward, const T* dinv, int first = 0,
              int tile = -1) {
  if (tile < 0) tile = G.tile;
  for (int ci = first; ci < G.ncol; ++ci) {
    const int c = forward ? ci : G.ncol - 1 - ci;
    if (G.cslice[c + 1] <= G.cslice[c]) continue;
    switch (tile) {
      case 1: gs_colour<T, K, 1>(ctx, G, c, b, x, dinv); break;
      case 2: gs_colour<T, K, 2>(ctx, G, c, b, x, dinv); break;
      case 3: gs_colour<T, K, 3>(ctx, G, c, b, x, dinv); break;
      case 4: gs_colour<T, K, 4>(ctx, G, c, b, x, dinv); break;
      case 5: gs_colour<T, K, 5>(ctx, G, c, b, x, dinv); break;
      case 6: gs_colour<T, K, 6>(ctx, G, c, b, x, dinv); break;
      default: gs_colour<T, K, 0>(ctx, G, c, b, x, dinv); break;
    }
  }
}

template <class T>
T* tmp_of(GLevel& g);
template <>
double* tmp_of<double>(GLevel& g) { return g.t64.p; }
template <>
float* tmp_of<float>(GLevel& g) { return g.t32.p; }
template <class T>
const T* winvd_of(const GLevel& g);
template <>
const double* winvd_of<double>(const GLevel& g) { return g.winvd64.p; }
template <>
const float* winvd_of<float>(const GLevel& g) { return g.winvd32.p; }

// nu smoothing sweeps on (b, x): multicolour Gauss-Seidel or SOR with
// per-row weights (colours forward or reversed), or weighted Jacobi
// (order-free; ping-pong through the level's scratch vector, one launch per sweep)
// Row weights of a colour-ordered sweep (Gauss-Seidel: 1 / A_ii; SOR: omega_i /
// A_ii), or null for the Jacobi smoothers
template <class T>
const T* sweep_dinv(const SolverState* S, const GLevel& G) {
  if (S->smoother == 0) return invd_of<T>(G);
  if (S->smoother == 2 && S->wsweep == 1) return winvd_of<T>(G);
  return nullptr;
}

// nu cell-block Schwarz sweeps: r = b - A x into the level's scratch vector,
// then the weighted block products of both block classes added into x (the
// same map before and after the coarse correction).  x_zero: x is zero on
// entry, so the first sweep's residual is b itself and is not computed.
// a block class (8 or 16 wide) of at least this many blocks at a depth is
// relaxed colour by colour without atomics (8 launches); a smaller one in one
// launch with atomic adds
constexpr long long BLOCK_COLOUR_MIN = 1LL << 19;

template <class T, int K>
void block_smooth(SolverState* S, GLevel& G, const T* b, T* x, int nu, bool x_zero) {
  camfe_ctx ctx = S->ctx;
  hipStream_t st = ctx->stream;
  constexpr bool dbl = std::is_same<T, double>::value;
  const T* inv8 = dbl ? (const T*)G.binv8_64.p : (const T*)G.binv8_32.p;
  const T* inv16 = dbl ? (const T*)G.binv16_64.p : (const T*)G.binv16_32.p;
  const T* w8 = dbl ? (const T*)G.bw8_64.p : (const T*)G.bw8_32.p;
  const T* w16 = dbl ? (const T*)G.bw16_64.p : (const T*)G.bw16_32.p;
  const T* sc = dbl ? (const T*)G.bs64.p : (const T*)G.bs32.p;
  const T om = (T)(S->block_omega > 0 ? S->block_omega : G.block_omega);
  T* rbuf = tmp_of<T>(G);
  for (int it = 0; it < nu; ++it) {
    const T* r = b;
    if (it > 0 || !x_zero) {
      CAMFE_TIMED(ctx, KT_RESIDUAL, (pass_bytes<T, K>(G.nnz, (long long)G.n)), (k_residual<T, T, K>),
                  (unsigned)G.nslices, SL * SW, 0, st, G.sl_meta.p, (int)G.nslices, G.scol.p, G.scol16.p, G.sbase.p,
                  sval_of<T>(G), b, (const T*)x, rbuf, (double*)nullptr);
      r = rbuf;
    }
    // each block class separately: colour by colour with plain adds (no two
    // blocks of a colour share a function) when it is large, else one
    // launch with atomic adds; the launches of a sweep run in order
    const long long cmin = S->block_colour_min > 0 ? S->block_colour_min : BLOCK_COLOUR_MIN;
    const double b8 = 36 * sizeof(T) / 8.0 + 4 + 3.0 * K * sizeof(T);     // bytes per block row
    const double b16 = 136 * sizeof(T) / 16.0 + 4 + 3.0 * K * sizeof(T);
    if (G.nb8 >= cmin) {
      for (int k = 0; k < 8; ++k) {
        const long long a = G.bc8[k], e = G.bc8[k + 1];
        if (e > a)
          CAMFE_TIMED(ctx, KT_GS, ((double)(e - a) * 8 * b8), (k_block_apply<T, K, 8, false>),
                      grid_for((size_t)(e - a) * 8, 256), 256, 0, st, a, e, G.bidx8.p, inv8, w8, sc, (const T*)r, om,
                      x);
      }
    } else if (G.nb8) {
      CAMFE_TIMED(ctx, KT_GS, ((double)G.nb8 * 8 * b8), (k_block_apply<T, K, 8, true>),
                  grid_for((size_t)G.nb8 * 8, 256), 256, 0, st, 0LL, G.nb8, G.bidx8.p, inv8, w8, sc, (const T*)r,
                  om, x);
    }
    if (G.nb16 >= cmin) {
      for (int k = 0; k < 8; ++k) {
        const long long a = G.bc16[k], e = G.bc16[k + 1];
        if (e > a)
          CAMFE_TIMED(ctx, KT_GS, ((double)(e - a) * 16 * b16), (k_block_apply<T, K, 16, false>),
                      grid_for((size_t)(e - a) * 16, 256), 256, 0, st, a, e, G.bidx16.p, inv16, w16, sc,
                      (const T*)r, om, x);
      }
    } else if (G.nb16) {
      CAMFE_TIMED(ctx, KT_GS, ((double)G.nb16 * 16 * b16), (k_block_apply<T, K, 16, true>),
                  grid_for((size_t)G.nb16 * 16, 256), 256, 0, st, 0LL, G.nb16, G.bidx16.p, inv16, w16, sc,
                  (const T*)r, om, x);
    }
  }
}

// uniform values in [-1, 1) from a counter (splitmix64 of seed + i)
__global__ void k_hash_fill(long long n, unsigned long long seed, double* v) {
  const long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  unsigned long long z = seed + 0x9E3779B97F4A7C15ULL * (unsigned long long)(i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z ^= z >> 31;
  v[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}
__global__ void k_scale_into(long long n, double a, const double* y, double* v) {
  const long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n) v[i] = a * y[i];
}

// Automatic damping of the cell-block smoother, per depth.  The block
// operator B = sum_B w_B R_B^T A_B^-1 R_B is symmetric and B A is
// A-self-adjoint; one sweep maps the error e to (I - omega B A) e, a
// contraction only while omega lambda_max(B A) < 2.  The weights bound what
// blocks sharing functions add, but blocks that share none still couple
// through A (functions of neighbouring cells are nearly parallel where the
// surface crosses cells in thin pieces), and lambda_max grows past 2 at fine
// depths.  So lambda_max is estimated by BLOCK_POWER steps of the power
// method in the A inner product from a fixed pseudo-random start (the
// Rayleigh quotient (A v . B A v) / (v . A v) approaches it from below), and
// the damping set to 4 / (3 lambda), the Richardson choice that damps the
// upper half of the spectrum by at least 1/3, capped at 1.
constexpr int BLOCK_POWER = 20;

void estimate_block_damping(SolverState* S) {
  camfe_ctx ctx = S->ctx;
  hipStream_t st = ctx->stream;
  DArr<double> dd(3);
  for (int d = S->d0; d <= S->D; ++d) {
    GLevel& G = S->lev[d];
    G.block_lambda = G.block_omega = 0;
    if (!G.nb8 && !G.nb16) continue;
    const long long n = (long long)G.n, nb = (n + BLK - 1) / BLK;
    double* v = G.x64.p;
    double* zero_b = G.b64.p;
    double* r = G.r64.p;
    double* y = G.t64.p;
    hipLaunchKernelGGL((k_fill<double>), grid_for(n, BLK), BLK, 0, st, zero_b, n, 0.0);
    hipLaunchKernelGGL(k_hash_fill, grid_for(n, BLK), BLK, 0, st, n, 0x5EEDB10CULL + (unsigned long long)d, v);
    double lam = 0;
    for (int it = 0; it < BLOCK_POWER; ++it) {
      // r = -A v, y = B r = -B A v
      hipLaunchKernelGGL((k_residual<double, double, 1>), (unsigned)G.nslices, SL * SW, 0, st, G.sl_meta.p,
                         (int)G.nslices, G.scol.p, G.scol16.p, G.sbase.p, G.sval64.p, (const double*)zero_b, (const double*)v, r,
                         (double*)nullptr);
      hipLaunchKernelGGL((k_fill<double>), grid_for(n, BLK), BLK, 0, st, y, n, 0.0);
      if (G.nb8)
        hipLaunchKernelGGL((k_block_apply<double, 1, 8, true>), grid_for((size_t)G.nb8 * 8, 256), 256, 0, st, 0LL,
                           G.nb8, G.bidx8.p, (const double*)G.binv8_64.p, (const double*)G.bw8_64.p,
                           (const double*)G.bs64.p, (const double*)r, 1.0, y);
      if (G.nb16)
        hipLaunchKernelGGL((k_block_apply<double, 1, 16, true>), grid_for((size_t)G.nb16 * 16, 256), 256, 0, st,
                           0LL, G.nb16, G.bidx16.p, (const double*)G.binv16_64.p, (const double*)G.bw16_64.p,
                           (const double*)G.bs64.p, (const double*)r, 1.0, y);
      const double* pa[3] = {y, v, y};
      const double* pb[3] = {r, r, y};
      for (int q = 0; q < 3; ++q) {
        hipLaunchKernelGGL(k_dot<1>, (unsigned)nb, BLK, 0, st, n, pa[q], pb[q], S->part.p);
        hipLaunchKernelGGL(k_finalize<1>, 1, 1024, 0, st, (const double*)S->part.p, (int)nb, dd.p + q);
      }
      double h[3];
      copy_out(ctx, h, dd.p, 3);
      if (!(h[2] > 0.0) || !(h[1] < 0.0)) break;   // B A v = 0: nothing to damp
      lam = std::max(lam, -h[0] / h[1]);
      hipLaunchKernelGGL(k_scale_into, grid_for(n, BLK), BLK, 0, st, n, 1.0 / std::sqrt(h[2]), (const double*)y,
                         v);
    }
    check_launch();
    G.block_lambda = lam;
    G.block_omega = lam > 0 ? std::min(1.0, 4.0 / (3.0 * lam)) : 1.0;
  }
}

template <class T, int K>
// first0: x was zero and the first sweep's colour-0 rows are already relaxed
// (by the kernel that zeroed x), so that sweep starts at colour 1; x_zero: x
// is zero on entry (used by the cell-block sweep)
void smooth(SolverState* S, GLevel& G, const T* b, T* x, int nu, bool forward, bool first0 = false,
            bool x_zero = false) {
  camfe_ctx ctx = S->ctx;
  if (S->smoother == 3) {
    block_smooth<T, K>(S, G, b, x, nu, x_zero);
    return;
  }
  if (const T* dinv = sweep_dinv<T>(S, G)) {
    for (int i = 0; i < nu; ++i) gs_sweep<T, K>(ctx, G, b, x, forward, dinv, i == 0 && first0 && forward ? 1 : 0);
    return;
  }
  T* a = x;
  T* t = tmp_of<T>(G);
  for (int i = 0; i < nu; ++i) {
    CAMFE_TIMED(ctx, KT_GS, (pass_bytes<T, K>(G.nnz, (long long)G.n) + (double)G.n * sizeof(T)), (k_jacobi<T, K>),
                (unsigned)G.nslices, SL * SW, 0, ctx->stream, G.sl_meta.p, (int)G.nslices,
                G.scol.p, G.scol16.p, G.sbase.p, sval_of<T>(G), winvd_of<T>(G), b, (const T*)a, t);
    std::swap(a, t);
  }
  if (a != x)
    hipLaunchKernelGGL((k_convert<T, T>), grid_for(G.n * K, BLK), BLK, 0, ctx->stream, (const T*)a,
                       (long long)(G.n * K), x);
}

// batched solver: direct solves of the meshes whose coarsest depth is this level
template <class T, int K>
void coarse_batched(SolverState* S, GLevel& G, const T* b, T* x) {
  if (!G.ncb) return;
  hipLaunchKernelGGL((k_coarse_b<T, K>), grid_for((size_t)G.cb_rows * 64, BLK), BLK, 0, S->ctx->stream, G.ncb,
                     G.cb_rowoff.p, G.cb_cum.p, G.cb_aoff.p, (const double*)G.cb_a64.p, b, x,
                     (const int*)G.cbmem.p, (const int*)S->mact.p);
}

// One cycle at depth d on (b, x) of that depth, x given (zero on entry below
// the top): the coarse problem gets S->gamma cycles, the first from zero (one:
// V-cycle, two: W-cycle, Section 5.2).
// first0: as for smooth() (x zero, colour 0 of the first pre-sweep done)
template <class T, int K>
void vcycle(SolverState* S, int d, const T* b, T* x, int nu1, int nu2, bool first0 = false, bool x_zero = false) {
  camfe_ctx ctx = S->ctx;
  hipStream_t st = ctx->stream;
  GLevel& G = S->lev[d];
  if (d == S->d0 && S->batch) {
    smooth<T, K>(S, G, b, x, nu1, true, false, x_zero);
    coarse_batched<T, K>(S, G, b, x);
    smooth<T, K>(S, G, b, x, nu2, false);
    return;
  }
  if (d == S->d0) {
    if (S->direct) {
      const double w = (double)S->n0 * S->n0 * sizeof(double) + 2.0 * S->n0 * K * sizeof(T);
      CAMFE_TIMED(ctx, KT_COARSE, w, (k_coarse<T, K>), grid_for((size_t)S->n0 * 64, BLK), BLK, 0, st,
                  (const double*)S->Ainv64.p, S->n0, b, x);
    } else {
      smooth<T, K>(S, G, b, x, nu1, true, false, x_zero);
      smooth<T, K>(S, G, b, x, nu2, false);
    }
    return;
  }
  smooth<T, K>(S, G, b, x, nu1, true, first0, x_zero);
  T* r = Vec<T>::r(G);
  CAMFE_TIMED(ctx, KT_RESIDUAL, (pass_bytes<T, K>(G.nnz, (long long)G.n)), (k_residual<T, T, K>),
              (unsigned)G.nslices, SL * SW, 0, st, G.sl_meta.p,
              (int)G.nslices, G.scol.p, G.scol16.p, G.sbase.p, sval_of<T>(G), b, (const T*)x, r, (double*)nullptr);
  GLevel& C = S->lev[d - 1];
  T* bc = Vec<T>::b(C);
  T* xc = Vec<T>::x(C);
  // transfers: parent map (4 B per entry) plus the vectors read and written;
  // above the coarsest depth of a single system (colour-major rows) the
  // restriction also takes the coarse depth's first colour-0 relaxation
  const T* cdinv = (!S->batch && nu1 > 0 && d - 1 > S->d0) ? sweep_dinv<T>(S, C) : nullptr;
  CAMFE_TIMED(ctx, KT_RESTRICT, (4.0 * G.pnnz + ((double)G.n + C.n) * K * sizeof(T)), (k_restrict<T, K>),
              grid_for(C.n * RL, BLK), BLK, 0, st, G.Rptr.p, G.Rcol.p, rw_of<T>(G), (long long)C.n, (const T*)r, bc,
              xc, cdinv, cdinv ? (long long)C.coff[1] : 0LL, (const int*)C.blkmem.p, (const int*)S->mact.p);
  const int c1 = S->nu_coarse > 0 ? S->nu_coarse : nu1, c2 = S->nu_coarse > 0 ? S->nu_coarse : nu2;
  // the restriction zeroes x_c (or relaxes its colour 0 when cdinv is set)
  for (int g = 0; g < S->gamma; ++g)
    vcycle<T, K>(S, d - 1, bc, xc, c1, c2, g == 0 && cdinv != nullptr, g == 0 && cdinv == nullptr);
  CAMFE_TIMED(ctx, KT_PROLONG, (4.0 * G.pnnz + ((double)C.n + 2.0 * G.n) * K * sizeof(T)), (k_prolong<T, K>),
              grid_for(G.n, BLK), BLK, 0, st, G.Pptr.p, G.Pcol.p, pw_of<T>(G), (long long)G.n, (const T*)xc, x,
              (const int*)G.blkmem.p, (const int*)S->mact.p);
  if (G.ncb) coarse_batched<T, K>(S, G, b, x);   // meshes that bottom out here
  smooth<T, K>(S, G, b, x, nu2, false);
}

// z = V(r) at the finest depth (z zeroed first); FP32 cycles convert in and out
template <int K>
void precondition(SolverState* S, const double* r, double* z, int nu1, int nu2) {
  hipStream_t st = S->ctx->stream;
  GLevel& G = S->lev[S->D];
  const long long nk = (long long)G.n * K;
  if (S->precision == 0) {
    hipLaunchKernelGGL((k_fill<double>), grid_for(nk, BLK), BLK, 0, st, z, nk, 0.0);
    vcycle<double, K>(S, S->D, r, z, nu1, nu2, false, true);
  } else {
    hipLaunchKernelGGL((k_convert<double, float>), grid_for(nk, BLK), BLK, 0, st, r, nk, G.b32.p);
    hipLaunchKernelGGL((k_fill<float>), grid_for(nk, BLK), BLK, 0, st, G.x32.p, nk, 0.0f);
    vcycle<float, K>(S, S->D, G.b32.p, G.x32.p, nu1, nu2, false, true);
    hipLaunchKernelGGL((k_convert<float, double>), grid_for(nk, BLK), BLK, 0, st, G.x32.p, nk, z);
  }
}

// out[q] = sum of nb per-block partials
template <int K>
void finalize(SolverState* S, long long nb, double* out) {
  hipLaunchKernelGGL(k_finalize<K>, 1, 1024, 0, S->ctx->stream, (const double*)S->part.p, (int)nb, out);
}

// out[q] = a_q . b_q over the finest depth
template <int K>
void dot(SolverState* S, const double* a, const double* b, double* out) {
  const long long n = (long long)S->lev[S->D].n;
  const long long nb = (n + BLK - 1) / BLK;
  hipLaunchKernelGGL(k_dot<K>, (unsigned)nb, BLK, 0, S->ctx->stream, n, a, b, S->part.p);
  finalize<K>(S, nb, out);
}

// r = b - A x at the finest depth in FP64; nrm (nullable) receives ||r_q||^2
template <int K>
void residual64(SolverState* S, const double* b, const double* x, double* r, double* nrm) {
  GLevel& G = S->lev[S->D];
  camfe_ctx ctx = S->ctx;
  CAMFE_TIMED(ctx, KT_RESIDUAL, (pass_bytes<double, K>(G.nnz, (long long)G.n)), (k_residual<double, double, K>),
              (unsigned)G.nslices, SL * SW, 0, ctx->stream, G.sl_meta.p,
              (int)G.nslices, G.scol.p, G.scol16.p, G.sbase.p, G.sval64.p, b, x, r, nrm ? S->part.p : (double*)nullptr);
  if (nrm) finalize<K>(S, (long long)G.nslices, nrm);
}

void dcopy(camfe_ctx ctx, void* dst, const void* src, size_t bytes) {
  if (bytes) CAMFE_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, ctx->stream));
}

struct SolveResult {
  int it = 0, cycles = 0;
  double rel = 0;
  bool judged_gs = false;   // the judge continued with plain Gauss-Seidel
  double judge_rel[2] = {0.0, 0.0};   // residuals after the judge's iterations (smoother, GS)
};

// Record `enqueue` into a graph once (keyed), replay it on the context stream.
// Capture runs on a private stream (the context stream may be the legacy
// default stream, which cannot be captured) with the timer off.
void run_graph(SolverState* S, long long key, const std::function<void()>& enqueue) {
  camfe_ctx ctx = S->ctx;
  auto it = S->graphs.find(key);
  if (it == S->graphs.end()) {
    if (!S->cap) CAMFE_HIP(hipStreamCreateWithFlags(&S->cap, hipStreamNonBlocking));
    hipStream_t saved = ctx->stream;
    const bool saved_on = ctx->timer.on;
    ctx->stream = S->cap;
    ctx->timer.on = false;
    hipGraph_t graph = nullptr;
    CAMFE_HIP(hipStreamBeginCapture(S->cap, hipStreamCaptureModeThreadLocal));
    try {
      enqueue();
    } catch (...) {
      (void)hipStreamEndCapture(S->cap, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      ctx->stream = saved;
      ctx->timer.on = saved_on;
      throw;
    }
    CAMFE_HIP(hipStreamEndCapture(S->cap, &graph));
    ctx->stream = saved;
    ctx->timer.on = saved_on;
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    CAMFE_HIP(e);
    it = S->graphs.emplace(key, ex).first;
  }
  CAMFE_HIP(hipGraphLaunch(it->second, ctx->stream));
}

// One CG step: q = A p, x += alpha p, r -= alpha q (||r||^2 into rr), z = V(r),
// p = z + beta p.  All scalars stay on the device.
template <int K>
void cg_step(SolverState* S, int nu1, int nu2) {
  camfe_ctx ctx = S->ctx;
  GLevel& G = S->lev[S->D];
  const size_t n = G.n;
  const long long nb = (long long)((n + BLK - 1) / BLK);
  double* sc = S->sc.p;
  CAMFE_TIMED(ctx, KT_SPMV, ((double)G.nnz * 8 + 2.0 * n * K * 8), k_spmv_dot<K>, (unsigned)G.nslices, SL * SW, 0,
              ctx->stream, G.sl_meta.p, (int)G.nslices, G.scol.p, G.scol16.p, G.sbase.p, G.sval64.p,
              (const double*)S->P.p, S->Q.p, S->part.p);
  finalize<K>(S, (long long)G.nslices, sc + K);
  hipStream_t st = ctx->stream;
  // the top depth's first colour-0 relaxation goes into the update (a
  // colour-ordered smoother above the coarsest depth)
  const bool first0 = nu1 > 0 && S->D > S->d0 && sweep_dinv<double>(S, G) != nullptr;
  const long long n0c = first0 ? (long long)G.coff[1] : 0LL;
  if (S->precision == 0) {
    CAMFE_TIMED(ctx, KT_CG_VEC, (7.0 * n * K * 8), (k_cg_update_v<K, 0>), (unsigned)nb, BLK, 0, st, (long long)n,
                (const double*)sc, S->X.p, S->R.p, (const double*)S->P.p, (const double*)S->Q.p, S->part2.p, S->Z.p,
                (float*)nullptr, (float*)nullptr, first0 ? sweep_dinv<double>(S, G) : (const double*)nullptr,
                (const float*)nullptr, n0c);
    vcycle<double, K>(S, S->D, S->R.p, S->Z.p, nu1, nu2, first0, !first0);
    hipLaunchKernelGGL((k_dot_rz<K, 0>), (unsigned)nb, BLK, 0, st, (long long)n, (const double*)S->R.p, S->Z.p,
                       (const float*)nullptr, S->part.p);
  } else {
    CAMFE_TIMED(ctx, KT_CG_VEC, (6.0 * n * K * 8 + 8.0 * n * K), (k_cg_update_v<K, 1>), (unsigned)nb, BLK, 0, st,
                (long long)n, (const double*)sc, S->X.p, S->R.p, (const double*)S->P.p, (const double*)S->Q.p,
                S->part2.p, (double*)nullptr, G.b32.p, G.x32.p, (const double*)nullptr,
                first0 ? sweep_dinv<float>(S, G) : (const float*)nullptr, n0c);
    vcycle<float, K>(S, S->D, G.b32.p, G.x32.p, nu1, nu2, first0, !first0);
    hipLaunchKernelGGL((k_dot_rz<K, 1>), (unsigned)nb, BLK, 0, st, (long long)n, (const double*)S->R.p, S->Z.p,
                       (const float*)G.x32.p, S->part.p);
  }
  hipLaunchKernelGGL(k_finalize_cg<K>, 1, 1024, 0, st, (const double*)S->part.p, (const double*)S->part2.p, (int)nb,
                     sc);
  hipLaunchKernelGGL(k_cg_direction<K>, (unsigned)nb, BLK, 0, st, (long long)n, (const double*)(sc + 5 * K),
                     (const double*)S->Z.p, S->P.p);
}

// One stationary step: x += V(b - A x); r = b - A x (||r||^2 into rr)
template <int K>
void stationary_step(SolverState* S, int nu1, int nu2) {
  camfe_ctx ctx = S->ctx;
  GLevel& G = S->lev[S->D];
  const long long nk = (long long)G.n * K;
  precondition<K>(S, S->R.p, S->Z.p, nu1, nu2);
  hipStream_t st = ctx->stream;
  hipLaunchKernelGGL(k_axpy_inplace<K>, grid_for(nk, BLK), BLK, 0, st, (long long)G.n, S->X.p, (const double*)S->Z.p);
  residual64<K>(S, S->B.p, S->X.p, S->R.p, S->sc.p + 2 * K);
}

// Solve columns [c0, c0 + K) of the problem (device canonical b, x col-major)
template <int K>
SolveResult solve_block(camfe_sys s, SolverState* S, const camfe_solve_opts& o, const double* db, double* dx, int kk,
                        int c0) {
  camfe_ctx ctx = s->h->ctx;
  hipStream_t st = ctx->stream;
  GLevel& G = S->lev[S->D];
  const size_t n = G.n;
  const long long nk = (long long)n * K;
  unsigned gn = grid_for(n, BLK), gnk = grid_for(nk, BLK);
  double* sc = S->sc.p;   // rz[K] pq[K] rr[K] rzn[K] bb[K] beta[K]
  hipLaunchKernelGGL(k_gather_in<K>, gn, BLK, 0, st, db, (long long)n, c0, kk, G.iperm.p, S->B.p);
  if (o.x0_given)
    hipLaunchKernelGGL(k_gather_in<K>, gn, BLK, 0, st, (const double*)dx, (long long)n, c0, kk, G.iperm.p, S->X.p);
  else
    hipLaunchKernelGGL((k_fill<double>), gnk, BLK, 0, st, S->X.p, nk, 0.0);
  hipLaunchKernelGGL((k_fill<double>), 1, 64, 0, st, sc, (long long)(8 * KMAXS), 0.0);
  dot<K>(S, S->B.p, S->B.p, sc + 4 * K);
  residual64<K>(S, S->B.p, S->X.p, S->R.p, sc + 2 * K);
  check_launch();
  double hb[3 * KMAXS];
  copy_out(ctx, hb, sc + 2 * K, 3 * K);   // rr[K], rz_new[K], bb[K]
  double bn[KMAXS];
  for (int c = 0; c < K; ++c) bn[c] = std::sqrt(hb[2 * K + c]);
  auto relmax = [&](const double* rr) {
    double m = 0;
    for (int c = 0; c < K && c0 + c < kk; ++c) {
      double v = bn[c] > 0 ? std::sqrt(rr[c]) / bn[c] : std::sqrt(rr[c]);
      if (!(v <= m)) m = v;   // keeps NaN
    }
    return m;
  };
  SolveResult res;
  res.rel = relmax(hb);
  const int nu1 = o.nu_pre, nu2 = o.nu_post;
  // captured steps are replayed `check_every` times between convergence checks
  const bool use_graph = !ctx->timer.on;
  const int check_every = 4;
  auto gkey = [&] {   // the smoother may change during a judged solve
    return (((((((long long)K * 2 + S->precision) * 64 + nu1) * 64 + nu2) * 2 + o.method) * 4 + S->smoother) * 4 +
            S->gamma) * 64 + S->nu_coarse;
  };
  auto run_steps = [&](int m, bool cg) {
    for (int i = 0; i < m; ++i) {
      if (use_graph)
        run_graph(S, gkey(), [&] { if (cg) cg_step<K>(S, nu1, nu2); else stationary_step<K>(S, nu1, nu2); });
      else if (cg)
        cg_step<K>(S, nu1, nu2);
      else
        stationary_step<K>(S, nu1, nu2);
    }
    check_launch();
    double rr[KMAXS];
    copy_out(ctx, rr, sc + 2 * K, K);
    return relmax(rr);
  };
  // a replacement smoother whose iteration runs away is stopped early (the
  // caller then redoes the solve with Gauss-Seidel)
  const double rel0 = res.rel;
  auto diverging = [&] { return S->smoother != 0 && res.rel > 1e2 * rel0; };
  if (o.method == 1) {
    while (res.rel > o.rtol && res.it < o.max_iter) {
      const int m = std::min(check_every, o.max_iter - res.it);
      res.rel = run_steps(m, false);
      res.it += m;
      res.cycles += m;
      if (!std::isfinite(res.rel) || diverging()) break;
    }
  } else if (res.rel > o.rtol && o.max_iter > 0) {
    // conjugate gradients preconditioned by one V-cycle
    auto cg_start = [&] {
      precondition<K>(S, S->R.p, S->Z.p, nu1, nu2);
      ++res.cycles;
      hipLaunchKernelGGL((k_convert<double, double>), gnk, BLK, 0, st, (const double*)S->Z.p, nk, S->P.p);
      dot<K>(S, S->R.p, S->Z.p, sc);
    };
    cg_start();
    const int nj = std::min(o.judge, o.max_iter);
    const int requested = S->smoother;   // restored below for the next column block
    if (S->smoother != 0 && nj > 0) {
      // Gauss-Seidel judges the replacement smoother: each runs nj CG
      // iterations from the start, and the one with the smaller residual
      // continues (its state kept, the other's iterations counted)
      const int smoother = S->smoother;
      res.rel = run_steps(nj, true);
      res.it += nj;
      res.cycles += nj;
      res.judge_rel[0] = res.rel;
      if (!(res.rel <= o.rtol)) {
        DArr<double> xs(nk), rs(nk), ps(nk), scs(8 * KMAXS);
        dcopy(ctx, xs.p, S->X.p, nk * sizeof(double));
        dcopy(ctx, rs.p, S->R.p, nk * sizeof(double));
        dcopy(ctx, ps.p, S->P.p, nk * sizeof(double));
        dcopy(ctx, scs.p, sc, 8 * KMAXS * sizeof(double));
        const double rel_a = res.rel;
        S->smoother = 0;
        if (o.x0_given)
          hipLaunchKernelGGL(k_gather_in<K>, gn, BLK, 0, st, (const double*)dx, (long long)n, c0, kk, G.iperm.p,
                             S->X.p);
        else
          hipLaunchKernelGGL((k_fill<double>), gnk, BLK, 0, st, S->X.p, nk, 0.0);
        residual64<K>(S, S->B.p, S->X.p, S->R.p, nullptr);
        cg_start();
        const double rel_b = run_steps(nj, true);
        res.it += nj;
        res.cycles += nj;
        res.judge_rel[1] = rel_b;
        if (rel_b < rel_a || !std::isfinite(rel_a)) {
          res.rel = rel_b;
          res.judged_gs = true;
        } else {
          S->smoother = smoother;
          dcopy(ctx, S->X.p, xs.p, nk * sizeof(double));
          dcopy(ctx, S->R.p, rs.p, nk * sizeof(double));
          dcopy(ctx, S->P.p, ps.p, nk * sizeof(double));
          dcopy(ctx, sc, scs.p, 8 * KMAXS * sizeof(double));
        }
      }
    }
    while (res.it < o.max_iter && !(res.rel <= o.rtol)) {
      const int m = std::min(check_every, o.max_iter - res.it);
      res.rel = run_steps(m, true);
      res.it += m;
      res.cycles += m;
      if (res.rel <= o.rtol || !std::isfinite(res.rel) || diverging()) break;
    }
    // true residual of the final iterate
    residual64<K>(S, S->B.p, S->X.p, S->R.p, sc + 2 * K);
    double rr[KMAXS];
    copy_out(ctx, rr, sc + 2 * K, K);
    res.rel = relmax(rr);
    S->smoother = requested;
  }
  hipLaunchKernelGGL(k_scatter_out<K>, gn, BLK, 0, st, (const double*)S->X.p, (long long)n, c0, kk, G.iperm.p, dx);
  check_launch();
  return res;
}

// ------------------------------------------------------------------ batch
// Many systems solved side by side.  Level bd of the batch holds, for every
// mesh m, its depth D_m - (Lmax - bd) when that is not below its coarsest
// depth: the finest depths line up at the top and each mesh bottoms out at
// its own coarsest depth, where its dense inverse is applied.  Rows are
// mesh-major (each mesh's rows padded to whole BLK-row blocks); slices are
// colour-major across meshes, so one launch per colour relaxes every mesh.
struct BatchMember {
  size_t n = 0;            // functions at the finest depth
  long long rowoff = 0;    // first row at the finest batch level
  DArr<int> iperm;         // canonical -> internal order at the finest depth
};

template <class T>
std::vector<T> to_host(camfe_ctx ctx, const DArr<T>& a, size_t n) {
  std::vector<T> h(n);
  if (n) copy_out(ctx, h.data(), a.p, n);
  return h;
}

__global__ void k_copy_add(const int* src, long long n, int add, int* dst) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n) dst[i] = src[i] + add;
}

inline long long pad_rows(long long n) { return (n + BLK - 1) / BLK * BLK; }


}  // namespace
}  // namespace camfe

struct camfe_batch_s {
  camfe_ctx ctx = nullptr;
  double t = 0, coarse_eps = 0;
  std::vector<camfe::BatchMember> mem;
  std::unique_ptr<camfe::SolverState> S;
};

namespace camfe {
namespace {

void build_batch(camfe_batch_s* Bt, const std::vector<SolverState*>& ms) {
  camfe_ctx ctx = Bt->ctx;
  const int nm = (int)ms.size();
  int Lmax = 0;
  for (auto* m : ms) Lmax = std::max(Lmax, m->D - m->d0);
  std::unique_ptr<SolverState> S(new SolverState());
  S->ctx = ctx;
  S->t = Bt->t;
  S->coarse_eps = Bt->coarse_eps;
  S->D = Lmax;
  S->d0 = 0;
  S->batch = true;
  S->nmesh = nm;
  S->lev.resize(Lmax + 1);
  auto mdepth = [&](int m, int bd) { return ms[m]->D - (Lmax - bd); };
  auto present = [&](int m, int bd) { return mdepth(m, bd) >= ms[m]->d0; };
  std::vector<std::vector<long long>> rowoff(Lmax + 1, std::vector<long long>(nm, -1));
  for (int bd = 0; bd <= Lmax; ++bd) {
    GLevel& G = S->lev[bd];
    G.d = bd;
    G.ncol = ms[0]->lev[ms[0]->D].ncol;
    long long off = 0;
    for (int m = 0; m < nm; ++m)
      if (present(m, bd)) {
        rowoff[bd][m] = off;
        off += pad_rows((long long)ms[m]->lev[mdepth(m, bd)].n);
      }
    G.n = (size_t)off;
    // slice metadata, colour-major across meshes
    struct Meta { std::vector<int> ptr, row0, rows; };
    std::vector<Meta> meta(nm);
    for (int m = 0; m < nm; ++m)
      if (present(m, bd)) {
        const GLevel& M = ms[m]->lev[mdepth(m, bd)];
        meta[m].ptr = to_host(ctx, M.sl_ptr, M.nslices + 1);
        meta[m].row0 = to_host(ctx, M.sl_row0, M.nslices);
        meta[m].rows = to_host(ctx, M.sl_rows, M.nslices);
      }
    std::vector<int> hp(1, 0), hrow0, hrows, hsm;
    G.cslice.assign(G.ncol + 1, 0);
    G.coff.assign(G.ncol + 1, 0);
    G.cnnz.assign(G.ncol, 0);
    G.nnz = 0;
    struct Chunk { int m; long long src, dst, cnt; };
    std::vector<Chunk> chunks;
    for (int c = 0; c < G.ncol; ++c) {
      G.cslice[c] = (int)hrow0.size();
      G.coff[c + 1] = G.coff[c];
      for (int m = 0; m < nm; ++m) {
        if (!present(m, bd)) continue;
        const GLevel& M = ms[m]->lev[mdepth(m, bd)];
        const int s0 = M.cslice[c], s1 = M.cslice[c + 1];
        if (s1 > s0) chunks.push_back({m, meta[m].ptr[s0], hp.back(), (long long)meta[m].ptr[s1] - meta[m].ptr[s0]});
        for (int sl = s0; sl < s1; ++sl) {
          hrow0.push_back((int)(meta[m].row0[sl] + rowoff[bd][m]));
          hrows.push_back(meta[m].rows[sl]);
          hsm.push_back(m);
          hp.push_back(hp.back() + meta[m].ptr[sl + 1] - meta[m].ptr[sl]);
        }
        G.coff[c + 1] += M.coff[c + 1] - M.coff[c];
        G.cnnz[c] += M.cnnz[c];
      }
    }
    G.cslice[G.ncol] = (int)hrow0.size();
    for (int m = 0; m < nm; ++m)
      if (present(m, bd)) G.nnz += ms[m]->lev[mdepth(m, bd)].nnz;
    G.nslices = hrow0.size();
    G.snnz = (size_t)hp.back();
    G.sl_ptr.alloc(G.nslices + 1);
    G.sl_row0.alloc(std::max<size_t>(G.nslices, 1));
    G.sl_rows.alloc(std::max<size_t>(G.nslices, 1));
    copy_in(ctx, G.sl_ptr.p, hp.data(), hp.size());
    if (G.nslices) {
      copy_in(ctx, G.sl_row0.p, hrow0.data(), G.nslices);
      copy_in(ctx, G.sl_rows.p, hrows.data(), G.nslices);
    }
    pack_meta(ctx, G, hp, hrow0, hrows);
    // the full records, and the member of each slice and of each BLK-row block
    G.sl_meta_all.alloc(G.sl_meta.n);
    dcopy(ctx, G.sl_meta_all.p, G.sl_meta.p, G.sl_meta.n * sizeof(int4));
    hsm.resize(std::max<size_t>(G.nslices, 1), 0);
    G.slmem.alloc(hsm.size());
    copy_in(ctx, G.slmem.p, hsm.data(), hsm.size());
    {
      std::vector<int> bm(std::max<size_t>(G.n / BLK, 1), 0);
      for (int m = 0; m < nm; ++m)
        if (present(m, bd))
          for (long long r = rowoff[bd][m]; r < rowoff[bd][m] + pad_rows((long long)ms[m]->lev[mdepth(m, bd)].n);
               r += BLK)
            bm[r / BLK] = m;
      G.blkmem.alloc(bm.size());
      copy_in(ctx, G.blkmem.p, bm.data(), bm.size());
    }
    G.scol.alloc(G.snnz);
    G.sval64.alloc(G.snnz);
    G.sval32.alloc(G.snnz);
    for (const Chunk& ch : chunks) {
      const GLevel& M = ms[ch.m]->lev[mdepth(ch.m, bd)];
      dcopy(ctx, G.sval64.p + ch.dst, M.sval64.p + ch.src, ch.cnt * sizeof(double));
      dcopy(ctx, G.sval32.p + ch.dst, M.sval32.p + ch.src, ch.cnt * sizeof(float));
      hipLaunchKernelGGL(k_copy_add, grid_for(ch.cnt, BLK), BLK, 0, ctx->stream, M.scol.p + ch.src, ch.cnt,
                         (int)rowoff[bd][ch.m], G.scol.p + ch.dst);
    }
    check_launch();
    G.invd64.alloc(G.n);
    G.invd32.alloc(G.n);
    zero(ctx, G.invd64.p, G.n);
    zero(ctx, G.invd32.p, G.n);
    for (int m = 0; m < nm; ++m)
      if (present(m, bd)) {
        const GLevel& M = ms[m]->lev[mdepth(m, bd)];
        dcopy(ctx, G.invd64.p + rowoff[bd][m], M.invd64.p, M.n * sizeof(double));
        dcopy(ctx, G.invd32.p + rowoff[bd][m], M.invd32.p, M.n * sizeof(float));
      }
    const size_t nk = G.n * KMAXS;
    for (DArr<double>* v : {&G.x64, &G.b64, &G.r64, &G.t64}) { v->alloc(nk); zero(ctx, v->p, nk); }
    for (DArr<float>* v : {&G.x32, &G.b32, &G.r32, &G.t32}) { v->alloc(nk); zero(ctx, v->p, nk); }
    // meshes solved directly at this level
    std::vector<int> cro, ccum(1, 0), cmem;
    std::vector<long long> caoff;
    long long atot = 0;
    for (int m = 0; m < nm; ++m)
      if (present(m, bd) && mdepth(m, bd) == ms[m]->d0 && ms[m]->direct) {
        cmem.push_back(m);
        cro.push_back((int)rowoff[bd][m]);
        ccum.push_back(ccum.back() + ms[m]->n0);
        caoff.push_back(atot);
        atot += (long long)ms[m]->n0 * ms[m]->n0;
      }
    G.ncb = (int)cro.size();
    G.cb_rows = ccum.back();
    if (G.ncb) {
      G.cb_rowoff.alloc(G.ncb);
      G.cb_cum.alloc(G.ncb + 1);
      G.cb_aoff.alloc(G.ncb);
      copy_in(ctx, G.cb_rowoff.p, cro.data(), cro.size());
      copy_in(ctx, G.cb_cum.p, ccum.data(), ccum.size());
      copy_in(ctx, G.cb_aoff.p, caoff.data(), caoff.size());
      G.cbmem.alloc(G.ncb);
      copy_in(ctx, G.cbmem.p, cmem.data(), cmem.size());
      G.cb_a64.alloc(atot);
      int j = 0;
      for (int m = 0; m < nm; ++m)
        if (present(m, bd) && mdepth(m, bd) == ms[m]->d0 && ms[m]->direct) {
          const size_t na = (size_t)ms[m]->n0 * ms[m]->n0;
          dcopy(ctx, G.cb_a64.p + caoff[j], ms[m]->Ainv64.p, na * sizeof(double));
          ++j;
        }
    }
  }
  // transfers between batch levels bd (fine) and bd - 1
  for (int bd = 1; bd <= Lmax; ++bd) {
    GLevel& F = S->lev[bd];
    GLevel& Cc = S->lev[bd - 1];
    std::vector<int> pcnt(F.n + 1, 0), rcnt(Cc.n + 1, 0);
    struct TChunk { int m; long long psrc_n, pdst_row, rsrc_n, rdst_row; };
    std::vector<TChunk> tch;
    for (int m = 0; m < nm; ++m) {
      if (!present(m, bd - 1)) continue;
      const GLevel& MF = ms[m]->lev[mdepth(m, bd)];
      std::vector<int> mp = to_host(ctx, MF.Pptr, MF.n + 1);
      std::vector<int> mr = to_host(ctx, MF.Rptr, ms[m]->lev[mdepth(m, bd - 1)].n + 1);
      for (size_t i = 0; i < MF.n; ++i) pcnt[rowoff[bd][m] + i + 1] = mp[i + 1] - mp[i];
      const size_t ncm = ms[m]->lev[mdepth(m, bd - 1)].n;
      for (size_t i = 0; i < ncm; ++i) rcnt[rowoff[bd - 1][m] + i + 1] = mr[i + 1] - mr[i];
      tch.push_back({m, (long long)mp[MF.n], rowoff[bd][m], (long long)mr[ncm], rowoff[bd - 1][m]});
    }
    for (size_t i = 0; i < F.n; ++i) pcnt[i + 1] += pcnt[i];
    for (size_t i = 0; i < Cc.n; ++i) rcnt[i + 1] += rcnt[i];
    const long long pn = pcnt[F.n];
    F.pnnz = pn;
    F.Pptr.alloc(F.n + 1);
    F.Rptr.alloc(Cc.n + 1);
    copy_in(ctx, F.Pptr.p, pcnt.data(), pcnt.size());
    copy_in(ctx, F.Rptr.p, rcnt.data(), rcnt.size());
    F.Pcol.alloc(std::max<long long>(pn, 1));
    F.Pw64.alloc(std::max<long long>(pn, 1));
    F.Pw32.alloc(std::max<long long>(pn, 1));
    F.Rcol.alloc(std::max<long long>(pn, 1));
    F.Rw64.alloc(std::max<long long>(pn, 1));
    F.Rw32.alloc(std::max<long long>(pn, 1));
    for (const TChunk& t : tch) {
      const GLevel& MF = ms[t.m]->lev[mdepth(t.m, bd)];
      const long long pd = pcnt[t.pdst_row], rd = rcnt[t.rdst_row];
      hipLaunchKernelGGL(k_copy_add, grid_for(t.psrc_n, BLK), BLK, 0, ctx->stream, MF.Pcol.p, t.psrc_n,
                         (int)rowoff[bd - 1][t.m], F.Pcol.p + pd);
      dcopy(ctx, F.Pw64.p + pd, MF.Pw64.p, t.psrc_n * sizeof(double));
      dcopy(ctx, F.Pw32.p + pd, MF.Pw32.p, t.psrc_n * sizeof(float));
      hipLaunchKernelGGL(k_copy_add, grid_for(t.rsrc_n, BLK), BLK, 0, ctx->stream, MF.Rcol.p, t.rsrc_n,
                         (int)rowoff[bd][t.m], F.Rcol.p + rd);
      dcopy(ctx, F.Rw64.p + rd, MF.Rw64.p, t.rsrc_n * sizeof(double));
      dcopy(ctx, F.Rw32.p + rd, MF.Rw32.p, t.rsrc_n * sizeof(float));
    }
    check_launch();
  }
  // finest level: mesh of every block, outer vectors, scalars
  const GLevel& T = S->lev[Lmax];
  const size_t nb = T.n / BLK;
  std::vector<int> bm(std::max<size_t>(nb, 1), 0), bs(nm + 1, 0);
  Bt->mem.resize(nm);
  for (int m = 0; m < nm; ++m) {
    const long long b0 = rowoff[Lmax][m] / BLK;
    const long long cnt = pad_rows((long long)ms[m]->lev[ms[m]->D].n) / BLK;
    for (long long b = b0; b < b0 + cnt; ++b) bm[b] = m;
    bs[m] = (int)b0;
    bs[m + 1] = (int)(b0 + cnt);
    BatchMember& me = Bt->mem[m];
    me.n = ms[m]->lev[ms[m]->D].n;
    me.rowoff = rowoff[Lmax][m];
    me.iperm.alloc(me.n);
    dcopy(ctx, me.iperm.p, ms[m]->lev[ms[m]->D].iperm.p, me.n * sizeof(int));
  }
  S->bmesh.alloc(bm.size());
  S->bstart.alloc(nm + 1);
  copy_in(ctx, S->bmesh.p, bm.data(), bm.size());
  copy_in(ctx, S->bstart.p, bs.data(), bs.size());
  const size_t n = T.n * KMAXS;
  for (DArr<double>* v : {&S->X, &S->R, &S->Z, &S->P, &S->Q, &S->B}) { v->alloc(n); zero(ctx, v->p, n); }
  S->sc.alloc((size_t)nm * SCS);
  zero(ctx, S->sc.p, S->sc.n);
  S->mact.alloc(nm);
  {
    std::vector<int> on(nm, 1);
    copy_in(ctx, S->mact.p, on.data(), on.size());
  }
  S->part.alloc((std::max(T.nslices, nb) + 1) * KMAXS);
  ctx->sync();
  Bt->S = std::move(S);
}

template <int K>
void dot_seg(SolverState* S, const double* a, const double* b, int off) {
  const GLevel& G = S->lev[S->D];
  const long long nb = (long long)(G.n / BLK);
  hipLaunchKernelGGL(k_dot_b<K>, (unsigned)nb, BLK, 0, S->ctx->stream, (long long)G.n, (const int*)S->bmesh.p,
                     (const int*)S->mact.p, a, b, S->part.p);
  hipLaunchKernelGGL(k_finalize_seg<K>, (unsigned)S->nmesh, BLK, 0, S->ctx->stream, (const double*)S->part.p,
                     S->bstart.p, S->sc.p, off);
}

// One batched CG step (per-mesh scalars; frozen columns keep x and r)
template <int K>
void cg_step_b(SolverState* S, int nu1, int nu2) {
  camfe_ctx ctx = S->ctx;
  GLevel& G = S->lev[S->D];
  const size_t n = G.n;
  const long long nb = (long long)(n / BLK);
  CAMFE_TIMED(ctx, KT_SPMV, ((double)G.nnz * 8 + 2.0 * n * K * 8), k_spmv_dot<K>, (unsigned)G.nslices, SL * SW, 0,
              ctx->stream, G.sl_meta.p, (int)G.nslices, G.scol.p, G.scol16.p, G.sbase.p, G.sval64.p,
              (const double*)S->P.p, S->Q.p, S->part.p);
  dot_seg<K>(S, S->P.p, S->Q.p, K);
  CAMFE_TIMED(ctx, KT_CG_VEC, (6.0 * n * K * 8), k_cg_update_b<K>, (unsigned)nb, BLK, 0, ctx->stream, (long long)n,
              (const int*)S->bmesh.p, (const double*)S->sc.p, S->X.p, S->R.p, (const double*)S->P.p,
              (const double*)S->Q.p, S->part.p);
  hipLaunchKernelGGL(k_finalize_seg<K>, (unsigned)S->nmesh, BLK, 0, ctx->stream, (const double*)S->part.p,
                     S->bstart.p, S->sc.p, 2 * K);
  precondition<K>(S, S->R.p, S->Z.p, nu1, nu2);
  dot_seg<K>(S, S->R.p, S->Z.p, 3 * K);
  hipStream_t st = ctx->stream;
  hipLaunchKernelGGL(k_cg_direction_b<K>, (unsigned)nb, BLK, 0, st, (long long)n, (const int*)S->bmesh.p,
                     (const double*)S->sc.p, (const double*)S->Z.p, S->P.p);
  hipLaunchKernelGGL(k_copy_rz_b<K>, grid_for((size_t)S->nmesh * K, 64), 64, 0, st, S->nmesh, S->sc.p);
}

// Solve columns [c0, c0 + K) of every mesh; res[m] gets the mesh's result
template <int K>
void batch_solve_block(camfe_batch_s* Bt, const camfe_solve_opts& o, const std::vector<DArr<double>>& db,
                       std::vector<DArr<double>>& dx, const std::vector<int>& kk, int c0,
                       std::vector<SolveResult>& res) {
  SolverState* S = Bt->S.get();
  camfe_ctx ctx = S->ctx;
  hipStream_t st = ctx->stream;
  GLevel& G = S->lev[S->D];
  const int nm = S->nmesh;
  const long long nk = (long long)G.n * K;
  const unsigned gnk = grid_for(nk, BLK);
  // every outer vector starts at zero: the rows that pad each member to whole
  // blocks are written by no kernel but enter the per-block dot products, so
  // what an earlier pass (another column count, another layout) left there
  // must not survive
  for (double* v : {S->B.p, S->X.p, S->R.p, S->Z.p, S->P.p, S->Q.p})
    hipLaunchKernelGGL((k_fill<double>), gnk, BLK, 0, st, v, nk, 0.0);
  for (int m = 0; m < nm; ++m) {
    const BatchMember& me = Bt->mem[m];
    if (c0 >= kk[m]) continue;
    hipLaunchKernelGGL(k_gather_in<K>, grid_for(me.n, BLK), BLK, 0, st, (const double*)db[m].p, (long long)me.n, c0,
                       kk[m], me.iperm.p, S->B.p + me.rowoff * K);
    if (o.x0_given)
      hipLaunchKernelGGL(k_gather_in<K>, grid_for(me.n, BLK), BLK, 0, st, (const double*)dx[m].p, (long long)me.n,
                         c0, kk[m], me.iperm.p, S->X.p + me.rowoff * K);
  }
  std::vector<double> rel((size_t)nm * K, 0.0);
  // relative residual per (mesh, column); act = 1 while above rtol.  A column
  // once frozen stays frozen (its x and r no longer change), and a member
  // whose columns are all frozen is gated off: its slices are emptied and
  // the gated kernels skip its blocks, so the batch costs what its members
  // still iterating cost.  The gated members' scalars are not maintained, so
  // the frozen state is kept here, not re-derived from them.
  std::vector<char> live((size_t)nm * K, 1);
  std::vector<int> mon(nm, 1), mon_dev;   // mon_dev: flags on the device (unknown at first)
  std::vector<double> hs((size_t)nm * SCS);
  auto update = [&](bool set_act) {
    bool any = false;
    for (int m = 0; m < nm; ++m) {
      bool mlive = false;
      for (int c = 0; c < K; ++c) {
        double* sc = hs.data() + (size_t)m * SCS;
        const bool col = c0 + c < kk[m];
        const double bn = std::sqrt(sc[4 * K + c]);
        const double v = !col ? 0.0 : (bn > 0 ? std::sqrt(sc[2 * K + c]) / bn : std::sqrt(sc[2 * K + c]));
        if (!set_act) {   // final residuals: every column's
          rel[(size_t)m * K + c] = v;
          continue;
        }
        char& lv = live[(size_t)m * K + c];
        if (lv) rel[(size_t)m * K + c] = v;
        lv = lv && col && std::isfinite(v) && v > o.rtol;
        sc[5 * K + c] = lv ? 1.0 : 0.0;
        mlive = mlive || lv;
      }
      mon[m] = mlive ? 1 : 0;
      any = any || mlive;
    }
    return any;
  };
  // push the members' active flags and re-gate the slice records of every level
  auto gate = [&](const std::vector<int>& on) {
    if (on == mon_dev) return;
    mon_dev = on;
    copy_in(ctx, S->mact.p, on.data(), on.size());
    for (int bd = S->d0; bd <= S->D; ++bd) {
      GLevel& L = S->lev[bd];
      if (L.nslices)
        hipLaunchKernelGGL(k_gate_meta, grid_for(L.nslices, BLK), BLK, 0, st, (long long)L.nslices,
                           (const int4*)L.sl_meta_all.p, (const int*)L.slmem.p, (const int*)S->mact.p, L.sl_meta.p);
    }
  };
  // every member on, and every slice record whole again when this returns or throws
  struct Ungate {
    SolverState* S;
    ~Ungate() {
      std::vector<int> on(S->nmesh, 1);
      (void)hipMemcpyAsync(S->mact.p, on.data(), on.size() * sizeof(int), hipMemcpyHostToDevice, S->ctx->stream);
      for (int bd = S->d0; bd <= S->D; ++bd) {
        GLevel& L = S->lev[bd];
        (void)hipMemcpyAsync(L.sl_meta.p, L.sl_meta_all.p, L.sl_meta.n * sizeof(int4), hipMemcpyDeviceToDevice,
                             S->ctx->stream);
      }
      (void)hipStreamSynchronize(S->ctx->stream);
    }
  } ungate{S};
  gate(std::vector<int>(nm, 1));
  hipLaunchKernelGGL((k_fill<double>), grid_for(S->sc.n, BLK), BLK, 0, st, S->sc.p, (long long)S->sc.n, 0.0);
  dot_seg<K>(S, S->B.p, S->B.p, 4 * K);
  hipLaunchKernelGGL((k_residual<double, double, K>), (unsigned)G.nslices, SL * SW, 0, st, G.sl_meta.p,
                     (int)G.nslices, G.scol.p, G.scol16.p, G.sbase.p, G.sval64.p, (const double*)S->B.p, (const double*)S->X.p, S->R.p,
                     (double*)nullptr);
  dot_seg<K>(S, S->R.p, S->R.p, 2 * K);
  check_launch();
  copy_out(ctx, hs.data(), S->sc.p, hs.size());
  bool any = update(true);
  copy_in(ctx, S->sc.p, hs.data(), hs.size());
  gate(mon);
  const std::vector<int> mon0 = mon;   // members that take the first cycle
  int it = 0, cycles = 0;
  std::vector<int> mit(nm, 0);   // iterations each member took part in
  const int nu1 = o.nu_pre, nu2 = o.nu_post;
  const bool use_graph = !ctx->timer.on;
  const int check_every = 4;
  const long long gkey = (((((long long)K * 2 + S->precision) * 64 + nu1) * 64 + nu2) * 8 + 5) * 64 + S->nu_coarse;
  if (any && o.max_iter > 0) {
    precondition<K>(S, S->R.p, S->Z.p, nu1, nu2);
    ++cycles;
    hipLaunchKernelGGL((k_convert<double, double>), gnk, BLK, 0, st, (const double*)S->Z.p, nk, S->P.p);
    dot_seg<K>(S, S->R.p, S->Z.p, 0);
    while (any && it < o.max_iter) {
      const int mm = std::min(check_every, o.max_iter - it);
      for (int i = 0; i < mm; ++i) {
        if (use_graph) run_graph(S, gkey, [&] { cg_step_b<K>(S, nu1, nu2); });
        else cg_step_b<K>(S, nu1, nu2);
      }
      check_launch();
      it += mm;
      cycles += mm;
      for (int m = 0; m < nm; ++m) mit[m] += mon[m] ? mm : 0;
      copy_out(ctx, hs.data(), S->sc.p, hs.size());
      any = update(true);
      copy_in(ctx, S->sc.p, hs.data(), hs.size());
      gate(mon);
    }
    // true residuals of the final iterates, over every member
    gate(std::vector<int>(nm, 1));
    hipLaunchKernelGGL((k_residual<double, double, K>), (unsigned)G.nslices, SL * SW, 0, st, G.sl_meta.p,
                       (int)G.nslices, G.scol.p, G.scol16.p, G.sbase.p, G.sval64.p, (const double*)S->B.p, (const double*)S->X.p, S->R.p,
                       (double*)nullptr);
    dot_seg<K>(S, S->R.p, S->R.p, 2 * K);
    copy_out(ctx, hs.data(), S->sc.p, hs.size());
    update(false);
  }
  for (int m = 0; m < nm; ++m) {
    const BatchMember& me = Bt->mem[m];
    if (c0 >= kk[m]) continue;
    hipLaunchKernelGGL(k_scatter_out<K>, grid_for(me.n, BLK), BLK, 0, st, (const double*)(S->X.p + me.rowoff * K),
                       (long long)me.n, c0, kk[m], me.iperm.p, dx[m].p);
    SolveResult& r = res[m];
    r.it = std::max(r.it, mit[m]);
    r.cycles += mit[m] + (cycles > 0 && mon0[m] ? 1 : 0);
    for (int c = 0; c < K; ++c)
      if (c0 + c < kk[m] && !(rel[(size_t)m * K + c] <= r.rel)) r.rel = rel[(size_t)m * K + c];
  }
  check_launch();
}

}  // namespace

// The values of M (or L) changed with the structure kept: repack A = M + t L
// into the existing SELL arrays of every depth and refactor the coarsest
// depth, in place.  Learned weights are recomputed at the next solve.
void refresh_solver(camfe_sys s) {
  SolverState* S = s->solver;
  if (!S) return;
  camfe_ctx ctx = s->h->ctx;
  auto t0 = std::chrono::steady_clock::now();
  for (int d = S->d0; d <= S->D; ++d) {
    GLevel& G = S->lev[d];
    const SLevel& L = s->lev[d];
    const long long threads = (long long)G.nslices * SL;
    hipLaunchKernelGGL(k_sell_fill, grid_for(threads, BLK), BLK, 0, ctx->stream, L.ptr.p, L.col.p, L.M.p, L.L.p,
                       S->t, G.perm.p, G.iperm.p, G.sl_ptr.p, G.sl_row0.p, G.sl_rows.p, (long long)G.nslices,
                       G.scol.p, G.sval64.p, G.sval32.p, G.invd64.p, G.invd32.p);
    check_launch();
  }
  setup_coarsest(s, S);
  S->wkind = 0;
  S->model = nullptr;
  ctx->sync();
  S->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// solver state for (t, coarse_eps), rebuilt when either changes
SolverState* ensure_solver(camfe_sys s, double t, double coarse_eps) {
  SolverState* S = s->solver;
  if (!S || S->t != t || S->coarse_eps != coarse_eps) {
    destroy_solver(S);
    s->solver = nullptr;
    s->solver = setup(s, t, 0, coarse_eps);
    S = s->solver;
  }
  return S;
}

// Coarse-grid correction of the V-cycle at depth d > d0 on four columns
// (n_d x 4 row-major, internal order), with B_c one plain FP64 Gauss-Seidel
// V(2,2)-cycle at depth d-1 (a symmetric operator):
//   adjoint == 0: out = e - P B_c P^T A e
//   adjoint == 1: out = e - A P B_c P^T e   (the transpose of the first)
void coarse_correction(SolverState* S, int d, const double* e, double* out, bool adjoint) {
  camfe_ctx ctx = S->ctx;
  hipStream_t st = ctx->stream;
  GLevel& G = S->lev[d];
  GLevel& C = S->lev[d - 1];
  constexpr int K = KMAXS;
  const long long nk = (long long)G.n * K;
  const int sm = S->smoother;
  S->smoother = 0;
  double* r = G.r64.p;
  if (!adjoint) {
    // r = 0 - A e, b_c = P^T r = -P^T A e
    hipLaunchKernelGGL((k_fill<double>), grid_for(nk, BLK), BLK, 0, st, G.t64.p, nk, 0.0);
    hipLaunchKernelGGL((k_residual<double, double, K>), (unsigned)G.nslices, SL * SW, 0, st, G.sl_meta.p,
                       (int)G.nslices, G.scol.p, G.scol16.p, G.sbase.p, G.sval64.p, (const double*)G.t64.p, e, r, (double*)nullptr);
  } else {
    hipLaunchKernelGGL((k_convert<double, double>), grid_for(nk, BLK), BLK, 0, st, e, nk, r);
  }
  hipLaunchKernelGGL((k_restrict<double, K>), grid_for(C.n * RL, BLK), BLK, 0, st, G.Rptr.p, G.Rcol.p, G.Rw64.p,
                     (long long)C.n, (const double*)r, C.b64.p, C.x64.p, (const double*)nullptr, 0LL,
                     (const int*)nullptr, (const int*)nullptr);
  vcycle<double, K>(S, d - 1, C.b64.p, C.x64.p, 2, 2);
  if (!adjoint) {
    // out = e + P x_c  (x_c = -B_c P^T A e)
    hipLaunchKernelGGL((k_convert<double, double>), grid_for(nk, BLK), BLK, 0, st, e, nk, out);
    hipLaunchKernelGGL((k_prolong<double, K>), grid_for(G.n, BLK), BLK, 0, st, G.Pptr.p, G.Pcol.p, G.Pw64.p,
                       (long long)G.n, (const double*)C.x64.p, out, (const int*)nullptr, (const int*)nullptr);
  } else {
    // t = P x_c (x_c = B_c P^T e), out = e - A t
    hipLaunchKernelGGL((k_fill<double>), grid_for(nk, BLK), BLK, 0, st, G.t64.p, nk, 0.0);
    hipLaunchKernelGGL((k_prolong<double, K>), grid_for(G.n, BLK), BLK, 0, st, G.Pptr.p, G.Pcol.p, G.Pw64.p,
                       (long long)G.n, (const double*)C.x64.p, G.t64.p, (const int*)nullptr,
                       (const int*)nullptr);
    hipLaunchKernelGGL((k_residual<double, double, K>), (unsigned)G.nslices, SL * SW, 0, st, G.sl_meta.p,
                       (int)G.nslices, G.scol.p, G.scol16.p, G.sbase.p, G.sval64.p, e, (const double*)G.t64.p, out, (double*)nullptr);
  }
  S->smoother = sm;
  check_launch();
}

// one FP64 Gauss-Seidel V(nu1, nu2)-cycle at depth d on A e = 0 for four
// columns (x: n_d x 4 row-major, internal order), in place
void plain_vcycle_at(SolverState* S, int d, double* x, int nu1, int nu2) {
  const long long nk = (long long)S->lev[d].n * KMAXS;
  hipLaunchKernelGGL((k_fill<double>), grid_for(nk, BLK), BLK, 0, S->ctx->stream, S->B.p, nk, 0.0);
  const int sm = S->smoother;
  S->smoother = 0;
  vcycle<double, KMAXS>(S, d, S->B.p, x, nu1, nu2);
  S->smoother = sm;
  check_launch();
}

}  // namespace camfe

using namespace camfe;

namespace camfe {
// Solve (M + t L) X = B for k device columns (canonical order, n x k
// column-major) with the multicolour Gauss-Seidel cycles of o (smoother 0);
// X is the start when o.x0_given.  For callers inside the library.
SolveSummary solve_device(camfe_sys s, const camfe_solve_opts& o, const double* db, double* dx, int k) {
  SolverState* S = ensure_solver(s, o.t, o.coarse_eps);
  S->precision = o.precision;
  S->smoother = 0;
  struct GammaScope {
    SolverState* S;
    ~GammaScope() { S->gamma = 1; }
  } gamma_scope{S};
  S->gamma = o.cycle == 2 ? 2 : 1;
  SolveSummary tot;
  for (int c0 = 0; c0 < k; c0 += KMAXS) {
    const int kb = std::min(KMAXS, k - c0);
    SolveResult r;
    switch (kb) {
      case 1: r = solve_block<1>(s, S, o, db, dx, k, c0); break;
      case 2: r = solve_block<2>(s, S, o, db, dx, k, c0); break;
      case 3: r = solve_block<3>(s, S, o, db, dx, k, c0); break;
      default: r = solve_block<4>(s, S, o, db, dx, k, c0); break;
    }
    tot.iterations = std::max(tot.iterations, r.it);
    tot.cycles += r.cycles;
    if (!(r.rel <= tot.rel)) tot.rel = r.rel;
  }
  return tot;
}
}  // namespace camfe

extern "C" {

camfe_status camfe_measure_kernel(camfe_sys s, const char* kernel, int precision, int reps, double* avg_ms,
                                  double* bytes_per_launch) {
  return guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s && kernel && reps > 0 && (precision == 0 || precision == 1), CAMFE_EINVAL, "bad argument");
    SolverState* S = s->solver;
    CAMFE_REQUIRE(S, CAMFE_ESTATE, "no solver state: call camfe_solve first");
    camfe_ctx ctx = s->h->ctx;
    ctx->use_device();
    GLevel& G = S->lev[S->D];
    const std::string name(kernel);
    int kid = -1;
    if (name == "gs_colour") kid = 0;
    else if (name == "residual") kid = 1;
    else if (name == "spmv_dot") kid = 2;
    else if (name == "empty") kid = 3;
    else if (name == "copy") kid = 4;
    // "vcycle" or "vcycle:<sweeps at the finest depth>,<sweeps below>"
    int cyc_nu = 2, cyc_nc = 0;
    if (name == "vcycle") kid = 5;
    else if (name.rfind("vcycle:", 0) == 0) {
      int a = 0, c = 0;
      char tail = 0;
      CAMFE_REQUIRE(std::sscanf(name.c_str() + 7, "%d,%d%c", &a, &c, &tail) == 2 && a >= 1 && a <= 16 && c >= 0 &&
                        c <= 16,
                    CAMFE_EINVAL, "vcycle schedule: vcycle:<1-16>,<0-16>");
      kid = 5;
      cyc_nu = a;
      cyc_nc = c;
    }
    CAMFE_REQUIRE(kid >= 0, CAMFE_EINVAL,
                  "measurable kernels: gs_colour, residual, spmv_dot, empty, copy, vcycle[:nu,nu_below]");
    const long long nk = (long long)G.n;
    hipStream_t st = ctx->stream;
    hipLaunchKernelGGL((k_fill<double>), grid_for(nk, BLK), BLK, 0, st, G.b64.p, nk, 1.0);
    hipLaunchKernelGGL((k_fill<double>), grid_for(nk, BLK), BLK, 0, st, G.x64.p, nk, 0.0);
    hipLaunchKernelGGL((k_fill<float>), grid_for(nk, BLK), BLK, 0, st, G.b32.p, nk, 1.0f);
    hipLaunchKernelGGL((k_fill<float>), grid_for(nk, BLK), BLK, 0, st, G.x32.p, nk, 0.0f);
    // launches per repetition and algorithmic bytes of a colour sweep
    double launches = 0, sweep_bytes = 0;
    for (int c = 0; c < G.ncol; ++c)
      if (G.cslice[c + 1] > G.cslice[c]) {
        launches += 1;
        sweep_bytes += precision == 0 ? pass_bytes<double, 1>(G.cnnz[c], G.coff[c + 1] - G.coff[c])
                                      : pass_bytes<float, 1>(G.cnnz[c], G.coff[c + 1] - G.coff[c]);
      }
    double bytes = sweep_bytes;
    if (kid == 1) {
      launches = 1;
      bytes = precision == 0 ? pass_bytes<double, 1>(G.nnz, nk) : pass_bytes<float, 1>(G.nnz, nk);
    }
    if (kid == 2) { launches = 1; bytes = (double)G.nnz * 8 + 2.0 * nk * 8; }
    if (kid == 3) bytes = 0;
    if (kid == 5) { launches = 1; bytes = 0; }   // one whole cycle per repetition; bytes left to the caller
    // the copy moves a colour launch's average bytes (half read, half written)
    // per launch, rotating through NCP buffer pairs so that, like the colours'
    // matrices, its data does not stay in the L2 caches between launches
    constexpr int NCP = 16;
    const long long m16 = std::max(1LL, (long long)(sweep_bytes / std::max(launches, 1.0) / 32.0 + 0.5));
    DArr<double2> csrc, cdst;
    if (kid == 4) {
      csrc.alloc((size_t)m16 * NCP);
      cdst.alloc((size_t)m16 * NCP);
      hipLaunchKernelGGL((k_fill<double>), grid_for(2 * m16 * NCP, BLK), BLK, 0, st, (double*)csrc.p,
                         2 * m16 * NCP, 1.0);
      bytes = 32.0 * m16 * launches;
    }
    auto enqueue = [&] {
      int cp = 0;
      for (int r = 0; r < reps; ++r) {
        if (kid == 0) {
          if (precision == 0) gs_sweep<double, 1>(ctx, G, G.b64.p, G.x64.p, true, G.invd64.p);
          else gs_sweep<float, 1>(ctx, G, G.b32.p, G.x32.p, true, G.invd32.p);
        } else if (kid == 1) {
          if (precision == 0)
            hipLaunchKernelGGL((k_residual<double, double, 1>), (unsigned)G.nslices, SL * SW, 0,
                               ctx->stream, G.sl_meta.p, (int)G.nslices, G.scol.p, G.scol16.p, G.sbase.p,
                               G.sval64.p, (const double*)G.b64.p, (const double*)G.x64.p, G.r64.p, (double*)nullptr);
          else
            hipLaunchKernelGGL((k_residual<float, float, 1>), (unsigned)G.nslices, SL * SW, 0,
                               ctx->stream, G.sl_meta.p, (int)G.nslices, G.scol.p, G.scol16.p, G.sbase.p,
                               G.sval32.p, (const float*)G.b32.p, (const float*)G.x32.p, G.r32.p, (double*)nullptr);
        } else if (kid == 2) {
          hipLaunchKernelGGL(k_spmv_dot<1>, (unsigned)G.nslices, SL * SW, 0, ctx->stream, G.sl_meta.p,
                             (int)G.nslices, G.scol.p, G.scol16.p, G.sbase.p, G.sval64.p, (const double*)G.x64.p, G.r64.p, S->part.p);
        } else if (kid == 5) {
          // one plain Gauss-Seidel V-cycle from a zero guess, as the
          // preconditioner of a CG step applies it (one column)
          if (precision == 0) {
            hipLaunchKernelGGL((k_fill<double>), grid_for(nk, BLK), BLK, 0, st, G.x64.p, nk, 0.0);
            vcycle<double, 1>(S, S->D, G.b64.p, G.x64.p, cyc_nu, cyc_nu);
          } else {
            hipLaunchKernelGGL((k_fill<float>), grid_for(nk, BLK), BLK, 0, st, G.x32.p, nk, 0.0f);
            vcycle<float, 1>(S, S->D, G.b32.p, G.x32.p, cyc_nu, cyc_nu);
          }
        } else {
          for (int c = 0; c < G.ncol; ++c) {
            const int s0 = G.cslice[c], s1 = G.cslice[c + 1];
            if (s1 == s0) continue;
            if (kid == 3) {
              hipLaunchKernelGGL(k_nop, (unsigned)(s1 - s0), SL * SW, 0, ctx->stream);
            } else {
              const long long o = (long long)(cp++ % NCP) * m16;
              hipLaunchKernelGGL(k_copy16, grid_for(m16, BLK), BLK, 0, ctx->stream, (const double2*)csrc.p + o,
                                 cdst.p + o, m16);
            }
          }
        }
      }
    };
    struct CycleScope {   // the measured cycle is the plain one, whatever the last solve used
      SolverState* S;
      int sm, g, nc;
      ~CycleScope() { S->smoother = sm; S->gamma = g; S->nu_coarse = nc; }
    } cycle_scope{S, S->smoother, S->gamma, S->nu_coarse};
    if (kid == 5) { S->smoother = 0; S->gamma = 1; S->nu_coarse = cyc_nc; }
    const long long sched = kid == 5 ? (long long)(cyc_nu * 17 + cyc_nc) : 0;
    const long long key = -1 - ((((long long)kid * 2 + precision) * 512 + sched) << 20) - reps;
    // reference graphs are not kept: the copy's buffers end with this call
    struct DropGraph {
      SolverState* S;
      long long key;
      bool on;
      ~DropGraph() {
        auto it = on ? S->graphs.find(key) : S->graphs.end();
        if (it == S->graphs.end()) return;
        (void)hipStreamSynchronize(S->ctx->stream);
        (void)hipGraphExecDestroy(it->second);
        S->graphs.erase(it);
      }
    } drop{S, key, kid >= 3};
    run_graph(S, key, enqueue);   // instantiate and warm
    ctx->sync();
    hipEvent_t e0, e1;
    CAMFE_HIP(hipEventCreate(&e0));
    CAMFE_HIP(hipEventCreate(&e1));
    CAMFE_HIP(hipEventRecord(e0, ctx->stream));
    run_graph(S, key, enqueue);
    CAMFE_HIP(hipEventRecord(e1, ctx->stream));
    CAMFE_HIP(hipEventSynchronize(e1));
    float ms = 0;
    CAMFE_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (avg_ms) *avg_ms = ms / (reps * launches);
    if (bytes_per_launch) *bytes_per_launch = bytes / launches;
  });
}

}  // extern "C"

namespace camfe {
namespace {
// Time of one forward colour sweep (all colours, one right-hand side) at level
// G with tile v: reps sweeps captured once into a graph, replayed between two
// events after a warm replay; ms per sweep.  Overwrites the level's scratch.
double time_tile(SolverState* S, GLevel& G, int precision, int v, int reps) {
  camfe_ctx ctx = S->ctx;
  hipStream_t st = ctx->stream;
  const long long nk = (long long)G.n;
  hipLaunchKernelGGL((k_fill<double>), grid_for(nk, BLK), BLK, 0, st, G.b64.p, nk, 1.0);
  hipLaunchKernelGGL((k_fill<double>), grid_for(nk, BLK), BLK, 0, st, G.x64.p, nk, 0.0);
  hipLaunchKernelGGL((k_fill<float>), grid_for(nk, BLK), BLK, 0, st, G.b32.p, nk, 1.0f);
  hipLaunchKernelGGL((k_fill<float>), grid_for(nk, BLK), BLK, 0, st, G.x32.p, nk, 0.0f);
  const long long key = -(1LL << 40) - ((long long)G.d << 16) - ((long long)v << 8) - precision;
  auto enqueue = [&] {
    for (int r = 0; r < reps; ++r) {
      if (precision == 0) gs_sweep<double, 1>(ctx, G, G.b64.p, G.x64.p, true, G.invd64.p, 0, v);
      else gs_sweep<float, 1>(ctx, G, G.b32.p, G.x32.p, true, G.invd32.p, 0, v);
    }
  };
  struct Drop {
    SolverState* S;
    long long key;
    ~Drop() {
      auto it = S->graphs.find(key);
      if (it == S->graphs.end()) return;
      (void)hipStreamSynchronize(S->ctx->stream);
      (void)hipGraphExecDestroy(it->second);
      S->graphs.erase(it);
    }
  } drop{S, key};
  run_graph(S, key, enqueue);
  hipEvent_t e0, e1;
  CAMFE_HIP(hipEventCreate(&e0));
  CAMFE_HIP(hipEventCreate(&e1));
  CAMFE_HIP(hipEventRecord(e0, st));
  run_graph(S, key, enqueue);
  CAMFE_HIP(hipEventRecord(e1, st));
  CAMFE_HIP(hipEventSynchronize(e1));
  float ms = 0;
  CAMFE_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

// every level of S (from d_lo up): the fastest tile for the colour sweep,
// written into the levels and returned per level (index d - d_lo)
std::vector<int> autotune_levels(SolverState* S, int d_lo, int precision, int reps, std::vector<double>* best_ms) {
  std::vector<int> pick;
  for (int d = d_lo; d <= S->D; ++d) {
    GLevel& G = S->lev[d];
    int bv = 0;
    double bt = 0;
    for (int v = 0; v < NTILE; ++v) {
      const double ms = time_tile(S, G, precision, v, reps);
      if (v == 0 || ms < bt) { bt = ms; bv = v; }
    }
    G.tile = bv;
    pick.push_back(bv);
    if (best_ms) best_ms->push_back(bt);
  }
  S->drop_graphs();   // captured cycles hold the old tiles
  S->ctx->sync();
  return pick;
}
}  // namespace
}  // namespace camfe

extern "C" {

camfe_status camfe_system_autotune(camfe_sys s, double t, int precision, int reps, int32_t* tile, double* ms,
                                   int cap, int* nlevels) {
  return guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s && (precision == 0 || precision == 1) && reps > 0, CAMFE_EINVAL, "bad argument");
    camfe_hier h = s->h;
    const int nl = h->D - h->d0 + 1;
    if (nlevels) *nlevels = nl;
    if (cap == 0) return;
    CAMFE_REQUIRE(cap >= nl, CAMFE_ETOOSMALL, "capacity below the number of depths");
    h->ctx->use_device();
    SolverState* S = ensure_solver(s, t, s->solver ? s->solver->coarse_eps : DEFAULT_COARSE_EPS);
    std::vector<double> best;
    std::vector<int> pick = autotune_levels(S, h->d0, precision, reps, &best);
    s->tiles.assign(h->D + 1, 0);
    for (int i = 0; i < nl; ++i) {
      s->tiles[h->d0 + i] = pick[i];
      if (tile) tile[i] = pick[i];
      if (ms) ms[i] = best[i];
    }
  });
}

camfe_status camfe_block_damping(camfe_sys s, double t, double coarse_eps, double* omega, double* lambda, int cap,
                                 int* nlevels) {
  return guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s, CAMFE_EINVAL, "null system");
    camfe_hier h = s->h;
    CAMFE_REQUIRE(h->degree == 1, CAMFE_EINVAL, "the cell-block smoother is defined for degree 1");
    const int nl = h->D - h->d0 + 1;
    if (nlevels) *nlevels = nl;
    if (cap == 0) return;
    CAMFE_REQUIRE(cap >= nl, CAMFE_ETOOSMALL, "capacity below the number of depths");
    h->ctx->use_device();
    SolverState* S = ensure_solver(s, t, coarse_eps);
    if (!S->blocks_ready) {
      build_cell_blocks(s, S);
      estimate_block_damping(S);
    }
    for (int i = 0; i < nl; ++i) {
      if (omega) omega[i] = S->lev[h->d0 + i].block_omega;
      if (lambda) lambda[i] = S->lev[h->d0 + i].block_lambda;
    }
  });
}

camfe_status camfe_batch_autotune(camfe_batch b, int precision, int reps, int32_t* tile, double* ms, int cap,
                                  int* nlevels) {
  return guarded([&] {
    if (b) set_current_ctx(b->ctx);
    CAMFE_REQUIRE(b && (precision == 0 || precision == 1) && reps > 0, CAMFE_EINVAL, "bad argument");
    SolverState* S = b->S.get();
    const int nl = S->D + 1;
    if (nlevels) *nlevels = nl;
    if (cap == 0) return;
    CAMFE_REQUIRE(cap >= nl, CAMFE_ETOOSMALL, "capacity below the number of levels");
    b->ctx->use_device();
    std::vector<double> best;
    std::vector<int> pick = autotune_levels(S, 0, precision, reps, &best);
    for (int i = 0; i < nl; ++i) {
      if (tile) tile[i] = pick[i];
      if (ms) ms[i] = best[i];
    }
  });
}

camfe_status camfe_solve(camfe_sys s, const camfe_solve_opts* o, const double* b, int k, double* x,
                         camfe_solve_stats* stats) {
  camfe_status rc = CAMFE_OK;
  camfe_status g = guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s && o && b && x && k > 0, CAMFE_EINVAL, "bad argument");
    CAMFE_REQUIRE(o->precision == 0 || o->precision == 1, CAMFE_EINVAL, "precision must be 0 or 1");
    CAMFE_REQUIRE(o->method == 0 || o->method == 1, CAMFE_EINVAL, "method must be 0 or 1");
    CAMFE_REQUIRE(o->nu_pre >= 0 && o->nu_post >= 0 && o->max_iter >= 0, CAMFE_EINVAL, "bad sweep counts");
    CAMFE_REQUIRE(o->method != 0 || o->nu_pre == o->nu_post, CAMFE_EINVAL,
                  "CG needs a symmetric V-cycle: nu_pre must equal nu_post");
    CAMFE_REQUIRE(o->judge >= 0, CAMFE_EINVAL, "judge must be >= 0");
    CAMFE_REQUIRE(o->cycle >= 0 && o->cycle <= 2, CAMFE_EINVAL, "cycle must be 0, 1 (V) or 2 (W)");
    CAMFE_REQUIRE(o->nu_coarse >= 0 && o->nu_coarse < 64, CAMFE_EINVAL, "nu_coarse must lie in [0, 64)");
    camfe_hier h = s->h;
    camfe_ctx ctx = h->ctx;
    ctx->use_device();
    CAMFE_REQUIRE(o->smoother >= 0 && o->smoother <= 3, CAMFE_EINVAL, "smoother must be 0, 1, 2 or 3");
    CAMFE_REQUIRE(o->smoother != 1 || (o->omega > 0 && o->omega < 2), CAMFE_EINVAL, "omega must lie in (0, 2)");
    CAMFE_REQUIRE(o->smoother != 3 || (o->omega >= 0 && o->omega <= 1), CAMFE_EINVAL,
                  "block damping omega must lie in [0, 1] (0: automatic per depth)");
    CAMFE_REQUIRE(o->smoother != 3 || h->degree == 1, CAMFE_EINVAL, "the cell-block smoother is defined for degree 1");
    CAMFE_REQUIRE(o->smoother != 2 || s->model, CAMFE_ESTATE, "learned smoother requested but no model attached");
    SolverState* S = ensure_solver(s, o->t, o->coarse_eps);
    S->precision = o->precision;   // both precisions share one setup
    // the cycle shape holds for this call only (other users of the state,
    // such as smoother training, take V-cycles)
    struct GammaScope {
      SolverState* S;
      ~GammaScope() { S->gamma = 1; S->nu_coarse = 0; }
    } gamma_scope{S};
    S->gamma = o->cycle == 2 ? 2 : 1;
    S->nu_coarse = o->nu_coarse;
    const bool stale = o->smoother != S->wkind || (o->smoother == 1 && o->omega != S->omega) ||
                       (o->smoother == 2 && s->model != S->model);
    if (o->smoother == 3) {
      if (!S->blocks_ready) {
        build_cell_blocks(s, S);
        estimate_block_damping(S);
      }
      if (S->block_colour_min != s->block_colour_min) {   // captured cycles hold the launch pattern
        S->drop_graphs();
        S->block_colour_min = s->block_colour_min;
      }
      if (S->block_omega != o->omega) {   // captured cycles hold the damping as a kernel argument
        S->drop_graphs();
        S->block_omega = o->omega;
      }
    } else if (o->smoother != 0 && stale) {
      set_smoother_weights(s, S, o->smoother, o->omega, o->smoother == 2 ? s->model : nullptr);
    }
    S->smoother = o->smoother;
    const size_t n = S->lev[h->D].n;
    DArr<double> db(n * (size_t)k), dx(n * (size_t)k);
    copy_in(ctx, db.p, b, db.n);
    if (o->x0_given) copy_in(ctx, dx.p, (const double*)x, dx.n);
    auto t0 = std::chrono::steady_clock::now();
    auto run_all = [&](const camfe_solve_opts& oo) {
      SolveResult tot;
      for (int c0 = 0; c0 < k; c0 += KMAXS) {
        const int kb = std::min(KMAXS, k - c0);
        SolveResult r;
        switch (kb) {
          case 1: r = solve_block<1>(s, S, oo, db.p, dx.p, k, c0); break;
          case 2: r = solve_block<2>(s, S, oo, db.p, dx.p, k, c0); break;
          case 3: r = solve_block<3>(s, S, oo, db.p, dx.p, k, c0); break;
          default: r = solve_block<4>(s, S, oo, db.p, dx.p, k, c0); break;
        }
        tot.it = std::max(tot.it, r.it);
        tot.cycles += r.cycles;
        tot.judged_gs = tot.judged_gs || r.judged_gs;
        for (int j = 0; j < 2; ++j) tot.judge_rel[j] = std::max(tot.judge_rel[j], r.judge_rel[j]);
        if (!(r.rel <= tot.rel)) tot.rel = r.rel;
      }
      return tot;
    };
    SolveResult tot = run_all(*o);
    int fell_back = tot.judged_gs ? 2 : 0;
    // (stationary cycles of the cell-block smoother, a contraction, are
    // returned as asked; under CG a failed block solve is redone too)
    if (o->smoother != 0 && !(o->smoother == 3 && o->method == 1) && !tot.judged_gs && !(tot.rel <= o->rtol)) {
      // the Jacobi smoother failed (diverged or stalled): Gauss-Seidel redoes the solve
      camfe_solve_opts go = *o;
      go.smoother = 0;
      S->smoother = 0;
      if (o->x0_given) copy_in(ctx, dx.p, (const double*)x, dx.n);
      SolveResult t2 = run_all(go);
      t2.it += tot.it;
      t2.cycles += tot.cycles;
      t2.judge_rel[0] = tot.judge_rel[0];
      t2.judge_rel[1] = tot.judge_rel[1];
      tot = t2;
      fell_back = 1;
    }
    ctx->sync();
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    copy_out(ctx, x, dx.p, dx.n);
    ctx->sync();
    if (stats) {
      stats->iterations = tot.it;
      stats->fell_back = fell_back;
      stats->cycles = tot.cycles;
      stats->eps_regularised = S->direct ? 1 : 0;
      stats->rel_residual = tot.rel;
      stats->seconds = secs;
      stats->setup_seconds = S->setup_seconds;
      stats->judge_rel[0] = tot.judge_rel[0];
      stats->judge_rel[1] = tot.judge_rel[1];
    }
    if (!(tot.rel <= o->rtol)) rc = CAMFE_ENOCONV;
  });
  if (g != CAMFE_OK) return g;
  if (rc != CAMFE_OK) set_last_error("solver stopped above rtol");
  return rc;
}

camfe_status camfe_batch_create(camfe_ctx ctx, camfe_sys const* systems, int nsys, double t, double coarse_eps,
                                camfe_batch* out) {
  return guarded([&] {
    if (ctx) set_current_ctx(ctx);
    CAMFE_REQUIRE(ctx && systems && nsys >= 1 && out, CAMFE_EINVAL, "bad argument");
    ctx->use_device();
    auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<camfe_batch_s> B(new camfe_batch_s());
    B->ctx = ctx;
    B->t = t;
    B->coarse_eps = coarse_eps;
    std::vector<SolverState*> ms;
    for (int i = 0; i < nsys; ++i) {
      camfe_sys s = systems[i];
      CAMFE_REQUIRE(s && s->h->ctx == ctx, CAMFE_EINVAL, "systems must belong to the context");
      CAMFE_REQUIRE(s->h->degree == systems[0]->h->degree, CAMFE_EINVAL, "systems must share the degree");
      ms.push_back(ensure_solver(s, t, coarse_eps));
    }
    build_batch(B.get(), ms);
    B->S->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = B.release();
  });
}

camfe_status camfe_batch_info(camfe_batch b, int* levels, int64_t* rows) {
  return guarded([&] {
    if (b) set_current_ctx(b->ctx);
    CAMFE_REQUIRE(b, CAMFE_EINVAL, "null batch");
    if (levels) *levels = b->S->D + 1;
    if (rows) *rows = (int64_t)b->S->lev[b->S->D].n;
  });
}

camfe_status camfe_batch_solve(camfe_batch bt, const camfe_solve_opts* o, const double* const* b, const int* k,
                               double* const* x, camfe_solve_stats* stats) {
  camfe_status rc = CAMFE_OK;
  camfe_status g = guarded([&] {
    if (bt) set_current_ctx(bt->ctx);
    CAMFE_REQUIRE(bt && o && b && k && x, CAMFE_EINVAL, "bad argument");
    CAMFE_REQUIRE(o->t == bt->t && o->coarse_eps == bt->coarse_eps, CAMFE_EINVAL,
                  "t and coarse_eps must be those the batch was built for");
    CAMFE_REQUIRE(o->method == 0 && o->smoother == 0, CAMFE_EINVAL,
                  "batched solves use CG with the Gauss-Seidel V-cycle");
    CAMFE_REQUIRE(o->precision == 0 || o->precision == 1, CAMFE_EINVAL, "precision must be 0 or 1");
    CAMFE_REQUIRE(o->cycle == 0 || o->cycle == 1, CAMFE_EINVAL, "the batched solve takes V-cycles (cycle 0 or 1)");
    CAMFE_REQUIRE(o->nu_pre >= 0 && o->nu_post >= 0 && o->max_iter >= 0 && o->nu_pre == o->nu_post, CAMFE_EINVAL,
                  "bad sweep counts (CG needs nu_pre == nu_post)");
    CAMFE_REQUIRE(o->nu_coarse >= 0 && o->nu_coarse < 64, CAMFE_EINVAL, "nu_coarse must lie in [0, 64)");
    SolverState* S = bt->S.get();
    camfe_ctx ctx = bt->ctx;
    ctx->use_device();
    S->precision = o->precision;
    struct CoarseScope {   // the batch's later calls start from the default again
      SolverState* S;
      ~CoarseScope() { S->nu_coarse = 0; }
    } coarse_scope{S};
    S->nu_coarse = o->nu_coarse;
    const int nm = S->nmesh;
    std::vector<int> kk(k, k + nm);
    int kmax = 0;
    for (int m = 0; m < nm; ++m) {
      CAMFE_REQUIRE(kk[m] >= 1 && b[m] && x[m], CAMFE_EINVAL, "every mesh needs k >= 1, b and x");
      kmax = std::max(kmax, kk[m]);
    }
    std::vector<DArr<double>> db(nm), dx(nm);
    for (int m = 0; m < nm; ++m) {
      const size_t nn = bt->mem[m].n * (size_t)kk[m];
      db[m].alloc(nn);
      dx[m].alloc(nn);
      copy_in(ctx, db[m].p, b[m], nn);
      if (o->x0_given) copy_in(ctx, dx[m].p, (const double*)x[m], nn);
    }
    auto t0 = std::chrono::steady_clock::now();
    std::vector<SolveResult> res(nm);
    for (int c0 = 0; c0 < kmax; c0 += KMAXS) {
      switch (std::min(KMAXS, kmax - c0)) {
        case 1: batch_solve_block<1>(bt, *o, db, dx, kk, c0, res); break;
        case 2: batch_solve_block<2>(bt, *o, db, dx, kk, c0, res); break;
        case 3: batch_solve_block<3>(bt, *o, db, dx, kk, c0, res); break;
        default: batch_solve_block<4>(bt, *o, db, dx, kk, c0, res); break;
      }
    }
    ctx->sync();
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int m = 0; m < nm; ++m) {
      copy_out(ctx, x[m], dx[m].p, dx[m].n);
      if (stats) {
        stats[m].iterations = res[m].it;
        stats[m].fell_back = 0;
        stats[m].cycles = res[m].cycles;
        stats[m].eps_regularised = 0;
        stats[m].rel_residual = res[m].rel;
        stats[m].seconds = secs;
        stats[m].setup_seconds = S->setup_seconds;
        stats[m].judge_rel[0] = stats[m].judge_rel[1] = 0.0;
      }
      if (!(res[m].rel <= o->rtol)) rc = CAMFE_ENOCONV;
    }
    ctx->sync();
  });
  if (g != CAMFE_OK) return g;
  if (rc != CAMFE_OK) set_last_error("solver stopped above rtol for at least one mesh");
  return rc;
}

void camfe_batch_destroy(camfe_batch b) {
  if (!b) return;
  (void)hipSetDevice(b->ctx->device);
  (void)hipStreamSynchronize(b->ctx->stream);
  delete b;
}

}  // extern "C"

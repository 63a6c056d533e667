// Finite-element assembly on the GPU (Section 3.1 Eq. 2; Section 5.1):
//   M_ij = int b_i b_j,  L_ij = int <grad_M b_i, grad_M b_j>,  b_i = int f b_i
// by exact quadrature over each triangle fragment clipped to a cell.
//
// Work unit: one wavefront takes a chunk of (cell, triangle) pairs of one
// cell.  Per pair the triangle is clipped against the six cell planes with
// one polygon vertex per lane (ballots give each lane its output slot), the
// polygon is fanned from its first vertex and every sub-triangle gets a
// collapsed Gauss-Legendre rule.  Eight (degree 1) or four (degree 2)
// quadrature points at a time, the 64 lanes evaluate (function slot, point)
// pairs and the FP64 matrix cores contract them: M_e += Phi W Phi^T and
// L_e += sum_axes G W G^T with v_mfma_f64_16x16x4 (operands: lane l holds
// row/column l % 16 at k = l / 16; result: lane l, register r holds row
// l / 16 + 4 r, column l % 16).  Consecutive pairs whose eight (27) rows
// coincide share one element block, which is scattered with atomics when the
// rows change.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace camfe {
namespace {

constexpr int BLK = 256;
constexpr int CHUNK = 32;     // pairs per work item
constexpr int KMAX = 4;       // right-hand-side columns per assembly pass

typedef double d4 __attribute__((ext_vector_type(4)));

__constant__ double c_glx[2][8];   // Gauss-Legendre nodes on [0,1]: [0] 4-point, [1] 7-point
__constant__ double c_glw[2][8];

// Gauss-Legendre rule on [0,1] (Newton iteration on the Legendre recurrence)
void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 60; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (p0 - z * p1) / (1.0 - z * z);
      double step = p1 / dp;
      z -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    x[i] = 0.5 * (1.0 + z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
  }
}

void upload_rules() {
  static bool done = false;
  if (done) return;
  double x[2][8] = {{0}}, w[2][8] = {{0}};
  gauss_legendre(4, x[0], w[0]);
  gauss_legendre(7, x[1], w[1]);
  CAMFE_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_glx), x, sizeof(x)));
  CAMFE_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_glw), w, sizeof(w)));
  done = true;
}

__device__ inline long long lower_bound_u64(const u64* a, long long lo, long long hi, u64 key) {
  while (lo < hi) {
    long long mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}
__device__ inline int find_col(const int* col, int lo, int hi, int c) {
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (col[mid] < c) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// 1D basis piece j of the degree on one cell, local coordinate l in [0,1]
template <int DEG>
__device__ inline void basis1d(int j, double l, double& b, double& db) {
  if (DEG == 1) {
    b = j ? l : 1.0 - l;
    db = j ? 1.0 : -1.0;
  } else {
    if (j == 0) { b = 0.5 * (1.0 - l) * (1.0 - l); db = -(1.0 - l); }
    else if (j == 1) { b = 0.75 - (l - 0.5) * (l - 0.5); db = -2.0 * (l - 0.5); }
    else { b = 0.5 * l * l; db = l; }
  }
}

// --------------------------------------------------------- work chunks
__global__ void k_cell_heads(const u64* pairs, long long n, int* flag) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n) flag[i] = (i == 0 || (pairs[i] >> TRI_BITS) != (pairs[i - 1] >> TRI_BITS)) ? 1 : 0;
}
__global__ void k_cell_starts(const int* flag, const int* pos, long long n, int* start) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n && flag[i]) start[pos[i]] = (int)i;
}
__global__ void k_chunk_count(const int* start, int ncell, long long npairs, int* cnt) {
  long long c = blockIdx.x * (long long)BLK + threadIdx.x;
  if (c >= ncell) return;
  long long e = (c + 1 < ncell) ? start[c + 1] : npairs;
  cnt[c] = (int)((e - start[c] + CHUNK - 1) / CHUNK);
}
__global__ void k_chunk_fill(const int* start, const int* coff, int ncell, long long npairs, int2* chunks) {
  long long c = blockIdx.x * (long long)BLK + threadIdx.x;
  if (c >= ncell) return;
  long long b = start[c], e = (c + 1 < ncell) ? start[c + 1] : npairs;
  int o = coff[c];
  for (long long p = b; p < e; p += CHUNK) chunks[o++] = make_int2((int)p, (int)min((long long)CHUNK, e - p));
}

// ------------------------------------------------- superset row structure
// Row (k, i) may couple with every function at the supports k + delta.  The
// functions of support g are cfirst[g] .. cfirst[g + 1] - 1, ascending in g,
// so emitting the neighbouring supports in ascending order writes a sorted row
// (the supports, at most 27 or 125, are sorted instead of the row's entries:
// coarse split depths have rows of thousands).
template <int DEG, bool FILL>
__global__ void k_struct(const u64* fkey, long long nf, const u64* ckey, long long ncorn, const int* cfirst,
                         int* cnt, const int* ptr, int* col) {
  long long f = blockIdx.x * (long long)BLK + threadIdx.x;
  if (f >= nf) return;
  constexpr int R = DEG == 1 ? 1 : 2;
  constexpr int NS = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
  long long c[3];
  demorton(fkey[f], c);
  int gs[FILL ? NS : 1];
  int ng = 0, m = 0;
  for (int dz = -R; dz <= R; ++dz)
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        long long x = c[0] + dx, y = c[1] + dy, z = c[2] + dz;
        if (x < 0 || y < 0 || z < 0) continue;
        u64 k = morton((u64)x, (u64)y, (u64)z);
        long long g = lower_bound_u64(ckey, 0, ncorn, k);
        if (g < ncorn && ckey[g] == k) {
          if (FILL) {
            int p = ng++;
            while (p > 0 && gs[p - 1] > (int)g) { gs[p] = gs[p - 1]; --p; }
            gs[p] = (int)g;
          } else {
            m += cfirst[g + 1] - cfirst[g];
          }
        }
      }
  if (!FILL) {
    cnt[f] = m;
    return;
  }
  const int o = ptr[f];
  for (int i = 0; i < ng; ++i)
    for (int q = cfirst[gs[i]]; q < cfirst[gs[i] + 1]; ++q) col[o + m++] = q;
}

// ------------------------------------------------------------ assembly
struct AsmArgs {
  const u64* pairs;
  const int* pair_rows;
  const int2* chunks;
  int nchunk;
  const double* U;
  const int* F;
  const double* nrm;
  double sc;          // 2^(d - D)
  double hd2;         // (world cell size at depth d)^2
  const double* tri_w;
  const int* ptr;
  const int* col;
  double* M;          // nullable
  double* L;          // nullable
  const double* fv;   // per-vertex values, nv x k column-major (nullable)
  long long nv;
  int k;              // columns in this pass (<= KMAX)
  double* rhs;        // n x ldr column-major (column offset applied by caller)
  long long ldr;
  int grad_rhs;       // rhs receives int <grad f, grad b_i> instead of int f b_i
  unsigned long long* npts;   // nullable: quadrature points processed (measurement)
  double* pcache;     // degree 1, mass only: each pair's unweighted 8 x 8 block (36 packed entries)
};

// position of (r, c), r <= c, in a packed upper triangle of 8 x 8
__host__ __device__ constexpr int upk8(int r, int c) { return r * (17 - r) / 2 + c - r; }

// CACHE (degree 1, mass only): every pair's unweighted element block also
// goes to a.pcache, so that later re-weightings skip clipping and quadrature.
// RHS: the launch fills right-hand sides (a.rhs) instead of matrices (a.M),
// fixed at compile time so that each variant holds only its own registers.
// The kernel is bound by the latency of its per-pair chain (triangle loads,
// clipping rounds, LDS, atomics), so occupancy matters: the degree-1 matrix
// variant is held to 96 registers (5 waves per SIMD, a few spilled values;
// at 80 and 6 waves the spills cost twice the time), the others to their
// spill-free counts (4 waves for degree-1 loads, 2-3 for degree 2).
template <int DEG, bool CACHE = false, bool RHS = false>
__global__ __launch_bounds__(64, DEG == 1 ? (RHS ? 4 : 5) : 2) void k_assemble(AsmArgs a) {
  constexpr int W = DEG == 1 ? 2 : 3;
  constexpr int NB = W * W * W;
  constexpr int T = DEG == 1 ? 1 : 2;       // 16-row tiles per block
  constexpr int NQ = DEG == 1 ? 4 : 7;
  constexpr int Q = NQ * NQ;
  constexpr int RI = DEG == 1 ? 0 : 1;
  // quadrature points per matrix-core step: degree 1 fills the 16 rows with
  // its 8 functions at two sets of 4 points (rows and columns f + 8 h hold
  // function f at point set h; the element block is the sum of the two
  // diagonal 8x8 blocks of the product), degree 2 its 27 functions at 4 points
  constexpr int PG = DEG == 1 ? 8 : 4;
  constexpr int PMAX = 16;   // clipped polygon vertices (9 in exact arithmetic)
  __shared__ double poly[PMAX][6];
  __shared__ double sarea[PMAX];
  const int lane = threadIdx.x;
  const int slot = lane & 15;
  const int pt = lane >> 4;
  const u64 lt_mask = (1ULL << lane) - 1ULL;
  const bool want_mat = !RHS && a.M != nullptr;
  const bool want_rhs = RHS && a.rhs != nullptr;
  unsigned long long wave_pts = 0;   // quadrature points of this wavefront (measurement)
  static_assert(!CACHE || DEG == 1, "the block cache holds degree-1 blocks");
  d4 accP = (d4){0, 0, 0, 0};        // CACHE: this pair's block

  for (int ch = blockIdx.x; ch < a.nchunk; ch += gridDim.x) {
    const int2 cd = a.chunks[ch];
    d4 accM[T * (T + 1) / 2], accL[T * (T + 1) / 2];
#pragma unroll
    for (int i = 0; i < T * (T + 1) / 2; ++i) { accM[i] = (d4){0, 0, 0, 0}; accL[i] = (d4){0, 0, 0, 0}; }
    double accB[T][KMAX];
#pragma unroll
    for (int i = 0; i < T; ++i)
#pragma unroll
      for (int c = 0; c < KMAX; ++c) accB[i][c] = 0.0;
    int cur_row = -1;   // row of local function `lane` (lanes < NB)
    bool have = false;

    for (int pi = 0; pi <= cd.y; ++pi) {
      // rows of the next pair (or a sentinel after the last pair)
      int new_row = -2;
      if (pi < cd.y && lane < NB) new_row = a.pair_rows[(long long)(cd.x + pi) * NB + lane];
      const bool changed = __any(lane < NB && new_row != cur_row);
      if (have && (changed || pi == cd.y)) {
        // ---- scatter the element block
        if (want_mat && DEG == 1) {
          // lane (pt, slot < 8) holds rows pt and pt + 4 of column slot of the
          // first diagonal block; the lane 8 above it, the same entries of the second
          const double m0 = accM[0][0] + __shfl(accM[0][2], lane + 8);
          const double m1 = accM[0][1] + __shfl(accM[0][3], lane + 8);
          const double l0 = accL[0][0] + __shfl(accL[0][2], lane + 8);
          const double l1 = accL[0][1] + __shfl(accL[0][3], lane + 8);
          const int colrow = __shfl(cur_row, slot & 7);
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            const int rowrow = __shfl(cur_row, pt + 4 * r);
            if (slot < 8) {
              const int e1 = a.ptr[rowrow + 1];
              const int p = find_col(a.col, a.ptr[rowrow], e1, colrow);
              if (p < e1 && a.col[p] == colrow) {
                atomicAdd(a.M + p, r == 0 ? m0 : m1);
                if (a.L) atomicAdd(a.L + p, r == 0 ? l0 : l1);
              }
            }
          }
        } else if (want_mat) {
          int ti = 0;
#pragma unroll
          for (int I = 0; I < T; ++I)
#pragma unroll
            for (int J = I; J < T; ++J, ++ti) {
              const int b = 16 * J + slot;
              const int colrow = __shfl(cur_row, b < NB ? b : 0);
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int aa = 16 * I + pt + 4 * r;   // row of accumulator register r
                const int rowrow = __shfl(cur_row, aa < NB ? aa : 0);
                if (aa < NB && b < NB) {
                  const double mv = accM[ti][r], lv = accL[ti][r];
                  const int e1 = a.ptr[rowrow + 1];
                  int p = find_col(a.col, a.ptr[rowrow], e1, colrow);
                  if (p < e1 && a.col[p] == colrow) {
                    atomicAdd(a.M + p, mv);
                    if (a.L) atomicAdd(a.L + p, lv);
                  }
                  if (I != J) {
                    const int e2 = a.ptr[colrow + 1];
                    int p2 = find_col(a.col, a.ptr[colrow], e2, rowrow);
                    if (p2 < e2 && a.col[p2] == rowrow) {
                      atomicAdd(a.M + p2, mv);
                      if (a.L) atomicAdd(a.L + p2, lv);
                    }
                  }
                }
              }
            }
        }
        if (want_rhs) {
#pragma unroll
          for (int i = 0; i < T; ++i)
#pragma unroll
            for (int c = 0; c < KMAX; ++c) {
              if (c >= a.k) continue;
              double v = accB[i][c];
              if (DEG == 1) v += __shfl_xor(v, 8);
              v += __shfl_xor(v, 16);
              v += __shfl_xor(v, 32);
              accB[i][c] = v;
            }
#pragma unroll
          for (int i = 0; i < T; ++i) {
            const int j = 16 * i + slot;   // (degree 1: slots 8-15 repeat functions 0-7)
            const int rr = __shfl(cur_row, j < NB ? j : 0);
            if (pt == 0 && j < NB)
              for (int c = 0; c < a.k; ++c) atomicAdd(a.rhs + (long long)c * a.ldr + rr, accB[i][c]);
          }
        }
#pragma unroll
        for (int i = 0; i < T * (T + 1) / 2; ++i) { accM[i] = (d4){0, 0, 0, 0}; accL[i] = (d4){0, 0, 0, 0}; }
#pragma unroll
        for (int i = 0; i < T; ++i)
#pragma unroll
          for (int c = 0; c < KMAX; ++c) accB[i][c] = 0.0;
        have = false;
      }
      if (pi == cd.y) break;
      cur_row = new_row;
      have = true;

      // ---- clip the triangle to the closed cell (one polygon vertex per lane)
      const u64 key = a.pairs[cd.x + pi];
      const int t = (int)(key & TRI_MASK);
      long long cc[3];
      demorton(key >> TRI_BITS, cc);
      double P[6] = {0, 0, 0, 0, 0, 0};
      if (lane < 3) {
        const int v = a.F[3 * t + lane];
        for (int q = 0; q < 3; ++q) P[q] = a.U[3 * (long long)v + q] * a.sc;
        P[3] = lane == 0 ? 1.0 : 0.0;
        P[4] = lane == 1 ? 1.0 : 0.0;
        P[5] = lane == 2 ? 1.0 : 0.0;
      }
      int n = 3;
      // a triangle inside the closed cell (the common case at fine depths,
      // where triangles are smaller than cells) is its own clipped polygon:
      // every plane would keep all three vertices in order, so the clipping
      // is skipped with the same result
      bool inside = true;
      if (lane < 3)
#pragma unroll
        for (int q = 0; q < 3; ++q) inside = inside && P[q] >= (double)cc[q] && P[q] <= (double)cc[q] + 1.0;
      const bool all_in = __all(inside);
      if (all_in) {
        if (lane < 3)
#pragma unroll
          for (int q = 0; q < 6; ++q) poly[lane][q] = P[q];
        __syncthreads();
      }
      for (int pl = 0; pl < 6 && n >= 3 && !all_in; ++pl) {
        const int ax = pl >> 1;
        const bool ge = (pl & 1) == 0;
        const double v = (double)cc[ax] + (ge ? 0.0 : 1.0);
        const int src = lane + 1 < n ? lane + 1 : 0;
        double Qv[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) Qv[q] = __shfl(P[q], src);
        const bool act = lane < n;
        const bool inP = act && (ge ? P[ax] >= v : P[ax] <= v);
        const bool inQ = act && (ge ? Qv[ax] >= v : Qv[ax] <= v);
        const bool cross = act && (inP != inQ);
        const u64 bP = __ballot(inP), bC = __ballot(cross);
        const int pos = __popcll(bP & lt_mask) + __popcll(bC & lt_mask);
        const int nn = __popcll(bP) + __popcll(bC);
        if (inP && pos < PMAX)
#pragma unroll
          for (int q = 0; q < 6; ++q) poly[pos][q] = P[q];
        if (cross) {
          const double lam = (v - P[ax]) / (Qv[ax] - P[ax]);
          double R[6];
#pragma unroll
          for (int q = 0; q < 6; ++q) R[q] = P[q] + lam * (Qv[q] - P[q]);
          R[ax] = v;
          const int o = pos + (inP ? 1 : 0);
          if (o < PMAX)
#pragma unroll
            for (int q = 0; q < 6; ++q) poly[o][q] = R[q];
        }
        __syncthreads();
        n = nn < PMAX ? nn : PMAX;
        if (lane < n)
#pragma unroll
          for (int q = 0; q < 6; ++q) P[q] = poly[lane][q];
        __syncthreads();
      }
      if (n < 3) continue;
      // the final polygon is in poly[0..n) (written by the last plane)
      const double nx = a.nrm[3 * t], ny = a.nrm[3 * t + 1], nz = a.nrm[3 * t + 2];
      const double tw = a.tri_w ? a.tri_w[t] : 1.0;
      double fvv[3][KMAX];
      if (want_rhs) {
        for (int m = 0; m < 3; ++m) {
          const int v = a.F[3 * t + m];
          for (int c = 0; c < KMAX; ++c) fvv[m][c] = c < a.k ? a.fv[(long long)c * a.nv + v] : 0.0;
        }
        if (a.grad_rhs) {
          // fvv becomes the gradient of f on the triangle, in depth-d cell
          // units: (f1 - f0) (e2 x n) / |n|^2 + (f2 - f0) (n x e1) / |n|^2
          // with e1, e2 the edges from corner 0 and n = e1 x e2 (zero on a
          // triangle without area)
          double q0[3], e1[3], e2[3];
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            q0[q] = a.U[3 * (long long)a.F[3 * t] + q] * a.sc;
            e1[q] = a.U[3 * (long long)a.F[3 * t + 1] + q] * a.sc - q0[q];
            e2[q] = a.U[3 * (long long)a.F[3 * t + 2] + q] * a.sc - q0[q];
          }
          const double n0 = e1[1] * e2[2] - e1[2] * e2[1];
          const double n1 = e1[2] * e2[0] - e1[0] * e2[2];
          const double n2 = e1[0] * e2[1] - e1[1] * e2[0];
          const double nn = n0 * n0 + n1 * n1 + n2 * n2;
          const double inv = nn > 0.0 ? 1.0 / nn : 0.0;
          const double g1[3] = {(e2[1] * n2 - e2[2] * n1) * inv, (e2[2] * n0 - e2[0] * n2) * inv,
                                (e2[0] * n1 - e2[1] * n0) * inv};
          const double g2[3] = {(n1 * e1[2] - n2 * e1[1]) * inv, (n2 * e1[0] - n0 * e1[2]) * inv,
                                (n0 * e1[1] - n1 * e1[0]) * inv};
#pragma unroll
          for (int c = 0; c < KMAX; ++c) {
            const double d1 = fvv[1][c] - fvv[0][c], d2 = fvv[2][c] - fvv[0][c];
#pragma unroll
            for (int q = 0; q < 3; ++q) fvv[q][c] = d1 * g1[q] + d2 * g2[q];
          }
        }
      }
      const int npts = (n - 2) * Q;
      wave_pts += (unsigned long long)npts;
      // area of each fan sub-triangle, once (lane s - 1 takes sub-triangle s)
      if (lane < n - 2) {
        const double* A0 = poly[0];
        const double* A1 = poly[lane + 1];
        const double* A2 = poly[lane + 2];
        double e1[3], e2[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) { e1[q] = A1[q] - A0[q]; e2[q] = A2[q] - A0[q]; }
        const double cx = e1[1] * e2[2] - e1[2] * e2[1];
        const double cy = e1[2] * e2[0] - e1[0] * e2[2];
        const double cz = e1[0] * e2[1] - e1[1] * e2[0];
        sarea[lane] = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
      }
      __syncthreads();
      for (int p0 = 0; p0 < npts; p0 += PG) {
        const int p = p0 + pt + (DEG == 1 ? 4 * (slot >> 3) : 0);
        double val[T], gx[T], gy[T], gz[T];
        double wl = 0.0, wm = 0.0, wmu = 0.0, bar[3] = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < T; ++i) { val[i] = gx[i] = gy[i] = gz[i] = 0.0; }
        if (p < npts) {
          const int s = p / Q + 1;
          const int qi = p - (s - 1) * Q;
          const int iu = qi / NQ, iv = qi - iu * NQ;
          const double* A0 = poly[0];
          const double* A1 = poly[s];
          const double* A2 = poly[s + 1];
          double e1[3], e2[3];
#pragma unroll
          for (int q = 0; q < 3; ++q) { e1[q] = A1[q] - A0[q]; e2[q] = A2[q] - A0[q]; }
          const double area = sarea[s - 1];
          const double u = c_glx[RI][iu], wu = c_glw[RI][iu];
          const double xi = u, eta = (1.0 - u) * c_glx[RI][iv];
          wl = 2.0 * area * wu * c_glw[RI][iv] * (1.0 - u);
          wmu = wl * a.hd2;
          wm = wmu * tw;
          double lc[3];
#pragma unroll
          for (int q = 0; q < 3; ++q) lc[q] = A0[q] + xi * e1[q] + eta * e2[q] - (double)cc[q];
          if (want_rhs && !a.grad_rhs)   // barycentric coordinates: the value load only
#pragma unroll
            for (int q = 0; q < 3; ++q) bar[q] = A0[3 + q] + xi * (A1[3 + q] - A0[3 + q]) + eta * (A2[3 + q] - A0[3 + q]);
#pragma unroll
          for (int i = 0; i < T; ++i) {
            const int j = DEG == 1 ? (slot & 7) : 16 * i + slot;
            if (j < NB) {
              const int jx = j % W, jy = (j / W) % W, jz = j / (W * W);
              double bx, dbx, by, dby, bz, dbz;
              basis1d<DEG>(jx, lc[0], bx, dbx);
              basis1d<DEG>(jy, lc[1], by, dby);
              basis1d<DEG>(jz, lc[2], bz, dbz);
              const double g0 = dbx * by * bz, g1 = bx * dby * bz, g2 = bx * by * dbz;
              const double gn = g0 * nx + g1 * ny + g2 * nz;
              val[i] = bx * by * bz;
              gx[i] = g0 - gn * nx;
              gy[i] = g1 - gn * ny;
              gz[i] = g2 - gn * nz;
            }
          }
        }
        if (CACHE) {
          accP = __builtin_amdgcn_mfma_f64_16x16x4f64(val[0], wmu * val[0], accP, 0, 0, 0);
        } else if (want_mat) {
          int ti = 0;
#pragma unroll
          for (int I = 0; I < T; ++I)
#pragma unroll
            for (int J = I; J < T; ++J, ++ti) {
              accM[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(val[I], wm * val[J], accM[ti], 0, 0, 0);
              accL[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(gx[I], wl * gx[J], accL[ti], 0, 0, 0);
              accL[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(gy[I], wl * gy[J], accL[ti], 0, 0, 0);
              accL[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(gz[I], wl * gz[J], accL[ti], 0, 0, 0);
            }
        }
        if (want_rhs && a.grad_rhs) {
          // surface gradients in cell units with the cell-unit weight: the
          // Dirichlet form is invariant under the scaling
#pragma unroll
          for (int c = 0; c < KMAX; ++c)
            if (c < a.k)   // (columns past k stay zero)
#pragma unroll
              for (int i = 0; i < T; ++i)
                accB[i][c] += wl * (gx[i] * fvv[0][c] + gy[i] * fvv[1][c] + gz[i] * fvv[2][c]);
        } else if (want_rhs) {
#pragma unroll
          for (int c = 0; c < KMAX; ++c) {
            if (c >= a.k) continue;
            const double fx = bar[0] * fvv[0][c] + bar[1] * fvv[1][c] + bar[2] * fvv[2][c];
#pragma unroll
            for (int i = 0; i < T; ++i) accB[i][c] += wm * val[i] * fx;
          }
        }
      }
      if (CACHE) {
        // the pair's block (sum of the two diagonal 8 x 8 blocks, as in the
        // scatter), stored as its upper triangle; then weighted into the run's block
        const double e0 = accP[0] + __shfl(accP[2], lane + 8);
        const double e1 = accP[1] + __shfl(accP[3], lane + 8);
        const long long base = (long long)(cd.x + pi) * 36;
        if (slot < 8 && pt <= slot) a.pcache[base + upk8(pt, slot)] = e0;
        if (slot < 8 && pt + 4 <= slot) a.pcache[base + upk8(pt + 4, slot)] = e1;
#pragma unroll
        for (int q = 0; q < 4; ++q) accM[0][q] += tw * accP[q];
        accP = (d4){0, 0, 0, 0};
      }
    }
  }
  if (a.npts && lane == 0 && wave_pts) atomicAdd(a.npts, wave_pts);
}

// M from the cached unweighted blocks of every pair: one wavefront per chunk
// of pairs, lane (r, c) = entry (r, c) of the element block; blocks of
// consecutive pairs with the same eight rows are summed, each weighted by its
// triangle's weight, and scattered when the rows change
__global__ __launch_bounds__(64) void k_mass_cached(const int2* chunks, int nchunk, const u64* pairs,
                                                    const int* pair_rows, const double* pcache, const double* tri_w,
                                                    const int* ptr, const int* col, double* M) {
  const int lane = threadIdx.x;
  const int r = lane >> 3, c = lane & 7;
  const int e = upk8(min(r, c), max(r, c));
  for (int ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    const int2 cd = chunks[ch];
    int cur_row = -1;
    bool have = false;
    double acc = 0.0;
    for (int pi = 0; pi <= cd.y; ++pi) {
      int new_row = -2;
      if (pi < cd.y && lane < 8) new_row = pair_rows[(long long)(cd.x + pi) * 8 + lane];
      const bool changed = __any(lane < 8 && new_row != cur_row);
      if (have && (changed || pi == cd.y)) {
        const int rowrow = __shfl(cur_row, r), colrow = __shfl(cur_row, c);
        const int e1 = ptr[rowrow + 1];
        const int p = find_col(col, ptr[rowrow], e1, colrow);
        if (p < e1 && col[p] == colrow) atomicAdd(M + p, acc);
        acc = 0.0;
        have = false;
      }
      if (pi == cd.y) break;
      cur_row = new_row;
      have = true;
      const long long q = cd.x + pi;
      const double w = tri_w ? tri_w[(int)(pairs[q] & TRI_MASK)] : 1.0;
      acc += w * pcache[q * 36 + e];
    }
  }
}

// ---------------------------------------------------------- compaction
__global__ void k_nz_count(const int* ptr, const double* M, const double* L, long long n, int* cnt) {
  long long r = blockIdx.x * (long long)BLK + threadIdx.x;
  if (r >= n) return;
  int c = 0;
  for (int e = ptr[r]; e < ptr[r + 1]; ++e) c += (M[e] != 0.0 || L[e] != 0.0) ? 1 : 0;
  cnt[r] = c;
}
__global__ void k_nz_fill(const int* ptr, const int* col, const double* M, const double* L, long long n,
                          const int* nptr, int* ncol, double* nM, double* nL) {
  long long r = blockIdx.x * (long long)BLK + threadIdx.x;
  if (r >= n) return;
  int o = nptr[r];
  for (int e = ptr[r]; e < ptr[r + 1]; ++e)
    if (M[e] != 0.0 || L[e] != 0.0) {
      ncol[o] = col[e];
      nM[o] = M[e];
      nL[o] = L[e];
      ++o;
    }
}
__global__ void k_set_last(int* ptr, long long n, const int* cnt, const int* off) {
  ptr[n] = off[n - 1] + cnt[n - 1];
}

// y = (alpha M + beta L) x, x and y n x k row-major
// y = (alpha M + beta L) x, x and y n x k row-major; M or L null = absent.
// Eight lanes per row, each taking every eighth entry, partial sums combined
// by shuffles; columns in groups of four.
constexpr int CL = 8;
__global__ __launch_bounds__(BLK) void k_csr_apply(const int* ptr, const int* col, const double* M, const double* L,
                                                   double alpha, double beta, long long n, int k, const double* x,
                                                   double* y) {
  const long long r = (blockIdx.x * (long long)BLK + threadIdx.x) / CL;
  const int sub = threadIdx.x % CL;
  const bool ok = r < n;
  const int e0 = ok ? ptr[r] : 0, e1 = ok ? ptr[r + 1] : 0;
  for (int c0 = 0; c0 < k; c0 += 4) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int e = e0 + sub; e < e1; e += CL) {
      const double a = (M ? alpha * M[e] : 0.0) + (L ? beta * L[e] : 0.0);
      const double* xr = x + (long long)col[e] * k;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (c0 + q < k) acc[q] += a * xr[c0 + q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double v = acc[q];
      for (int o = CL / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (ok && sub == 0 && c0 + q < k) y[r * k + c0 + q] = v;
    }
  }
}

// layout changes between column-major (n x k) and row-major (n x k)
__global__ void k_transpose(const double* in, long long n, int k, double* out, int to_rowmajor) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n * k) return;
  long long r = i / k;
  int c = (int)(i - r * k);
  if (to_rowmajor) out[i] = in[(long long)c * n + r];
  else out[(long long)c * n + r] = in[i];
}

__global__ void k_linear_coeffs(const u64* fkey, long long n, int degree, const double* cube, double hd,
                                double* X) {
  long long f = blockIdx.x * (long long)BLK + threadIdx.x;
  if (f >= n) return;
  long long c[3];
  demorton(fkey[f], c);
  for (int a = 0; a < 3; ++a) {
    double g = degree == 1 ? (double)c[a] : (double)c[a] - 0.5;
    X[(long long)a * n + f] = cube[a] + g * hd;
  }
}

template <int DEG>
__global__ void k_eval_vertices(const double* U, long long nv, int D, const int* vt_ptr, const int* vt_tri,
                                const u64* ent, long long nent, const int* ent_func, const double* x, long long n,
                                int k, double* out) {
  constexpr int W = DEG == 1 ? 2 : 3;
  long long v = blockIdx.x * (long long)BLK + threadIdx.x;
  if (v >= nv) return;
  for (int c = 0; c < k; ++c) out[(long long)c * nv + v] = 0.0;
  if (vt_ptr[v] == vt_ptr[v + 1]) return;
  const int t = vt_tri[vt_ptr[v]];
  const long long top = (1LL << D) - 1;
  long long cc[3];
  double lc[3];
  for (int a = 0; a < 3; ++a) {
    double u = U[3 * v + a];
    cc[a] = max(0LL, min(top, (long long)floor(u)));
    lc[a] = u - (double)cc[a];
  }
  for (int jz = 0; jz < W; ++jz)
    for (int jy = 0; jy < W; ++jy)
      for (int jx = 0; jx < W; ++jx) {
        double bx, by, bz, d;
        basis1d<DEG>(jx, lc[0], bx, d);
        basis1d<DEG>(jy, lc[1], by, d);
        basis1d<DEG>(jz, lc[2], bz, d);
        double phi = bx * by * bz;
        if (phi == 0.0) continue;
        u64 key = (morton((u64)(cc[0] + jx), (u64)(cc[1] + jy), (u64)(cc[2] + jz)) << TRI_BITS) | (u64)t;
        long long p = lower_bound_u64(ent, 0, nent, key);
        if (p >= nent || ent[p] != key) continue;
        int r = ent_func[p];
        for (int c = 0; c < k; ++c) out[(long long)c * nv + v] += phi * x[(long long)c * n + r];
      }
}

// ---------------------------------------------------------- host side
struct Chunks {
  DArr<int2> c;
  int n = 0;
};

Chunks make_chunks(camfe_ctx ctx, const HLevel& L) {
  Chunks out;
  const size_t np = L.npairs;
  if (np == 0) return out;
  DArr<int> flag(np), pos(np);
  unsigned g = grid_for(np, BLK);
  hipLaunchKernelGGL(k_cell_heads, g, BLK, 0, ctx->stream, L.pairs.p, (long long)np, flag.p);
  exclusive_scan(ctx, flag.p, pos.p, np);
  int ncell = read_scalar(ctx, pos.p + np - 1) + read_scalar(ctx, flag.p + np - 1);
  DArr<int> start(ncell), cnt(ncell), off(ncell);
  hipLaunchKernelGGL(k_cell_starts, g, BLK, 0, ctx->stream, flag.p, pos.p, (long long)np, start.p);
  hipLaunchKernelGGL(k_chunk_count, grid_for(ncell, BLK), BLK, 0, ctx->stream, start.p, ncell, (long long)np, cnt.p);
  exclusive_scan(ctx, cnt.p, off.p, ncell);
  out.n = read_scalar(ctx, off.p + ncell - 1) + read_scalar(ctx, cnt.p + ncell - 1);
  out.c.alloc(out.n);
  hipLaunchKernelGGL(k_chunk_fill, grid_for(ncell, BLK), BLK, 0, ctx->stream, start.p, off.p, ncell, (long long)np,
                     out.c.p);
  check_launch();
  return out;
}

// Launch one assembly pass.  With the timer on, the pass counts its quadrature
// points and records the flops of the dense contractions it performed:
// M_e and the three gradient products, 2 NB^2 flops each per point.
void launch_assemble(camfe_hier h, int d, const Chunks& ch, AsmArgs a) {
  if (ch.n == 0) return;
  camfe_ctx ctx = h->ctx;
  unsigned grid = (unsigned)std::min(ch.n, 1 << 20);
  DArr<unsigned long long> cnt;
  const bool timed = ctx->timer.on && a.M != nullptr;
  if (timed) {
    cnt.alloc(1);
    zero(ctx, cnt.p, 1);
    a.npts = cnt.p;
  }
  if (a.rhs && h->degree == 1)
    CAMFE_TIMED(ctx, KT_ASSEMBLE, 0.0, (k_assemble<1, false, true>), grid, 64, 0, ctx->stream, a);
  else if (a.rhs)
    CAMFE_TIMED(ctx, KT_ASSEMBLE, 0.0, (k_assemble<2, false, true>), grid, 64, 0, ctx->stream, a);
  else if (h->degree == 1)
    CAMFE_TIMED(ctx, KT_ASSEMBLE, 0.0, k_assemble<1>, grid, 64, 0, ctx->stream, a);
  else
    CAMFE_TIMED(ctx, KT_ASSEMBLE, 0.0, k_assemble<2>, grid, 64, 0, ctx->stream, a);
  check_launch();
  if (timed) {
    const double NB = h->NB();
    ctx->timer.pending.back().work = (double)read_scalar(ctx, cnt.p) * 2.0 * NB * NB * (a.L ? 4.0 : 1.0);
  }
}

AsmArgs base_args(camfe_hier h, int d, const Chunks& ch) {
  const HLevel& L = h->lev[d];
  AsmArgs a;
  std::memset(&a, 0, sizeof(a));
  a.pairs = L.pairs.p;
  a.pair_rows = L.pair_rows.p;
  a.chunks = ch.c.p;
  a.nchunk = ch.n;
  a.U = h->U.p;
  a.F = h->F.p;
  a.nrm = h->nrm.p;
  a.sc = std::ldexp(1.0, d - h->D);
  const double hd = h->cube[3] / std::ldexp(1.0, d);
  a.hd2 = hd * hd;
  a.nv = (long long)h->nv;
  return a;
}

}  // namespace

// Assemble M (and L) at depth d into the system's CSR (built here the first time)
void assemble_level(camfe_sys s, int d, bool want_L, bool want_M) {
  camfe_hier h = s->h;
  camfe_ctx ctx = h->ctx;
  upload_rules();
  const HLevel& L = h->lev[d];
  SLevel& S = s->lev[d];
  Chunks ch = make_chunks(ctx, L);
  if (S.ptr.n == 0) {
    // superset structure, assembly, then compaction to the entries that are hit
    const size_t n = L.nfun;
    DArr<int> cnt(n), sptr(n + 1);
    unsigned g = grid_for(n, BLK);
    if (h->degree == 1)
      hipLaunchKernelGGL((k_struct<1, false>), g, BLK, 0, ctx->stream, L.fkey.p, (long long)n, L.ckey.p,
                         (long long)L.ncorn, L.cfirst.p, cnt.p, (const int*)nullptr, (int*)nullptr);
    else
      hipLaunchKernelGGL((k_struct<2, false>), g, BLK, 0, ctx->stream, L.fkey.p, (long long)n, L.ckey.p,
                         (long long)L.ncorn, L.cfirst.p, cnt.p, (const int*)nullptr, (int*)nullptr);
    check_launch();
    exclusive_scan(ctx, cnt.p, sptr.p, n);
    hipLaunchKernelGGL(k_set_last, 1, 1, 0, ctx->stream, sptr.p, (long long)n, cnt.p, sptr.p);
    const int snnz = read_scalar(ctx, sptr.p + n);
    DArr<int> scol(snnz);
    if (h->degree == 1)
      hipLaunchKernelGGL((k_struct<1, true>), g, BLK, 0, ctx->stream, L.fkey.p, (long long)n, L.ckey.p,
                         (long long)L.ncorn, L.cfirst.p, (int*)nullptr, sptr.p, scol.p);
    else
      hipLaunchKernelGGL((k_struct<2, true>), g, BLK, 0, ctx->stream, L.fkey.p, (long long)n, L.ckey.p,
                         (long long)L.ncorn, L.cfirst.p, (int*)nullptr, sptr.p, scol.p);
    check_launch();
    DArr<double> sM(snnz), sL(snnz);
    zero(ctx, sM.p, snnz);
    zero(ctx, sL.p, snnz);
    AsmArgs a = base_args(h, d, ch);
    a.tri_w = s->tri_w.n ? s->tri_w.p : nullptr;
    a.ptr = sptr.p;
    a.col = scol.p;
    a.M = sM.p;
    a.L = sL.p;
    launch_assemble(h, d, ch, a);
    hipLaunchKernelGGL(k_nz_count, g, BLK, 0, ctx->stream, sptr.p, sM.p, sL.p, (long long)n, cnt.p);
    S.n = n;
    S.ptr.alloc(n + 1);
    exclusive_scan(ctx, cnt.p, S.ptr.p, n);
    hipLaunchKernelGGL(k_set_last, 1, 1, 0, ctx->stream, S.ptr.p, (long long)n, cnt.p, S.ptr.p);
    S.nnz = (size_t)read_scalar(ctx, S.ptr.p + n);
    S.col.alloc(S.nnz);
    S.M.alloc(S.nnz);
    S.L.alloc(S.nnz);
    hipLaunchKernelGGL(k_nz_fill, g, BLK, 0, ctx->stream, sptr.p, scol.p, sM.p, sL.p, (long long)n, S.ptr.p,
                       S.col.p, S.M.p, S.L.p);
    check_launch();
    ctx->sync();
    return;
  }
  // re-assembly into the existing structure
  if (want_M) zero(ctx, S.M.p, S.nnz);
  if (want_L) zero(ctx, S.L.p, S.nnz);
  AsmArgs a = base_args(h, d, ch);
  a.tri_w = s->tri_w.n ? s->tri_w.p : nullptr;
  a.ptr = S.ptr.p;
  a.col = S.col.p;
  if (want_M && want_L) {
    a.M = S.M.p;
    a.L = S.L.p;
    launch_assemble(h, d, ch, a);
  } else if (want_M) {
    a.M = S.M.p;
    a.L = nullptr;
    launch_assemble(h, d, ch, a);
  }
  ctx->sync();
}

// M at depth d for new triangle weights.  Degree 1: the first call runs the
// quadrature once more and keeps every pair's unweighted element block (36
// doubles per pair, when that fits in a quarter of the free device memory);
// later calls only weight and scatter the kept blocks.  Degree 2, or no room:
// the full mass assembly.
void reassemble_mass_level(camfe_sys s, int d) {
  camfe_hier h = s->h;
  camfe_ctx ctx = h->ctx;
  if (h->degree != 1) {
    assemble_level(s, d, false, true);
    return;
  }
  if (s->mcache.size() <= (size_t)d) s->mcache.resize(d + 1);
  DArr<double>& C = s->mcache[d];
  const HLevel& L = h->lev[d];
  SLevel& S = s->lev[d];
  const size_t need = L.npairs * 36;
  if (C.n != need) {
    size_t free_b = 0, total_b = 0;
    CAMFE_HIP(hipMemGetInfo(&free_b, &total_b));
    if (need * sizeof(double) > free_b / 4) {
      assemble_level(s, d, false, true);
      return;
    }
    upload_rules();
    Chunks ch = make_chunks(ctx, L);
    C.alloc(need);
    zero(ctx, C.p, need);
    zero(ctx, S.M.p, S.nnz);
    AsmArgs a = base_args(h, d, ch);
    a.tri_w = s->tri_w.n ? s->tri_w.p : nullptr;
    a.ptr = S.ptr.p;
    a.col = S.col.p;
    a.M = S.M.p;
    a.pcache = C.p;
    if (ch.n) {
      CAMFE_TIMED(ctx, KT_ASSEMBLE, 0.0, (k_assemble<1, true>), (unsigned)std::min(ch.n, 1 << 20), 64, 0,
                  ctx->stream, a);
    }
    check_launch();
    ctx->sync();
    return;
  }
  Chunks ch = make_chunks(ctx, L);
  zero(ctx, S.M.p, S.nnz);
  if (ch.n)
    hipLaunchKernelGGL(k_mass_cached, (unsigned)std::min(ch.n, 1 << 20), 64, 0, ctx->stream, ch.c.p, ch.n,
                       L.pairs.p, L.pair_rows.p, (const double*)C.p,
                       (const double*)(s->tri_w.n ? s->tri_w.p : nullptr), S.ptr.p, S.col.p, S.M.p);
  check_launch();
  ctx->sync();
}

void load_vector_dev(camfe_sys s, const double* d_fv, int k, double* d_b, bool grad) {
  camfe_hier h = s->h;
  camfe_ctx ctx = h->ctx;
  upload_rules();
  const int d = h->D;
  const HLevel& L = h->lev[d];
  Chunks ch = make_chunks(ctx, L);
  zero(ctx, d_b, L.nfun * (size_t)k);
  for (int c0 = 0; c0 < k; c0 += KMAX) {
    AsmArgs a = base_args(h, d, ch);
    a.tri_w = nullptr;
    a.fv = d_fv + (size_t)c0 * h->nv;
    a.k = std::min(KMAX, k - c0);
    a.rhs = d_b + (size_t)c0 * L.nfun;
    a.ldr = (long long)L.nfun;
    a.grad_rhs = grad ? 1 : 0;
    launch_assemble(h, d, ch, a);
  }
  ctx->sync();
}

void csr_apply(camfe_ctx ctx, const SLevel& L, double alpha, double beta, const double* x, int k, double* y) {
  hipLaunchKernelGGL(k_csr_apply, grid_for(L.n * CL, BLK), BLK, 0, ctx->stream, L.ptr.p, L.col.p,
                     (const double*)(alpha != 0.0 ? L.M.p : nullptr), (const double*)(beta != 0.0 ? L.L.p : nullptr),
                     alpha, beta, (long long)L.n, k, x, y);
  check_launch();
}

void to_rowmajor(camfe_ctx ctx, const double* in, size_t n, int k, double* out) {
  hipLaunchKernelGGL(k_transpose, grid_for(n * k, BLK), BLK, 0, ctx->stream, in, (long long)n, k, out, 1);
  check_launch();
}
void to_colmajor(camfe_ctx ctx, const double* in, size_t n, int k, double* out) {
  hipLaunchKernelGGL(k_transpose, grid_for(n * k, BLK), BLK, 0, ctx->stream, in, (long long)n, k, out, 0);
  check_launch();
}

}  // namespace camfe

using namespace camfe;

// host or device vertex values in, host or device b out
static camfe_status load_common(camfe_sys s, const double* vertex_f, int k, double* b, bool grad) {
  return guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s && vertex_f && b && k > 0, CAMFE_EINVAL, "bad argument");
    require_mesh(s);
    camfe_hier h = s->h;
    camfe_ctx ctx = h->ctx;
    ctx->use_device();
    const size_t n = h->lev[h->D].nfun;
    DArr<double> fv(h->nv * (size_t)k), bd(n * (size_t)k);
    copy_in(ctx, fv.p, vertex_f, fv.n);
    load_vector_dev(s, fv.p, k, bd.p, grad);
    copy_out(ctx, b, bd.p, bd.n);
    ctx->sync();
  });
}

extern "C" {

camfe_status camfe_assemble(camfe_hier h, const double* tri_weight, camfe_sys* out) {
  return guarded([&] {
    if (h) set_current_ctx(h->ctx);
    CAMFE_REQUIRE(h && out, CAMFE_EINVAL, "null argument");
    camfe_ctx ctx = h->ctx;
    ctx->use_device();
    std::unique_ptr<camfe_sys_s> s(new camfe_sys_s());
    s->h = h;
    s->lev.resize(h->D + 1);
    if (tri_weight) {
      s->tri_w.alloc(h->nt);
      copy_in(ctx, s->tri_w.p, tri_weight, h->nt);
    }
    for (int d = h->d0; d <= h->D; ++d) assemble_level(s.get(), d, true, true);
    *out = s.release();
  });
}

camfe_status camfe_reassemble_mass(camfe_sys s, const double* tri_weight) {
  return guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s, CAMFE_EINVAL, "null system");
    require_mesh(s);
    camfe_ctx ctx = s->h->ctx;
    ctx->use_device();
    if (tri_weight) {
      if (s->tri_w.n != s->h->nt) s->tri_w.alloc(s->h->nt);
      copy_in(ctx, s->tri_w.p, tri_weight, s->h->nt);
    } else {
      s->tri_w.release();
    }
    for (int d = s->h->d0; d <= s->h->D; ++d) reassemble_mass_level(s, d);
    refresh_solver(s);
  });
}

camfe_status camfe_export_matrix(camfe_sys s, int depth, int which, int64_t* rowptr, int32_t* col, double* val,
                                 int64_t cap, int64_t* nnz) {
  return guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s && (which == 0 || which == 1), CAMFE_EINVAL, "bad argument");
    camfe_hier h = s->h;
    CAMFE_REQUIRE(depth >= h->d0 && depth <= h->D, CAMFE_ESTATE, "depth not assembled");
    const SLevel& L = s->lev[depth];
    if (nnz) *nnz = (int64_t)L.nnz;
    if (cap == 0) return;
    CAMFE_REQUIRE(cap >= (int64_t)L.nnz, CAMFE_ETOOSMALL, "export capacity too small");
    camfe_ctx ctx = h->ctx;
    ctx->use_device();
    if (rowptr) {
      std::vector<int> hp(L.n + 1);
      copy_out(ctx, hp.data(), L.ptr.p, L.n + 1);
      ctx->sync();
      std::vector<int64_t> h64(hp.begin(), hp.end());
      copy_out(ctx, rowptr, h64.data(), L.n + 1);
      ctx->sync();
    }
    if (col) copy_out(ctx, (int*)col, L.col.p, L.nnz);
    if (val) copy_out(ctx, val, which == 0 ? L.M.p : L.L.p, L.nnz);
    ctx->sync();
  });
}


camfe_status camfe_load_vector(camfe_sys s, const double* vertex_f, int k, double* b) {
  return load_common(s, vertex_f, k, b, false);
}

camfe_status camfe_gradient_load(camfe_sys s, const double* vertex_f, int k, double* b) {
  return load_common(s, vertex_f, k, b, true);
}

camfe_status camfe_apply(camfe_sys s, int which, double t, const double* x, int k, double* y) {
  return guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s && x && y && k > 0 && which >= 0 && which <= 2, CAMFE_EINVAL, "bad argument");
    camfe_hier h = s->h;
    camfe_ctx ctx = h->ctx;
    ctx->use_device();
    const SLevel& L = s->lev[h->D];
    DArr<double> xc(L.n * (size_t)k), xr(L.n * (size_t)k), yr(L.n * (size_t)k);
    copy_in(ctx, xc.p, x, xc.n);
    to_rowmajor(ctx, xc.p, L.n, k, xr.p);
    double al = which == 1 ? 0.0 : 1.0, be = which == 0 ? 0.0 : (which == 1 ? 1.0 : t);
    csr_apply(ctx, L, al, be, xr.p, k, yr.p);
    to_colmajor(ctx, yr.p, L.n, k, xc.p);
    copy_out(ctx, y, xc.p, xc.n);
    ctx->sync();
  });
}

// true when p is device memory of the given device (clears the runtime's
// error state when p is unknown to it, as plain host memory is)
static bool device_memory_of(const void* p, int device) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == device;
}

camfe_status camfe_apply_noalloc(camfe_sys s, int which, double t, const double* x, int k, double* y) {
  return guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s && x && y && k > 0 && which >= 0 && which <= 2, CAMFE_EINVAL, "bad argument");
    camfe_hier h = s->h;
    camfe_ctx ctx = h->ctx;
    ctx->use_device();
    const SLevel& L = s->lev[h->D];
    CAMFE_REQUIRE(L.n * (size_t)k <= NOALLOC_BLOCK, CAMFE_EINVAL,
                  "n x k = " + std::to_string(L.n * (size_t)k) + " exceeds the scratch limit of 2^20 values");
    CAMFE_REQUIRE(device_memory_of(x, ctx->device) && device_memory_of(y, ctx->device), CAMFE_EINVAL,
                  "x and y must be device memory of the context's device");
    CAMFE_REQUIRE(ctx->noalloc_scratch, CAMFE_ESTATE, "no device scratch for this context");
    double* xr = ctx->noalloc_scratch;
    double* yr = ctx->noalloc_scratch + NOALLOC_BLOCK;
    to_rowmajor(ctx, x, L.n, k, xr);
    double al = which == 1 ? 0.0 : 1.0, be = which == 0 ? 0.0 : (which == 1 ? 1.0 : t);
    csr_apply(ctx, L, al, be, xr, k, yr);
    to_colmajor(ctx, yr, L.n, k, y);
    ctx->sync();
  });
}

camfe_status camfe_linear_coeffs(camfe_sys s, double* X) {
  return guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s && X, CAMFE_EINVAL, "bad argument");
    require_mesh(s);
    camfe_hier h = s->h;
    camfe_ctx ctx = h->ctx;
    ctx->use_device();
    const HLevel& L = h->lev[h->D];
    DArr<double> Xd(3 * L.nfun);
    const double hd = h->cube[3] / std::ldexp(1.0, h->D);
    hipLaunchKernelGGL(k_linear_coeffs, grid_for(L.nfun, BLK), BLK, 0, ctx->stream, L.fkey.p, (long long)L.nfun,
                       h->degree, h->cubed.p, hd, Xd.p);
    check_launch();
    copy_out(ctx, X, Xd.p, Xd.n);
    ctx->sync();
  });
}

camfe_status camfe_eval_vertices(camfe_sys s, const double* x, int k, double* vertex_out) {
  return guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s && x && vertex_out && k > 0, CAMFE_EINVAL, "bad argument");
    require_mesh(s);
    camfe_hier h = s->h;
    camfe_ctx ctx = h->ctx;
    ctx->use_device();
    const HLevel& L = h->lev[h->D];
    DArr<double> xd(L.nfun * (size_t)k), od(h->nv * (size_t)k);
    copy_in(ctx, xd.p, x, xd.n);
    unsigned g = grid_for(h->nv, BLK);
    if (h->degree == 1)
      hipLaunchKernelGGL(k_eval_vertices<1>, g, BLK, 0, ctx->stream, h->U.p, (long long)h->nv, h->D, h->vt_ptr.p,
                         h->vt_tri.p, L.ent.p, (long long)L.nent, L.ent_func.p, xd.p, (long long)L.nfun, k, od.p);
    else
      hipLaunchKernelGGL(k_eval_vertices<2>, g, BLK, 0, ctx->stream, h->U.p, (long long)h->nv, h->D, h->vt_ptr.p,
                         h->vt_tri.p, L.ent.p, (long long)L.nent, L.ent_func.p, xd.p, (long long)L.nfun, k, od.p);
    check_launch();
    copy_out(ctx, vertex_out, od.p, od.n);
    ctx->sync();
  });
}

void camfe_system_destroy(camfe_sys s) {
  if (!s) return;
  (void)hipSetDevice(s->h->ctx->device);
  (void)hipStreamSynchronize(s->h->ctx->stream);
  delete s;
}

}  // extern "C"

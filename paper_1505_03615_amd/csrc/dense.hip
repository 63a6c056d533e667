// Dense symmetric positive definite inverse for the coarsest depth: blocked
// right-looking Cholesky A = L L^T (diagonal blocks factored in LDS, panels by
// triangular solves, trailing updates by a tiled FP64 MFMA GEMM), then the inverse
// of L bottom up (all diagonal blocks at once, then doubling block sizes, two
// batched GEMMs per level), then A^-1 = L^-T L^-1 by one more GEMM.  All matrices are n x n
// row-major in device memory.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace camfe {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int NB = 32;      // block size of the factorisation and of the triangular inverse
constexpr int TM = 64;      // GEMM tile (four wavefronts of 32 x 32 on the FP64 matrix cores)
constexpr int TK = 16;      // GEMM k-chunk staged in LDS

// One TM x TM tile (ti, tj) of C = beta C + alpha op(A) op(B) on an M x N
// output; op(A)(i, p) = TA ? A[p][i] : A[i][p], op(B)(p, j) = TB ? B[j][p] :
// B[p][j].  lower != 0: only entries with j <= i are written.
template <bool TA, bool TB>
__device__ inline void dgemm_tile(int ti, int tj, int M, int N, int Kd, const double* A, long long lda,
                                  const double* B, long long ldb, double* C, long long ldc, double alpha, double beta,
                                  int lower) {
  if (lower && tj > ti) return;
  const int i0 = ti * TM, j0 = tj * TM;
  if (i0 >= M || j0 >= N) return;
  __shared__ double As[TK][TM + 1];
  __shared__ double Bs[TK][TM + 1];
  // four wavefronts, each a 32 x 32 quadrant of the tile as 2 x 2 blocks of
  // v_mfma_f64_16x16x4 (operand lane l: row/column l % 16 at k = l / 16;
  // result lane l, register r: row l / 16 + 4 r, column l % 16)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int qr = 32 * (w >> 1), qc = 32 * (w & 1);
  const int sl = lane & 15, kq = lane >> 4;
  d4 acc[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = (d4){0.0, 0.0, 0.0, 0.0};
  for (int p0 = 0; p0 < Kd; p0 += TK) {
    for (int e = threadIdx.x; e < TM * TK; e += 256) {
      int r, p;
      if (TA) { p = e / TM; r = e % TM; } else { r = e / TK; p = e % TK; }
      const int gi = i0 + r, gp = p0 + p;
      As[p][r] = (gi < M && gp < Kd) ? (TA ? A[(long long)gp * lda + gi] : A[(long long)gi * lda + gp]) : 0.0;
      int c, q;
      if (TB) { c = e / TK; q = e % TK; } else { q = e / TM; c = e % TM; }
      const int gj = j0 + c, gq = p0 + q;
      Bs[q][c] = (gj < N && gq < Kd) ? (TB ? B[(long long)gj * ldb + gq] : B[(long long)gq * ldb + gj]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k0 = 0; k0 < TK; k0 += 4) {
      const double a0 = As[k0 + kq][qr + sl], a1 = As[k0 + kq][qr + 16 + sl];
      const double b0 = Bs[k0 + kq][qc + sl], b1 = Bs[k0 + kq][qc + 16 + sl];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + qr + 16 * u + kq + 4 * r, gj = j0 + qc + 16 * v + sl;
        if (gi < M && gj < N && (!lower || gj <= gi)) {
          double* c = C + (long long)gi * ldc + gj;
          *c = (beta == 0.0 ? 0.0 : beta * *c) + alpha * acc[u][v][r];
        }
      }
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_dgemm(int M, int N, int Kd, const double* A, long long lda, const double* B,
                                               long long ldb, double* C, long long ldc, double alpha, double beta,
                                               int lower) {
  dgemm_tile<TA, TB>(blockIdx.y, blockIdx.x, M, N, Kd, A, lda, B, ldb, C, ldc, alpha, beta, lower);
}

// One level of the bottom-up triangular inverse: for every pair z of
// neighbouring diagonal blocks of size h (rows o = 2 h z .. o + h and
// o + h .. min(o + 2h, n)), whose inverses W11 and W22 are in place,
// STEP 1: T_z = L21 W11, STEP 2: W21 = -W22 T_z (T_z at T + z h^2, leading dimension h)
template <int STEP>
__global__ __launch_bounds__(256) void k_trinv_level(const double* L, double* W, double* T, long long n, int h) {
  const long long o = 2LL * h * blockIdx.z;
  const int mz = (int)(std::min((long long)2 * h, n - o) - h);   // rows of the second block (> 0)
  double* Tz = T + (long long)blockIdx.z * h * h;
  if (STEP == 1)
    dgemm_tile<false, false>(blockIdx.y, blockIdx.x, mz, h, h, L + (o + h) * n + o, n, W + o * n + o, n, Tz, h,
                             1.0, 0.0, 0);
  else
    dgemm_tile<false, false>(blockIdx.y, blockIdx.x, mz, h, mz, W + (o + h) * n + (o + h), n, Tz, h,
                             W + (o + h) * n + o, n, -1.0, 0.0, 0);
}

// Cholesky of the kb x kb diagonal block at (k0, k0) in LDS; writes L_kk with
// zeros above its diagonal.  A non-positive pivot sets *fail.
__global__ __launch_bounds__(256) void k_potrf_diag(double* A, long long n, int k0, int kb, int* fail) {
  __shared__ double L[NB][NB + 1];
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int i = e / NB, j = e % NB;
    L[i][j] = (i < kb && j < kb) ? A[(long long)(k0 + i) * n + k0 + j] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    if (threadIdx.x == 0) {
      double a = L[j][j];
      if (!(a > 0.0)) { *fail = 1; a = 1.0; }
      L[j][j] = sqrt(a);
    }
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < kb; i += 256) L[i][j] /= L[j][j];
    __syncthreads();
    const int m = kb - j - 1;
    for (int e = threadIdx.x; e < m * m; e += 256) {
      const int i = j + 1 + e / m, k = j + 1 + e % m;
      if (k <= i) L[i][k] -= L[i][j] * L[k][j];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < kb * kb; e += 256) {
    const int i = e / kb, j = e % kb;
    A[(long long)(k0 + i) * n + k0 + j] = j <= i ? L[i][j] : 0.0;
  }
}

// rows i >= k0 + kb of the panel: x L_kk^T = a, x overwriting A[i][k0 .. k0+kb)
__global__ __launch_bounds__(64) void k_trsm_panel(double* A, long long n, int k0, int kb) {
  __shared__ double L[NB][NB + 1];
  for (int e = threadIdx.x; e < NB * NB; e += 64) {
    const int i = e / NB, j = e % NB;
    L[i][j] = (i < kb && j < kb) ? A[(long long)(k0 + i) * n + k0 + j] : 0.0;
  }
  __syncthreads();
  const long long i = (long long)k0 + kb + blockIdx.x * 64LL + threadIdx.x;
  if (i >= n) return;
  double* row = A + i * n + k0;
  double x[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < kb) {
      double v = row[j];
      for (int p = 0; p < j; ++p) v -= x[p] * L[j][p];
      x[j] = v / L[j][j];
    }
  }
#pragma unroll
  for (int j = 0; j < NB; ++j)
    if (j < kb) row[j] = x[j];
}

// inverse of the lower-triangular diagonal block number blockIdx.x (rows
// r0 = NB blockIdx.x .. r0 + rb) of L into the same block of W
__global__ __launch_bounds__(64) void k_trtri_diag(const double* L, double* W, long long n) {
  const int r0 = blockIdx.x * NB;
  const int rb = (int)std::min((long long)NB, n - r0);
  __shared__ double T[NB][NB + 1];
  for (int e = threadIdx.x; e < NB * NB; e += 64) {
    const int i = e / NB, j = e % NB;
    T[i][j] = (i < rb && j < rb) ? L[(long long)(r0 + i) * n + r0 + j] : 0.0;
  }
  __syncthreads();
  // column c of the inverse: forward substitution of T y = e_c
  const int c = threadIdx.x;
  if (c >= rb) return;
  double y[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (i < rb) {
      double v = i == c ? 1.0 : 0.0;
      for (int p = c; p < i; ++p) v -= T[i][p] * y[p];
      y[i] = i < c ? 0.0 : v / T[i][i];
    }
  }
#pragma unroll
  for (int i = 0; i < NB; ++i)
    if (i < rb) W[(long long)(r0 + i) * n + r0 + c] = y[i];
}

__global__ void k_zero_upper(double* A, long long n) {
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= n * n) return;
  if (e % n > e / n) A[e] = 0.0;
}

// Ainv[r][c] = s_r s_c C[max(r,c)][min(r,c)] (C holds the lower triangle)
__global__ void k_sym_scale(const double* C, long long n, const double* s, double* out) {
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= n * n) return;
  const long long r = e / n, c = e % n;
  out[e] = (r >= c ? C[r * n + c] : C[c * n + r]) * s[r] * s[c];
}

template <bool TA, bool TB>
void gemm(camfe_ctx ctx, int M, int N, int Kd, const double* A, long long lda, const double* B, long long ldb,
          double* C, long long ldc, double alpha, double beta, bool lower) {
  if (M <= 0 || N <= 0) return;
  dim3 grid((N + TM - 1) / TM, (M + TM - 1) / TM);
  hipLaunchKernelGGL((k_dgemm<TA, TB>), grid, dim3(256), 0, ctx->stream, M, N, Kd, A, lda, B, ldb, C, ldc, alpha,
                     beta, lower ? 1 : 0);
}

// W = inverse of the lower-triangular L (n x n), bottom up: every NB x NB
// diagonal block in one launch, then levels of doubling block size, each
// pairing neighbouring inverted blocks with two batched GEMMs
void trinv(camfe_ctx ctx, const double* L, double* W, double* T, long long n) {
  const int nb = (int)((n + NB - 1) / NB);
  hipLaunchKernelGGL(k_trtri_diag, nb, 64, 0, ctx->stream, L, W, n);
  for (long long h = NB; h < n; h *= 2) {
    const unsigned pairs = (unsigned)((n - h + 2 * h - 1) / (2 * h));   // pairs with a second block
    const unsigned tiles = (unsigned)((h + TM - 1) / TM);
    dim3 grid(tiles, tiles, pairs);
    hipLaunchKernelGGL(k_trinv_level<1>, grid, 256, 0, ctx->stream, L, W, T, n, (int)h);
    hipLaunchKernelGGL(k_trinv_level<2>, grid, 256, 0, ctx->stream, L, W, T, n, (int)h);
  }
}

}  // namespace

// A (n x n, symmetric positive definite, destroyed) -> out = diag(s) A^-1 diag(s).
// Throws CAMFE_ESINGULAR on a non-positive pivot.
void spd_inverse_scaled(camfe_ctx ctx, double* A, int n, const double* s, double* out) {
  const long long nn = (long long)n * n;
  // Cholesky, lower triangle in place
  zero(ctx, ctx->d_flag, 1);
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int kb = std::min(NB, n - k0);
    hipLaunchKernelGGL(k_potrf_diag, 1, 256, 0, ctx->stream, A, (long long)n, k0, kb, ctx->d_flag);
    const int m = n - k0 - kb;
    if (m > 0) {
      hipLaunchKernelGGL(k_trsm_panel, (m + 63) / 64, 64, 0, ctx->stream, A, (long long)n, k0, kb);
      // trailing lower triangle: A22 -= P P^T, P = A[k0+kb.., k0 .. k0+kb)
      const double* P = A + (long long)(k0 + kb) * n + k0;
      double* A22 = A + (long long)(k0 + kb) * n + (k0 + kb);
      gemm<false, true>(ctx, m, m, kb, P, n, P, n, A22, n, -1.0, 1.0, true);
    }
  }
  check_launch();
  const int fail = read_scalar(ctx, ctx->d_flag);
  CAMFE_REQUIRE(fail == 0, CAMFE_ESINGULAR, "coarsest Cholesky failed (increase coarse_eps)");
  hipLaunchKernelGGL(k_zero_upper, grid_for(nn, 256), 256, 0, ctx->stream, A, (long long)n);
  // W = L^-1, recursively: inv([L11 0; L21 L22]) = [W11 0; -W22 L21 W11  W22]
  DArr<double> W(nn), T(nn);
  zero(ctx, W.p, W.n);
  trinv(ctx, A, W.p, T.p, n);
  // A^-1 = W^T W (lower triangle into A), then scale and mirror
  gemm<true, false>(ctx, n, n, n, W.p, n, W.p, n, A, n, 1.0, 0.0, true);
  hipLaunchKernelGGL(k_sym_scale, grid_for(nn, 256), 256, 0, ctx->stream, (const double*)A, (long long)n, s, out);
  check_launch();
  ctx->sync();
}

}  // namespace camfe

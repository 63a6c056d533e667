// Smallest generalised eigenpairs L x = lambda M x of the estimated
// Laplace-Beltrami operator (Section 5.1) by shift-invert subspace iteration.
// Each step solves (L + sigma M) Y = M X with the multigrid-preconditioned CG
// of the solver, then a Rayleigh-Ritz step: the k x k Gram matrices
// G_L = Y^T L Y and G_M = Y^T M Y (block reductions), the small problem
// G_L c = theta G_M c in one workgroup (Cholesky of G_M, cyclic Jacobi
// rotations), and X = Y C.  Blocks live row-major (n x k, row i contiguous)
// for the matrix products and the Gram reductions; the solver takes them
// column-major.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace camfe {
namespace {

constexpr int BLK = 256;
constexpr int KE = 32;        // largest block
constexpr int GR = 64;        // rows per Gram tile

// x[i][j] uniform in (-1, 1) from SplitMix64 of (seed, i k + j)
__global__ void k_random_block(long long n, int k, unsigned long long seed, double* x) {
  long long e = blockIdx.x * (long long)BLK + threadIdx.x;
  if (e >= n * k) return;
  unsigned long long z = seed + 0x9E3779B97F4A7C15ULL * (unsigned long long)(e + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z ^= z >> 31;
  x[e] = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
}

// out (column-major) = in (row-major) * scale_j, scale_j = a / (theta_j + b)
// when theta is given, else a
__global__ void k_to_col_scaled(long long n, int k, const double* in, const double* theta, double a, double b,
                                double* out) {
  long long e = blockIdx.x * (long long)BLK + threadIdx.x;
  if (e >= n * k) return;
  const long long i = e / k;
  const int j = (int)(e - i * k);
  const double sc = theta ? a / (theta[j] + b) : a;
  out[(long long)j * n + i] = in[e] * sc;
}

// Per-block partial Gram matrices: part[b][0][p][q] = sum_i Y[i][p] A[i][q],
// part[b][1][p][q] = sum_i Y[i][p] B[i][q] over the block's rows; each
// thread owns entries e = tid, tid + BLK, ... of the k x k matrix
__global__ __launch_bounds__(BLK) void k_gram2(long long n, int k, const double* Y, const double* A, const double* B,
                                               double* part) {
  __shared__ double ty[GR * KE], ta[GR * KE], tb[GR * KE];
  const int kk = k * k;
  double accA[KE * KE / BLK], accB[KE * KE / BLK];
#pragma unroll
  for (int m = 0; m < KE * KE / BLK; ++m) accA[m] = accB[m] = 0.0;
  const long long tiles = (n + GR - 1) / GR;
  for (long long t = blockIdx.x; t < tiles; t += gridDim.x) {
    const long long r0 = t * GR;
    const int rows = n - r0 < GR ? (int)(n - r0) : GR;
    for (int e = threadIdx.x; e < GR * k; e += BLK) {
      const bool in = e < rows * k;
      ty[e] = in ? Y[r0 * k + e] : 0.0;
      ta[e] = in ? A[r0 * k + e] : 0.0;
      tb[e] = in ? B[r0 * k + e] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < KE * KE / BLK; ++m) {
      const int e = threadIdx.x + m * BLK;
      if (e < kk) {
        const int p = e / k, q = e - p * k;
        double sa = 0.0, sb = 0.0;
        for (int r = 0; r < rows; ++r) {
          const double y = ty[r * k + p];
          sa += y * ta[r * k + q];
          sb += y * tb[r * k + q];
        }
        accA[m] += sa;
        accB[m] += sb;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < KE * KE / BLK; ++m) {
    const int e = threadIdx.x + m * BLK;
    if (e < kk) {
      part[(long long)blockIdx.x * 2 * kk + e] = accA[m];
      part[(long long)blockIdx.x * 2 * kk + kk + e] = accB[m];
    }
  }
}

// out[e] = sum over nb blocks of part[b][e], e < len (blocks of stride len)
__global__ void k_sum_parts(const double* part, int nb, int len, double* out) {
  const int e = blockIdx.x * BLK + threadIdx.x;
  if (e >= len) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(long long)b * len + e];
  out[e] = s;
}

// G_L c = theta G_M c for k <= KE in one workgroup of SG threads: G_M = R R^T
// (lower R, column by column), A = R^-1 G_L R^-T (one column, then one row,
// per thread), cyclic Jacobi on A in the round-robin order of Brent and Luk
// (each round rotates k/2 disjoint index pairs at once; rotations of disjoint
// pairs commute, so a round equals the same rotations done one by one) until
// the off-diagonal mass is below 1e-30 of the total (at most 64 sweeps), then
// C = R^-T Q with the columns in ascending order of theta.
// flag: 1 when G_M is not positive definite.
constexpr int SG = 64;
__global__ __launch_bounds__(SG) void k_small_geig(int k, const double* GL, const double* GM, double* theta,
                                                   double* C, int* flag) {
  __shared__ double R[KE * KE], A[KE * KE], Q[KE * KE];
  __shared__ double rc[KE / 2], rs[KE / 2];
  __shared__ int rp[KE / 2], rq[KE / 2];
  __shared__ double red[2 * SG];
  __shared__ int bad, done, ord[KE];
  const int tid = threadIdx.x;
  for (int e = tid; e < k * k; e += SG) {
    const int tr = (e % k) * k + e / k;
    R[e] = 0.5 * (GM[e] + GM[tr]);
    A[e] = 0.5 * (GL[e] + GL[tr]);
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  // Cholesky, one column at a time
  for (int j = 0; j < k; ++j) {
    if (tid == 0) {
      double d = R[j * k + j];
      for (int p = 0; p < j; ++p) d -= R[j * k + p] * R[j * k + p];
      if (!(d > 0.0)) bad = 1;
      R[j * k + j] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < k; i += SG) {
      double v = R[i * k + j];
      for (int p = 0; p < j; ++p) v -= R[i * k + p] * R[j * k + p];
      R[i * k + j] = v / R[j * k + j];
    }
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) *flag = 1;
    return;   // uniform: every thread read the same shared flag
  }
  for (int e = tid; e < k * k; e += SG)
    if (e % k > e / k) R[e] = 0.0;   // upper part
  __syncthreads();
  // A <- R^-1 A: thread c solves column c
  for (int c = tid; c < k; c += SG)
    for (int i = 0; i < k; ++i) {
      double v = A[i * k + c];
      for (int p = 0; p < i; ++p) v -= R[i * k + p] * A[p * k + c];
      A[i * k + c] = v / R[i * k + i];
    }
  __syncthreads();
  // A <- A R^-T: thread r solves row r
  for (int r = tid; r < k; r += SG)
    for (int i = 0; i < k; ++i) {
      double v = A[r * k + i];
      for (int p = 0; p < i; ++p) v -= A[r * k + p] * R[i * k + p];
      A[r * k + i] = v / R[i * k + i];
    }
  __syncthreads();
  for (int e = tid; e < k * k; e += SG) {
    const int i = e / k, j = e % k;
    if (i < j) {
      const double v = 0.5 * (A[i * k + j] + A[j * k + i]);
      A[i * k + j] = v;
      A[j * k + i] = v;
    }
    Q[e] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  const int m = (k + 1) & ~1;   // even number of slots; slot k (odd k) idles
  for (int sweep = 0; sweep < 64; ++sweep) {
    // off-diagonal and total mass, one row per thread
    double off = 0.0, tot = 0.0;
    for (int r = tid; r < k; r += SG)
      for (int j = 0; j < k; ++j) {
        const double v = A[r * k + j] * A[r * k + j];
        tot += v;
        if (j != r) off += v;
      }
    red[tid] = off;
    red[SG + tid] = tot;
    __syncthreads();
    if (tid == 0) {
      double so = 0.0, st = 0.0;
      for (int t = 0; t < SG; ++t) { so += red[t]; st += red[SG + t]; }
      done = so <= 1e-30 * st;
    }
    __syncthreads();
    if (done) break;
    for (int round = 0; round < m - 1; ++round) {
      // pair i: slots i and m - 1 - i of [0, 1 + (round + 0) % (m - 1), ...]
      if (tid < m / 2) {
        const int a = tid == 0 ? 0 : 1 + (tid - 1 + round) % (m - 1);
        const int b = 1 + (m - 2 - tid + round) % (m - 1);
        const int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, sn = 0.0;
        if (q < k) {
          const double apq = A[p * k + q];
          if (apq != 0.0) {
            const double tau = (A[q * k + q] - A[p * k + p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = t * c;
          }
        }
        rp[tid] = p;
        rq[tid] = q < k ? q : p;   // an idle pair rotates nothing
        rc[tid] = c;
        rs[tid] = sn;
      }
      __syncthreads();
      // columns p, q of A and Q: thread r owns row r
      for (int r = tid; r < k; r += SG)
        for (int i = 0; i < m / 2; ++i) {
          const int p = rp[i], q = rq[i];
          if (p == q) continue;
          const double c = rc[i], sn = rs[i];
          const double ap = A[r * k + p], aq = A[r * k + q];
          A[r * k + p] = c * ap - sn * aq;
          A[r * k + q] = sn * ap + c * aq;
          const double qp = Q[r * k + p], qq = Q[r * k + q];
          Q[r * k + p] = c * qp - sn * qq;
          Q[r * k + q] = sn * qp + c * qq;
        }
      __syncthreads();
      // rows p, q of A: thread r owns column r
      for (int r = tid; r < k; r += SG)
        for (int i = 0; i < m / 2; ++i) {
          const int p = rp[i], q = rq[i];
          if (p == q) continue;
          const double c = rc[i], sn = rs[i];
          const double ap = A[p * k + r], aq = A[q * k + r];
          A[p * k + r] = c * ap - sn * aq;
          A[q * k + r] = sn * ap + c * aq;
        }
      __syncthreads();
    }
  }
  if (tid == 0) {
    for (int i = 0; i < k; ++i) ord[i] = i;
    for (int i = 0; i < k; ++i) {
      int mi = i;
      for (int j = i + 1; j < k; ++j)
        if (A[ord[j] * k + ord[j]] < A[ord[mi] * k + ord[mi]]) mi = j;
      const int tmp = ord[i]; ord[i] = ord[mi]; ord[mi] = tmp;
    }
    *flag = 0;
  }
  __syncthreads();
  // C = R^-T Q: thread j back-substitutes column j
  for (int j = tid; j < k; j += SG) {
    const int src = ord[j];
    theta[j] = A[src * k + src];
    for (int i = k - 1; i >= 0; --i) {
      double v = Q[i * k + src];
      for (int p = i + 1; p < k; ++p) v -= R[p * k + i] * C[p * k + j];
      C[i * k + j] = v / R[i * k + i];
    }
  }
}

// out_m = in_m C for the three row-major blocks (n x k times k x k)
__global__ void k_combine3(long long n, int k, const double* C, const double* y0, const double* y1, const double* y2,
                           double* x0, double* x1, double* x2) {
  __shared__ double c[KE * KE];
  for (int e = threadIdx.x; e < k * k; e += BLK) c[e] = C[e];
  __syncthreads();
  long long e = blockIdx.x * (long long)BLK + threadIdx.x;
  if (e >= n * k) return;
  const long long i = e / k;
  const int j = (int)(e - i * k);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int p = 0; p < k; ++p) {
    const double w = c[p * k + j];
    a0 += y0[i * k + p] * w;
    a1 += y1[i * k + p] * w;
    a2 += y2[i * k + p] * w;
  }
  x0[e] = a0;
  x1[e] = a1;
  x2[e] = a2;
}

// per-block partial column sums of |LX - theta MX|^2 and |MX|^2 (2k values)
__global__ __launch_bounds__(BLK) void k_eig_resid(long long n, int k, const double* LX, const double* MX,
                                                   const double* theta, double* part) {
  __shared__ double sr[BLK], sm[BLK];
  // thread (row slot, column): BLK / k rows per pass
  const int j = threadIdx.x % k, slot = threadIdx.x / k, slots = BLK / k;
  double r2 = 0.0, m2 = 0.0;
  if (slot < slots) {
    const double th = theta[j];
    for (long long i = (long long)blockIdx.x * slots + slot; i < n; i += (long long)gridDim.x * slots) {
      const double mx = MX[i * k + j], r = LX[i * k + j] - th * mx;
      r2 += r * r;
      m2 += mx * mx;
    }
  }
  sr[threadIdx.x] = r2;
  sm[threadIdx.x] = m2;
  __syncthreads();
  if (threadIdx.x < k) {
    double a = 0.0, b = 0.0;
    for (int s = 0; s < slots; ++s) { a += sr[s * k + threadIdx.x]; b += sm[s * k + threadIdx.x]; }
    part[(long long)blockIdx.x * 2 * k + threadIdx.x] = a;
    part[(long long)blockIdx.x * 2 * k + k + threadIdx.x] = b;
  }
}

// evecs (column-major, first nev columns) from the row-major block
__global__ void k_take_cols(long long n, int k, int nev, const double* x, double* out) {
  long long e = blockIdx.x * (long long)BLK + threadIdx.x;
  if (e >= n * nev) return;
  const int j = (int)(e / n);
  const long long i = e - (long long)j * n;
  out[e] = x[i * k + j];
}

}  // namespace
}  // namespace camfe

using namespace camfe;

extern "C" {

camfe_status camfe_eigs(camfe_sys s, const camfe_eig_opts* o, double* evals, double* evecs, camfe_eig_stats* stats) {
  camfe_status rc = CAMFE_OK;
  camfe_status g = guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s && o && evals, CAMFE_EINVAL, "bad argument");
    const int k = o->block > 0 ? o->block : std::min(KE, o->nev + 8);
    CAMFE_REQUIRE(o->nev >= 1 && o->nev <= k && k <= KE, CAMFE_EINVAL, "need 1 <= nev <= block <= 32");
    CAMFE_REQUIRE(o->sigma > 0.0 && std::isfinite(o->sigma), CAMFE_EINVAL, "sigma must be positive");
    CAMFE_REQUIRE(o->max_iter >= 1 && o->tol > 0.0 && o->solve_rtol > 0.0, CAMFE_EINVAL, "bad iteration limits");
    CAMFE_REQUIRE(o->precision == 0 || o->precision == 1, CAMFE_EINVAL, "precision must be 0 or 1");
    camfe_hier h = s->h;
    camfe_ctx ctx = h->ctx;
    ctx->use_device();
    hipStream_t st = ctx->stream;
    const SLevel& Lv = s->lev[h->D];
    const long long n = (long long)Lv.n;
    CAMFE_REQUIRE(n >= k, CAMFE_EINVAL, "block wider than the system");
    const long long nk = n * k;
    const unsigned gnk = grid_for((size_t)nk, BLK);
    auto t0 = std::chrono::steady_clock::now();
    DArr<double> X(nk), Y(nk), LY(nk), MY(nk), LX(nk), MX(nk), cb(nk), cx(nk);
    const int kk = k * k;
    const int nbg = (int)std::min<long long>(1024, (n + GR - 1) / GR);
    const int nbr = (int)std::min<long long>(1024, (n + BLK - 1) / BLK);
    DArr<double> part((size_t)std::max(nbg * 2 * kk, nbr * 2 * k)), G(2 * kk), C(kk), theta(k), rn(2 * k);
    DArr<int> flag(1);
    hipLaunchKernelGGL(k_random_block, gnk, BLK, 0, st, n, k, (unsigned long long)o->seed, X.p);
    csr_apply(ctx, Lv, 1.0, 0.0, X.p, k, MX.p);
    camfe_solve_opts so{};
    so.t = 1.0 / o->sigma;
    so.rtol = o->solve_rtol;
    so.max_iter = 2000;
    so.nu_pre = so.nu_post = 2;
    so.method = 0;
    so.precision = o->precision;
    so.coarse_eps = 1e-6;
    so.cycle = 1;
    int it = 0, cycles = 0;
    double worst = INFINITY, loose = 1.0;
    std::vector<double> th(k), r(2 * k);
    bool have_theta = false;
    while (it < o->max_iter) {
      // (M + L / sigma) Y = M X / sigma, started from X_j / (theta_j + sigma)
      hipLaunchKernelGGL(k_to_col_scaled, gnk, BLK, 0, st, n, k, (const double*)MX.p, (const double*)nullptr,
                         1.0 / o->sigma, 0.0, cb.p);
      if (have_theta)
        hipLaunchKernelGGL(k_to_col_scaled, gnk, BLK, 0, st, n, k, (const double*)X.p, (const double*)theta.p, 1.0,
                           o->sigma, cx.p);
      so.x0_given = have_theta ? 1 : 0;
      // inexact shift-invert: each solve only needs an error well below the
      // wanted pairs' current residual (at least solve_rtol)
      so.rtol = std::max(o->solve_rtol, 1e-2 * loose);
      SolveSummary ss = solve_device(s, so, cb.p, cx.p, k);
      cycles += ss.cycles;
      to_rowmajor(ctx, cx.p, (size_t)n, k, Y.p);
      csr_apply(ctx, Lv, 0.0, 1.0, Y.p, k, LY.p);
      csr_apply(ctx, Lv, 1.0, 0.0, Y.p, k, MY.p);
      hipLaunchKernelGGL(k_gram2, nbg, BLK, 0, st, n, k, (const double*)Y.p, (const double*)LY.p,
                         (const double*)MY.p, part.p);
      hipLaunchKernelGGL(k_sum_parts, grid_for(2 * kk, BLK), BLK, 0, st, (const double*)part.p, nbg, 2 * kk, G.p);
      hipLaunchKernelGGL(k_small_geig, 1, SG, 0, st, k, (const double*)G.p, (const double*)(G.p + kk), theta.p, C.p,
                         flag.p);
      check_launch();
      CAMFE_REQUIRE(read_scalar(ctx, flag.p) == 0, CAMFE_ESINGULAR, "the block's M Gram matrix is not positive definite");
      hipLaunchKernelGGL(k_combine3, gnk, BLK, 0, st, n, k, (const double*)C.p, (const double*)Y.p,
                         (const double*)LY.p, (const double*)MY.p, X.p, LX.p, MX.p);
      hipLaunchKernelGGL(k_eig_resid, nbr, BLK, 0, st, n, k, (const double*)LX.p, (const double*)MX.p,
                         (const double*)theta.p, part.p);
      hipLaunchKernelGGL(k_sum_parts, 1, BLK, 0, st, (const double*)part.p, nbr, 2 * k, rn.p);
      check_launch();
      copy_out(ctx, th.data(), theta.p, (size_t)k);
      copy_out(ctx, r.data(), rn.p, (size_t)(2 * k));
      ctx->sync();
      have_theta = true;
      ++it;
      worst = 0.0;
      for (int j = 0; j < o->nev; ++j) {
        const double v = std::sqrt(r[j]) / ((std::fabs(th[j]) + o->sigma) * std::sqrt(r[k + j]));
        if (!(v <= worst)) worst = v;   // keeps NaN
      }
      loose = std::isfinite(worst) ? std::min(worst, 1.0) : 1.0;
      if (worst <= o->tol) break;
    }
    copy_out(ctx, evals, theta.p, (size_t)o->nev);
    if (evecs) {
      DArr<double> ev((size_t)(n * o->nev));
      hipLaunchKernelGGL(k_take_cols, grid_for((size_t)(n * o->nev), BLK), BLK, 0, st, n, k, o->nev,
                         (const double*)X.p, ev.p);
      copy_out(ctx, evecs, ev.p, ev.n);
    }
    ctx->sync();
    if (stats) {
      stats->iterations = it;
      stats->solve_cycles = cycles;
      stats->max_residual = worst;
      stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!(worst <= o->tol)) rc = CAMFE_ENOCONV;
  });
  if (g != CAMFE_OK) return g;
  if (rc != CAMFE_OK) set_last_error("eigensolver stopped above tol");
  return rc;
}

}  // extern "C"

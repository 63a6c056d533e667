// Learned smoother: per-row relaxation weights for weighted Jacobi, predicted
// by a small MLP per (relative) depth from the row's local stencil, trained on
// the GPU on error samples that the plain multigrid cycle leaves behind.
//
// Features of row i (function k at depth d, degree 1), 30 values:
//   [0..26]  sum over columns j whose support is k + delta of A_ij / A_ii,
//            delta in {-1,0,1}^3 (index (dx+1) + 3 (dy+1) + 9 (dz+1))
//   [27]     clamp(log10(A_ii / max_j A_jj), -30, 0) / 10
//   [28]     M_ii / A_ii
//   [29]     (D - d) / 10
// MLP 30 -> 32 (ReLU) -> 32 (ReLU) -> 1, s = 2 sigmoid(z); rows of zero
// computed mass get omega = 0.  Inference weights are BF16 (FP32 debug mode),
// accumulation FP32.
// The network's output s = 2 sigmoid(z) in (0, 2) is scaled by the l1-Jacobi
// bound c_i = A_ii / sum_j |A_ij|: omega_i = c_i s_i.  Then 2 W^-1 - A (W the
// diagonal of omega_i / A_ii) is strictly diagonally dominant, so every sweep
// contracts the A-norm of the error whatever the network outputs, and the
// V-cycle stays a symmetric positive definite preconditioner for CG.
//
// Training loss per depth (samples e_0^s, nu sweeps):
//   e_{k+1} = e_k - omega * D^-1 A e_k,   L = mean_s log(|A e_nu^s|^2 / |A e_0^s|^2)
// dL/domega from the adjoint sweeps, then back-propagation through the MLP,
// Adam on FP32 master weights.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <vector>

#include "solver.hpp"

namespace camfe {

constexpr int NF = 30;
constexpr int NH = 32;
constexpr int O_W1 = 0;                   // W1[i][j]: feature i -> hidden j
constexpr int O_B1 = O_W1 + NF * NH;      // 960
constexpr int O_W2 = O_B1 + NH;           // 992, W2[a][b]
constexpr int O_B2 = O_W2 + NH * NH;      // 2016
constexpr int O_W3 = O_B2 + NH;           // 2048
constexpr int O_B3 = O_W3 + NH;           // 2080
constexpr int NP = O_B3 + 1;              // 2081
constexpr int FSTRIDE = 32;               // floats per row in memory: 30 features, then c_i
constexpr int C_L1 = 30;                  // c_i = A_ii / sum_j |A_ij| (not a network input)

}  // namespace camfe

struct camfe_model_s {
  int levels = 1;
  int sweep = 0;          // 0: damped Jacobi with l1-bounded weights; 1: multicolour SOR
  int bf16 = 1;
  std::vector<float> w;   // levels * NP, FP32 master weights
};

namespace camfe {
namespace {

constexpr int BLK = 256;

__device__ inline float bf16_to_float(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

template <class WT>
__device__ inline float wload(const WT* p, int i);
template <>
__device__ inline float wload<float>(const float* p, int i) { return p[i]; }
template <>
__device__ inline float wload<uint16_t>(const uint16_t* p, int i) { return bf16_to_float(p[i]); }

// ---------------------------------------------------------------- features
__global__ void k_max_diag(const double* invd, long long n, unsigned long long* out) {
  __shared__ double sh[BLK];
  double m = 0.0;
  for (long long i = blockIdx.x * (long long)BLK + threadIdx.x; i < n; i += (long long)gridDim.x * BLK)
    if (invd[i] > 0.0) m = fmax(m, 1.0 / invd[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = BLK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(sh[0]));   // positive doubles order as integers
}

__global__ void k_features(const int* ptr, const int* col, const double* M, const double* L, double t,
                           const u64* fkey, const int* perm, long long n, double maxdiag, float level, float* feat) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  float* fo = feat + i * FSTRIDE;
  for (int q = 0; q < FSTRIDE; ++q) fo[q] = 0.0f;
  const int f = perm[i];
  double aii = 0.0, mii = 0.0;
  for (int e = ptr[f]; e < ptr[f + 1]; ++e)
    if (col[e] == f) { aii = M[e] + t * L[e]; mii = M[e]; }
  if (!(aii > 0.0)) return;
  long long ck[3];
  demorton(fkey[f], ck);
  double asum = 0.0;
  for (int e = ptr[f]; e < ptr[f + 1]; ++e) {
    asum += fabs(M[e] + t * L[e]);
    long long cj[3];
    demorton(fkey[col[e]], cj);
    const int dx = (int)(cj[0] - ck[0]), dy = (int)(cj[1] - ck[1]), dz = (int)(cj[2] - ck[2]);
    if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1) continue;
    fo[(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)] += (float)((M[e] + t * L[e]) / aii);
  }
  double lg = log10(aii / maxdiag);
  lg = fmin(0.0, fmax(-30.0, lg));
  fo[27] = (float)(lg / 10.0);
  fo[28] = (float)(mii / aii);
  fo[29] = level / 10.0f;
  fo[C_L1] = (float)(aii / asum);
}

// ------------------------------------------------------------------- MLP
template <class WT>
__device__ inline void load_weights(const WT* w, float* sw) {
  for (int i = threadIdx.x; i < NP; i += blockDim.x) sw[i] = wload<WT>(w, i);
  __syncthreads();
}

// forward of one row; returns z and fills the hidden activations when asked
__device__ inline float mlp_row(const float* sw, const float* f, float* a1, float* a2) {
  float h1[NH];
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    float s = sw[O_B1 + j];
#pragma unroll
    for (int i = 0; i < NF; ++i) s = fmaf(f[i], sw[O_W1 + i * NH + j], s);
    if (a1) a1[j] = s;
    h1[j] = fmaxf(s, 0.0f);
  }
  float z = sw[O_B3];
#pragma unroll
  for (int b = 0; b < NH; ++b) {
    float s = sw[O_B2 + b];
#pragma unroll
    for (int a = 0; a < NH; ++a) s = fmaf(h1[a], sw[O_W2 + a * NH + b], s);
    if (a2) a2[b] = s;
    z = fmaf(fmaxf(s, 0.0f), sw[O_W3 + b], z);
  }
  return z;
}

__device__ inline bool row_active(const float* f) {
  // zero-mass rows have all-zero features (a real row has the diagonal entry 1)
  return f[13] != 0.0f;
}

// omega per row (internal order) and the Jacobi weights omega / A_ii
template <class WT>
__global__ __launch_bounds__(BLK) void k_mlp_omega(const float* feat, long long n, const WT* w, int l1,
                                                   const double* invd, double* omega, double* winvd64,
                                                   float* winvd32) {
  __shared__ float sw[NP];
  load_weights<WT>(w, sw);
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  float f[NF];
#pragma unroll
  for (int q = 0; q < NF; ++q) f[q] = feat[i * FSTRIDE + q];
  double om = 0.0;
  if (row_active(f)) {
    const float z = mlp_row(sw, f, nullptr, nullptr);
    // Jacobi: omega = c 2 sigmoid(z); SOR: omega = 1/2 + sigmoid(z), a band around Gauss-Seidel
    om = l1 ? (double)feat[i * FSTRIDE + C_L1] * (2.0 / (1.0 + exp(-(double)z)))
            : 0.5 + 1.0 / (1.0 + exp(-(double)z));
  }
  if (omega) omega[i] = om;
  if (winvd64) winvd64[i] = om * invd[i];
  if (winvd32) winvd32[i] = fabs(om * invd[i]) < 3.0e38 ? (float)(om * invd[i]) : 0.0f;
}

// per-row back-propagation: dz -> hidden deltas (recomputing the forward)
template <class WT>
__global__ __launch_bounds__(BLK) void k_mlp_backward_rows(const float* feat, long long n, const WT* w,
                                                           const double* dz, float* h1o, float* h2o, float* d1o,
                                                           float* d2o) {
  __shared__ float sw[NP];
  load_weights<WT>(w, sw);
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  float f[NF], a1[NH], a2[NH];
#pragma unroll
  for (int q = 0; q < NF; ++q) f[q] = feat[i * FSTRIDE + q];
  const bool act = row_active(f);
  mlp_row(sw, f, a1, a2);
  const float g = act ? (float)dz[i] : 0.0f;
  float d2[NH];
#pragma unroll
  for (int b = 0; b < NH; ++b) {
    d2[b] = a2[b] > 0.0f ? g * sw[O_W3 + b] : 0.0f;
    h2o[i * NH + b] = fmaxf(a2[b], 0.0f);
    d2o[i * NH + b] = d2[b];
  }
#pragma unroll
  for (int a = 0; a < NH; ++a) {
    float s = 0.0f;
#pragma unroll
    for (int b = 0; b < NH; ++b) s = fmaf(sw[O_W2 + a * NH + b], d2[b], s);
    h1o[i * NH + a] = fmaxf(a1[a], 0.0f);
    d1o[i * NH + a] = a1[a] > 0.0f ? s : 0.0f;
  }
}

// parameter gradients: each block sums GROWS rows, staged CH rows at a time
// in LDS (features, both hidden layers' activations and deltas, dz), then one
// FP64 atomic per parameter and block
constexpr int GROWS = 512;
constexpr int CH = 64;
constexpr int KS = 4;       // error samples (columns) per depth in the loss
__global__ __launch_bounds__(BLK) void k_param_grad(const float* feat, const float* h1, const float* h2,
                                                    const float* d1, const float* d2, const double* dz,
                                                    long long n, double* grad) {
  __shared__ float sf[CH][NF + 1], sh1[CH][NH + 1], sh2[CH][NH + 1], sd1[CH][NH + 1], sd2[CH][NH + 1];
  __shared__ float sdz[CH];
  const long long r0 = blockIdx.x * (long long)GROWS;
  const long long r1 = min(n, r0 + GROWS);
  double acc[(NP + BLK - 1) / BLK];
#pragma unroll
  for (int u = 0; u < (NP + BLK - 1) / BLK; ++u) acc[u] = 0.0;
  for (long long c0 = r0; c0 < r1; c0 += CH) {
    const int cn = (int)min((long long)CH, r1 - c0);
    for (int e = threadIdx.x; e < CH * NH; e += BLK) {
      const int r = e / NH, j = e % NH;
      const bool ok = r < cn;
      const long long g = c0 + r;
      if (j < NF) sf[r][j] = ok ? feat[g * FSTRIDE + j] : 0.0f;
      sh1[r][j] = ok ? h1[g * NH + j] : 0.0f;
      sh2[r][j] = ok ? h2[g * NH + j] : 0.0f;
      sd1[r][j] = ok ? d1[g * NH + j] : 0.0f;
      sd2[r][j] = ok ? d2[g * NH + j] : 0.0f;
    }
    for (int r = threadIdx.x; r < CH; r += BLK) sdz[r] = r < cn ? (float)dz[c0 + r] : 0.0f;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < (NP + BLK - 1) / BLK; ++u) {
      const int p = threadIdx.x + u * BLK;
      if (p >= NP) continue;
      float s = 0.0f;
      if (p < O_B1) {
        const int i = p / NH, j = p % NH;
        for (int r = 0; r < cn; ++r) s = fmaf(sf[r][i], sd1[r][j], s);
      } else if (p < O_W2) {
        const int j = p - O_B1;
        for (int r = 0; r < cn; ++r) s += sd1[r][j];
      } else if (p < O_B2) {
        const int a = (p - O_W2) / NH, bq = (p - O_W2) % NH;
        for (int r = 0; r < cn; ++r) s = fmaf(sh1[r][a], sd2[r][bq], s);
      } else if (p < O_W3) {
        const int j = p - O_B2;
        for (int r = 0; r < cn; ++r) s += sd2[r][j];
      } else if (p < O_B3) {
        const int j = p - O_W3;
        for (int r = 0; r < cn; ++r) s = fmaf(sh2[r][j], sdz[r], s);
      } else {
        for (int r = 0; r < cn; ++r) s += sdz[r];
      }
      acc[u] += (double)s;
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < (NP + BLK - 1) / BLK; ++u) {
    const int p = threadIdx.x + u * BLK;
    if (p < NP) atomicAdd(grad + p, acc[u]);
  }
}

__global__ void k_adam(float* w, const double* g, double scale, float* m, float* v, int np, float lr, float b1,
                       float b2, float eps, int step) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const float gi = (float)(g[i] * scale);
  m[i] = b1 * m[i] + (1.0f - b1) * gi;
  v[i] = b2 * v[i] + (1.0f - b2) * gi * gi;
  const float mh = m[i] / (1.0f - powf(b1, (float)step));
  const float vh = v[i] / (1.0f - powf(b2, (float)step));
  w[i] -= lr * mh / (sqrtf(vh) + eps);
}

// ------------------------------------------------------------- sweeps
// counter-based normal samples: splitmix64 of (seed, index), Box-Muller
__device__ inline unsigned long long splitmix64(unsigned long long x) {
  x += 0x9e3779b97f4a7c15ULL;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
  return x ^ (x >> 31);
}
__global__ void k_rand_normal(unsigned long long seed, long long m, double* out) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= m) return;
  const unsigned long long a = splitmix64(seed ^ splitmix64(2 * (unsigned long long)i));
  const unsigned long long b = splitmix64(seed ^ splitmix64(2 * (unsigned long long)i + 1));
  const double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740993.0);
  const double u2 = (b >> 11) * (1.0 / 9007199254740992.0);
  out[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// rows [r0, r1) relax: u = invd * y, e_out = e_in - omega * u; other rows
// keep e and get u = 0
template <int K>
__global__ void k_jac_fwd(long long n, long long r0, long long r1, const double* invd, const double* om,
                          const double* y, const double* e_in, double* u, double* e_out) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  const bool in = i >= r0 && i < r1;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const double uv = in ? invd[i] * y[i * K + q] : 0.0;
    u[i * K + q] = uv;
    e_out[i * K + q] = e_in[i * K + q] - (in ? om[i] * uv : 0.0);
  }
}
// g = coef_q * y (per column)
template <int K>
__global__ void k_scale_cols(long long n, const double* coef, const double* y, double* g) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int q = 0; q < K; ++q) g[i * K + q] = coef[q] * y[i * K + q];
}
// rows [r0, r1): gomega -= sum_q g * u and v = invd * omega * g; v = 0 elsewhere
template <int K>
__global__ void k_adj(long long n, long long r0, long long r1, const double* invd, const double* om,
                      const double* g, const double* u, double* gom, double* v) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  const bool in = i >= r0 && i < r1;
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    s += g[i * K + q] * u[i * K + q];
    v[i * K + q] = in ? invd[i] * om[i] * g[i * K + q] : 0.0;
  }
  if (in) gom[i] -= s;
}
template <int K>
__global__ void k_sub(long long n, double* g, const double* y) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n * K) g[i] -= y[i];
}
// Jacobi: omega = c s, s = 2 sigmoid(z): d omega / dz = c s (1 - s / 2) = omega (1 - s / 2)
// SOR: omega = 1/2 + sigma, sigma = sigmoid(z): d omega / dz = sigma (1 - sigma)
__global__ void k_dz(long long n, const double* gom, const double* om, const float* feat, int l1, double* dz) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  if (l1) {
    const double c = (double)feat[i * FSTRIDE + C_L1];
    const double sg = c > 0.0 ? om[i] / c : 0.0;
    dz[i] = gom[i] * om[i] * (1.0 - 0.5 * sg);
  } else {
    const double sg = om[i] > 0.0 ? om[i] - 0.5 : 0.0;
    dz[i] = gom[i] * sg * (1.0 - sg);
  }
}
// column sums of squares (one block per column block, FP64 atomics per block)
template <int K>
__global__ void k_colnorm2(long long n, const double* y, double* out) {
  __shared__ double sh[BLK];
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  for (int q = 0; q < K; ++q) {
    double v = i < n ? y[i * K + q] * y[i * K + q] : 0.0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = BLK / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out + q, sh[0]);
    __syncthreads();
  }
}
template <int K>
__global__ void k_gather_cols(const double* src, long long n, int kk, const int* iperm, double* dst) {
  long long f = blockIdx.x * (long long)BLK + threadIdx.x;
  if (f >= n) return;
  const int i = iperm[f];
#pragma unroll
  for (int q = 0; q < K; ++q) dst[(long long)i * K + q] = q < kk ? src[(long long)q * n + f] : 0.0;
}
__global__ void k_fill_d(double* p, long long n, double v) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f(float* p, long long n, float v) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n) p[i] = v;
}
// out[perm[i]] = v[i]: internal order to canonical order
__global__ void k_scatter_canon(const double* v, long long n, const int* perm, double* out) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n) out[perm[i]] = v[i];
}
// columns [c0, KS) of the n x KS row-major src into dst
__global__ void k_take_cols(const double* src, long long n, int c0, double* dst) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  for (int q = c0; q < KS; ++q) dst[i * KS + q] = src[i * KS + q];
}
inline unsigned long long splitmix64_host(unsigned long long x) {
  x += 0x9e3779b97f4a7c15ULL;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
  return x ^ (x >> 31);
}

// y = A x on the rows of slices [s0, s0 + ns) at depth d, FP64, K columns
// (SELL, plain one-row-per-thread loop)
template <int K>
__global__ void k_apply_sell(const int* sl_ptr, const int* row0, const int* rows, long long s0, long long ns,
                             const int* scol, const double* sval, const double* x, double* y) {
  long long g = blockIdx.x * (long long)BLK + threadIdx.x;
  if (g / SL >= ns) return;
  long long s = s0 + g / SL;
  int lane = (int)(g % SL);
  if (lane >= rows[s]) return;
  const int w = (sl_ptr[s + 1] - sl_ptr[s]) / SL;
  const long long base = sl_ptr[s] + lane;
  double acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0.0;
  for (int j = 0; j < w; ++j) {
    const double a = sval[base + (long long)j * SL];
    const int c = scol[base + (long long)j * SL];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = fma(a, x[(long long)c * K + q], acc[q]);
  }
  const int i = row0[s] + lane;
#pragma unroll
  for (int q = 0; q < K; ++q) y[(long long)i * K + q] = acc[q];
}

// round-to-nearest-even to BF16 (the 16 high bits of the FP32 pattern)
__global__ void k_to_bf16(const float* w, int n, uint16_t* h) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t u = __float_as_uint(w[i]);
  if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
  h[i] = (uint16_t)(u >> 16);
}

__global__ void k_scale_invd(const double* invd, long long n, double omega, double* w64, float* w32) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  w64[i] = omega * invd[i];
  w32[i] = fabs(omega * invd[i]) < 3.0e38 ? (float)(omega * invd[i]) : 0.0f;
}

// ------------------------------------------------------------ host side
template <class T>
void need(DArr<T>& a, size_t n) {
  if (a.n < n) a.alloc(n);
}

void features(camfe_sys s, SolverState* S, int d, DArr<float>& feat) {
  camfe_ctx ctx = s->h->ctx;
  const GLevel& G = S->lev[d];
  const SLevel& L = s->lev[d];
  const HLevel& H = s->h->lev[d];
  CAMFE_REQUIRE(s->h->degree == 1, CAMFE_EINVAL, "the learned smoother is defined for degree 1 (27-point stencils)");
  DArr<unsigned long long> mx(1);
  zero(ctx, mx.p, 1);
  hipLaunchKernelGGL(k_max_diag, 64, BLK, 0, ctx->stream, G.invd64.p, (long long)G.n, mx.p);
  check_launch();
  unsigned long long bits = read_scalar(ctx, mx.p);
  double maxdiag;
  std::memcpy(&maxdiag, &bits, 8);
  if (!(maxdiag > 0)) maxdiag = 1.0;
  feat.alloc(G.n * FSTRIDE);
  hipLaunchKernelGGL(k_features, grid_for(G.n, BLK), BLK, 0, ctx->stream, L.ptr.p, L.col.p, L.M.p, L.L.p, S->t,
                     H.fkey.p, G.perm.p, (long long)G.n, maxdiag, (float)(s->h->D - d), feat.p);
  check_launch();
}

// one MLP's weights on the device: FP32 master copy and its BF16 rounding
struct WView {
  const float* f = nullptr;
  const uint16_t* h = nullptr;
  bool bf16 = true;
};

struct DevWeights {
  DArr<float> f;
  DArr<uint16_t> h;
  WView upload(camfe_ctx ctx, const float* w, bool use_bf16) {
    need(f, NP);
    need(h, NP);
    copy_in(ctx, f.p, w, NP);
    hipLaunchKernelGGL(k_to_bf16, grid_for(NP, BLK), BLK, 0, ctx->stream, (const float*)f.p, NP, h.p);
    check_launch();
    WView v;
    v.f = f.p;
    v.h = h.p;
    v.bf16 = use_bf16;
    return v;
  }
};

void mlp_omega(camfe_ctx ctx, const float* feat, size_t n, const WView& W, bool l1, const double* invd,
               double* omega, double* w64, float* w32) {
  if (W.bf16)
    hipLaunchKernelGGL(k_mlp_omega<uint16_t>, grid_for(n, BLK), BLK, 0, ctx->stream, feat, (long long)n, W.h,
                       l1 ? 1 : 0, invd, omega, w64, w32);
  else
    hipLaunchKernelGGL(k_mlp_omega<float>, grid_for(n, BLK), BLK, 0, ctx->stream, feat, (long long)n, W.f,
                       l1 ? 1 : 0, invd, omega, w64, w32);
  check_launch();
}

// Work vectors of the loss and gradient, grown on demand and reused
struct GradWork {
  DArr<double> om, gom, dz, e, u, y, g, v, coef, nrm;
  DArr<float> h1, h2, d1, d2;
  std::vector<double> hn;
};

}  // namespace
void coarse_correction(SolverState* S, int d, const double* e, double* out, bool adjoint);   // solve.hip
namespace {

// Loss of one depth for the samples E0 (internal order, n x KS row-major, the
// columns from kk on zero) and, when grad is given, dL/dparams added to grad
// (device, NP doubles).  Returns the loss (mean over the kk samples).  sweep 0:
// nu damped Jacobi sweeps with l1-bounded weights; sweep 1: nu multicolour SOR
// sweeps, one relaxation step per colour (rows of one colour are contiguous in
// the internal order and do not couple).  cycle = 0: the nu sweeps alone;
// cycle = 1: a two-grid cycle, nu pre-sweeps (colours forward), the coarse
// correction e - P B_c P^T A e with B_c the plain V-cycle one depth down
// (needs d > d0), nu post-sweeps (colours reversed).
double loss_grad_level(camfe_ctx ctx, SolverState* S, int d, const float* feat, const WView& W, int sweep, int nu,
                       int cycle, const double* E0, int kk, double* grad, GradWork& w) {
  const GLevel& G = S->lev[d];
  const size_t n = G.n;
  const int K = KS;
  const unsigned gn = grid_for(n, BLK);
  struct Step { int cc; long long r0, r1, s0, s1; };
  std::vector<Step> steps;
  auto sweeps = [&](bool forward) {
    for (int it = 0; it < nu; ++it) {
      if (sweep == 0) {
        steps.push_back({0, 0, (long long)n, 0, (long long)G.nslices});
      } else {
        for (int ci = 0; ci < G.ncol; ++ci) {
          const int c = forward ? ci : G.ncol - 1 - ci;
          steps.push_back({0, G.coff[c], G.coff[c + 1], G.cslice[c], G.cslice[c + 1]});
        }
      }
    }
  };
  sweeps(true);
  if (cycle) {
    CAMFE_REQUIRE(d > S->d0, CAMFE_EINVAL, "the two-grid loss needs a coarser depth");
    steps.push_back({1, 0, 0, 0, 0});
    sweeps(false);
  }
  const size_t ns = steps.size();
  need(w.om, n);
  need(w.gom, n);
  need(w.dz, n);
  need(w.e, n * K * (ns + 1));
  need(w.u, n * K * (ns > 0 ? ns : 1));
  need(w.y, n * K);
  need(w.g, n * K);
  need(w.v, n * K);
  need(w.coef, K);
  need(w.nrm, 2 * K);
  hipStream_t st = ctx->stream;
  mlp_omega(ctx, feat, n, W, sweep == 0, G.invd64.p, w.om.p, nullptr, nullptr);
  CAMFE_HIP(hipMemcpyAsync(w.e.p, E0, n * K * sizeof(double), hipMemcpyDeviceToDevice, st));
  auto apply_range = [&](long long s0, long long s1, const double* x, double* y) {
    if (s1 <= s0) return;
    hipLaunchKernelGGL(k_apply_sell<KS>, grid_for((size_t)(s1 - s0) * SL, BLK), BLK, 0, st, G.sl_ptr.p,
                       G.sl_row0.p, G.sl_rows.p, s0, s1 - s0, G.scol.p, G.sval64.p, x, y);
  };
  auto apply = [&](const double* x, double* y) { apply_range(0, (long long)G.nslices, x, y); };
  for (size_t k = 0; k < ns; ++k) {
    if (steps[k].cc) {
      coarse_correction(S, d, w.e.p + k * n * K, w.e.p + (k + 1) * n * K, false);
      continue;
    }
    apply_range(steps[k].s0, steps[k].s1, w.e.p + k * n * K, w.y.p);
    hipLaunchKernelGGL(k_jac_fwd<KS>, gn, BLK, 0, st, (long long)n, steps[k].r0, steps[k].r1, G.invd64.p,
                       (const double*)w.om.p, (const double*)w.y.p, (const double*)(w.e.p + k * n * K),
                       w.u.p + k * n * K, w.e.p + (k + 1) * n * K);
  }
  zero(ctx, w.nrm.p, 2 * K);
  apply(w.e.p, w.y.p);
  hipLaunchKernelGGL(k_colnorm2<KS>, gn, BLK, 0, st, (long long)n, (const double*)w.y.p, w.nrm.p);
  apply(w.e.p + ns * n * K, w.y.p);   // r = A e_final, kept in y for the backward pass
  hipLaunchKernelGGL(k_colnorm2<KS>, gn, BLK, 0, st, (long long)n, (const double*)w.y.p, w.nrm.p + K);
  check_launch();
  double nr[2 * KS];
  copy_out(ctx, nr, w.nrm.p, 2 * K);
  double loss = 0.0, coef[KS];
  for (int q = 0; q < K; ++q) {
    coef[q] = 0.0;
    if (q < kk) {
      loss += std::log(nr[K + q] / nr[q]) / kk;
      coef[q] = 2.0 / kk / nr[K + q];
    }
  }
  if (!grad) return loss;
  // adjoint: g_nu = coef A r; per sweep k (last first) gomega -= g_{k+1} u_k and
  // g_k = g_{k+1} - A (D^-1 omega g_{k+1})
  copy_in(ctx, w.coef.p, coef, K);
  apply(w.y.p, w.v.p);
  hipLaunchKernelGGL(k_scale_cols<KS>, gn, BLK, 0, st, (long long)n, (const double*)w.coef.p, (const double*)w.v.p,
                     w.g.p);
  hipLaunchKernelGGL(k_fill_d, gn, BLK, 0, st, w.gom.p, (long long)n, 0.0);
  for (long long k = (long long)ns - 1; k >= 0; --k) {
    if (steps[k].cc) {
      // g <- (I - P B_c P^T A)^T g = g - A P B_c P^T g
      coarse_correction(S, d, w.g.p, w.v.p, true);
      CAMFE_HIP(hipMemcpyAsync(w.g.p, w.v.p, n * K * sizeof(double), hipMemcpyDeviceToDevice, st));
      continue;
    }
    hipLaunchKernelGGL(k_adj<KS>, gn, BLK, 0, st, (long long)n, steps[k].r0, steps[k].r1, G.invd64.p,
                       (const double*)w.om.p, (const double*)w.g.p, (const double*)(w.u.p + k * n * K), w.gom.p,
                       w.v.p);
    if (k > 0) {
      apply(w.v.p, w.y.p);
      hipLaunchKernelGGL(k_sub<KS>, grid_for(n * K, BLK), BLK, 0, st, (long long)n, w.g.p, (const double*)w.y.p);
    }
  }
  hipLaunchKernelGGL(k_dz, gn, BLK, 0, st, (long long)n, (const double*)w.gom.p, (const double*)w.om.p, feat,
                     sweep == 0 ? 1 : 0, w.dz.p);
  need(w.h1, n * NH);
  need(w.h2, n * NH);
  need(w.d1, n * NH);
  need(w.d2, n * NH);
  if (W.bf16)
    hipLaunchKernelGGL(k_mlp_backward_rows<uint16_t>, gn, BLK, 0, st, feat, (long long)n, W.h, (const double*)w.dz.p,
                       w.h1.p, w.h2.p, w.d1.p, w.d2.p);
  else
    hipLaunchKernelGGL(k_mlp_backward_rows<float>, gn, BLK, 0, st, feat, (long long)n, W.f, (const double*)w.dz.p,
                       w.h1.p, w.h2.p, w.d1.p, w.d2.p);
  hipLaunchKernelGGL(k_param_grad, (unsigned)((n + GROWS - 1) / GROWS), BLK, 0, st, feat, (const float*)w.h1.p,
                     (const float*)w.h2.p, (const float*)w.d1.p, (const float*)w.d2.p, (const double*)w.dz.p,
                     (long long)n, grad);
  check_launch();
  return loss;
}

}  // namespace

SolverState* ensure_solver(camfe_sys s, double t, double coarse_eps);                   // solve.hip
void plain_vcycle_at(SolverState* S, int d, double* x, int nu1, int nu2);              // solve.hip, n x 4, b = 0

void set_smoother_weights(camfe_sys s, SolverState* S, int smoother, double omega, const void* model) {
  camfe_ctx ctx = s->h->ctx;
  DevWeights W;
  for (int d = S->d0; d <= S->D; ++d) {
    GLevel& G = S->lev[d];
    need(G.winvd64, G.n);
    need(G.winvd32, G.n);
    if (smoother == 1) {
      hipLaunchKernelGGL(k_scale_invd, grid_for(G.n, BLK), BLK, 0, ctx->stream, G.invd64.p, (long long)G.n, omega,
                         G.winvd64.p, G.winvd32.p);
      check_launch();
    } else {
      const camfe_model_s* m = (const camfe_model_s*)model;
      const int l = std::min(S->D - d, m->levels - 1);
      DArr<float> feat;
      features(s, S, d, feat);
      WView v = W.upload(ctx, m->w.data() + (size_t)l * NP, m->bf16 != 0);
      mlp_omega(ctx, feat.p, G.n, v, m->sweep == 0, G.invd64.p, nullptr, G.winvd64.p, G.winvd32.p);
      ctx->sync();
    }
  }
  ctx->sync();
  S->wkind = smoother;
  S->wsweep = smoother == 2 ? ((const camfe_model_s*)model)->sweep : 0;
  S->omega = omega;
  S->model = model;
  S->drop_graphs();
}

}  // namespace camfe

using namespace camfe;

extern "C" {

camfe_status camfe_model_create(const float* params, int levels, int bf16, int sweep, camfe_model* out) {
  return guarded([&] {
    CAMFE_REQUIRE(out && levels >= 1 && levels <= 32 && (sweep == 0 || sweep == 1), CAMFE_EINVAL, "bad argument");
    std::unique_ptr<camfe_model_s> m(new camfe_model_s());
    m->levels = levels;
    m->bf16 = bf16 ? 1 : 0;
    m->sweep = sweep;
    m->w.assign((size_t)levels * NP, 0.0f);
    if (params) {
      std::memcpy(m->w.data(), params, m->w.size() * sizeof(float));
    } else {
      // uniform (He-scaled) weights from a fixed LCG, zero biases, and w3 small
      // so that s = 2 sigmoid(z) starts near 1 (plain l1-Jacobi)
      uint64_t st = 0x1234567ULL;
      auto urand = [&]() {
        st = st * 6364136223846793005ULL + 1442695040888963407ULL;
        return ((st >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
      };
      for (int l = 0; l < levels; ++l) {
        float* w = m->w.data() + (size_t)l * NP;
        for (int i = 0; i < NF * NH; ++i) w[O_W1 + i] = (float)(urand() * std::sqrt(6.0 / NF));
        for (int i = 0; i < NH * NH; ++i) w[O_W2 + i] = (float)(urand() * std::sqrt(6.0 / NH));
        for (int i = 0; i < NH; ++i) w[O_W3 + i] = (float)(urand() * 0.1);
        w[O_B3] = 0.0f;
      }
    }
    *out = m.release();
  });
}

camfe_status camfe_model_params(camfe_model m, float* params, int64_t cap, int64_t* n, int* levels, int* bf16,
                                int* sweep) {
  return guarded([&] {
    CAMFE_REQUIRE(m, CAMFE_EINVAL, "null model");
    if (n) *n = (int64_t)m->w.size();
    if (levels) *levels = m->levels;
    if (bf16) *bf16 = m->bf16;
    if (sweep) *sweep = m->sweep;
    if (cap == 0) return;
    CAMFE_REQUIRE(params && cap >= (int64_t)m->w.size(), CAMFE_ETOOSMALL, "export capacity too small");
    std::memcpy(params, m->w.data(), m->w.size() * sizeof(float));
  });
}

void camfe_model_destroy(camfe_model m) { delete m; }

// File record: tag, four little-endian int32 (levels, bf16, sweep, NP), then
// levels * NP little-endian FP32.  This library targets little-endian hosts
// only (x86-64), so the in-memory order is the file order.
static const char MODEL_TAG[8] = {'C', 'A', 'M', 'F', 'E', 'S', 'M', '1'};

camfe_status camfe_smoother_save(camfe_model m, const char* path) {
  return guarded([&] {
    CAMFE_REQUIRE(m && path, CAMFE_EINVAL, "null model or path");
    std::FILE* f = std::fopen(path, "wb");
    CAMFE_REQUIRE(f, CAMFE_EDEVICE, std::string("cannot open ") + path + " for writing");
    const int32_t head[4] = {m->levels, m->bf16, m->sweep, NP};
    bool ok = std::fwrite(MODEL_TAG, 1, 8, f) == 8 && std::fwrite(head, sizeof(int32_t), 4, f) == 4 &&
              std::fwrite(m->w.data(), sizeof(float), m->w.size(), f) == m->w.size();
    ok = (std::fclose(f) == 0) && ok;
    CAMFE_REQUIRE(ok, CAMFE_EDEVICE, std::string("writing ") + path + " failed");
  });
}

camfe_status camfe_smoother_load(const char* path, camfe_model* out) {
  return guarded([&] {
    CAMFE_REQUIRE(path && out, CAMFE_EINVAL, "null path or output handle");
    std::FILE* f = std::fopen(path, "rb");
    CAMFE_REQUIRE(f, CAMFE_EINVAL, std::string("cannot open ") + path);
    std::unique_ptr<std::FILE, int (*)(std::FILE*)> guard(f, std::fclose);
    char tag[8];
    int32_t head[4];
    CAMFE_REQUIRE(std::fread(tag, 1, 8, f) == 8 && std::memcmp(tag, MODEL_TAG, 8) == 0, CAMFE_EINVAL,
                  "not a smoother model file");
    CAMFE_REQUIRE(std::fread(head, sizeof(int32_t), 4, f) == 4, CAMFE_EINVAL, "truncated model header");
    CAMFE_REQUIRE(head[0] >= 1 && head[0] <= 32 && (head[1] == 0 || head[1] == 1) &&
                      (head[2] == 0 || head[2] == 1) && head[3] == NP,
                  CAMFE_EINVAL, "model header out of range");
    std::vector<float> w((size_t)head[0] * NP);
    CAMFE_REQUIRE(std::fread(w.data(), sizeof(float), w.size(), f) == w.size(), CAMFE_EINVAL,
                  "model file shorter than its header says");
    char extra;
    CAMFE_REQUIRE(std::fread(&extra, 1, 1, f) == 0, CAMFE_EINVAL, "model file longer than its header says");
    camfe_model m = nullptr;
    camfe_status rc = camfe_model_create(w.data(), head[0], head[1], head[2], &m);
    if (rc != CAMFE_OK) throw Error(rc, "model creation failed");
    *out = m;
  });
}

camfe_status camfe_smoother_attach(camfe_sys s, camfe_model m) {
  return guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s, CAMFE_EINVAL, "null system");
    CAMFE_REQUIRE(!m || s->h->degree == 1, CAMFE_EINVAL, "the learned smoother is defined for degree 1");
    s->model = m;
    if (s->solver) s->solver->model = nullptr;   // weights are recomputed at the next solve
  });
}

camfe_status camfe_smoother_omega(camfe_sys s, camfe_model m, int depth, double t, double* omega) {
  return guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s && m && omega, CAMFE_EINVAL, "bad argument");
    camfe_hier h = s->h;
    CAMFE_REQUIRE(depth >= h->d0 && depth <= h->D, CAMFE_ESTATE, "depth not assembled");
    camfe_ctx ctx = h->ctx;
    ctx->use_device();
    SolverState* S = ensure_solver(s, t, DEFAULT_COARSE_EPS);
    const GLevel& G = S->lev[depth];
    DArr<float> feat;
    features(s, S, depth, feat);
    DevWeights W;
    const int l = std::min(S->D - depth, m->levels - 1);
    WView v = W.upload(ctx, m->w.data() + (size_t)l * NP, m->bf16 != 0);
    DArr<double> om(G.n), out(G.n);
    mlp_omega(ctx, feat.p, G.n, v, m->sweep == 0, G.invd64.p, om.p, nullptr, nullptr);
    hipLaunchKernelGGL(k_scatter_canon, grid_for(G.n, BLK), BLK, 0, ctx->stream, (const double*)om.p,
                       (long long)G.n, G.perm.p, out.p);
    check_launch();
    copy_out(ctx, omega, out.p, G.n);
  });
}

camfe_status camfe_smoother_loss_grad(camfe_sys s, int depth, double t, const float* params, int bf16, int sweep,
                                      int cycle, const double* e0, int nsamples, int nu, double* loss,
                                      double* grad) {
  return guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s && params && e0 && loss && nsamples >= 1 && nsamples <= KS && nu >= 0 &&
                      (sweep == 0 || sweep == 1) && (cycle == 0 || cycle == 1),
                  CAMFE_EINVAL, "bad argument");
    camfe_hier h = s->h;
    CAMFE_REQUIRE(depth >= h->d0 && depth <= h->D, CAMFE_ESTATE, "depth not assembled");
    camfe_ctx ctx = h->ctx;
    ctx->use_device();
    SolverState* S = ensure_solver(s, t, DEFAULT_COARSE_EPS);
    const GLevel& G = S->lev[depth];
    DArr<float> feat;
    features(s, S, depth, feat);
    DevWeights W;
    WView v = W.upload(ctx, params, bf16 != 0);
    DArr<double> e0c(G.n * (size_t)nsamples), E(G.n * KS);
    copy_in(ctx, e0c.p, e0, e0c.n);
    hipLaunchKernelGGL(k_gather_cols<KS>, grid_for(G.n, BLK), BLK, 0, ctx->stream, (const double*)e0c.p,
                       (long long)G.n, nsamples, G.iperm.p, E.p);
    DArr<double> gd(NP);
    zero(ctx, gd.p, NP);
    GradWork w;
    CAMFE_REQUIRE(!cycle || depth > S->d0, CAMFE_ESTATE, "the two-grid loss needs a depth above the coarsest");
    *loss = loss_grad_level(ctx, S, depth, feat.p, v, sweep, nu, cycle, E.p, nsamples, grad ? gd.p : nullptr, w);
    if (grad) copy_out(ctx, grad, gd.p, NP);
  });
}

camfe_status camfe_smoother_train(camfe_ctx ctx, camfe_sys const* systems, int nsys, const camfe_train_opts* o,
                                  camfe_model* out, double* loss_history) {
  return guarded([&] {
    if (ctx) set_current_ctx(ctx);
    CAMFE_REQUIRE(ctx && systems && nsys >= 1 && o && out, CAMFE_EINVAL, "bad argument");
    CAMFE_REQUIRE(o->levels >= 1 && o->levels <= 32 && o->steps >= 0 && o->nu >= 1 && o->lr > 0 &&
                      o->samples >= 0 && o->samples <= 2 && (o->sweep == 0 || o->sweep == 1) &&
                      (o->cycle == 0 || o->cycle == 1),
                  CAMFE_EINVAL, "bad options");
    for (int i = 0; i < nsys; ++i) {
      const double ti = o->t_each ? o->t_each[i] : o->t;
      CAMFE_REQUIRE(ti >= 0.0 && std::isfinite(ti), CAMFE_EINVAL, "t must be finite and >= 0");
      if (o->t_each)   // one solver state per system: a repeated system cannot take two t
        for (int j = 0; j < i; ++j) CAMFE_REQUIRE(systems[j] != systems[i], CAMFE_EINVAL, "repeated system");
    }
    ctx->use_device();
    camfe_model m0 = nullptr;
    camfe_status rc = camfe_model_create(nullptr, o->levels, o->bf16, o->sweep, &m0);
    if (rc != CAMFE_OK) throw Error(rc, "model creation failed");
    std::unique_ptr<camfe_model_s> mp(m0);
    // per (system, depth above the coarsest): features and KS error samples,
    // each the error that one plain Gauss-Seidel V-cycle leaves from a random start
    struct Item {
      SolverState* S;
      int d, l;
      DArr<float> feat;
      DArr<double> E;
    };
    std::vector<std::unique_ptr<Item>> items;
    unsigned long long seed = o->seed;
    for (int i = 0; i < nsys; ++i) {
      camfe_sys s = systems[i];
      CAMFE_REQUIRE(s && s->h->ctx == ctx, CAMFE_EINVAL, "systems must belong to the context");
      CAMFE_REQUIRE(s->h->degree == 1, CAMFE_EINVAL, "the learned smoother is defined for degree 1");
      SolverState* S = ensure_solver(s, o->t_each ? o->t_each[i] : o->t, DEFAULT_COARSE_EPS);
      const int saved = S->smoother;
      S->smoother = 0;
      for (int d = S->d0 + 1; d <= S->D; ++d) {
        std::unique_ptr<Item> it(new Item());
        it->S = S;
        it->d = d;
        it->l = std::min(S->D - d, o->levels - 1);
        features(s, S, d, it->feat);
        const GLevel& G = S->lev[d];
        it->E.alloc(G.n * KS);
        hipLaunchKernelGGL(k_rand_normal, grid_for(G.n * KS, BLK), BLK, 0, ctx->stream,
                           splitmix64_host(seed + 0x1000ULL * i + d), (long long)(G.n * KS), it->E.p);
        check_launch();
        if (o->samples == 1) {
          plain_vcycle_at(S, d, it->E.p, 2, 2);
        } else if (o->samples == 2) {
          DArr<double> tmp(G.n * KS);
          CAMFE_HIP(hipMemcpyAsync(tmp.p, it->E.p, tmp.bytes(), hipMemcpyDeviceToDevice, ctx->stream));
          plain_vcycle_at(S, d, tmp.p, 2, 2);
          hipLaunchKernelGGL(k_take_cols, grid_for(G.n, BLK), BLK, 0, ctx->stream, (const double*)tmp.p,
                             (long long)G.n, 2, it->E.p);
          check_launch();
          ctx->sync();
        }
        items.push_back(std::move(it));
      }
      S->smoother = saved;
      S->drop_graphs();
    }
    ctx->sync();
    CAMFE_REQUIRE(!items.empty(), CAMFE_EINVAL, "no depth above the coarsest to train on");
    const int L = o->levels;
    const size_t np = (size_t)L * NP;
    DArr<float> wdev(np), mom(np), vel(np);
    DArr<uint16_t> wbf(np);
    copy_in(ctx, wdev.p, mp->w.data(), np);
    hipLaunchKernelGGL((k_fill_f), grid_for(np, BLK), BLK, 0, ctx->stream, mom.p, (long long)np, 0.0f);
    hipLaunchKernelGGL((k_fill_f), grid_for(np, BLK), BLK, 0, ctx->stream, vel.p, (long long)np, 0.0f);
    DArr<double> grad(np);
    std::vector<int> cnt(L, 0);
    for (auto& it : items) cnt[it->l]++;
    GradWork w;
    for (int step = 1; step <= o->steps; ++step) {
      hipLaunchKernelGGL(k_fill_d, grid_for(np, BLK), BLK, 0, ctx->stream, grad.p, (long long)np, 0.0);
      hipLaunchKernelGGL(k_to_bf16, grid_for(np, BLK), BLK, 0, ctx->stream, (const float*)wdev.p, (int)np, wbf.p);
      check_launch();
      double tot = 0.0;
      for (auto& it : items) {
        WView v;
        v.f = wdev.p + (size_t)it->l * NP;
        v.h = wbf.p + (size_t)it->l * NP;
        v.bf16 = o->bf16 != 0;
        tot += loss_grad_level(ctx, it->S, it->d, it->feat.p, v, o->sweep, o->nu, o->cycle, it->E.p, KS,
                               grad.p + (size_t)it->l * NP, w);
      }
      if (loss_history) loss_history[step - 1] = tot / items.size();
      for (int l = 0; l < L; ++l)
        if (cnt[l])
          hipLaunchKernelGGL(k_adam, grid_for(NP, BLK), BLK, 0, ctx->stream, wdev.p + (size_t)l * NP,
                             (const double*)(grad.p + (size_t)l * NP), 1.0 / cnt[l], mom.p + (size_t)l * NP,
                             vel.p + (size_t)l * NP, NP, (float)o->lr, 0.9f, 0.999f, 1e-8f, step);
      check_launch();
    }
    copy_out(ctx, mp->w.data(), wdev.p, np);
    *out = mp.release();
  });
}

}  // extern "C"

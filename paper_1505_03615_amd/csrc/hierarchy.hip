// Hierarchy construction on the GPU: grid placement, triangle/cell pairs,
// octree aggregation, support lists, the connectivity-aware split and the
// prolongation of Eq. (4).
//
// Every floating-point predicate here is evaluated with plain IEEE adds and
// multiplies in a fixed order (the library is built with -ffp-contract=off),
// so the discrete structure is a deterministic function of the input.
#include <algorithm>
#include <map>
#include <mutex>
#include <string>

#include "internal.hpp"

namespace camfe {

namespace {

constexpr int BLK = 256;

// ------------------------------------------------------------ predicates
// Separating axis A for points P[0..np): the open box of half-size h at the
// origin projects to (-r, r) with r = h (|A0| + |A1| + |A2|); the axis
// separates (touching counts) iff min >= r or max <= -r.  Zero axes are skipped.
template <int NP>
__device__ inline bool axis_sep(double a0, double a1, double a2, const double (&P)[NP][3], double h) {
  if (a0 == 0.0 && a1 == 0.0 && a2 == 0.0) return false;
  double mn = 0.0, mx = 0.0;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    double p = a0 * P[i][0] + a1 * P[i][1] + a2 * P[i][2];
    if (i == 0 || p < mn) mn = p;
    if (i == 0 || p > mx) mx = p;
  }
  double r = h * (fabs(a0) + fabs(a1) + fabs(a2));
  return mn >= r || mx <= -r;
}

template <int NP>
__device__ inline bool box_cross_sep(const double (&P)[NP][3], const double f[3], double h) {
  if (axis_sep<NP>(1.0, 0.0, 0.0, P, h)) return true;
  if (axis_sep<NP>(0.0, 1.0, 0.0, P, h)) return true;
  if (axis_sep<NP>(0.0, 0.0, 1.0, P, h)) return true;
  if (axis_sep<NP>(0.0, -f[2], f[1], P, h)) return true;
  if (axis_sep<NP>(f[2], 0.0, -f[0], P, h)) return true;
  return axis_sep<NP>(-f[1], f[0], 0.0, P, h);
}

// triangle (translated to the box centre) meets the open box
__device__ inline bool tri_meets_box(const double (&v)[3][3], double h) {
  double f[3][3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int a = 0; a < 3; ++a) f[j][a] = v[(j + 1) % 3][a] - v[j][a];
  double n0 = f[0][1] * f[1][2] - f[0][2] * f[1][1];
  double n1 = f[0][2] * f[1][0] - f[0][0] * f[1][2];
  double n2 = f[0][0] * f[1][1] - f[0][1] * f[1][0];
  if (axis_sep<3>(n0, n1, n2, v, h)) return false;
#pragma unroll
  for (int j = 0; j < 3; ++j)
    if (box_cross_sep<3>(v, f[j], h)) return false;
  return true;
}

// closed segment (translated) meets the open box
__device__ inline bool seg_meets_box(const double P[3], const double Q[3], double h) {
  double pts[2][3] = {{P[0], P[1], P[2]}, {Q[0], Q[1], Q[2]}};
  double f[3] = {Q[0] - P[0], Q[1] - P[1], Q[2] - P[2]};
  return !box_cross_sep<2>(pts, f, h);
}

// support box of a support key at depth d (degree 1: corner k, [k-1, k+1]^3;
// degree 2: stored node S = o + 1, box [S-2, S+1]^3)
__device__ inline void support_box(int degree, u64 skey, double C[3], double* H) {
  long long c[3];
  demorton(skey, c);
#pragma unroll
  for (int a = 0; a < 3; ++a) C[a] = degree == 1 ? (double)c[a] : (double)c[a] - 0.5;
  *H = degree == 1 ? 1.0 : 1.5;
}

__device__ inline long long lower_bound_u64(const u64* a, long long lo, long long hi, u64 key) {
  while (lo < hi) {
    long long mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// ------------------------------------------------------------- grid placement
__global__ void k_minmax(const double* V, long long nv, double* part) {
  __shared__ double smn[3][BLK], smx[3][BLK];
  double mn[3] = {1e308, 1e308, 1e308}, mx[3] = {-1e308, -1e308, -1e308};
  for (long long v = blockIdx.x * (long long)BLK + threadIdx.x; v < nv; v += (long long)gridDim.x * BLK)
    for (int a = 0; a < 3; ++a) {
      double x = V[3 * v + a];
      mn[a] = fmin(mn[a], x);
      mx[a] = fmax(mx[a], x);
    }
  for (int a = 0; a < 3; ++a) { smn[a][threadIdx.x] = mn[a]; smx[a][threadIdx.x] = mx[a]; }
  __syncthreads();
  for (int s = BLK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int a = 0; a < 3; ++a) {
        smn[a][threadIdx.x] = fmin(smn[a][threadIdx.x], smn[a][threadIdx.x + s]);
        smx[a][threadIdx.x] = fmax(smx[a][threadIdx.x], smx[a][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int a = 0; a < 3; ++a) { part[6 * blockIdx.x + a] = smn[a][0]; part[6 * blockIdx.x + 3 + a] = smx[a][0]; }
}

// cube: side s = 1.125 x largest extent, centred; or the explicit box
__global__ void k_cube(const double* part, int nblk, int D, double bx, double by, double bz, double bs,
                       double* cube) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double o[3], s;
  if (bs > 0) {
    o[0] = bx; o[1] = by; o[2] = bz; s = bs;
  } else {
    double mn[3], mx[3];
    for (int a = 0; a < 3; ++a) { mn[a] = part[a]; mx[a] = part[3 + a]; }
    for (int b = 1; b < nblk; ++b)
      for (int a = 0; a < 3; ++a) {
        mn[a] = fmin(mn[a], part[6 * b + a]);
        mx[a] = fmax(mx[a], part[6 * b + 3 + a]);
      }
    double ext = fmax(fmax(mx[0] - mn[0], mx[1] - mn[1]), mx[2] - mn[2]);
    s = 1.125 * ext;
    for (int a = 0; a < 3; ++a) o[a] = (mn[a] + mx[a]) * 0.5 - s * 0.5;
  }
  cube[0] = o[0]; cube[1] = o[1]; cube[2] = o[2]; cube[3] = s;
  cube[4] = ldexp(1.0, D) / s;
}

enum { FLAG_OUTSIDE = 1, FLAG_INDEX = 2, FLAG_DEGEN = 4, FLAG_PLANE = 8, FLAG_CHI = 16, FLAG_NONFINITE = 32 };

__global__ void k_grid_coords(const double* V, long long nv, const double* cube, double N, double* U,
                              int* flag) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= 3 * nv) return;
  int a = (int)(i % 3);
  double x = V[i];
  double u = (x - cube[a]) * cube[4];
  if (!isfinite(x)) atomicOr(flag, FLAG_NONFINITE);
  if (!(u >= 0.0 && u <= N)) atomicOr(flag, FLAG_OUTSIDE);
  U[i] = u;
}

__global__ void k_tri_check(const int* F, long long nt, long long nv, const double* U, double* nrm,
                            int* flag) {
  long long t = blockIdx.x * (long long)BLK + threadIdx.x;
  if (t >= nt) return;
  int f0 = F[3 * t], f1 = F[3 * t + 1], f2 = F[3 * t + 2];
  if (f0 < 0 || f1 < 0 || f2 < 0 || f0 >= nv || f1 >= nv || f2 >= nv || f0 == f1 || f1 == f2 || f0 == f2) {
    atomicOr(flag, FLAG_INDEX);
    return;
  }
  const double* p0 = U + 3 * (long long)f0;
  const double* p1 = U + 3 * (long long)f1;
  const double* p2 = U + 3 * (long long)f2;
  double e0[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
  double e1[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
  double n[3] = {e0[1] * e1[2] - e0[2] * e1[1], e0[2] * e1[0] - e0[0] * e1[2], e0[0] * e1[1] - e0[1] * e1[0]};
  if (n[0] == 0.0 && n[1] == 0.0 && n[2] == 0.0) atomicOr(flag, FLAG_DEGEN);
  for (int a = 0; a < 3; ++a)
    if (p0[a] == p1[a] && p1[a] == p2[a] && floor(p0[a]) == p0[a]) atomicOr(flag, FLAG_PLANE);
  double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int a = 0; a < 3; ++a) nrm[3 * t + a] = n[a] / nn;
}

// --------------------------------------------------------- finest pairs
__device__ inline void tri_cells(const double* U, const int* F, long long t, long long top,
                                 const double* (&p)[3], long long lo[3], long long hi[3]) {
  for (int i = 0; i < 3; ++i) p[i] = U + 3 * (long long)F[3 * t + i];
  for (int a = 0; a < 3; ++a) {
    double mn = fmin(fmin(p[0][a], p[1][a]), p[2][a]);
    double mx = fmax(fmax(p[0][a], p[1][a]), p[2][a]);
    lo[a] = max(0LL, min(top, (long long)floor(mn)));
    hi[a] = max(0LL, min(top, (long long)floor(mx)));
  }
}

// WRITE = false: count the cells each triangle meets; true: write their keys
template <bool WRITE>
__global__ void k_pairs(const double* U, const int* F, long long nt, long long top, long long* cnt,
                        const long long* off, u64* out) {
  long long t = blockIdx.x * (long long)BLK + threadIdx.x;
  if (t >= nt) return;
  const double* p[3];
  long long lo[3], hi[3];
  tri_cells(U, F, t, top, p, lo, hi);
  long long c = 0, w = WRITE ? off[t] : 0;
  for (long long z = lo[2]; z <= hi[2]; ++z)
    for (long long y = lo[1]; y <= hi[1]; ++y)
      for (long long x = lo[0]; x <= hi[0]; ++x) {
        double cen[3] = {(double)x + 0.5, (double)y + 0.5, (double)z + 0.5};
        double v[3][3];
        for (int i = 0; i < 3; ++i)
          for (int a = 0; a < 3; ++a) v[i][a] = p[i][a] - cen[a];
        if (tri_meets_box(v, 0.5)) {
          if (WRITE) out[w++] = (morton((u64)x, (u64)y, (u64)z) << TRI_BITS) | (u64)t;
          else ++c;
        }
      }
  if (!WRITE) cnt[t] = c;
}

// ------------------------------------------------------------ unique / flags
__global__ void k_head_flags(const u64* k, long long n, int shift, int* flag) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  flag[i] = (i == 0 || (k[i] >> shift) != (k[i - 1] >> shift)) ? 1 : 0;
}
__global__ void k_compact_heads(const u64* k, const int* flag, const int* pos, long long n, u64* out) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  if (flag[i]) out[pos[i]] = k[i];
}
__global__ void k_parent_keys(const u64* in, long long n, u64* out) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  u64 k = in[i];
  out[i] = (((k >> TRI_BITS) >> 3) << TRI_BITS) | (k & TRI_MASK);
}

// --------------------------------------------------------- support entries
// (support, triangle) candidates of the pairs taken in triangle order
// (pairs_by_tri, with each pair's index in the cell-ordered list): a stable
// sort on the support bits alone then orders them by (support, triangle).
// vals = cell-ordered pair index * NB + corner.
__global__ void k_support_emit(const u64* pairs_by_tri, const uint32_t* pair_index, long long np, int W,
                               u64* keys, uint32_t* vals) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  const int NB = W * W * W;
  if (i >= np * NB) return;
  long long q = i / NB;
  int j = (int)(i - q * NB);
  u64 k = pairs_by_tri[q];
  long long c[3];
  demorton(k >> TRI_BITS, c);
  int jx = j % W, jy = (j / W) % W, jz = j / (W * W);
  u64 s = morton((u64)(c[0] + jx), (u64)(c[1] + jy), (u64)(c[2] + jz));
  keys[i] = (s << TRI_BITS) | (k & TRI_MASK);
  vals[i] = pair_index[q] * (uint32_t)NB + (uint32_t)j;
}
__global__ void k_iota_u32(uint32_t* v, long long n) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n) v[i] = (uint32_t)i;
}
// unique entries + map from (pair, j) to its entry
__global__ void k_entries_scatter(const u64* keys, const uint32_t* vals, const int* flag, const int* pos,
                                  long long n, u64* ent, int* entry_of) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  int e = pos[i] + flag[i] - 1;   // inclusive rank - 1
  if (flag[i]) ent[e] = keys[i];
  entry_of[vals[i]] = e;
}

// group (support) of each entry: corner id = inclusive scan of head flags - 1
__global__ void k_corner_start(const int* flag, const int* pos, long long n, int* cstart, int* cid) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  if (flag[i]) cstart[pos[i]] = (int)i;
  cid[i] = pos[i] + flag[i] - 1;
}

// ------------------------------------------------------------- union-find
__device__ inline int uf_load(int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

__device__ inline int uf_find(int* parent, int x) {
  int p = uf_load(parent + x);
  while (p != x) {
    int gp = uf_load(parent + p);
    if (gp != p) __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = p;
    p = gp;
  }
  return x;
}

// hook the larger root under the smaller one: every root is its set's minimum
__device__ inline void uf_union(int* parent, int a, int b) {
  while (true) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a < b) { int t = a; a = b; b = t; }
    int old = atomicCAS(parent + a, a, b);
    if (old == a) return;
  }
}

__global__ void k_uf_init(int* parent, long long n) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n) parent[i] = (int)i;
}

// Links of entry e = (k, t): shared edges of t that reach into the open
// support, and vertices of t inside it; t is joined with the smallest
// triangle on that edge (vertex) that is active at k.  Two shortcuts keep
// the same components: when t itself comes first among the edge's (vertex's)
// triangles there is nothing to join, so no search is made; and a vertex
// inside the box by more than rounding whose triangles form one fan (vfan)
// adds no link, since its edges all reach into the box and their links
// already join every triangle at it (all of which are active at k).
__global__ void k_uf_link(const u64* ent, long long n, const int* cid, const int* cstart, int ncorn,
                          const int* F, const double* U, double sc, int degree, const int* tri_edge,
                          const int* edge_ptr, const int* edge_tri, const int* vt_ptr, const int* vt_tri,
                          const int* vfan, int* parent) {
  long long e = blockIdx.x * (long long)BLK + threadIdx.x;
  if (e >= n) return;
  const u64 key = ent[e];
  const u64 skey = key >> TRI_BITS;
  const int t = (int)(key & TRI_MASK);
  const int g = cid[e];
  const long long gs = cstart[g];
  const long long ge = (g + 1 < ncorn) ? cstart[g + 1] : n;
  if (ge - gs < 2) return;
  double C[3], H;
  support_box(degree, skey, C, &H);
  for (int j = 0; j < 3; ++j) {
    int a = F[3 * t + j], b = F[3 * t + (j + 1) % 3];
    int lo = min(a, b), hi = max(a, b);
    double pa[3], pb[3];
    for (int q = 0; q < 3; ++q) {
      pa[q] = U[3 * (long long)lo + q] * sc - C[q];
      pb[q] = U[3 * (long long)hi + q] * sc - C[q];
    }
    if (seg_meets_box(pa, pb, H)) {
      int eid = tri_edge[3 * t + j];
      for (int r = edge_ptr[eid]; r < edge_ptr[eid + 1]; ++r) {
        int t2 = edge_tri[r];
        if (t2 == t) break;
        u64 k2 = (skey << TRI_BITS) | (u64)t2;
        long long p = lower_bound_u64(ent, gs, ge, k2);
        if (p < ge && ent[p] == k2) {
          if (p != e) uf_union(parent, (int)e, (int)p);
          break;
        }
      }
    }
    int v = F[3 * t + j];
    bool inside = true, deep = true;
    for (int q = 0; q < 3; ++q) {
      const double z = fabs(U[3 * (long long)v + q] * sc - C[q]);
      inside = inside && z < H;
      deep = deep && z < H * (1.0 - 1e-12);
    }
    if (inside && !(deep && vfan[v])) {
      for (int r = vt_ptr[v]; r < vt_ptr[v + 1]; ++r) {
        int t2 = vt_tri[r];
        if (t2 == t) break;
        u64 k2 = (skey << TRI_BITS) | (u64)t2;
        long long p = lower_bound_u64(ent, gs, ge, k2);
        if (p < ge && ent[p] == k2) {
          if (p != e) uf_union(parent, (int)e, (int)p);
          break;
        }
      }
    }
  }
}

// root of every entry into a separate array.  The walk only reads parent:
// path halving here would let one thread overwrite another's final root with
// a stale ancestor (a valid pointer for union-find, but not the root that the
// function numbering needs).
__global__ void k_uf_roots(const int* parent, long long n, int* root) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  int x = (int)i, p = parent[x];
  while (p != x) {
    x = p;
    p = parent[x];
  }
  root[i] = x;
}

// without the split: every entry belongs to its support's first entry
__global__ void k_parent_is_group_head(const int* cid, const int* cstart, long long n, int* parent) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n) parent[i] = cstart[cid[i]];
}

__global__ void k_root_flags(const int* parent, long long n, int* isroot) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n) isroot[i] = parent[i] == (int)i ? 1 : 0;
}

__global__ void k_functions(const u64* ent, const int* parent, const int* rank, const int* cid,
                            const int* cstart, long long n, u64* fkey, int* fcomp, int* frep,
                            int* ent_func) {
  long long e = blockIdx.x * (long long)BLK + threadIdx.x;
  if (e >= n) return;
  int r = parent[e];
  ent_func[e] = rank[r];
  if (r == (int)e) {
    int f = rank[e];
    fkey[f] = ent[e] >> TRI_BITS;
    frep[f] = (int)(ent[e] & TRI_MASK);
    fcomp[f] = f - rank[cstart[cid[e]]];
  }
}

__global__ void k_corners(const u64* ent, const int* cstart, const int* rank, int ncorn, int nfun,
                          u64* ckey, int* cfirst) {
  long long g = blockIdx.x * (long long)BLK + threadIdx.x;
  if (g > ncorn) return;
  if (g == ncorn) { cfirst[g] = nfun; return; }
  ckey[g] = ent[cstart[g]] >> TRI_BITS;
  cfirst[g] = rank[cstart[g]];
}

__global__ void k_pair_rows(const int* entry_of, const int* ent_func, long long n, int* rows) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n) rows[i] = ent_func[entry_of[i]];
}

// --------------------------------------------------------------- adjacency
// edge keys: (smaller vertex << vbits) | larger vertex, vbits bits per vertex
__global__ void k_edge_emit(const int* F, long long nt, int vbits, u64* keys, uint32_t* vals) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= 3 * nt) return;
  long long t = i / 3;
  int j = (int)(i - 3 * t);
  int a = F[3 * t + j], b = F[3 * t + (j + 1) % 3];
  u64 lo = (u64)min(a, b), hi = (u64)max(a, b);
  keys[i] = (lo << vbits) | hi;
  vals[i] = (uint32_t)i;
}
__global__ void k_edge_fill(const uint32_t* vals, const int* flag, const int* pos, long long n, int* tri_edge,
                            int* edge_ptr, int* edge_tri) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  int id = pos[i] + flag[i] - 1;
  tri_edge[vals[i]] = id;
  edge_tri[i] = (int)(vals[i] / 3);
  if (flag[i]) edge_ptr[id] = (int)i;
}
// vertex keys: (vertex << tbits) | triangle, tbits bits per triangle
__global__ void k_vert_emit(const int* F, long long nt, int tbits, u64* keys) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= 3 * nt) return;
  keys[i] = ((u64)F[i] << tbits) | (u64)(i / 3);
}
__global__ void k_vt_fill(const u64* keys, long long n, long long nv, int tbits, int* vt_ptr, int* vt_tri) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  const u64 tmask = (1ULL << tbits) - 1ULL;
  long long v = (long long)(keys[i] >> tbits);
  vt_tri[i] = (int)(keys[i] & tmask);
  long long pv = (i == 0) ? -1 : (long long)(keys[i - 1] >> tbits);
  for (long long w = pv + 1; w <= v; ++w) vt_ptr[w] = (int)i;
  if (i == n - 1)
    for (long long w = v + 1; w <= nv; ++w) vt_ptr[w] = (int)n;
}

// 1 when the triangles at vertex v form a single fan: connected through
// edges at v (two triangles share the edge (v, w) when both hold w).  Up to
// 32 triangles per vertex are examined; a vertex with more counts as not
// a single fan (its vertex links are kept, which is always correct).
__global__ void k_vertex_fans(const int* F, const int* vt_ptr, const int* vt_tri, long long nv, int* vfan) {
  long long v = blockIdx.x * (long long)BLK + threadIdx.x;
  if (v >= nv) return;
  const int p0 = vt_ptr[v], k = vt_ptr[v + 1] - p0;
  if (k > 32) { vfan[v] = 0; return; }
  int w1[32], w2[32], lab[32];
  for (int i = 0; i < k; ++i) {
    const int t = vt_tri[p0 + i];
    int o[2], m = 0;
    for (int j = 0; j < 3; ++j) {
      const int u = F[3 * t + j];
      if (u != (int)v && m < 2) o[m++] = u;
    }
    w1[i] = o[0];
    w2[i] = m > 1 ? o[1] : o[0];
    lab[i] = i;
  }
  // label propagation over the shared-edge graph (at most k rounds)
  for (bool moved = true; moved;) {
    moved = false;
    for (int i = 0; i < k; ++i)
      for (int j = i + 1; j < k; ++j)
        if ((w1[i] == w1[j] || w1[i] == w2[j] || w2[i] == w1[j] || w2[i] == w2[j]) && lab[i] != lab[j]) {
          const int m = min(lab[i], lab[j]);
          lab[i] = lab[j] = m;
          moved = true;
        }
  }
  int one = 1;
  for (int i = 0; i < k; ++i) one = one && lab[i] == 0;
  vfan[v] = one;
}

// ----------------------------------------------------------- prolongation
// per axis: parents of fine index x at the coarser depth and their weights
__device__ inline int parents_1d(int degree, long long x, long long par[2], double w[2]) {
  if (degree == 1) {
    if ((x & 1) == 0) { par[0] = x >> 1; w[0] = 1.0; return 1; }
    par[0] = (x - 1) >> 1; w[0] = 0.5;
    par[1] = (x + 1) >> 1; w[1] = 0.5;
    return 2;
  }
  // stored nodes: x - 2X in {-2, -1, 0, 1} with weights 1/4, 3/4, 3/4, 1/4
  int n = 0;
  for (int m = -2; m <= 1; ++m) {
    long long d = x - m;
    if (d & 1) continue;
    par[n] = d >> 1;
    w[n] = (m == -2 || m == 1) ? 0.25 : 0.75;
    ++n;
  }
  return n;
}

__global__ void k_prolong_count(const u64* fkey, long long nf, int degree, int* cnt) {
  long long f = blockIdx.x * (long long)BLK + threadIdx.x;
  if (f >= nf) return;
  long long c[3];
  demorton(fkey[f], c);
  int total = 1;
  for (int a = 0; a < 3; ++a) {
    long long par[2];
    double w[2];
    total *= parents_1d(degree, c[a], par, w);
  }
  cnt[f] = total;
}

__global__ void k_prolong_fill(const u64* fkey, const int* frep, long long nf, int degree, const int* ptr,
                               const u64* cent, long long ncent, const int* cent_func, int* col, double* w,
                               int* flag) {
  long long f = blockIdx.x * (long long)BLK + threadIdx.x;
  if (f >= nf) return;
  long long c[3];
  demorton(fkey[f], c);
  long long par[3][2];
  double pw[3][2];
  int np[3];
  for (int a = 0; a < 3; ++a) np[a] = parents_1d(degree, c[a], par[a], pw[a]);
  int cols[8];
  double ws[8];
  int m = 0;
  const u64 rep = (u64)frep[f];
  for (int iz = 0; iz < np[2]; ++iz)
    for (int iy = 0; iy < np[1]; ++iy)
      for (int ix = 0; ix < np[0]; ++ix) {
        u64 K = morton((u64)par[0][ix], (u64)par[1][iy], (u64)par[2][iz]);
        u64 key = (K << TRI_BITS) | rep;
        long long p = lower_bound_u64(cent, 0, ncent, key);
        int cc = -1;
        if (p < ncent && cent[p] == key) cc = cent_func[p];
        else atomicOr(flag, FLAG_CHI);
        // insertion by column
        int q = m++;
        double wv = pw[0][ix] * pw[1][iy] * pw[2][iz];
        while (q > 0 && cols[q - 1] > cc) { cols[q] = cols[q - 1]; ws[q] = ws[q - 1]; --q; }
        cols[q] = cc;
        ws[q] = wv;
      }
  int o = ptr[f];
  for (int i = 0; i < m; ++i) { col[o + i] = cols[i]; w[o + i] = ws[i]; }
}

// -------------------------------------------------------------- host side
struct Flags {
  DArr<int> f, pos;
};

// unique of sorted keys (by full value) -> out, returns count
size_t unique_sorted(camfe_ctx ctx, const u64* in, size_t n, DArr<u64>& out) {
  if (n == 0) { out.alloc(0); return 0; }
  DArr<int> flag(n), pos(n);
  unsigned g = grid_for(n, BLK);
  hipLaunchKernelGGL(k_head_flags, g, BLK, 0, ctx->stream, in, (long long)n, 0, flag.p);
  exclusive_scan(ctx, flag.p, pos.p, n);
  int last_pos = read_scalar(ctx, pos.p + n - 1), last_flag = read_scalar(ctx, flag.p + n - 1);
  size_t m = (size_t)last_pos + last_flag;
  out.alloc(m);
  hipLaunchKernelGGL(k_compact_heads, g, BLK, 0, ctx->stream, in, flag.p, pos.p, (long long)n, out.p);
  check_launch();
  return m;
}

int sbits(int d) { return std::max(d + 1, 2); }

void build_adjacency(camfe_hier h) {
  camfe_ctx ctx = h->ctx;
  const size_t n3 = 3 * h->nt;
  DArr<u64> keys(n3);
  DArr<uint32_t> vals(n3);
  unsigned g = grid_for(n3, BLK);
  // bits that hold any vertex index and any triangle index
  auto bits_for = [](size_t count) {
    int b = 1;
    while (b < 31 && (size_t(1) << b) < count) ++b;
    return b;
  };
  const int vbits = bits_for(h->nv), tbits = bits_for(h->nt);
  hipLaunchKernelGGL(k_edge_emit, g, BLK, 0, ctx->stream, h->F.p, (long long)h->nt, vbits, keys.p, vals.p);
  check_launch();
  sort_pairs(ctx, keys.p, vals.p, n3, 2 * vbits);
  DArr<int> flag(n3), pos(n3);
  hipLaunchKernelGGL(k_head_flags, g, BLK, 0, ctx->stream, keys.p, (long long)n3, 0, flag.p);
  exclusive_scan(ctx, flag.p, pos.p, n3);
  h->ne = (size_t)read_scalar(ctx, pos.p + n3 - 1) + read_scalar(ctx, flag.p + n3 - 1);
  h->tri_edge.alloc(n3);
  h->edge_ptr.alloc(h->ne + 1);
  h->edge_tri.alloc(n3);
  hipLaunchKernelGGL(k_edge_fill, g, BLK, 0, ctx->stream, vals.p, flag.p, pos.p, (long long)n3, h->tri_edge.p,
                     h->edge_ptr.p, h->edge_tri.p);
  int n3i = (int)n3;
  copy_in(ctx, h->edge_ptr.p + h->ne, &n3i, 1);
  ctx->sync();
  hipLaunchKernelGGL(k_vert_emit, g, BLK, 0, ctx->stream, h->F.p, (long long)h->nt, tbits, keys.p);
  sort_keys(ctx, keys.p, n3, vbits + tbits);
  h->vt_ptr.alloc(h->nv + 1);
  h->vt_tri.alloc(n3);
  hipLaunchKernelGGL(k_vt_fill, g, BLK, 0, ctx->stream, keys.p, (long long)n3, (long long)h->nv, tbits,
                     h->vt_ptr.p, h->vt_tri.p);
  h->vfan.alloc(std::max<size_t>(h->nv, 1));
  hipLaunchKernelGGL(k_vertex_fans, grid_for(h->nv, BLK), BLK, 0, ctx->stream, h->F.p, h->vt_ptr.p, h->vt_tri.p,
                     (long long)h->nv, h->vfan.p);
  check_launch();
  ctx->sync();
}

// supports, split and functions of one depth, plus the (pair, j) -> function map
void build_functions(camfe_hier h, int d) {
  camfe_ctx ctx = h->ctx;
  HLevel& L = h->lev[d];
  const int W = h->W(), NB = h->NB();
  const size_t nraw = L.npairs * (size_t)NB;
  CAMFE_REQUIRE(nraw < (1ULL << 31), CAMFE_EINVAL, "too many (support, triangle) candidates at one depth");
  DArr<u64> keys(nraw);
  DArr<uint32_t> vals(nraw);
  unsigned g = grid_for(nraw, BLK);
  {
    // the pairs in triangle order (3 digit passes), so that the candidates
    // need sorting on their support bits only
    DArr<u64> by_tri(L.npairs);
    DArr<uint32_t> index(L.npairs);
    CAMFE_HIP(hipMemcpyAsync(by_tri.p, L.pairs.p, L.npairs * sizeof(u64), hipMemcpyDeviceToDevice, ctx->stream));
    hipLaunchKernelGGL(k_iota_u32, grid_for(L.npairs, BLK), BLK, 0, ctx->stream, index.p, (long long)L.npairs);
    check_launch();
    sort_pairs(ctx, by_tri.p, index.p, L.npairs, TRI_BITS);
    hipLaunchKernelGGL(k_support_emit, g, BLK, 0, ctx->stream, by_tri.p, index.p, (long long)L.npairs, W, keys.p,
                       vals.p);
    check_launch();
  }
  sort_pairs(ctx, keys.p, vals.p, nraw, 3 * sbits(d) + TRI_BITS, TRI_BITS);
  DArr<int> entry_of(nraw);
  {
    DArr<int> flag(nraw), pos(nraw);
    hipLaunchKernelGGL(k_head_flags, g, BLK, 0, ctx->stream, keys.p, (long long)nraw, 0, flag.p);
    exclusive_scan(ctx, flag.p, pos.p, nraw);
    L.nent = (size_t)read_scalar(ctx, pos.p + nraw - 1) + read_scalar(ctx, flag.p + nraw - 1);
    L.ent.alloc(L.nent);
    hipLaunchKernelGGL(k_entries_scatter, g, BLK, 0, ctx->stream, keys.p, vals.p, flag.p, pos.p,
                       (long long)nraw, L.ent.p, entry_of.p);
    check_launch();
  }
  keys.release();
  vals.release();
  // supports = runs of entries with one support key
  const size_t n = L.nent;
  unsigned ge = grid_for(n, BLK);
  DArr<int> cflag(n), cpos(n), cid(n);
  hipLaunchKernelGGL(k_head_flags, ge, BLK, 0, ctx->stream, L.ent.p, (long long)n, TRI_BITS, cflag.p);
  exclusive_scan(ctx, cflag.p, cpos.p, n);
  L.ncorn = (size_t)read_scalar(ctx, cpos.p + n - 1) + read_scalar(ctx, cflag.p + n - 1);
  DArr<int> cstart(L.ncorn);
  hipLaunchKernelGGL(k_corner_start, ge, BLK, 0, ctx->stream, cflag.p, cpos.p, (long long)n, cstart.p, cid.p);
  check_launch();
  // components: parent ends as the root (smallest entry) of each component
  DArr<int> parent(n);
  if (h->split) {
    DArr<int> link(n);
    hipLaunchKernelGGL(k_uf_init, ge, BLK, 0, ctx->stream, link.p, (long long)n);
    const double sc = ldexp(1.0, d - h->D);
    CAMFE_TIMED(ctx, KT_UF_LINK, 0.0, k_uf_link, ge, BLK, 0, ctx->stream, L.ent.p, (long long)n, cid.p, cstart.p,
                (int)L.ncorn, h->F.p, h->U.p, sc, h->degree, h->tri_edge.p, h->edge_ptr.p, h->edge_tri.p,
                h->vt_ptr.p, h->vt_tri.p, h->vfan.p, link.p);
    check_launch();
    hipLaunchKernelGGL(k_uf_roots, ge, BLK, 0, ctx->stream, (const int*)link.p, (long long)n, parent.p);
  } else {
    hipLaunchKernelGGL(k_parent_is_group_head, ge, BLK, 0, ctx->stream, cid.p, cstart.p, (long long)n, parent.p);
  }
  check_launch();
  // functions = roots, numbered in entry order (support key, then smallest triangle)
  DArr<int> isroot(n), rank(n);
  hipLaunchKernelGGL(k_root_flags, ge, BLK, 0, ctx->stream, parent.p, (long long)n, isroot.p);
  exclusive_scan(ctx, isroot.p, rank.p, n);
  L.nfun = (size_t)read_scalar(ctx, rank.p + n - 1) + read_scalar(ctx, isroot.p + n - 1);
  L.fkey.alloc(L.nfun);
  L.fcomp.alloc(L.nfun);
  L.frep.alloc(L.nfun);
  L.ent_func.alloc(n);
  hipLaunchKernelGGL(k_functions, ge, BLK, 0, ctx->stream, L.ent.p, parent.p, rank.p, cid.p, cstart.p,
                     (long long)n, L.fkey.p, L.fcomp.p, L.frep.p, L.ent_func.p);
  L.ckey.alloc(L.ncorn);
  L.cfirst.alloc(L.ncorn + 1);
  hipLaunchKernelGGL(k_corners, grid_for(L.ncorn + 1, BLK), BLK, 0, ctx->stream, L.ent.p, cstart.p, rank.p,
                     (int)L.ncorn, (int)L.nfun, L.ckey.p, L.cfirst.p);
  L.pair_rows.alloc(nraw);
  hipLaunchKernelGGL(k_pair_rows, g, BLK, 0, ctx->stream, entry_of.p, L.ent_func.p, (long long)nraw,
                     L.pair_rows.p);
  check_launch();
  ctx->sync();
  L.built = true;
}

void build_prolongation(camfe_hier h, int d) {
  camfe_ctx ctx = h->ctx;
  HLevel& F_ = h->lev[d];
  HLevel& C_ = h->lev[d - 1];
  const size_t nf = F_.nfun;
  F_.P_ptr.alloc(nf + 1);
  unsigned g = grid_for(nf, BLK);
  int last_cnt = 0, last_off = 0;
  {
    DArr<int> cnt(nf);
    hipLaunchKernelGGL(k_prolong_count, g, BLK, 0, ctx->stream, F_.fkey.p, (long long)nf, h->degree, cnt.p);
    check_launch();
    exclusive_scan(ctx, cnt.p, F_.P_ptr.p, nf);
    last_cnt = read_scalar(ctx, cnt.p + nf - 1);
    last_off = read_scalar(ctx, F_.P_ptr.p + nf - 1);
  }
  F_.pnnz = (size_t)last_off + last_cnt;
  int tot = (int)F_.pnnz;
  copy_in(ctx, F_.P_ptr.p + nf, &tot, 1);
  F_.P_col.alloc(F_.pnnz);
  F_.P_w.alloc(F_.pnnz);
  zero(ctx, ctx->d_flag, 1);
  hipLaunchKernelGGL(k_prolong_fill, g, BLK, 0, ctx->stream, F_.fkey.p, F_.frep.p, (long long)nf, h->degree,
                     F_.P_ptr.p, C_.ent.p, (long long)C_.nent, C_.ent_func.p, F_.P_col.p, F_.P_w.p,
                     ctx->d_flag);
  check_launch();
  int fl = read_scalar(ctx, ctx->d_flag);
  CAMFE_REQUIRE(fl == 0, CAMFE_EDEVICE, "prolongation: representative triangle missing from a parent support");
}

void count_cells(camfe_hier h, int d) {
  HLevel& L = h->lev[d];
  if (L.npairs == 0) { L.ncells = 0; return; }
  camfe_ctx ctx = h->ctx;
  DArr<int> flag(L.npairs), pos(L.npairs);
  unsigned g = grid_for(L.npairs, BLK);
  hipLaunchKernelGGL(k_head_flags, g, BLK, 0, ctx->stream, L.pairs.p, (long long)L.npairs, TRI_BITS, flag.p);
  exclusive_scan(ctx, flag.p, pos.p, L.npairs);
  L.ncells = (size_t)read_scalar(ctx, pos.p + L.npairs - 1) + read_scalar(ctx, flag.p + L.npairs - 1);
}

void build(camfe_hier h, const double* V, const int32_t* F) {
  camfe_ctx ctx = h->ctx;
  const int D = h->D;
  const size_t nv = h->nv, nt = h->nt;
  DArr<double> Vd(3 * nv);
  h->F.alloc(3 * nt);
  copy_in(ctx, Vd.p, V, 3 * nv);
  copy_in(ctx, h->F.p, (const int*)F, 3 * nt);
  // grid placement (A1)
  const int nblk = 64;
  DArr<double> part(6 * nblk);
  h->cubed.alloc(5);
  hipLaunchKernelGGL(k_minmax, nblk, BLK, 0, ctx->stream, Vd.p, (long long)nv, part.p);
  hipLaunchKernelGGL(k_cube, 1, 64, 0, ctx->stream, part.p, nblk, D, h->cube[0], h->cube[1], h->cube[2],
                     h->cube[3], h->cubed.p);
  check_launch();
  h->U.alloc(3 * nv);
  h->nrm.alloc(3 * nt);
  zero(ctx, ctx->d_flag, 1);
  hipLaunchKernelGGL(k_grid_coords, grid_for(3 * nv, BLK), BLK, 0, ctx->stream, Vd.p, (long long)nv, h->cubed.p,
                     ldexp(1.0, D), h->U.p, ctx->d_flag);
  hipLaunchKernelGGL(k_tri_check, grid_for(nt, BLK), BLK, 0, ctx->stream, h->F.p, (long long)nt, (long long)nv,
                     h->U.p, h->nrm.p, ctx->d_flag);
  check_launch();
  copy_out(ctx, h->cube, h->cubed.p, 5);
  int fl = read_scalar(ctx, ctx->d_flag);
  CAMFE_REQUIRE(!(fl & FLAG_NONFINITE), CAMFE_EINVAL, "non-finite vertex coordinate");
  CAMFE_REQUIRE(!(fl & FLAG_INDEX), CAMFE_EINVAL, "triangle index out of range or repeated");
  CAMFE_REQUIRE(!(fl & FLAG_OUTSIDE), CAMFE_EINVAL, "vertex outside the grid cube");
  CAMFE_REQUIRE(!(fl & FLAG_DEGEN), CAMFE_EINVAL, "degenerate triangle");
  CAMFE_REQUIRE(!(fl & FLAG_PLANE), CAMFE_EINVAL, "triangle lies in a grid plane (not in general position)");
  Vd.release();
  build_adjacency(h);
  h->lev.clear();
  h->lev.resize(D + 1);
  for (int d = 0; d <= D; ++d) h->lev[d].d = d;
  // finest pairs (A2): count, scan, write, sort
  {
    HLevel& L = h->lev[D];
    DArr<long long> cnt(nt), off(nt);
    unsigned g = grid_for(nt, BLK);
    const long long top = (1LL << D) - 1;
    hipLaunchKernelGGL(k_pairs<false>, g, BLK, 0, ctx->stream, h->U.p, h->F.p, (long long)nt, top, cnt.p,
                       (const long long*)nullptr, (u64*)nullptr);
    check_launch();
    exclusive_scan64(ctx, cnt.p, off.p, nt);
    L.npairs = (size_t)(read_scalar(ctx, off.p + nt - 1) + read_scalar(ctx, cnt.p + nt - 1));
    L.pairs.alloc(L.npairs);
    CAMFE_TIMED(ctx, KT_PAIRS, 0.0, k_pairs<true>, g, BLK, 0, ctx->stream, h->U.p, h->F.p, (long long)nt, top,
                cnt.p, off.p, L.pairs.p);
    check_launch();
    sort_keys(ctx, L.pairs.p, L.npairs, 3 * D + TRI_BITS);
    count_cells(h, D);
  }
  // depths D, D-1, ..., 0: pairs by aggregation; functions down to the coarsest depth
  h->d0 = D;
  bool stopped = false;
  for (int d = D; d >= 0; --d) {
    HLevel& L = h->lev[d];
    if (d < D) {
      HLevel& Fn = h->lev[d + 1];
      DArr<u64> tmp(Fn.npairs);
      hipLaunchKernelGGL(k_parent_keys, grid_for(Fn.npairs, BLK), BLK, 0, ctx->stream, Fn.pairs.p,
                         (long long)Fn.npairs, tmp.p);
      check_launch();
      sort_keys(ctx, tmp.p, Fn.npairs, 3 * d + TRI_BITS);
      L.npairs = unique_sorted(ctx, tmp.p, Fn.npairs, L.pairs);
      count_cells(h, d);
    }
    if (stopped) continue;
    build_functions(h, d);
    h->d0 = d;
    if (d <= h->min_depth || (h->max_coarse > 0 && (long long)L.nfun <= h->max_coarse)) stopped = true;
  }
  // prolongation with chi (A6)
  for (int d = D; d > h->d0; --d) build_prolongation(h, d);
  ctx->sync();
}

template <class T>
void export_array(camfe_ctx ctx, T* dst, const T* src, size_t n) {
  if (dst && n) copy_out(ctx, dst, src, n);
}

__global__ void k_split_keys(const u64* k, long long n, u64* key, int* tri) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n) return;
  if (key) key[i] = k[i] >> TRI_BITS;
  if (tri) tri[i] = (int)(k[i] & TRI_MASK);
}

// distinct cells of the sorted pair keys: the head of each run writes its cell
__global__ void k_cell_scatter(const u64* pairs, long long n, const int* flag, const int* pos, u64* out) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i >= n || !flag[i]) return;
  out[pos[i]] = pairs[i] >> TRI_BITS;
}

__global__ void k_widen(const int* in, long long n, long long* out) {
  long long i = blockIdx.x * (long long)BLK + threadIdx.x;
  if (i < n) out[i] = in[i];
}

camfe_status check_cap(int64_t cap, size_t n, int64_t* nout) {
  if (nout) *nout = (int64_t)n;
  if (cap == 0) return CAMFE_OK;
  if (cap < (int64_t)n) throw Error(CAMFE_ETOOSMALL, "export capacity too small");
  return CAMFE_OK;
}

const HLevel& level_of(camfe_hier h, int depth, bool need_functions) {
  if (h) set_current_ctx(h->ctx);
  CAMFE_REQUIRE(h != nullptr, CAMFE_EINVAL, "null hierarchy");
  CAMFE_REQUIRE(depth >= 0 && depth <= h->D, CAMFE_EINVAL, "depth out of range");
  const HLevel& L = h->lev[depth];
  if (need_functions) CAMFE_REQUIRE(L.built, CAMFE_ESTATE, "depth below the coarsest depth built");
  return L;
}

}  // namespace
}  // namespace camfe

using namespace camfe;

namespace {
thread_local std::string g_last_error;
thread_local camfe_ctx g_current_ctx = nullptr;

// Scratch of camfe_apply_noalloc (two row-major n x k blocks).  Each device
// holds its own copy at its own address; host code uses only the address that
// hipGetSymbolAddress gives for the current device, never the array's name.
__device__ __align__(256) double scratch[2 * NOALLOC_BLOCK];
std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_addr;   // device ordinal -> address of its scratch

// the current device's scratch address, looked up once per device
double* scratch_address(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) return it->second;
  double* p = nullptr;
  CAMFE_HIP(hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch)));
  CAMFE_REQUIRE(p != nullptr, CAMFE_EDEVICE, "no address for the device scratch");
  g_scratch_addr[device] = p;
  return p;
}
}

camfe_ctx camfe::current_ctx() { return g_current_ctx; }
void camfe::set_current_ctx(camfe_ctx ctx) { g_current_ctx = ctx; }

void camfe::set_last_error(const std::string& msg) {
  g_last_error = msg;
  if (g_current_ctx) {
    std::lock_guard<std::mutex> lk(g_current_ctx->err_mu);
    g_current_ctx->last_error = msg;
  }
}

extern "C" {

const char* camfe_last_error(void) { return g_last_error.c_str(); }

const char* camfe_ctx_last_error(camfe_ctx ctx) {
  if (!ctx) return "null context";
  std::lock_guard<std::mutex> lk(ctx->err_mu);
  return ctx->last_error.c_str();
}

camfe_status camfe_ctx_create(int device, void* hip_stream, camfe_ctx* out) {
  return guarded([&] {
    CAMFE_REQUIRE(out != nullptr, CAMFE_EINVAL, "null output handle");
    int ndev = 0;
    CAMFE_HIP(hipGetDeviceCount(&ndev));
    CAMFE_REQUIRE(device >= 0 && device < ndev, CAMFE_EINVAL, "device ordinal out of range");
    std::unique_ptr<camfe_ctx_s> c(new camfe_ctx_s());
    c->device = device;
    CAMFE_HIP(hipSetDevice(device));
    c->noalloc_scratch = scratch_address(device);
    if (hip_stream) {
      c->stream = (hipStream_t)hip_stream;
    } else {
      CAMFE_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
    CAMFE_HIP(hipMalloc((void**)&c->d_flag, sizeof(int)));
    pool_attach_stream(device, c->stream);
    *out = c.release();
  });
}

void camfe_ctx_destroy(camfe_ctx ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->scratch.release();
  ctx->scratch2.release();
  pool_detach_stream(ctx->device, ctx->stream);
  if (ctx->d_flag) (void)hipFree(ctx->d_flag);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

camfe_status camfe_ctx_kernel_timing(camfe_ctx ctx, int enable) {
  return guarded([&] {
    if (ctx) set_current_ctx(ctx);
    CAMFE_REQUIRE(ctx, CAMFE_EINVAL, "null context");
    ctx->use_device();
    if (enable) ctx->timer.reset();
    else ctx->timer.resolve();
    ctx->timer.on = enable != 0;
  });
}

camfe_status camfe_ctx_kernel_time(camfe_ctx ctx, const char* kernel, double* total_ms, int64_t* launches,
                                   double* work) {
  return guarded([&] {
    if (ctx) set_current_ctx(ctx);
    CAMFE_REQUIRE(ctx && kernel, CAMFE_EINVAL, "null argument");
    ctx->use_device();
    ctx->timer.resolve();
    for (int k = 0; k < KT_COUNT; ++k)
      if (std::string(kernel) == kernel_name(k)) {
        if (total_ms) *total_ms = ctx->timer.total_ms[k];
        if (launches) *launches = ctx->timer.count[k];
        if (work) *work = ctx->timer.work[k];
        return;
      }
    throw Error(CAMFE_EINVAL, std::string("unknown kernel name ") + kernel);
  });
}

camfe_status camfe_hierarchy_build(camfe_ctx ctx, const double* V, int64_t nv, const int32_t* F, int64_t nt,
                                   const camfe_hier_opts* o, camfe_hier* out) {
  return guarded([&] {
    if (ctx) set_current_ctx(ctx);
    CAMFE_REQUIRE(ctx && V && F && o && out, CAMFE_EINVAL, "null argument");
    CAMFE_REQUIRE(o->depth >= 1 && o->depth <= 12, CAMFE_EINVAL, "depth must be in [1, 12]");
    CAMFE_REQUIRE(o->degree == 1 || o->degree == 2, CAMFE_EINVAL, "degree must be 1 or 2");
    CAMFE_REQUIRE(nv > 0 && nt > 0, CAMFE_EINVAL, "empty mesh");
    CAMFE_REQUIRE(nt < (1LL << TRI_BITS), CAMFE_EINVAL, "at most 2^24 - 1 triangles");
    CAMFE_REQUIRE(nv < (1LL << 31), CAMFE_EINVAL, "too many vertices");
    ctx->use_device();
    std::unique_ptr<camfe_hier_s> h(new camfe_hier_s());
    h->ctx = ctx;
    h->D = o->depth;
    h->degree = o->degree;
    h->split = o->split ? 1 : 0;
    h->min_depth = std::max(0, std::min(o->min_depth, o->depth));
    h->max_coarse = o->max_coarse;
    h->nv = (size_t)nv;
    h->nt = (size_t)nt;
    if (o->box_side > 0) {
      h->cube[0] = o->box_origin[0]; h->cube[1] = o->box_origin[1]; h->cube[2] = o->box_origin[2];
      h->cube[3] = o->box_side;
    } else {
      h->cube[3] = 0.0;
    }
    build(h.get(), V, F);
    *out = h.release();
  });
}

camfe_status camfe_hierarchy_levels(camfe_hier h, int* finest, int* coarsest) {
  return guarded([&] {
    if (h) set_current_ctx(h->ctx);
    CAMFE_REQUIRE(h, CAMFE_EINVAL, "null hierarchy");
    if (finest) *finest = h->D;
    if (coarsest) *coarsest = h->d0;
  });
}

camfe_status camfe_hierarchy_cube(camfe_hier h, double out4[4]) {
  return guarded([&] {
    if (h) set_current_ctx(h->ctx);
    CAMFE_REQUIRE(h && out4, CAMFE_EINVAL, "null argument");
    for (int i = 0; i < 4; ++i) out4[i] = h->cube[i];
  });
}

camfe_status camfe_hierarchy_info(camfe_hier h, int depth, int64_t* n_cells, int64_t* n_pairs,
                                  int64_t* n_functions) {
  return guarded([&] {
    const HLevel& L = level_of(h, depth, false);
    if (n_cells) *n_cells = (int64_t)L.ncells;
    if (n_pairs) *n_pairs = (int64_t)L.npairs;
    if (n_functions) *n_functions = L.built ? (int64_t)L.nfun : -1;
  });
}

camfe_status camfe_export_cells(camfe_hier h, int depth, uint64_t* keys, int64_t cap, int64_t* n) {
  return guarded([&] {
    const HLevel& L = level_of(h, depth, false);
    check_cap(cap, L.ncells, n);
    if (cap == 0 || L.ncells == 0) return;
    CAMFE_REQUIRE(keys, CAMFE_EINVAL, "null output array");
    camfe_ctx ctx = h->ctx;
    ctx->use_device();
    DArr<int> flag(L.npairs), pos(L.npairs);
    DArr<u64> k(L.ncells);
    unsigned g = grid_for(L.npairs, BLK);
    hipLaunchKernelGGL(k_head_flags, g, BLK, 0, ctx->stream, L.pairs.p, (long long)L.npairs, TRI_BITS, flag.p);
    check_launch();
    exclusive_scan(ctx, flag.p, pos.p, L.npairs);
    hipLaunchKernelGGL(k_cell_scatter, g, BLK, 0, ctx->stream, L.pairs.p, (long long)L.npairs, flag.p, pos.p, k.p);
    check_launch();
    export_array(ctx, (u64*)keys, k.p, L.ncells);
    ctx->sync();
  });
}

camfe_status camfe_export_pairs(camfe_hier h, int depth, uint64_t* cell_key, int32_t* tri, int64_t cap,
                                int64_t* n) {
  return guarded([&] {
    const HLevel& L = level_of(h, depth, false);
    check_cap(cap, L.npairs, n);
    if (cap == 0 || L.npairs == 0) return;
    camfe_ctx ctx = h->ctx;
    ctx->use_device();
    DArr<u64> k(L.npairs);
    DArr<int> t(L.npairs);
    hipLaunchKernelGGL(k_split_keys, grid_for(L.npairs, BLK), BLK, 0, ctx->stream, L.pairs.p,
                       (long long)L.npairs, k.p, t.p);
    check_launch();
    export_array(ctx, (u64*)cell_key, k.p, L.npairs);
    export_array(ctx, (int*)tri, t.p, L.npairs);
    ctx->sync();
  });
}

camfe_status camfe_export_functions(camfe_hier h, int depth, uint64_t* key, int32_t* comp, int32_t* rep,
                                    int64_t cap, int64_t* n) {
  return guarded([&] {
    const HLevel& L = level_of(h, depth, true);
    check_cap(cap, L.nfun, n);
    if (cap == 0) return;
    camfe_ctx ctx = h->ctx;
    ctx->use_device();
    export_array(ctx, (u64*)key, L.fkey.p, L.nfun);
    export_array(ctx, (int*)comp, L.fcomp.p, L.nfun);
    export_array(ctx, (int*)rep, L.frep.p, L.nfun);
    ctx->sync();
  });
}

camfe_status camfe_export_support_entries(camfe_hier h, int depth, uint64_t* key, int32_t* tri, int32_t* func,
                                          int64_t cap, int64_t* n) {
  return guarded([&] {
    const HLevel& L = level_of(h, depth, true);
    check_cap(cap, L.nent, n);
    if (cap == 0 || L.nent == 0) return;
    camfe_ctx ctx = h->ctx;
    ctx->use_device();
    DArr<u64> k(L.nent);
    DArr<int> t(L.nent);
    hipLaunchKernelGGL(k_split_keys, grid_for(L.nent, BLK), BLK, 0, ctx->stream, L.ent.p, (long long)L.nent,
                       k.p, t.p);
    check_launch();
    export_array(ctx, (u64*)key, k.p, L.nent);
    export_array(ctx, (int*)tri, t.p, L.nent);
    export_array(ctx, (int*)func, L.ent_func.p, L.nent);
    ctx->sync();
  });
}

camfe_status camfe_export_prolongation(camfe_hier h, int depth, int64_t* rowptr, int32_t* col, double* w,
                                       int64_t cap, int64_t* nnz) {
  return guarded([&] {
    const HLevel& L = level_of(h, depth, true);
    CAMFE_REQUIRE(depth > h->d0, CAMFE_ESTATE, "no prolongation into the coarsest depth");
    check_cap(cap, L.pnnz, nnz);
    if (cap == 0) return;
    camfe_ctx ctx = h->ctx;
    ctx->use_device();
    if (rowptr) {
      DArr<long long> p64(L.nfun + 1);
      hipLaunchKernelGGL(k_widen, grid_for(L.nfun + 1, BLK), BLK, 0, ctx->stream, L.P_ptr.p,
                         (long long)(L.nfun + 1), p64.p);
      check_launch();
      export_array(ctx, (long long*)rowptr, p64.p, L.nfun + 1);
      ctx->sync();
    }
    export_array(ctx, (int*)col, L.P_col.p, L.pnnz);
    export_array(ctx, w, L.P_w.p, L.pnnz);
    ctx->sync();
  });
}

void camfe_hierarchy_destroy(camfe_hier h) {
  if (!h) return;
  (void)hipSetDevice(h->ctx->device);
  (void)hipStreamSynchronize(h->ctx->stream);
  delete h;
}

}  // extern "C"

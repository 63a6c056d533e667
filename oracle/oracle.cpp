// CPU oracle for the connectivity-aware multilevel finite-element system of
// Chuang & Kazhdan, "A Connectivity-Aware Multi-level Finite-Element System for
// Solving Laplace-Beltrami Equations" (arXiv 1505.03615).
//
// TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, sequential FP64
// restatement of what the method computes.  Only the test suite, the smoke
// check and the benchmark's CPU-baseline leg load it.  It shares no code,
// header, table or constant generator with the HIP library, and the HIP
// library never loads it.
//
// Build: g++ -O2 -ffp-contract=off -shared -fPIC (no -march=native), so every
// floating-point predicate below is evaluated with plain IEEE-754 adds and
// multiplies in the stated order.  A second build with -fopenmp (used only for
// the benchmark's all-cores timing) shares the rows of one colour and of the
// residual, matrix-vector and prolongation loops among threads; each row is
// still computed by one thread in the same order, so its results are the same
// bits as the sequential build's.
//
// Steps, with the passage each follows:
//   cube / grid coordinates ........ Section 3.2, Definition 1 (grid G^N embedding;
//                                    placement is not specified: 1.125 x extent, centred)
//   finest triangle/cell pairs ..... Section 4.2 (keep functions whose support meets
//                                    the surface), Definition 2
//   octree aggregation .............. Section 4.3 (successively finer grids)
//   supports, links, components ..... Section 4.2 (one function per connected
//                                    component of supp(b_k) restricted to the mesh)
//   prolongation with chi ........... Section 3.2 Eq. (3), Section 4.3 Eq. (4),
//                                    Observation of Section 4.1
//   quadrature + assembly ........... Section 3.1 Eq. (2) (stiffness with the
//                                    surface gradient, load), Section 5.1 (mass)
//   V-cycle with Gauss-Seidel ....... Section 3.2 / 4.3 (multigrid on nested spaces),
//                                    Section 5.2 (Gauss-Seidel smoothing), the
//                                    Discussion closing Section 5 (eps * Id for
//                                    singular systems)
//   gradient constraint, W-cycle .... Section 5.2 (colour fitting: int <grad f,
//                                    grad b_i>, one W-cycle, minimum depth)
//
// Parity pins for every function here live in tests/test_oracle_*.py.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

namespace {

typedef std::pair<uint64_t, int> KeyTri;

// ---------------------------------------------------------------- Morton keys
// bit b of x -> 3b, of y -> 3b+1, of z -> 3b+2
uint64_t morton3(long x, long y, long z) {
  uint64_t k = 0;
  for (int b = 0; b < 21; ++b) {
    k |= (uint64_t)((x >> b) & 1) << (3 * b);
    k |= (uint64_t)((y >> b) & 1) << (3 * b + 1);
    k |= (uint64_t)((z >> b) & 1) << (3 * b + 2);
  }
  return k;
}
void demorton3(uint64_t k, long c[3]) {
  c[0] = c[1] = c[2] = 0;
  for (int b = 0; b < 21; ++b) {
    c[0] |= (long)((k >> (3 * b)) & 1) << b;
    c[1] |= (long)((k >> (3 * b + 1)) & 1) << b;
    c[2] |= (long)((k >> (3 * b + 2)) & 1) << b;
  }
}

// ------------------------------------------------------- separating axes
// Projection of the points P[0..np) on axis A; the open box of half-size h at
// the origin projects to (-r, r), r = h(|A0|+|A1|+|A2|).  The axis separates
// (touching counts as separated) iff min >= r or max <= -r.  All-zero axes
// carry no information and are skipped.
bool axis_separates(const double A[3], const double P[][3], int np, double h) {
  if (A[0] == 0.0 && A[1] == 0.0 && A[2] == 0.0) return false;
  double mn = 0, mx = 0;
  for (int i = 0; i < np; ++i) {
    double p = A[0] * P[i][0] + A[1] * P[i][1] + A[2] * P[i][2];
    if (i == 0 || p < mn) mn = p;
    if (i == 0 || p > mx) mx = p;
  }
  double r = h * (std::fabs(A[0]) + std::fabs(A[1]) + std::fabs(A[2]));
  return mn >= r || mx <= -r;
}

// box axes e_a and the three axes e_a x f for one direction f
bool box_and_cross_axes_separate(const double P[][3], int np, const double f[3], double h) {
  for (int a = 0; a < 3; ++a) {
    double A[3] = {0.0, 0.0, 0.0};
    A[a] = 1.0;
    if (axis_separates(A, P, np, h)) return true;
  }
  double ax[3] = {0.0, -f[2], f[1]};
  double ay[3] = {f[2], 0.0, -f[0]};
  double az[3] = {-f[1], f[0], 0.0};
  return axis_separates(ax, P, np, h) || axis_separates(ay, P, np, h) ||
         axis_separates(az, P, np, h);
}

// Triangle (vertices already translated to the box centre) against the open
// box of half-size h: the 13-axis separating-axis test (box normals, triangle
// normal, edge x box-axis cross products).
bool triangle_meets_open_box(const double v[3][3], double h) {
  double f[3][3];
  for (int j = 0; j < 3; ++j)
    for (int a = 0; a < 3; ++a) f[j][a] = v[(j + 1) % 3][a] - v[j][a];
  double n[3] = {f[0][1] * f[1][2] - f[0][2] * f[1][1], f[0][2] * f[1][0] - f[0][0] * f[1][2],
                 f[0][0] * f[1][1] - f[0][1] * f[1][0]};
  if (axis_separates(n, v, 3, h)) return false;
  for (int j = 0; j < 3; ++j)
    if (box_and_cross_axes_separate(v, 3, f[j], h)) return false;
  return true;
}

// Closed segment [P,Q] (translated to the box centre) against the open box.
bool segment_meets_open_box(const double P[3], const double Q[3], double h) {
  double pts[2][3] = {{P[0], P[1], P[2]}, {Q[0], Q[1], Q[2]}};
  double f[3] = {Q[0] - P[0], Q[1] - P[1], Q[2] - P[2]};
  return !box_and_cross_axes_separate(pts, 2, f, h);
}

// ------------------------------------------------------------- union-find
struct DSU {
  std::vector<int> p;
  explicit DSU(int n) : p(n) { std::iota(p.begin(), p.end(), 0); }
  int find(int x) {
    while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
    return x;
  }
  void unite(int a, int b) {
    a = find(a); b = find(b);
    if (a == b) return;
    if (a < b) p[b] = a; else p[a] = b;
  }
};

// ----------------------------------------------------------- data per depth
struct Level {
  int d = 0;
  std::vector<KeyTri> pairs;            // (cell Morton key, triangle), sorted
  std::vector<KeyTri> stri;             // (support key, triangle) sorted, unique
  std::vector<int> stri_func;           // function index of each stri entry
  std::vector<uint64_t> fkey;           // per function: support key
  std::vector<int> fcomp, frep;         // component number, representative (min) triangle
  // prolongation from depth d-1 to d: rows = functions at d, cols at d-1
  std::vector<long> Pptr;
  std::vector<int> Pcol;
  std::vector<double> Pw;
  // assembled matrices (CSR over functions, columns ascending)
  std::vector<long> Aptr;
  std::vector<int> Acol;
  std::vector<double> Mval, Lval;
  bool assembled = false;
};

struct Hier {
  int D = 0, degree = 1, split = 1, min_depth = 0;
  long max_coarse = 0;
  int d0 = 0;             // coarsest depth built
  double o[3] = {0, 0, 0}, s = 1.0;
  long nv = 0, nt = 0;
  std::vector<double> U;  // grid coordinates at depth D, nv x 3
  std::vector<double> V;  // world positions, nv x 3
  std::vector<int> F;     // nt x 3
  std::vector<Level> lev; // index = depth
  // mesh adjacency: edge (sorted vertex pair) -> incident triangles; vertex -> triangles
  std::vector<std::pair<std::pair<int, int>, int>> edge_tri;  // sorted
  std::vector<long> vt_ptr;
  std::vector<int> vt_tri;
  double timing[4] = {0, 0, 0, 0};  // build, assemble, setup, solve seconds
  std::string err;
};

int width(int degree) { return degree == 1 ? 2 : 3; }  // supports per axis touching one cell

// Support box of a function key at depth d, in depth-d grid units.
// Degree 1: corner k, box [k-1, k+1]^3 (centre k, half-size 1).
// Degree 2: stored node S = o+1 for the quadratic B-spline on cell o, box
// [o-1, o+2]^3 (centre S - 1/2, half-size 3/2).
void support_box(int degree, uint64_t key, double C[3], double* H) {
  long c[3];
  demorton3(key, c);
  for (int a = 0; a < 3; ++a) C[a] = degree == 1 ? (double)c[a] : (double)c[a] - 0.5;
  *H = degree == 1 ? 1.0 : 1.5;
}

// grid coordinates at depth d (exact power-of-two scaling of the depth-D ones)
void vert_at(const Hier& h, int v, int d, double out[3]) {
  double sc = std::ldexp(1.0, d - h.D);
  for (int a = 0; a < 3; ++a) out[a] = h.U[3 * (long)v + a] * sc;
}

// ----------------------------------------------------------- hierarchy build
bool build(Hier& h, const double* V, const int* F, const double* box) {
  const int D = h.D;
  const long nv = h.nv, nt = h.nt;
  // grid placement: bounding cube, 1.125 x the largest extent, centred
  if (box && box[3] > 0) {
    for (int a = 0; a < 3; ++a) h.o[a] = box[a];
    h.s = box[3];
  } else {
    double mn[3], mx[3];
    for (int a = 0; a < 3; ++a) { mn[a] = V[a]; mx[a] = V[a]; }
    for (long v = 0; v < nv; ++v)
      for (int a = 0; a < 3; ++a) {
        mn[a] = std::min(mn[a], V[3 * v + a]);
        mx[a] = std::max(mx[a], V[3 * v + a]);
      }
    double ext = std::max(std::max(mx[0] - mn[0], mx[1] - mn[1]), mx[2] - mn[2]);
    h.s = 1.125 * ext;
    for (int a = 0; a < 3; ++a) h.o[a] = (mn[a] + mx[a]) * 0.5 - h.s * 0.5;
  }
  const double inv = std::ldexp(1.0, D) / h.s;
  const double N = std::ldexp(1.0, D);
  h.U.resize(3 * nv);
  for (long v = 0; v < nv; ++v)
    for (int a = 0; a < 3; ++a) {
      double u = (V[3 * v + a] - h.o[a]) * inv;
      if (!(u >= 0.0 && u <= N)) { h.err = "vertex outside the grid cube"; return false; }
      h.U[3 * v + a] = u;
    }
  h.F.assign(F, F + 3 * nt);
  for (long t = 0; t < nt; ++t) {
    const int* f = &h.F[3 * t];
    for (int j = 0; j < 3; ++j)
      if (f[j] < 0 || f[j] >= nv) { h.err = "triangle index out of range"; return false; }
    const double* p0 = &h.U[3 * (long)f[0]];
    const double* p1 = &h.U[3 * (long)f[1]];
    const double* p2 = &h.U[3 * (long)f[2]];
    double e0[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
    double e1[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
    double n[3] = {e0[1] * e1[2] - e0[2] * e1[1], e0[2] * e1[0] - e0[0] * e1[2],
                   e0[0] * e1[1] - e0[1] * e1[0]};
    if (n[0] == 0.0 && n[1] == 0.0 && n[2] == 0.0) { h.err = "degenerate triangle"; return false; }
    for (int a = 0; a < 3; ++a)
      if (p0[a] == p1[a] && p1[a] == p2[a] && std::floor(p0[a]) == p0[a]) {
        h.err = "triangle lies in a grid plane (not in general position)";
        return false;
      }
  }

  // mesh adjacency
  h.edge_tri.clear();
  for (long t = 0; t < nt; ++t)
    for (int j = 0; j < 3; ++j) {
      int a = h.F[3 * t + j], b = h.F[3 * t + (j + 1) % 3];
      h.edge_tri.push_back({{std::min(a, b), std::max(a, b)}, (int)t});
    }
  std::sort(h.edge_tri.begin(), h.edge_tri.end());
  h.vt_ptr.assign(nv + 1, 0);
  for (long t = 0; t < nt; ++t)
    for (int j = 0; j < 3; ++j) h.vt_ptr[h.F[3 * t + j] + 1]++;
  for (long v = 0; v < nv; ++v) h.vt_ptr[v + 1] += h.vt_ptr[v];
  h.vt_tri.assign(3 * nt, 0);
  {
    std::vector<long> fill(h.vt_ptr.begin(), h.vt_ptr.end() - 1);
    for (long t = 0; t < nt; ++t)
      for (int j = 0; j < 3; ++j) h.vt_tri[fill[h.F[3 * t + j]]++] = (int)t;
  }

  h.lev.assign(D + 1, Level());
  for (int d = 0; d <= D; ++d) h.lev[d].d = d;

  // finest pairs: t meets the open cell, by the 13-axis test on candidate
  // cells of the triangle's integer bounding box
  {
    std::vector<KeyTri>& P = h.lev[D].pairs;
    const long top = (1L << D) - 1;
    for (long t = 0; t < nt; ++t) {
      const double* p[3] = {&h.U[3 * (long)h.F[3 * t]], &h.U[3 * (long)h.F[3 * t + 1]],
                            &h.U[3 * (long)h.F[3 * t + 2]]};
      long lo[3], hi[3];
      for (int a = 0; a < 3; ++a) {
        double mn = std::min(std::min(p[0][a], p[1][a]), p[2][a]);
        double mx = std::max(std::max(p[0][a], p[1][a]), p[2][a]);
        lo[a] = std::max(0L, std::min(top, (long)std::floor(mn)));
        hi[a] = std::max(0L, std::min(top, (long)std::floor(mx)));
      }
      for (long z = lo[2]; z <= hi[2]; ++z)
        for (long y = lo[1]; y <= hi[1]; ++y)
          for (long x = lo[0]; x <= hi[0]; ++x) {
            double cen[3] = {(double)x + 0.5, (double)y + 0.5, (double)z + 0.5};
            double v[3][3];
            for (int i = 0; i < 3; ++i)
              for (int a = 0; a < 3; ++a) v[i][a] = p[i][a] - cen[a];
            if (triangle_meets_open_box(v, 0.5)) P.push_back({morton3(x, y, z), (int)t});
          }
    }
    std::sort(P.begin(), P.end());
  }
  // coarser pairs: parent cell (each coordinate halved) of every finer pair
  for (int d = D - 1; d >= 0; --d) {
    std::vector<KeyTri>& P = h.lev[d].pairs;
    for (const KeyTri& kt : h.lev[d + 1].pairs) P.push_back({kt.first >> 3, kt.second});
    std::sort(P.begin(), P.end());
    P.erase(std::unique(P.begin(), P.end()), P.end());
  }

  // functions per depth, from the finest down; stop at the coarsest depth d0
  const int W = width(h.degree);
  h.d0 = 0;
  for (int d = D; d >= 0; --d) {
    Level& L = h.lev[d];
    // active sets A_k: every support containing the cell of a pair
    L.stri.clear();
    for (const KeyTri& kt : L.pairs) {
      long c[3];
      demorton3(kt.first, c);
      for (int jz = 0; jz < W; ++jz)
        for (int jy = 0; jy < W; ++jy)
          for (int jx = 0; jx < W; ++jx)
            L.stri.push_back({morton3(c[0] + jx, c[1] + jy, c[2] + jz), kt.second});
    }
    std::sort(L.stri.begin(), L.stri.end());
    L.stri.erase(std::unique(L.stri.begin(), L.stri.end()), L.stri.end());
    L.stri_func.assign(L.stri.size(), -1);
    L.fkey.clear(); L.fcomp.clear(); L.frep.clear();
    // per support: union-find of its active triangles
    size_t g0 = 0;
    while (g0 < L.stri.size()) {
      size_t g1 = g0;
      const uint64_t key = L.stri[g0].first;
      while (g1 < L.stri.size() && L.stri[g1].first == key) ++g1;
      const int m = (int)(g1 - g0);
      std::vector<int> comp_of(m, 0);
      if (h.split) {
        double C[3], H;
        support_box(h.degree, key, C, &H);
        DSU dsu(m);
        // position of triangle t inside this support's list, or -1
        auto local = [&](int t) -> int {
          auto it = std::lower_bound(L.stri.begin() + g0, L.stri.begin() + g1, KeyTri(key, t));
          return (it != L.stri.begin() + g1 && it->second == t) ? (int)(it - L.stri.begin() - g0) : -1;
        };
        for (int i = 0; i < m; ++i) {
          const int t = L.stri[g0 + i].second;
          const int* f = &h.F[3 * (long)t];
          for (int j = 0; j < 3; ++j) {
            // shared edge whose points reach into the open support
            int a = std::min(f[j], f[(j + 1) % 3]), b = std::max(f[j], f[(j + 1) % 3]);
            double pa[3], pb[3];
            vert_at(h, a, d, pa);
            vert_at(h, b, d, pb);
            for (int q = 0; q < 3; ++q) { pa[q] -= C[q]; pb[q] -= C[q]; }
            if (segment_meets_open_box(pa, pb, H)) {
              auto lo = std::lower_bound(h.edge_tri.begin(), h.edge_tri.end(),
                                         std::make_pair(std::make_pair(a, b), -1));
              for (auto it = lo; it != h.edge_tri.end() && it->first.first == a && it->first.second == b; ++it) {
                int li = local(it->second);
                if (li >= 0) dsu.unite(i, li);
              }
            }
            // shared vertex inside the open support
            const int v = f[j];
            double pv[3];
            vert_at(h, v, d, pv);
            bool inside = true;
            for (int q = 0; q < 3; ++q) inside = inside && std::fabs(pv[q] - C[q]) < H;
            if (inside) {
              for (long r = h.vt_ptr[v]; r < h.vt_ptr[v + 1]; ++r) {
                int li = local(h.vt_tri[r]);
                if (li >= 0) dsu.unite(i, li);
              }
            }
          }
        }
        // components numbered by increasing minimum triangle; the union-find
        // keeps the smallest local index (= smallest triangle) as root
        int nc = 0;
        std::vector<int> num(m, -1);
        for (int i = 0; i < m; ++i) {
          int r = dsu.find(i);
          if (num[r] < 0) num[r] = nc++;
          comp_of[i] = num[r];
        }
      }
      const int first = (int)L.fkey.size();
      int ncomp = 0;
      for (int i = 0; i < m; ++i) ncomp = std::max(ncomp, comp_of[i] + 1);
      for (int c = 0; c < ncomp; ++c) {
        L.fkey.push_back(key);
        L.fcomp.push_back(c);
        L.frep.push_back(-1);
      }
      for (int i = 0; i < m; ++i) {
        int fi = first + comp_of[i];
        L.stri_func[g0 + i] = fi;
        if (L.frep[fi] < 0) L.frep[fi] = L.stri[g0 + i].second;  // smallest triangle first
      }
      g0 = g1;
    }
    const long n = (long)L.fkey.size();
    h.d0 = d;
    // coarsest depth: the finest depth with n_d <= max_coarse, but not below
    // min_depth (when max_coarse <= 0 only min_depth decides)
    if (d <= h.min_depth || (h.max_coarse > 0 && n <= h.max_coarse)) break;
  }

  // prolongation (Eq. 4): fine function (k', i') with representative t*
  // receives coarse function (K, label_K(t*)) with the B-spline refinement weight
  for (int d = D; d > h.d0; --d) {
    Level& Lf = h.lev[d];
    Level& Lc = h.lev[d - 1];
    const long n = (long)Lf.fkey.size();
    Lf.Pptr.assign(n + 1, 0);
    Lf.Pcol.clear(); Lf.Pw.clear();
    for (long f = 0; f < n; ++f) {
      long k[3];
      demorton3(Lf.fkey[f], k);
      long par[3][2];
      double w[3][2];
      int np[3];
      for (int a = 0; a < 3; ++a) {
        np[a] = 0;
        if (h.degree == 1) {
          // hat refinement 1/2 (1 2 1): k' = 2K + m, m in {-1,0,1}
          if (k[a] % 2 == 0) { par[a][0] = k[a] / 2; w[a][0] = 1.0; np[a] = 1; }
          else {
            par[a][0] = (k[a] - 1) / 2; w[a][0] = 0.5;
            par[a][1] = (k[a] + 1) / 2; w[a][1] = 0.5; np[a] = 2;
          }
        } else {
          // quadratic refinement 1/4 (1 3 3 1) on stored indices S = o+1:
          // S' - 2S in {-2,-1,0,1} with weights 1/4, 3/4, 3/4, 1/4
          const long Sp = k[a];
          for (int mm = -2; mm <= 1; ++mm) {
            if (((Sp - mm) % 2 + 2) % 2 != 0) continue;
            par[a][np[a]] = (Sp - mm) / 2;
            w[a][np[a]] = (mm == -2 || mm == 1) ? 0.25 : 0.75;
            np[a]++;
          }
        }
      }
      std::vector<std::pair<int, double>> row;
      for (int iz = 0; iz < np[2]; ++iz)
        for (int iy = 0; iy < np[1]; ++iy)
          for (int ix = 0; ix < np[0]; ++ix) {
            uint64_t K = morton3(par[0][ix], par[1][iy], par[2][iz]);
            auto it = std::lower_bound(Lc.stri.begin(), Lc.stri.end(), KeyTri(K, Lf.frep[f]));
            if (it == Lc.stri.end() || it->first != K || it->second != Lf.frep[f]) {
              h.err = "prolongation: representative triangle missing from a parent support";
              return false;
            }
            row.push_back({Lc.stri_func[it - Lc.stri.begin()], w[0][ix] * w[1][iy] * w[2][iz]});
          }
      std::sort(row.begin(), row.end());
      for (auto& e : row) { Lf.Pcol.push_back(e.first); Lf.Pw.push_back(e.second); }
      Lf.Pptr[f + 1] = (long)Lf.Pcol.size();
    }
  }
  return true;
}

// --------------------------------------------------------------- quadrature
// Gauss-Legendre nodes/weights on [0,1] by Newton on P_n
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0); w.assign(n, 0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1; p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    double p0 = 1, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1; p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1);
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1 - z * z) * dp * dp);
  }
}

// 1D basis pieces on one cell, local coordinate l in [0,1], j = index of the
// support among the W touching the cell along this axis
double b1d(int degree, int j, double l) {
  if (degree == 1) return j == 0 ? 1.0 - l : l;
  if (j == 0) return 0.5 * (1.0 - l) * (1.0 - l);
  if (j == 1) return 0.75 - (l - 0.5) * (l - 0.5);
  return 0.5 * l * l;
}
double db1d(int degree, int j, double l) {
  if (degree == 1) return j == 0 ? -1.0 : 1.0;
  if (j == 0) return -(1.0 - l);
  if (j == 1) return -2.0 * (l - 0.5);
  return l;
}

struct PV { double x[3]; double l[3]; };  // polygon vertex: position + barycentrics

// Sutherland-Hodgman against the closed half-space x_a >= v (ge) or x_a <= v
std::vector<PV> clip(const std::vector<PV>& in, int a, double v, bool ge) {
  std::vector<PV> out;
  const size_t n = in.size();
  for (size_t i = 0; i < n; ++i) {
    const PV& P = in[i];
    const PV& Q = in[(i + 1) % n];
    bool inP = ge ? P.x[a] >= v : P.x[a] <= v;
    bool inQ = ge ? Q.x[a] >= v : Q.x[a] <= v;
    if (inP) out.push_back(P);
    if (inP != inQ) {
      double lam = (v - P.x[a]) / (Q.x[a] - P.x[a]);
      PV R;
      for (int b = 0; b < 3; ++b) {
        R.x[b] = P.x[b] + lam * (Q.x[b] - P.x[b]);
        R.l[b] = P.l[b] + lam * (Q.l[b] - P.l[b]);
      }
      R.x[a] = v;
      out.push_back(R);
    }
  }
  return out;
}

struct RowAcc { std::vector<int> col; std::vector<double> m, l; };

void row_add(RowAcc& r, int c, double m, double l) {
  for (size_t i = 0; i < r.col.size(); ++i)
    if (r.col[i] == c) { r.m[i] += m; r.l[i] += l; return; }
  r.col.push_back(c); r.m.push_back(m); r.l.push_back(l);
}

int func_of(const Level& L, uint64_t key, int t) {
  auto it = std::lower_bound(L.stri.begin(), L.stri.end(), KeyTri(key, t));
  if (it == L.stri.end() || it->first != key || it->second != t) return -1;
  return L.stri_func[it - L.stri.begin()];
}

// Integrate over every (cell, triangle) fragment at depth d:
//   M_ij = int b_i b_j,  L_ij = int <grad_M b_i, grad_M b_j>,  b_i += int f b_i
// with grad_M the tangential (surface) gradient on each flat triangle.
// tri_w (nullable) scales each triangle's contribution to M only (area ratio
// of an evolved surface; the stiffness stays that of the original surface).  fv (nullable, nv x k col-major) gives per-vertex values of
// f, interpolated linearly inside each triangle; rhs is n x k col-major.
// rhs (nullable) receives b_i = int f b_i, or with grad_rhs the gradient
// constraint b_i = int <grad f, grad b_i> of the colour-fitting problem
// (Section 5.2), for f linear on each triangle from per-vertex values fv.
bool assemble_level(Hier& h, int d, const double* tri_w, const double* fv, int k, double* rhs,
                    bool want_matrix, bool grad_rhs = false) {
  Level& L = h.lev[d];
  const int W = width(h.degree);
  const int NB = W * W * W;
  const int nq = h.degree == 1 ? 4 : 7;
  std::vector<double> gx, gw;
  gauss_legendre01(nq, gx, gw);
  const double hd = h.s / std::ldexp(1.0, d);   // world size of a depth-d cell
  const double sc = std::ldexp(1.0, d - h.D);
  const long n = (long)L.fkey.size();
  std::vector<RowAcc> rows(want_matrix ? n : 0);
  if (rhs) std::fill(rhs, rhs + n * k, 0.0);
  for (const KeyTri& kt : L.pairs) {
    const int t = kt.second;
    long c[3];
    demorton3(kt.first, c);
    int ridx[27];
    for (int jz = 0; jz < W; ++jz)
      for (int jy = 0; jy < W; ++jy)
        for (int jx = 0; jx < W; ++jx) {
          int r = func_of(L, morton3(c[0] + jx, c[1] + jy, c[2] + jz), t);
          if (r < 0) { h.err = "assembly: (support, triangle) label missing"; return false; }
          ridx[jx + W * jy + W * W * jz] = r;
        }
    // unit normal of the triangle (direction is scale-invariant)
    const int* f = &h.F[3 * (long)t];
    std::vector<PV> poly(3);
    for (int i = 0; i < 3; ++i) {
      for (int a = 0; a < 3; ++a) poly[i].x[a] = h.U[3 * (long)f[i] + a] * sc;
      for (int b = 0; b < 3; ++b) poly[i].l[b] = (i == b) ? 1.0 : 0.0;
    }
    double e0[3], e1[3];
    for (int a = 0; a < 3; ++a) { e0[a] = poly[1].x[a] - poly[0].x[a]; e1[a] = poly[2].x[a] - poly[0].x[a]; }
    double nrm[3] = {e0[1] * e1[2] - e0[2] * e1[1], e0[2] * e1[0] - e0[0] * e1[2],
                     e0[0] * e1[1] - e0[1] * e1[0]};
    double nn = std::sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
    for (int a = 0; a < 3; ++a) nrm[a] /= nn;
    // clip to the closed cell, planes x>=, x<=, y>=, y<=, z>=, z<=
    for (int a = 0; a < 3 && poly.size() >= 3; ++a) {
      poly = clip(poly, a, (double)c[a], true);
      if (poly.size() >= 3) poly = clip(poly, a, (double)c[a] + 1.0, false);
    }
    if (poly.size() < 3) continue;
    const double tw = tri_w ? tri_w[t] : 1.0;
    // gradient of f on the triangle in world units: sum over corners m of
    // f_m grad(lambda_m), where grad(lambda_1) = (e2 x n)/|n|^2 and
    // grad(lambda_2) = (n x e1)/|n|^2 with e1, e2 the edges from corner 0 and
    // n = e1 x e2 (each is orthogonal to the opposite edge and to n, and rises
    // by 1 along its own edge); zero on a triangle of zero area
    std::vector<double> gf(grad_rhs ? 3 * (size_t)k : 0, 0.0);
    if (grad_rhs) {
      double w1[3], w2[3];
      for (int a = 0; a < 3; ++a) {
        w1[a] = h.V[3 * (size_t)f[1] + a] - h.V[3 * (size_t)f[0] + a];
        w2[a] = h.V[3 * (size_t)f[2] + a] - h.V[3 * (size_t)f[0] + a];
      }
      const double nw[3] = {w1[1] * w2[2] - w1[2] * w2[1], w1[2] * w2[0] - w1[0] * w2[2],
                            w1[0] * w2[1] - w1[1] * w2[0]};
      const double n2 = nw[0] * nw[0] + nw[1] * nw[1] + nw[2] * nw[2];
      if (n2 > 0.0) {
        const double gl1[3] = {(w2[1] * nw[2] - w2[2] * nw[1]) / n2, (w2[2] * nw[0] - w2[0] * nw[2]) / n2,
                               (w2[0] * nw[1] - w2[1] * nw[0]) / n2};
        const double gl2[3] = {(nw[1] * w1[2] - nw[2] * w1[1]) / n2, (nw[2] * w1[0] - nw[0] * w1[2]) / n2,
                               (nw[0] * w1[1] - nw[1] * w1[0]) / n2};
        for (int col = 0; col < k; ++col) {
          const double* fc = fv + (size_t)col * h.nv;
          const double d1 = fc[f[1]] - fc[f[0]], d2 = fc[f[2]] - fc[f[0]];
          for (int a = 0; a < 3; ++a) gf[3 * (size_t)col + a] = d1 * gl1[a] + d2 * gl2[a];
        }
      }
    }
    std::vector<double> Me(NB * NB, 0.0), Le(NB * NB, 0.0);
    std::vector<double> be((size_t)NB * (k > 0 ? k : 1), 0.0);
    // fan from vertex 0; collapsed Gauss-Legendre on each sub-triangle
    for (size_t s = 1; s + 1 < poly.size(); ++s) {
      const PV& P0 = poly[0];
      const PV& P1 = poly[s];
      const PV& P2 = poly[s + 1];
      double a1[3], a2[3];
      for (int a = 0; a < 3; ++a) { a1[a] = P1.x[a] - P0.x[a]; a2[a] = P2.x[a] - P0.x[a]; }
      double cr[3] = {a1[1] * a2[2] - a1[2] * a2[1], a1[2] * a2[0] - a1[0] * a2[2],
                      a1[0] * a2[1] - a1[1] * a2[0]};
      double area = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      for (int iu = 0; iu < nq; ++iu)
        for (int iv = 0; iv < nq; ++iv) {
          double xi = gx[iu], eta = (1.0 - gx[iu]) * gx[iv];
          // tri_w weights the mass only (M_t of an evolved surface, L_0 fixed)
          double wq = 2.0 * area * gw[iu] * gw[iv] * (1.0 - gx[iu]) * hd * hd;
          double wqm = wq * tw;
          double x[3], lam[3];
          for (int a = 0; a < 3; ++a) {
            x[a] = P0.x[a] + xi * a1[a] + eta * a2[a];
            lam[a] = P0.l[a] + xi * (P1.l[a] - P0.l[a]) + eta * (P2.l[a] - P0.l[a]);
          }
          double lc[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
          double phi[27], g[27][3];
          for (int jz = 0; jz < W; ++jz)
            for (int jy = 0; jy < W; ++jy)
              for (int jx = 0; jx < W; ++jx) {
                int j = jx + W * jy + W * W * jz;
                double bx = b1d(h.degree, jx, lc[0]), by = b1d(h.degree, jy, lc[1]),
                       bz = b1d(h.degree, jz, lc[2]);
                phi[j] = bx * by * bz;
                double gr[3] = {db1d(h.degree, jx, lc[0]) * by * bz / hd,
                                bx * db1d(h.degree, jy, lc[1]) * bz / hd,
                                bx * by * db1d(h.degree, jz, lc[2]) / hd};
                double gn = gr[0] * nrm[0] + gr[1] * nrm[1] + gr[2] * nrm[2];
                for (int a = 0; a < 3; ++a) g[j][a] = gr[a] - gn * nrm[a];
              }
          if (want_matrix)
            for (int i = 0; i < NB; ++i)
              for (int j = 0; j < NB; ++j) {
                Me[i * NB + j] += wqm * phi[i] * phi[j];
                Le[i * NB + j] += wq * (g[i][0] * g[j][0] + g[i][1] * g[j][1] + g[i][2] * g[j][2]);
              }
          if (rhs && grad_rhs)
            for (int col = 0; col < k; ++col) {
              const double* gc = &gf[3 * (size_t)col];
              for (int i = 0; i < NB; ++i)
                be[(size_t)col * NB + i] += wq * (gc[0] * g[i][0] + gc[1] * g[i][1] + gc[2] * g[i][2]);
            }
          else if (rhs)
            for (int col = 0; col < k; ++col) {
              const double* fc = fv + (size_t)col * h.nv;
              double fx = lam[0] * fc[f[0]] + lam[1] * fc[f[1]] + lam[2] * fc[f[2]];
              for (int i = 0; i < NB; ++i) be[(size_t)col * NB + i] += wq * phi[i] * fx;
            }
        }
    }
    if (want_matrix)
      for (int i = 0; i < NB; ++i)
        for (int j = 0; j < NB; ++j) row_add(rows[ridx[i]], ridx[j], Me[i * NB + j], Le[i * NB + j]);
    if (rhs)
      for (int col = 0; col < k; ++col)
        for (int i = 0; i < NB; ++i) rhs[(size_t)col * n + ridx[i]] += be[(size_t)col * NB + i];
  }
  if (want_matrix) {
    L.Aptr.assign(n + 1, 0);
    L.Acol.clear(); L.Mval.clear(); L.Lval.clear();
    for (long r = 0; r < n; ++r) {
      std::vector<int> ord(rows[r].col.size());
      std::iota(ord.begin(), ord.end(), 0);
      std::sort(ord.begin(), ord.end(), [&](int a, int b) { return rows[r].col[a] < rows[r].col[b]; });
      for (int i : ord) {
        L.Acol.push_back(rows[r].col[i]);
        L.Mval.push_back(rows[r].m[i]);
        L.Lval.push_back(rows[r].l[i]);
      }
      L.Aptr[r + 1] = (long)L.Acol.size();
    }
    L.assembled = true;
  }
  return true;
}

// ------------------------------------------------------------------- solver
struct SysLevel {
  long n = 0;
  const std::vector<long>* ptr = nullptr;
  const std::vector<int>* col = nullptr;
  std::vector<double> a;          // A = M + t L values (same pattern)
  std::vector<double> diag;
  std::vector<std::vector<long>> colour_rows;  // rows of each colour, canonical order
  // dense Cholesky factor at the coarsest level (lower, row-major)
  std::vector<double> chol;
  bool direct = false;
  const Level* lev = nullptr;
  // cell-block Schwarz smoother: function lists of the blocks, the inverse of
  // each block (m x m row-major) and each block's weight
  std::vector<std::vector<long>> blocks;
  std::vector<std::vector<double>> binv;
  std::vector<double> bweight;
  double block_omega = 1.0;       // damping of this level's block corrections
};

int colour_of(int degree, uint64_t key) {
  long c[3];
  demorton3(key, c);
  if (degree == 1) return (int)((c[0] & 1) + 2 * (c[1] & 1) + 4 * (c[2] & 1));
  return (int)((c[0] % 3) + 3 * (c[1] % 3) + 9 * (c[2] % 3));
}

bool cholesky(std::vector<double>& A, long n) {
  for (long j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (long p = 0; p < j; ++p) s -= A[j * n + p] * A[j * n + p];
    if (!(s > 0.0)) return false;
    double ljj = std::sqrt(s);
    A[j * n + j] = ljj;
    for (long i = j + 1; i < n; ++i) {
      double v = A[i * n + j];
      for (long p = 0; p < j; ++p) v -= A[i * n + p] * A[j * n + p];
      A[i * n + j] = v / ljj;
    }
    for (long i = 0; i < j; ++i) A[i * n + j] = 0.0;
  }
  return true;
}

void chol_solve(const std::vector<double>& Lf, long n, double* x) {
  for (long i = 0; i < n; ++i) {
    double v = x[i];
    for (long p = 0; p < i; ++p) v -= Lf[i * n + p] * x[p];
    x[i] = v / Lf[i * n + i];
  }
  for (long i = n - 1; i >= 0; --i) {
    double v = x[i];
    for (long p = i + 1; p < n; ++p) v -= Lf[p * n + i] * x[p];
    x[i] = v / Lf[i * n + i];
  }
}

struct Solver {
  Hier* h = nullptr;
  std::vector<SysLevel> sl;   // index = depth
  int nu1 = 2, nu2 = 2;
  int gamma = 1;              // coarse corrections per level: 1 V-cycle, 2 W-cycle
  int nu_coarse = 0;          // sweeps each way below the finest depth (0: nu1, nu2)
  int eps_used = 0;
  int smoother = 0;           // 0 multicolour Gauss-Seidel, 1 cell-block Schwarz
};

void gs_sweep(const SysLevel& S, const double* b, double* x, int k, bool forward);
void residual(const SysLevel& S, const double* b, const double* x, int k, double* r);

// Entry (r, c) of A at one level (0 when not stored)
double a_entry(const SysLevel& S, long r, long c) {
  long lo = (*S.ptr)[r], hi = (*S.ptr)[r + 1];
  while (lo < hi) {
    long mid = (lo + hi) / 2;
    if ((*S.col)[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  return lo < (*S.ptr)[r + 1] && (*S.col)[lo] == c ? S.a[lo] : 0.0;
}

// Cell blocks of the Schwarz smoother at depth d (trilinear functions only).
// A block holds, for one occupied cell, every function whose support
// contains the cell and whose component holds one of the cell's triangles:
// the functions at the cell's 8 corners, one per component met in the cell.
// Functions of zero computed mass are left out.  A cell with more than
// BLOCK_CAP such functions (many separate pieces of surface in one cell, at
// coarse split depths) gives one single-function block per function instead.
// Each block's inverse is that of its unit-diagonal-scaled matrix plus eps I,
// scaled back: D^-1/2 (D^-1/2 A_b D^-1/2 + eps I)^-1 D^-1/2 (the coarsest
// solve's treatment, which keeps exactly dependent functions bounded).
constexpr int BLOCK_CAP = 16;

void build_blocks(const Hier& h, int d, SysLevel& S, double eps) {
  const Level& L = h.lev[d];
  S.blocks.clear();
  S.binv.clear();
  std::vector<std::vector<long>> raw;
  size_t p = 0;
  while (p < L.pairs.size()) {
    const uint64_t cell = L.pairs[p].first;
    long c[3];
    demorton3(cell, c);
    std::vector<long> fs;
    size_t q = p;
    for (; q < L.pairs.size() && L.pairs[q].first == cell; ++q)
      for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
          for (int dx = 0; dx < 2; ++dx) {
            int f = func_of(L, morton3(c[0] + dx, c[1] + dy, c[2] + dz), L.pairs[q].second);
            if (f >= 0 && S.diag[f] > 0.0) fs.push_back(f);
          }
    std::sort(fs.begin(), fs.end());
    fs.erase(std::unique(fs.begin(), fs.end()), fs.end());
    if ((int)fs.size() > BLOCK_CAP) {
      for (long f : fs) raw.push_back({f});
    } else if (!fs.empty()) {
      raw.push_back(fs);
    }
    p = q;
  }
  // weight of a block: 1 / (the largest number of blocks holding one of its
  // functions), so that the weights of the blocks holding any function sum to
  // at most 1
  std::vector<double> mult(S.n, 0.0);
  for (const auto& b : raw)
    for (long f : b) mult[f] += 1.0;
  S.bweight.clear();
  for (const auto& b : raw) {
    double mx = 0.0;
    for (long f : b) mx = std::max(mx, mult[f]);
    S.bweight.push_back(1.0 / mx);
  }
  for (const auto& b : raw) {
    const long m = (long)b.size();
    std::vector<double> sc(m), A((size_t)m * m), inv((size_t)m * m, 0.0);
    for (long i = 0; i < m; ++i) sc[i] = 1.0 / std::sqrt(S.diag[b[i]]);
    for (long i = 0; i < m; ++i)
      for (long j = 0; j < m; ++j) A[i * m + j] = a_entry(S, b[i], b[j]) * sc[i] * sc[j];
    for (long i = 0; i < m; ++i) A[i * m + i] += eps;
    if (!cholesky(A, m)) throw std::runtime_error("cell block not positive definite");
    for (long j = 0; j < m; ++j) {
      std::vector<double> e(m, 0.0);
      e[j] = 1.0;
      chol_solve(A, m, e.data());
      for (long i = 0; i < m; ++i) inv[i * m + j] = sc[i] * e[i] * sc[j];
    }
    S.blocks.push_back(b);
    S.binv.push_back(inv);
  }
}

// One cell-block Schwarz sweep: r = b - A x, then
//   x += omega sum over blocks B of w_B R_B^T A_B^-1 R_B r
// with w_B the block's weight.  The map is symmetric (the same before and
// after the coarse correction): the error goes to (I - omega B A) e with B
// the weighted block sum, an A-norm contraction only while omega times the
// largest eigenvalue of B A stays below 2.  The weights bound what blocks
// sharing a function add, but not the coupling of blocks that share none,
// so that eigenvalue can pass 2 and the damping is the caller's to choose.
void block_sweep(const SysLevel& S, const double* b, double* x, int k, double omega) {
  std::vector<double> r((size_t)S.n * k), u((size_t)S.n * k, 0.0);
  residual(S, b, x, k, r.data());
  for (size_t bi = 0; bi < S.blocks.size(); ++bi) {
    const std::vector<long>& blk = S.blocks[bi];
    const long m = (long)blk.size();
    for (int q = 0; q < k; ++q)
      for (long i = 0; i < m; ++i) {
        double acc = 0.0;
        for (long j = 0; j < m; ++j) acc += S.binv[bi][i * m + j] * r[(size_t)q * S.n + blk[j]];
        u[(size_t)q * S.n + blk[i]] += S.bweight[bi] * acc;
      }
  }
  for (size_t e = 0; e < u.size(); ++e) x[e] += omega * u[e];
}

void smooth(const Solver& sv, const SysLevel& S, const double* b, double* x, int k, bool forward) {
  if (sv.smoother == 1) block_sweep(S, b, x, k, S.block_omega);
  else gs_sweep(S, b, x, k, forward);
}

// one Gauss-Seidel sweep over all colours (forward or reverse), x n x k col-major
void gs_sweep(const SysLevel& S, const double* b, double* x, int k, bool forward) {
  const int nc = (int)S.colour_rows.size();
  for (int ci = 0; ci < nc; ++ci) {
    int c = forward ? ci : nc - 1 - ci;
    const std::vector<long>& rows = S.colour_rows[c];
    // rows of one colour never couple: in the OpenMP build they are shared out
    // (each row computed by one thread exactly as here, so no result changes)
#pragma omp parallel for schedule(static)
    for (long j = 0; j < (long)rows.size(); ++j)
      for (int q = 0; q < k; ++q) {
        const long r = rows[j];
        const double* xq = x + (size_t)q * S.n;
        double acc = 0.0;
        if (S.diag[r] == 0.0) continue;   // zero-mass function: all-zero row, nothing to relax
        for (long e = (*S.ptr)[r]; e < (*S.ptr)[r + 1]; ++e) acc += S.a[e] * xq[(*S.col)[e]];
        x[(size_t)q * S.n + r] += (b[(size_t)q * S.n + r] - acc) / S.diag[r];
      }
  }
}

void residual(const SysLevel& S, const double* b, const double* x, int k, double* r) {
  for (int q = 0; q < k; ++q)
#pragma omp parallel for schedule(static)
    for (long i = 0; i < S.n; ++i) {
      double acc = 0.0;
      for (long e = (*S.ptr)[i]; e < (*S.ptr)[i + 1]; ++e) acc += S.a[e] * x[(size_t)q * S.n + (*S.col)[e]];
      r[(size_t)q * S.n + i] = b[(size_t)q * S.n + i] - acc;
    }
}

void matvec(const SysLevel& S, const double* x, int k, double* y) {
  for (int q = 0; q < k; ++q)
#pragma omp parallel for schedule(static)
    for (long i = 0; i < S.n; ++i) {
      double acc = 0.0;
      for (long e = (*S.ptr)[i]; e < (*S.ptr)[i + 1]; ++e) acc += S.a[e] * x[(size_t)q * S.n + (*S.col)[e]];
      y[(size_t)q * S.n + i] = acc;
    }
}

// One multigrid cycle at depth d on (b, x), x given: nu1 forward sweeps, the
// coarse correction (gamma cycles at depth d - 1 from zero), nu2 reverse
// sweeps; the coarsest depth is solved directly or relaxed.
void vcycle(Solver& sv, int d, const double* b, double* x, int k) {
  SysLevel& S = sv.sl[d];
  const bool coarse = d < sv.h->D && sv.nu_coarse > 0;
  const int nu1 = coarse ? sv.nu_coarse : sv.nu1, nu2 = coarse ? sv.nu_coarse : sv.nu2;
  if (d == sv.h->d0) {
    if (S.direct) {
      // x = D^-1/2 (D^-1/2 A D^-1/2 + eps I)^-1 D^-1/2 b
      for (int q = 0; q < k; ++q) {
        double* xq = x + (size_t)q * S.n;
        for (long i = 0; i < S.n; ++i)
          xq[i] = S.diag[i] > 0.0 ? b[(size_t)q * S.n + i] / std::sqrt(S.diag[i]) : 0.0;
        chol_solve(S.chol, S.n, xq);
        for (long i = 0; i < S.n; ++i) xq[i] = S.diag[i] > 0.0 ? xq[i] / std::sqrt(S.diag[i]) : 0.0;
      }
    } else {
      for (int s = 0; s < nu1; ++s) smooth(sv, S, b, x, k, true);
      for (int s = 0; s < nu2; ++s) smooth(sv, S, b, x, k, false);
    }
    return;
  }
  for (int s = 0; s < nu1; ++s) smooth(sv, S, b, x, k, true);
  std::vector<double> r((size_t)S.n * k);
  residual(S, b, x, k, r.data());
  const Level& Lf = sv.h->lev[d];
  SysLevel& C = sv.sl[d - 1];
  std::vector<double> bc((size_t)C.n * k, 0.0), xc((size_t)C.n * k, 0.0);
  for (int q = 0; q < k; ++q)
    for (long i = 0; i < S.n; ++i)
      for (long e = Lf.Pptr[i]; e < Lf.Pptr[i + 1]; ++e)
        bc[(size_t)q * C.n + Lf.Pcol[e]] += Lf.Pw[e] * r[(size_t)q * S.n + i];
  // the coarse problem gets gamma cycles from zero (one: V-cycle, two: W-cycle)
  for (int g = 0; g < sv.gamma; ++g) vcycle(sv, d - 1, bc.data(), xc.data(), k);
  for (int q = 0; q < k; ++q)
#pragma omp parallel for schedule(static)
    for (long i = 0; i < S.n; ++i)
      for (long e = Lf.Pptr[i]; e < Lf.Pptr[i + 1]; ++e)
        x[(size_t)q * S.n + i] += Lf.Pw[e] * xc[(size_t)q * C.n + Lf.Pcol[e]];
  for (int s = 0; s < nu2; ++s) smooth(sv, S, b, x, k, false);
}

double col_norm(const double* v, long n) {
  double s = 0;
  for (long i = 0; i < n; ++i) s += v[i] * v[i];
  return std::sqrt(s);
}

}  // namespace

// =================================================================== C ABI
extern "C" {

struct OracleHandle { Hier h; };

const char* oracle_error(void* hp) { return ((OracleHandle*)hp)->h.err.c_str(); }

// Returns a handle (never null); oracle_ok() tells whether the build succeeded.
void* oracle_build(const double* V, long nv, const int* F, long nt, int depth, int degree,
                   int split, int min_depth, long max_coarse, const double* box) {
  OracleHandle* H = new OracleHandle();
  Hier& h = H->h;
  h.D = depth; h.degree = degree; h.split = split; h.min_depth = min_depth;
  h.max_coarse = max_coarse; h.nv = nv; h.nt = nt;
  auto t0 = std::chrono::steady_clock::now();
  if (depth < 1 || depth > 12 || (degree != 1 && degree != 2) || nt <= 0 || nv <= 0 ||
      nt >= (1L << 24)) {
    h.err = "invalid arguments";
  } else {
    h.V.assign(V, V + 3 * nv);
    if (!build(h, V, F, box) && h.err.empty()) h.err = "build failed";
  }
  h.timing[0] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return H;
}
int oracle_ok(void* hp) { return ((OracleHandle*)hp)->h.err.empty() ? 1 : 0; }
void oracle_free(void* hp) { delete (OracleHandle*)hp; }

void oracle_cube(void* hp, double* out4) {
  Hier& h = ((OracleHandle*)hp)->h;
  out4[0] = h.o[0]; out4[1] = h.o[1]; out4[2] = h.o[2]; out4[3] = h.s;
}
int oracle_coarsest(void* hp) { return ((OracleHandle*)hp)->h.d0; }
double oracle_timing(void* hp, int i) { return ((OracleHandle*)hp)->h.timing[i]; }

// what: 0 pairs, 1 functions, 2 (support, triangle) entries, 3 prolongation nnz,
//       4 matrix nnz, 5 occupied cells
long oracle_count(void* hp, int d, int what) {
  Hier& h = ((OracleHandle*)hp)->h;
  if (d < 0 || d > h.D) return -1;
  const Level& L = h.lev[d];
  switch (what) {
    case 0: return (long)L.pairs.size();
    case 1: return (d >= h.d0) ? (long)L.fkey.size() : -1;
    case 2: return (d >= h.d0) ? (long)L.stri.size() : -1;
    case 3: return (d > h.d0) ? (long)L.Pcol.size() : -1;
    case 4: return L.assembled ? (long)L.Acol.size() : -1;
    case 5: {
      long c = 0;
      for (size_t i = 0; i < L.pairs.size(); ++i)
        if (i == 0 || L.pairs[i].first != L.pairs[i - 1].first) ++c;
      return c;
    }
  }
  return -1;
}

void oracle_pairs(void* hp, int d, uint64_t* key, int* tri) {
  const Level& L = ((OracleHandle*)hp)->h.lev[d];
  for (size_t i = 0; i < L.pairs.size(); ++i) { key[i] = L.pairs[i].first; tri[i] = L.pairs[i].second; }
}
void oracle_functions(void* hp, int d, uint64_t* key, int* comp, int* rep) {
  const Level& L = ((OracleHandle*)hp)->h.lev[d];
  for (size_t i = 0; i < L.fkey.size(); ++i) { key[i] = L.fkey[i]; comp[i] = L.fcomp[i]; rep[i] = L.frep[i]; }
}
void oracle_support_entries(void* hp, int d, uint64_t* key, int* tri, int* func) {
  const Level& L = ((OracleHandle*)hp)->h.lev[d];
  for (size_t i = 0; i < L.stri.size(); ++i) {
    key[i] = L.stri[i].first; tri[i] = L.stri[i].second; func[i] = L.stri_func[i];
  }
}
void oracle_prolongation(void* hp, int d, long* ptr, int* col, double* w) {
  const Level& L = ((OracleHandle*)hp)->h.lev[d];
  std::copy(L.Pptr.begin(), L.Pptr.end(), ptr);
  std::copy(L.Pcol.begin(), L.Pcol.end(), col);
  std::copy(L.Pw.begin(), L.Pw.end(), w);
}

// Assemble M and L at every built depth; tri_w nullable.
int oracle_assemble(void* hp, const double* tri_w) {
  Hier& h = ((OracleHandle*)hp)->h;
  if (!h.err.empty()) return -1;
  auto t0 = std::chrono::steady_clock::now();
  for (int d = h.d0; d <= h.D; ++d)
    if (!assemble_level(h, d, tri_w, nullptr, 0, nullptr, true)) return -1;
  h.timing[1] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return 0;
}

void oracle_matrix(void* hp, int d, long* ptr, int* col, double* mval, double* lval) {
  const Level& L = ((OracleHandle*)hp)->h.lev[d];
  std::copy(L.Aptr.begin(), L.Aptr.end(), ptr);
  std::copy(L.Acol.begin(), L.Acol.end(), col);
  std::copy(L.Mval.begin(), L.Mval.end(), mval);
  std::copy(L.Lval.begin(), L.Lval.end(), lval);
}

// b = int f b_i at depth d (finest by default), f per-vertex (nv x k col-major)
int oracle_load_vector(void* hp, int d, const double* fv, int k, double* b) {
  Hier& h = ((OracleHandle*)hp)->h;
  if (!h.err.empty() || d < h.d0 || d > h.D) return -1;
  return assemble_level(h, d, nullptr, fv, k, b, false) ? 0 : -1;
}

// b_i = int <grad f, grad b_i> at depth d (the gradient constraint of the
// screened Poisson colour fit, Section 5.2), f per-vertex (nv x k col-major)
int oracle_gradient_load(void* hp, int d, const double* fv, int k, double* b) {
  Hier& h = ((OracleHandle*)hp)->h;
  if (!h.err.empty() || d < h.d0 || d > h.D) return -1;
  return assemble_level(h, d, nullptr, fv, k, b, false, true) ? 0 : -1;
}

// Solve (M + t L) x = b at the finest depth.
// mode 0: stationary multigrid, x <- x + V(b - A x) with V a (nu1, nu2) cycle,
//         a V-cycle (gamma 1) or a W-cycle (gamma 2, Section 5.2); below the
//         finest depth nu_coarse sweeps each way when it is positive.
// mode 1: conjugate gradients preconditioned by one V-cycle (V is symmetric:
//         forward colour order before the coarse correction, reverse after,
//         nu1 == nu2, exact coarse solve), one independent CG per column.
// The coarsest level is solved with a Cholesky factor of the unit-diagonal
// scaled matrix plus coarse_eps * Id (the eps * Id remedy that the Discussion
// closing Section 5 gives for singular systems), when it holds at most
// max_coarse rows;
// otherwise it is only relaxed.
// b, x: n x k col-major; x0_given: start from x, else x = 0.
// stats[0] = V-cycles applied, stats[1] = max relative residual, stats[2] =
// eps used (always 1 with a direct coarsest solve), stats[3] = seconds.
// history (nullable, max_iter+1 entries) receives the max relative residual
// before the first and after every iteration (true residual).
int oracle_solve(void* hp, double t, double rtol, int max_iter, int nu1, int nu2,
                 const double* b, int k, double* x, int x0_given, double* stats,
                 double* history, int mode, double coarse_eps, int gamma, int nu_coarse, int smoother,
                 double block_omega, const double* level_omega) {
  Hier& h = ((OracleHandle*)hp)->h;
  if (!h.err.empty()) return -1;
  if (gamma < 1 || gamma > 2) { h.err = "gamma must be 1 or 2"; return -1; }
  if (nu_coarse < 0) { h.err = "nu_coarse must be >= 0"; return -1; }
  if (smoother < 0 || smoother > 1 || (smoother == 1 && h.degree != 1)) {
    h.err = "smoother: 0 Gauss-Seidel, 1 cell blocks (degree 1)";
    return -1;
  }
  auto t0 = std::chrono::steady_clock::now();
  Solver sv;
  sv.h = &h; sv.nu1 = nu1; sv.nu2 = nu2; sv.gamma = gamma; sv.nu_coarse = nu_coarse; sv.smoother = smoother;
  sv.sl.assign(h.D + 1, SysLevel());
  for (int d = h.d0; d <= h.D; ++d) {
    Level& L = h.lev[d];
    if (!L.assembled) { h.err = "solve before assemble"; return -1; }
    SysLevel& S = sv.sl[d];
    S.lev = &L;
    S.n = (long)L.fkey.size();
    S.ptr = &L.Aptr; S.col = &L.Acol;
    S.a.resize(L.Mval.size());
    for (size_t e = 0; e < L.Mval.size(); ++e) S.a[e] = L.Mval[e] + t * L.Lval[e];
    S.diag.assign(S.n, 0.0);
    for (long r = 0; r < S.n; ++r)
      for (long e = L.Aptr[r]; e < L.Aptr[r + 1]; ++e)
        if (L.Acol[e] == r) S.diag[r] = S.a[e];
    const int ncol = h.degree == 1 ? 8 : 27;
    S.colour_rows.assign(ncol, {});
    for (long r = 0; r < S.n; ++r) S.colour_rows[colour_of(h.degree, L.fkey[r])].push_back(r);
    // block damping: one value for every depth, or level_omega[d - d0]
    S.block_omega = level_omega ? level_omega[d - h.d0] : block_omega;
    if (smoother == 1) {
      try {
        build_blocks(h, d, S, coarse_eps);
      } catch (const std::exception& e) {
        h.err = e.what();
        return -1;
      }
    }
  }
  {
    SysLevel& S = sv.sl[h.d0];
    if (h.max_coarse > 0 && S.n <= h.max_coarse) {
      S.direct = true;
      // factor D^-1/2 A D^-1/2 + eps I (unit diagonal before the shift)
      S.chol.assign((size_t)S.n * S.n, 0.0);
      for (long r = 0; r < S.n; ++r)
        for (long e = (*S.ptr)[r]; e < (*S.ptr)[r + 1]; ++e) {
          long c = (*S.col)[e];
          if (S.diag[r] > 0.0 && S.diag[c] > 0.0)
            S.chol[(size_t)r * S.n + c] = S.a[e] / std::sqrt(S.diag[r] * S.diag[c]);
        }
      // a zero-mass function gets an identity row (its right-hand side is 0)
      for (long r = 0; r < S.n; ++r) S.chol[(size_t)r * S.n + r] = (S.diag[r] > 0.0 ? S.chol[(size_t)r * S.n + r] : 1.0) + coarse_eps;
      sv.eps_used = 1;
      if (!cholesky(S.chol, S.n)) { h.err = "coarse Cholesky failed"; return -1; }
    }
  }
  auto t1 = std::chrono::steady_clock::now();
  h.timing[2] = std::chrono::duration<double>(t1 - t0).count();
  SysLevel& Sf = sv.sl[h.D];
  const long n = Sf.n;
  if (!x0_given) std::fill(x, x + n * k, 0.0);
  std::vector<double> bn(k), r((size_t)n * k);
  for (int q = 0; q < k; ++q) bn[q] = col_norm(b + (size_t)q * n, n);
  auto relres = [&]() {
    residual(Sf, b, x, k, r.data());
    double m = 0;
    for (int q = 0; q < k; ++q) {
      double rn = col_norm(r.data() + (size_t)q * n, n);
      double v = bn[q] > 0 ? rn / bn[q] : rn;
      if (!(v <= m)) m = v;   // keeps NaN
    }
    return m;
  };
  double rr = relres();
  if (history) history[0] = rr;
  int it = 0, cycles = 0;
  if (mode == 0) {
    std::vector<double> e((size_t)n * k);
    while (rr > rtol && it < max_iter) {
      std::fill(e.begin(), e.end(), 0.0);
      vcycle(sv, h.D, r.data(), e.data(), k);   // r holds b - A x from relres()
      for (size_t i = 0; i < e.size(); ++i) x[i] += e[i];
      ++it; ++cycles;
      rr = relres();
      if (history) history[it] = rr;
      if (!std::isfinite(rr)) break;
    }
  } else {
    // one CG per column; r = b - A x already computed
    std::vector<double> z((size_t)n * k, 0.0), p((size_t)n * k), q((size_t)n * k);
    std::vector<double> rz(k, 0.0);
    std::vector<char> done(k, 0);
    for (int c = 0; c < k; ++c) {
      double rn = col_norm(r.data() + (size_t)c * n, n);
      done[c] = (bn[c] > 0 ? rn / bn[c] : rn) <= rtol;
    }
    vcycle(sv, h.D, r.data(), z.data(), k);
    ++cycles;
    for (int c = 0; c < k; ++c) {
      double s = 0;
      for (long i = 0; i < n; ++i) s += r[(size_t)c * n + i] * z[(size_t)c * n + i];
      rz[c] = s;
    }
    p = z;
    while (rr > rtol && it < max_iter) {
      matvec(Sf, p.data(), k, q.data());   // q = A p
      for (int c = 0; c < k; ++c) {
        if (done[c]) continue;
        double pq = 0;
        for (long i = 0; i < n; ++i) pq += p[(size_t)c * n + i] * q[(size_t)c * n + i];
        double alpha = pq != 0.0 ? rz[c] / pq : 0.0;
        for (long i = 0; i < n; ++i) {
          x[(size_t)c * n + i] += alpha * p[(size_t)c * n + i];
          r[(size_t)c * n + i] -= alpha * q[(size_t)c * n + i];
        }
        double rn = col_norm(r.data() + (size_t)c * n, n);
        if ((bn[c] > 0 ? rn / bn[c] : rn) <= rtol) done[c] = 1;
      }
      ++it;
      std::vector<double> rsave = r;
      rr = relres();   // true residual of the current iterate
      r = rsave;
      if (history) history[it] = rr;
      if (rr <= rtol || !std::isfinite(rr)) break;
      for (int c = 0; c < k; ++c) done[c] = 0;
      std::fill(z.begin(), z.end(), 0.0);
      vcycle(sv, h.D, r.data(), z.data(), k);
      ++cycles;
      for (int c = 0; c < k; ++c) {
        double s = 0;
        for (long i = 0; i < n; ++i) s += r[(size_t)c * n + i] * z[(size_t)c * n + i];
        double beta = rz[c] != 0.0 ? s / rz[c] : 0.0;
        rz[c] = s;
        for (long i = 0; i < n; ++i) p[(size_t)c * n + i] = z[(size_t)c * n + i] + beta * p[(size_t)c * n + i];
      }
    }
  }
  h.timing[3] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
  if (stats) {
    stats[0] = cycles; stats[1] = rr; stats[2] = sv.eps_used; stats[3] = h.timing[3];
    stats[4] = it;
  }
  return rr <= rtol ? 0 : 1;
}

// y = A x at depth d with A = M + t L (x, y n x k col-major)
int oracle_apply(void* hp, int d, double t, const double* x, int k, double* y) {
  Hier& h = ((OracleHandle*)hp)->h;
  if (d < h.d0 || d > h.D || !h.lev[d].assembled) return -1;
  const Level& L = h.lev[d];
  const long n = (long)L.fkey.size();
  for (int q = 0; q < k; ++q)
    for (long i = 0; i < n; ++i) {
      double acc = 0;
      for (long e = L.Aptr[i]; e < L.Aptr[i + 1]; ++e)
        acc += (L.Mval[e] + t * L.Lval[e]) * x[(size_t)q * n + L.Acol[e]];
      y[(size_t)q * n + i] = acc;
    }
  return 0;
}

// One forward multicolour Gauss-Seidel sweep at depth d (for sweep-level checks)
int oracle_gs_sweep(void* hp, int d, double t, const double* b, int k, double* x, int forward) {
  Hier& h = ((OracleHandle*)hp)->h;
  if (d < h.d0 || d > h.D || !h.lev[d].assembled) return -1;
  const Level& L = h.lev[d];
  SysLevel S;
  S.n = (long)L.fkey.size();
  S.ptr = &L.Aptr; S.col = &L.Acol;
  S.a.resize(L.Mval.size());
  for (size_t e = 0; e < L.Mval.size(); ++e) S.a[e] = L.Mval[e] + t * L.Lval[e];
  S.diag.assign(S.n, 0.0);
  for (long r = 0; r < S.n; ++r)
    for (long e = L.Aptr[r]; e < L.Aptr[r + 1]; ++e)
      if (L.Acol[e] == r) S.diag[r] = S.a[e];
  S.colour_rows.assign(h.degree == 1 ? 8 : 27, {});
  for (long r = 0; r < S.n; ++r) S.colour_rows[colour_of(h.degree, L.fkey[r])].push_back(r);
  gs_sweep(S, b, x, k, forward != 0);
  return 0;
}

// One cell-block Schwarz sweep at depth d (for sweep-level checks; forward
// and backward are the same map); eps as in the solver's block inverses
int oracle_block_sweep(void* hp, int d, double t, const double* b, int k, double* x, int forward, double eps,
                       double omega) {
  Hier& h = ((OracleHandle*)hp)->h;
  if (d < h.d0 || d > h.D || !h.lev[d].assembled || h.degree != 1) return -1;
  const Level& L = h.lev[d];
  SysLevel S;
  S.n = (long)L.fkey.size();
  S.ptr = &L.Aptr; S.col = &L.Acol;
  S.a.resize(L.Mval.size());
  for (size_t e = 0; e < L.Mval.size(); ++e) S.a[e] = L.Mval[e] + t * L.Lval[e];
  S.diag.assign(S.n, 0.0);
  for (long r = 0; r < S.n; ++r)
    for (long e = L.Aptr[r]; e < L.Aptr[r + 1]; ++e)
      if (L.Acol[e] == r) S.diag[r] = S.a[e];
  try {
    build_blocks(h, d, S, eps);
  } catch (const std::exception& e) {
    h.err = e.what();
    return -1;
  }
  (void)forward;   // the block sweep is the same map in both directions
  block_sweep(S, b, x, k, omega);
  return 0;
}

// Values at mesh vertices of u = sum_i x_i b_i (finest depth), using for each
// vertex the smallest triangle that contains it to pick each corner's component.
int oracle_eval_vertices(void* hp, const double* x, int k, double* out) {
  Hier& h = ((OracleHandle*)hp)->h;
  const int D = h.D;
  const Level& L = h.lev[D];
  const long n = (long)L.fkey.size();
  const int W = width(h.degree);
  const long top = (1L << D) - 1;
  for (long v = 0; v < h.nv; ++v) {
    for (int q = 0; q < k; ++q) out[(size_t)q * h.nv + v] = 0.0;
    if (h.vt_ptr[v] == h.vt_ptr[v + 1]) continue;
    const int t = h.vt_tri[h.vt_ptr[v]];
    long c[3];
    double lc[3];
    for (int a = 0; a < 3; ++a) {
      double u = h.U[3 * v + a];
      c[a] = std::max(0L, std::min(top, (long)std::floor(u)));
      lc[a] = u - (double)c[a];
    }
    for (int jz = 0; jz < W; ++jz)
      for (int jy = 0; jy < W; ++jy)
        for (int jx = 0; jx < W; ++jx) {
          double phi = b1d(h.degree, jx, lc[0]) * b1d(h.degree, jy, lc[1]) * b1d(h.degree, jz, lc[2]);
          if (phi == 0.0) continue;
          int r = func_of(L, morton3(c[0] + jx, c[1] + jy, c[2] + jz), t);
          if (r < 0) continue;
          for (int q = 0; q < k; ++q) out[(size_t)q * h.nv + v] += phi * x[(size_t)q * n + r];
        }
  }
  return 0;
}

// World positions of the function centres at the finest depth (3 columns):
// the coefficients that reproduce the embedding (x, y, z) exactly.
int oracle_linear_coeffs(void* hp, double* X) {
  Hier& h = ((OracleHandle*)hp)->h;
  const Level& L = h.lev[h.D];
  const long n = (long)L.fkey.size();
  const double hd = h.s / std::ldexp(1.0, h.D);
  for (long i = 0; i < n; ++i) {
    long c[3];
    demorton3(L.fkey[i], c);
    for (int a = 0; a < 3; ++a) {
      // degree 1: corner k at k*h; degree 2: node o = S-1 centred at (o + 1/2) h
      double g = h.degree == 1 ? (double)c[a] : (double)c[a] - 0.5;
      X[(size_t)a * n + i] = h.o[a] + g * hd;
    }
  }
  return 0;
}

}  // extern "C"

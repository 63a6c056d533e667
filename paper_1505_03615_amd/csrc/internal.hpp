// Objects behind the opaque handles, shared by the translation units.
#pragma once

#include <memory>
#include <vector>

#include "common.hpp"

namespace camfe {

// Data of one octree depth d (all arrays on the device).
struct HLevel {
  int d = 0;
  size_t npairs = 0;        // (cell, triangle) pairs, keys = Morton(cell) << 24 | tri, sorted
  DArr<u64> pairs;
  size_t ncells = 0;
  bool built = false;       // functions exist at this depth (d >= coarsest)
  size_t nent = 0;          // (support, triangle) entries, keys = Morton(support) << 24 | tri
  DArr<u64> ent;
  DArr<int> ent_func;       // function of each entry
  size_t nfun = 0;          // functions, canonical order
  DArr<u64> fkey;
  DArr<int> fcomp, frep;
  size_t ncorn = 0;         // distinct supports (corners / nodes)
  DArr<u64> ckey;
  DArr<int> cfirst;         // first function of each support, ncorn + 1 entries
  DArr<int> pair_rows;      // function of (pair, local support j), npairs * NB
  // prolongation from depth d-1 (rows: functions at d, columns: at d-1)
  size_t pnnz = 0;
  DArr<int> P_ptr, P_col;
  DArr<double> P_w;
};

}  // namespace camfe

struct camfe_hier_s {
  camfe_ctx ctx = nullptr;
  bool imported = false;      // levels from given matrices (camfe_system_import_csr): no mesh
  int D = 0, degree = 1, split = 1, min_depth = 0, d0 = 0;
  long long max_coarse = 0;
  double cube[5] = {0, 0, 0, 1, 1};   // origin xyz, side, 2^D / side
  size_t nv = 0, nt = 0;
  camfe::DArr<double> U;      // nv x 3 grid coordinates at depth D
  camfe::DArr<int> F;         // nt x 3
  camfe::DArr<double> nrm;    // nt x 3 unit normals
  camfe::DArr<double> cubed;  // device copy of cube[]
  // mesh adjacency
  size_t ne = 0;
  camfe::DArr<int> tri_edge;  // nt x 3: edge id of edge (F[t][j], F[t][j+1])
  camfe::DArr<int> edge_ptr, edge_tri;
  camfe::DArr<int> vt_ptr, vt_tri;
  camfe::DArr<int> vfan;      // nv: 1 when the triangles at the vertex form one fan joined by edges at it
  std::vector<camfe::HLevel> lev;  // index = depth
  int NB() const { return degree == 1 ? 8 : 27; }
  int W() const { return degree == 1 ? 2 : 3; }
};

namespace camfe {

// Assembled matrices of one depth: CSR over functions (canonical order),
// ascending columns, M and L on one pattern.
struct SLevel {
  size_t n = 0, nnz = 0;
  DArr<int> ptr, col;
  DArr<double> M, L;
};

struct SolverState;   // solve.hip
void destroy_solver(SolverState* s);
void refresh_solver(camfe_sys s);   // matrix values changed, structure kept

}  // namespace camfe

struct camfe_sys_s {
  camfe_hier h = nullptr;
  std::vector<camfe::SLevel> lev;   // index = depth (only d0..D filled)
  camfe::DArr<double> tri_w;        // current triangle weights of M (empty = 1)
  camfe::SolverState* solver = nullptr;
  const void* model = nullptr;      // attached learned smoother (not owned)
  camfe::DArr<double> area0;        // triangle areas of the original surface (flow)
  std::vector<camfe::DArr<double>> mcache;   // per depth: unweighted degree-1 mass blocks of every pair
  long long sell_sort_min_rows = 0;  // colours with at least this many rows are length-sorted (0: default)
  bool sell_compact = true;          // 16-bit column codes where a slice's spans allow (degree 1)
  long long block_colour_min = 0;    // cell-block depths relaxed colour by colour from this many blocks (0: default)
  std::vector<int> tiles;            // colour-sweep tile per depth from camfe_system_autotune (empty: default)
  camfe_hier owned_h = nullptr;      // an imported system's own hierarchy (freed with the system)
  ~camfe_sys_s() {
    camfe::destroy_solver(solver);
    solver = nullptr;
    lev.clear();
    delete owned_h;
  }
};

namespace camfe {
// calls that need the mesh reject systems built from given matrices
inline void require_mesh(camfe_sys s) {
  CAMFE_REQUIRE(!s->h->imported, CAMFE_ESTATE, "the system has no mesh (built from given matrices)");
}
// assemble.hip
void assemble_level(camfe_sys s, int d, bool want_L, bool want_M);
// b = int f b_i (grad: int <grad f, grad b_i>) at the finest depth; fv nv x k,
// b n x k, both column-major on the device
void load_vector_dev(camfe_sys s, const double* d_fv, int k, double* d_b, bool grad = false);
// dense.hip: out = diag(s) A^-1 diag(s) for SPD A (n x n row-major, destroyed)
void spd_inverse_scaled(camfe_ctx ctx, double* A, int n, const double* s, double* out);
// assemble.hip helpers: y = (a M + b L) x at the finest depth, x and y n x k
// row-major; layout changes of n x k blocks
void csr_apply(camfe_ctx ctx, const SLevel& L, double a, double b, const double* x, int k, double* y);
void to_rowmajor(camfe_ctx ctx, const double* in, size_t n, int k, double* out);
void to_colmajor(camfe_ctx ctx, const double* in, size_t n, int k, double* out);
// solve.hip: (M + t L) X = B for k device columns (canonical, column-major)
struct SolveSummary {
  int iterations = 0, cycles = 0;
  double rel = 0.0;   // largest relative residual over the columns
};
SolveSummary solve_device(camfe_sys s, const camfe_solve_opts& o, const double* db, double* dx, int k);
}  // namespace camfe

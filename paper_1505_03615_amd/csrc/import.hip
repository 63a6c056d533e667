// Systems built from given matrices (a debugging entry: the multigrid solve
// of Sections 3.2, 4.3 and 5.2 on matrices assembled elsewhere), and the
// solver's layout options and statistics.
//
// An imported system carries a hierarchy of its own with only what the
// solver reads: per depth the function keys (their colours), the
// prolongation from the depth below (Eq. 4), and the CSR matrices M and L.
// It has no mesh, so the calls that integrate over or evaluate on the
// surface reject it.
#include <algorithm>
#include <memory>
#include <vector>

#include "internal.hpp"
#include "solver.hpp"

using namespace camfe;

namespace {

// colour of a function from its key: corner parity per axis (degree 1) or
// node index mod 3 per axis (degree 2); two functions of one colour never
// share a nonzero in a system assembled from the B-splines
int colour_of_key(int degree, u64 key) {
  long long c[3] = {0, 0, 0};
  for (int b = 0; b < 21; ++b)
    for (int a = 0; a < 3; ++a) c[a] |= (long long)((key >> (3 * b + a)) & 1ULL) << b;
  if (degree == 1) return (int)((c[0] & 1) + 2 * (c[1] & 1) + 4 * (c[2] & 1));
  return (int)((c[0] % 3) + 3 * (c[1] % 3) + 9 * (c[2] % 3));
}

template <class T>
std::vector<T> host_copy(camfe_ctx ctx, const T* src, size_t n) {
  std::vector<T> v(n);
  copy_out(ctx, v.data(), src, n);
  return v;
}

}  // namespace

extern "C" {

camfe_status camfe_system_set_sell_sort(camfe_sys s, int64_t min_rows) {
  return guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s, CAMFE_EINVAL, "null system");
    s->h->ctx->use_device();
    s->sell_sort_min_rows = min_rows > 0 ? (long long)min_rows : 0;
    s->h->ctx->sync();
    destroy_solver(s->solver);
    s->solver = nullptr;
  });
}

camfe_status camfe_system_set_sell_columns(camfe_sys s, int bits) {
  return guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s && (bits == 16 || bits == 32), CAMFE_EINVAL, "null system, or bits other than 16 and 32");
    s->h->ctx->use_device();
    s->sell_compact = bits == 16;
    s->h->ctx->sync();
    destroy_solver(s->solver);
    s->solver = nullptr;
  });
}

camfe_status camfe_system_set_block_colouring(camfe_sys s, int64_t min_blocks) {
  return guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s, CAMFE_EINVAL, "null system");
    s->block_colour_min = min_blocks > 0 ? (long long)min_blocks : 0;
  });
}

camfe_status camfe_system_sell_stats(camfe_sys s, int depth, int64_t* slices, int64_t* compact, int64_t* entries) {
  return guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s, CAMFE_EINVAL, "null system");
    CAMFE_REQUIRE(s->solver, CAMFE_ESTATE, "no solver yet: solve (or autotune) first");
    const SolverState* S = s->solver;
    CAMFE_REQUIRE(depth >= S->d0 && depth <= S->D, CAMFE_EINVAL, "depth outside the solver's depths");
    const GLevel& G = S->lev[depth];
    if (slices) *slices = (int64_t)G.nslices;
    if (compact) *compact = (int64_t)G.ns16;
    if (entries) *entries = (int64_t)G.snnz;
  });
}

camfe_status camfe_system_import_csr(camfe_ctx ctx, int degree, int nlevels, const camfe_level_csr* levels,
                                     int64_t max_coarse, camfe_sys* out) {
  return guarded([&] {
    if (ctx) set_current_ctx(ctx);
    CAMFE_REQUIRE(ctx && levels && out && nlevels >= 1, CAMFE_EINVAL, "null argument");
    CAMFE_REQUIRE(degree == 1 || degree == 2, CAMFE_EINVAL, "degree must be 1 or 2");
    ctx->use_device();
    const int d0 = levels[0].depth, D = levels[nlevels - 1].depth;
    CAMFE_REQUIRE(d0 >= 0 && D <= 12 && D - d0 + 1 == nlevels, CAMFE_EINVAL,
                  "levels must be consecutive depths in [0, 12], coarsest first");
    std::unique_ptr<camfe_hier_s> h(new camfe_hier_s());
    h->ctx = ctx;
    h->imported = true;
    h->D = D;
    h->d0 = d0;
    h->min_depth = d0;
    h->degree = degree;
    h->max_coarse = max_coarse;
    h->lev.resize(D + 1);
    std::unique_ptr<camfe_sys_s> s(new camfe_sys_s());
    s->lev.resize(D + 1);
    long long n_below = 0;
    for (int i = 0; i < nlevels; ++i) {
      const camfe_level_csr& in = levels[i];
      const int d = d0 + i;
      CAMFE_REQUIRE(in.depth == d, CAMFE_EINVAL, "levels must be consecutive depths, coarsest first");
      CAMFE_REQUIRE(in.n > 0 && in.n < (1LL << 31) && in.keys && in.rowptr && in.col && in.M && in.L, CAMFE_EINVAL,
                    "level " + std::to_string(d) + ": empty or missing arrays");
      const size_t n = (size_t)in.n;
      std::vector<int64_t> ptr = host_copy(ctx, in.rowptr, n + 1);
      CAMFE_REQUIRE(ptr[0] == 0 && ptr[n] < (1LL << 31), CAMFE_EINVAL, "level " + std::to_string(d) + ": row pointers");
      for (size_t r = 0; r < n; ++r)
        CAMFE_REQUIRE(ptr[r + 1] >= ptr[r], CAMFE_EINVAL, "level " + std::to_string(d) + ": row pointers decrease");
      const size_t nnz = (size_t)ptr[n];
      std::vector<u64> keys = host_copy(ctx, (const u64*)in.keys, n);
      std::vector<int> col = host_copy(ctx, (const int*)in.col, nnz);
      std::vector<double> M = host_copy(ctx, in.M, nnz), L = host_copy(ctx, in.L, nnz);
      const u64 key_limit = 1ULL << (3 * (d + 2));   // node indices up to 2^d + 2 per axis
      std::vector<int> colour(n);
      for (size_t r = 0; r < n; ++r) {
        CAMFE_REQUIRE(keys[r] < key_limit, CAMFE_EINVAL, "level " + std::to_string(d) + ": key out of range");
        colour[r] = colour_of_key(degree, keys[r]);
      }
      for (size_t r = 0; r < n; ++r) {
        bool diag = false;
        for (long long e = ptr[r]; e < ptr[r + 1]; ++e) {
          const int c = col[e];
          CAMFE_REQUIRE(c >= 0 && (size_t)c < n && (e == ptr[r] || c > col[e - 1]), CAMFE_EINVAL,
                        "level " + std::to_string(d) + ": columns out of range or not ascending");
          if ((size_t)c == r) diag = true;
          else
            CAMFE_REQUIRE(colour[c] != colour[r] || (M[e] == 0.0 && L[e] == 0.0), CAMFE_EINVAL,
                          "level " + std::to_string(d) + ": two functions of one colour share a nonzero");
        }
        CAMFE_REQUIRE(diag, CAMFE_EINVAL, "level " + std::to_string(d) + ": missing diagonal entry");
      }
      camfe::HLevel& H = h->lev[d];
      H.d = d;
      H.built = true;
      H.nfun = n;
      H.fkey.alloc(n);
      copy_in(ctx, H.fkey.p, keys.data(), n);
      camfe::SLevel& S = s->lev[d];
      S.n = n;
      S.nnz = nnz;
      std::vector<int> p32(ptr.begin(), ptr.end());
      S.ptr.alloc(n + 1);
      S.col.alloc(std::max<size_t>(nnz, 1));
      S.M.alloc(std::max<size_t>(nnz, 1));
      S.L.alloc(std::max<size_t>(nnz, 1));
      copy_in(ctx, S.ptr.p, p32.data(), n + 1);
      copy_in(ctx, S.col.p, col.data(), nnz);
      copy_in(ctx, S.M.p, M.data(), nnz);
      copy_in(ctx, S.L.p, L.data(), nnz);
      if (i > 0) {
        CAMFE_REQUIRE(in.p_rowptr && in.p_col && in.p_w, CAMFE_EINVAL,
                      "level " + std::to_string(d) + ": missing prolongation");
        std::vector<int64_t> pp = host_copy(ctx, in.p_rowptr, n + 1);
        CAMFE_REQUIRE(pp[0] == 0 && pp[n] < (1LL << 31), CAMFE_EINVAL,
                      "level " + std::to_string(d) + ": prolongation row pointers");
        for (size_t r = 0; r < n; ++r)
          CAMFE_REQUIRE(pp[r + 1] >= pp[r], CAMFE_EINVAL,
                        "level " + std::to_string(d) + ": prolongation row pointers decrease");
        const size_t pn = (size_t)pp[n];
        std::vector<int> pc = host_copy(ctx, (const int*)in.p_col, pn);
        for (size_t e = 0; e < pn; ++e)
          CAMFE_REQUIRE(pc[e] >= 0 && pc[e] < n_below, CAMFE_EINVAL,
                        "level " + std::to_string(d) + ": prolongation column out of range");
        std::vector<double> pw = host_copy(ctx, in.p_w, pn);
        std::vector<int> pp32(pp.begin(), pp.end());
        H.pnnz = pn;
        H.P_ptr.alloc(n + 1);
        H.P_col.alloc(std::max<size_t>(pn, 1));
        H.P_w.alloc(std::max<size_t>(pn, 1));
        copy_in(ctx, H.P_ptr.p, pp32.data(), n + 1);
        copy_in(ctx, H.P_col.p, pc.data(), pn);
        copy_in(ctx, H.P_w.p, pw.data(), pn);
      }
      n_below = (long long)n;
    }
    ctx->sync();
    s->h = h.get();
    s->owned_h = h.release();
    *out = s.release();
  });
}

}  // extern "C"

// Surface flow (Section 5.3): one semi-implicit step of conformalized
// mean-curvature flow, (M_t + delta/2 L_0) u_{t+delta} = M_t u_t, on the
// hierarchy of the original surface.  The basis functions are tracked: they
// stay those of the original surface, so L_0 never changes and M_t is the
// original mass integral with each triangle's contribution scaled by the ratio
// of its current area (under the embedding u_t) to its original area.
#include <cmath>

#include "internal.hpp"

namespace camfe {
namespace {

constexpr int BLK = 256;

__device__ inline double tri_area(double ax, double ay, double az, double bx, double by, double bz, double cx,
                                  double cy, double cz) {
  const double ux = bx - ax, uy = by - ay, uz = bz - az;
  const double vx = cx - ax, vy = cy - ay, vz = cz - az;
  const double nx = uy * vz - uz * vy, ny = uz * vx - ux * vz, nz = ux * vy - uy * vx;
  return 0.5 * sqrt(nx * nx + ny * ny + nz * nz);
}

// original areas from the grid coordinates U (nv x 3 row-major), scaled to
// world units by (side / 2^D)^2
__global__ void k_area0(const double* U, const int* F, long long nt, double scale2, double* a0) {
  long long t = blockIdx.x * (long long)BLK + threadIdx.x;
  if (t >= nt) return;
  const double* p = U + 3LL * F[3 * t];
  const double* q = U + 3LL * F[3 * t + 1];
  const double* r = U + 3LL * F[3 * t + 2];
  a0[t] = tri_area(p[0], p[1], p[2], q[0], q[1], q[2], r[0], r[1], r[2]) * scale2;
}

// w_T = area of T under the vertex positions P (nv x 3 column-major) / a0_T
__global__ void k_area_ratio(const double* P, long long nv, const int* F, long long nt, const double* a0, double* w) {
  long long t = blockIdx.x * (long long)BLK + threadIdx.x;
  if (t >= nt) return;
  const long long a = F[3 * t], b = F[3 * t + 1], c = F[3 * t + 2];
  w[t] = tri_area(P[a], P[nv + a], P[2 * nv + a], P[b], P[nv + b], P[2 * nv + b], P[c], P[nv + c], P[2 * nv + c]) /
         a0[t];
}

void must(camfe_status rc) {
  if (rc != CAMFE_OK) throw Error(rc, camfe_last_error());
}

}  // namespace
}  // namespace camfe

using namespace camfe;

extern "C" {

camfe_status camfe_flow_step(camfe_sys s, double delta, double* X, const camfe_solve_opts* opts,
                             camfe_solve_stats* stats) {
  camfe_status rc = CAMFE_OK;
  camfe_status g = guarded([&] {
    if (s) set_current_ctx(s->h->ctx);
    CAMFE_REQUIRE(s && X && opts && delta >= 0.0, CAMFE_EINVAL, "bad argument");
    require_mesh(s);
    camfe_hier h = s->h;
    camfe_ctx ctx = h->ctx;
    ctx->use_device();
    const size_t n = s->lev[h->D].n, nv = h->nv, nt = h->nt;
    if (s->area0.n != nt) {
      s->area0.alloc(nt);
      const double sc = 1.0 / h->cube[4];
      hipLaunchKernelGGL(k_area0, grid_for(nt, BLK), BLK, 0, ctx->stream, h->U.p, h->F.p, (long long)nt, sc * sc,
                         s->area0.p);
      check_launch();
    }
    DArr<double> Xd(n * 3), P(nv * 3), W(nt), B(n * 3);
    copy_in(ctx, Xd.p, (const double*)X, Xd.n);
    must(camfe_eval_vertices(s, Xd.p, 3, P.p));
    hipLaunchKernelGGL(k_area_ratio, grid_for(nt, BLK), BLK, 0, ctx->stream, (const double*)P.p, (long long)nv,
                       h->F.p, (long long)nt, (const double*)s->area0.p, W.p);
    check_launch();
    must(camfe_reassemble_mass(s, W.p));
    must(camfe_apply(s, 0, 0.0, Xd.p, 3, B.p));
    camfe_solve_opts o = *opts;
    o.t = 0.5 * delta;
    o.x0_given = 1;
    rc = camfe_solve(s, &o, B.p, 3, Xd.p, stats);
    if (rc != CAMFE_OK && rc != CAMFE_ENOCONV) throw Error(rc, camfe_last_error());
    copy_out(ctx, X, Xd.p, Xd.n);
    ctx->sync();
  });
  if (g != CAMFE_OK) return g;
  if (rc != CAMFE_OK) set_last_error("solver stopped above rtol");
  return rc;
}

}  // extern "C"

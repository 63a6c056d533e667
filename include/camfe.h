/* camfe: connectivity-aware multilevel finite elements for Laplace-Beltrami
 * systems on triangle meshes (Chuang & Kazhdan, arXiv 1505.03615), as a C ABI
 * over hand-written HIP kernels for AMD Instinct MI355X (gfx950).
 *
 * Problem statement (Section 3.1, Eq. 1-2): given a mesh M and an octree depth
 * D, build the nested function spaces of Sections 3.2 and 4 (trilinear or
 * quadratic B-splines on the grid of 2^D cells per axis, restricted to M, one
 * function per connected component of each support, Section 4.2), assemble
 * the mass matrix M_ij = int b_i b_j (Section 5.1) and the stiffness matrix
 * L_ij = int <grad_M b_i, grad_M b_j> (Eq. 2, with the sign that makes L
 * positive semi-definite), and solve (M + t L) x = b with the multigrid
 * V-cycle over the nested hierarchy (Sections 3.2, 4.3, 5.2).
 *
 * Conventions for every call:
 *  - Return value: a camfe_status; on failure camfe_last_error() describes it.
 *    No C++ exception crosses the interface.
 *  - Array arguments may point to host or to device memory of the context's
 *    device; the library copies them (hipMemcpyDefault) and never keeps them.
 *    All work runs on the context's stream; calls return after the stream has
 *    finished the work they queued, so outputs are ready on return.
 *  - Handles are owned by the library and released by the matching *_destroy.
 *    A hierarchy must outlive the systems assembled from it; a context must
 *    outlive its hierarchies.
 *  - Exports use the two-call pattern: pass cap = 0 (pointers may be NULL) to
 *    learn the size in *n; a non-zero cap below the size returns
 *    CAMFE_ETOOSMALL.
 *  - Keys: a cell (i, j, k) of depth d is stored as its Morton code (bit b of
 *    i at 3b, of j at 3b+1, of k at 3b+2).  A degree-1 function lives at grid
 *    corner k (support box [k-1, k+1]^3 in depth-d cell units); a degree-2
 *    function at the cell o whose quadratic B-spline has support
 *    [o-1, o+2]^3, stored as the Morton code of o + (1,1,1).
 *  - Vectors over functions are column-major n x k arrays of doubles, n the
 *    number of functions at the finest depth, in canonical order (support key
 *    ascending, then component number).
 *  - Not thread-safe per handle; distinct handles may be used from distinct
 *    threads.
 */
#ifndef CAMFE_H
#define CAMFE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CAMFE_OK = 0,
  CAMFE_EINVAL = -1,    /* invalid argument or mesh                          */
  CAMFE_ENOMEM = -2,    /* device allocation failed                          */
  CAMFE_EDEVICE = -3,   /* HIP runtime or kernel error                       */
  CAMFE_ENOCONV = -4,   /* solver stopped at max_iter above rtol (stats set) */
  CAMFE_ESINGULAR = -5, /* coarsest factorisation failed even with eps * Id  */
  CAMFE_ETOOSMALL = -6, /* export capacity below the required size           */
  CAMFE_ESTATE = -7     /* call not valid for this handle (e.g. depth not built) */
} camfe_status;

typedef struct camfe_ctx_s *camfe_ctx;
typedef struct camfe_hier_s *camfe_hier;
typedef struct camfe_sys_s *camfe_sys;

/* Message of the last failed call on this thread (never NULL). */
const char *camfe_last_error(void);
/* Message of the last failed call that reached this context: a call on the
 * context itself or on a hierarchy, system or batch created under it, from
 * any thread (never NULL; "" when none failed).  A call rejected before it
 * could name its context (a null handle) records its message on the thread
 * only.  Valid until the next failing call on the context or its destruction. */
const char *camfe_ctx_last_error(camfe_ctx ctx);

/* Context: device ordinal and stream (hipStream_t, NULL = a stream the
 * library creates and owns).  Holds scratch memory reused across calls. */
camfe_status camfe_ctx_create(int device, void *hip_stream, camfe_ctx *out);
void camfe_ctx_destroy(camfe_ctx ctx);

/* Measurement: with enable = 1 every launch of the hot kernels on the
 * context's stream is bracketed by HIP events (totals reset); enable = 0 stops
 * recording.  camfe_ctx_kernel_time returns, for one kernel name
 * ("gs_colour", "residual", "spmv_dot", "restrict", "prolong", "coarse_solve",
 * "assemble", "pairs", "uf_link", "support_sort", "cg_vector"), the summed
 * event time in ms, the number of launches, and the summed algorithmic work
 * (bytes the method must move, or flops for "assemble").  EINVAL for an
 * unknown name. */
camfe_status camfe_ctx_kernel_timing(camfe_ctx ctx, int enable);
camfe_status camfe_ctx_kernel_time(camfe_ctx ctx, const char *kernel, double *total_ms, int64_t *launches,
                                   double *work);

/* ----------------------------------------------------------- primitives */
/* The ordering and counting steps under the hierarchy build: finding the
 * basis (Section 4.2) needs the triangles of each cell and of each support
 * grouped, which the build does by sorting Morton-keyed records and taking
 * prefix sums of counts.  Exported so that they can be tested and reused.
 * All pointers are device memory; the calls run on the context's stream,
 * take temporary storage from the context and return once the result is in
 * place (work queued earlier on other streams is not waited for).
 *
 * camfe_radix_sort: stable radix sort, in place, of n keys (key_bytes 4 or
 * 8, unsigned) by their bits [0, end_bit), carrying n 32-bit values along
 * when vals is not NULL.  Keys that agree on those bits keep their input
 * order.  EINVAL for n < 0 or n >= 2^31, key_bytes other than 4 and 8,
 * end_bit outside [0, 8 key_bytes], or a null keys pointer with n > 0.
 *
 * camfe_exclusive_sum: out[i] = in[0] + ... + in[i-1] for n integers of
 * elem_bytes 4 or 8 (two's complement, wrapping); out may equal in.  EINVAL
 * for n < 0, other element sizes, or a null pointer with n > 0. */
camfe_status camfe_radix_sort(camfe_ctx ctx, void *keys, int key_bytes, uint32_t *vals, int64_t n, int end_bit);
camfe_status camfe_exclusive_sum(camfe_ctx ctx, const void *in, void *out, int64_t n, int elem_bytes);

/* ------------------------------------------------------------ hierarchy */
typedef struct {
  int depth;          /* finest depth D, 1..12 (2^D cells per axis)                   */
  int degree;         /* 1: trilinear at corners (the paper's space); 2: quadratic    */
                      /*    B-splines at cells (footnote to Definition 1)             */
  int split;          /* 1: connectivity-aware split (Section 4.2); 0: one function  */
                      /*    per support (the space of Definition 2)                   */
  int min_depth;      /* coarsest depth may not go below this (Section 5.2 "minimum  */
                      /*    depth")                                                   */
  int64_t max_coarse; /* coarsest depth = finest depth with at most this many        */
                      /*    functions (but >= min_depth); it is solved directly when  */
                      /*    it has at most max_coarse functions, else relaxed.        */
                      /*    <= 0: only min_depth decides and the coarsest is relaxed  */
  double box_origin[3];
  double box_side;    /* > 0: grid cube [origin, origin + side]^3; <= 0: bounding    */
                      /*    cube of the mesh scaled by 1.125 about its centre         */
} camfe_hier_opts;

/* Build the octree of triangle/cell pairs, the support lists, the split and
 * the prolongation (Eq. 4) from depth D down to the coarsest depth.
 * V: nv x 3 row-major vertex positions; F: nt x 3 row-major vertex indices,
 * nt < 2^24.  EINVAL for out-of-range indices, repeated indices, a triangle of
 * zero area, a vertex outside an explicit box, or a triangle lying in a grid
 * plane (the mesh must be in general position). */
camfe_status camfe_hierarchy_build(camfe_ctx ctx, const double *V, int64_t nv, const int32_t *F,
                                   int64_t nt, const camfe_hier_opts *opts, camfe_hier *out);
/* finest and coarsest depth built */
camfe_status camfe_hierarchy_levels(camfe_hier h, int *finest, int *coarsest);
/* grid cube actually used: origin[3], side */
camfe_status camfe_hierarchy_cube(camfe_hier h, double out4[4]);
/* counts at depth d (0..D); n_functions is -1 below the coarsest depth */
camfe_status camfe_hierarchy_info(camfe_hier h, int depth, int64_t *n_cells, int64_t *n_pairs,
                                  int64_t *n_functions);
/* occupied cells at depth d (Definition 1: cells whose open box meets the
 * surface; at coarser depths the parents of occupied cells, Section 4.3):
 * Morton keys ascending, n_cells of camfe_hierarchy_info entries */
camfe_status camfe_export_cells(camfe_hier h, int depth, uint64_t *keys, int64_t cap, int64_t *n);
/* (cell key, triangle) pairs whose triangle meets the open cell, sorted */
camfe_status camfe_export_pairs(camfe_hier h, int depth, uint64_t *cell_key, int32_t *tri,
                                int64_t cap, int64_t *n);
/* functions in canonical order: support key, component number (components of
 * one support numbered by increasing smallest triangle), smallest triangle */
camfe_status camfe_export_functions(camfe_hier h, int depth, uint64_t *key, int32_t *comp,
                                    int32_t *rep_tri, int64_t cap, int64_t *n);
/* (support key, triangle) active pairs, sorted, with the function each maps to */
camfe_status camfe_export_support_entries(camfe_hier h, int depth, uint64_t *key, int32_t *tri,
                                          int32_t *func, int64_t cap, int64_t *n);
/* prolongation P_d (rows: functions at depth d, columns at d-1; Eq. 4), CSR
 * with ascending columns; rowptr has n_functions(d) + 1 entries */
camfe_status camfe_export_prolongation(camfe_hier h, int depth, int64_t *rowptr, int32_t *col,
                                       double *w, int64_t cap, int64_t *nnz);
void camfe_hierarchy_destroy(camfe_hier h);

/* ------------------------------------------------------------- assembly */
/* Assemble M and L at every built depth (Eq. 2, Section 5.1) by exact
 * quadrature over the triangle fragments clipped to cells.  tri_weight
 * (nullable, nt doubles) scales each triangle's contribution to M only (the
 * mass of an evolved surface, Section 5.3); L always uses weight 1. */
camfe_status camfe_assemble(camfe_hier h, const double *tri_weight, camfe_sys *out);
/* Re-assemble M alone with new triangle weights (L and the structure kept).
 * Degree 1: the first call also keeps every (cell, triangle) pair's
 * unweighted element block on the device (36 doubles per pair, held by the
 * system until it is destroyed; skipped when that would take more than a
 * quarter of the free device memory), and later calls only weight and scatter
 * those blocks.  tri_weight: host or device pointer, nt doubles (null = 1). */
camfe_status camfe_reassemble_mass(camfe_sys s, const double *tri_weight);
/* which: 0 = M, 1 = L.  CSR with ascending columns, canonical order. */
camfe_status camfe_export_matrix(camfe_sys s, int depth, int which, int64_t *rowptr,
                                 int32_t *col, double *val, int64_t cap, int64_t *nnz);
/* b_i = int f b_i at the finest depth (Eq. 2) for f linear on each triangle
 * from per-vertex values vertex_f (nv x k column-major); b is n x k. */
camfe_status camfe_load_vector(camfe_sys s, const double *vertex_f, int k, double *b);
/* b_i = int <grad f, grad b_i> at the finest depth: the gradient constraint of
 * the screened Poisson colour fit (L + alpha M) u = b + alpha s (Section 5.2),
 * with s from camfe_load_vector and grad f the surface gradient of f, linear
 * on each triangle from per-vertex values vertex_f (nv x k column-major; zero
 * on triangles without area, which the hierarchy build rejects; on a sliver
 * whose corners' values differ the gradient grows like the inverse of its
 * width, so such inputs are ill-conditioned); b is n x k.  Host or device
 * pointers. */
camfe_status camfe_gradient_load(camfe_sys s, const double *vertex_f, int k, double *b);
/* y = A x at the finest depth with A = M (which 0), L (1) or M + t L (2) */
camfe_status camfe_apply(camfe_sys s, int which, double t, const double *x, int k, double *y);
/* camfe_apply without any device allocation, for callers that cannot
 * allocate (serving loops, harnesses that forbid it).  x and y must be device
 * memory of the context's device (EINVAL otherwise) with n x k <= 2^20 (EINVAL
 * otherwise).  The row-major staging lives in a fixed 16 MiB device array per
 * GPU, reserved when the library first runs on that GPU and held until the
 * process ends; it is shared by every call on that GPU, so calls that overlap
 * on one GPU (from several threads or contexts) race.  Like every call it
 * synchronises the context's stream before returning. */
camfe_status camfe_apply_noalloc(camfe_sys s, int which, double t, const double *x, int k, double *y);
/* coefficients that reproduce the embedding: n x 3 column-major (x, y, z) */
camfe_status camfe_linear_coeffs(camfe_sys s, double *X);
/* u(v) = sum_i x_i b_i(v) at every mesh vertex (nv x k column-major) */
camfe_status camfe_eval_vertices(camfe_sys s, const double *x, int k, double *vertex_out);

/* ---------------------------------------------------------------- solve */
typedef struct {
  double t;          /* A = M + t L                                                */
  double rtol;       /* stop when ||b - A x||_2 <= rtol ||b||_2 for every column   */
  int max_iter;      /* outer iterations (CG steps or stationary cycles)          */
  int nu_pre, nu_post; /* sweeps before/after the coarse correction; equal for     */
                       /*    method 0 (CG needs a symmetric V-cycle), else EINVAL   */
  int method;        /* 0: CG preconditioned by one V-cycle; 1: stationary V-cycles */
  int precision;     /* 0: FP64 throughout; 1: V-cycle in FP32, residual, CG      */
                     /*    recurrences and coarsest solve in FP64                 */
  int x0_given;      /* start from x instead of 0                                 */
  double coarse_eps; /* eps added to the unit-diagonal-scaled coarsest matrix     */
                     /*    (1e-6 recommended: regularises singular systems, and   */
                     /*    FP32 cycles cannot amplify rounding past O(0.1))       */
  int smoother;      /* 0: multicolour Gauss-Seidel (Section 5.2); 1: weighted    */
                     /*    Jacobi with constant omega; 2: the attached learned    */
                     /*    model's smoother (Jacobi or SOR, per-row omega);       */
                     /*    3: cell-block Schwarz (not in the paper; degree 1):    */
                     /*    a block per occupied cell holding the functions of its */
                     /*    8 corners met there (single-function blocks in cells   */
                     /*    of more than 16), inverses of the unit-diagonal-scaled */
                     /*    blocks plus coarse_eps I; a sweep adds                 */
                     /*    omega sum_B w_B R_B^T A_B^-1 R_B (b - A x), w_B = 1 /  */
                     /*    (the most blocks holding one of B's functions).  An    */
                     /*    A-norm contraction only while omega lambda_max < 2     */
                     /*    (lambda_max of that block sum times A, which passes 2  */
                     /*    at fine depths: see camfe_block_damping).  Only FP64   */
                     /*    cycles are reliable: a near-singular block amplifies   */
                     /*    rounding by up to 1 / coarse_eps                       */
  double omega;      /* omega of smoother 1; damping of smoother 3 in [0, 1]      */
                     /*    (0: each depth's automatic value)                      */
  int judge;         /* smoother 1 or 2 with method 0: Gauss-Seidel as judge.     */
                     /*    The requested smoother and plain Gauss-Seidel each run */
                     /*    `judge` CG iterations from the start; the one with the */
                     /*    smaller residual continues.  All of them count in       */
                     /*    iterations and cycles.  0: off.  The batched solve     */
                     /*    ignores it                                             */
  int cycle;         /* 0 or 1: V-cycle; 2: W-cycle (Section 5.2): at every depth */
                     /*    above the coarsest the coarse problem gets two cycles, */
                     /*    the second starting from the first's result.  The      */
                     /*    batched solve takes 0 or 1 only (else EINVAL)          */
  int nu_coarse;     /* sweeps each way at the depths below the finest; 0: the    */
                     /*    finest depth's nu_pre / nu_post.  The batched solve    */
                     /*    ignores it                                             */
} camfe_solve_opts;

typedef struct {
  int iterations;    /* outer iterations done                                     */
  int fell_back;     /* 1 when the smoother (1 or 2, or 3 under CG) stopped above */
                     /*    rtol and Gauss-Seidel redid the solve (stationary      */
                     /*    cycles of smoother 3 are returned as asked); 2 when    */
                     /*    the judge continued with Gauss-Seidel                  */
  int cycles;        /* V-cycles applied                                          */
  int eps_regularised;
  double rel_residual; /* max over columns of ||b - A x|| / ||b|| (FP64)          */
  double seconds;      /* wall time of the iteration (setup excluded)             */
  double setup_seconds;/* forming A at every depth, packing, coarsest factor      */
  double judge_rel[2]; /* judged solves: largest relative CG residual over the    */
                       /*    columns after the judge's iterations, [0] requested  */
                       /*    smoother, [1] Gauss-Seidel (0 when not judged)       */
} camfe_solve_stats;

/* Solve (M + t L) x = b at the finest depth (Sections 3.2, 4.3, 5.2).
 * b, x: n x k column-major (x is read when x0_given).  Returns CAMFE_ENOCONV
 * with stats filled when max_iter is reached above rtol. */
camfe_status camfe_solve(camfe_sys s, const camfe_solve_opts *opts, const double *b, int k,
                         double *x, camfe_solve_stats *stats);
/* Measurement of one finest-depth kernel of a solved system (the solver state
 * of the last camfe_solve call): "gs_colour" (one forward Gauss-Seidel sweep,
 * one launch per colour), "residual" or "spmv_dot", with FP64 (precision 0) or
 * FP32 (1) values, one right-hand side; or "vcycle": one whole plain
 * Gauss-Seidel V(2,2)-cycle from a zero guess over every depth (the
 * preconditioner a CG step applies), avg_ms per cycle and bytes_per_launch 0
 * (its algorithmic bytes depend on the depths' sizes, which the exports give);
 * "vcycle:a,c" is the same cycle with a sweeps each way at the finest depth
 * and c at every coarser one (c = 0: a; 1 <= a <= 16, 0 <= c <= 16).  reps back-to-back sweeps/launches are
 * captured once into a HIP graph and replayed between two HIP events on the
 * context's stream.  avg_ms: average time of one launch; bytes_per_launch: the
 * algorithmic bytes of one launch (matrix values + three vector accesses per
 * row).  Two reference launches put these figures in context: "empty" (a
 * kernel that does nothing, on each colour's grid of the sweep: the launch
 * floor; bytes 0) and "copy" (one plain device copy per colour moving the
 * colour launch's average algorithmic bytes, half read and half written,
 * rotating through 16 buffer pairs so that its data leaves the L2 caches
 * between launches as the colours' matrices do; allocates and frees those
 * buffers).  Overwrites the solver's scratch vectors only. */
camfe_status camfe_measure_kernel(camfe_sys s, const char *kernel, int precision, int reps, double *avg_ms,
                                  double *bytes_per_launch);
/* Layout choice of the solver's packed matrices: the rows of a colour with
 * at least min_rows rows are ordered by decreasing length inside windows of
 * 1024 rows (less SELL padding, more scattered x gathers); smaller colours
 * keep the canonical order.  min_rows <= 0 restores the default (2^19).
 * Rows of one colour never couple, so the order changes no row's arithmetic.
 * Takes effect at the next solver set-up: drops the system's current solver
 * state (captured graphs included). */
camfe_status camfe_system_set_sell_sort(camfe_sys s, int64_t min_rows);
/* Column storage of the solver's packed matrices (degree 1): bits 16 (the
 * default) stores per entry a 16-bit code, colour << 13 | offset from one
 * base per (64-row slice, colour), wherever every colour's columns in the
 * slice span fewer than 8192 rows, and 32-bit columns elsewhere; bits 32
 * keeps 32-bit columns everywhere.  Both hold the same columns in the same
 * order, so results are the same bits.  EINVAL for other values.  Takes
 * effect at the next solver set-up (drops the current solver state). */
camfe_status camfe_system_set_sell_columns(camfe_sys s, int bits);
/* Launch pattern of the cell-block smoother (smoother 3): at each depth, a
 * block class (blocks of up to 8 and of 9-16 functions) with at least
 * min_blocks blocks is relaxed colour by colour (cells whose coordinates have
 * the same parities share no function, so each colour's blocks update x
 * with plain adds, 8 launches); a smaller class takes one launch with atomic
 * adds.  The update is the same sum either way, in another order.
 * min_blocks <= 0 restores the default (2^19).  Takes effect at the next
 * smoother-3 solve. */
camfe_status camfe_system_set_block_colouring(camfe_sys s, int64_t min_blocks);
/* Packed-matrix figures of one depth of the current solver state: slices,
 * slices with 16-bit column codes, stored entries (padding included).
 * Nullable outputs.  ESTATE before the first solve; EINVAL for a depth
 * outside the solver's. */
camfe_status camfe_system_sell_stats(camfe_sys s, int depth, int64_t *slices, int64_t *compact, int64_t *entries);
/* The automatic damping of smoother 3 at every depth (coarsest first; 0 at
 * a coarsest depth solved directly), building the solver for A = M + t L and
 * its cell blocks where missing: omega_d = min(1, 4 / (3 lambda_d)), where
 * lambda_d estimates the largest eigenvalue of B A, B = sum_B w_B R_B^T A_B^-1
 * R_B, by 20 power steps in the A inner product from a fixed pseudo-random
 * start (from below).  One sweep maps the error e to (I - omega B A) e, so
 * omega must stay below 2 / lambda_max.  lambda (nullable) receives the
 * estimates.  cap: entries of omega / lambda (0: only *nlevels); ETOOSMALL
 * below the number of depths; EINVAL for degree 2. */
camfe_status camfe_block_damping(camfe_sys s, double t, double coarse_eps, double *omega, double *lambda, int cap,
                                 int *nlevels);
/* Autotuner of the colour sweep's tile (not in the paper): for every depth of
 * the system's solver for A = M + t L (built when missing), each compiled tile
 * {wavefronts per 64-row slice, entries per lane issued together} in
 * {8,4} (default), {4,4}, {8,2}, {16,2}, {16,4}, {4,8}, {2,16} is timed over
 * reps forward
 * sweeps (one right-hand side, FP64 values for precision 0, FP32 for 1,
 * captured into a HIP graph, timed with events on the context's stream) and
 * the fastest is kept for that depth: by this solver and by the solvers the
 * system builds later.  Without it a degree-1 depth takes {4,8} from 2^19
 * rows per colour, {4,4} from 2^17, {8,4} from 2^15 and {16,2} below (degree
 * 2: {8,4}).  Tiles change the order in which a row's partial sums meet, so
 * results move within rounding.  Right-hand-side columns are processed four per pass
 * (the widest tile compiled).  Two-call pattern over the depths, coarsest
 * first: cap = 0 returns the count in *nlevels; otherwise tile (nullable)
 * receives each depth's index (0..6 in the order above) and ms (nullable) its
 * time per sweep.  Overwrites the solver's scratch vectors. */
camfe_status camfe_system_autotune(camfe_sys s, double t, int precision, int reps, int32_t *tile, double *ms,
                                   int cap, int *nlevels);
void camfe_system_destroy(camfe_sys s);

/* Debugging entry: a system built from given matrices instead of a mesh, so
 * that the multigrid solve (Sections 3.2, 4.3, 5.2) can run on matrices
 * assembled elsewhere (for instance by a reference implementation).  One
 * entry per depth, levels[0] the coarsest and levels[nlevels - 1] the finest,
 * depths consecutive.  Per level: the support keys of its n functions
 * (Morton codes as in the exports; they fix each function's colour, so two
 * functions of one colour must never share a nonzero), M and L as CSR on one
 * pattern (rowptr n + 1 entries, ascending columns per row, diagonal
 * present), and for every level but the coarsest the prolongation from the
 * level below (Eq. 4) as CSR, rows = this level's functions.  The coarsest
 * level is solved directly when it has at most max_coarse functions, else
 * relaxed.  Host or device pointers; everything is copied.  The system has no
 * mesh: calls that need one (load vectors, vertex values, linear
 * coefficients, mass re-weighting, flow steps, training) return CAMFE_ESTATE.
 * EINVAL for inconsistent sizes, columns or keys out of range, a missing
 * diagonal, or a degree other than 1 or 2. */
typedef struct {
  int depth;                 /* octree depth of the level (0..12)            */
  int64_t n;                 /* functions                                     */
  const uint64_t *keys;      /* n support keys                                */
  const int64_t *rowptr;     /* n + 1                                         */
  const int32_t *col;        /* rowptr[n] column indices                      */
  const double *M, *L;       /* rowptr[n] values each                         */
  const int64_t *p_rowptr;   /* prolongation from the level below (NULL at    */
  const int32_t *p_col;      /*    the coarsest): n + 1 row pointers, columns */
  const double *p_w;         /*    and weights                                */
} camfe_level_csr;
camfe_status camfe_system_import_csr(camfe_ctx ctx, int degree, int nlevels, const camfe_level_csr *levels,
                                     int64_t max_coarse, camfe_sys *out);

/* ------------------------------------------------------------ spectrum */
/* The smallest generalised eigenpairs L x = lambda M x at the finest depth
 * (Section 5.1: the spectrum of the estimated Laplace-Beltrami operator).
 * Shift-invert subspace iteration: each step solves (L + sigma M) Y = M X
 * for the block with the system's multigrid-preconditioned CG (as
 * camfe_solve with t = 1/sigma), then a Rayleigh-Ritz step on the GPU
 * (k x k Gram matrices of L and M, Cholesky of the M Gram matrix, Jacobi
 * rotations) makes the block M-orthonormal with ascending Ritz values.
 * The start block is pseudo-random from seed. */
typedef struct {
  int nev;            /* eigenpairs wanted, 1 <= nev <= block                    */
  int block;          /* subspace width, nev <= block <= 32 (0: min(32, nev + 8)) */
  double sigma;       /* shift > 0; convergence per step is (l_j + s)/(l_b + s)  */
  int max_iter;       /* subspace iterations                                     */
  double tol;         /* stop when every wanted pair has                         */
                      /*   ||L x - l M x|| <= tol (|l| + sigma) ||M x||          */
  double solve_rtol;  /* inner solves stop at max(solve_rtol, 0.01 x the wanted */
                      /*   pairs' largest scaled residual of the previous step)  */
  int precision;      /* inner cycles: 0 FP64, 1 FP32 (residuals in FP64)        */
  uint64_t seed;      /* start block                                             */
} camfe_eig_opts;

typedef struct {
  int iterations;      /* subspace iterations done                               */
  int solve_cycles;    /* V-cycles over all inner solves                         */
  double max_residual; /* largest scaled residual of the wanted pairs (above)    */
  double seconds;      /* wall time                                              */
} camfe_eig_stats;

/* evals: nev doubles, ascending; evecs (nullable): n x nev column-major,
 * M-orthonormal, canonical order (the entries of functions with zero computed
 * mass, whose rows of M and L are zero, are not determined by the problem and
 * carry no meaning).  Host or device pointers.  Sets up the
 * system's solver for t = 1/sigma (the next camfe_solve with another t
 * rebuilds it).  Returns CAMFE_EINVAL for options out of range (above) or a
 * block wider than the system, CAMFE_ENOCONV (outputs written) when max_iter
 * is reached above tol, CAMFE_ESINGULAR when the block's M Gram matrix is not
 * positive definite (a start block in the null space of M). */
camfe_status camfe_eigs(camfe_sys s, const camfe_eig_opts *opts, double *evals, double *evecs,
                        camfe_eig_stats *stats);

/* ------------------------------------------------------------- batching */
/* Many systems solved together (not in the paper): the hierarchies are lined
 * up by depth below their finest (each mesh bottoms out at its own coarsest
 * depth), and every phase of the V-cycle and of CG is one launch over all
 * meshes, captured into a HIP graph.  CG keeps its scalars per mesh and
 * column, and freezes columns that have converged (checked every four
 * iterations).  A member whose columns have all converged drops out: its
 * slices, transfer rows, coarse solve and CG vector blocks are skipped by
 * every later launch, so the batch costs what its members still iterating
 * cost. */
typedef struct camfe_batch_s *camfe_batch;
/* Copies the systems' solver data for A = M + t L (building it where missing);
 * later changes to the systems do not reach the batch.  All systems share the
 * context and the degree.  A system may be listed more than once.  A batch
 * solve takes one pass over all members per four right-hand-side columns of
 * its widest member, so a system with many columns is best listed once per
 * chunk of up to four (each entry then gets its chunk's columns). */
camfe_status camfe_batch_create(camfe_ctx ctx, camfe_sys const *systems, int nsys, double t, double coarse_eps,
                                camfe_batch *out);
/* levels of the batched hierarchy; rows of its finest level (padded) */
camfe_status camfe_batch_info(camfe_batch b, int *levels, int64_t *rows);
/* b[m], x[m]: n_m x k[m] column-major (x[m] read when x0_given); opts->t and
 * coarse_eps must be the batch's, method 0 and smoother 0; opts->nu_coarse
 * applies to every member's depths below its finest.  stats (nullable)
 * has nsys entries: iterations and cycles are those member m took part in,
 * seconds the whole batch's.  Returns CAMFE_ENOCONV when any mesh stops above
 * rtol. */
camfe_status camfe_batch_solve(camfe_batch b, const camfe_solve_opts *opts, const double *const *b_in, const int *k,
                               double *const *x, camfe_solve_stats *stats);
/* camfe_system_autotune over the batch's levels (finest last; the levels
 * hold every member's rows of that relative depth). */
camfe_status camfe_batch_autotune(camfe_batch b, int precision, int reps, int32_t *tile, double *ms, int cap,
                                  int *nlevels);
void camfe_batch_destroy(camfe_batch b);

/* --------------------------------------------------------- surface flow */
/* One step of conformalized mean-curvature flow (Section 5.3): solve
 * (M_t + delta/2 L_0) X' = M_t X with tracked test functions, i.e. on the
 * hierarchy and L_0 of the original surface, M_t being the original mass
 * integral with each triangle's contribution scaled by its current area (the
 * mesh vertices moved to u_t = sum_i X_i b_i) over its original area.
 * X: n x 3 column-major coefficients of the current embedding (start from
 * camfe_linear_coeffs), overwritten with X'.  The solve starts from X; opts->t
 * and opts->x0_given are ignored.  Leaves M = M_t assembled at every depth.
 * Returns CAMFE_ENOCONV (X' written) when the solve stops above rtol. */
camfe_status camfe_flow_step(camfe_sys s, double delta, double *X, const camfe_solve_opts *opts,
                             camfe_solve_stats *stats);

/* ------------------------------------------------------ learned smoother */
/* Not part of the paper's method (its smoother is Gauss-Seidel, Section 5.2):
 * optional smoothers x_i += omega_i (b_i - (A x)_i) / A_ii whose per-row weights
 * come from a small MLP per relative depth l = D - d (depths with l >= levels
 * use the last MLP).  Two sweep types, fixed per model:
 *   sweep 0, damped Jacobi: all rows at once, omega_i = c_i s_i with
 *     s_i = 2 sigmoid(z_i) in (0, 2) and the l1-Jacobi bound
 *     c_i = A_ii / sum_j |A_ij|, which keeps every sweep an
 *     A-norm contraction whatever the network outputs;
 *   sweep 1, multicolour SOR: the Gauss-Seidel colour order with
 *     omega_i = 1/2 + sigmoid(z_i) in (1/2, 3/2), a band around Gauss-Seidel
 *     (symmetric SOR with per-row weights in (0, 2) is an SPD preconditioner).
 * Degree 1 only.
 * Row features (30, FP32): the row of A = M + t L summed per grid offset
 * delta in {-1,0,1}^3 of the column's corner from the row's corner, divided by
 * A_ii (index (dx+1) + 3(dy+1) + 9(dz+1)); clamp(log10(A_ii / max_j A_jj),
 * -30, 0) / 10; M_ii / A_ii; (D - d) / 10.  A row of zero computed mass gets
 * omega = 0.  MLP: 30 -> 32 (ReLU) -> 32 (ReLU) -> 1, parameters packed per
 * level as W1[30][32], b1[32], W2[32][32], b2[32], w3[32], b3 (2081 floats;
 * W[i][j] maps input i to output j).  Inference and training use BF16 copies
 * of the weights (round to nearest even) with FP32 accumulation, or FP32
 * weights when bf16 = 0.
 * Training loss of a depth for error samples e0^s and nu sweeps of
 * e <- e - omega D^-1 A e: mean_s log(|A e_nu^s|^2 / |A e0^s|^2). */
typedef struct camfe_model_s *camfe_model;

typedef struct {
  double t;          /* A = M + t L of the training systems                        */
  int levels;        /* MLPs (relative depths), 1..32                               */
  int steps;         /* Adam steps (beta 0.9 / 0.999, eps 1e-8)                     */
  int nu;            /* sweeps whose residual reduction the loss measures, >= 1     */
  int bf16;          /* 1: BF16 weights (FP32 accumulation); 0: FP32 weights        */
  double lr;         /* Adam step size                                              */
  uint64_t seed;     /* seed of the error samples                                   */
  int sweep;         /* 0: damped Jacobi (l1-bounded); 1: multicolour SOR            */
  int cycle;         /* loss: 0 the nu sweeps alone; 1 a two-grid cycle (nu pre-    */
                     /*    sweeps, coarse correction with the plain V-cycle one     */
                     /*    depth down, nu post-sweeps in reverse colour order)      */
  int samples;       /* error samples per depth (four): 0 normal random vectors;    */
                     /*    1 the error one plain Gauss-Seidel V(2,2) cycle on       */
                     /*    A e = 0 leaves from such a vector; 2 two of each         */
  const double *t_each; /* nullable host array of nsys values: t of each system    */
                     /*    (replaces t; each system may then appear only once)      */
} camfe_train_opts;

/* Model from packed FP32 parameters (levels x 2081, copied) or, with params
 * NULL, a fixed deterministic initialisation (s near 1: l1-Jacobi for sweep 0,
 * Gauss-Seidel for sweep 1). */
camfe_status camfe_model_create(const float *params, int levels, int bf16, int sweep, camfe_model *out);
/* Model as a file: a plain binary record (no serialised objects) of the
 * 8-byte tag "CAMFESM1", four little-endian int32 (levels, bf16, sweep, 2081
 * parameters per level) and levels x 2081 little-endian FP32 parameters.
 * save: EINVAL for a null model or path, EDEVICE when the file cannot be
 * written.  load: EINVAL when the file cannot be read, has another tag, sizes
 * out of range, or a length that does not match its header; on success *out
 * is a new model (camfe_model_destroy). */
camfe_status camfe_smoother_save(camfe_model m, const char *path);
camfe_status camfe_smoother_load(const char *path, camfe_model *out);
/* Two-call export of the packed parameters; levels, bf16 and sweep may be NULL. */
camfe_status camfe_model_params(camfe_model m, float *params, int64_t cap, int64_t *n, int *levels, int *bf16,
                                int *sweep);
void camfe_model_destroy(camfe_model m);
/* Attach a model (not owned; must outlive its use by camfe_solve) or detach
 * with NULL.  smoother = 2 in camfe_solve needs an attached model (ESTATE). */
camfe_status camfe_smoother_attach(camfe_sys s, camfe_model m);
/* omega_i = c_i s_i of every function at one assembled depth (canonical
 * order, n_d doubles) for A = M + t L. */
camfe_status camfe_smoother_omega(camfe_sys s, camfe_model m, int depth, double t, double *omega);
/* Training loss at one depth for one MLP's parameters (2081 floats), a sweep
 * type and nsamples (1..4) error samples e0 (n_d x nsamples column-major,
 * canonical order), with its gradient (2081 doubles; grad may be NULL).
 * cycle 0: nu sweeps (an SOR sweep relaxes colour 0, then 1, ...); cycle 1: a
 * two-grid cycle, nu sweeps, e - P B_c P^T A e with B_c one plain FP64
 * Gauss-Seidel V(2,2)-cycle at depth - 1 (ESTATE at the coarsest depth), nu
 * sweeps with the colours reversed.  Loss log(|A e_end|^2 / |A e0|^2) averaged
 * over the samples.  Sweeps, correction and adjoints run in FP64; the MLP in
 * FP32 or BF16 weights. */
camfe_status camfe_smoother_loss_grad(camfe_sys s, int depth, double t, const float *params, int bf16, int sweep,
                                      int cycle, const double *e0, int nsamples, int nu, double *loss, double *grad);
/* Train a model on the GPU: for every system and depth above the coarsest,
 * four error samples (opts->samples), then opts->steps Adam steps on the mean
 * loss (opts->cycle) per MLP.
 * loss_history (nullable) receives the mean loss over all depths before each
 * step.  The systems' solver state for opts->t is built when missing. */
camfe_status camfe_smoother_train(camfe_ctx ctx, camfe_sys const *systems, int nsys, const camfe_train_opts *opts,
                                  camfe_model *out, double *loss_history);

#ifdef __cplusplus
}
#endif
#endif /* CAMFE_H */
